// LWE key switching LWE_{s'}(kN) -> LWE_s(n) (TFHE ePrint 2018/421, Sec. 4):
// out = (0^n, b') - sum_{i<kN} sum_{j<t} KSK[i][j][v_ij], where v_ij is the
// j-th most significant base-2^b digit of a'_i rounded (ties up) to t*b bits.
//
// A workgroup owns a tile of 64 output words x 64 ciphertexts; thread
// (word x, group y) accumulates 16 ciphertexts of one output word.  For each
// (i, j) the 2^b table rows of the word are read once (coalesced across the
// 64 words of the tile) and selected per ciphertext; the rounded inputs of
// the tile are staged in LDS one chunk of 64 input coefficients at a time.
#include "fhesql_internal.h"

namespace {

constexpr int TW = 64;       // output words per tile
constexpr int TC = 64;       // ciphertexts per tile
constexpr int THREADS = 256;
constexpr int PER = TC / (THREADS / TW);  // ciphertexts per thread (16)
constexpr int ICH = 64;      // input coefficients per LDS chunk

template <typename T, int V>
__global__ __launch_bounds__(THREADS) void keyswitch_kernel(const T* __restrict__ big, const T* __restrict__ ksk,
                                                            T* out, const uint64_t* out_ptrs, int B, int n,
                                                            int kN, int t, int bb) {
    __shared__ uint32_t rt[TC][ICH + 1];
    const int tx = threadIdx.x % TW, ty = threadIdx.x / TW;
    const int w = blockIdx.x * TW + tx;
    const int c0 = blockIdx.y * TC;
    const int tb = t * bb;
    T acc[PER];
#pragma unroll
    for (int s = 0; s < PER; s++) {
        const int c = c0 + ty + s * (THREADS / TW);
        acc[s] = (w == n && c < B) ? big[(size_t)c * (kN + 1) + kN] : (T)0;
    }
    const size_t row = (size_t)(n + 1);
    for (int i0 = 0; i0 < kN; i0 += ICH) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < TC * ICH; idx += THREADS) {
            const int cc = idx / ICH, ii = idx % ICH;
            const int c = c0 + cc;
            uint32_t r = 0;
            if (c < B && i0 + ii < kN) r = (uint32_t)round_top<T>(big[(size_t)c * (kN + 1) + i0 + ii], tb);
            rt[cc][ii] = r;
        }
        __syncthreads();
        const int iend = min(ICH, kN - i0);
        if (w <= n) {
            for (int ii = 0; ii < iend; ii++) {
                const T* base = ksk + ((size_t)(i0 + ii) * t) * V * row + w;
                for (int j = 0; j < t; j++) {
                    T tab[V];
#pragma unroll
                    for (int v = 0; v < V; v++) tab[v] = base[((size_t)j * V + v) * row];
                    const int sh = (t - 1 - j) * bb;
#pragma unroll
                    for (int s = 0; s < PER; s++) {
                        const uint32_t v = (rt[ty + s * (THREADS / TW)][ii] >> sh) & (V - 1);
                        T sel = tab[0];
#pragma unroll
                        for (int q = 1; q < V; q++) sel = v == (uint32_t)q ? tab[q] : sel;
                        acc[s] -= sel;
                    }
                }
            }
        }
    }
    if (w <= n) {
#pragma unroll
        for (int s = 0; s < PER; s++) {
            const int c = c0 + ty + s * (THREADS / TW);
            if (c >= B) continue;
            T* dst = out_ptrs ? (T*)(uintptr_t)out_ptrs[c] : out + (size_t)c * row;
            dst[w] = acc[s];
        }
    }
}

template <typename T>
int launch_ks_t(tfhe_ctx* c, const void* big, void* out, const uint64_t* out_ptrs, uint32_t B, hipStream_t s) {
    const int n = (int)c->p.n, kN = (int)(c->p.k * c->p.N), t = (int)c->p.ks_t, bb = (int)c->p.ks_base_bits;
    dim3 grid((n + 1 + TW - 1) / TW, (B + TC - 1) / TC);
    const T* k = (const T*)c->d_ksk;
    switch (bb) {
        case 1: hipLaunchKernelGGL((keyswitch_kernel<T, 2>), grid, dim3(THREADS), 0, s, (const T*)big, k, (T*)out, out_ptrs, (int)B, n, kN, t, bb); break;
        case 2: hipLaunchKernelGGL((keyswitch_kernel<T, 4>), grid, dim3(THREADS), 0, s, (const T*)big, k, (T*)out, out_ptrs, (int)B, n, kN, t, bb); break;
        case 3: hipLaunchKernelGGL((keyswitch_kernel<T, 8>), grid, dim3(THREADS), 0, s, (const T*)big, k, (T*)out, out_ptrs, (int)B, n, kN, t, bb); break;
        case 4: hipLaunchKernelGGL((keyswitch_kernel<T, 16>), grid, dim3(THREADS), 0, s, (const T*)big, k, (T*)out, out_ptrs, (int)B, n, kN, t, bb); break;
        default: return ctx_fail(c, TFHE_EINVAL, "key-switching base must be 2^1..2^4");
    }
    return hip_check(c, hipGetLastError(), "launch keyswitch");
}

}  // namespace

int launch_keyswitch(tfhe_ctx* c, const void* big_in, void* out, const uint64_t* out_ptrs, uint32_t B,
                     hipStream_t s) {
    if (B == 0) return TFHE_OK;
    TimedLaunch tl(c, s, 1, B);
    return c->q == 32 ? launch_ks_t<uint32_t>(c, big_in, out, out_ptrs, B, s)
                      : launch_ks_t<uint64_t>(c, big_in, out, out_ptrs, B, s);
}
