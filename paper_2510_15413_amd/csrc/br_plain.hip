// Blind rotation + sample extraction with a plain scalar-integer external
// product: the baseline for the limb-split MFMA kernel.  Same definition
// (TFHE ePrint 2018/421, Alg. 3): ACC <- ACC + ExtProd(BSK_i, X^{abar_i} ACC - ACC)
// for i = 0..n-1, each negacyclic product computed with wrapping u32/u64
// multiply-adds.  A workgroup owns PB ciphertexts; the accumulators, the
// digits of the step and the sign-extended key block of one (u,p) live in
// LDS.  Thread t accumulates the outputs o = t, t+256, ... (component v = o/N,
// coefficient o%N) of all PB ciphertexts.
#include "fhesql_internal.h"

namespace {

constexpr int THREADS = 256;

struct PlainArgs {
    const void* lwe;
    const void* bsk;          // [n][2l][2][N] words
    const void* tv;
    const int32_t* tv_index;
    void* out;                // [B][N+1]
    int B, n, N, l, bg_bits;
};

template <typename T, int PB, int OUTS>
__global__ __launch_bounds__(THREADS) void br_plain_kernel(PlainArgs a) {
    const int n = a.n, N = a.N, l = a.l, bgb = a.bg_bits, NB = 2 * l;
    const int lg2n = __builtin_ctz(2 * N);
    const int tid = threadIdx.x;
    const int ct0 = blockIdx.x * PB;
    const T* lwe = (const T*)a.lwe;
    const T* bsk = (const T*)a.bsk;

    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    T* acc = (T*)smem;                                   // [PB][2][N]
    T* kx = acc + (size_t)PB * 2 * N;                    // [2][2N] extended key
    int8_t* dg = (int8_t*)(kx + (size_t)2 * 2 * N);      // [2l][N][PB]
    uint16_t* abar = (uint16_t*)(dg + (size_t)NB * N * PB);  // [PB][n]

    for (int idx = tid; idx < PB * n; idx += THREADS) {
        const int c = idx / n, i = idx - c * n;
        const int gi = ct0 + c;
        abar[idx] = gi < a.B ? (uint16_t)mod_switch<T>(lwe[(size_t)gi * (n + 1) + i], lg2n) : 0;
    }
    for (int idx = tid; idx < PB * N; idx += THREADS) {
        const int c = idx / N, j = idx - c * N;
        const int gi = ct0 + c;
        T body = 0;
        if (gi < a.B) {
            const int bb = (int)mod_switch<T>(lwe[(size_t)gi * (n + 1) + n], lg2n);
            const int e = (2 * N - bb) & (2 * N - 1);
            const T* tv = (const T*)a.tv + (size_t)(a.tv_index ? a.tv_index[gi] : 0) * N;
            body = monomial_coef<T>([&](int s) -> T { return tv[s]; }, N, e, j);
        }
        acc[((size_t)c * 2 + 0) * N + j] = 0;
        acc[((size_t)c * 2 + 1) * N + j] = body;
    }
    __syncthreads();

    const int half = 1 << (bgb - 1);
    const uint32_t bgm = (1u << bgb) - 1;
    uint32_t off = 0;
    for (int p = 0; p < l; p++) off += (uint32_t)half << (p * bgb);
    int ov[OUTS], oj[OUTS];
#pragma unroll
    for (int s = 0; s < OUTS; s++) {
        const int o = tid + s * THREADS;
        ov[s] = o < 2 * N ? o / N : -1;
        oj[s] = o < 2 * N ? o % N : 0;
    }

    for (int i = 0; i < n; i++) {
        // digits of X^{abar} ACC - ACC
        for (int idx = tid; idx < PB * 2 * N; idx += THREADS) {
            const int c = idx % PB, rest = idx / PB;
            const int j = rest % N, u = rest / N;
            const T* P = acc + ((size_t)c * 2 + u) * N;
            T rot = monomial_coef<T>([&](int s) -> T { return P[s]; }, N, abar[c * n + i], j);
            uint32_t y = (uint32_t)round_top<T>((T)(rot - P[j]), l * bgb) + off;
            for (int p = 0; p < l; p++) {
                int d = (int)((y >> ((l - 1 - p) * bgb)) & bgm) - half;
                dg[((size_t)(u * l + p) * N + j) * PB + c] = (int8_t)d;
            }
        }
        T sum[OUTS][PB];
#pragma unroll
        for (int s = 0; s < OUTS; s++)
#pragma unroll
            for (int c = 0; c < PB; c++) sum[s][c] = 0;
        for (int ub = 0; ub < NB; ub++) {
            __syncthreads();  // digits ready; previous key block consumed
            const T* K = bsk + ((size_t)i * NB + ub) * 2 * N;
            for (int idx = tid; idx < 2 * 2 * N; idx += THREADS) {
                const int v = idx / (2 * N), x = idx - v * 2 * N;
                // kx[v][x] = Kext[x - N]: K[x-N] for x >= N, -K[x] for x < N
                kx[idx] = x >= N ? K[(size_t)v * N + x - N] : (T)(0 - K[(size_t)v * N + x]);
            }
            __syncthreads();
            const int8_t* D = dg + (size_t)ub * N * PB;
            for (int kk = 0; kk < N; kk++) {
                T dv[PB];
#pragma unroll
                for (int c = 0; c < PB; c++) dv[c] = (T)(int64_t)D[kk * PB + c];
#pragma unroll
                for (int s = 0; s < OUTS; s++) {
                    if (ov[s] < 0) continue;
                    const T key = kx[(size_t)ov[s] * 2 * N + N + oj[s] - kk];
#pragma unroll
                    for (int c = 0; c < PB; c++) sum[s][c] += key * dv[c];
                }
            }
        }
        __syncthreads();  // all digit reads of this step are done
#pragma unroll
        for (int s = 0; s < OUTS; s++) {
            if (ov[s] < 0) continue;
#pragma unroll
            for (int c = 0; c < PB; c++) acc[((size_t)c * 2 + ov[s]) * N + oj[s]] += sum[s][c];
        }
        __syncthreads();
    }

    T* out = (T*)a.out;
    for (int idx = tid; idx < PB * (N + 1); idx += THREADS) {
        const int c = idx / (N + 1), j = idx - c * (N + 1);
        const int gi = ct0 + c;
        if (gi >= a.B) continue;
        const T* A0 = acc + (size_t)c * 2 * N;
        T val;
        if (j == 0) val = A0[0];
        else if (j < N) val = (T)(0 - A0[N - j]);
        else val = A0[N];
        out[(size_t)gi * (N + 1) + j] = val;
    }
}

template <typename T, int PB>
size_t plain_lds(const tfhe_ctx* c) {
    const size_t N = c->p.N, l = c->p.l;
    return (size_t)PB * 2 * N * sizeof(T) + 4 * N * sizeof(T) + 2 * l * N * PB + (size_t)PB * c->p.n * 2 + 16;
}

template <typename T, int PB, int OUTS>
int launch_plain_o(tfhe_ctx* c, const PlainArgs& a, hipStream_t s) {
    const size_t lds = plain_lds<T, PB>(c);
    auto k = br_plain_kernel<T, PB, OUTS>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_check(c, e, "hipFuncSetAttribute(br_plain)");
    hipLaunchKernelGGL(k, dim3((a.B + PB - 1) / PB), dim3(THREADS), lds, s, a);
    return hip_check(c, hipGetLastError(), "launch br_plain");
}

template <typename T, int PB>
int launch_plain_t(tfhe_ctx* c, const PlainArgs& a, hipStream_t s) {
    switch ((2 * a.N + THREADS - 1) / THREADS) {
        case 1: return launch_plain_o<T, PB, 1>(c, a, s);
        case 2: return launch_plain_o<T, PB, 2>(c, a, s);
        case 4: return launch_plain_o<T, PB, 4>(c, a, s);
        case 8: return launch_plain_o<T, PB, 8>(c, a, s);
        case 16: return launch_plain_o<T, PB, 16>(c, a, s);
    }
    return ctx_fail(c, TFHE_EINVAL, "unsupported N for the plain kernel");
}

}  // namespace

int launch_br_plain(tfhe_ctx* c, const void* lwe_in, const void* tv, const int32_t* tv_index,
                    void* big_out, uint32_t B, hipStream_t s) {
    PlainArgs a;
    a.lwe = lwe_in;
    a.bsk = c->d_bsk;
    a.tv = tv;
    a.tv_index = tv_index;
    a.out = big_out;
    a.B = (int)B;
    a.n = (int)c->p.n;
    a.N = (int)c->p.N;
    a.l = (int)c->p.l;
    a.bg_bits = (int)c->p.bg_bits;
    const size_t max_lds = 160 * 1024;
    if (c->q == 32) {
        if (plain_lds<uint32_t, 4>(c) <= max_lds) return launch_plain_t<uint32_t, 4>(c, a, s);
        if (plain_lds<uint32_t, 2>(c) <= max_lds) return launch_plain_t<uint32_t, 2>(c, a, s);
        return launch_plain_t<uint32_t, 1>(c, a, s);
    }
    if (plain_lds<uint64_t, 2>(c) <= max_lds) return launch_plain_t<uint64_t, 2>(c, a, s);
    return launch_plain_t<uint64_t, 1>(c, a, s);
}
