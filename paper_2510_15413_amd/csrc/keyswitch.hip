// LWE key switching LWE_{s'}(kN) -> LWE_s(n) (TFHE ePrint 2018/421, Sec. 4):
// out = (0^n, b') - sum_{i<kN} sum_{j<t} KSK[i][j][v_ij], where v_ij is the
// j-th most significant base-2^b digit of a'_i rounded (ties up) to t*b bits.
//
// Digits.  A pre-pass rounds every mask coefficient a'_i of the batch to its
// top t*b bits once and stores them coefficient-major, dig[i][c] (16-bit
// when t*b <= 16, else 32-bit): the word tiles of one ciphertext group then
// read one coalesced row of digits per coefficient instead of each tile
// re-reading (and re-rounding) the strided full-width words of every
// ciphertext, which halves or quarters the bytes each XCD pulls per tile
// and keeps them in L2 while the tiles that share them run.
//
// Mapping.  Lanes are ciphertexts: a workgroup of 4 waves owns 256
// ciphertexts (64 per wave) and a tile of WPW output words, and every lane
// accumulates those WPW words of its own ciphertext in registers.  The digit
// that picks a table row is then a per-lane value, so the pick is an LDS
// address rather than a select chain.  For each input coefficient i the
// t*2^b table rows restricted to the tile's words are staged in LDS (double
// buffered; each thread loads its share of the next coefficients into
// registers while the current ones are consumed; 32-bit words stage up to 8
// coefficients per barrier), and each lane reads the row its digit selects
// with 16-byte LDS reads.  Rows are padded by 16 bytes so that the
// lanes' distinct rows fall on different bank groups.
//
// Placement.  Workgroups are dealt round-robin to the 8 XCDs, each with its
// own L2.  The grid is one-dimensional and a workgroup's (word tile,
// ciphertext group) is taken from a tile-major or group-major order cut into
// 8 contiguous runs, one per XCD: tile-major when the table is larger than
// the batch's inputs (each XCD then fetches only its tiles' columns of the
// table, whose rows start on 128-byte lines), group-major otherwise (each XCD
// fetches only its groups' inputs).
#include "fhesql_internal.h"

namespace {

constexpr int THREADS = 256;
constexpr int TC = 256;     // ciphertexts per workgroup (one per thread)
constexpr int PMAX = 8;     // staged elements per thread and coefficient (t*2^b*WPW <= PMAX*THREADS)

template <typename T>
struct Vec16;  // 16 bytes of table words
template <>
struct Vec16<uint32_t> {
    typedef uint32_t type __attribute__((ext_vector_type(4)));
    static constexpr int N = 4;
};
template <>
struct Vec16<uint64_t> {
    typedef uint64_t type __attribute__((ext_vector_type(2)));
    static constexpr int N = 2;
};

// Rounded digits of a 64 x 64 block (ciphertexts x coefficients): rows of
// the ciphertexts are read coalesced, turned in LDS, and written as rows of
// the coefficient-major digit array.
template <typename T, typename D>
__global__ __launch_bounds__(THREADS) void ks_digits_kernel(const T* __restrict__ big, D* __restrict__ dig, int B,
                                                            int kN, int tb) {
    __shared__ uint32_t blk[64][65];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
#pragma unroll
    for (int m = 0; m < 16; m++) {
        const int r = w + 4 * m, c = c0 + r, i = i0 + lane;
        blk[r][lane] = (c < B && i < kN) ? (uint32_t)round_top<T>(big[(size_t)c * (kN + 1) + i], tb) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; m++) {
        const int col = w + 4 * m, c = c0 + lane, i = i0 + col;
        if (c < B && i < kN) dig[(size_t)i * B + c] = (D)blk[lane][col];
    }
}

struct KsPlace {
    int tiles, groups;  // word tiles and ciphertext groups
    int per;            // workgroups per XCD run (the grid is 8 * per)
    int tile_major;     // 1: runs of consecutive tiles, 0: runs of consecutive groups
};

template <typename T, typename D, int V, int WPW, int P>
__global__ __launch_bounds__(THREADS) void keyswitch_kernel(const T* __restrict__ big, const D* __restrict__ dig,
                                                            const T* __restrict__ ksk, T* out,
                                                            const uint64_t* out_ptrs, int B, int n, int kN, int t,
                                                            int bb, int ks_row, KsPlace pl) {
    typedef typename Vec16<T>::type vec;
    constexpr int EV = Vec16<T>::N;          // words per 16-byte read
    constexpr int RS = WPW + EV;             // LDS row stride in words (16-byte pad)
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    T* tab = (T*)smem;                       // [2][P][t*V][RS]
    const int TS = t * V * RS;               // words per coefficient
    const int tid = threadIdx.x;
    // workgroup L runs on XCD L % 8 as the (L / 8)-th of that XCD's run
    const int z = (int)(blockIdx.x % 8) * pl.per + (int)(blockIdx.x / 8);
    if (z >= pl.tiles * pl.groups) return;  // padding of the last run
    const int tile = pl.tile_major ? z / pl.groups : z % pl.tiles;
    const int grp = pl.tile_major ? z % pl.groups : z / pl.tiles;
    const int c = grp * TC + tid;
    const int w0 = tile * WPW;
    const size_t row = (size_t)ks_row;  // table row stride in words
    const int E = t * V * WPW;               // staged words per coefficient
    const bool live = c < B;
    const D* digc = dig + (live ? c : 0);  // coefficient i's digits at digc[i * B]

    T acc[WPW];
#pragma unroll
    for (int k = 0; k < WPW; k++) acc[k] = (w0 + k == n && live) ? big[(size_t)c * (kN + 1) + kN] : (T)0;

    // Subtract the rows that coefficient value r selects, from the rows of
    // one coefficient staged at cbuf.
    auto consume = [&](const T* cbuf, uint32_t r) {
        for (int j = 0; j < t; j++) {
            const uint32_t d = (r >> ((t - 1 - j) * bb)) & (V - 1);
            const vec* rp = (const vec*)(cbuf + (j * V + d) * RS);
#pragma unroll
            for (int q = 0; q < WPW / EV; q++) {
                const vec x = rp[q];
#pragma unroll
                for (int e = 0; e < EV; e++) acc[q * EV + e] -= x[e];
            }
        }
    };
    T pf[PMAX];
    if constexpr (P == 1) {
        // One coefficient per barrier: this thread's share of its tile rows,
        // element e = tid + m*THREADS is word e % WPW of row (j, v) =
        // (e / WPW / V, e / WPW % V).
#define KS_FETCH(I)                                                                     \
    do {                                                                                \
        _Pragma("unroll") for (int m = 0; m < PMAX; m++) {                              \
            const int e = tid + m * THREADS;                                            \
            const int k = e % WPW, jv = e / WPW;                                        \
            pf[m] = (e < E && w0 + k <= n) ? ksk[((size_t)(I) * t * V + jv) * row + w0 + k] : (T)0; \
        }                                                                               \
    } while (0)
#define KS_STAGE(BUF)                                                                   \
    do {                                                                                \
        _Pragma("unroll") for (int m = 0; m < PMAX; m++) {                              \
            const int e = tid + m * THREADS;                                            \
            if (e < E) tab[(size_t)(BUF) * TS + (e / WPW) * RS + e % WPW] = pf[m];      \
        }                                                                               \
    } while (0)
        KS_FETCH(0);
        KS_STAGE(0);
        __syncthreads();
        for (int i = 0; i < kN; i++) {
            if (i + 1 < kN) KS_FETCH(i + 1);
            const uint32_t r = live ? (uint32_t)digc[(size_t)i * B] : 0u;
            consume(tab + (size_t)(i & 1) * TS, r);
            if (i + 1 < kN) KS_STAGE((i + 1) & 1);
            __syncthreads();
        }
#undef KS_FETCH
#undef KS_STAGE
    } else {
        // P coefficients per barrier.  Element e = tid + m*THREADS is word
        // e' % WPW of row (e' / WPW) of coefficient e / E (e' = e % E); its
        // offsets relative to the group's first coefficient are formed once.
        int gofs[PMAX], lofs[PMAX];
#pragma unroll
        for (int m = 0; m < PMAX; m++) {
            const int e = tid + m * THREADS;
            const int ci = e / E, er = e - ci * E;
            const int k = er % WPW, jv = er / WPW;
            const bool take = e < P * E;
            gofs[m] = take && w0 + k <= n ? (ci * t * V + jv) * (int)row + w0 + k : -1;  // -1: stage a zero
            lofs[m] = take ? ci * TS + jv * RS + k : -1;                                 // -1: nothing to stage
        }
        auto fetch = [&](int i0) {
            const T* kg = ksk + (size_t)i0 * t * V * row;
#pragma unroll
            for (int m = 0; m < PMAX; m++) pf[m] = gofs[m] >= 0 ? kg[gofs[m]] : (T)0;
        };
        auto stage = [&](int buf) {
#pragma unroll
            for (int m = 0; m < PMAX; m++)
                if (lofs[m] >= 0) tab[(size_t)buf * P * TS + lofs[m]] = pf[m];
        };
        fetch(0);
        stage(0);
        __syncthreads();
        for (int i0 = 0, g = 0; i0 < kN; i0 += P, g++) {
            // this group's coefficients first, so that waiting for them does
            // not wait for the next group's rows
            uint32_t rr[P];
#pragma unroll
            for (int ii = 0; ii < P; ii++) rr[ii] = live ? (uint32_t)digc[(size_t)(i0 + ii) * B] : 0u;
            if (i0 + P < kN) fetch(i0 + P);
            const T* tbuf = tab + (size_t)(g & 1) * P * TS;
#pragma unroll
            for (int ii = 0; ii < P; ii++) consume(tbuf + ii * TS, rr[ii]);
            if (i0 + P < kN) stage((g + 1) & 1);
            __syncthreads();
        }
    }
    if (!live) return;
    T* dst = out_ptrs ? (T*)(uintptr_t)out_ptrs[c] : out + (size_t)c * (n + 1);
#pragma unroll
    for (int k = 0; k < WPW; k++)
        if (w0 + k <= n) dst[w0 + k] = acc[k];
}

// ---- 32-bit words: the key switch as int8 matrix products.
//
// out[c][w] = [w == n] b'_c - sum_k X[c][k] Y[k][w]  (mod 2^32), with X the
// one-hot digit matrix, X[c][(i*t + j)*V + v] = [digit_ij(c) == v], and Y the
// table rows.  Y is split into balanced int8 limbs, Y = sum_m 2^{8m} Y_m; each
// limb product is exact in int32 (kN*t ones per row of X, |limb| <= 128), and
// the limb sums are combined mod 2^32 at the end.  v_mfma_i32_16x16x64_i8
// takes A = a 16-word tile of Y_m (each word's 64 k of a chunk contiguous,
// staged in LDS chunk by chunk, double-buffered) and B = 16 ciphertexts'
// one-hot rows of the chunk, formed in registers from the digits (a lane's 16
// bytes are PPL = 16/V consecutive (i, j) pairs, one byte set per pair).  A
// workgroup of 4 waves owns TW word tiles (one: two would hold 268 registers
// per lane, one wave per SIMD) and 64 KM_CT ciphertexts (KM_CT tiles of 16
// per wave: 4, or 2 when the grid would not fill the CUs), so each staged A
// fragment feeds KM_CT MFMAs; a wave's output tile holds 4 consecutive words
// of one ciphertext per lane.

template <int V, typename D, int TW, int KM_CT>
__global__ __launch_bounds__(THREADS) void ks_mfma_kernel(const uint32_t* __restrict__ big, const D* __restrict__ dig,
                                                          const int8_t* __restrict__ ytab, uint32_t* out,
                                                          const uint64_t* out_ptrs, int B, int n, int kN, int t,
                                                          int bb, int Wp, KsPlace pl) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    constexpr int PPL = 16 / V;                 // (i, j) pairs in a lane's 16 bytes of a chunk
    constexpr int CHU = TW * 4 * 16 * 4;        // 16-byte units of table per chunk: TW tiles x 4 limbs x 16 words x 64 k
    constexpr int UPT = CHU / THREADS;          // units per thread
    static_assert(CHU % THREADS == 0, "whole units per thread");
    __shared__ __attribute__((aligned(16))) int8_t tb[2][CHU * 16];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int z = (int)(blockIdx.x % 8) * pl.per + (int)(blockIdx.x / 8);
    if (z >= pl.tiles * pl.groups) return;  // padding of the last run
    const int tile = pl.tile_major ? z / pl.groups : z % pl.tiles;
    const int grp = pl.tile_major ? z % pl.groups : z / pl.tiles;
    const int w0 = tile * TW * 16;
    const size_t K = (size_t)kN * t * V;
    const int NCH = (int)(K / 64);
    const size_t plane = (size_t)Wp * K;  // bytes of one limb plane
    const int g = lane >> 4;
    const int cl = grp * 64 * KM_CT + wave * 16 * KM_CT + (lane & 15);  // this lane's ciphertext of tile 0 (tile ct: + 16 ct)

    // table staging: unit u = tid + q*THREADS is row R = u/4 (limb m = R / (16 TW), word
    // w0 + R % (16 TW)), 16 bytes `part` = u % 4 of the chunk's 64
    const int8_t* src[UPT];
    int dst[UPT];
#pragma unroll
    for (int q = 0; q < UPT; q++) {
        const int u = tid + q * THREADS, R = u >> 2, part = u & 3;
        const int m = R / (16 * TW), w = w0 + R % (16 * TW);
        src[q] = w < Wp ? ytab + (size_t)m * plane + (size_t)w * K + 16 * part : nullptr;
        dst[q] = R * 64 + 16 * part;
    }
    uint4 st[UPT];
    auto fetch = [&](int ch) {
#pragma unroll
        for (int q = 0; q < UPT; q++) st[q] = src[q] ? *(const uint4*)(src[q] + (size_t)ch * 64) : make_uint4(0, 0, 0, 0);
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < UPT; q++) *(uint4*)(tb[buf] + dst[q]) = st[q];
    };

    // digits of a lane's pairs in chunk ch for ciphertext tile ct: the pairs
    // P0 .. P0+PPL-1 (P0 = (64 ch + 16 g) / V) touch rows i0 and i0 + 1
    auto digit_rows = [&](int ch, int ct, uint32_t& lo, uint32_t& hi, int& j0) {
        const int P0 = (64 * ch + 16 * g) / V;
        const int i0 = P0 / t;
        j0 = P0 - i0 * t;
        const int c = cl + 16 * ct;
        const bool live = c < B;
        lo = live ? (uint32_t)dig[(size_t)i0 * B + c] : 0u;
        hi = live && i0 + 1 < kN ? (uint32_t)dig[(size_t)(i0 + 1) * B + c] : 0u;
    };
    auto onehot = [&](uint32_t lo, uint32_t hi, int j0) -> v4i {
        uint32_t wv[4] = {0, 0, 0, 0};
        int j = j0;
        bool up = false;
#pragma unroll
        for (int p = 0; p < PPL; p++) {
            const uint32_t r = up ? hi : lo;
            const int d = (int)((r >> ((t - 1 - j) * bb)) & (V - 1));
            const int pos = p * V + d;  // byte of the lane's 16
#pragma unroll
            for (int e = 0; e < 4; e++) wv[e] |= (pos >> 2) == e ? 1u << (8 * (pos & 3)) : 0u;
            if (++j == t) { j = 0; up = true; }
        }
        return v4i{(int)wv[0], (int)wv[1], (int)wv[2], (int)wv[3]};
    };

    v4i acc[TW][KM_CT][4];
#pragma unroll
    for (int wt = 0; wt < TW; wt++)
#pragma unroll
        for (int ct = 0; ct < KM_CT; ct++)
#pragma unroll
            for (int m = 0; m < 4; m++) acc[wt][ct][m] = v4i{0, 0, 0, 0};

    fetch(0);
    stage(0);
    uint32_t dlo[KM_CT], dhi[KM_CT];
    int dj0 = 0;
#pragma unroll
    for (int ct = 0; ct < KM_CT; ct++) digit_rows(0, ct, dlo[ct], dhi[ct], dj0);
    __syncthreads();
    for (int ch = 0; ch < NCH; ch++) {
        const int buf = ch & 1;
        if (ch + 1 < NCH) fetch(ch + 1);
        v4i bx[KM_CT];
#pragma unroll
        for (int ct = 0; ct < KM_CT; ct++) bx[ct] = onehot(dlo[ct], dhi[ct], dj0);
        if (ch + 1 < NCH) {
#pragma unroll
            for (int ct = 0; ct < KM_CT; ct++) digit_rows(ch + 1, ct, dlo[ct], dhi[ct], dj0);
        }
#pragma unroll
        for (int wt = 0; wt < TW; wt++)
#pragma unroll
            for (int m = 0; m < 4; m++) {
                const v4i a = *(const v4i*)(tb[buf] + ((m * TW + wt) * 16 + (lane & 15)) * 64 + 16 * g);
#pragma unroll
                for (int ct = 0; ct < KM_CT; ct++)
                    acc[wt][ct][m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bx[ct], acc[wt][ct][m], 0, 0, 0);
            }
        if (ch + 1 < NCH) stage(buf ^ 1);
        __syncthreads();
    }
    // lane holds words w0 + 16 wt + 4g + e of ciphertext cl + 16 ct
#pragma unroll
    for (int ct = 0; ct < KM_CT; ct++) {
        const int c = cl + 16 * ct;
        if (c >= B) continue;
        uint32_t* dstp = out_ptrs ? (uint32_t*)(uintptr_t)out_ptrs[c] : out + (size_t)c * (n + 1);
        const uint32_t body = big[(size_t)c * (kN + 1) + kN];
#pragma unroll
        for (int wt = 0; wt < TW; wt++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int w = w0 + 16 * wt + 4 * g + e;
                if (w > n) continue;
                uint32_t val = 0;
#pragma unroll
                for (int m = 0; m < 4; m++) val += (uint32_t)acc[wt][ct][m][e] << (8 * m);
                dstp[w] = (w == n ? body : 0u) - val;
            }
    }
}

template <int V, typename D, int TW, int KM_CT>
int launch_mfma_ct(tfhe_ctx* c, const uint32_t* big, const D* dig, uint32_t* out, const uint64_t* out_ptrs,
                   uint32_t B, hipStream_t s) {
    const int n = (int)c->p.n, kN = (int)(c->p.k * c->p.N), t = (int)c->p.ks_t, bb = (int)c->p.ks_base_bits;
    KsPlace pl;
    pl.tiles = (c->ks_wp / 16 + TW - 1) / TW;
    pl.groups = (int)((B + 64 * KM_CT - 1) / (64 * KM_CT));
    pl.per = (pl.tiles * pl.groups + 7) / 8;
    const double table = 4.0 * c->ks_wp * kN * t * V, inputs = (double)B * kN * sizeof(D);
    pl.tile_major = table > inputs ? 1 : 0;
    hipLaunchKernelGGL((ks_mfma_kernel<V, D, TW, KM_CT>), dim3(8 * pl.per), dim3(THREADS), 0, s, big, dig,
                       (const int8_t*)c->d_ksk8, out, out_ptrs, (int)B, n, kN, t, bb, c->ks_wp, pl);
    return hip_check(c, hipGetLastError(), "launch ks_mfma");
}

template <int V, typename D, int TW>
int launch_mfma_ks(tfhe_ctx* c, const uint32_t* big, void* dig_ws, uint32_t* out, const uint64_t* out_ptrs,
                   uint32_t B, hipStream_t s) {
    const int kN = (int)(c->p.k * c->p.N), t = (int)c->p.ks_t, bb = (int)c->p.ks_base_bits;
    D* dig = (D*)dig_ws;
    hipLaunchKernelGGL((ks_digits_kernel<uint32_t, D>), dim3((kN + 63) / 64, (B + 63) / 64), dim3(THREADS), 0, s,
                       big, dig, (int)B, kN, t * bb);
    // 4 ciphertext tiles per wave, or 2 when that leaves CUs idle (measured:
    // 4096 ciphertexts at n = 64 0.069 -> 0.052 ms; 4 is faster once the grid
    // fills the chip)
    const int cus = c->prop.multiProcessorCount > 0 ? c->prop.multiProcessorCount : 256;
    const int64_t wgs4 = (int64_t)((c->ks_wp / 16 + TW - 1) / TW) * ((B + 255) / 256);
    if (wgs4 < cus) return launch_mfma_ct<V, D, TW, 2>(c, big, dig, out, out_ptrs, B, s);
    return launch_mfma_ct<V, D, TW, 4>(c, big, dig, out, out_ptrs, B, s);
}

template <typename T, typename D, int V, int WPW, int P>
int launch_p(tfhe_ctx* c, const T* big, void* dig_ws, T* out, const uint64_t* out_ptrs, uint32_t B, hipStream_t s) {
    const int n = (int)c->p.n, kN = (int)(c->p.k * c->p.N), t = (int)c->p.ks_t, bb = (int)c->p.ks_base_bits;
    constexpr int RS = WPW + Vec16<T>::N;
    const size_t lds = 2ull * P * t * V * RS * sizeof(T);
    D* dig = (D*)dig_ws;
    hipLaunchKernelGGL((ks_digits_kernel<T, D>), dim3((kN + 63) / 64, (B + 63) / 64), dim3(THREADS), 0, s, big, dig,
                       (int)B, kN, t * bb);
    auto k = keyswitch_kernel<T, D, V, WPW, P>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_check(c, e, "hipFuncSetAttribute(keyswitch)");
    KsPlace pl;
    pl.tiles = (n + 1 + WPW - 1) / WPW;
    pl.groups = (int)((B + TC - 1) / TC);
    pl.per = (pl.tiles * pl.groups + 7) / 8;
    const double table = (double)kN * t * V * (n + 1), inputs = (double)B * (kN + 1);
    pl.tile_major = table > inputs ? 1 : 0;
    hipLaunchKernelGGL(k, dim3(8 * pl.per), dim3(THREADS), lds, s, big, (const D*)dig, (const T*)c->d_ksk, out,
                       out_ptrs, (int)B, n, kN, t, bb, (int)c->ks_row, pl);
    return hip_check(c, hipGetLastError(), "launch keyswitch");
}

// Coefficients staged per barrier: with 32-bit words the largest of 8, 4, 2
// whose rows fit the staging registers and that divides kN (fewer barriers
// for short LWE tiles); with 64-bit words one, which measured faster.
template <typename T, typename D, int V, int WPW>
int launch_v(tfhe_ctx* c, const T* big, void* dig, T* out, const uint64_t* out_ptrs, uint32_t B, hipStream_t s) {
    const int kN = (int)(c->p.k * c->p.N), t = (int)c->p.ks_t;
    const int E = t * V * WPW;
    if (E > PMAX * THREADS) return ctx_fail(c, TFHE_EINVAL, "key-switching levels exceed the staging tile");
    if constexpr (sizeof(T) == 4) {
        if (8 * E <= PMAX * THREADS && kN % 8 == 0) return launch_p<T, D, V, WPW, 8>(c, big, dig, out, out_ptrs, B, s);
        if (4 * E <= PMAX * THREADS && kN % 4 == 0) return launch_p<T, D, V, WPW, 4>(c, big, dig, out, out_ptrs, B, s);
        if (2 * E <= PMAX * THREADS && kN % 2 == 0) return launch_p<T, D, V, WPW, 2>(c, big, dig, out, out_ptrs, B, s);
    }
    return launch_p<T, D, V, WPW, 1>(c, big, dig, out, out_ptrs, B, s);
}

// 16 words per lane.  For short LWE (n + 1 <= 128) 8 words per lane would
// waste fewer padded words in the last tile, but twice the tiles re-read the
// input and redo the digit extraction: at n = 64, 16 words measured 30%
// faster for 32768 ciphertexts and 3% slower for 4096.
template <typename T, int V>
int launch_w(tfhe_ctx* c, const void* big, void* dig, void* out, const uint64_t* out_ptrs, uint32_t B,
             hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        // the MFMA form: a lane's pairs of a chunk must span at most two rows i
        if (c->d_ksk8 && 16 / V <= (int)c->p.ks_t) {
            const uint32_t* b32 = (const uint32_t*)big;
            uint32_t* o32 = (uint32_t*)out;
            if (c->p.ks_t * c->p.ks_base_bits <= 16) return launch_mfma_ks<V, uint16_t, 1>(c, b32, dig, o32, out_ptrs, B, s);
            return launch_mfma_ks<V, uint32_t, 1>(c, b32, dig, o32, out_ptrs, B, s);
        }
    }
    if (c->p.ks_t * c->p.ks_base_bits <= 16)
        return launch_v<T, uint16_t, V, 16>(c, (const T*)big, dig, (T*)out, out_ptrs, B, s);
    return launch_v<T, uint32_t, V, 16>(c, (const T*)big, dig, (T*)out, out_ptrs, B, s);
}

template <typename T>
int launch_ks_t(tfhe_ctx* c, const void* big, void* dig, void* out, const uint64_t* out_ptrs, uint32_t B,
                hipStream_t s) {
    switch (c->p.ks_base_bits) {
        case 1: return launch_w<T, 2>(c, big, dig, out, out_ptrs, B, s);
        case 2: return launch_w<T, 4>(c, big, dig, out, out_ptrs, B, s);
        case 3: return launch_w<T, 8>(c, big, dig, out, out_ptrs, B, s);
        case 4: return launch_w<T, 16>(c, big, dig, out, out_ptrs, B, s);
        default: return ctx_fail(c, TFHE_EINVAL, "key-switching base must be 2^1..2^4");
    }
}

}  // namespace

size_t ks_digits_bytes(const tfhe_ctx* c, uint32_t B) {
    const size_t d = c->p.ks_t * c->p.ks_base_bits <= 16 ? 2 : 4;
    return ((size_t)B * c->p.k * c->p.N * d + 255) & ~(size_t)255;
}

int launch_keyswitch(tfhe_ctx* c, const void* big_in, void* out, const uint64_t* out_ptrs, uint32_t B, void* dig,
                     size_t dig_cap, hipStream_t s) {
    if (B == 0) return TFHE_OK;
    if (!dig || dig_cap < ks_digits_bytes(c, B)) return ctx_fail(c, TFHE_EINVAL, "key-switch digit buffer too small");
    TimedLaunch tl(c, s, 1, B);
    return c->q == 32 ? launch_ks_t<uint32_t>(c, big_in, dig, out, out_ptrs, B, s)
                      : launch_ks_t<uint64_t>(c, big_in, dig, out, out_ptrs, B, s);
}
