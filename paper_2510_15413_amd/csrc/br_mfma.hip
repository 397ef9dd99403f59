// Blind rotation + sample extraction with an exact limb-split int8 MFMA
// external product (gfx950, v_mfma_i32_16x16x64_i8).
//
// TFHE bootstrapping (ePrint 2018/421, Alg. 3 / Sec. 4): for i = 0..n-1,
//   ACC <- ACC + ExtProd(BSK_i, X^{abar_i} ACC - ACC),
// ExtProd(G, C)_v = sum_{u,p} Dec_p(C_u) * G[u*l+p-1][v] (negacyclic products).
//
// Mapping.  For one step and one (u, p, v), all ciphertexts of a batch share
// the key polynomial K = G[u*l+p-1][v], so the products of the batch are one
// matrix product Out[N x B] = T(K)[N x N] . D[N x B] with the negacyclic
// Toeplitz matrix T(K)[j][kk] = Kext[j - kk] (Kext[t] = K[t] for t >= 0 and
// -K[t+N] for t < 0) and D the digit matrix of the batch.  K is split into
// balanced int8 limbs, K = sum_m 2^{8m} K_m (mod 2^q); each limb product is
// exact in int32 (|limb| <= 128, |digit| <= Bg/2, N terms) and the sum
// sum_m 2^{8m} P_m is formed mod 2^q, so the result is bit-exact.
//
// Workgroup = 16 ciphertexts (the MFMA N dimension) for all n steps, 8 waves.
// Wave w owns output component v = w/4 and the row tiles J = (w%4) + 4a of
// 16 consecutive coefficients.  K chunks are 64 coefficients.  The A operand
// of tile (J, c) depends only on the diagonal c - a (Toeplitz), so one A
// fragment is loaded per diagonal and reused by every (a, c) on it.
// The key limbs of step i are stored (once per context) as reversed extended
// byte arrays S[x] = limb(Kext[N-1-x]); a lane's 16 A bytes are contiguous
// in S, unaligned by a per-lane constant.  At N = 1024 (32-bit words) the
// context also holds the 16 bytes at every offset of S in an aligned slot
// (the key windows) and each fragment is one 16-byte global load; otherwise
// the key is staged in LDS and a fragment is 5 words fixed with v_alignbyte,
// or for N <= 256 4 aligned words of one of four byte-shifted copies.
// Accumulators are laid out [v][N/4][16 cts][4 coefs].  With one row pass
// every wave keeps its rows in registers across the n steps and stores them
// at each step's end for the next rotate-diff: component 0 to LDS, component
// 1 to LDS too when both fit in 64 KB (small N), else parked in component
// 0's region during the step and in a per-workgroup global buffer at the
// end.  With several passes both components live in a global ping-pong
// buffer, and the first pass of a step caches its digits in global memory
// for the others.  Digits are formed into LDS.
#include <algorithm>

#include "fhesql_internal.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
constexpr int CTS = 16;
constexpr int THREADS = 512;
// N <= 256: each key slot holds four copies of the key bytes, copy j shifted
// down by j bytes, so that a lane reads its 16 A bytes as 4 aligned words of
// copy (b & 3) with no byte alignment on the critical path.  The 4 lanes of a
// row group that read one word of the single copy now read 4 copies; copy j
// starts KCOPY_PAD * j bytes further (24 words per copy), which puts the 32
// lanes of each half-wave on 32 distinct LDS banks.
constexpr int KCOPY_PAD = 96;

struct BrArgs {
    const void* lwe;          // [B][n+1] words
    const int8_t* bsk8;       // [n][2l][2][LIMBS][2N]
    const uint4* win;         // [n][2l][2][LIMBS][2N] 16-byte key windows, or null
    const void* tv;           // test polynomials [ntv][N] words
    const int32_t* tv_index;  // [B] or null
    void* out;                // [B][N+1] words
    void* ws;                 // accumulator buffers per workgroup (sized by acc_ws_bytes)
    int8_t* dcache;           // [grid][2l][N/64][1024] digit bytes (several row passes) or null
    int B, n, l, bg_bits;
};

template <typename T>
FHE_DEV size_t acc_idx(int N, int v, int j, int c) {
    return ((size_t)(v * (N >> 2) + (j >> 2)) * CTS + c) * 4 + (j & 3);
}

// Gadget digits of the rotate-diff X^{abar} ACC_u - ACC_u for 16 cts, written
// in the MFMA B-fragment layout: block (u*l+p, chunk) of 1 KB, lane (g,c) holds
// the 16 digits of coefficients 64*chunk + 16*g + 0..15 of ciphertext c.
// U components starting at u_lo, levels p_lo .. p_lo+p_n-1 of each: block
// (u-u_lo)*p_n + (p-p_lo).  One rotate-diff pass yields all levels formed.
// A work item is 4 consecutive coefficients of one ciphertext: its own 4
// words are one 16-byte group of the accumulator layout and the 4 rotated
// words straddle at most two such groups, so an item takes three vector
// loads; the loads of G items are issued together.  With GC the packed
// digits are also written to gdst at the same offsets (the digit cache).
// With DS > 1 the caller forms slice `ds` of DS equal slices of the items
// (the multi-workgroup blind rotation spreads one group's digits over DS
// workgroups).
// With acopy the item's own accumulator words are also copied there (same
// layout), which seeds the next accumulator of the multi-workgroup path.
// TH: threads that share the work (the first TH of the workgroup, or with
// TH = THREADS / 2 either half, each half forming its own slice).
template <typename T, int R, int U, bool GC = false, int DS = 1, bool AC = false, int TH = THREADS>
FHE_DEV void digits_phase(const T* __restrict__ src, int ab, int8_t* dbuf, int u_lo, int p_lo, int p_n, int l,
                          int bgb, int8_t* gdst = nullptr, int ds = 0, T* acopy = nullptr) {
    typedef T vec4 __attribute__((ext_vector_type(4)));
    constexpr int N = R * 64;
    constexpr int NG = N / 4;  // 4-word groups per component
    constexpr int ITEMS = CTS * U * NG / DS;
    static_assert((CTS * U * NG) % (DS * CTS) == 0, "digit slices must hold whole groups of 16 items");
    static_assert(THREADS % TH == 0 && TH % CTS == 0, "thread subsets must hold whole ciphertext groups");
    const int it0 = ds * ITEMS;
    constexpr int IPT = (ITEMS + TH - 1) / TH;
    constexpr int G = IPT < 4 ? IPT : 4;
    constexpr int Q = Torus<T>::Q;
    // Level p of the balanced decomposition of x is field p of
    // y = round_top(x, l*bgb) + off, minus half (off = half at every level).
    // With F = off << shr (shr = Q - l*bgb >= 1, as l*bgb <= 31), the word
    // z = (x + 2^(shr-1) + F) ^ F holds field p of y with its top bit flipped
    // at bit shr + (l-1-p)*bgb, and that field read as a signed bgb-bit
    // number is the digit (t ^ half = t - half mod 2^bgb, sign in the top bit).
    const int shr = Q - l * bgb;
    const int half = 1 << (bgb - 1);
    uint32_t off = 0;
    for (int p = 0; p < l; p++) off += (uint32_t)half << (p * bgb);
    const T F = (T)off << shr;
    const T C = ((T)1 << (shr - 1)) + F;
    // the fields sit in the word's low half at q = 32, in its high half at q = 64
    const int fb = Q == 32 ? shr : shr - 32;
    // the item addresses below do not change from step to step; an opaque
    // thread index keeps them from being hoisted out of the caller's step
    // loop (held there they would crowd out the MFMA phase's registers)
    int tix = TH == THREADS ? (int)threadIdx.x : (int)(threadIdx.x & (TH - 1));
    __asm__ volatile("" : "+v"(tix));
    const int c = tix & (CTS - 1);  // fixed per thread (TH % 16 == 0); ab is its abar_i
    const int neg = ab >= N;
    const int es = neg ? ab - N : ab;
    // coefficient 4kg+e reads rotated index 4kg+e-es: group kg-qs (+1), word e+sh
    const int sh = (4 - (es & 3)) & 3;
    const int qs = (es + 3) >> 2;  // 4kg - es = 4(kg - qs) + sh
    const bool s1 = (sh & 1) != 0, s2 = (sh & 2) != 0;
    // word e+sh lies in the second group for e = 1 (sh = 3), 2 (sh >= 2), 3 (sh >= 1)
    const bool hi1 = sh == 3, hi2 = s2, hi3 = sh != 0;
    // all ones when the rotation exponent is at least N (X^N = -1)
    const T negm = neg ? ~(T)0 : (T)0;
    // item it = tix + k*TH covers group (it0 + it) >> 4 of the U
    // components (all unsigned, so that the divisions are shifts)
    const unsigned rest0 = ((unsigned)it0 + (unsigned)tix) >> 4;
    constexpr unsigned RSTEP = TH / CTS;
    const vec4* Pc = (const vec4*)src + c;
    for (int k0 = 0; k0 < IPT; k0 += G) {
        vec4 dv[G], r0[G], r1[G];
        int kq[G];
#pragma unroll
        for (int k = 0; k < G; k++) {
            if (ITEMS % TH != 0 && (unsigned)tix + (unsigned)(k0 + k) * TH >= (unsigned)ITEMS) continue;
            const unsigned rest = rest0 + (unsigned)(k0 + k) * RSTEP;
            const unsigned kg = rest & (NG - 1);
            const unsigned ub = (U == 1 ? 0u : rest / NG) + (unsigned)u_lo;
            const vec4* P = Pc + (size_t)ub * NG * CTS;
            const int q0 = (int)kg - qs;
            kq[k] = q0;
            dv[k] = P[kg * CTS];
            if (AC) ((vec4*)acopy + c + (size_t)ub * NG * CTS)[kg * CTS] = dv[k];
            r0[k] = P[(unsigned)(q0 & (NG - 1)) * CTS];
            r1[k] = P[(unsigned)((q0 + 1) & (NG - 1)) * CTS];
        }
#pragma unroll
        for (int k = 0; k < G; k++) {
            if (ITEMS % TH != 0 && (unsigned)tix + (unsigned)(k0 + k) * TH >= (unsigned)ITEMS) continue;
            const unsigned rest = rest0 + (unsigned)(k0 + k) * RSTEP;
            const int kg = (int)(rest & (NG - 1));
            const int u = (U == 1 ? 0 : (int)(rest / NG)) + u_lo;
            // negacyclic sign as a mask (all ones: negate): a group below
            // zero wraps with a sign flip, on top of the exponent's
            const T m0 = (T)(int64_t)(kq[k] >> 31) ^ negm;
            const T m1 = (T)(int64_t)((kq[k] + 1) >> 31) ^ negm;
            // word e+sh of the 7 words r0[0..3], r1[0..2]: two selects by the
            // bits of sh (named values, not an array: an indexed array would
            // be placed in scratch memory)
            const T q0w = s1 ? r0[k][1] : r0[k][0], q1w = s1 ? r0[k][2] : r0[k][1];
            const T q2w = s1 ? r0[k][3] : r0[k][2], q3w = s1 ? r1[k][0] : r0[k][3];
            const T q4w = s1 ? r1[k][1] : r1[k][0], q5w = s1 ? r1[k][2] : r1[k][1];
            const T v0 = s2 ? q2w : q0w, v1 = s2 ? q3w : q1w, v2 = s2 ? q4w : q2w, v3 = s2 ? q5w : q3w;
            // (v ^ m) - m is v or -v
            auto field_word = [&](T v, T m, T d) -> uint32_t {
                const T z = (T)(((T)(C - d) + (T)((T)(v ^ m) - m)) ^ F);
                return Q == 32 ? (uint32_t)z : (uint32_t)((uint64_t)z >> 32);
            };
            uint32_t zz[4];
            zz[0] = field_word(v0, m0, dv[k][0]);
            zz[1] = field_word(v1, hi1 ? m1 : m0, dv[k][1]);
            zz[2] = field_word(v2, hi2 ? m1 : m0, dv[k][2]);
            zz[3] = field_word(v3, hi3 ? m1 : m0, dv[k][3]);
            // coefficients 4kg..4kg+3: chunk kg/16, lane group (kg/4)%4, bytes 4(kg%4)..
            const unsigned ukg = (unsigned)kg;
            const unsigned obase = (ukg >> 4) * 1024u + ((ukg >> 2) & 3u) * 256u + (unsigned)c * 16u + (ukg & 3u) * 4u +
                                   (unsigned)((u - u_lo) * p_n) * (unsigned)(R * 1024);
            for (int p = p_lo; p < p_lo + p_n; p++) {
                const int pos = fb + (l - 1 - p) * bgb;
                const int d0 = __builtin_amdgcn_sbfe((int)zz[0], pos, bgb);
                const int d1 = __builtin_amdgcn_sbfe((int)zz[1], pos, bgb);
                const int d2 = __builtin_amdgcn_sbfe((int)zz[2], pos, bgb);
                const int d3 = __builtin_amdgcn_sbfe((int)zz[3], pos, bgb);
                // low bytes of the four digits, coefficient e in byte e
                const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)d1, (uint32_t)d0, 0x0C0C0400u);
                const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)d3, (uint32_t)d2, 0x0C0C0400u);
                const uint32_t packed = p01 | (p23 << 16);
                const unsigned o = obase + (unsigned)(p - p_lo) * (unsigned)(R * 1024);
                *(uint32_t*)(dbuf + o) = packed;
                if (GC) *(uint32_t*)(gdst + o) = packed;
            }
        }
    }
}

struct ARaw {
    uint32_t w[5];
};

// The 5 words at p covering a lane's 16 A bytes (which start sh bytes into
// the first), or with shifted copies (KC = 4) the 4 words of the fragment.
template <int KC>
FHE_DEV ARaw afrag_raw(const uint8_t* p) {
    const uint32_t* w = (const uint32_t*)p;
    ARaw r;
#pragma unroll
    for (int k = 0; k < (KC == 4 ? 4 : 5); k++) r.w[k] = w[k];
    return r;
}

template <int KC>
FHE_DEV v4i afrag_combine(const ARaw& r, int sh) {
    v4i a;
    if (KC == 4) {
        a[0] = (int)r.w[0];
        a[1] = (int)r.w[1];
        a[2] = (int)r.w[2];
        a[3] = (int)r.w[3];
        return a;
    }
    a[0] = (int)__builtin_amdgcn_alignbyte(r.w[1], r.w[0], sh);
    a[1] = (int)__builtin_amdgcn_alignbyte(r.w[2], r.w[1], sh);
    a[2] = (int)__builtin_amdgcn_alignbyte(r.w[3], r.w[2], sh);
    a[3] = (int)__builtin_amdgcn_alignbyte(r.w[4], r.w[3], sh);
    return a;
}

// Small rings (N <= 256, 32-bit words, the step-keyed schedule): a limb's diagonal
// iteration is only RP <= 4 MFMAs, shorter than an LDS read, so the limbs
// are unrolled and each fragment of limb m+1 is requested as soon as
// limb m's iteration that uses it has issued its MFMAs (every diagonal
// fragment serves one iteration), a limb ahead of its use, leaving no LDS
// wait inside a limb and holding one set of 2RP-1 fragments.
template <typename T, int R, int KC>
FHE_DEV void mfma_block_small(const uint8_t* kslot, const int8_t* dblk, int v, int jr, T (&delta)[R][4]) {
    constexpr int N = R * 64;
    constexpr int NL = Torus<T>::LIMBS;
    constexpr int CP = R;
    constexpr int NF = 2 * CP - 1;                                 // diagonals -(CP-1) .. CP-1
    constexpr int KCS = 2 * NL * 2 * N + KCOPY_PAD;                // copy stride
    static_assert(KC == 4 && NL == 4, "small-ring block: four shifted key copies, 32-bit words");
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    const int sh0 = ((N - 1) - 16 * jr - r + 16 * g) & 3;
    // fragment k (diagonal k - (CP-1)) of limb m at byte 2N m + 64 k of this
    // lane's copy past the base, which is moved down by 64 (CP-1) so that
    // every offset is a positive immediate (it stays inside LDS: the key
    // slot follows the digit buffer)
    int sbo = (N - 1) - 16 * jr - r + 16 * g - sh0 - 64 * (CP - 1);
    __asm__ volatile("" : "+v"(sbo));
    const uint8_t* S0 = kslot + (size_t)sh0 * KCS + (size_t)v * NL * (2 * N) + sbo;
    v4i bf[CP];
#pragma unroll
    for (int cc = 0; cc < CP; cc++) bf[cc] = *(const v4i*)(dblk + (size_t)cc * 1024 + lane * 16);
    ARaw F[NF];
#pragma unroll
    for (int k = 0; k < NF; k++) F[k] = afrag_raw<4>(S0 + 64 * k);
#pragma unroll
    for (int m = 0; m < NL; m++) {
        if (m == 0) __builtin_amdgcn_s_setprio(3);
        else if (m == 1) __builtin_amdgcn_s_setprio(2);
        else if (m == 2) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        v4i acc[CP];
#pragma unroll
        for (int s = 0; s < CP; s++) {
            // iteration s: MFMA (a, c = (a+s) mod CP) on diagonal c - a, which
            // is s (fragment s + CP - 1) or s - CP (fragment s - 1)
#pragma unroll
            for (int a = 0; a < CP; a++) {
                const int k = a + s < CP ? s + CP - 1 : s - 1;
                const v4i A = afrag_combine<4>(F[k], 0);
                acc[a] = s == 0 ? __builtin_amdgcn_mfma_i32_16x16x64_i8(A, bf[(a + s) % CP], v4i{0, 0, 0, 0}, 0, 0, 0)
                                : __builtin_amdgcn_mfma_i32_16x16x64_i8(A, bf[(a + s) % CP], acc[a], 0, 0, 0);
            }
            if (m + 1 < NL) {
                const uint8_t* Sn = S0 + (size_t)(m + 1) * (2 * N);
                F[s + CP - 1] = afrag_raw<4>(Sn + 64 * (s + CP - 1));
                if (s > 0) F[s - 1] = afrag_raw<4>(Sn + 64 * (s - 1));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int a = 0; a < CP; a++)
#pragma unroll
            for (int e = 0; e < 4; e++) delta[a][e] += (T)((T)(int64_t)acc[a][e] << (8 * m));
    }
    __builtin_amdgcn_s_setprio(0);
}

// Windowed key (N = 1024, 32-bit words, one row pass): every A fragment is
// one 16-byte-aligned global load.  The window array holds, for every limb
// of every key polynomial and every byte offset x of its reversed extended
// byte array S, the 16 bytes S[x .. x+15] at 16-byte slot x, so lane (r, g)
// of a wave finds its fragment of diagonal d at slot x0 + 64 d and the 64
// lanes of a wave read one contiguous kilobyte.  No key is staged in LDS,
// no byte alignment is done, and consecutive blocks need no barrier.  The
// fragments of iteration t (limb t / CP, diagonal pair t % CP) are requested
// two iterations ahead through a ring of 4 register slots, carried across
// blocks by the caller (wnext is the block that runs next, whose first two
// iterations the last ones request).
template <typename T, int R>
FHE_DEV void mfma_block_wk(const uint4* __restrict__ wblk, const uint4* __restrict__ wnext, const int8_t* dblk,
                           int v, int jr, T (&delta)[R][4], v4i (&F0)[4], v4i (&F1)[4]) {
    constexpr int N = R * 64;
    constexpr int NL = Torus<T>::LIMBS;
    constexpr int CP = R;
    constexpr int IT = NL * CP;  // iterations per block
    static_assert(CP == 16 && NL == 4, "windowed key: 16 chunks, four limbs");
    const int lane = threadIdx.x & 63;
    v4i bf[CP];
#pragma unroll
    for (int cc = 0; cc < CP; cc++) bf[cc] = *(const v4i*)(dblk + (size_t)cc * 1024 + lane * 16);
#pragma unroll
    for (int m = 0; m < NL; m++) {
        if (m == 0) __builtin_amdgcn_s_setprio(3);
        else if (m == 1) __builtin_amdgcn_s_setprio(2);
        else if (m == 2) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        v4i acc[CP];
#pragma unroll
        for (int s = 0; s < CP; s++) {
            const int t = m * CP + s;
            {
                // request iteration t + 2 (of the next block past the end)
                const int tn = (t + 2) % IT;
                const uint4* b = (t + 2 < IT ? wblk : wnext) + (size_t)(tn / CP) * (2 * N);
                const int sn = tn % CP;
                F0[(t + 2) & 3] = __builtin_bit_cast(v4i, b[64 * sn]);
                if (sn > 0) F1[(t + 2) & 3] = __builtin_bit_cast(v4i, b[64 * (sn - CP)]);
            }
#pragma unroll
            for (int a = 0; a < CP; a++) {
                const v4i A = a + s < CP ? F0[t & 3] : F1[t & 3];
                acc[a] = s == 0 ? __builtin_amdgcn_mfma_i32_16x16x64_i8(A, bf[(a + s) % CP], v4i{0, 0, 0, 0}, 0, 0, 0)
                                : __builtin_amdgcn_mfma_i32_16x16x64_i8(A, bf[(a + s) % CP], acc[a], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int a = 0; a < CP; a++)
#pragma unroll
            for (int e = 0; e < 4; e++) delta[a][e] += (T)((T)(int64_t)acc[a][e] << (8 * m));
    }
    __builtin_amdgcn_s_setprio(0);
}

// One (u,p) key block for this wave: all limbs, the pass's RP row tiles.
// KC = 4: the slot holds four copies of the key bytes, copy j shifted down by
// j bytes, so a lane reads its 16 bytes as 4 aligned words of copy (b & 3).
template <typename T, int R, int RP, int KC>
FHE_DEV void mfma_block(const uint8_t* kslot, const int8_t* dblk, int v, int jr, int pass,
                        T (&delta)[RP][4]) {
    constexpr int N = R * 64;
    constexpr int NL = Torus<T>::LIMBS;
    constexpr int CP = R < 16 ? R : 16;
    constexpr int KCS = 2 * NL * 2 * N + (KC == 4 ? KCOPY_PAD : 0);  // copy stride
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    const int sh0 = ((N - 1) - 16 * jr - r + 16 * g) & 3;
    const int lanebase = (N - 1) - 16 * jr - r + 16 * g - (KC == 4 ? sh0 : 0);
    const int sh = KC == 4 ? 0 : sh0;
    for (int cg = 0; cg < R / CP; cg++) {
        v4i bf[CP];
#pragma unroll
        for (int cc = 0; cc < CP; cc++)
            bf[cc] = *(const v4i*)(dblk + (size_t)(cg * CP + cc) * 1024 + lane * 16);
        // one limb: its MFMA products for this block in acc[] (int32, exact)
        auto limb = [&](int m, v4i(&acc)[RP]) {
            // Issue priority falls limb by limb, so of the two waves sharing a
            // SIMD the one further along yields to the other (at equal
            // priority the older wave wins, and the younger one would finish
            // the block alone, leaving gaps in the matrix pipe).
            if (m == 0) __builtin_amdgcn_s_setprio(3);
            else if (m == 1) __builtin_amdgcn_s_setprio(2);
            else if (m == 2) __builtin_amdgcn_s_setprio(1);
            else __builtin_amdgcn_s_setprio(0);
            const uint8_t* S = kslot + (KC == 4 ? (size_t)sh0 * KCS : 0) + (size_t)(v * NL + m) * (2 * N);
#pragma unroll
            for (int a = 0; a < RP; a++) acc[a] = v4i{0, 0, 0, 0};
            // Diagonals d = c - a (local) in wrapped pairs: iteration s takes
            // d = s for a <= CP-1-s and d = s - CP for the other a, so every
            // iteration issues RP independent MFMAs (one per accumulator).
            // The raw LDS loads of iteration s+1 are issued before the MFMAs
            // of iteration s and combined after them.  The fragment of
            // diagonal d starts at byte db + 64 d, d in (-CP, CP); the base is
            // moved down by 64 (CP-1) bytes so that every word offset is a
            // positive immediate (it stays inside LDS: the key slot lies
            // after the digit buffer, which is at least 1 KB per chunk).
            const int db = lanebase + 64 * (cg * CP - pass * RP);
            int sbo = (db & ~3) - 64 * (CP - 1);
            __asm__ volatile("" : "+v"(sbo));  // keep the rebased offset as the base
            const uint8_t* Sb = S + sbo;
            ARaw r0 = afrag_raw<KC>(Sb + 64 * (CP - 1)), r1;
            v4i A0 = afrag_combine<KC>(r0, sh), A1 = A0;
#pragma unroll
            for (int s = 0; s < CP; s++) {
                const bool wrap_next = s + 1 >= CP - RP + 1;
                if (s + 1 < CP) {
                    r0 = afrag_raw<KC>(Sb + 64 * (s + CP));
                    if (wrap_next) r1 = afrag_raw<KC>(Sb + 64 * s);
                }
#pragma unroll
                for (int a = 0; a < RP; a++) {
                    if (a + s < CP)
                        acc[a] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A0, bf[a + s], acc[a], 0, 0, 0);
                    else
                        acc[a] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A1, bf[a + s - CP], acc[a], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
                if (s + 1 < CP) {
                    A0 = afrag_combine<KC>(r0, sh);
                    if (wrap_next) A1 = afrag_combine<KC>(r1, sh);
                }
            }
        };
        // limbs whose shifted product has a nonzero low word: full fold
#pragma unroll 1
        for (int m = 0; m < (NL < 4 ? NL : 4); m++) {
            v4i acc[RP];
            limb(m, acc);
#pragma unroll
            for (int a = 0; a < RP; a++)
#pragma unroll
                for (int e = 0; e < 4; e++)
                    delta[a][e] += (T)((T)(int64_t)acc[a][e] << (8 * m));
        }
        if constexpr (NL > 4) {
            // q = 64, limbs 4..7: the shifted product has a zero low word, so
            // only the low 32 bits of the limb sum reach the high word
#pragma unroll 1
            for (int m = 4; m < NL; m++) {
                v4i acc[RP];
                limb(m, acc);
#pragma unroll
                for (int a = 0; a < RP; a++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
                        u32x2 w = __builtin_bit_cast(u32x2, delta[a][e]);
                        w.y += (uint32_t)acc[a][e] << (8 * m - 32);
                        delta[a][e] = __builtin_bit_cast(T, w);
                    }
            }
        }
    }
    __builtin_amdgcn_s_setprio(0);
}

// DG: digit blocks formed per rotate-diff pass -- 0 all (k+1)l blocks of a
// step up front (key double-buffered), -1 the l blocks of one component
// before that component's MFMA blocks with accumulator component 0 held in
// LDS (key double-buffered), -2 (both components in LDS, small N) the
// step-keyed schedule described at its loop, else DG consecutive levels of
// one component just before their MFMA blocks.
template <typename T, int R, int RP, int DG>
__global__ __launch_bounds__(THREADS, 1) __attribute__((amdgpu_waves_per_eu(2, 2))) void br_mfma_kernel(BrArgs a) {
    constexpr int N = R * 64;
    constexpr int NL = Torus<T>::LIMBS;
    constexpr int KSLOT = 2 * NL * 2 * N;  // bytes of one (u,p) key block
    constexpr int KV = (KSLOT / 16 + THREADS - 1) / THREADS;
    constexpr int KC = R <= 4 ? 4 : 1;   // shifted key copies per slot
    constexpr int KCS = KSLOT + (KC == 4 ? KCOPY_PAD : 0);  // copy stride
    constexpr int LG = __builtin_ctz(2 * N);
    constexpr bool ACCL = DG < 0;
    constexpr bool SK = DG == -2;    // all key blocks of a step staged together
    constexpr bool WK = DG == -3;    // key fragments loaded from the global window array
    constexpr bool DALL = DG <= 0;   // a step's digits formed before its blocks run
    constexpr bool DOUBLE = DALL && !SK && !WK;
    constexpr int NPASS = R / RP;
    static_assert(!ACCL || NPASS == 1, "LDS accumulator mode needs one row pass");
    // small N: accumulator component 1 in LDS as well (right after component 0)
    constexpr bool ACC1L = ACCL && 2 * N * CTS * (int)sizeof(T) <= 65536;
    static_assert(!SK || ACC1L, "the step-keyed schedule keeps both components in LDS");
    // Several row passes with digits formed per group: the first pass also
    // writes each group's digits to a per-workgroup global cache (L2
    // resident) and the later passes of the step copy them back to LDS.
    constexpr bool DCACHE = !DALL && NPASS > 1;
    constexpr int DCU = (DALL ? 1 : DG) * R * 64;  // uint4 per digit group
    constexpr int DCV = (DCU + THREADS - 1) / THREADS;
    const int n = a.n, l = a.l, NB = 2 * l;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ct0 = blockIdx.x * CTS;
    const T* lwe = (const T*)a.lwe;

    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    int8_t* dbuf = (int8_t*)smem;
    size_t off = (size_t)(SK || WK ? NB : ACCL ? l : DALL ? NB : DG) * R * 1024;
    uint8_t* kbuf = smem + off;
    off += (size_t)(SK ? NB : WK ? 0 : DOUBLE ? 2 : 1) * KC * KCS;
    T* acc0 = (T*)(smem + off);  // ACCL: accumulator component 0, [N/4][16 cts][4]

    // With all digits of a step formed before its blocks (DALL) the
    // accumulator is updated in place; otherwise two buffers alternate.
    // With component 0 in LDS (ACCL) only the component-1 half of a
    // workgroup's slot is used; the slot keeps its full 2N*CTS-word stride,
    // which measured about 1% faster at the standard set than packing the
    // component-1 halves (and moved a tenth of the HBM bytes).
    T* ws0 = (T*)a.ws + (size_t)blockIdx.x * (DALL ? 1 : 2) * (2 * N * CTS);
    T* ws1 = DALL ? ws0 : ws0 + 2 * N * CTS;
    T* const acc1 = (ACC1L ? acc0 : ws0) + (size_t)N * CTS;  // ACCL: component 1 (LDS or global)

    // this thread's ciphertext in the digit phases and its abar_i, one step ahead
    const int cd = tid & (CTS - 1);
    const T* lwe_cd = lwe + (size_t)(ct0 + cd < a.B ? ct0 + cd : 0) * (n + 1);
    const bool cd_live = ct0 + cd < a.B;
    T a_next = cd_live ? lwe_cd[0] : (T)0;  // raw a_{i+1}; switched when used

    // ---- prologue: accumulator = (0, X^{-bbar} testv)
    for (int idx = tid; idx < CTS * N; idx += THREADS) {
        const int c = idx & (CTS - 1), j = idx >> 4;
        const int gi = ct0 + c;
        T body = 0;
        if (gi < a.B) {
            const int bb = (int)mod_switch<T>(lwe[(size_t)gi * (n + 1) + n], LG);
            const int e = (2 * N - bb) & (2 * N - 1);
            const T* tv = (const T*)a.tv + (size_t)(a.tv_index ? a.tv_index[gi] : 0) * N;
            body = monomial_coef<T>([&](int s) -> T { return tv[s]; }, N, e, j);
        }
        if (ACCL) acc0[acc_idx<T>(N, 0, j, c)] = 0;
        else ws0[acc_idx<T>(N, 0, j, c)] = 0;
        (ACC1L ? acc0 : ws0)[acc_idx<T>(N, 1, j, c)] = body;
    }

    const int v = wave >> 2, jr = wave & 3;
    constexpr int KU = KSLOT / 16;  // uint4 per key block
    uint4 pre[KV];
    uint32_t pnx[KV];  // KC = 4: the word after each uint4
#define KEY_LOAD(SRCPTR)                                                   \
    do {                                                                   \
        const uint4* ks_ = (SRCPTR);                                       \
        _Pragma("unroll") for (int q_ = 0; q_ < KV; q_++) {                \
            const int idx_ = tid + q_ * THREADS;                           \
            pre[q_] = (KU % THREADS == 0 || idx_ < KU) ? ks_[idx_ < KU ? idx_ : 0] : make_uint4(0, 0, 0, 0); \
            if (KC == 4) pnx[q_] = idx_ + 1 < KU ? *(const uint32_t*)(ks_ + idx_ + 1) : 0u; \
        }                                                                  \
    } while (0)
#define KEY_STORE(DSTPTR)                                                  \
    do {                                                                   \
        uint4* kd_ = (uint4*)(DSTPTR);                                     \
        _Pragma("unroll") for (int q_ = 0; q_ < KV; q_++) {                \
            const int idx_ = tid + q_ * THREADS;                           \
            if (KU % THREADS == 0 || idx_ < KU) {                          \
                kd_[idx_] = pre[q_];                                       \
                if (KC == 4) {                                             \
                    const uint4 w_ = pre[q_];                              \
                    _Pragma("unroll") for (int j_ = 1; j_ < 4; j_++)       \
                        kd_[j_ * (KCS / 16) + idx_] = make_uint4(          \
                            __builtin_amdgcn_alignbyte(w_.y, w_.x, j_),    \
                            __builtin_amdgcn_alignbyte(w_.z, w_.y, j_),    \
                            __builtin_amdgcn_alignbyte(w_.w, w_.z, j_),    \
                            __builtin_amdgcn_alignbyte(pnx[q_], w_.w, j_)); \
                }                                                          \
            }                                                              \
        }                                                                  \
    } while (0)
    const uint4* kbase = (const uint4*)a.bsk8;
    if (DOUBLE) {
        KEY_LOAD(kbase);
        KEY_STORE(kbuf);
    }
    // SK: the l key blocks of one component (half h of a step), staged
    // through registers, thread idx taking uint4 idx of the half (up to l = 4)
    constexpr int KVH = SK ? (4 * KU + THREADS - 1) / THREADS : 1;
    uint4 hk[KVH];
    uint32_t hn[KVH];  // KC = 4: the word after each uint4 (0 at a block's end)
    auto key_load_half = [&](int step, int h) {
        const uint4* ks = kbase + ((size_t)step * NB + (size_t)h * l) * KU;
#pragma unroll
        for (int q = 0; q < KVH; q++) {
            const int idx = tid + q * THREADS;
            if (idx < l * KU) {
                hk[q] = ks[idx];
                if (KC == 4) hn[q] = (idx % KU) + 1 < KU ? *(const uint32_t*)(ks + idx + 1) : 0u;
            }
        }
    };
    auto key_store_half = [&](int h) {
#pragma unroll
        for (int q = 0; q < KVH; q++) {
            const int idx = tid + q * THREADS;
            if (idx < l * KU) {
                const int w = idx % KU;
                uint4* kd = (uint4*)(kbuf + (size_t)(h * l + idx / KU) * KC * KCS);
                kd[w] = hk[q];
                if (KC == 4) {
                    const uint4 x = hk[q];
#pragma unroll
                    for (int j = 1; j < 4; j++)
                        kd[j * (KCS / 16) + w] = make_uint4(__builtin_amdgcn_alignbyte(x.y, x.x, j),
                                                            __builtin_amdgcn_alignbyte(x.z, x.y, j),
                                                            __builtin_amdgcn_alignbyte(x.w, x.z, j),
                                                            __builtin_amdgcn_alignbyte(hn[q], x.w, j));
                }
            }
        }
    };
    if constexpr (SK) {
        key_load_half(0, 0);
        key_store_half(0);
        key_load_half(0, 1);
        key_store_half(1);
    }
    __syncthreads();

    T* src = ws0;
    T* dst = ws1;
    int t = 0;  // linear key-block counter over (i, pass, ub)
    // With one pass and in-place accumulators each wave keeps its own rows
    // in registers across steps (the fold accumulates straight into them) and
    // only stores them for the next step's digit phases.
    constexpr bool REGACC = DALL && NPASS == 1;
    typedef T vec4 __attribute__((ext_vector_type(4)));
    constexpr size_t STEP4 = (size_t)(64 / 4) * CTS * 4;  // 4 row tiles further
    const size_t rbase = acc_idx<T>(N, v, 16 * jr + 4 * (lane >> 4), lane & 15);
    // this wave's rows live in LDS (accumulator components held there) or in
    // the global buffer; the branch is wave-uniform and keeps each access
    // in its own address space (a selected pointer would be a flat access)
    const bool rows_lds = ACCL && (v == 0 || ACC1L);
    // ACCL without room for component 1 in LDS: component 0's LDS region is
    // dead from the end of its digit phase to the end of the step, so the
    // component-1 waves park their rows there for the component-1 digit
    // phase (no global round trip); they reach global memory only at the end
    constexpr bool PARK = ACCL && !ACC1L && REGACC;
    const size_t rbase0 = rbase - (size_t)v * N * CTS;  // the same rows in component 0's layout
    T accr[REGACC ? RP : 1][4];
    if (REGACC) {
        auto get = [&](const T* base) {
#pragma unroll
            for (int q = 0; q < (REGACC ? RP : 1); q++) {
                const vec4 x = *(const vec4*)(base + rbase + q * STEP4);
#pragma unroll
                for (int e = 0; e < 4; e++) accr[q][e] = x[e];
            }
        };
        if (rows_lds) get(acc0);
        else get(ws0);
    }
    // Step-keyed schedule (SK): three barriers per step.  The digits of
    // component 0 are formed first; the digits of component 1 are formed
    // while component 0's blocks run (the v = 0 waves before their blocks,
    // the v = 1 waves after theirs, so that on each SIMD one wave's digit
    // work meets the other's MFMAs), into their own l blocks of the digit
    // buffer.  The key area holds all 2l blocks of a step; the next step's
    // component-0 half is stored once this step's component-0 blocks are
    // done (after the second barrier), its component-1 half at the start of
    // the next step (its blocks start after that step's second barrier).
    if constexpr (SK) {
        int8_t* dbuf1 = dbuf + (size_t)l * R * 1024;
        auto block = [&](int ub) {
            const uint8_t* ks = kbuf + (size_t)ub * KC * KCS;
            const int8_t* db = dbuf + (size_t)ub * R * 1024;
            if constexpr (KC == 4 && NL == 4) mfma_block_small<T, R, KC>(ks, db, v, jr, accr);
            else mfma_block<T, R, RP, KC>(ks, db, v, jr, 0, accr);
        };
        for (int i = 0; i < n; i++) {
            const int ab = cd_live ? (int)mod_switch<T>(a_next, LG) : 0;
            if (i + 1 < n) a_next = lwe_cd[i + 1];
            if (i > 0) key_store_half(1);
            digits_phase<T, R, 1>(acc0, ab, dbuf, 0, 0, l, l, a.bg_bits);
            if (i + 1 < n) key_load_half(i + 1, 0);
            __syncthreads();
            if (v == 0) digits_phase<T, R, 1, false, 2, false, THREADS / 2>(acc1, ab, dbuf1, 0, 0, l, l, a.bg_bits,
                                                                            nullptr, 0);
            for (int ub = 0; ub < l; ub++) block(ub);
            if (v == 1) digits_phase<T, R, 1, false, 2, false, THREADS / 2>(acc1, ab, dbuf1, 0, 0, l, l, a.bg_bits,
                                                                            nullptr, 1);
            __syncthreads();
            if (i + 1 < n) {
                key_store_half(0);
                key_load_half(i + 1, 1);
            }
            for (int ub = l; ub < NB; ub++) block(ub);
            uint32_t ro = (uint32_t)rbase;
            __asm__ volatile("" : "+v"(ro));
#pragma unroll
            for (int q = 0; q < RP; q++) {
                vec4 o;
#pragma unroll
                for (int e = 0; e < 4; e++) o[e] = accr[q][e];
                *(vec4*)(acc0 + ro + q * STEP4) = o;
            }
            __syncthreads();
        }
    }
    // Windowed-key schedule (WK): the key blocks of a step run back to back
    // (the key is read from the window array, not staged); four barriers per
    // step: after component 0's digits, after parking component 1's rows,
    // between the components' blocks and at the step end.
    if constexpr (WK) {
        v4i F0[4], F1[4];  // fragment ring of mfma_block_wk
        constexpr size_t BLK = (size_t)2 * NL * 2 * N;  // windows per (u,p) block
        const size_t vo = (size_t)v * NL * 2 * N + (size_t)((N - 1) - 16 * jr - (lane & 15) + 16 * (lane >> 4));
        auto wbase = [&](int i, int ub) { return a.win + ((size_t)i * NB + ub) * BLK + vo; };
        {
            const uint4* b = wbase(0, 0);
            F0[0] = __builtin_bit_cast(v4i, b[0]);
            F0[1] = __builtin_bit_cast(v4i, b[64]);
            F1[1] = __builtin_bit_cast(v4i, b[64 * (1 - 16)]);
        }
        for (int i = 0; i < n; i++) {
            const int ab = cd_live ? (int)mod_switch<T>(a_next, LG) : 0;
            if (i + 1 < n) a_next = lwe_cd[i + 1];
            digits_phase<T, R, 1>(acc0, ab, dbuf, 0, 0, l, l, a.bg_bits);
            __syncthreads();
            if constexpr (PARK) if (v == 1) {
                // this step's component-1 input rows (no fold has touched them yet)
                uint32_t ro = (uint32_t)rbase0;
                __asm__ volatile("" : "+v"(ro));
#pragma unroll
                for (int q = 0; q < RP; q++) {
                    vec4 o;
#pragma unroll
                    for (int e = 0; e < 4; e++) o[e] = accr[q][e];
                    *(vec4*)(acc0 + ro + q * STEP4) = o;
                }
            }
            __syncthreads();
            // component 1's digits are formed into their own l blocks while
            // component 0's blocks run: the v = 0 waves before their blocks,
            // the v = 1 waves after theirs (one of each per SIMD)
            int8_t* dbuf1 = dbuf + (size_t)l * R * 1024;
            const T* rows1 = PARK ? acc0 : acc1;
            if (v == 0) digits_phase<T, R, 1, false, 2, false, THREADS / 2>(rows1, ab, dbuf1, 0, 0, l, l, a.bg_bits,
                                                                            nullptr, 0);
            for (int ub = 0; ub < NB; ub++) {
                if (ub == l) {
                    if (v == 1) digits_phase<T, R, 1, false, 2, false, THREADS / 2>(rows1, ab, dbuf1, 0, 0, l, l,
                                                                                    a.bg_bits, nullptr, 1);
                    __syncthreads();
                }
                const uint4* nxt = ub + 1 < NB ? wbase(i, ub + 1) : i + 1 < n ? wbase(i + 1, 0) : wbase(i, ub);
                mfma_block_wk<T, R>(wbase(i, ub), nxt, dbuf + (size_t)ub * R * 1024, v, jr, accr, F0, F1);
            }
            uint32_t ro = (uint32_t)rbase;
            __asm__ volatile("" : "+v"(ro));
            if (rows_lds) {
#pragma unroll
                for (int q = 0; q < RP; q++) {
                    vec4 o;
#pragma unroll
                    for (int e = 0; e < 4; e++) o[e] = accr[q][e];
                    *(vec4*)(acc0 + ro + q * STEP4) = o;
                }
            }
            __syncthreads();
        }
    }
    if constexpr (!SK && !WK) for (int i = 0; i < n; i++) {
        const int ab = cd_live ? (int)mod_switch<T>(a_next, LG) : 0;
        if (i + 1 < n) a_next = lwe_cd[i + 1];
        if (DALL && !ACCL) {
            digits_phase<T, R, 2>(src, ab, dbuf, 0, 0, l, l, a.bg_bits);
            __syncthreads();
        }
        for (int pass = 0; pass < NPASS; pass++) {
            T dlocal[REGACC ? 1 : RP][4];
            T(&delta)[RP][4] = *reinterpret_cast<T(*)[RP][4]>(REGACC ? (void*)accr : (void*)dlocal);
            if (!REGACC) {
#pragma unroll
                for (int q = 0; q < RP; q++)
#pragma unroll
                    for (int e = 0; e < 4; e++) delta[q][e] = 0;
            }
            for (int ub = 0; ub < NB; ub++, t++) {
                if (ACCL && ub % l == 0) {
                    // digits of component ub/l (its MFMA blocks of the last
                    // component ended with a barrier)
                    if (ub == 0) digits_phase<T, R, 1>(acc0, ab, dbuf, 0, 0, l, l, a.bg_bits);
                    else digits_phase<T, R, 1>(PARK ? acc0 : acc1, ab, dbuf, 0, 0, l, l, a.bg_bits);
                    __syncthreads();
                    if constexpr (PARK) if (ub == 0 && v == 1) {
                        // this step's component-1 input rows (no fold has touched them yet)
                        uint32_t ro = (uint32_t)rbase0;
                        __asm__ volatile("" : "+v"(ro));
#pragma unroll
                        for (int q = 0; q < RP; q++) {
                            vec4 o;
#pragma unroll
                            for (int e = 0; e < 4; e++) o[e] = accr[q][e];
                            *(vec4*)(acc0 + ro + q * STEP4) = o;
                        }
                    }
                }
                if (!DALL && ub % DG == 0) {
                    int8_t* gc = DCACHE ? a.dcache + ((size_t)blockIdx.x * NB + ub) * R * 1024 : nullptr;
                    if (!DCACHE || pass == 0) {
                        digits_phase<T, R, 1, DCACHE>(src, ab, dbuf, ub / l, ub % l, DG, l, a.bg_bits, gc);
                    } else {
                        uint4 dc[DCV];
#pragma unroll
                        for (int q = 0; q < DCV; q++) {
                            const int idx = tid + q * THREADS;
                            if (DCU % THREADS == 0 || idx < DCU) dc[q] = ((const uint4*)gc)[idx];
                        }
#pragma unroll
                        for (int q = 0; q < DCV; q++) {
                            const int idx = tid + q * THREADS;
                            if (DCU % THREADS == 0 || idx < DCU) ((uint4*)dbuf)[idx] = dc[q];
                        }
                    }
                }
                if (DOUBLE) {
                    // prefetch the next block of the (i, pass, ub) sequence
                    int ni = i, nub = ub + 1, npass = pass;
                    if (nub == NB) { nub = 0; npass++; if (npass == NPASS) { npass = 0; ni++; } }
                    if (ni < n) KEY_LOAD(kbase + ((size_t)ni * NB + nub) * KU);
                } else {
                    KEY_LOAD(kbase + ((size_t)i * NB + ub) * KU);
                    KEY_STORE(kbuf);
                    __syncthreads();
                }
                // (double-buffered: the slot read below was stored before the
                // previous block's closing barrier)
                const uint8_t* kslot = kbuf + (DOUBLE ? (size_t)(t & 1) * KC * KCS : 0);
                const int8_t* dblk = dbuf + (size_t)(ACCL ? ub % l : DALL ? ub : ub % DG) * R * 1024;
                mfma_block<T, R, RP, KC>(kslot, dblk, v, jr, pass, delta);
                if (DOUBLE) KEY_STORE(kbuf + (size_t)((t + 1) & 1) * KC * KCS);
                __syncthreads();
            }
            if (REGACC) {
                // opaque per step, so the row addresses are formed here
                // instead of being held across the step loop
                uint32_t ro = (uint32_t)rbase;
                __asm__ volatile("" : "+v"(ro));
                auto put = [&](T* base) {
#pragma unroll
                    for (int q = 0; q < RP; q++) {
                        vec4 o;
#pragma unroll
                        for (int e = 0; e < 4; e++) o[e] = delta[q][e];
                        *(vec4*)(base + ro + q * STEP4) = o;
                    }
                };
                if (rows_lds) put(acc0);
                else if (!PARK) put(ACCL ? ws0 : dst);
                continue;
            }
            // dst rows of this pass = src rows + delta (16-byte accesses; all
            // loads issued before the stores).  Row tile J = jr + 4a holds
            // coefficients 16J + 4(lane>>4) + e of ciphertext lane&15.
            {
                const size_t base0 = acc_idx<T>(N, v, 16 * (jr + 4 * pass * RP) + 4 * (lane >> 4), lane & 15);
                constexpr size_t STEP = (size_t)(64 / 4) * CTS * 4;  // 4 row tiles further
                // opaque per step, so the 2*RP row addresses are formed here
                // instead of being hoisted out of the step loop
                uint32_t bo = (uint32_t)base0;
                __asm__ volatile("" : "+v"(bo));  // (the offset, so the pointers stay global)
                const T* ps = src + bo;
                T* pd = dst + bo;
                vec4 cur[RP];
#pragma unroll
                for (int q = 0; q < RP; q++) cur[q] = *(const vec4*)(ps + q * STEP);
#pragma unroll
                for (int q = 0; q < RP; q++) {
                    vec4 o;
#pragma unroll
                    for (int e = 0; e < 4; e++) o[e] = (T)(cur[q][e] + delta[q][e]);
                    *(vec4*)(pd + q * STEP) = o;
                }
            }
        }
        __syncthreads();
        T* tmp = src;
        src = dst;
        dst = tmp;
    }

#undef KEY_LOAD
#undef KEY_STORE
    if constexpr (PARK) {
        if (v == 1) {
#pragma unroll
            for (int q = 0; q < RP; q++) {
                vec4 o;
#pragma unroll
                for (int e = 0; e < 4; e++) o[e] = accr[q][e];
                *(vec4*)(ws0 + rbase + q * STEP4) = o;
            }
        }
        __syncthreads();
    }
    // ---- sample extraction: a'_0 = A[0], a'_j = -A[N-j], b' = B[0]
    const T* A0 = ACCL ? (const T*)acc0 : src;
    T* out = (T*)a.out;
    for (int idx = tid; idx < CTS * (N + 1); idx += THREADS) {
        const int c = idx / (N + 1), j = idx - c * (N + 1);
        const int gi = ct0 + c;
        if (gi >= a.B) continue;
        T val;
        if (j == 0) val = A0[acc_idx<T>(N, 0, 0, c)];
        else if (j < N) val = (T)(0 - A0[acc_idx<T>(N, 0, N - j, c)]);
        else val = (ACC1L ? (const T*)acc0 : (const T*)src)[acc_idx<T>(N, 1, 0, c)];
        out[(size_t)gi * (N + 1) + j] = val;
    }
}

// ------------------------------------------------ multi-workgroup path
//
// A batch of few ciphertexts leaves most CUs idle in the kernel above (one
// workgroup runs a group of 16 ciphertexts through all n steps).  Here every
// step is two launches over all groups: split_digits_kernel forms the
// step's digits of every group into global memory (DS workgroups per group
// and component), and split_mfma_kernel spreads each group's output rows over
// R/RP workgroups -- workgroup `pass` computes the row tiles the persistent
// kernel's row pass `pass` computes, with the same mfma_block -- and writes
// ACC + delta to the other accumulator buffer.  The arithmetic is the
// persistent kernel's (integer sums mod 2^q), so the bits are the same.

struct SplitArgs {
    const void* lwe;          // [B][n+1] words
    const int8_t* bsk8;       // [n][2l][2][LIMBS][2N]
    const void* tv;           // test polynomials [ntv][N] words
    const int32_t* tv_index;  // [B] or null
    void* out;                // [B][N+1] words
    void* acc;                // [2][G][2N*16] words (ping-pong)
    int8_t* dig;              // [G][2l][N/64][1024] digit bytes of the step
    int B, G, n, l, bg_bits, step;
};

// Row tiles per wave of the multi-workgroup path (each key fragment feeds
// that many MFMAs, which hides the LDS latency of the next one).
constexpr int SPLIT_RP = 4;

// Digit slices per group and component: 1024 items (of 4 coefficients) each.
template <int R>
constexpr int split_ds() { return R >= 4 ? R / 4 : 1; }

template <typename T, int R>
__global__ __launch_bounds__(THREADS) void split_init_kernel(SplitArgs a) {
    constexpr int N = R * 64;
    constexpr int LG = __builtin_ctz(2 * N);
    const int g = blockIdx.x;
    const T* lwe = (const T*)a.lwe;
    T* acc = (T*)a.acc + (size_t)g * 2 * N * CTS;
    for (int idx = threadIdx.x; idx < CTS * N; idx += THREADS) {
        const int c = idx & (CTS - 1), j = idx >> 4;
        const int gi = g * CTS + c;
        T body = 0;
        if (gi < a.B) {
            const int bb = (int)mod_switch<T>(lwe[(size_t)gi * (a.n + 1) + a.n], LG);
            const int e = (2 * N - bb) & (2 * N - 1);
            const T* tv = (const T*)a.tv + (size_t)(a.tv_index ? a.tv_index[gi] : 0) * N;
            body = monomial_coef<T>([&](int s) -> T { return tv[s]; }, N, e, j);
        }
        acc[acc_idx<T>(N, 0, j, c)] = 0;
        acc[acc_idx<T>(N, 1, j, c)] = body;
    }
}

// grid (G, 2 components, DS slices): digits of step a.step for every level.
template <typename T, int R>
__global__ __launch_bounds__(THREADS) void split_digits_kernel(SplitArgs a) {
    constexpr int N = R * 64;
    constexpr int LG = __builtin_ctz(2 * N);
    constexpr int DS = split_ds<R>();
    const int g = blockIdx.x, u = blockIdx.y, ds = blockIdx.z;
    const int cd = threadIdx.x & (CTS - 1);
    const int gi = g * CTS + cd;
    const T* lwe = (const T*)a.lwe;
    const int ab = gi < a.B ? (int)mod_switch<T>(lwe[(size_t)gi * (a.n + 1) + a.step], LG) : 0;
    const T* src = (const T*)a.acc + ((size_t)(a.step & 1) * a.G + g) * 2 * N * CTS;
    T* next = (T*)a.acc + ((size_t)((a.step + 1) & 1) * a.G + g) * 2 * N * CTS;
    int8_t* dst = a.dig + ((size_t)g * 2 * a.l + (size_t)u * a.l) * R * 1024;
    // also seeds the next accumulator with this one (the MFMA launch adds to it)
    digits_phase<T, R, 1, false, DS, true>(src, ab, dst, u, 0, a.l, a.l, a.bg_bits, nullptr, ds, next);
}

// grid (G, R/RP, KS): row pass blockIdx.y of group blockIdx.x over the
// (u,p) blocks of K-slice blockIdx.z (2l/KS consecutive blocks) for step
// a.step; its partial sums are added to the next accumulator (seeded with
// this step's by the digit launch) -- with atomic adds when several slices
// share the rows, which keeps the sum exact mod 2^q in any order.
template <typename T, int R, int RP>
__global__ __launch_bounds__(THREADS, 1) void split_mfma_kernel(SplitArgs a) {
    constexpr int N = R * 64;
    constexpr int NL = Torus<T>::LIMBS;
    constexpr int KSLOT = 2 * NL * 2 * N;  // bytes of one (u,p) key block
    constexpr int KU = KSLOT / 16;         // uint4 per key block
    constexpr int KV = (KU + THREADS - 1) / THREADS;
    constexpr int DU = R * 64;             // uint4 per digit block (R KB)
    constexpr int DV = (DU + THREADS - 1) / THREADS;
    const int g = blockIdx.x, pass = blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int NB = 2 * a.l;
    const int KS = (int)gridDim.z;
    const int ub0 = blockIdx.z * (NB / KS), ub1 = ub0 + NB / KS;
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    int8_t* dslot = (int8_t*)smem;       // digit block (R KB), then the key block
    uint8_t* kslot = smem + (size_t)R * 1024;
    const uint4* kbase = (const uint4*)a.bsk8 + (size_t)a.step * NB * KU;
    const uint4* dbase = (const uint4*)(a.dig + (size_t)g * NB * R * 1024);
    // Staged through registers as native 4-word vectors: held as HIP's
    // uint4 across the block loop the arrays were placed in scratch memory,
    // and each prefetch then waited for its loads at once.
    typedef uint32_t w4 __attribute__((ext_vector_type(4)));
    const w4* kbv = (const w4*)kbase;
    const w4* dbv = (const w4*)dbase;
    w4 kp[KV], dp[DV];
#define SPLIT_LOAD(UB)                                                          \
    do {                                                                        \
        _Pragma("unroll") for (int q_ = 0; q_ < KV; q_++) {                     \
            const int idx_ = tid + q_ * THREADS;                                \
            if (KU % THREADS == 0 || idx_ < KU) kp[q_] = kbv[(size_t)(UB) * KU + idx_]; \
        }                                                                       \
        _Pragma("unroll") for (int q_ = 0; q_ < DV; q_++) {                     \
            const int idx_ = tid + q_ * THREADS;                                \
            if (DU % THREADS == 0 || idx_ < DU) dp[q_] = dbv[(size_t)(UB) * DU + idx_]; \
        }                                                                       \
    } while (0)
#define SPLIT_STORE()                                                           \
    do {                                                                        \
        _Pragma("unroll") for (int q_ = 0; q_ < KV; q_++) {                     \
            const int idx_ = tid + q_ * THREADS;                                \
            if (KU % THREADS == 0 || idx_ < KU) ((w4*)kslot)[idx_] = kp[q_]; \
        }                                                                       \
        _Pragma("unroll") for (int q_ = 0; q_ < DV; q_++) {                     \
            const int idx_ = tid + q_ * THREADS;                                \
            if (DU % THREADS == 0 || idx_ < DU) ((w4*)dslot)[idx_] = dp[q_]; \
        }                                                                       \
    } while (0)
    const int v = wave >> 2, jr = wave & 3;
    T delta[RP][4];
#pragma unroll
    for (int q = 0; q < RP; q++)
#pragma unroll
        for (int e = 0; e < 4; e++) delta[q][e] = 0;
    SPLIT_LOAD(ub0);
    for (int ub = ub0; ub < ub1; ub++) {
        SPLIT_STORE();
        __syncthreads();
        if (ub + 1 < ub1) SPLIT_LOAD(ub + 1);  // in flight during this block's MFMAs
        mfma_block<T, R, RP, 1>(kslot, dslot, v, jr, pass, delta);
        __syncthreads();
    }
#undef SPLIT_LOAD
#undef SPLIT_STORE
    // Row tile J = jr + 4(pass RP + q) holds coefficients 16J + 4(lane>>4) + e
    // of ciphertext lane&15.
    T* dst = (T*)a.acc + ((size_t)((a.step + 1) & 1) * a.G + g) * 2 * N * CTS;
    const size_t base0 = acc_idx<T>(N, v, 16 * (jr + 4 * pass * RP) + 4 * (lane >> 4), lane & 15);
    constexpr size_t STEP = (size_t)(64 / 4) * CTS * 4;  // 4 row tiles further
    typedef T vec4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int q = 0; q < RP; q++) {
        T* row = dst + base0 + q * STEP;
        if (KS == 1) {
            const vec4 cur = *(const vec4*)row;
            vec4 o;
#pragma unroll
            for (int e = 0; e < 4; e++) o[e] = (T)(cur[e] + delta[q][e]);
            *(vec4*)row = o;
        } else {
#pragma unroll
            for (int e = 0; e < 4; e++) atomicAdd(row + e, delta[q][e]);
        }
    }
}

// Sample extraction from the final accumulators: a'_0 = A[0], a'_j = -A[N-j], b' = B[0].
template <typename T, int R>
__global__ __launch_bounds__(THREADS) void split_extract_kernel(SplitArgs a) {
    constexpr int N = R * 64;
    const int g = blockIdx.x;
    const T* A0 = (const T*)a.acc + ((size_t)(a.n & 1) * a.G + g) * 2 * N * CTS;
    T* out = (T*)a.out;
    for (int idx = threadIdx.x; idx < CTS * (N + 1); idx += THREADS) {
        const int c = idx / (N + 1), j = idx - c * (N + 1);
        const int gi = g * CTS + c;
        if (gi >= a.B) continue;
        T val;
        if (j == 0) val = A0[acc_idx<T>(N, 0, 0, c)];
        else if (j < N) val = (T)(0 - A0[acc_idx<T>(N, 0, N - j, c)]);
        else val = A0[acc_idx<T>(N, 1, 0, c)];
        out[(size_t)gi * (N + 1) + j] = val;
    }
}

template <typename T, int R>
int launch_split_t(tfhe_ctx* c, SplitArgs a, int KS, hipStream_t s) {
    constexpr int N = R * 64;
    constexpr int NL = Torus<T>::LIMBS;
    constexpr int RP = SPLIT_RP;
    if (KS < 1 || (2 * a.l) % KS) return ctx_fail(c, TFHE_EINVAL, "K slices must divide the 2l key blocks");
    // (+16: the last limb's fragments read up to 4 bytes past the key block)
    const size_t lds = (size_t)R * 1024 + 2ull * NL * 2 * N + 16;
    auto km = split_mfma_kernel<T, R, RP>;
    hipError_t e = hipFuncSetAttribute((const void*)km, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_check(c, e, "hipFuncSetAttribute(split_mfma)");
    auto ki = split_init_kernel<T, R>;
    auto kd = split_digits_kernel<T, R>;
    auto kx = split_extract_kernel<T, R>;
    hipLaunchKernelGGL(ki, dim3(a.G), dim3(THREADS), 0, s, a);
    for (int i = 0; i < a.n; i++) {
        a.step = i;
        hipLaunchKernelGGL(kd, dim3(a.G, 2, split_ds<R>()), dim3(THREADS), 0, s, a);
        hipLaunchKernelGGL(km, dim3(a.G, R / RP, KS), dim3(THREADS), lds, s, a);
    }
    hipLaunchKernelGGL(kx, dim3(a.G), dim3(THREADS), 0, s, a);
    return hip_check(c, hipGetLastError(), "launch split blind rotation");
}

template <typename T, int R, int RP, int DG>
int launch_t(tfhe_ctx* c, const BrArgs& a, size_t lds, hipStream_t s) {
    auto k = br_mfma_kernel<T, R, RP, DG>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_check(c, e, "hipFuncSetAttribute(br_mfma)");
    const unsigned grid = (a.B + CTS - 1) / CTS;
    hipLaunchKernelGGL(k, dim3(grid), dim3(THREADS), lds, s, a);
    return hip_check(c, hipGetLastError(), "launch br_mfma");
}

// LDS bytes of the kernel with digit group dg (0 = all blocks of a step,
// -1 = one component's blocks plus accumulator component 0, -2 = all digit
// and key blocks of a step plus both accumulator components).
size_t lds_need(const tfhe_ctx* c, int dg) {
    const int N = c->p.N, l = c->p.l;
    const int NL = c->q == 32 ? 4 : 8;
    const size_t kslot = N <= 256 ? 4 * (2ull * NL * 2 * N + KCOPY_PAD) : 2ull * NL * 2 * N;
    if (dg == -2) return 2ull * l * (N / 64) * 1024 + 2ull * l * kslot + 2ull * N * CTS * word_bytes(c);
    if (dg == -3) return 2ull * l * (N / 64) * 1024 + (size_t)N * CTS * word_bytes(c);
    size_t b = (size_t)(dg < 0 ? l : dg == 0 ? 2 * l : dg) * (N / 64) * 1024;
    b += (dg <= 0 ? 2 : 1) * kslot;
    if (dg < 0) b += (size_t)N * CTS * word_bytes(c) * (2ull * N * CTS * word_bytes(c) <= 65536 ? 2 : 1);
    return b;
}

constexpr int kNoFit = -100;

// Row tiles per pass instantiated for (q, N) and the row_pass knob.
int plan_rp(const tfhe_ctx* c) {
    const int N = (int)c->p.N, rp = c->row_pass;
    if (c->q == 32) {
        switch (N) {
            case 64: return 1;
            case 256: return rp == 2 ? 2 : 4;
            case 512: return rp == 4 ? 4 : 8;
            case 1024: return rp == 8 ? 8 : 16;
            case 2048: return 8;
        }
    } else {
        switch (N) {
            case 64: return 1;
            case 256: case 512: case 1024: return 4;
            case 2048: return rp == 4 ? 4 : 8;
        }
    }
    return 0;
}

// Largest digit grouping that fits LDS and the digit_blocks knob (0 auto,
// 1 one block, 2 pairs of levels when l is even, 3 all blocks of a step with
// the accumulator in global memory, 4 one component's blocks with
// accumulator component 0 in LDS).  Auto prefers, with one row pass, the
// step-keyed schedule when both accumulator components fit in LDS (small N,
// l <= 4) and it costs no occupancy for a batch of B, else the
// per-component grouping that keeps component 0 in LDS.
int plan_dg(const tfhe_ctx* c, int R, int rp, uint32_t B) {
    const size_t max_lds = (size_t)c->prop.maxSharedMemoryPerMultiProcessor > 0
                               ? (size_t)c->prop.maxSharedMemoryPerMultiProcessor
                               : (size_t)160 * 1024;
    const bool both_lds = 2ull * c->p.N * CTS * word_bytes(c) <= 65536;
    if (rp == R && c->digit_blocks == 0 && c->d_win && lds_need(c, -3) <= max_lds) return -3;
    if (rp == R && c->digit_blocks == 0 && both_lds && c->p.l <= 4 && lds_need(c, -2) <= max_lds) {
        // The step-keyed schedule stages a whole step's keys, which can leave
        // room for fewer workgroups per CU than the per-component one (at
        // N = 256: one instead of two): take it when it keeps two per CU, or
        // when the batch's groups all fit at its occupancy.
        const int cus = c->prop.multiProcessorCount > 0 ? c->prop.multiProcessorCount : 256;
        const uint64_t groups = ((uint64_t)B + CTS - 1) / CTS;
        const size_t per_cu = max_lds / lds_need(c, -2);
        if (per_cu >= 2 || lds_need(c, -1) > max_lds / 2 || groups <= (uint64_t)cus * per_cu) return -2;
    }
    if (rp == R && (c->digit_blocks == 0 || c->digit_blocks == 4) && lds_need(c, -1) <= max_lds) return -1;
    if ((c->digit_blocks == 0 || c->digit_blocks == 3) && lds_need(c, 0) <= max_lds) return 0;
    if (c->digit_blocks != 1 && c->p.l % 2 == 0 && lds_need(c, 2) <= max_lds) return 2;
    if (lds_need(c, 1) > max_lds) return kNoFit;
    return 1;
}

template <typename T, int R, int RP>
int dispatch_dg(tfhe_ctx* c, const BrArgs& a, int dg, hipStream_t s) {
    if constexpr (RP == R) {
        if (dg == -1) return launch_t<T, R, RP, -1>(c, a, lds_need(c, -1), s);
    }
    if constexpr (RP == R && 2 * R * 64 * CTS * sizeof(T) <= 65536) {
        if (dg == -2) return launch_t<T, R, RP, -2>(c, a, lds_need(c, -2), s);
    }
    if constexpr (sizeof(T) == 4 && R == 16 && RP == 16) {
        if (dg == -3) return launch_t<T, R, RP, -3>(c, a, lds_need(c, -3), s);
    }
    if (dg == 0) return launch_t<T, R, RP, 0>(c, a, lds_need(c, 0), s);
    if (dg == 2) return launch_t<T, R, RP, 2>(c, a, lds_need(c, 2), s);
    if (dg == 1) return launch_t<T, R, RP, 1>(c, a, lds_need(c, 1), s);
    return ctx_fail(c, TFHE_EINVAL, "parameters exceed LDS capacity of the MFMA kernel");
}

// Accumulator buffers per workgroup (words of 2N * CTS per buffer): none
// when both components stay in LDS, one buffer (of which component 0 in LDS
// leaves the first half unused) when a step's digits are formed before its
// blocks, else two alternating buffers.  Then (several row passes with
// per-group digits) the digit cache.
size_t acc_ws_bytes(const tfhe_ctx* c, uint32_t B) {
    const int R = (int)c->p.N / 64, rp = plan_rp(c);
    if (rp <= 0) return 0;
    const int dg = plan_dg(c, R, rp, B);
    if (dg == kNoFit) return 0;
    const size_t grid = (B + CTS - 1) / CTS;
    const size_t comp = (size_t)c->p.N * CTS * word_bytes(c);  // one component of a workgroup
    if (dg < 0) return 2 * comp <= 65536 ? 0 : grid * 2 * comp;
    return grid * (dg == 0 ? 1 : 2) * 2 * comp;
}

// Groups of 16 ciphertexts up to which a batch takes the multi-workgroup
// path: the split_groups knob, by default half the CUs for N >= 512 (at the
// standard set it is still 6% faster at 128 groups; at N = 256 a group's
// step is too short to gain, so only on request).
int64_t split_limit(const tfhe_ctx* c) {
    const int R = (int)c->p.N / 64;
    if (R < 4) return 0;
    const int cus = c->prop.multiProcessorCount > 0 ? c->prop.multiProcessorCount : 256;
    if (c->split_groups >= 0) return c->split_groups;
    return R >= 8 ? cus / 2 : 0;
}

// K slices of the multi-workgroup path for a batch of B (0 = the persistent
// kernel): the most (a divisor of the 2l key blocks) that keep the launch
// within two workgroups per CU, at least one.
int split_ks(const tfhe_ctx* c, uint32_t B) {
    const int R = (int)c->p.N / 64;
    if (B == 0 || R < SPLIT_RP) return 0;
    const int cus = c->prop.multiProcessorCount > 0 ? c->prop.multiProcessorCount : 256;
    const int64_t lim = split_limit(c);
    const int64_t G = (B + CTS - 1) / CTS;
    if (G > lim) return 0;
    const int NB = 2 * (int)c->p.l;
    int ks = 1;
    for (int d = 1; d <= NB; d++)
        if (NB % d == 0 && G * (R / SPLIT_RP) * d <= 2 * cus) ks = d;
    return ks;
}

size_t split_ws_bytes(const tfhe_ctx* c, uint32_t B) {
    const size_t G = (B + CTS - 1) / CTS;
    return 2 * G * 2 * (size_t)c->p.N * CTS * word_bytes(c) + G * 2 * (size_t)c->p.l * (c->p.N / 64) * 1024;
}

size_t dcache_bytes(const tfhe_ctx* c, uint32_t B) {
    const int R = (int)c->p.N / 64, rp = plan_rp(c);
    if (rp <= 0 || R / rp <= 1 || plan_dg(c, R, rp, B) <= 0) return 0;
    const size_t grid = (B + CTS - 1) / CTS;
    return grid * 2 * (size_t)c->p.l * R * 1024;
}

}  // namespace

// Row tiles per pass instantiated for each (q, N); the first is the default.
bool mfma_row_pass_supported(const tfhe_ctx* c, int rp) {
    const int N = (int)c->p.N;
    if (c->q == 32) {
        if (N == 64) return rp == 1;
        if (N == 256) return rp == 4 || rp == 2;
        if (N == 512) return rp == 8 || rp == 4;
        if (N == 1024) return rp == 16 || rp == 8;
        if (N == 2048) return rp == 8;
        return false;
    }
    if (N == 64) return rp == 1;
    if (N == 256 || N == 512 || N == 1024) return rp == 4;
    if (N == 2048) return rp == 8 || rp == 4;
    return false;
}

size_t mfma_ws_bytes(const tfhe_ctx* c, uint32_t B) {
    if (split_ks(c, B)) return split_ws_bytes(c, B);
    return acc_ws_bytes(c, B) + dcache_bytes(c, B);
}

// Largest workspace of any batch of at most Bmax ciphertexts (the split
// path's need grows with B below its threshold, the persistent kernel's
// with B above it).
size_t mfma_ws_bytes_upto(const tfhe_ctx* c, uint32_t Bmax) {
    size_t need = mfma_ws_bytes(c, Bmax);
    const uint64_t bs = std::min<uint64_t>(Bmax, (uint64_t)split_limit(c) * CTS);
    if (bs) need = std::max(need, split_ws_bytes(c, (uint32_t)bs));
    return need;
}

template <typename T, int R>
int dispatch_split(tfhe_ctx* c, const SplitArgs& a, int ks, hipStream_t s) {
    return launch_split_t<T, R>(c, a, ks, s);
}

int launch_br_mfma(tfhe_ctx* c, const void* lwe_in, const void* tv, const int32_t* tv_index,
                   void* big_out, uint32_t B, void* ws, size_t ws_cap, hipStream_t s) {
    const int N = (int)c->p.N;
    const int rp = plan_rp(c);
    if (N < 64 || rp <= 0) return ctx_fail(c, TFHE_EINVAL, "unsupported N for the MFMA kernel");
    const int dg = plan_dg(c, N / 64, rp, B);
    if (dg == kNoFit) return ctx_fail(c, TFHE_EINVAL, "parameters exceed LDS capacity of the MFMA kernel");
    // the tuning may have changed since the workspace was sized
    const size_t need = mfma_ws_bytes(c, B);
    if ((need && !ws) || need > ws_cap)
        return ctx_fail(c, TFHE_EINVAL, "blind-rotation workspace too small for the current tuning");
    if (const int srp = split_ks(c, B)) {
        SplitArgs sa;
        sa.lwe = lwe_in;
        sa.bsk8 = c->d_bsk8;
        sa.tv = tv;
        sa.tv_index = tv_index;
        sa.out = big_out;
        sa.acc = ws;
        const uint32_t G = (B + CTS - 1) / CTS;
        sa.dig = (int8_t*)ws + 2 * (size_t)G * 2 * N * CTS * word_bytes(c);
        sa.B = (int)B;
        sa.G = (int)G;
        sa.n = (int)c->p.n;
        sa.l = (int)c->p.l;
        sa.bg_bits = (int)c->p.bg_bits;
        sa.step = 0;
        if (c->q == 32) {
            switch (N) {
                case 256: return dispatch_split<uint32_t, 4>(c, sa, srp, s);
                case 512: return dispatch_split<uint32_t, 8>(c, sa, srp, s);
                case 1024: return dispatch_split<uint32_t, 16>(c, sa, srp, s);
                case 2048: return dispatch_split<uint32_t, 32>(c, sa, srp, s);
            }
        } else {
            switch (N) {
                case 256: return dispatch_split<uint64_t, 4>(c, sa, srp, s);
                case 512: return dispatch_split<uint64_t, 8>(c, sa, srp, s);
                case 1024: return dispatch_split<uint64_t, 16>(c, sa, srp, s);
                case 2048: return dispatch_split<uint64_t, 32>(c, sa, srp, s);
            }
        }
        return ctx_fail(c, TFHE_EINVAL, "unsupported N for the multi-workgroup blind rotation");
    }
    BrArgs a;
    a.lwe = lwe_in;
    a.bsk8 = c->d_bsk8;
    a.win = (const uint4*)c->d_win;
    a.tv = tv;
    a.tv_index = tv_index;
    a.out = big_out;
    a.ws = ws;
    a.dcache = dcache_bytes(c, B) ? (int8_t*)ws + acc_ws_bytes(c, B) : nullptr;
    a.B = (int)B;
    a.n = (int)c->p.n;
    a.l = (int)c->p.l;
    a.bg_bits = (int)c->p.bg_bits;
    if (c->q == 32) {
        switch (N) {
            case 64: return dispatch_dg<uint32_t, 1, 1>(c, a, dg, s);
            case 256: return rp == 2 ? dispatch_dg<uint32_t, 4, 2>(c, a, dg, s) : dispatch_dg<uint32_t, 4, 4>(c, a, dg, s);
            case 512: return rp == 4 ? dispatch_dg<uint32_t, 8, 4>(c, a, dg, s) : dispatch_dg<uint32_t, 8, 8>(c, a, dg, s);
            case 1024:
                return rp == 8 ? dispatch_dg<uint32_t, 16, 8>(c, a, dg, s) : dispatch_dg<uint32_t, 16, 16>(c, a, dg, s);
            case 2048: return dispatch_dg<uint32_t, 32, 8>(c, a, dg, s);
        }
    } else {
        switch (N) {
            case 64: return dispatch_dg<uint64_t, 1, 1>(c, a, dg, s);
            case 256: return dispatch_dg<uint64_t, 4, 4>(c, a, dg, s);
            case 512: return dispatch_dg<uint64_t, 8, 4>(c, a, dg, s);
            case 1024: return dispatch_dg<uint64_t, 16, 4>(c, a, dg, s);
            case 2048:
                return rp == 4 ? dispatch_dg<uint64_t, 32, 4>(c, a, dg, s) : dispatch_dg<uint64_t, 32, 8>(c, a, dg, s);
        }
    }
    return ctx_fail(c, TFHE_EINVAL, "unsupported N for the MFMA kernel");
}
