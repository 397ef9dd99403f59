/*
 * tfhe_oracle.c -- plain, slow CPU reference of the FHE-SQL oblivious-selection
 * hot path.  TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no code
 * with the GPU library.
 *
 * The FHE-SQL paper (Section 2.2 and Section 4.3) evaluates its WHERE mask and
 * masked select with TFHE gate bootstrapping but does not define TFHE's
 * internals; it cites the TFHE paper (Chillotti, Gama, Georgieva, Izabachene,
 * "TFHE: Fast Fully Homomorphic Encryption over the Torus", ePrint 2018/421).
 * Every function below follows that paper's definitions, written out on the
 * discretised torus Z/2^q (q <= 64) with wrapping unsigned arithmetic:
 *   - LWE / GLWE / GGSW ciphertexts and their phases (TFHE Sec. 2 and 3),
 *   - the signed gadget decomposition (TFHE Def. 3.7 / Lemma 3.7 reading),
 *   - the external product and CMux (TFHE Sec. 3.4),
 *   - blind rotation, sample extraction and key switching (TFHE Alg. 3 and
 *     Sec. 4), gate bootstrapping (TFHE Sec. 4.2) and programmable
 *     bootstrapping with a test polynomial.
 * Rounding ties go up (add half, floor) everywhere; gadget digits lie in
 * [-Bg/2, Bg/2).  Values are held in uint64_t and reduced mod 2^q.
 *
 * Parameter vector p[8] = {q, n, k, N, bg_bits, l, ks_bits, ks_t}.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t tor;

enum { PQ = 0, PN = 1, PK = 2, PBIGN = 3, PBG = 4, PL = 5, PKSB = 6, PKST = 7 };

static tor qmask(int q) { return q >= 64 ? ~(tor)0 : (((tor)1 << q) - 1); }

/* 2^e mod 2^q (e may be >= q, then 0). */
static tor pow2(int q, int e) { return e >= q ? 0 : ((tor)1 << e); }

/* Round x (a q-bit value) to its top `bits` bits, half-up; result in [0, 2^bits). */
tor or_round_top(int q, int bits, tor x) {
    x &= qmask(q);
    if (bits >= q) return x;
    int sh = q - bits;
    tor r = ((x + ((tor)1 << (sh - 1))) & qmask(q)) >> sh;
    return r;
}

/* Modulus switch to Z_2N:  floor((x + 2^(q-log2(2N)-1)) / 2^(q-log2(2N))) mod 2N. */
tor or_mod_switch(int q, int N, tor x) {
    int lg = 0;
    while ((1 << lg) < 2 * N) lg++;
    return or_round_top(q, lg, x);
}

/* Signed gadget decomposition of x with base 2^bg_bits and l levels.
 * d[0] is the most significant level (p = 1), d[l-1] the least (p = l).
 * Digits lie in [-Bg/2, Bg/2) and sum_p d_p 2^(q - p*bg_bits) equals the
 * rounding of x to l*bg_bits bits (mod 2^q). */
void or_decompose(int q, int bg_bits, int l, tor x, int64_t *d) {
    tor xt = or_round_top(q, l * bg_bits, x);
    int64_t bg = (int64_t)1 << bg_bits;
    int64_t carry = 0;
    for (int p = l; p >= 1; p--) {
        int64_t r = (int64_t)((xt >> ((l - p) * bg_bits)) & (tor)(bg - 1)) + carry;
        if (r >= bg / 2) { d[p - 1] = r - bg; carry = 1; }
        else { d[p - 1] = r; carry = 0; }
    }
}

/* Negacyclic product c = a * b in Z_2^q[X]/(X^N + 1), schoolbook:
 * c_i = sum_{j<=i} a_j b_{i-j} - sum_{j>i} a_j b_{N+i-j}.  c must not alias. */
void or_negacyclic_mul(int q, int N, const tor *a, const tor *b, tor *c) {
    if (q <= 32) {
        /* Same definition in 32-bit wrapping arithmetic (2^q divides 2^32). */
        uint32_t *acc = (uint32_t *)calloc((size_t)N, sizeof(uint32_t));
        uint32_t *bb = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
        for (int j = 0; j < N; j++) bb[j] = (uint32_t)b[j];
        for (int i = 0; i < N; i++) {
            uint32_t ai = (uint32_t)a[i];
            for (int j = 0; j < N - i; j++) acc[i + j] += ai * bb[j];
            for (int j = N - i; j < N; j++) acc[i + j - N] -= ai * bb[j];
        }
        for (int i = 0; i < N; i++) c[i] = (tor)acc[i] & qmask(q);
        free(acc);
        free(bb);
        return;
    }
    tor *acc = (tor *)calloc((size_t)N, sizeof(tor));
    for (int i = 0; i < N; i++) {
        tor ai = a[i];
        for (int j = 0; j < N - i; j++) acc[i + j] += ai * b[j];
        for (int j = N - i; j < N; j++) acc[i + j - N] -= ai * b[j];
    }
    for (int i = 0; i < N; i++) c[i] = acc[i] & qmask(q);
    free(acc);
}

/* out = X^e * p in Z_2^q[X]/(X^N+1), e in [0, 2N). */
void or_monomial_mul(int q, int N, int64_t e, const tor *p, tor *out) {
    e %= 2 * N;
    if (e < 0) e += 2 * N;
    int neg = 0;
    if (e >= N) { e -= N; neg = 1; }
    for (int i = 0; i < N; i++) {
        tor v;
        if (i >= e) v = p[i - e];
        else v = (tor)0 - p[i - e + N];
        if (neg) v = (tor)0 - v;
        out[i] = v & qmask(q);
    }
}

/* ---------------------------------------------------------------- phases */

/* LWE phase b - <a, s>.  ct = (a_0..a_{n-1}, b). */
tor or_lwe_phase(int q, int n, const tor *key, const tor *ct) {
    tor acc = ct[n];
    for (int i = 0; i < n; i++) acc -= ct[i] * key[i];
    return acc & qmask(q);
}

/* GLWE phase B - sum_j A_j * S_j.  ct = (A_0..A_{k-1}, B), each N words. */
void or_glwe_phase(int q, int k, int N, const tor *S, const tor *ct, tor *out) {
    tor *tmp = (tor *)malloc((size_t)N * sizeof(tor));
    memcpy(out, ct + (size_t)k * N, (size_t)N * sizeof(tor));
    for (int j = 0; j < k; j++) {
        or_negacyclic_mul(q, N, ct + (size_t)j * N, S + (size_t)j * N, tmp);
        for (int i = 0; i < N; i++) out[i] = (out[i] - tmp[i]) & qmask(q);
    }
    free(tmp);
}

/* ------------------------------------------------------------- encryption */

/* LWE encryption of mu: b = <a, s> + mu + e (mask a and error e given). */
void or_lwe_encrypt(int q, int n, const tor *key, const tor *mask, tor err, tor mu, tor *out) {
    tor acc = mu + err;
    for (int i = 0; i < n; i++) {
        out[i] = mask[i] & qmask(q);
        acc += out[i] * key[i];
    }
    out[n] = acc & qmask(q);
}

/* GLWE encryption of msg (N coefficients): A_j = mask_j, B = sum_j A_j*S_j + e + msg. */
void or_glwe_encrypt(int q, int k, int N, const tor *S, const tor *masks, const tor *errs,
                     const tor *msg, tor *out) {
    tor *tmp = (tor *)malloc((size_t)N * sizeof(tor));
    tor *B = out + (size_t)k * N;
    for (int i = 0; i < N; i++) B[i] = (errs[i] + (msg ? msg[i] : 0)) & qmask(q);
    for (int j = 0; j < k; j++) {
        for (int i = 0; i < N; i++) out[(size_t)j * N + i] = masks[(size_t)j * N + i] & qmask(q);
        or_negacyclic_mul(q, N, out + (size_t)j * N, S + (size_t)j * N, tmp);
        for (int i = 0; i < N; i++) B[i] = (B[i] + tmp[i]) & qmask(q);
    }
    free(tmp);
}

/* GGSW encryption of an integer m: (k+1)*l rows, row r = u*l + (p-1) is a GLWE
 * encryption of zero with m * 2^(q - p*bg_bits) added to coefficient 0 of
 * component u (component k is the body B).
 * masks: [(k+1)l][k][N], errs: [(k+1)l][N], out: [(k+1)l][k+1][N]. */
void or_ggsw_encrypt(const int *P, const tor *S, tor m, const tor *masks, const tor *errs, tor *out) {
    int q = P[PQ], k = P[PK], N = P[PBIGN], bg = P[PBG], l = P[PL];
    size_t glwe = (size_t)(k + 1) * N;
    for (int u = 0; u <= k; u++) {
        for (int p = 1; p <= l; p++) {
            int r = u * l + (p - 1);
            tor *row = out + (size_t)r * glwe;
            or_glwe_encrypt(q, k, N, S, masks + (size_t)r * k * N, errs + (size_t)r * N, NULL, row);
            row[(size_t)u * N] = (row[(size_t)u * N] + m * pow2(q, q - p * bg)) & qmask(q);
        }
    }
}

/* Bootstrapping key: BSK_i = GGSW_S(s_i), i = 0..n-1.
 * masks: [n][(k+1)l][k][N], errs: [n][(k+1)l][N], out: [n][(k+1)l][k+1][N]. */
void or_bsk_gen(const int *P, const tor *s, const tor *S, const tor *masks, const tor *errs, tor *out) {
    int n = P[PN], k = P[PK], N = P[PBIGN], l = P[PL];
    size_t rows = (size_t)(k + 1) * l;
    for (int i = 0; i < n; i++)
        or_ggsw_encrypt(P, S, s[i], masks + (size_t)i * rows * k * N, errs + (size_t)i * rows * N,
                        out + (size_t)i * rows * (k + 1) * N);
}

/* Key-switching table: KSK[i][j][v] = LWE_s(v * s'_i * 2^(q - (j+1)*ks_bits)),
 * i < kN, j < t, v < 2^ks_bits; every entry (v = 0 included) is a fresh noisy
 * encryption.  s' is the extracted key (s'_{jN+i} = S_j[i]).
 * masks: [kN][t][2^b][n], errs: [kN][t][2^b], out: [kN][t][2^b][n+1]. */
void or_ksk_gen(const int *P, const tor *sx, const tor *s, const tor *masks, const tor *errs, tor *out) {
    int q = P[PQ], n = P[PN], k = P[PK], N = P[PBIGN], b = P[PKSB], t = P[PKST];
    int V = 1 << b;
    for (int i = 0; i < k * N; i++)
        for (int j = 0; j < t; j++)
            for (int v = 0; v < V; v++) {
                size_t e = ((size_t)i * t + j) * V + v;
                tor mu = ((tor)v * sx[i] * pow2(q, q - (j + 1) * b)) & qmask(q);
                or_lwe_encrypt(q, n, s, masks + e * n, errs[e], mu, out + e * (n + 1));
            }
}

/* --------------------------------------------------------- bootstrapping */

/* External product GGSW (x) GLWE: out_v = sum_{u<=k} sum_{p=1..l} Dec_p(C_u) * G[u*l+p-1][v],
 * the decomposition taken coefficient-wise. ggsw: [(k+1)l][k+1][N]. */
void or_ext_product(const int *P, const tor *ggsw, const tor *glwe, tor *out) {
    int q = P[PQ], k = P[PK], N = P[PBIGN], bg = P[PBG], l = P[PL];
    size_t glwe_w = (size_t)(k + 1) * N;
    tor *dig = (tor *)malloc((size_t)l * N * sizeof(tor));
    tor *tmp = (tor *)malloc((size_t)N * sizeof(tor));
    int64_t *d = (int64_t *)malloc((size_t)l * sizeof(int64_t));
    memset(out, 0, glwe_w * sizeof(tor));
    for (int u = 0; u <= k; u++) {
        for (int i = 0; i < N; i++) {
            or_decompose(q, bg, l, glwe[(size_t)u * N + i], d);
            for (int p = 0; p < l; p++) dig[(size_t)p * N + i] = (tor)d[p] & qmask(q);
        }
        for (int p = 1; p <= l; p++) {
            const tor *row = ggsw + (size_t)(u * l + p - 1) * glwe_w;
            for (int v = 0; v <= k; v++) {
                or_negacyclic_mul(q, N, dig + (size_t)(p - 1) * N, row + (size_t)v * N, tmp);
                for (int i = 0; i < N; i++)
                    out[(size_t)v * N + i] = (out[(size_t)v * N + i] + tmp[i]) & qmask(q);
            }
        }
    }
    free(dig);
    free(tmp);
    free(d);
}

/* Blind rotation of the test polynomial testv (N words) by the phase of the
 * LWE ciphertext lwe (n+1 words):
 *   ACC = (0, ..., 0, X^{-MS(b)} testv);
 *   for i = 0..n-1 (in this order): ACC <- ACC + ExtProd(BSK_i, X^{MS(a_i)} ACC - ACC).
 * acc_out: (k+1)N words. */
void or_blind_rotate(const int *P, const tor *bsk, const tor *lwe, const tor *testv, tor *acc_out) {
    int q = P[PQ], n = P[PN], k = P[PK], N = P[PBIGN], l = P[PL];
    size_t glwe_w = (size_t)(k + 1) * N;
    size_t ggsw_w = (size_t)(k + 1) * l * glwe_w;
    tor *rot = (tor *)malloc(glwe_w * sizeof(tor));
    tor *ep = (tor *)malloc(glwe_w * sizeof(tor));
    memset(acc_out, 0, glwe_w * sizeof(tor));
    int64_t bbar = (int64_t)or_mod_switch(q, N, lwe[n]);
    or_monomial_mul(q, N, 2 * N - bbar, testv, acc_out + (size_t)k * N);
    for (int i = 0; i < n; i++) {
        int64_t abar = (int64_t)or_mod_switch(q, N, lwe[i]);
        for (int u = 0; u <= k; u++) {
            or_monomial_mul(q, N, abar, acc_out + (size_t)u * N, rot + (size_t)u * N);
            for (int j = 0; j < N; j++)
                rot[(size_t)u * N + j] = (rot[(size_t)u * N + j] - acc_out[(size_t)u * N + j]) & qmask(q);
        }
        or_ext_product(P, bsk + (size_t)i * ggsw_w, rot, ep);
        for (size_t j = 0; j < glwe_w; j++) acc_out[j] = (acc_out[j] + ep[j]) & qmask(q);
    }
    free(rot);
    free(ep);
}

/* Sample extraction of coefficient 0: a'_{jN} = A_j[0], a'_{jN+i} = -A_j[N-i], b' = B[0].
 * out: kN + 1 words. */
void or_sample_extract(const int *P, const tor *glwe, tor *out) {
    int q = P[PQ], k = P[PK], N = P[PBIGN];
    for (int j = 0; j < k; j++) {
        const tor *A = glwe + (size_t)j * N;
        out[(size_t)j * N] = A[0];
        for (int i = 1; i < N; i++) out[(size_t)j * N + i] = ((tor)0 - A[N - i]) & qmask(q);
    }
    out[(size_t)k * N] = glwe[(size_t)k * N];
}

/* Key switching LWE(kN) -> LWE(n): out = (0^n, b') - sum_{i,j} KSK[i][j][digit_j(round(a'_i))],
 * with a'_i rounded half-up to t*ks_bits bits and split into t unsigned digits,
 * most significant first.  ksk: [kN][t][2^b][n+1]. */
void or_keyswitch(const int *P, const tor *ksk, const tor *in, tor *out) {
    int q = P[PQ], n = P[PN], k = P[PK], N = P[PBIGN], b = P[PKSB], t = P[PKST];
    int V = 1 << b;
    for (int w = 0; w < n; w++) out[w] = 0;
    out[n] = in[(size_t)k * N];
    for (int i = 0; i < k * N; i++) {
        tor at = or_round_top(q, t * b, in[i]);
        for (int j = 1; j <= t; j++) {
            int v = (int)((at >> ((t - j) * b)) & (tor)(V - 1));
            const tor *row = ksk + (((size_t)i * t + (j - 1)) * V + v) * (n + 1);
            for (int w = 0; w <= n; w++) out[w] = (out[w] - row[w]) & qmask(q);
        }
    }
}

/* Bootstrap without key switch: SE(BR(lwe, testv)); out: kN + 1 words. */
void or_bootstrap(const int *P, const tor *bsk, const tor *lwe, const tor *testv, tor *out) {
    size_t glwe_w = (size_t)(P[PK] + 1) * P[PBIGN];
    tor *acc = (tor *)malloc(glwe_w * sizeof(tor));
    or_blind_rotate(P, bsk, lwe, testv, acc);
    or_sample_extract(P, acc, out);
    free(acc);
}

/* Gate test polynomial: every coefficient 2^(q-3) (the torus value 1/8). */
void or_gate_testv(int q, int N, tor *testv) {
    for (int i = 0; i < N; i++) testv[i] = pow2(q, q - 3);
}

/* Programmable bootstrap test polynomial for a table f over Z_p with output
 * scale delta_out: coefficient j encodes f(m(j)), m(j) = floor((j p + N/2) / N);
 * where m(j) = p (the last half-box) the coefficient is -delta_out f(0), so
 * the negacyclic wrap returns f(0) for phases just below 0. */
void or_lut_testv(int q, int N, int p, const tor *f, tor delta_out, tor *testv) {
    for (int j = 0; j < N; j++) {
        int64_t m = ((int64_t)j * p + N / 2) / N;
        if (m >= p) testv[j] = ((tor)0 - delta_out * f[0]) & qmask(q);
        else testv[j] = (delta_out * f[m]) & qmask(q);
    }
}

/* Full bootstrap KS(SE(BR(lwe, testv))); out: n + 1 words. */
void or_pbs(const int *P, const tor *bsk, const tor *ksk, const tor *lwe, const tor *testv, tor *out) {
    size_t big = (size_t)P[PK] * P[PBIGN] + 1;
    tor *tmp = (tor *)malloc(big * sizeof(tor));
    or_bootstrap(P, bsk, lwe, testv, tmp);
    or_keyswitch(P, ksk, tmp, out);
    free(tmp);
}

/* Gate bootstrap: PBS with the gate test polynomial. */
void or_gate_bootstrap(const int *P, const tor *bsk, const tor *ksk, const tor *lwe, tor *out) {
    tor *tv = (tor *)malloc((size_t)P[PBIGN] * sizeof(tor));
    or_gate_testv(P[PQ], P[PBIGN], tv);
    or_pbs(P, bsk, ksk, lwe, tv, out);
    free(tv);
}

/* Linear combination of LWE ciphertexts: out = (0^n, c) + sum_j w_j ct_j.
 * ins: [nin][n+1] words, w: nin signed weights. */
void or_lincomb(int q, int n, int nin, const tor *ins, const int64_t *w, tor c, tor *out) {
    for (int i = 0; i < n; i++) out[i] = 0;
    out[n] = c & qmask(q);
    for (int j = 0; j < nin; j++)
        for (int i = 0; i <= n; i++)
            out[i] = (out[i] + (tor)w[j] * ins[(size_t)j * (n + 1) + i]) & qmask(q);
}
