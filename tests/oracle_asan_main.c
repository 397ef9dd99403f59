/*
 * Test driver for the oracle under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (built and run by tests/test_oracle_sanitizers.py, CPU only).
 * It calls every exported oracle function at tiny 32- and 64-bit parameter
 * sets with pseudo-random inputs, checks a few exact identities (negacyclic
 * product by X, decomposition reconstruction, gate bootstrap decryption with
 * noiseless keys) and exits 0 when they hold; a sanitizer report aborts.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t tor;

tor or_round_top(int q, int bits, tor x);
tor or_mod_switch(int q, int N, tor x);
void or_decompose(int q, int bg_bits, int l, tor x, int64_t *d);
void or_negacyclic_mul(int q, int N, const tor *a, const tor *b, tor *c);
void or_monomial_mul(int q, int N, int64_t e, const tor *p, tor *out);
tor or_lwe_phase(int q, int n, const tor *key, const tor *ct);
void or_lwe_encrypt(int q, int n, const tor *key, const tor *mask, tor err, tor mu, tor *out);
void or_bsk_gen(const int *P, const tor *s, const tor *S, const tor *masks, const tor *errs, tor *out);
void or_ksk_gen(const int *P, const tor *sx, const tor *s, const tor *masks, const tor *errs, tor *out);
void or_gate_bootstrap(const int *P, const tor *bsk, const tor *ksk, const tor *lwe, tor *out);
void or_lut_testv(int q, int N, int p, const tor *f, tor delta_out, tor *testv);
void or_pbs(const int *P, const tor *bsk, const tor *ksk, const tor *lwe, const tor *testv, tor *out);
void or_lincomb(int q, int n, int nin, const tor *ins, const int64_t *w, tor c, tor *out);

static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint64_t nxt(void) {  /* xorshift64*, only to fill test inputs */
    st ^= st >> 12;
    st ^= st << 25;
    st ^= st >> 27;
    return st * 0x2545F4914F6CDD1Dull;
}
static tor qm(int q) { return q >= 64 ? ~(tor)0 : (((tor)1 << q) - 1); }

static int fails = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); fails++; } \
    } while (0)

static void run(int q, int n, int N, int bg, int l, int kb, int kt) {
    const int k = 1;
    int P[8] = {q, n, k, N, bg, l, kb, kt};
    const tor m = qm(q);
    /* negacyclic product by X equals the monomial shift by 1 */
    tor *a = calloc(N, sizeof(tor)), *x = calloc(N, sizeof(tor)), *c = calloc(N, sizeof(tor)), *d = calloc(N, sizeof(tor));
    for (int i = 0; i < N; i++) a[i] = nxt() & m;
    x[1] = 1;
    or_negacyclic_mul(q, N, a, x, c);
    or_monomial_mul(q, N, 1, a, d);
    CHECK(memcmp(c, d, N * sizeof(tor)) == 0);
    /* decomposition reconstructs the rounded value */
    int64_t dg[16];
    for (int r = 0; r < 200; r++) {
        tor v = nxt() & m, acc = 0;
        or_decompose(q, bg, l, v, dg);
        for (int p = 1; p <= l; p++) acc = (acc + (tor)dg[p - 1] * ((tor)1 << (q - p * bg))) & m;
        CHECK(acc == ((or_round_top(q, l * bg, v) << (q - l * bg)) & m));
        CHECK(or_mod_switch(q, N, v) < (tor)(2 * N));
    }
    /* keys (binary), noiseless BSK and KSK */
    tor *s = calloc(n, sizeof(tor)), *S = calloc(N, sizeof(tor));
    for (int i = 0; i < n; i++) s[i] = nxt() & 1;
    for (int i = 0; i < N; i++) S[i] = nxt() & 1;
    size_t rows = (size_t)(k + 1) * l, V = (size_t)1 << kb;
    tor *bm = malloc((size_t)n * rows * k * N * sizeof(tor)), *be = calloc((size_t)n * rows * N, sizeof(tor));
    for (size_t i = 0; i < (size_t)n * rows * k * N; i++) bm[i] = nxt() & m;
    tor *bsk = malloc((size_t)n * rows * (k + 1) * N * sizeof(tor));
    or_bsk_gen(P, s, S, bm, be, bsk);
    size_t ke = (size_t)k * N * kt * V;
    tor *km = malloc(ke * n * sizeof(tor)), *kerr = calloc(ke, sizeof(tor));
    for (size_t i = 0; i < ke * n; i++) km[i] = nxt() & m;
    tor *ksk = malloc(ke * (n + 1) * sizeof(tor));
    or_ksk_gen(P, S, s, km, kerr, ksk);
    /* AND of fresh noiseless encryptions decrypts to the truth table */
    tor *mask = malloc(n * sizeof(tor)), *ct = malloc(2 * (n + 1) * sizeof(tor));
    tor *lin = malloc((n + 1) * sizeof(tor)), *out = malloc((n + 1) * sizeof(tor));
    const tor e8 = (tor)1 << (q - 3);
    for (int bx = 0; bx < 2; bx++)
        for (int by = 0; by < 2; by++) {
            for (int j = 0; j < 2; j++) {
                for (int i = 0; i < n; i++) mask[i] = nxt() & m;
                int b = j ? by : bx;
                or_lwe_encrypt(q, n, s, mask, 0, b ? e8 : ((tor)0 - e8) & m, ct + (size_t)j * (n + 1));
            }
            int64_t w[2] = {1, 1};
            or_lincomb(q, n, 2, ct, w, ((tor)0 - e8) & m, lin);
            or_gate_bootstrap(P, bsk, ksk, lin, out);
            tor ph = or_lwe_phase(q, n, s, out);
            int bit = ph != 0 && ph < ((tor)1 << (q - 1));
            CHECK(bit == (bx & by));
        }
    /* a programmable bootstrap with a small table */
    tor f[4] = {0, 1, 2, 3}, *tv = malloc(N * sizeof(tor));
    or_lut_testv(q, N, 4, f, (tor)1 << (q - 3), tv);
    or_pbs(P, bsk, ksk, lin, tv, out);
    free(a); free(x); free(c); free(d); free(s); free(S); free(bm); free(be); free(bsk);
    free(km); free(kerr); free(ksk); free(mask); free(ct); free(lin); free(out); free(tv);
}

int main(void) {
    run(32, 16, 64, 8, 2, 2, 5);
    run(64, 16, 128, 6, 4, 3, 6);
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
