"""Pins of the oracle's TFHE primitives against brute force, closed forms and
exact identities (the paper prints no numeric test vector for this path, so
each pin comes from the mathematics of the TFHE definitions it cites)."""
import itertools
import random

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from helpers import py_monomial, torus_dist


def _rand_poly(rng, q, N):
    return np.array([rng.randrange(1 << q) for _ in range(N)], dtype=np.uint64)


# ------------------------------------------------------------- negacyclic

@pytest.mark.parametrize("q,N", [(32, 1), (32, 2), (32, 8), (32, 64), (64, 16), (64, 64), (8, 16), (20, 32)])
def test_negacyclic_vs_full_product_reduction(q, N):
    rng = random.Random(q * 1000 + N)
    for _ in range(3):
        a, b = _rand_poly(rng, q, N), _rand_poly(rng, q, N)
        full = [0] * (2 * N)
        for i in range(N):
            for j in range(N):
                full[i + j] += int(a[i]) * int(b[j])
        # reduce X^N = -1 on the full (degree < 2N-1) product
        expect = [(full[i] - full[i + N]) % (1 << q) for i in range(N)]
        assert [int(v) for v in oracle.negacyclic_mul(q, a, b)] == expect


def test_negacyclic_algebra():
    rng = random.Random(7)
    q, N = 32, 32
    a, b, c = (_rand_poly(rng, q, N) for _ in range(3))
    ab = oracle.negacyclic_mul(q, a, b)
    assert np.array_equal(ab, oracle.negacyclic_mul(q, b, a))
    assert np.array_equal(oracle.negacyclic_mul(q, ab, c),
                          oracle.negacyclic_mul(q, a, oracle.negacyclic_mul(q, b, c)))
    # X^N = -1: multiplying by X^(N-1) then X gives -a.
    x1 = np.zeros(N, dtype=np.uint64); x1[1] = 1
    xn1 = np.zeros(N, dtype=np.uint64); xn1[N - 1] = 1
    neg = oracle.negacyclic_mul(q, oracle.negacyclic_mul(q, a, xn1), x1)
    assert [int(v) for v in neg] == [(-int(v)) % (1 << q) for v in a]


@pytest.mark.parametrize("q,N", [(32, 16), (64, 8)])
def test_monomial_matches_exponent_rule(q, N):
    rng = random.Random(3)
    a = _rand_poly(rng, q, N)
    for e in range(0, 2 * N):
        assert [int(v) for v in oracle.monomial_mul(q, e, a)] == py_monomial(q, N, e, a)
        mono = np.zeros(N, dtype=np.uint64)
        mono[e % N] = 1 if e < N else (1 << q) - 1
        assert np.array_equal(oracle.monomial_mul(q, e, a), oracle.negacyclic_mul(q, a, mono))


# ---------------------------------------------------------- decomposition

@pytest.mark.parametrize("bg,l", [(2, 2), (3, 2), (2, 3), (1, 4)])
def test_decomposition_exhaustive_tiny_torus(bg, l):
    q = 8
    half = 1 << (q - l * bg - 1) if q > l * bg else 0
    recon = {}
    for digs in itertools.product(range(-(1 << (bg - 1)), 1 << (bg - 1)), repeat=l):
        r = sum(d << (q - (p + 1) * bg) for p, d in enumerate(digs)) % (1 << q)
        assert r not in recon  # the digit tuples are in bijection with the grid
        recon[r] = list(digs)
    assert len(recon) == 1 << (l * bg)
    for x in range(1 << q):
        d = oracle.decompose(q, bg, l, x)
        assert all(-(1 << (bg - 1)) <= v < (1 << (bg - 1)) for v in d)
        r = sum(v << (q - (p + 1) * bg) for p, v in enumerate(d)) % (1 << q)
        assert recon[r] == d
        # r is the nearest grid point, ties rounded up
        assert torus_dist(q, r, x) <= half
        if torus_dist(q, r, x) == half and half:
            assert (r - x) % (1 << q) == half


@pytest.mark.parametrize("q,bg,l", [(32, 8, 2), (32, 7, 3), (64, 6, 4), (32, 2, 5), (64, 16, 4)])
def test_decomposition_random_wide(q, bg, l):
    rng = random.Random(q + bg + l)
    half = 1 << (q - l * bg - 1) if q > l * bg else 0
    vals = [rng.randrange(1 << q) for _ in range(3000)]
    vals += [0, (1 << q) - 1, half, max(half - 1, 0), ((1 << q) - half) % (1 << q), 1 << (q - 1)]
    for x in vals:
        d = oracle.decompose(q, bg, l, x)
        assert all(-(1 << (bg - 1)) <= v < (1 << (bg - 1)) for v in d)
        r = sum(v << (q - (p + 1) * bg) for p, v in enumerate(d)) % (1 << q)
        assert r % (1 << max(q - l * bg, 0)) == 0
        assert torus_dist(q, r, x) <= half


def test_mod_switch_exhaustive():
    q, N = 10, 4
    step = (1 << q) // (2 * N)
    for x in range(1 << q):
        m = oracle.mod_switch(q, N, x)
        assert 0 <= m < 2 * N
        assert torus_dist(q, m * step, x) <= step // 2
        if torus_dist(q, m * step, x) == step // 2:
            assert (m * step - x) % (1 << q) == step // 2


# ----------------------------------------------------- ciphertext identities

def _keys(p, seed):
    s, S = si.secret_keys(p, seed)
    return s, S


def _round_grid(q, bits, x):
    step = 1 << (q - bits)
    return (((int(x) + step // 2) // step) * step) % (1 << q)


@pytest.mark.parametrize("pname", ["tiny", "tiny64"])
def test_sample_extract_phase(pname):
    p = si.PARAMS[pname]
    s, S = _keys(p, 5)
    rng = random.Random(1)
    for _ in range(5):
        C = _rand_poly(rng, p.q, (p.k + 1) * p.N)
        se = oracle.sample_extract(p, C)
        assert oracle.lwe_phase(p.q, oracle.extracted_key(S), se) == int(oracle.glwe_phase(p, S, C)[0])


@pytest.mark.parametrize("pname", ["tiny", "tiny64"])
def test_glwe_encrypt_phase_is_message_plus_error(pname):
    p = si.PARAMS[pname]
    s, S = _keys(p, 6)
    rng = random.Random(2)
    masks = _rand_poly(rng, p.q, p.k * p.N)
    errs = _rand_poly(rng, 8, p.N)
    msg = _rand_poly(rng, p.q, p.N)
    ct = oracle.glwe_encrypt(p, S, masks, errs, msg)
    ph = oracle.glwe_phase(p, S, ct)
    assert [int(v) for v in ph] == [(int(m) + int(e)) % (1 << p.q) for m, e in zip(msg, errs)]


@pytest.mark.parametrize("pname", ["tiny", "toy", "tiny64"])
@pytest.mark.parametrize("m", [0, 1, 3])
def test_ext_product_noiseless_identity(pname, m):
    """Noiseless GGSW(m) (random masks, zero errors): the phase of the external
    product is m times the phase of the gadget-rounded GLWE input."""
    p = si.PARAMS[pname]
    s, S = _keys(p, 7)
    rows = (p.k + 1) * p.l
    masks = si.torus(9, 3, rows * p.k * p.N, p.q).reshape(rows, p.k, p.N)
    errs = np.zeros((rows, p.N), dtype=np.uint64)
    G = oracle.ggsw_encrypt(p, S, m, masks, errs)
    rng = random.Random(m)
    C = _rand_poly(rng, p.q, (p.k + 1) * p.N)
    out = oracle.ext_product(p, G, C)
    Cr = np.array([_round_grid(p.q, p.l * p.bg_bits, v) for v in C], dtype=np.uint64)
    want = [(m * int(v)) % (1 << p.q) for v in oracle.glwe_phase(p, S, Cr)]
    assert [int(v) for v in oracle.glwe_phase(p, S, out)] == want
    # trivial GGSW(1) (zero masks, zero errors) returns the rounded input itself
    G1 = oracle.ggsw_encrypt(p, S, 1, np.zeros_like(masks), errs)
    assert np.array_equal(oracle.ext_product(p, G1, C), Cr)


@pytest.mark.parametrize("pname", ["tiny", "tiny64"])
def test_blind_rotate_trivial_key_rotates_exactly(pname):
    """With a trivial bootstrapping key (zero masks and errors) blind rotation
    returns (0, X^{-phi} testv), phi = MS(b) - sum MS(a_i) s_i mod 2N."""
    p = si.PARAMS[pname]
    s, S = _keys(p, 8)
    rows = (p.k + 1) * p.l
    zero_m = np.zeros((p.n, rows, p.k, p.N), dtype=np.uint64)
    zero_e = np.zeros((p.n, rows, p.N), dtype=np.uint64)
    bsk = oracle.bsk_gen(p, s, S, zero_m, zero_e)
    rng = random.Random(11)
    step = 1 << (p.q - p.l * p.bg_bits)
    for t in range(6):
        lwe = _rand_poly(rng, p.q, p.n + 1)
        testv = np.array([rng.randrange(1 << (p.l * p.bg_bits)) * step for _ in range(p.N)], dtype=np.uint64)
        acc = oracle.blind_rotate(p, bsk, lwe, testv)
        phi = (oracle.mod_switch(p.q, p.N, lwe[p.n])
               - sum(oracle.mod_switch(p.q, p.N, lwe[i]) * int(s[i]) for i in range(p.n))) % (2 * p.N)
        assert not acc[:p.k * p.N].any()
        assert [int(v) for v in acc[p.k * p.N:]] == py_monomial(p.q, p.N, (2 * p.N - phi) % (2 * p.N), testv)


@pytest.mark.parametrize("pname", ["tiny", "toy", "tiny64"])
def test_keyswitch_noiseless_identity(pname):
    """Noiseless key-switching table: the output phase under s is
    b' - sum_i round_{t*b}(a'_i) s'_i exactly."""
    p = si.PARAMS[pname]
    s, S = _keys(p, 12)
    sx = oracle.extracted_key(S)
    V = 1 << p.ks_bits
    masks = si.torus(13, 5, p.k * p.N * p.ks_t * V * p.n, p.q).reshape(p.k * p.N, p.ks_t, V, p.n)
    errs = np.zeros((p.k * p.N, p.ks_t, V), dtype=np.uint64)
    ksk = oracle.ksk_gen(p, sx, s, masks, errs)
    rng = random.Random(5)
    for _ in range(4):
        big = _rand_poly(rng, p.q, p.k * p.N + 1)
        out = oracle.keyswitch(p, ksk, big)
        want = int(big[-1])
        for i in range(p.k * p.N):
            want -= _round_grid(p.q, p.ks_t * p.ks_bits, big[i]) * int(sx[i])
        assert oracle.lwe_phase(p.q, s, out) == want % (1 << p.q)


def test_lut_testv_boxes_exact():
    """Every phase in the half-open box of width N/p centred on m N/p rotates
    the test polynomial to f(m) at coefficient 0 (trivial key, q = 64)."""
    p = si.TINY64
    N = p.N
    for plain in (4, 8, 32):
        f = np.array([(7 * m + 3) % plain for m in range(plain)], dtype=np.uint64)
        delta = 1 << (p.q - 6)
        tv = oracle.lut_testv(p, plain, f, delta)
        for phi in range(2 * N):
            coef0 = py_monomial(p.q, N, (2 * N - phi) % (2 * N), tv)[0]
            # box index of phi: nearest multiple of N/plain (half-up)
            m = ((phi * plain + N // 2) // N) % (2 * plain)
            if m < plain:
                assert coef0 == (int(f[m]) * delta) % (1 << p.q), (plain, phi)
            else:  # phases with the padding bit set give the negated table
                assert coef0 == (-int(f[m - plain]) * delta) % (1 << p.q), (plain, phi)
