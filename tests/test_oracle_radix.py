"""Pins of the radix (programmable bootstrapping) circuits: plaintext truth
of every netlist, exhaustive at two blocks, and encrypted runs on the small
64-bit parameter set checked after decryption."""
import itertools
import random

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import circuits as C

PB = C.RadixPlainBackend()


def blocks(v, nb):
    return [(v >> (4 * i)) & 15 for i in range(nb)]


def value(bl):
    return sum(int(b) << (4 * i) for i, b in enumerate(bl))


def test_tables_stay_in_range():
    for name, tab in C.radix_tables().items():
        assert len(tab) == C.RADIX_P and all(0 <= x < C.RADIX_P for x in tab), name


def test_plain_compare_exhaustive_two_blocks():
    for a, c in itertools.product(range(256), repeat=2):
        for op, f in (("lt", a < c), ("eq", a == c), ("gt", a > c)):
            assert C.radix_compare(PB, op, blocks(a, 2), blocks(c, 2)) == (16 if f else 0), (op, a, c)


@pytest.mark.parametrize("nb", [3, 4, 8])
def test_plain_compare_select_add_random(nb):
    rng = random.Random(nb)
    M = 1 << (4 * nb)
    for _ in range(500):
        a, c, v = rng.randrange(M), rng.randrange(M), rng.randrange(M)
        if rng.random() < 0.1:
            c = a
        m = C.radix_compare(PB, "lt", blocks(a, nb), blocks(c, nb))
        assert m == (16 if a < c else 0)
        assert value(C.radix_select(PB, m, blocks(v, nb))) == (v if a < c else 0)
        assert value(C.radix_add(PB, blocks(a, nb), blocks(v, nb))) == (a + v) % M


def test_plain_sum_wraps():
    rng = random.Random(5)
    for rows in (1, 2, 3, 7, 16):
        vals = [rng.randrange(1 << 32) for _ in range(rows)]
        assert value(C.radix_sum(PB, [blocks(v, 8) for v in vals])) == sum(vals) % (1 << 32)


def _enc_blocks(p, K, vals, nb, seed):
    delta = 1 << (p.q - 6)
    bl = np.array([blocks(int(v), nb) for v in vals], dtype=np.uint64).ravel()
    m, e = si.lwe_randomness(p, seed, bl.size)
    return oracle.lwe_encrypt(p, K.s, m, e, bl * np.uint64(delta)).reshape(len(vals), nb, p.n + 1)


def _dec_blocks(p, K, cts):
    delta = 1 << (p.q - 6)
    out = []
    for c in cts.reshape(-1, p.n + 1):
        ph = oracle.lwe_phase(p.q, K.s, c)
        out.append(((ph + delta // 2) // delta) % (2 * C.RADIX_P))
    return np.array(out).reshape(cts.shape[:-1])


def test_encrypted_radix_small_64bit():
    p = si.TINY64
    K = oracle.Keys(p, 91)
    nb = 2
    a_vals, c_val, v_vals = [3, 200, 77], 77, [15, 255, 128]
    A = _enc_blocks(p, K, a_vals, nb, 1)
    Cc = _enc_blocks(p, K, [c_val], nb, 2)[0]
    V = _enc_blocks(p, K, v_vals, nb, 3)
    be = C.RadixCipherBackend(p, K)
    sels = []
    for r, a in enumerate(a_vals):
        for op, f in (("lt", a < c_val), ("eq", a == c_val), ("gt", a > c_val)):
            m = C.radix_compare(be, op, list(A[r]), list(Cc))
            assert _dec_blocks(p, K, m[None])[0] == (16 if f else 0), (a, op)
        m = C.radix_compare(be, "lt", list(A[r]), list(Cc))
        sel = C.radix_select(be, m, list(V[r]))
        assert value(_dec_blocks(p, K, np.stack(sel))) == (v_vals[r] if a < c_val else 0)
        sels.append(sel)
    tot = C.radix_sum(be, sels)
    want = sum(v for a, v in zip(a_vals, v_vals) if a < c_val) % 256
    assert value(_dec_blocks(p, K, np.stack(tot))) == want


def test_lazy_radix_evaluator_matches_eager():
    """The depth-parallel radix evaluator gives the eager backend's
    ciphertexts word for word (compare, select and a 3-row SUM)."""
    p = si.TINY64
    K = oracle.Keys(p, 93)
    nb = 3
    a_vals, c_val, v_vals = [5, 300, 4000], 300, [17, 4095, 1234]
    A = _enc_blocks(p, K, a_vals, nb, 4)
    Cc = _enc_blocks(p, K, [c_val], nb, 5)[0]
    V = _enc_blocks(p, K, v_vals, nb, 6)

    def circuit(be):
        ms = [C.radix_compare(be, "lt", list(A[r]), list(Cc)) for r in range(3)]
        ss = [C.radix_select(be, ms[r], list(V[r])) for r in range(3)]
        return ms, ss, C.radix_sum(be, ss)

    em, es, et = circuit(C.RadixCipherBackend(p, K))
    lz = C.LazyRadixBackend(p)
    lm, ls, lt = circuit(lz)
    C.evaluate_radix(p, K, lz, threads=4)
    assert np.array_equal(C.resolve_radix(p, K, lm), np.stack(em))
    assert np.array_equal(C.resolve_radix(p, K, ls), np.stack([np.stack(s) for s in es]))
    assert np.array_equal(C.resolve_radix(p, K, lt), np.stack(et))
