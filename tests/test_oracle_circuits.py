"""Pins of the oracle's gates and SQL circuits: plaintext truth of every
netlist (exhaustive at 4-bit width) and decrypt-checked encrypted runs."""
import itertools
import random

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import circuits as C
from helpers import enc_bits, dec_bits, bits_to_int

PB = C.PlainBackend()
W = 4


def _bits(v, w=W):
    return [(v >> j) & 1 for j in range(w)]


def test_plain_gate_tables():
    table = {
        "AND": lambda x, y: x & y, "NAND": lambda x, y: 1 - (x & y),
        "OR": lambda x, y: x | y, "NOR": lambda x, y: 1 - (x | y),
        "XOR": lambda x, y: x ^ y, "XNOR": lambda x, y: 1 - (x ^ y),
        "ANDNY": lambda x, y: (1 - x) & y,
    }
    for op, f in table.items():
        for x, y in itertools.product((0, 1), repeat=2):
            assert int(PB.gate(op, x, y)) == f(x, y)
    for x, y, z in itertools.product((0, 1), repeat=3):
        assert int(PB.gate("MAJ", x, y, z)) == int(x + y + z >= 2)


def test_gate_lincombs_on_noiseless_phases():
    """Each gate's constant and weights put the phase of the combination on the
    correct side of zero for every input pair (values +-1/8, q = 32)."""
    q = 32
    e8 = 1 << (q - 3)
    for op, (c8, w) in C.GATES.items():
        for xs in itertools.product((0, 1), repeat=len(w)):
            ph = c8 * e8 + sum(wi * (e8 if b else -e8) for wi, b in zip(w, xs))
            ph %= 1 << q
            got = 1 if 0 < ph < (1 << (q - 1)) else 0
            assert got == int(PB.gate(op, *xs)), (op, xs)
            # and the combined phase stays at least 1/8 away from 0 and 1/2
            d = min(ph, (1 << q) - ph, abs(ph - (1 << (q - 1))))
            assert d >= e8, (op, xs)


def test_plain_predicates_exhaustive():
    for a, c in itertools.product(range(16), repeat=2):
        A, Cb = _bits(a), _bits(c)
        assert PB_bool(C.eq(PB, A, Cb)) == (a == c)
        assert PB_bool(C.lt(PB, A, Cb)) == (a < c)
        assert PB_bool(C.gt(PB, A, Cb)) == (a > c)
    for a, lo, hi in itertools.product(range(16), repeat=3):
        assert PB_bool(C.between(PB, _bits(a), _bits(lo), _bits(hi))) == (lo <= a <= hi)


def PB_bool(x):
    return bool(x)


@pytest.mark.parametrize("w", [1, 2, 3, 5, 8, 16])
def test_plain_predicates_random_widths(w):
    rng = random.Random(w)
    for _ in range(300):
        a, c, d = (rng.randrange(1 << w) for _ in range(3))
        lo, hi = min(c, d), max(c, d)
        assert bool(C.eq(PB, _bits(a, w), _bits(c, w))) == (a == c)
        assert bool(C.eq(PB, _bits(a, w), _bits(a, w)))
        assert bool(C.lt(PB, _bits(a, w), _bits(c, w))) == (a < c)
        assert bool(C.between(PB, _bits(a, w), _bits(lo, w), _bits(hi, w))) == (lo <= a <= hi)


def test_plain_select_and_sum():
    rng = random.Random(3)
    for m, v in itertools.product((0, 1), range(16)):
        out = C.select(PB, bool(m), _bits(v))
        assert bits_to_int([int(b) for b in out]) == (v if m else 0)
    for rows in list(range(1, 10)) + [17, 33]:
        vals = [rng.randrange(256) for _ in range(rows)]
        res = C.sum_tree(PB, [_bits(v, 8) for v in vals])
        assert bits_to_int([int(b) for b in res]) == sum(vals)
        assert len(res) == 8 + (rows - 1).bit_length()


def test_encrypted_gates_tiny(tiny_keys):
    p = si.TINY
    be = C.CipherBackend(p, tiny_keys)
    xs = [0, 1, 0, 1, 0, 1, 0, 1]
    ys = [0, 0, 1, 1, 0, 0, 1, 1]
    zs = [0, 0, 0, 0, 1, 1, 1, 1]
    X = enc_bits(p, tiny_keys, xs, 41)
    Y = enc_bits(p, tiny_keys, ys, 42)
    Z = enc_bits(p, tiny_keys, zs, 43)
    for op in C.GATES:
        for i in range(8):
            args = (X[i], Y[i], Z[i]) if op == "MAJ" else (X[i], Y[i])
            got = oracle.decrypt_bit(p.q, tiny_keys.s, be.gate(op, *args))
            want = int(PB.gate(op, *([xs[i], ys[i], zs[i]] if op == "MAJ" else [xs[i], ys[i]])))
            assert got == want, (op, i)


def test_encrypted_predicates_tiny(tiny_keys):
    p = si.TINY
    rng = random.Random(9)
    pairs = [(rng.randrange(16), rng.randrange(16)) for _ in range(10)] + [(5, 5), (0, 15), (15, 0)]
    for idx, (a, c) in enumerate(pairs):
        be = C.CipherBackend(p, tiny_keys)
        A = list(enc_bits(p, tiny_keys, _bits(a), 100 + idx))
        Cc = list(enc_bits(p, tiny_keys, _bits(c), 200 + idx))
        assert dec_bits(p, tiny_keys, C.eq(be, A, Cc)) == int(a == c)
        assert dec_bits(p, tiny_keys, C.lt(be, A, Cc)) == int(a < c)
        assert dec_bits(p, tiny_keys, C.gt(be, A, Cc)) == int(a > c)
        lo, hi = sorted((c, (c + 5) % 16))
        Lo = list(enc_bits(p, tiny_keys, _bits(lo), 300 + idx))
        Hi = list(enc_bits(p, tiny_keys, _bits(hi), 400 + idx))
        assert dec_bits(p, tiny_keys, C.between(be, A, Lo, Hi)) == int(lo <= a <= hi)
    assert be.count == 4 * 2 - 1 + 4 + 4 + 2 * 4 + 1


def test_encrypted_mask_select_sum_tiny(tiny_keys):
    p = si.TINY
    rows = 6
    col1, col2 = si.table(si.DATA_SEED_BASE + 100, rows, W)
    col1[2] = 7
    c1 = enc_bits(p, tiny_keys, si.column_bits(col1, W), 500).reshape(rows, W, p.n + 1)
    c2 = enc_bits(p, tiny_keys, si.column_bits(col2, W), 501).reshape(rows, W, p.n + 1)
    lit = enc_bits(p, tiny_keys, _bits(7), 502)
    masks = C.mask_rows(p, tiny_keys, "eq", c1, lit)
    sel = C.select_rows(p, tiny_keys, masks, c2)
    m = dec_bits(p, tiny_keys, masks)
    assert m.tolist() == [int(v == 7) for v in col1]
    got = [bits_to_int(r) for r in dec_bits(p, tiny_keys, sel)]
    assert got == [int(v) if int(u) == 7 else 0 for u, v in zip(col1, col2)]
    be = C.CipherBackend(p, tiny_keys)
    total = C.sum_tree(be, [list(r) for r in sel])
    assert bits_to_int(dec_bits(p, tiny_keys, np.stack(total))) == sum(got)


def test_pbs_lut_tiny64():
    """Programmable bootstrap with a table over Z_8 (64-bit torus, padding bit)."""
    p = si.TINY64
    keys = oracle.Keys(p, 77)
    plain = 8
    delta = 1 << (p.q - 4)  # 2^q / (2 * plain)
    f = np.array([(3 * m + 1) % plain for m in range(plain)], dtype=np.uint64)
    tv = oracle.lut_testv(p, plain, f, delta)
    ms = [0, 1, 5, 7]
    masks, errs = si.lwe_randomness(p, 78, len(ms))
    cts = oracle.lwe_encrypt(p, keys.s, masks, errs, [m * delta for m in ms])
    for m, ct in zip(ms, cts):
        out = oracle.pbs(p, keys.bsk, keys.ksk, ct, tv)
        ph = oracle.lwe_phase(p.q, keys.s, out)
        dec = ((ph + delta // 2) // delta) % (2 * plain)
        assert dec == int(f[m]), (m, dec)
