"""Pins of the oracle's expression-tree evaluation (Homomorphic Expression
Tree, Section 4.3 B): the circuits against integer semantics (exhaustive
comparisons and selections at 3 bits, seeded random DAGs at 4 bits), the
If-Then-Else linear step on every input, and encrypted runs decrypted against
the same integer semantics."""
import itertools

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import circuits as C
from helpers import enc_bits, dec_bits, bits_to_int

PB = C.PlainBackend()


def _bits(v, w):
    return [bool((v >> j) & 1) for j in range(w)]


def _plain_root(nodes, cols, lits, w):
    out = C.expr_eval(PB, nodes, [_bits(c, w) for c in cols], [_bits(x, w) for x in lits], w)
    return bits_to_int(out) if isinstance(out, list) else bool(out)


def test_compare_ops_exhaustive():
    w = 3
    for op in si.CMP_NAMES:
        nodes = [{"kind": "column", "col": 0}, {"kind": "column", "col": 1},
                 {"kind": "cmp", "op": op, "a": 0, "b": 1}]
        for a, b in itertools.product(range(8), repeat=2):
            ref = {"eq": a == b, "ne": a != b, "lt": a < b, "le": a <= b, "gt": a > b, "ge": a >= b}[op]
            assert _plain_root(nodes, [a, b], [], w) == ref, (op, a, b)


def test_selection_exhaustive():
    w = 3
    for kind in ("max", "min"):
        nodes = [{"kind": "column", "col": 0}, {"kind": "column", "col": 1}, {"kind": kind, "a": 0, "b": 1}]
        for a, b in itertools.product(range(8), repeat=2):
            assert _plain_root(nodes, [a, b], [], w) == (max(a, b) if kind == "max" else min(a, b))
    nodes = [{"kind": "column", "col": 0}, {"kind": "column", "col": 1}, {"kind": "column", "col": 2},
             {"kind": "const", "value": 4}, {"kind": "cmp", "op": "lt", "a": 0, "b": 3},
             {"kind": "ite", "c": 4, "a": 1, "b": 2}]
    for a, x, y in itertools.product(range(8), repeat=3):
        assert _plain_root(nodes, [a, x, y], [], w) == (x if a < 4 else y)


def test_mux_linear_step_every_input():
    """AND(c,x) + ANDNY(c,y) + 1/8 is a valid bit equal to c ? x : y."""
    for c, x, y in itertools.product((False, True), repeat=3):
        assert C.mux(PB, c, x, y) == (x if c else y)
    # the two AND terms are never both TRUE, which is what keeps the sum a bit
    with pytest.raises(ValueError):
        PB.lin([True, True], [1, 1], 1)


def test_boolean_connectives_and_not():
    w = 2
    for kind in ("and", "or", "xor"):
        nodes = [{"kind": "column", "col": 0}, {"kind": "const", "value": 1},
                 {"kind": "cmp", "op": "eq", "a": 0, "b": 1},
                 {"kind": "column", "col": 1}, {"kind": "const", "value": 2},
                 {"kind": "cmp", "op": "ge", "a": 3, "b": 4},
                 {"kind": kind, "a": 2, "b": 5}, {"kind": "not", "a": 6}]
        for a, b in itertools.product(range(4), repeat=2):
            p, q = a == 1, b >= 2
            ref = {"and": p and q, "or": p or q, "xor": p != q}[kind]
            assert _plain_root(nodes, [a, b], [], w) == (not ref)


def test_random_trees_against_integer_semantics():
    w = 4
    for seed in range(60):
        root = "bool" if seed % 2 == 0 else "value"
        nodes = si.random_expr(si.DATA_SEED_BASE + 500 + seed, 3, 2, w, depth=3, root=root)
        vals = si.uniform_ints(si.DATA_SEED_BASE + 700 + seed, si.TAG_DATA, 5 * 8, w).reshape(8, 5)
        for row in vals.tolist():
            cols, lits = row[:3], row[3:]
            assert _plain_root(nodes, cols, lits, w) == C.expr_plain(nodes, cols, lits, w), (seed, row)


def test_paper_example_semantics():
    """age > 18 AND salary < 1000 over 11-bit values."""
    w = 11
    nodes = si.paper_where_example()
    for age, salary in [(18, 999), (19, 999), (19, 1000), (40, 0), (0, 0), (2047, 2047), (19, 12)]:
        assert _plain_root(nodes, [age, salary], [], w) == (age > 18 and salary < 1000)


def test_validation():
    w = 2
    with pytest.raises(ValueError):  # operand after the node
        C.expr_eval(PB, [{"kind": "not", "a": 1}, {"kind": "column", "col": 0}], [_bits(0, w)], [], w)
    with pytest.raises(ValueError):  # and of values
        C.expr_eval(PB, [{"kind": "column", "col": 0}, {"kind": "and", "a": 0, "b": 0}], [_bits(0, w)], [], w)
    with pytest.raises(ValueError):  # compare of booleans
        nodes = [{"kind": "column", "col": 0}, {"kind": "cmp", "op": "eq", "a": 0, "b": 0},
                 {"kind": "cmp", "op": "eq", "a": 1, "b": 1}]
        C.expr_eval(PB, nodes, [_bits(0, w)], [], w)


def test_not_is_exact_negation(tiny_keys):
    p = si.TINY
    ct = enc_bits(p, tiny_keys, [1, 0], si.DATA_SEED_BASE + 41)
    be = C.CipherBackend(p, tiny_keys)
    for c in ct:
        n = be.neg(c)
        assert oracle.lwe_phase(p.q, tiny_keys.s, n) == (-oracle.lwe_phase(p.q, tiny_keys.s, c)) % (1 << p.q)
    assert dec_bits(p, tiny_keys, [be.neg(c) for c in ct]).tolist() == [0, 1]


@pytest.mark.parametrize("seed,root", [(3, "bool"), (4, "value"), (5, "bool")])
def test_encrypted_trees_decrypt_to_integer_semantics(tiny_keys, seed, root):
    p = si.TINY
    w = 3
    rows = 4
    nodes = si.random_expr(si.DATA_SEED_BASE + 900 + seed, 2, 1, w, depth=2, root=root)
    vals = si.uniform_ints(si.DATA_SEED_BASE + 950 + seed, si.TAG_DATA, rows * 3, w).reshape(rows, 3)
    cols = [enc_bits(p, tiny_keys, si.column_bits(vals[:, k], w), si.DATA_SEED_BASE + 960 + seed, tag_hi=k)
            .reshape(rows, w, p.n + 1) for k in range(2)]
    lit = enc_bits(p, tiny_keys, si.column_bits(vals[:1, 2], w), si.DATA_SEED_BASE + 970 + seed).reshape(w, p.n + 1)
    out = C.expr_rows(p, tiny_keys, nodes, cols, [lit], w)
    dec = dec_bits(p, tiny_keys, out)
    for r in range(rows):
        ref = C.expr_plain(nodes, [int(vals[r, 0]), int(vals[r, 1])], [int(vals[0, 2])], w)
        got = bits_to_int(dec[r]) if root == "value" else bool(dec[r])
        assert got == ref, (seed, r, nodes)


def test_encrypted_paper_example(tiny_keys):
    p = si.TINY
    w = 11
    vals = [(18, 999), (19, 999), (19, 1000), (200, 5)]
    age = enc_bits(p, tiny_keys, si.column_bits(np.array([a for a, _ in vals]), w), si.DATA_SEED_BASE + 980)
    sal = enc_bits(p, tiny_keys, si.column_bits(np.array([b for _, b in vals]), w), si.DATA_SEED_BASE + 981)
    cols = [age.reshape(len(vals), w, p.n + 1), sal.reshape(len(vals), w, p.n + 1)]
    out = C.expr_rows(p, tiny_keys, si.paper_where_example(), cols, [], w)
    assert dec_bits(p, tiny_keys, out).tolist() == [int(a > 18 and b < 1000) for a, b in vals]
