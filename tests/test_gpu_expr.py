"""GPU parity of expression trees (Section 4.3 B) through sql_expr_eval: every
output ciphertext word-for-word against the oracle's evaluation of the same
node list on the same seeded keys and inputs, plus decryption against integer
semantics."""
import sys

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import circuits as C
from helpers import enc_bits, dec_bits, bits_to_int

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_15413_amd as fs  # noqa: E402
from gpu_util import to_dev, from_dev, context, empty  # noqa: E402

_KEYS, _CTX = {}, {}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup(pname):
    if pname not in _KEYS:
        p = si.PARAMS[pname]
        _KEYS[pname] = oracle.Keys(p, si.KEY_SEED_BASE + 9)
        _CTX[pname] = context(p, _KEYS[pname])
    return si.PARAMS[pname], _KEYS[pname], _CTX[pname]


def enc_col(p, K, vals, w, seed, k):
    return enc_bits(p, K, si.column_bits(np.asarray(vals), w), seed, tag_hi=k).reshape(len(vals), w, p.n + 1)


def enc_lit(p, K, v, w, seed):
    return enc_bits(p, K, [(int(v) >> j) & 1 for j in range(w)], seed).reshape(w, p.n + 1)


def run_both(p, K, ctx, nodes, vals_cols, lit_vals, w, seed):
    """Encrypt, evaluate on the GPU and in the oracle; return (gpu, oracle,
    decrypted oracle output, root is value)."""
    rows = len(vals_cols[0])
    cols = [enc_col(p, K, v, w, seed + 1, k) for k, v in enumerate(vals_cols)]
    lits = [enc_lit(p, K, v, w, seed + 2 + i) for i, v in enumerate(lit_vals)]
    value_root = nodes[-1]["kind"] in C.VALUE_KINDS
    out = empty(p, rows, w, p.n + 1) if value_root else empty(p, rows, p.n + 1)
    say(f"expr: {p.name} rows={rows} w={w} nodes={len(nodes)} root={'value' if value_root else 'bool'}")
    ctx.sql_expr_eval(nodes, [to_dev(p, c) for c in cols], rows, w, out, lits=[to_dev(p, x) for x in lits])
    torch.cuda.synchronize()
    ref = C.expr_rows(p, K, nodes, cols, lits, w)
    return from_dev(p, out), ref, dec_bits(p, K, ref), value_root


def check_semantics(dec, nodes, vals_cols, lit_vals, w, value_root):
    for r in range(dec.shape[0]):
        ref = C.expr_plain(nodes, [int(v[r]) for v in vals_cols], [int(x) for x in lit_vals], w)
        got = bits_to_int(dec[r]) if value_root else bool(dec[r])
        assert got == ref, r


def test_paper_example_parity():
    """age > 18 AND salary < 1000 (11-bit values) with rows at the boundaries."""
    p, K, ctx = setup("toy")
    w = 11
    age = [18, 19, 19, 0, 2047, 40, 19, 100, 17]
    sal = [999, 999, 1000, 0, 2047, 12, 998, 1001, 5]
    nodes = si.paper_where_example()
    got, ref, dec, vr = run_both(p, K, ctx, nodes, [age, sal], [], w, 3100)
    assert np.array_equal(got, ref)
    check_semantics(dec, nodes, [age, sal], [], w, vr)


@pytest.mark.parametrize("op", si.CMP_NAMES)
def test_every_comparison_against_literal(op):
    p, K, ctx = setup("toy")
    w, rows = 5, 7
    vals = si.uniform_ints(si.DATA_SEED_BASE + 3200, si.TAG_DATA, rows, w)
    lit = int(vals[2])
    nodes = [{"kind": "column", "col": 0}, {"kind": "literal", "lit": 0}, {"kind": "cmp", "op": op, "a": 0, "b": 1}]
    got, ref, dec, vr = run_both(p, K, ctx, nodes, [vals], [lit], w, 3210)
    assert np.array_equal(got, ref)
    check_semantics(dec, nodes, [vals], [lit], w, vr)


@pytest.mark.parametrize("seed,root", [(0, "bool"), (1, "value"), (2, "bool"), (3, "value"), (4, "bool"),
                                       (5, "value")])
def test_random_trees_parity(seed, root):
    p, K, ctx = setup("toy")
    w, rows = 4, 9
    nodes = si.random_expr(si.DATA_SEED_BASE + 3300 + seed, 2, 1, w, depth=3, root=root)
    vals = si.uniform_ints(si.DATA_SEED_BASE + 3400 + seed, si.TAG_DATA, rows * 2 + 1, w)
    cols = [vals[:rows], vals[rows:2 * rows]]
    got, ref, dec, vr = run_both(p, K, ctx, nodes, cols, [int(vals[-1])], w, 3500 + 10 * seed)
    assert np.array_equal(got, ref), nodes
    check_semantics(dec, nodes, cols, [int(vals[-1])], w, vr)


def test_max_min_ite_and_plain_roots():
    """Value roots that are a column, a constant, MAX, MIN and an ITE; a
    boolean root that is a double negation."""
    p, K, ctx = setup("toy")
    w, rows = 4, 6
    a = [3, 9, 9, 0, 15, 7]
    b = [5, 2, 9, 15, 0, 8]
    trees = [
        [{"kind": "column", "col": 1}],
        [{"kind": "const", "value": 11}],
        [{"kind": "column", "col": 0}, {"kind": "column", "col": 1}, {"kind": "max", "a": 0, "b": 1}],
        [{"kind": "column", "col": 0}, {"kind": "column", "col": 1}, {"kind": "min", "a": 0, "b": 1}],
        [{"kind": "column", "col": 0}, {"kind": "const", "value": 8}, {"kind": "cmp", "op": "ge", "a": 0, "b": 1},
         {"kind": "column", "col": 1}, {"kind": "ite", "c": 2, "a": 3, "b": 1}],
        [{"kind": "column", "col": 0}, {"kind": "column", "col": 1}, {"kind": "cmp", "op": "le", "a": 0, "b": 1},
         {"kind": "not", "a": 2}, {"kind": "not", "a": 3}],
    ]
    for t, nodes in enumerate(trees):
        got, ref, dec, vr = run_both(p, K, ctx, nodes, [a, b], [], w, 3600 + 10 * t)
        assert np.array_equal(got, ref), t
        check_semantics(dec, nodes, [a, b], [], w, vr)


def test_q64_tree_parity():
    p, K, ctx = setup("tiny64")
    w, rows = 3, 5
    a = [1, 6, 4, 7, 0]
    b = [6, 1, 4, 0, 7]
    nodes = [{"kind": "column", "col": 0}, {"kind": "column", "col": 1}, {"kind": "cmp", "op": "ne", "a": 0, "b": 1},
             {"kind": "max", "a": 0, "b": 1}, {"kind": "const", "value": 5}, {"kind": "cmp", "op": "gt", "a": 3, "b": 4},
             {"kind": "xor", "a": 2, "b": 5}]
    got, ref, dec, vr = run_both(p, K, ctx, nodes, [a, b], [], w, 3700)
    assert np.array_equal(got, ref)
    check_semantics(dec, nodes, [a, b], [], w, vr)


def test_expr_errors_and_empty():
    p, K, ctx = setup("toy")
    w, rows = 2, 3
    col = to_dev(p, enc_col(p, K, [0, 1, 2], w, 3800, 0))
    out = empty(p, rows, p.n + 1)
    bad = [
        [{"kind": "not", "a": 1}, {"kind": "column", "col": 0}],                       # operand after node
        [{"kind": "column", "col": 0}, {"kind": "and", "a": 0, "b": 0}],               # AND of values
        [{"kind": "column", "col": 3}],                                                # column out of range
        [{"kind": "column", "col": 0}, {"kind": "cmp", "op": "zz", "a": 0, "b": 0}],   # unknown operator
        [{"kind": "column", "col": 0}, {"kind": "cmp", "op": "eq", "a": 0, "b": 0},
         {"kind": "ite", "c": 0, "a": 0, "b": 0}],                                     # ITE on a value
    ]
    for nodes in bad:
        with pytest.raises(fs.FheError):
            ctx.sql_expr_eval(nodes, [col], rows, w, out)
    with pytest.raises(fs.FheError):
        ctx.sql_expr_eval([{"kind": "column", "col": 0}], [col], rows, 0, out)
    with pytest.raises(fs.FheError):
        ctx.sql_expr_eval([], [col], rows, w, out)
    # zero rows: validated, nothing launched
    ctx.sql_expr_eval(si.paper_where_example(0, 0), [col], 0, w, out)


@pytest.mark.slow
def test_std_paper_example_sampled():
    """The paper's example over 4096 rows at the standard gate parameters in
    one call; the oracle recomputes three sampled rows."""
    import paper_2510_15413_amd as fs_
    p = si.STD
    K = oracle.Keys(p, si.KEY_SEED_BASE + 2)
    ctx = context(p, K)
    w, rows = 11, 4096
    age = si.uniform_ints(si.DATA_SEED_BASE + 3900, si.TAG_DATA, rows, w)
    sal = si.uniform_ints(si.DATA_SEED_BASE + 3901, si.TAG_DATA, rows, w)
    cols = [enc_col(p, K, age, w, 3910, 0), enc_col(p, K, sal, w, 3911, 1)]
    nodes = si.paper_where_example()
    out = empty(p, rows, p.n + 1)
    say("std paper example: 4096 rows")
    ctx.sql_expr_eval(nodes, [to_dev(p, c) for c in cols], rows, w, out)
    torch.cuda.synchronize()
    got = from_dev(p, out)
    dec = dec_bits(p, K, got)
    assert dec.tolist() == [int(a > 18 and s < 1000) for a, s in zip(age.tolist(), sal.tolist())]
    sample = [0, 1777, rows - 1]
    ref = C.expr_rows(p, K, nodes, [c[sample] for c in cols], [], w)
    assert np.array_equal(got[sample], ref)
    del fs_
