"""Obliviousness (the leakage of Section 5's ideal functionality: the query's
AST with literals redacted and the table's row count, nothing else): the
ordered launch schedule of the GPU path -- every blind-rotation and
key-switching launch with its ciphertext count -- is the same for real data,
an all-zero table and a different literal, for every predicate, the masked
select, the masked SUM and an expression tree."""
import sys

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from helpers import enc_bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_15413_amd as fs  # noqa: E402
from gpu_util import to_dev, context, empty  # noqa: E402

P = si.TOY
_K = {}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup():
    if "k" not in _K:
        _K["k"] = oracle.Keys(P, si.KEY_SEED_BASE + 11)
        _K["ctx"] = context(P, _K["k"])
    return _K["k"], _K["ctx"]


def enc_col(K, vals, w, seed):
    return to_dev(P, enc_bits(P, K, si.column_bits(np.asarray(vals), w), seed).reshape(len(vals), w, P.n + 1))


def enc_lit(K, v, w, seed):
    return to_dev(P, enc_bits(P, K, [(int(v) >> j) & 1 for j in range(w)], seed).reshape(w, P.n + 1))


def schedule(ctx, fn):
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    fn()
    torch.cuda.synchronize()
    log = ctx.timing_log()
    ctx.timing_enable(False)
    return log


@pytest.mark.parametrize("op", ["eq", "lt", "gt", "between"])
def test_scan_schedule_is_data_independent(op):
    K, ctx = setup()
    rows, w = 37, 5
    vals = si.uniform_ints(si.DATA_SEED_BASE + 4000, si.TAG_DATA, rows, w)
    cols = {"real": enc_col(K, vals, w, 4001), "zero": enc_col(K, np.zeros(rows, dtype=np.int64), w, 4002)}
    sel = enc_col(K, vals[::-1].copy(), w, 4003)
    lits = {"a": (enc_lit(K, 9, w, 4004), enc_lit(K, 20, w, 4005)),
            "b": (enc_lit(K, 0, w, 4006), enc_lit(K, 31, w, 4007))}
    logs = []
    for cname, lname in (("real", "a"), ("zero", "a"), ("real", "b")):
        col, (la, lb) = cols[cname], lits[lname]
        mask, out = empty(P, rows, P.n + 1), empty(P, rows, w, P.n + 1)

        def run():
            ctx.sql_mask_scan(col, rows, w, op, la, mask, lit_b=lb if op == "between" else None)
            ctx.sql_masked_select(mask, sel, rows, w, out)
        logs.append(schedule(ctx, run))
    say(op, "launches", len(logs[0]))
    assert len(logs[0]) > 0
    assert logs[0] == logs[1] == logs[2]


def test_sum_and_expression_schedules_are_data_independent():
    K, ctx = setup()
    rows, w = 21, 4
    vals = si.uniform_ints(si.DATA_SEED_BASE + 4100, si.TAG_DATA, rows, w)
    real, zero = enc_col(K, vals, w, 4101), enc_col(K, np.zeros(rows, dtype=np.int64), w, 4102)
    ones = enc_col(K, np.full(rows, 15), w, 4103)
    logs = []
    for col in (real, zero):
        masks = empty(P, rows, P.n + 1)
        width = fs.sum_width(w, rows)
        s = empty(P, width, P.n + 1)

        def run():
            ctx.sql_mask_scan(col, rows, w, "lt", enc_lit(K, 7, w, 4104), masks)
            ctx.sql_masked_sum(masks, col, rows, w, s)
        logs.append(schedule(ctx, run))
    assert len(logs[0]) > 0 and logs[0] == logs[1]
    # an expression tree whose plaintext constants (the redacted literals) differ
    elogs = []
    for consts in ((3, 12), (0, 15)):
        nodes = [{"kind": "column", "col": 0}, {"kind": "const", "value": consts[0]},
                 {"kind": "cmp", "op": "ge", "a": 0, "b": 1}, {"kind": "column", "col": 1},
                 {"kind": "const", "value": consts[1]}, {"kind": "cmp", "op": "ne", "a": 3, "b": 4},
                 {"kind": "and", "a": 2, "b": 5}, {"kind": "max", "a": 0, "b": 3},
                 {"kind": "ite", "c": 6, "a": 7, "b": 1}]
        for cset in ((real, ones), (zero, zero)):
            out = empty(P, rows, w, P.n + 1)
            elogs.append(schedule(ctx, lambda: ctx.sql_expr_eval(nodes, list(cset), rows, w, out)))
    assert len(elogs[0]) > 0
    assert all(e == elogs[0] for e in elogs)
