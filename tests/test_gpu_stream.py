"""Stream ordering of the C ABI: calls enqueue their work and return without
a host synchronization, calls on two streams that share the context's
workspace do not race, and a repeated graphed batch relaunches its cached
graph.  Every result is compared word for word with the oracle or with the
same call run alone."""
import sys

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import circuits as C
from helpers import enc_bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import to_dev, from_dev, context, empty  # noqa: E402

P = si.TOY
W = 4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def toy():
    K = oracle.Keys(P, si.KEY_SEED_BASE + 21)
    return K, context(P, K)


def table(K, rows, seed):
    col1, col2 = si.table(si.DATA_SEED_BASE + seed, rows, W)
    c1 = enc_bits(P, K, si.column_bits(col1, W), seed, tag_hi=1).reshape(rows, W, P.n + 1)
    c2 = enc_bits(P, K, si.column_bits(col2, W), seed, tag_hi=2).reshape(rows, W, P.n + 1)
    return col1, col2, c1, c2


def lit(K, value, seed):
    return enc_bits(P, K, si.column_bits(np.array([value]), W), seed, tag_hi=3).reshape(W, P.n + 1)


def test_back_to_back_calls_without_host_sync(toy):
    """Two masks and two selects enqueued on one stream with no host sync in
    between give the oracle's bits."""
    K, ctx = toy
    rows = 24
    col1, col2, c1, c2 = table(K, rows, 41)
    la, lb = lit(K, int(col1[3]), 42), lit(K, 9, 43)
    d1, d2, dla, dlb = to_dev(P, c1), to_dev(P, c2), to_dev(P, la), to_dev(P, lb)
    s = torch.cuda.Stream()
    m_eq, m_lt = empty(P, rows, P.n + 1), empty(P, rows, P.n + 1)
    s_eq, s_lt = empty(P, rows, W, P.n + 1), empty(P, rows, W, P.n + 1)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        ctx.sql_mask_scan(d1, rows, W, "eq", dla, m_eq)
        ctx.sql_masked_select(m_eq, d2, rows, W, s_eq)
        ctx.sql_mask_scan(d1, rows, W, "lt", dlb, m_lt)
        ctx.sql_masked_select(m_lt, d2, rows, W, s_lt)
    s.synchronize()
    om_eq = C.mask_rows(P, K, "eq", c1, la)
    om_lt = C.mask_rows(P, K, "lt", c1, lb)
    assert np.array_equal(from_dev(P, m_eq), om_eq)
    assert np.array_equal(from_dev(P, m_lt), om_lt)
    assert np.array_equal(from_dev(P, s_eq), C.select_rows(P, K, om_eq, c2))
    assert np.array_equal(from_dev(P, s_lt), C.select_rows(P, K, om_lt, c2))


def test_two_streams_share_the_workspace(toy):
    """A scan on one stream and a scan of another table on a second stream,
    enqueued with no host sync, give the bits of each scan run alone; a
    select on the second stream after it waits for the first reads the
    finished mask."""
    K, ctx = toy
    ra, rb = 48, 40
    a1, a2, ca1, ca2 = table(K, ra, 44)
    b1, _, cb1, _ = table(K, rb, 45)
    la, lb = lit(K, int(a1[5]), 46), lit(K, 7, 47)
    dA1, dA2, dB1, dla, dlb = (to_dev(P, x) for x in (ca1, ca2, cb1, la, lb))
    ref_a, ref_b = empty(P, ra, P.n + 1), empty(P, rb, P.n + 1)
    ref_sel = empty(P, ra, W, P.n + 1)
    ctx.sql_mask_scan(dA1, ra, W, "eq", dla, ref_a)
    ctx.sql_masked_select(ref_a, dA2, ra, W, ref_sel)
    ctx.sql_mask_scan(dB1, rb, W, "lt", dlb, ref_b)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        ma, mb = empty(P, ra, P.n + 1), empty(P, rb, P.n + 1)
        sel = empty(P, ra, W, P.n + 1)
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            ctx.sql_mask_scan(dA1, ra, W, "eq", dla, ma)
        with torch.cuda.stream(s2):
            ctx.sql_mask_scan(dB1, rb, W, "lt", dlb, mb)
            s2.wait_stream(s1)
            ctx.sql_masked_select(ma, dA2, ra, W, sel)
        torch.cuda.synchronize()
        say("two streams, repetition", rep)
        assert torch.equal(ma, ref_a)
        assert torch.equal(mb, ref_b)
        assert torch.equal(sel, ref_sel)
    assert np.array_equal(from_dev(P, ref_a), C.mask_rows(P, K, "eq", ca1, la))


def test_graphed_batch_is_captured_once(toy):
    """A repeated graphed sql_scan_batch relaunches its cached graph (one
    capture, one graph launch per call); every replay, with eager work and
    synchronizations in between, equals the ungraphed batch."""
    K, ctx = toy
    specs = [(9, "eq", 51), (17, "lt", 52), (5, "between", 53)]
    queries = []
    for rows, op, seed in specs:
        col1, col2, c1, c2 = table(K, rows, seed)
        la = lit(K, int(col1[0]), seed + 100)
        lb = lit(K, 12, seed + 200) if op == "between" else None
        queries.append(dict(col=to_dev(P, c1), sel_col=to_dev(P, c2), rows=rows, w=W, op=op,
                            lit_a=to_dev(P, la), lit_b=to_dev(P, lb) if lb is not None else None,
                            mask=empty(P, rows, P.n + 1), sel_out=empty(P, rows, W, P.n + 1)))
    ctx.sql_scan_batch(queries, use_graph=False)
    torch.cuda.synchronize()
    ref = [(q["mask"].clone(), q["sel_out"].clone()) for q in queries]
    _, _, ex1, _ = table(K, 11, 54)
    dex, lex = to_dev(P, ex1), to_dev(P, lit(K, 3, 55))
    mex = empty(P, 11, P.n + 1)
    cap0, launch0, _ = ctx.graph_stats()
    for rep in range(3):
        for q in queries:
            q["mask"].fill_(0)
            q["sel_out"].fill_(0)
        ctx.sql_scan_batch(queries, use_graph=True)
        ctx.sql_mask_scan(dex, 11, W, "gt", lex, mex)  # eager work between replays
        torch.cuda.synchronize()
        for q, (rm, rs) in zip(queries, ref):
            assert torch.equal(q["mask"], rm), rep
            assert torch.equal(q["sel_out"], rs), rep
    cap1, launch1, kept = ctx.graph_stats()
    assert cap1 - cap0 == 1
    assert launch1 - launch0 == 3
    assert kept >= 1
