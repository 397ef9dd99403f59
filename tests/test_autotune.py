"""The autotuner: candidate grid, cache miss (every candidate timed, the
fastest applied and stored), cache hit (applied without running), and --
on the GPU -- identical output bits under every candidate setting."""
import json

import pytest

import seeded_inputs as si
from paper_2510_15413_amd import autotune


def test_candidate_grid_covers_the_knobs():
    c = autotune.candidates(si.STD, batches=(4096, 65536))
    assert {x["row_pass"] for x in c} == {16, 8}
    assert {x["split_groups"] for x in c} == {-1, 0}
    assert {x["max_batch"] for x in c} == {4096, 65536}
    assert len(c) == 8
    t = autotune.candidates(si.TOY, batches=(4096,))
    assert {x["split_groups"] for x in t} == {-1}


class FakeCtx:
    """Records set_tuning calls (the knobs' effect is the library's)."""

    def __init__(self, p):
        self.p = p
        self.applied = []

    def set_tuning(self, **kw):
        self.applied.append(dict(kw))


def test_tune_miss_then_hit(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "_gpu_name", lambda: "test-gpu")
    cache = tmp_path / "tune.json"
    ctx = FakeCtx(si.TOY)
    cands = [{"max_batch": b, "row_pass": 4, "split_groups": -1} for b in (16, 32, 64)]
    cost = {16: 0.003, 32: 0.001, 64: 0.002}
    calls = []

    def run():
        import time
        mb = ctx.applied[-1]["max_batch"]
        calls.append(mb)
        time.sleep(cost[mb])
    best, times = autotune.tune(ctx, "w", run, cands=cands, reps=3, cache_path=str(cache))
    assert best["max_batch"] == 32
    assert ctx.applied[-1] == best
    assert len(times) == 3 and len(calls) == 3 * 4
    stored = json.loads(cache.read_text())
    key = autotune.cache_key(si.TOY, "w")
    assert stored[key]["best"] == best
    calls.clear()
    ctx2 = FakeCtx(si.TOY)
    best2, _ = autotune.tune(ctx2, "w", run, cands=cands, cache_path=str(cache))
    assert best2 == best and ctx2.applied == [best] and calls == []
    # another parameter set misses
    ctx3 = FakeCtx(si.STD)
    autotune.tune(ctx3, "w", lambda: None, cands=cands, cache_path=str(cache))
    assert len(json.loads(cache.read_text())) == 2


@pytest.mark.gpu
def test_every_candidate_gives_the_same_bits(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import numpy as np
    import oracle
    import paper_2510_15413_amd as fs
    from helpers import enc_bits
    from gpu_util import to_dev, empty
    p = si.TOY
    K = oracle.Keys(p, si.KEY_SEED_BASE + 5)
    ctx = fs.Context(p, K.bsk, K.ksk)
    w = 4
    qs = []
    for t, (rows, op) in enumerate(((37, "eq"), (80, "lt"), (21, "between"))):
        c1, c2 = si.table(si.DATA_SEED_BASE + 60 + t, rows, w)
        e1 = enc_bits(p, K, si.column_bits(c1, w), 60 + t).reshape(rows, w, p.n + 1)
        e2 = enc_bits(p, K, si.column_bits(c2, w), 70 + t).reshape(rows, w, p.n + 1)
        la = enc_bits(p, K, si.column_bits(np.array([int(c1[0])]), w), 80 + t).reshape(w, p.n + 1)
        lb = enc_bits(p, K, si.column_bits(np.array([13]), w), 90 + t).reshape(w, p.n + 1)
        qs.append(dict(col=to_dev(p, e1), sel_col=to_dev(p, e2), rows=rows, w=w, op=op, lit_a=to_dev(p, la),
                       lit_b=to_dev(p, lb) if op == "between" else None, mask=empty(p, rows, p.n + 1),
                       sel_out=empty(p, rows, w, p.n + 1)))
    outs = []

    def run():
        ctx.sql_scan_batch(qs, use_graph=True)
        torch.cuda.synchronize()
        outs.append([(q["mask"].clone(), q["sel_out"].clone()) for q in qs])
    cands = [{"max_batch": b, "row_pass": rp, "split_groups": sg}
             for b in (16, 100, 65536) for rp in (4, 2) for sg in (-1, 0, 1 << 20)]
    best, times = autotune.tune(ctx, "bits", run, cands=cands, cache_path=str(tmp_path / "t.json"))
    assert len(times) == len(cands)
    got = ctx.get_tuning()
    for k, v in best.items():
        assert got[k] == v, k
    ref = outs[0]
    for o in outs[1:]:
        for (m, s), (rm, rs) in zip(o, ref):
            assert torch.equal(m, rm) and torch.equal(s, rs)
    ctx.close()
