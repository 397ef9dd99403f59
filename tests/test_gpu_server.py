"""The continuous-batching server at the toy parameter set with queries of
tens to hundreds of rows (SELECT SUM(col2) WHERE col1 op c over prefixes of
one table, 8-bit columns): ticks smaller than a level, a budget that holds
two queries at a time, arrivals while others run.  Every sum decrypts to the
plaintext truth, two queries' sums equal the oracle's word for word, and a
query's bits equal those of the same query served alone."""
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
from gpu_util import to_dev, from_dev, empty  # noqa: E402

P = si.TOY
W = 8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_server_toy_queries_against_oracle():
    K = oracle.Keys(P, si.KEY_SEED_BASE + 31)
    ctx = fs.Context(P, K.bsk, K.ksk)
    rows_all = 160
    col1, col2 = si.table(si.DATA_SEED_BASE + 31, rows_all, W)
    c1 = enc_bits(P, K, si.column_bits(col1, W), 311).reshape(rows_all, W, P.n + 1)
    c2 = enc_bits(P, K, si.column_bits(col2, W), 312).reshape(rows_all, W, P.n + 1)
    d1, d2 = to_dev(P, c1), to_dev(P, c2)
    specs = [(60, "eq", int(col1[7]), None), (33, "lt", 90, None), (150, "gt", 200, None),
             (97, "between", 40, 170)]
    lits = {}
    for k, (_, _, a, b) in enumerate(specs):
        lits[k] = (enc_bits(P, K, [(a >> j) & 1 for j in range(W)], 320 + k),
                   enc_bits(P, K, [(b >> j) & 1 for j in range(W)], 330 + k) if b is not None else None)
    dl = {k: (to_dev(P, la), to_dev(P, lb) if lb is not None else None) for k, (la, lb) in lits.items()}

    def serve(indices, budget, stagger, max_batch):
        srv = fs.Server(ctx, budget, max_batch=max_batch)
        outs, ids, pending, ticks = {}, {}, list(indices), 0
        while pending or any(not srv.done(ids[i]) for i in ids):
            if pending and ticks % stagger == 0:
                i = pending.pop(0)
                rows, op, _, _ = specs[i]
                outs[i] = empty(P, fs.sum_width(W, rows), P.n + 1)
                ids[i] = srv.submit(d1[:rows], d2[:rows], rows, W, op, dl[i][0], outs[i], lit_b=dl[i][1])
            srv.step()
            ticks += 1
            assert ticks < 20000
        srv.close()
        return {i: from_dev(P, o) for i, o in outs.items()}, ticks

    probe = fs.Server(ctx, 1 << 34, max_batch=512)
    fixed = probe.bytes_in_use()
    probe.close()
    # temporaries of the two largest queries, not three (rows x ~(w + 3 w) LWEs each)
    per_row = 4 * W * (P.n + 1) * 4
    budget = fixed + 2 * 150 * per_row + (64 << 10)
    say("server: 4 queries, ticks of 512 gates")
    mixed, ticks = serve(range(4), budget, 5, 512)
    say(f"served in {ticks} ticks")
    alone = {}
    for i in (1, 3):
        alone.update(serve([i], 1 << 34, 1, 4096)[0])
    for i in (1, 3):
        assert np.array_equal(mixed[i], alone[i]), i
    for i, (rows, op, a, b) in enumerate(specs):
        c = col1[:rows]
        pred = {"eq": c == a, "lt": c < a, "gt": c > a, "between": (c >= a) & (c <= (b or 0))}[op]
        assert bits_to_int(dec_bits(P, K, mixed[i])) == int((col2[:rows] * pred).sum()), i
    # oracle end to end for the 60-row equality and the 33-row comparison
    lz = C.LazyBackend(P)
    roots = {}
    for i in (0, 1):
        rows, op, _, _ = specs[i]
        la, lb = lits[i]
        sel = []
        for r in range(rows):
            m = C.predicate(lz, op, list(c1[r]), list(la), list(lb) if lb is not None else None)
            sel.append(C.select(lz, m, list(c2[r])))
        roots[i] = C.sum_tree(lz, sel)
    say("oracle", len(lz.nodes), "bootstraps")
    C.evaluate(P, K, lz, threads=oracle.default_threads())
    for i in (0, 1):
        assert np.array_equal(mixed[i], C.resolve(P, roots[i])), i
    ctx.close()
