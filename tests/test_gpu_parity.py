"""GPU parity: every ciphertext the HIP library produces through the C ABI is
compared word for word with the CPU oracle on the same seeded keys and inputs
(the arithmetic is integer, so the tolerance is zero)."""
import random
import sys

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import circuits as C
from helpers import enc_bits, dec_bits, bits_to_int, edge_lwe, edge_big

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_15413_amd as fs  # noqa: E402
from gpu_util import to_dev, from_dev, context, empty  # noqa: E402

KERNELS = ["mfma", "plain"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_KEYS = {}
_CTX = {}


def keys_for(pname):
    if pname not in _KEYS:
        p = si.PARAMS[pname]
        _KEYS[pname] = oracle.Keys(p, si.KEY_SEED_BASE + 7)
    return _KEYS[pname]


def ctx_for(pname):
    if pname not in _CTX:
        _CTX[pname] = context(si.PARAMS[pname], keys_for(pname))
    return _CTX[pname]


def rand_lwe(p, count, seed):
    return si.torus(seed, 99, count * (p.n + 1), p.q).reshape(count, p.n + 1)


# ------------------------------------------------------------ key material

@pytest.mark.parametrize("pname", ["tiny", "toy", "tiny64"])
def test_device_keygen_matches_oracle(pname):
    p = si.PARAMS[pname]
    say("keygen", pname)
    K = keys_for(pname)
    s, S, bsk, ksk = fs.tfhe_keygen(p, K.seed)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(p, s), K.s)
    assert np.array_equal(from_dev(p, S), K.S)
    assert np.array_equal(from_dev(p, bsk), K.bsk.ravel())
    assert np.array_equal(from_dev(p, ksk), K.ksk.ravel())


@pytest.mark.parametrize("pname", ["toy", "tiny64"])
def test_device_encrypt_and_phase_match_oracle(pname):
    p = si.PARAMS[pname]
    K = keys_for(pname)
    count, start, tag_hi = 37, 5, 3
    mus = si.torus(4, 9, count, p.q)
    masks, errs = si.lwe_randomness(p, 21, count, tag_hi=tag_hi, start=start)
    want = oracle.lwe_encrypt(p, K.s, masks, errs, mus)
    got = fs.tfhe_lwe_encrypt(p, 21, to_dev(p, K.s), to_dev(p, mus), start=start, tag_hi=tag_hi)
    assert np.array_equal(from_dev(p, got), want)
    ph = from_dev(p, fs.tfhe_lwe_phase(p, to_dev(p, K.s), got))
    assert [int(v) for v in ph] == [oracle.lwe_phase(p.q, K.s, c) for c in want]


def test_device_rng_matches_seeded_inputs():
    got = fs.tfhe_rng_fill(1234, 77, 1000, start=33).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, si.raw(1234, 77, 1000, start=33))


# ------------------------------------------------------------- bootstrapping

@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("pname", ["tiny", "toy", "tiny64"])
@pytest.mark.parametrize("B", [1, 17, 40])
def test_bootstrap_parity(kernel, pname, B):
    p = si.PARAMS[pname]
    K = keys_for(pname)
    ctx = ctx_for(pname)
    ctx.set_kernel(kernel)
    say("bootstrap", kernel, pname, B)
    lwe = rand_lwe(p, B, 1000 + B)
    out = empty(p, B, p.k * p.N + 1)
    ctx.tfhe_bootstrap_batch(to_dev(p, lwe), out)
    # a random test polynomial too
    tv = si.torus(77, 5, p.N, p.q)
    out2 = empty(p, B, p.k * p.N + 1)
    ctx.tfhe_bootstrap_batch(to_dev(p, lwe), out2, testv=to_dev(p, tv))
    torch.cuda.synchronize()
    g1, g2 = from_dev(p, out), from_dev(p, out2)
    gtv = oracle.gate_testv(p)
    idx = list(range(B)) if B <= 17 else [0, 1, 15, 16, 17, 31, 32, B - 1]
    want = oracle.parallel_map(lambda i: (oracle.bootstrap(p, K.bsk, lwe[i], gtv),
                                          oracle.bootstrap(p, K.bsk, lwe[i], tv)), idx)
    for i, (w1, w2) in zip(idx, want):
        assert np.array_equal(g1[i], w1), (kernel, pname, B, i)
        assert np.array_equal(g2[i], w2), (kernel, pname, B, i)
    ctx.set_kernel("mfma")


@pytest.mark.parametrize("pname", ["tiny", "toy", "tiny64"])
def test_keyswitch_parity(pname):
    p = si.PARAMS[pname]
    K = keys_for(pname)
    ctx = ctx_for(pname)
    B = 70
    big = si.torus(5, 98, B * (p.k * p.N + 1), p.q).reshape(B, p.k * p.N + 1)
    out = empty(p, B, p.n + 1)
    ctx.tfhe_keyswitch_batch(to_dev(p, big), out)
    torch.cuda.synchronize()
    g = from_dev(p, out)
    for i in range(B):
        assert np.array_equal(g[i], oracle.keyswitch(p, K.ksk, big[i])), i


@pytest.mark.parametrize("op", list(C.GATES))
def test_gate_batch_parity(op):
    p = si.TOY
    K = keys_for("toy")
    ctx = ctx_for("toy")
    B = 12
    bits = si.bits(31, 1, 3 * B).reshape(3, B)
    X = [enc_bits(p, K, bits[j], 300 + j) for j in range(3)]
    out = empty(p, B, p.n + 1)
    ctx.tfhe_gate_batch(op, to_dev(p, X[0]), to_dev(p, X[1]), out,
                        z=to_dev(p, X[2]) if op == "MAJ" else None)
    torch.cuda.synchronize()
    g = from_dev(p, out)
    nin = 3 if op == "MAJ" else 2
    want = C.gate_batch(p, K, op, [[X[j][i] for j in range(nin)] for i in range(B)])
    assert np.array_equal(g, want)
    pb = C.PlainBackend()
    assert dec_bits(p, K, g).tolist() == [int(pb.gate(op, *[bits[j][i] for j in range(nin)])) for i in range(B)]


# --------------------------------------------------------------- SQL circuits

def _table(p, K, rows, w, seed, table_id=0):
    col1, col2 = si.table(si.DATA_SEED_BASE + seed, rows, w, table_id)
    c1 = enc_bits(p, K, si.column_bits(col1, w), seed * 10 + 1, tag_hi=table_id).reshape(rows, w, p.n + 1)
    c2 = enc_bits(p, K, si.column_bits(col2, w), seed * 10 + 2, tag_hi=table_id).reshape(rows, w, p.n + 1)
    return col1, col2, c1, c2


def _lit(p, K, v, w, seed):
    return enc_bits(p, K, [(int(v) >> j) & 1 for j in range(w)], seed)


def test_toy_query_full_parity():
    """32 rows of 4-bit columns: mask(col1 == 7) (4 XNOR + 3 AND per row), then
    mask AND each bit of col2: all 352 bootstrap outputs bit-exact."""
    p = si.TOY
    K = keys_for("toy")
    ctx = ctx_for("toy")
    rows, w = 32, 4
    col1, col2, c1, c2 = _table(p, K, rows, w, 1)
    lit = _lit(p, K, 7, w, 77)
    mask, sel = empty(p, rows, p.n + 1), empty(p, rows, w, p.n + 1)
    ctx.sql_mask_scan(to_dev(p, c1), rows, w, "eq", to_dev(p, lit), mask)
    ctx.sql_masked_select(mask, to_dev(p, c2), rows, w, sel)
    torch.cuda.synchronize()
    om = C.mask_rows(p, K, "eq", c1, lit)
    osel = C.select_rows(p, K, om, c2)
    assert np.array_equal(from_dev(p, mask), om)
    assert np.array_equal(from_dev(p, sel), osel)
    assert dec_bits(p, K, om).tolist() == [int(v == 7) for v in col1]
    got = [bits_to_int(b) for b in dec_bits(p, K, osel)]
    assert got == [int(b) if a == 7 else 0 for a, b in zip(col1, col2)]


@pytest.mark.parametrize("op", ["lt", "gt", "between", "eq"])
def test_toy_predicates_parity(op):
    p = si.TOY
    K = keys_for("toy")
    ctx = ctx_for("toy")
    rows, w = 13, 5
    col1, col2, c1, c2 = _table(p, K, rows, w, 2)
    lo, hi = 9, 22
    la = _lit(p, K, lo if op == "between" else int(col1[3]), w, 81)
    lb = _lit(p, K, hi, w, 82) if op == "between" else None
    mask = empty(p, rows, p.n + 1)
    ctx.sql_mask_scan(to_dev(p, c1), rows, w, op, to_dev(p, la), mask,
                      lit_b=to_dev(p, lb) if lb is not None else None)
    torch.cuda.synchronize()
    om = C.mask_rows(p, K, op, c1, la, lb)
    assert np.array_equal(from_dev(p, mask), om)
    c = lo if op == "between" else int(col1[3])
    truth = {"eq": lambda a: a == c, "lt": lambda a: a < c, "gt": lambda a: a > c,
             "between": lambda a: lo <= a <= hi}[op]
    assert dec_bits(p, K, om).tolist() == [int(truth(int(a))) for a in col1]


@pytest.mark.parametrize("rows", [1, 2, 5, 8])
def test_masked_sum_parity(rows):
    p = si.TINY
    K = keys_for("tiny")
    ctx = ctx_for("tiny")
    w = 3
    col1, col2, c1, c2 = _table(p, K, rows, w, 3)
    m_bits = [(i * 7 + 1) % 3 != 0 for i in range(rows)]
    m = enc_bits(p, K, m_bits, 55)
    width = fs.sum_width(w, rows)
    out = empty(p, width, p.n + 1)
    got_w = ctx.sql_masked_sum(to_dev(p, m), to_dev(p, c2), rows, w, out)
    torch.cuda.synchronize()
    assert got_w == width
    be = C.CipherBackend(p, K)
    sel = [C.select(be, m[r], list(c2[r])) for r in range(rows)]
    want = np.stack(C.sum_tree(be, sel)) if rows > 1 else np.stack(sel[0])
    assert np.array_equal(from_dev(p, out), want)
    assert bits_to_int(dec_bits(p, K, want)) == sum(int(v) for v, b in zip(col2, m_bits) if b)


@pytest.mark.parametrize("use_graph", [False, True])
def test_scan_batch_isolation_and_parity(use_graph):
    """Uneven tables with mixed predicates in one level-batched schedule give the
    same bits as each table alone, and match the oracle."""
    p = si.TOY
    K = keys_for("toy")
    ctx = ctx_for("toy")
    w = 4
    specs = [(5, "eq"), (17, "lt"), (9, "between")]
    qs, alone, tabs = [], [], []
    for t, (rows, op) in enumerate(specs):
        col1, col2, c1, c2 = _table(p, K, rows, w, 10 + t, table_id=t)
        la = _lit(p, K, int(col1[0]) if op == "eq" else 6, w, 90 + t)
        lb = _lit(p, K, 12, w, 95 + t) if op == "between" else None
        d = dict(col=to_dev(p, c1), sel_col=to_dev(p, c2), rows=rows, w=w, op=op, lit_a=to_dev(p, la),
                 lit_b=to_dev(p, lb) if lb is not None else None, mask=empty(p, rows, p.n + 1),
                 sel_out=empty(p, rows, w, p.n + 1))
        qs.append(d)
        tabs.append((col1, col2, c1, c2, la, lb))
        m1, s1 = empty(p, rows, p.n + 1), empty(p, rows, w, p.n + 1)
        ctx.sql_mask_scan(d["col"], rows, w, op, d["lit_a"], m1, lit_b=d["lit_b"])
        ctx.sql_masked_select(m1, d["sel_col"], rows, w, s1)
        alone.append((m1, s1))
    # three runs in a row with eager work and synchronizations between them;
    # every run (each a fresh capture and replay on the graph path) must
    # reproduce the tables computed alone
    for rep in range(3):
        for d in qs:
            d["mask"].fill_(0x5A5A5A5A)
            d["sel_out"].fill_(-1)
        scratch = torch.arange(4096, device="cuda", dtype=torch.int64).sum()
        torch.cuda.synchronize()
        ctx.sql_scan_batch(qs, use_graph=use_graph)
        torch.cuda.synchronize()
        del scratch
        for t, (d, (m1, s1)) in enumerate(zip(qs, alone)):
            assert torch.equal(d["mask"], m1), (rep, t)
            assert torch.equal(d["sel_out"], s1), (rep, t)
    # oracle end to end on the first two rows of every table
    for t, (d, (col1, col2, c1, c2, la, lb)) in enumerate(zip(qs, tabs)):
        op = specs[t][1]
        om = C.mask_rows(p, K, op, c1[:2], la, lb)
        assert np.array_equal(from_dev(p, d["mask"])[:2], om), t
        assert np.array_equal(from_dev(p, d["sel_out"])[:2], C.select_rows(p, K, om, c2[:2])), t


def test_errors_are_reported():
    p = si.TOY
    ctx = ctx_for("toy")
    x = empty(p, 4, p.n + 1)
    with pytest.raises(fs.FheError):
        ctx.sql_mask_scan(x, 4, 0, "eq", x, x)
    bad = si.Params("bad", 32, 64, 2, 256, 8, 2, 2, 5, 20, 25)
    with pytest.raises(fs.FheError):
        fs.Context(bad, np.zeros(10, dtype=np.uint64), np.zeros(10, dtype=np.uint64))
    # B = 0 is a no-op
    ctx.tfhe_bootstrap_batch(x, x, B=0)


def test_tuning_knobs_do_not_change_bits():
    """Splitting levels into small launches and the alternative MFMA row-pass
    variant give the same bits as the defaults."""
    p = si.TOY
    K = keys_for("toy")
    ctx = ctx_for("toy")
    rows, w = 21, 4
    col1, col2, c1, c2 = _table(p, K, rows, w, 20)
    lit = _lit(p, K, int(col1[2]), w, 120)
    outs = []
    for mb, rp in ((65536, 0), (16, 0), (48, 2), (65536, 4)):
        ctx.set_tuning(max_batch=mb, row_pass=rp)
        m, sel = empty(p, rows, p.n + 1), empty(p, rows, w, p.n + 1)
        ctx.sql_mask_scan(to_dev(p, c1), rows, w, "eq", to_dev(p, lit), m)
        ctx.sql_masked_select(m, to_dev(p, c2), rows, w, sel)
        torch.cuda.synchronize()
        outs.append((from_dev(p, m), from_dev(p, sel)))
    ctx.set_tuning(max_batch=65536, row_pass=0)
    for m, sel in outs[1:]:
        assert np.array_equal(m, outs[0][0]) and np.array_equal(sel, outs[0][1])
    om = C.mask_rows(p, K, "eq", c1[:3], lit)
    assert np.array_equal(outs[0][0][:3], om)
    with pytest.raises(fs.FheError):
        ctx.set_tuning(row_pass=3)


def test_server_isolation_parity_and_admission():
    """A query's encrypted SUM is the same bits alone, mixed with other queries
    in the continuous-batching server, and through the direct calls; it
    matches the oracle; a tiny budget queues queries instead of failing."""
    p = si.TINY
    K = keys_for("tiny")
    ctx = ctx_for("tiny")
    w = 4
    specs = [(7, "eq"), (12, "lt"), (5, "gt"), (1, "lt")]
    qs = []
    for t, (rows, op) in enumerate(specs):
        col1, col2, c1, c2 = _table(p, K, rows, w, 40 + t, table_id=t)
        lit = _lit(p, K, int(col1[0]) if op == "eq" else 9, w, 140 + t)
        width = fs.sum_width(w, rows)
        qs.append(dict(col=to_dev(p, c1), sum_col=to_dev(p, c2), rows=rows, w=w, op=op, lit_a=to_dev(p, lit),
                       width=width, host=(col1, col2, c1, c2, lit)))

    def run_server(indices, budget, stagger):
        srv = fs.Server(ctx, budget, max_batch=64)
        outs, ids = {}, {}
        pending = list(indices)
        ticks = 0
        while pending or any(not srv.done(ids[i]) for i in ids):
            if pending and (ticks % stagger == 0):
                i = pending.pop(0)
                outs[i] = empty(p, qs[i]["width"], p.n + 1)
                q = qs[i]
                ids[i] = srv.submit(q["col"], q["sum_col"], q["rows"], q["w"], q["op"], q["lit_a"], outs[i])
            srv.step()
            ticks += 1
            assert ticks < 5000
        srv.close()
        return {i: from_dev(p, outs[i]) for i in outs}

    alone = {}
    for i in range(len(qs)):
        alone.update(run_server([i], 1 << 34, 1))
    mixed = run_server(list(range(len(qs))), 1 << 34, 3)
    for i in range(len(qs)):
        assert np.array_equal(alone[i], mixed[i]), i
    # direct calls give the same bits
    q = qs[1]
    m = empty(p, q["rows"], p.n + 1)
    ctx.sql_mask_scan(q["col"], q["rows"], w, q["op"], q["lit_a"], m)
    s_dir = empty(p, q["width"], p.n + 1)
    ctx.sql_masked_sum(m, q["sum_col"], q["rows"], w, s_dir)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(p, s_dir), alone[1])
    # oracle end to end for queries 0 and 3, decrypted truth for all
    for i in (0, 3):
        col1, col2, c1, c2, lit = qs[i]["host"]
        be = C.CipherBackend(p, K)
        masks = [C.predicate(be, qs[i]["op"], list(c1[r]), list(lit)) for r in range(qs[i]["rows"])]
        sel = [C.select(be, masks[r], list(c2[r])) for r in range(qs[i]["rows"])]
        want = np.stack(C.sum_tree(be, sel)) if qs[i]["rows"] > 1 else np.stack(sel[0])
        assert np.array_equal(alone[i], want), i
    for i, q in enumerate(qs):
        col1, col2, c1, c2, lit = q["host"]
        c = int(col1[0]) if q["op"] == "eq" else 9
        pred = {"eq": col1 == c, "lt": col1 < c, "gt": col1 > c}[q["op"]]
        assert bits_to_int(dec_bits(p, K, alone[i])) == int((col2 * pred).sum()), i
    # admission: a budget just above one query's needs still completes all of them
    srv = fs.Server(ctx, 1 << 34, max_batch=64)
    base = srv.bytes_in_use()
    srv.close()
    tight = run_server(list(range(len(qs))), base + (24 << 10), 1)
    for i in range(len(qs)):
        assert np.array_equal(tight[i], alone[i]), i
    with pytest.raises(fs.FheError):
        fs.Server(ctx, 1024, max_batch=64)


def test_client_decrypt_and_filter_zero_rows():
    """Algorithm 1's client end: decrypt the server's selected rows on the
    device and drop the zero rows; what remains is exactly the matching rows
    with a non-zero value."""
    from paper_2510_15413_amd import client
    p = si.TOY
    K = keys_for("toy")
    ctx = ctx_for("toy")
    rows, w = 24, 4
    col1, col2, c1, c2 = _table(p, K, rows, w, 40)
    c = int(col1[5])
    lit = _lit(p, K, c, w, 41)
    mask, sel = empty(p, rows, p.n + 1), empty(p, rows, w, p.n + 1)
    ctx.sql_mask_scan(to_dev(p, c1), rows, w, "eq", to_dev(p, lit), mask)
    ctx.sql_masked_select(mask, to_dev(p, c2), rows, w, sel)
    torch.cuda.synchronize()
    key = to_dev(p, K.s)
    idx, vals = client.filter_zero_rows(p, key, sel)
    want = [r for r in range(rows) if col1[r] == c and col2[r] != 0]
    assert idx.cpu().tolist() == want
    assert vals[:, 0].cpu().tolist() == [int(col2[r]) for r in want]
    assert client.decrypt_values(p, key, to_dev(p, c2)).cpu().tolist() == [int(v) for v in col2]


def test_server_expression_queries():
    """SELECT SUM(col) WHERE <expression tree> through the server: the same
    bits alone, mixed with single-predicate queries, and through the direct
    calls (sql_expr_eval, then sql_masked_sum); oracle end to end for one
    query and decrypted truth for all."""
    p = si.TINY
    K = keys_for("tiny")
    ctx = ctx_for("tiny")
    w, rows = 4, 9
    vals = si.uniform_ints(si.DATA_SEED_BASE + 4200, si.TAG_DATA, 3 * rows, w).reshape(3, rows)
    cts = [enc_bits(p, K, si.column_bits(vals[k], w), 4210 + k).reshape(rows, w, p.n + 1) for k in range(3)]
    dcols = [to_dev(p, c) for c in cts]
    lit = _lit(p, K, 6, w, 4220).reshape(w, p.n + 1)
    trees = [
        [{"kind": "column", "col": 0}, {"kind": "literal", "lit": 0}, {"kind": "cmp", "op": "gt", "a": 0, "b": 1},
         {"kind": "column", "col": 1}, {"kind": "const", "value": 10}, {"kind": "cmp", "op": "lt", "a": 3, "b": 4},
         {"kind": "and", "a": 2, "b": 5}],
        [{"kind": "column", "col": 0}, {"kind": "column", "col": 1}, {"kind": "max", "a": 0, "b": 1},
         {"kind": "const", "value": 12}, {"kind": "cmp", "op": "le", "a": 2, "b": 3}, {"kind": "not", "a": 4}],
        [{"kind": "column", "col": 1}, {"kind": "const", "value": 3}, {"kind": "cmp", "op": "ne", "a": 0, "b": 1}],
    ]
    width = fs.sum_width(w, rows)

    def run_server(which, stagger):
        srv = fs.Server(ctx, 1 << 34, max_batch=64)
        outs, ids, pending, ticks = {}, {}, list(which), 0
        while pending or any(not srv.done(ids[i]) for i in ids):
            if pending and ticks % stagger == 0:
                i = pending.pop(0)
                outs[i] = empty(p, width, p.n + 1)
                if i < len(trees):
                    ids[i] = srv.submit_expr(trees[i], dcols, rows, w, dcols[2], outs[i], lits=[to_dev(p, lit)])
                else:  # a single-predicate query in the mix
                    ids[i] = srv.submit(dcols[0], dcols[2], rows, w, "lt", to_dev(p, lit), outs[i])
            srv.step()
            ticks += 1
            assert ticks < 5000
        srv.close()
        return {i: from_dev(p, outs[i]) for i in outs}

    alone = {}
    for i in range(len(trees)):
        alone.update(run_server([i], 1))
    mixed = run_server([3, 0, 1, 2], 2)
    for i in range(len(trees)):
        assert np.array_equal(alone[i], mixed[i]), i
        # direct calls
        m, s_dir = empty(p, rows, p.n + 1), empty(p, width, p.n + 1)
        ctx.sql_expr_eval(trees[i], dcols, rows, w, m, lits=[to_dev(p, lit)])
        ctx.sql_masked_sum(m, dcols[2], rows, w, s_dir)
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(p, s_dir), alone[i]), i
        pred = [C.expr_plain(trees[i], [int(vals[0][r]), int(vals[1][r])], [6], w) for r in range(rows)]
        assert bits_to_int(dec_bits(p, K, alone[i])) == sum(int(vals[2][r]) for r in range(rows) if pred[r]), i
    # oracle end to end for the first tree
    masks = C.expr_rows(p, K, trees[0], [cts[0], cts[1]], [lit], w)
    be = C.CipherBackend(p, K)
    sel = [C.select(be, masks[r], list(cts[2][r])) for r in range(rows)]
    assert np.array_equal(alone[0], np.stack(C.sum_tree(be, sel)))


@pytest.mark.parametrize("db", [1, 2])
def test_digit_cache_row_passes_and_server_workspace_check(db):
    """Several row passes with digits formed per group (the first pass caches
    each group's digits in global memory, the later passes reload them) give
    the default bits; a server whose blind-rotation workspace was sized under
    the default tuning refuses, with an error and without launching, a tick
    under this tuning, which needs the larger workspace."""
    p = si.TOY
    K = keys_for("toy")
    ctx = ctx_for("toy")
    rows, w = 19, 4
    col1, col2, c1, c2 = _table(p, K, rows, w, 60 + db)
    lit = _lit(p, K, 6, w, 62 + db)
    srv = fs.Server(ctx, 1 << 34, max_batch=64)
    outs = []
    try:
        for rp, dbk in ((0, 0), (2, db)):
            ctx.set_tuning(row_pass=rp, digit_blocks=dbk)
            m, sel = empty(p, rows, p.n + 1), empty(p, rows, w, p.n + 1)
            ctx.sql_mask_scan(to_dev(p, c1), rows, w, "lt", to_dev(p, lit), m)
            ctx.sql_masked_select(m, to_dev(p, c2), rows, w, sel)
            torch.cuda.synchronize()
            outs.append((from_dev(p, m), from_dev(p, sel)))
        out = empty(p, fs.sum_width(w, rows), p.n + 1)
        srv.submit(to_dev(p, c1), to_dev(p, c2), rows, w, "lt", to_dev(p, lit), out)
        with pytest.raises(fs.FheError, match="workspace"):
            for _ in range(64):
                srv.step()
    finally:
        ctx.set_tuning(row_pass=0, digit_blocks=0)
        torch.cuda.synchronize()
        srv.close()
    assert np.array_equal(outs[1][0], outs[0][0]) and np.array_equal(outs[1][1], outs[0][1])
    assert np.array_equal(dec_bits(p, K, outs[0][0]).astype(bool), col1 < 6)


# (q, N) pairs the MFMA kernel instantiates beyond the named parameter sets,
# with their row-pass variants: both accumulator components in LDS (q = 32,
# N = 512; q = 64, N <= 256), shifted key copies (q = 64, N <= 256), several
# row passes with the digit cache (q = 64, N = 1024) and the 32-bit 2048 ring
RINGS = [(32, 512, (8, 4)), (32, 2048, (8,)), (64, 64, (0,)), (64, 256, (0,)), (64, 1024, (0,))]


@pytest.mark.parametrize("q,N,passes", RINGS)
def test_bootstrap_every_ring_size(q, N, passes):
    """Gate bootstrapping at every other ring size the kernel supports gives
    the oracle's bits (n = 8 so that the oracle stays fast), for a batch of
    18 ciphertexts: one full workgroup and a ragged one."""
    bg, l, ksb, kst, sg = (7, 3, 2, 5, 25) if q == 32 else (6, 4, 3, 6, 51)
    p = si.Params(f"ring{q}_{N}", q, 8, 1, N, bg, l, ksb, kst, 20, sg)
    K = oracle.Keys(p, si.KEY_SEED_BASE + 50 + N + q)
    ctx = context(p, K)
    B = 18
    lwe = si.torus(9, N + q, B * (p.n + 1), p.q).reshape(B, p.n + 1)
    tv = oracle.gate_testv(p)
    idx = [0, 7, 15, 16, 17]
    want = oracle.parallel_map(lambda i: oracle.bootstrap(p, K.bsk, lwe[i], tv), idx)
    for rp in passes:
        say("ring", q, N, "row pass", rp)
        ctx.set_tuning(row_pass=rp)
        out = empty(p, B, p.N + 1)
        ctx.tfhe_bootstrap_batch(to_dev(p, lwe), out)
        torch.cuda.synchronize()
        g = from_dev(p, out)
        for i, w in zip(idx, want):
            assert np.array_equal(g[i], w), (q, N, rp, i)
    ctx.close()


@pytest.mark.parametrize("q,ks_bits,ks_t", [(32, 3, 8), (32, 4, 8), (64, 4, 8), (32, 2, 4), (32, 1, 8), (32, 1, 4)])
def test_keyswitch_staging_variants(q, ks_bits, ks_t):
    """Key switching with other key-switching bases, with an LWE of 41 words
    (a ragged word tile) and 300 ciphertexts (a ragged ciphertext group): the
    oracle's bits.  With 32-bit words the int8 MFMA form runs for every base
    whose one-hot bytes of a lane (16/2^b (i, j) pairs) span at most two
    table rows, i.e. 16/2^b <= t -- bases 2^3, 2^4, 2^2 x 4 and 2^1 x 8 --
    and the LDS gather kernel for 2^1 x 4 (8 pairs over 4 levels); with
    64-bit words the gather kernel (one staged coefficient per barrier)."""
    p = si.Params(f"ks{q}_{ks_bits}_{ks_t}", q, 40, 1, 256, 8 if q == 32 else 6, 2 if q == 32 else 4,
                  ks_bits, ks_t, 20, 25 if q == 32 else 51)
    K = oracle.Keys(p, si.KEY_SEED_BASE + 70 + ks_bits + q)
    ctx = context(p, K)
    B = 300
    big = si.torus(5, 99 + ks_bits, B * (p.k * p.N + 1), p.q).reshape(B, p.k * p.N + 1)
    out = empty(p, B, p.n + 1)
    ctx.tfhe_keyswitch_batch(to_dev(p, big), out)
    torch.cuda.synchronize()
    g = from_dev(p, out)
    for i in (0, 1, 127, 255, 256, 299):
        assert np.array_equal(g[i], oracle.keyswitch(p, K.ksk, big[i])), (q, ks_bits, i)
    ctx.close()


@pytest.mark.parametrize("kernel", KERNELS)
def test_edge_inputs_toy(kernel):
    """Blind rotation + extraction and key switching on the method's boundary
    inputs (exact modulus-switch ties, masks switching to 0, N and 2N-1, bbar
    = 0, the all-zero ciphertext, bodies at exactly +-1/8, key-switch rounding
    ties and the tie below 2^q): every output word equals the oracle's."""
    p = si.TOY
    K = keys_for("toy")
    ctx = ctx_for("toy")
    ctx.set_kernel(kernel)
    lwe = edge_lwe(p, 31)
    B = len(lwe)
    out = empty(p, B, p.N + 1)
    ks = empty(p, B, p.n + 1)
    ctx.tfhe_bootstrap_batch(to_dev(p, lwe), out)
    ctx.tfhe_keyswitch_batch(out, ks)
    big = edge_big(p, 32)
    ks2 = empty(p, len(big), p.n + 1)
    ctx.tfhe_keyswitch_batch(to_dev(p, big), ks2)
    torch.cuda.synchronize()
    ctx.set_kernel("mfma")
    g, gk, gk2 = from_dev(p, out), from_dev(p, ks), from_dev(p, ks2)
    tv = oracle.gate_testv(p)
    want = oracle.parallel_map(lambda i: oracle.bootstrap(p, K.bsk, lwe[i], tv), range(B))
    for i in range(B):
        assert np.array_equal(g[i], want[i]), ("bootstrap", i)
        assert np.array_equal(gk[i], oracle.keyswitch(p, K.ksk, want[i])), ("keyswitch", i)
    for i in range(len(big)):
        assert np.array_equal(gk2[i], oracle.keyswitch(p, K.ksk, big[i])), ("keyswitch edge", i)
