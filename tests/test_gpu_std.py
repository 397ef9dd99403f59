"""GPU parity at the standard 32-bit gate parameters (n=630, N=1024, l=3,
Bg=2^7, key switching 2^2 x 8) in the launch configuration the benchmark
times: bootstraps of a 4096-ciphertext batch and the 4096-row scan, checked
word for word against the oracle on sampled outputs (the oracle needs ~4 s
per bootstrap here), plus decryption of every row."""
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
from gpu_util import to_dev, from_dev, empty  # noqa: E402

P = si.STD


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def std():
    say("oracle keygen at n=630, N=1024")
    K = oracle.Keys(P, si.KEY_SEED_BASE + 2)
    ctx = fs.Context(P, K.bsk, K.ksk)
    return K, ctx


def test_std_device_keygen_matches_oracle(std):
    K, _ = std
    s, S, bsk, ksk = fs.tfhe_keygen(P, K.seed)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(P, s), K.s)
    assert np.array_equal(from_dev(P, S), K.S)
    assert np.array_equal(from_dev(P, bsk), K.bsk.ravel())
    assert np.array_equal(from_dev(P, ksk), K.ksk.ravel())


def test_std_bootstrap_batch_4096(std):
    K, ctx = std
    B = 4096
    lwe = si.torus(71, 99, B * (P.n + 1), P.q).reshape(B, P.n + 1)
    d_lwe = to_dev(P, lwe)
    out = empty(P, B, P.N + 1)
    say("mfma bootstrap batch", B)
    ctx.set_kernel("mfma")
    ctx.tfhe_bootstrap_batch(d_lwe, out)
    ks = empty(P, B, P.n + 1)
    ctx.tfhe_keyswitch_batch(out, ks)
    say("plain bootstrap batch 24")
    ctx.set_kernel("plain")
    out_p = empty(P, 24, P.N + 1)
    ctx.tfhe_bootstrap_batch(d_lwe[:24].contiguous(), out_p)
    ctx.set_kernel("mfma")
    torch.cuda.synchronize()
    g, gk = from_dev(P, out), from_dev(P, ks)
    assert np.array_equal(from_dev(P, out_p), g[:24])
    idx = [0, 1, 15, 16, 2047, 2048, 4080, 4095]
    tv = oracle.gate_testv(P)
    say("oracle bootstraps", len(idx))
    want = oracle.parallel_map(lambda i: oracle.bootstrap(P, K.bsk, lwe[i], tv), idx)
    for i, w_ in zip(idx, want):
        assert np.array_equal(g[i], w_), i
        assert np.array_equal(gk[i], oracle.keyswitch(P, K.ksk, g[i])), i


@pytest.mark.parametrize("dbk", [4, 1, 3])
def test_std_key_schedules(std, dbk):
    """The schedules that stage the key in LDS -- one component's blocks with
    component 0 of the accumulator in LDS (digit_blocks 4, also what a context
    without room for the key windows runs), one block at a time (1), all of a
    step's blocks with the accumulator in global memory (3) -- give the
    windowed-key default's bits on a ragged batch of two groups (with the
    multi-workgroup path for small batches switched off), and the oracle's on
    sampled outputs."""
    K, ctx = std
    B = 19
    lwe = si.torus(73, 90 + dbk, B * (P.n + 1), P.q).reshape(B, P.n + 1)
    d_lwe = to_dev(P, lwe)
    outs = []
    try:
        for tune in (0, dbk):
            say("std bootstrap, digit_blocks", tune)
            # split_groups=0: the one-workgroup-per-group kernel these schedules belong to
            ctx.set_tuning(digit_blocks=tune, split_groups=0)
            out = empty(P, B, P.N + 1)
            ctx.tfhe_bootstrap_batch(d_lwe, out)
            torch.cuda.synchronize()
            outs.append(from_dev(P, out))
    finally:
        ctx.set_tuning(digit_blocks=0, split_groups=-1)
    assert np.array_equal(outs[0], outs[1])
    tv = oracle.gate_testv(P)
    idx = [0, 18]
    want = oracle.parallel_map(lambda i: oracle.bootstrap(P, K.bsk, lwe[i], tv), idx)
    for i, w_ in zip(idx, want):
        assert np.array_equal(outs[1][i], w_), (dbk, i)


def test_std_edge_inputs(std):
    """The boundary inputs of the toy edge test at the standard parameters
    (lg = 11, key-switch rounding to 16 bits): every output word of the
    bootstrap, of the key switch of its outputs and of the key switch of the
    crafted big ciphertexts equals the oracle's."""
    K, ctx = std
    lwe = edge_lwe(P, 33)
    B = len(lwe)
    out = empty(P, B, P.N + 1)
    ks = empty(P, B, P.n + 1)
    ctx.tfhe_bootstrap_batch(to_dev(P, lwe), out)
    ctx.tfhe_keyswitch_batch(out, ks)
    big = edge_big(P, 34)
    ks2 = empty(P, len(big), P.n + 1)
    ctx.tfhe_keyswitch_batch(to_dev(P, big), ks2)
    torch.cuda.synchronize()
    g, gk, gk2 = from_dev(P, out), from_dev(P, ks), from_dev(P, ks2)
    tv = oracle.gate_testv(P)
    say("oracle bootstraps", B)
    want = oracle.parallel_map(lambda i: oracle.bootstrap(P, K.bsk, lwe[i], tv), range(B))
    for i in range(B):
        assert np.array_equal(g[i], want[i]), ("bootstrap", i)
        assert np.array_equal(gk[i], oracle.keyswitch(P, K.ksk, want[i])), ("keyswitch", i)
    for i in range(len(big)):
        assert np.array_equal(gk2[i], oracle.keyswitch(P, K.ksk, big[i])), ("keyswitch edge", i)


def _enc_table(K, rows, w, seed):
    col1, col2 = si.table(si.DATA_SEED_BASE + seed, rows, w)
    c1 = enc_bits(P, K, si.column_bits(col1, w), seed * 10 + 1).reshape(rows, w, P.n + 1)
    c2 = enc_bits(P, K, si.column_bits(col2, w), seed * 10 + 2).reshape(rows, w, P.n + 1)
    return col1, col2, c1, c2


@pytest.fixture(scope="module")
def scan4096(std):
    """The benchmark's step at full size, run once on the GPU: mask(col1 == c)
    + select(col2) and mask(col1 < c) over 4096 rows of 8-bit columns."""
    K, ctx = std
    rows, w = 4096, 8
    col1, col2, c1, c2 = _enc_table(K, rows, w, 2)
    c_eq, c_lt = int(col1[1234]), 100
    lit_eq = enc_bits(P, K, [(c_eq >> j) & 1 for j in range(w)], 501)
    lit_lt = enc_bits(P, K, [(c_lt >> j) & 1 for j in range(w)], 502)
    d1, d2 = to_dev(P, c1), to_dev(P, c2)
    m_eq, m_lt = empty(P, rows, P.n + 1), empty(P, rows, P.n + 1)
    s_eq = empty(P, rows, w, P.n + 1)
    say("scan eq + select + scan lt over", rows, "rows")
    ctx.sql_mask_scan(d1, rows, w, "eq", to_dev(P, lit_eq), m_eq)
    ctx.sql_masked_select(m_eq, d2, rows, w, s_eq)
    ctx.sql_mask_scan(d1, rows, w, "lt", to_dev(P, lit_lt), m_lt)
    torch.cuda.synchronize()
    return dict(rows=rows, w=w, col1=col1, col2=col2, c1=c1, c2=c2, c_eq=c_eq, c_lt=c_lt, lit_eq=lit_eq,
                lit_lt=lit_lt, m_eq=from_dev(P, m_eq), m_lt=from_dev(P, m_lt), s_eq=from_dev(P, s_eq))


def _oracle_rows(K, sc, sample, with_lt):
    """Level-parallel oracle evaluation of the step's circuits on rows."""
    lz = C.LazyBackend(P)
    roots = []
    for r in sample:
        m = C.eq(lz, list(sc["c1"][r]), list(sc["lit_eq"]))
        lt = C.lt(lz, list(sc["c1"][r]), list(sc["lit_lt"])) if with_lt else None
        roots.append((r, m, C.select(lz, m, list(sc["c2"][r])), lt))
    C.evaluate(P, K, lz, threads=oracle.default_threads())
    return roots


def test_std_scan_4096_rows(std, scan4096):
    """Every row decrypts to the plaintext truth; two rows (one matching)
    and one < chain are bit-exact to the oracle end to end."""
    K, ctx = std
    sc = scan4096
    rows, w, col1, col2, c_eq, c_lt = sc["rows"], sc["w"], sc["col1"], sc["col2"], sc["c_eq"], sc["c_lt"]
    gm_eq, gm_lt, gs = sc["m_eq"], sc["m_lt"], sc["s_eq"]
    dec = lambda cts: np.array([oracle.decrypt_bit(P.q, K.s, c) for c in cts.reshape(-1, P.n + 1)])  # noqa: E731
    assert (dec(gm_eq) == (col1 == c_eq)).all()
    assert (dec(gm_lt) == (col1 < c_lt)).all()
    vals = dec(gs).reshape(rows, w)
    assert [bits_to_int(v) for v in vals] == [int(b) if a == c_eq else 0 for a, b in zip(col1, col2)]
    say("oracle end to end on rows 1234, 4095 (+ < chain on 4095)")
    for r, m, sel, lt in _oracle_rows(K, sc, [1234, 4095], True):
        assert np.array_equal(gm_eq[r], C.resolve(P, m)), r
        assert np.array_equal(gs[r], C.resolve(P, sel)), r
        assert np.array_equal(gm_lt[r], C.resolve(P, lt)), r


def _sample64(rows):
    sample = sorted(set(int(x) % rows for x in si.uniform_ints(si.DATA_SEED_BASE + 64, si.TAG_SHAPE, 63, 16)))
    return sorted(set(sample) | {1234})[:64]


@pytest.mark.slow
@pytest.mark.parametrize("part", range(4))
def test_std_scan_64_row_sample(std, scan4096, part):
    """64 seeded rows of the 4096-row step bit-exact end to end, in four
    parts of 16 rows: the equality mask, the masked select and the < mask of
    each (1,984 oracle bootstraps in all, level-parallel on the host cores)."""
    K, _ = std
    sc = scan4096
    sample = _sample64(sc["rows"])
    assert len(sample) == 64
    part_rows = sample[16 * part:16 * (part + 1)]
    say("oracle end to end on seeded rows", part_rows)
    for r, m, sel, lt in _oracle_rows(K, sc, part_rows, True):
        assert np.array_equal(sc["m_eq"][r], C.resolve(P, m)), r
        assert np.array_equal(sc["s_eq"][r], C.resolve(P, sel)), r
        assert np.array_equal(sc["m_lt"][r], C.resolve(P, lt)), r


def test_std_server_small_queries(std):
    """Two small SUM queries served together at the standard parameters (the
    narrow levels take the multi-workgroup blind rotation): the oracle's
    bits, and the decrypted sums."""
    K, ctx = std
    w = 4
    col1, col2, c1, c2 = _enc_table(K, 6, w, 77)
    specs = [(6, "eq", int(col1[2])), (3, "lt", 9)]
    lits = [enc_bits(P, K, [(c >> j) & 1 for j in range(w)], 780 + k) for k, (_, _, c) in enumerate(specs)]
    srv = fs.Server(ctx, 1 << 34, max_batch=256)
    d1, d2 = to_dev(P, c1), to_dev(P, c2)
    outs, ids = [], []
    for k, (rows, op, _) in enumerate(specs):
        outs.append(empty(P, fs.sum_width(w, rows), P.n + 1))
        ids.append(srv.submit(d1[:rows], d2[:rows], rows, w, op, to_dev(P, lits[k]), outs[k]))
    ticks = 0
    while not all(srv.done(i) for i in ids):
        srv.step()
        ticks += 1
        assert ticks < 1000
    srv.close()
    say("std server done in", ticks, "ticks")
    lz = C.LazyBackend(P)
    roots = []
    for k, (rows, op, _) in enumerate(specs):
        sel = [C.select(lz, C.predicate(lz, op, list(c1[r]), list(lits[k])), list(c2[r])) for r in range(rows)]
        roots.append(C.sum_tree(lz, sel))
    say("oracle", len(lz.nodes), "bootstraps")
    C.evaluate(P, K, lz, threads=oracle.default_threads())
    for k, (rows, op, c) in enumerate(specs):
        g = from_dev(P, outs[k])
        assert np.array_equal(g, C.resolve(P, roots[k])), k
        pred = (col1[:rows] == c) if op == "eq" else (col1[:rows] < c)
        assert bits_to_int(dec_bits(P, K, g)) == int((col2[:rows] * pred).sum())
