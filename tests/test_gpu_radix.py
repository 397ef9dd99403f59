"""GPU parity of the 64-bit programmable-bootstrapping (radix) path: LUT
bootstraps, block-wise comparison, select and radix SUM against the oracle,
the per-block digit path of the MFMA kernel, and one sampled bootstrap at the
full 64-bit parameter set (n=750, N=2048, l=4, Bg=2^6)."""
import sys

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import circuits as C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_15413_amd as fs  # noqa: E402
from gpu_util import to_dev, from_dev, empty  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_K = {}


def keys(pname):
    if pname not in _K:
        p = si.PARAMS[pname]
        K = oracle.Keys(p, si.KEY_SEED_BASE + 4)
        _K[pname] = (K, fs.Context(p, K.bsk, K.ksk))
    return _K[pname]


def blocks(v, nb):
    return [(int(v) >> (4 * i)) & 15 for i in range(nb)]


def enc_blocks(p, K, vals, nb, seed):
    delta = 1 << (p.q - 6)
    bl = np.array([blocks(v, nb) for v in vals], dtype=np.uint64).ravel()
    m, e = si.lwe_randomness(p, seed, bl.size)
    return oracle.lwe_encrypt(p, K.s, m, e, bl * np.uint64(delta)).reshape(len(vals), nb, p.n + 1)


def dec_blocks(p, K, cts):
    delta = 1 << (p.q - 6)
    out = [((oracle.lwe_phase(p.q, K.s, c) + delta // 2) // delta) % 64 for c in cts.reshape(-1, p.n + 1)]
    return np.array(out).reshape(cts.shape[:-1])


def value(bl):
    return sum(int(b) << (4 * i) for i, b in enumerate(bl))


@pytest.mark.parametrize("digit_blocks", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("pname", ["toy", "tiny", "tiny64"])
def test_bootstrap_per_block_digit_path(pname, digit_blocks):
    """Every digit grouping gives the oracle's bits: the step-keyed schedule
    with both accumulator components in LDS (the default at N <= 512 with
    32-bit words), one component's blocks with accumulator component 0 in LDS
    (the default with one row pass otherwise, forced by 4), one (u,p) block at
    a time, two levels of a component at a time (the 2048-coefficient 64-bit
    set's grouping), and all blocks of a step with the accumulator in global
    memory."""
    p = si.PARAMS[pname]
    K, ctx = keys(pname)
    ctx.set_tuning(digit_blocks=digit_blocks)
    B = 19
    lwe = si.torus(8, 99, B * (p.n + 1), p.q).reshape(B, p.n + 1)
    out = empty(p, B, p.N + 1)
    ctx.tfhe_bootstrap_batch(to_dev(p, lwe), out)
    torch.cuda.synchronize()
    ctx.set_tuning(digit_blocks=0)
    g = from_dev(p, out)
    tv = oracle.gate_testv(p)
    for i in (0, 15, 16, 18):
        assert np.array_equal(g[i], oracle.bootstrap(p, K.bsk, lwe[i], tv)), i


@pytest.mark.parametrize("op", ["lt", "eq", "gt"])
def test_radix_compare_select_sum_tiny64(op):
    p = si.TINY64
    K, ctx = keys("tiny64")
    nb, rows = 3, 5
    a_vals = [5, 4000, 300, 300, 4095]
    c_val = 300
    v_vals = [17, 4095, 1234, 2000, 9]
    A, V = enc_blocks(p, K, a_vals, nb, 11), enc_blocks(p, K, v_vals, nb, 12)
    L = enc_blocks(p, K, [c_val], nb, 13)[0]
    dA, dV, dL = to_dev(p, A), to_dev(p, V), to_dev(p, L)
    mask = empty(p, rows, p.n + 1)
    sel = empty(p, rows, nb, p.n + 1)
    tot = empty(p, nb, p.n + 1)
    say("radix", op)
    ctx.sql_radix_mask_scan(dA, rows, nb, op, dL, mask)
    ctx.sql_radix_masked_select(mask, dV, rows, nb, sel)
    ctx.sql_radix_sum(sel, rows, nb, tot)
    torch.cuda.synchronize()
    gm, gs, gt = from_dev(p, mask), from_dev(p, sel), from_dev(p, tot)
    be = C.RadixCipherBackend(p, K)
    om = [C.radix_compare(be, op, list(A[r]), list(L)) for r in range(rows)]
    osel = [C.radix_select(be, om[r], list(V[r])) for r in range(rows)]
    otot = C.radix_sum(be, osel)
    assert np.array_equal(gm, np.stack(om))
    assert np.array_equal(gs, np.stack([np.stack(x) for x in osel]))
    assert np.array_equal(gt, np.stack(otot))
    f = {"lt": lambda a: a < c_val, "eq": lambda a: a == c_val, "gt": lambda a: a > c_val}[op]
    assert dec_blocks(p, K, gm).tolist() == [16 if f(a) else 0 for a in a_vals]
    want = sum(v for a, v in zip(a_vals, v_vals) if f(a)) % (1 << (4 * nb))
    assert value(dec_blocks(p, K, gt)) == want


def test_radix_sum_single_and_odd_rows():
    p = si.TINY64
    K, ctx = keys("tiny64")
    nb = 2
    for rows in (1, 3):
        vals = [200, 100, 7][:rows]
        X = enc_blocks(p, K, vals, nb, 30 + rows)
        out = empty(p, nb, p.n + 1)
        ctx.sql_radix_sum(to_dev(p, X), rows, nb, out)
        torch.cuda.synchronize()
        be = C.RadixCipherBackend(p, K)
        assert np.array_equal(from_dev(p, out), np.stack(C.radix_sum(be, [list(x) for x in X])))
        assert value(dec_blocks(p, K, from_dev(p, out))) == sum(vals) % 256


@pytest.mark.slow
def test_pbs64_full_parameters_sampled():
    """n=750, N=2048, l=4, Bg=2^6, key switching 2^3 x 6: a 64-ciphertext LUT
    bootstrap batch (per-block digit path, 8 limbs) sampled against the oracle,
    which needs ~45 s per bootstrap here."""
    p = si.PBS64
    say("oracle keygen at n=750 N=2048 q=64")
    K, ctx = keys("pbs64")
    B = 64
    delta = 1 << (p.q - 6)
    msgs = [(7 * i) % 32 for i in range(B)]
    m, e = si.lwe_randomness(p, 61, B)
    lwe = oracle.lwe_encrypt(p, K.s, m, e, [x * delta for x in msgs])
    tab = np.array(C.radix_tables()["msg"], dtype=np.uint64)
    tv = oracle.lut_testv(p, C.RADIX_P, tab, delta)
    big = empty(p, B, p.N + 1)
    out = empty(p, B, p.n + 1)
    ctx.tfhe_bootstrap_batch(to_dev(p, lwe), big, testv=to_dev(p, tv))
    ctx.tfhe_keyswitch_batch(big, out)
    torch.cuda.synchronize()
    g = from_dev(p, out)
    assert dec_blocks(p, K, g).tolist() == [x % 16 for x in msgs]
    say("oracle bootstrap, 1 sample")
    assert np.array_equal(g[37], oracle.pbs(p, K.bsk, K.ksk, lwe[37], tv))


# --------------------------------------------- full 64-bit parameter set

sys.path.insert(0, __import__("os").path.join(__import__("os").path.dirname(__file__), "golden"))
import pbs64_case as case  # noqa: E402


@pytest.fixture(scope="module")
def pbs64_keys():
    say("oracle keygen at n=750 N=2048 q=64")
    return keys("pbs64")


def test_pbs64_radix_rows_end_to_end(pbs64_keys):
    """Config-4 circuits at their own parameters (q=64, n=750, N=2048, l=4,
    Bg=2^6, key switching 2^3 x 6): the 8-block col1 < c compare, the masked
    select of col2 and the masked SUM over four rows whose comparisons come
    out below, equal and above, every output ciphertext word for word against
    the oracle (stored as SHA-256 prefixes by tests/golden/make_pbs64_golden.py)
    and decrypted against the integers."""
    K, ctx = pbs64_keys
    gold = case.read_golden()
    p = case.P
    col1, col2 = case.rows()
    c = case.literal()
    A, V = case.encrypt(K, col1, tag_hi=1), case.encrypt(K, col2, tag_hi=2)
    L = case.encrypt(K, [c], tag_hi=5)[0]
    rows = len(col1)
    mask = empty(p, rows, p.n + 1)
    sel = empty(p, rows, case.NB, p.n + 1)
    tot = empty(p, case.NB, p.n + 1)
    say("pbs64 radix compare + select + sum, 4 rows")
    ctx.sql_radix_mask_scan(to_dev(p, A), rows, case.NB, case.OP, to_dev(p, L), mask)
    ctx.sql_radix_masked_select(mask, to_dev(p, V), rows, case.NB, sel)
    ctx.sql_radix_sum(sel, rows, case.NB, tot)
    torch.cuda.synchronize()
    gm, gs, gt = from_dev(p, mask), from_dev(p, sel), from_dev(p, tot)
    truth = [a < c for a in col1]
    assert truth == [True, False, False, col1[3] < c]
    for r in range(rows):
        assert case.digest(gm[r]) == gold[("mask", r)][0], ("mask", r)
        assert case.decode(K, gm[r]) == (16 if truth[r] else 0)
        for i in range(case.NB):
            assert case.digest(gs[r, i]) == gold[("sel", r, i)][0], ("sel", r, i)
        assert value([case.decode(K, x) for x in gs[r]]) == (col2[r] if truth[r] else 0)
    for i in range(case.NB):
        assert case.digest(gt[i]) == gold[("sum", i)][0], ("sum", i)
    want = sum(v for v, f in zip(col2, truth) if f) % (1 << 32)
    assert value([case.decode(K, x) for x in gt]) == want


def test_pbs64_spot_checks_full_launch(pbs64_keys):
    """The first compare level of 512 rows (4096 programmable bootstraps with
    the CMP table, one 4096-ciphertext launch of the persistent kernel, then
    the key switch): every output decodes to CMP of its block difference,
    and 32 sampled outputs (including the first and the last) equal the
    oracle's word for word."""
    K, ctx = pbs64_keys
    gold = case.read_golden()
    p = case.P
    xs, plain, idx = case.spot_batch(K)
    B = len(xs)
    tab = np.array(C.radix_tables()["cmp"], dtype=np.uint64)
    tv = oracle.lut_testv(p, C.RADIX_P, tab, 1 << (p.q - 6))
    big = empty(p, B, p.N + 1)
    out = empty(p, B, p.n + 1)
    say("pbs64 spot batch", B)
    ctx.tfhe_bootstrap_batch(to_dev(p, xs), big, testv=to_dev(p, tv))
    ctx.tfhe_keyswitch_batch(big, out)
    torch.cuda.synchronize()
    g = from_dev(p, out)
    assert len(idx) >= 32
    for j in idx:
        assert case.digest(g[j]) == gold[("spot", j)][0], ("spot", j)
    tabl = C.radix_tables()["cmp"]
    dec = dec_blocks(p, K, g)
    assert dec.tolist() == [tabl[x] for x in plain]
