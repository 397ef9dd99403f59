"""Parity of the multi-workgroup blind rotation (small batches: each step
spread over many workgroups) with the persistent one-workgroup-per-group
kernel and with the oracle, at every ring size it serves (q = 32 with
N = 256, 512, 1024, 2048 and q = 64 with N = 512, 1024, 2048), with the key
blocks split over several workgroups whose sums meet in atomic adds (few
groups) and kept in one (many groups), ragged groups, and inside a circuit
(a SUM tree whose narrow levels take the split path)."""
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

from gpu_util import to_dev, from_dev, context, empty  # noqa: E402

ALWAYS = 1 << 20  # split_groups: every batch takes the split path
NEVER = 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_params(q, N):
    """n = 12 so the oracle is quick; the ring and gadget of the real sets."""
    if q == 32:
        l, bg = (2, 8) if N <= 256 else (3, 7)
        return si.Params(f"split{q}_{N}", 32, 12, 1, N, bg, l, 2, 8, 20, 25)
    return si.Params(f"split{q}_{N}", 64, 12, 1, N, 6, 4, 3, 6, 20, 51)


@pytest.mark.parametrize("q,N", [(32, 256), (32, 512), (32, 1024), (32, 2048), (64, 512), (64, 1024), (64, 2048)])
def test_split_matches_persistent_and_oracle(q, N):
    p = small_params(q, N)
    K = oracle.Keys(p, si.KEY_SEED_BASE + 80 + N + q)
    ctx = context(p, K)
    tv = oracle.gate_testv(p)
    for B, seed in ((1, 1), (17, 2), (40, 3)):
        lwe = si.torus(seed, 81, B * (p.n + 1), p.q).reshape(B, p.n + 1)
        d = to_dev(p, lwe)
        ref = empty(p, B, p.N + 1)
        ctx.set_tuning(split_groups=NEVER)
        ctx.tfhe_bootstrap_batch(d, ref)
        ctx.set_tuning(split_groups=ALWAYS)  # (few groups: key blocks over several workgroups)
        got = empty(p, B, p.N + 1)
        ctx.tfhe_bootstrap_batch(d, got)
        torch.cuda.synchronize()
        ctx.set_tuning(split_groups=-1)
        say("split", q, N, "B =", B)
        assert torch.equal(got, ref), (q, N, B)
        g = from_dev(p, ref)
        for i in sorted({0, B // 2, B - 1}):
            assert np.array_equal(g[i], oracle.bootstrap(p, K.bsk, lwe[i], tv)), (q, N, B, i)
    ctx.close()


@pytest.mark.parametrize("q,N", [(32, 1024), (64, 2048)])
def test_split_many_groups_one_k_slice(q, N):
    """Enough groups that the split path keeps all key blocks in one
    workgroup (no atomic adds): same bits as the persistent kernel on every
    ciphertext."""
    p = small_params(q, N)
    K = oracle.Keys(p, si.KEY_SEED_BASE + 90 + q)
    ctx = context(p, K)
    R = N // 64
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    G = (2 * cus) // (R // 4) + 3  # G * R/4 > 2 * CUs: one K slice
    B = 16 * G - 5
    lwe = si.torus(9, 91, B * (p.n + 1), p.q).reshape(B, p.n + 1)
    d = to_dev(p, lwe)
    ref, got = empty(p, B, p.N + 1), empty(p, B, p.N + 1)
    ctx.set_tuning(split_groups=NEVER)
    ctx.tfhe_bootstrap_batch(d, ref)
    ctx.set_tuning(split_groups=ALWAYS)
    ctx.tfhe_bootstrap_batch(d, got)
    torch.cuda.synchronize()
    ctx.set_tuning(split_groups=-1)
    assert torch.equal(got, ref)
    tv = oracle.gate_testv(p)
    g = from_dev(p, got)
    assert np.array_equal(g[B - 1], oracle.bootstrap(p, K.bsk, lwe[B - 1], tv))
    ctx.close()


def test_split_inside_sum_circuit():
    """A masked SUM over 6 rows at a 1024-coefficient ring: the tree's levels
    hold few gates and take the split path (default threshold); the sum is
    the oracle's, word for word."""
    p = si.Params("split_sum", 32, 24, 1, 1024, 7, 3, 2, 8, 20, 25)
    K = oracle.Keys(p, si.KEY_SEED_BASE + 95)
    ctx = context(p, K)
    rows, w = 6, 3
    vals = np.array([5, 7, 1, 6, 2, 7], dtype=np.uint64)
    masks = np.array([1, 0, 1, 1, 0, 1], dtype=np.uint64)
    col = enc_bits(p, K, si.column_bits(vals, w), 96).reshape(rows, w, p.n + 1)
    mk = enc_bits(p, K, masks, 97).reshape(rows, p.n + 1)
    width = 6
    out = empty(p, width, p.n + 1)
    ctx.sql_masked_sum(to_dev(p, mk), to_dev(p, col), rows, w, out)
    torch.cuda.synchronize()
    g = from_dev(p, out)
    assert bits_to_int(dec_bits(p, K, g)) == int((vals * masks).sum())
    lz = C.LazyBackend(p)
    sel = [C.select(lz, mk[r], list(col[r])) for r in range(rows)]
    tot = C.sum_tree(lz, sel)
    C.evaluate(p, K, lz)
    assert np.array_equal(g, C.resolve(p, tot))
    ctx.close()
