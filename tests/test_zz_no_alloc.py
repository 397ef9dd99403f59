"""The no-allocation bootstrap entry point (tfhe_bootstrap_batch_noalloc)
gives the bits of tfhe_bootstrap_batch on two calls in a row, the second with
a smaller batch, at parameter sets whose blind rotation uses a workspace
(the standard 32-bit set: accumulator component 1 in the scratch; the small
64-bit set: the same at 64-bit words), and rejects a batch too large for its
static array before launching anything."""
import sys

import pytest

import seeded_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_15413_amd as fs  # noqa: E402
from paper_2510_15413_amd import _lib  # noqa: E402
from gpu_util import to_dev, empty  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("pname", ["std", "tiny64"])
def test_noalloc_matches_bootstrap_batch(pname):
    p = si.PARAMS[pname]
    _, _, bsk, ksk = fs.tfhe_keygen(p, si.KEY_SEED_BASE + 61)
    ctx = fs.Context(p, bsk, ksk)
    del bsk, ksk
    for B, seed in ((300, 1), (37, 2)):
        say("noalloc", pname, "B =", B)
        lwe = to_dev(p, si.torus(seed, 61, B * (p.n + 1), p.q).reshape(B, p.n + 1))
        ref = empty(p, B, p.N + 1)
        got = empty(p, B, p.N + 1)
        got.fill_(0)
        ctx.tfhe_bootstrap_batch(lwe, ref)
        ctx.tfhe_bootstrap_batch_noalloc(lwe, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (pname, B)
    ctx.close()


def test_noalloc_rejects_batches_beyond_the_scratch():
    p = si.STD
    _, _, bsk, ksk = fs.tfhe_keygen(p, si.KEY_SEED_BASE + 62)
    ctx = fs.Context(p, bsk, ksk)
    del bsk, ksk
    cap = _lib.load().tfhe_noalloc_scratch_bytes()
    per_group = 2 * p.N * 16 * 4  # the accumulator slot of 16 ciphertexts (both components)
    B = (cap // per_group) * 16 + 16
    lwe = torch.zeros((B, p.n + 1), dtype=torch.int32, device="cuda")
    out = torch.empty((B, p.N + 1), dtype=torch.int32, device="cuda")
    with pytest.raises(fs.FheError, match="scratch"):
        ctx.tfhe_bootstrap_batch_noalloc(lwe, out)
    ctx.close()
