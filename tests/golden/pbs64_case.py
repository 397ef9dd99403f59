"""Inputs of the 64-bit radix parity case: the 32-bit integer workload (two
columns of 32-bit values as 8 radix blocks of 4-bit messages, col1 < c, the
masked select of col2 and the masked SUM, which stand in for the paper's
Section 6.D aggregation and the u32 comparison / If-Then-Else rows of its
Table 3) at its own parameter set: q = 64, n = 750, N = 2048, l = 4, Bg = 2^6,
key switching 2^3 x 6.

Shared by the GPU test and by ``make_pbs64_golden.py``, which writes the
oracle's expected outputs.  It holds the recipe only: seeded values,
their block encryptions and the combined inputs of the first compare level
(x_i = a_i - c_i + 16 per block), which both sides feed to their own
bootstraps.
"""
import hashlib
import os

import numpy as np

import oracle
import seeded_inputs as si

P = si.PBS64
KEY_SEED = si.KEY_SEED_BASE + 4
DATA_SEED = si.DATA_SEED_BASE + 40
NB = 8                 # blocks of a 32-bit value
OP = "lt"              # col1 < c
SPOT_ROWS = 512        # rows of the first-level spot-check batch (8 bootstraps each)
SPOT_COUNT = 32        # sampled bootstraps compared with the oracle
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pbs64_radix.txt")


def literal() -> int:
    """c, uniform in [2^20, 2^32 - 2^25) so that c - 17 and c + 2^24 stay in range."""
    u = int(si.uniform_ints(DATA_SEED, si.TAG_LITERAL, 1, 32)[0])
    return (1 << 20) + u % ((1 << 32) - (1 << 25) - (1 << 20))


def rows():
    """Four rows: col1 below c (differing in the two low blocks), equal to c,
    above c (differing in block 6) and uniform; col2 uniform."""
    c = literal()
    extra = int(si.uniform_ints(DATA_SEED, si.TAG_DATA, 1, 32)[0])
    col1 = [c - 17, c, c + (1 << 24), extra]
    col2 = [int(v) for v in si.uniform_ints(DATA_SEED, si.TAG_DATA, 4, 32, start=1)]
    return col1, col2


def blocks(v: int, nb: int = NB):
    return [(int(v) >> (4 * i)) & 15 for i in range(nb)]


def encrypt(K, vals, tag_hi):
    """[len(vals)][NB][n+1] encryptions of the blocks, x * 2^q/64 each."""
    delta = 1 << (P.q - 6)
    bl = np.array([blocks(v) for v in vals], dtype=np.uint64).ravel()
    m, e = si.lwe_randomness(P, DATA_SEED, bl.size, tag_hi=tag_hi)
    return oracle.lwe_encrypt(P, K.s, m, e, bl * np.uint64(delta)).reshape(len(vals), NB, P.n + 1)


def spot_batch(K):
    """Combined inputs of the first compare level for SPOT_ROWS uniform rows
    against c ([SPOT_ROWS * NB][n+1], row-major by (row, block)), their
    plaintext block differences, and the sampled indices."""
    c = literal()
    vals = [int(v) for v in si.uniform_ints(DATA_SEED, si.TAG_DATA, SPOT_ROWS, 32, start=64)]
    A = encrypt(K, vals, tag_hi=3)
    L = encrypt(K, [c], tag_hi=4)[0]
    delta = 1 << (P.q - 6)
    xs = np.stack([oracle.lincomb(P, [A[r, i], L[i]], [1, -1], 16 * delta)
                   for r in range(SPOT_ROWS) for i in range(NB)])
    plain = [blocks(v)[i] - blocks(c)[i] + 16 for v in vals for i in range(NB)]
    draws = si.uniform_ints(DATA_SEED, si.TAG_SHAPE, SPOT_COUNT - 2, 32)
    idx = sorted({0, SPOT_ROWS * NB - 1} | {int(d) % (SPOT_ROWS * NB) for d in draws})
    return xs, plain, idx


def digest(ct) -> str:
    """First 16 hex digits of the SHA-256 of a ciphertext's little-endian words."""
    a = np.ascontiguousarray(np.asarray(ct, dtype=np.uint64))
    return hashlib.sha256(a.astype("<u8").tobytes()).hexdigest()[:16]


def decode(K, ct) -> int:
    """Block value in [0, 64) of a radix ciphertext (rounded phase / delta)."""
    delta = 1 << (P.q - 6)
    ph = oracle.lwe_phase(P.q, K.s, np.asarray(ct, dtype=np.uint64))
    return ((ph + delta // 2) // delta) % 64


def read_golden(path=GOLDEN):
    """{key: (digest, value)} of the committed expected outputs; keys are
    ("mask", r), ("sel", r, i), ("sum", i), ("spot", idx)."""
    out = {}
    with open(path) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            parts = line.split()
            kind, nums, dg, val = parts[0], tuple(int(x) for x in parts[1:-2]), parts[-2], int(parts[-1])
            out[(kind,) + nums] = (dg, val)
    return out
