"""Writes pbs64_radix.txt: the oracle's outputs of the 64-bit radix parity
case (``pbs64_case``) as a SHA-256 prefix and the decoded block value per
ciphertext.  Calls only the oracle and the seeded input recipe.

    python tests/golden/make_pbs64_golden.py [threads]

About 15 minutes on 8 cores (each oracle bootstrap at N = 2048 takes ~26 s).
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import circuits as C  # noqa: E402
import pbs64_case as case  # noqa: E402


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else oracle.default_threads()
    t0 = time.time()
    p = case.P
    K = oracle.Keys(p, case.KEY_SEED)
    print(f"keys {time.time() - t0:.0f} s", flush=True)
    col1, col2 = case.rows()
    A = case.encrypt(K, col1, tag_hi=1)
    V = case.encrypt(K, col2, tag_hi=2)
    L = case.encrypt(K, [case.literal()], tag_hi=5)[0]
    lz = C.LazyRadixBackend(p)
    masks = [C.radix_compare(lz, case.OP, list(A[r]), list(L)) for r in range(len(col1))]
    sels = [C.radix_select(lz, masks[r], list(V[r])) for r in range(len(col1))]
    tot = C.radix_sum(lz, sels)
    C.evaluate_radix(p, K, lz, threads=threads,
                     progress=lambda d, n: print(f"depth {d}/{n} {time.time() - t0:.0f} s", flush=True))
    xs, _, idx = case.spot_batch(K)
    tv = oracle.lut_testv(p, C.RADIX_P, np.array(C.radix_tables()["cmp"], dtype=np.uint64), 1 << (p.q - 6))
    spots = oracle.parallel_map(lambda j: oracle.pbs(p, K.bsk, K.ksk, xs[j], tv), idx, threads)
    print(f"spot checks {time.time() - t0:.0f} s", flush=True)
    lines = ["# Oracle outputs of the 64-bit radix parity case (tests/golden/pbs64_case.py), written by",
             "# tests/golden/make_pbs64_golden.py: kind, indices, SHA-256 prefix of the ciphertext's",
             "# little-endian words, decoded block value.  mask r; sel r block; sum block; spot index",
             "# (first compare level, CMP table).",
             f"# literal {case.literal()} col1 {col1} col2 {col2} op {case.OP}"]
    for r, m in enumerate(masks):
        ct = C.resolve_radix(p, K, m)
        lines.append(f"mask {r} {case.digest(ct)} {case.decode(K, ct)}")
    for r, s in enumerate(sels):
        for i, b in enumerate(s):
            ct = C.resolve_radix(p, K, b)
            lines.append(f"sel {r} {i} {case.digest(ct)} {case.decode(K, ct)}")
    for i, b in enumerate(tot):
        ct = C.resolve_radix(p, K, b)
        lines.append(f"sum {i} {case.digest(ct)} {case.decode(K, ct)}")
    for j, ct in zip(idx, spots):
        lines.append(f"spot {j} {case.digest(ct)} {case.decode(K, ct)}")
    with open(case.GOLDEN, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {case.GOLDEN} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
