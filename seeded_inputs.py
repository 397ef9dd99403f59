"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This module holds random-number generation, parameter sets and workload
recipes only.  It contains none of the TFHE arithmetic (no encryption, no
rounding, no polynomial products): it produces the random numbers that key
generation and encryption consume, and plaintext tables.  Both the oracle
(``oracle/``) and the product (``paper_2510_15413_amd``) take these arrays as
inputs, so neither depends on the other.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; finaliser constants as published by Vigna).
It is used in counter form: the i-th value of stream (seed, tag) is
``mix64(K + (i + 1) * GAMMA)`` with ``K = mix64(seed ^ mix64(tag + GAMMA))``,
all mod 2^64, so any index can be generated independently (the GPU library
implements the same definition for large tables).

Noise: the TFHE paper (Chillotti et al., ePrint 2018/421, cited by the
FHE-SQL paper as its scheme) draws Gaussian errors.  Here an error of
standard deviation sigma = 2^-s on a q-bit torus is the centred Irwin-Hall
sum of twelve uniform 32-bit integers (variance exactly that of twelve
U(0,1) variables, i.e. 1, scaled to 2^(q-s)), rounded half-up to an integer.
This keeps the error values integer-exact across implementations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB

# Stream tags (upper 32 bits may carry a table / query id).
TAG_LWE_KEY = 1
TAG_GLWE_KEY = 2
TAG_BSK_MASK = 3
TAG_BSK_NOISE = 4
TAG_KSK_MASK = 5
TAG_KSK_NOISE = 6
TAG_CT_MASK = 7
TAG_CT_NOISE = 8
TAG_DATA = 9
TAG_LITERAL = 10
TAG_SHAPE = 11
TAG_EXPR = 12


def mix64_int(z: int) -> int:
    """SplitMix64 finaliser on a Python int (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * _M1) & MASK64
    z = ((z ^ (z >> 27)) * _M2) & MASK64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(_M1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(_M2)
        z ^= z >> np.uint64(31)
    return z


def stream_key(seed: int, tag: int) -> int:
    return mix64_int((seed & MASK64) ^ mix64_int(tag + GAMMA))


_CHUNK = 1 << 19


def raw(seed: int, tag: int, count: int, start: int = 0) -> np.ndarray:
    """Values start .. start+count-1 of stream (seed, tag), uint64."""
    key = np.uint64(stream_key(seed, tag))
    out = np.empty(count, dtype=np.uint64)
    for c0 in range(0, count, _CHUNK):
        c1 = min(count, c0 + _CHUNK)
        idx = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            state = key + idx * np.uint64(GAMMA)
        out[c0:c1] = _mix64_np(state)
    return out


def bits(seed: int, tag: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform bits (top bit of each value), uint64 0/1."""
    return raw(seed, tag, count, start) >> np.uint64(63)


def torus(seed: int, tag: int, count: int, q: int, start: int = 0) -> np.ndarray:
    """Uniform q-bit integers (top q bits of each value), uint64."""
    v = raw(seed, tag, count, start)
    if q == 64:
        return v
    return v >> np.uint64(64 - q)


def noise(seed: int, tag: int, count: int, q: int, sigma_log2: int,
          start: int = 0) -> np.ndarray:
    """Integer errors of std 2^(q - sigma_log2), as q-bit two's complement.

    Sample s uses stream values 6s .. 6s+5; each value contributes its high
    and low 32-bit halves to a sum of twelve uniforms.
    """
    out = np.empty(count, dtype=np.uint64)
    shift = 32 - q + sigma_log2
    step = _CHUNK // 6
    for c0 in range(0, count, step):
        c1 = min(count, c0 + step)
        v = raw(seed, tag, 6 * (c1 - c0), 6 * (start + c0)).reshape(c1 - c0, 6)
        hi = (v >> np.uint64(32)).astype(np.int64)
        lo = (v & np.uint64(0xFFFFFFFF)).astype(np.int64)
        s = hi.sum(axis=1) + lo.sum(axis=1) - np.int64(6 << 32)
        if shift > 0:
            e = (s + np.int64(1 << (shift - 1))) >> np.int64(shift)
        else:
            e = s << np.int64(-shift)
        out[c0:c1] = e.astype(np.uint64)
    if q < 64:
        out &= np.uint64((1 << q) - 1)
    return out


def uniform_ints(seed: int, tag: int, count: int, width_bits: int,
                 start: int = 0) -> np.ndarray:
    """Uniform unsigned integers in [0, 2^width_bits)."""
    return raw(seed, tag, count, start) >> np.uint64(64 - width_bits)


def uniform_unit(seed: int, tag: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits (workload shapes only)."""
    return (raw(seed, tag, count, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# --------------------------------------------------------------------------
# Parameter sets of the five workloads.
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Params:
    """TFHE parameters: torus bits q, LWE n, GLWE k and N, gadget base 2^bg_bits
    with l levels, key-switch base 2^ks_bits with ks_t levels, and the noise
    standard deviations 2^-lwe_sigma_log2 / 2^-glwe_sigma_log2."""
    name: str
    q: int
    n: int
    k: int
    N: int
    bg_bits: int
    l: int
    ks_bits: int
    ks_t: int
    lwe_sigma_log2: int
    glwe_sigma_log2: int

    def as_dict(self):
        return asdict(self)

    @property
    def lwe_words(self):
        return self.n + 1

    @property
    def big_lwe_words(self):
        return self.k * self.N + 1

    def bsk_words(self):
        return self.n * (self.k + 1) * self.l * (self.k + 1) * self.N

    def ksk_words(self):
        return self.k * self.N * self.ks_t * (1 << self.ks_bits) * (self.n + 1)


# Toy insecure gate-bootstrapping set (32 rows of 4-bit columns).
TOY = Params("toy", 32, 64, 1, 256, 8, 2, 2, 5, 20, 25)
# Standard 32-bit gate-bootstrapping set (4096 rows of 8-bit columns).
STD = Params("std", 32, 630, 1, 1024, 7, 3, 2, 8, 15, 25)
# 64-bit programmable bootstrapping set (radix blocks, LUTs).
PBS64 = Params("pbs64", 64, 750, 1, 2048, 6, 4, 3, 6, 20, 51)
# Tiny set used for exhaustive circuit checks on the CPU (insecure).
TINY = Params("tiny", 32, 16, 1, 64, 8, 2, 2, 5, 24, 30)
# Small 64-bit set that exercises the 64-bit path at low cost (insecure).
TINY64 = Params("tiny64", 64, 16, 1, 512, 6, 4, 3, 6, 24, 51)

PARAMS = {p.name: p for p in (TOY, STD, PBS64, TINY, TINY64)}

KEY_SEED_BASE = 0xF5E50000
DATA_SEED_BASE = 0xDA7A0000


# --------------------------------------------------------------------------
# Random material for key generation and encryption.
# --------------------------------------------------------------------------

def secret_keys(p: Params, seed: int):
    """Binary LWE key s (n) and GLWE key S (k*N), uint64 0/1."""
    s = bits(seed, TAG_LWE_KEY, p.n)
    S = bits(seed, TAG_GLWE_KEY, p.k * p.N)
    return s, S


def bsk_randomness(p: Params, seed: int):
    """Masks [n][(k+1)l][k][N] and errors [n][(k+1)l][N] of the GGSW rows."""
    rows = p.n * (p.k + 1) * p.l
    masks = torus(seed, TAG_BSK_MASK, rows * p.k * p.N, p.q).reshape(
        p.n, (p.k + 1) * p.l, p.k, p.N)
    errs = noise(seed, TAG_BSK_NOISE, rows * p.N, p.q, p.glwe_sigma_log2).reshape(
        p.n, (p.k + 1) * p.l, p.N)
    return masks, errs


def ksk_randomness(p: Params, seed: int):
    """Masks [kN][t][2^b][n] and errors [kN][t][2^b] of the key-switching table."""
    cnt = p.k * p.N * p.ks_t * (1 << p.ks_bits)
    masks = torus(seed, TAG_KSK_MASK, cnt * p.n, p.q).reshape(
        p.k * p.N, p.ks_t, 1 << p.ks_bits, p.n)
    errs = noise(seed, TAG_KSK_NOISE, cnt, p.q, p.lwe_sigma_log2).reshape(
        p.k * p.N, p.ks_t, 1 << p.ks_bits)
    return masks, errs


def lwe_randomness(p: Params, seed: int, count: int, tag_hi: int = 0, start: int = 0):
    """Masks [count][n] and errors [count] for fresh LWE encryptions."""
    masks = torus(seed, TAG_CT_MASK | (tag_hi << 32), count * p.n, p.q,
                  start=start * p.n).reshape(count, p.n)
    errs = noise(seed, TAG_CT_NOISE | (tag_hi << 32), count, p.q, p.lwe_sigma_log2,
                 start=start)
    return masks, errs


# --------------------------------------------------------------------------
# Plaintext workloads.
# --------------------------------------------------------------------------

def column_bits(values: np.ndarray, w: int) -> np.ndarray:
    """[rows][w] bits of each value, least significant bit first."""
    v = np.asarray(values, dtype=np.uint64)
    return ((v[:, None] >> np.arange(w, dtype=np.uint64)[None, :]) & np.uint64(1))


def table(seed: int, rows: int, w: int, table_id: int = 0):
    """Two uniform w-bit columns (col1, col2)."""
    col1 = uniform_ints(seed, TAG_DATA | (table_id << 32), rows, w)
    col2 = uniform_ints(seed, TAG_DATA | (table_id << 32), rows, w, start=rows)
    return col1, col2


def log_uniform_int(seed: int, tag: int, count: int, lo: float, hi: float) -> np.ndarray:
    u = uniform_unit(seed, tag, count)
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def uneven_tables(seed: int, count: int = 16, lo: int = 100, hi: int = 65536):
    """Row counts (log-uniform) and predicate kinds (uniform over eq, lt,
    between) of the batched multi-table scan."""
    rows = log_uniform_int(seed, TAG_SHAPE, count, lo, hi)
    ops = (uniform_ints(seed, TAG_SHAPE, count, 16, start=count) % np.uint64(3)).astype(np.int64)
    return rows, ops


CMP_NAMES = ("eq", "ne", "lt", "le", "gt", "ge")


def paper_where_example(age_col: int = 0, salary_col: int = 1, age_lit=18, salary_lit=1000):
    """Node list of the WHERE clause used as the expression-tree example of
    Section 4.3 B (age > 18 AND salary < 1000); the two numbers become
    plaintext constants."""
    return [
        {"kind": "column", "col": age_col},
        {"kind": "const", "value": age_lit},
        {"kind": "cmp", "op": "gt", "a": 0, "b": 1},
        {"kind": "column", "col": salary_col},
        {"kind": "const", "value": salary_lit},
        {"kind": "cmp", "op": "lt", "a": 3, "b": 4},
        {"kind": "and", "a": 2, "b": 5},
    ]


def random_expr(seed: int, ncols: int, nlits: int, w: int, depth: int = 3, root: str = "bool"):
    """A seeded random expression tree as a topologically ordered node list
    (operands precede their node; the last node is the root).  Boolean nodes
    draw from cmp/and/or/xor/not, value nodes from column/const/literal/
    max/min/ite; an operand is sometimes an earlier node of the same kind, so
    the result is a DAG with shared subexpressions."""
    draws = raw(seed, TAG_EXPR, 4096)
    pos = [0]

    def pick(n):
        v = int(draws[pos[0] % draws.size]) % n
        pos[0] += 1
        return v

    nodes, kinds = [], []

    def emit(nd, kind):
        nodes.append(nd)
        kinds.append(kind)
        return len(nodes) - 1

    def reuse(kind):
        cand = [i for i, k in enumerate(kinds) if k == kind]
        if cand and pick(4) == 0:
            return cand[pick(len(cand))]
        return None

    def value(d):
        r = reuse("value")
        if r is not None:
            return r
        leaf = d <= 0 or pick(3) != 0
        if leaf:
            t = pick(3 if nlits else 2)
            if t == 0:
                return emit({"kind": "column", "col": pick(ncols)}, "value")
            if t == 1:
                return emit({"kind": "const", "value": pick(1 << w)}, "value")
            return emit({"kind": "literal", "lit": pick(nlits)}, "value")
        t = pick(3)
        if t < 2:
            a, b = value(d - 1), value(d - 1)
            return emit({"kind": ("max", "min")[t], "a": a, "b": b}, "value")
        c = boolean(d - 1)
        a, b = value(d - 1), value(d - 1)
        return emit({"kind": "ite", "c": c, "a": a, "b": b}, "value")

    def boolean(d):
        r = reuse("bool")
        if r is not None:
            return r
        t = 0 if d <= 0 else pick(5)
        if t == 0:
            a, b = value(d - 1), value(d - 1)
            return emit({"kind": "cmp", "op": CMP_NAMES[pick(6)], "a": a, "b": b}, "bool")
        if t == 4:
            return emit({"kind": "not", "a": boolean(d - 1)}, "bool")
        a, b = boolean(d - 1), boolean(d - 1)
        return emit({"kind": ("and", "or", "xor")[t - 1], "a": a, "b": b}, "bool")

    if root == "bool":
        boolean(depth)
    else:
        value(depth)
    return nodes
