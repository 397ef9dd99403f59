"""CPU oracle for the FHE-SQL oblivious-selection hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_2510_15413_amd``); both take their random
material from ``seeded_inputs``.

The arithmetic lives in ``tfhe_oracle.c`` (plain C, schoolbook products); this
module marshals numpy arrays to it.  All torus values are uint64 arrays holding
q-bit integers.  See ``circuits.py`` for the gate and SQL netlists.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_tfhe.so")
SRC_PATH = os.path.join(_HERE, "tfhe_oracle.c")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_intp = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, portable x86-64-v2 code)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-march=x86-64-v2", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-o", tmp, SRC_PATH])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u64, i64, c_int = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
        sig = {
            "or_round_top": (u64, [c_int, c_int, u64]),
            "or_mod_switch": (u64, [c_int, c_int, u64]),
            "or_decompose": (None, [c_int, c_int, c_int, u64, _i64p]),
            "or_negacyclic_mul": (None, [c_int, c_int, _u64p, _u64p, _u64p]),
            "or_monomial_mul": (None, [c_int, c_int, i64, _u64p, _u64p]),
            "or_lwe_phase": (u64, [c_int, c_int, _u64p, _u64p]),
            "or_glwe_phase": (None, [c_int, c_int, c_int, _u64p, _u64p, _u64p]),
            "or_lwe_encrypt": (None, [c_int, c_int, _u64p, _u64p, u64, u64, _u64p]),
            "or_glwe_encrypt": (None, [c_int, c_int, c_int, _u64p, _u64p, _u64p, _u64p, _u64p]),
            "or_ggsw_encrypt": (None, [_intp, _u64p, u64, _u64p, _u64p, _u64p]),
            "or_bsk_gen": (None, [_intp, _u64p, _u64p, _u64p, _u64p, _u64p]),
            "or_ksk_gen": (None, [_intp, _u64p, _u64p, _u64p, _u64p, _u64p]),
            "or_ext_product": (None, [_intp, _u64p, _u64p, _u64p]),
            "or_blind_rotate": (None, [_intp, _u64p, _u64p, _u64p, _u64p]),
            "or_sample_extract": (None, [_intp, _u64p, _u64p]),
            "or_keyswitch": (None, [_intp, _u64p, _u64p, _u64p]),
            "or_bootstrap": (None, [_intp, _u64p, _u64p, _u64p, _u64p]),
            "or_gate_testv": (None, [c_int, c_int, _u64p]),
            "or_lut_testv": (None, [c_int, c_int, c_int, _u64p, u64, _u64p]),
            "or_pbs": (None, [_intp, _u64p, _u64p, _u64p, _u64p, _u64p]),
            "or_gate_bootstrap": (None, [_intp, _u64p, _u64p, _u64p, _u64p]),
            "or_lincomb": (None, [c_int, c_int, c_int, _u64p, _i64p, u64, _u64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(_u64p)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def pvec(p):
    """Parameter vector {q, n, k, N, bg_bits, l, ks_bits, ks_t}."""
    return (ctypes.c_int * 8)(p.q, p.n, p.k, p.N, p.bg_bits, p.l, p.ks_bits, p.ks_t)


def qmask(q: int) -> int:
    return (1 << q) - 1


# ------------------------------------------------------------ primitives

def round_top(q, bits, x) -> int:
    return int(lib().or_round_top(q, bits, int(x) & qmask(q)))


def mod_switch(q, N, x) -> int:
    return int(lib().or_mod_switch(q, N, int(x) & qmask(q)))


def decompose(q, bg_bits, l, x):
    d = (ctypes.c_int64 * l)()
    lib().or_decompose(q, bg_bits, l, int(x) & qmask(q), d)
    return [int(v) for v in d]


def negacyclic_mul(q, a, b):
    a, b = _u64(a), _u64(b)
    c = np.zeros_like(a)
    lib().or_negacyclic_mul(q, a.size, _p(a), _p(b), _p(c))
    return c


def monomial_mul(q, e, poly):
    poly = _u64(poly)
    out = np.zeros_like(poly)
    lib().or_monomial_mul(q, poly.size, int(e), _p(poly), _p(out))
    return out


def lwe_phase(q, key, ct) -> int:
    key, ct = _u64(key), _u64(ct)
    return int(lib().or_lwe_phase(q, key.size, _p(key), _p(ct)))


def lwe_phases(q, key, cts) -> np.ndarray:
    cts = _u64(cts).reshape(-1, np.asarray(key).size + 1)
    return np.array([lwe_phase(q, key, c) for c in cts], dtype=np.uint64)


def glwe_phase(p, S, ct):
    S, ct = _u64(S), _u64(ct)
    out = np.zeros(p.N, dtype=np.uint64)
    lib().or_glwe_phase(p.q, p.k, p.N, _p(S), _p(ct), _p(out))
    return out


def signed(q, x):
    """Read q-bit values as signed integers (numpy int64 or Python int)."""
    if isinstance(x, np.ndarray):
        v = x.astype(object)
        return np.array([int(t) - (1 << q) if int(t) >= (1 << (q - 1)) else int(t) for t in v.ravel()],
                        dtype=object).reshape(x.shape)
    x = int(x)
    return x - (1 << q) if x >= (1 << (q - 1)) else x


def decrypt_bit(q, key, ct) -> int:
    """Gate encoding: bit 1 iff the phase, as a signed q-bit integer, is > 0."""
    ph = lwe_phase(q, key, ct)
    return 1 if 0 < ph < (1 << (q - 1)) else 0


# ------------------------------------------------------------ encryption

def lwe_encrypt(p, key, masks, errs, mus):
    """Encrypt a batch: masks [M][n], errs [M], mus [M] -> [M][n+1]."""
    key, masks, errs, mus = _u64(key), _u64(masks), _u64(errs), _u64(mus)
    M = errs.size
    out = np.zeros((M, p.n + 1), dtype=np.uint64)
    L = lib()
    for i in range(M):
        L.or_lwe_encrypt(p.q, p.n, _p(key), _p(masks[i]), int(errs[i]), int(mus[i]) & qmask(p.q),
                         out[i].ctypes.data_as(_u64p))
    return out


def glwe_encrypt(p, S, masks, errs, msg=None):
    S, masks, errs = _u64(S), _u64(masks), _u64(errs)
    out = np.zeros((p.k + 1) * p.N, dtype=np.uint64)
    m = _u64(msg) if msg is not None else None
    lib().or_glwe_encrypt(p.q, p.k, p.N, _p(S), _p(masks), _p(errs),
                          _p(m) if m is not None else None, _p(out))
    return out


def ggsw_encrypt(p, S, m, masks, errs):
    S, masks, errs = _u64(S), _u64(masks), _u64(errs)
    out = np.zeros(((p.k + 1) * p.l, p.k + 1, p.N), dtype=np.uint64)
    lib().or_ggsw_encrypt(pvec(p), _p(S), int(m) & qmask(p.q), _p(masks), _p(errs), _p(out))
    return out


def bsk_gen(p, s, S, masks, errs):
    s, S, masks, errs = _u64(s), _u64(S), _u64(masks), _u64(errs)
    out = np.zeros((p.n, (p.k + 1) * p.l, p.k + 1, p.N), dtype=np.uint64)
    lib().or_bsk_gen(pvec(p), _p(s), _p(S), _p(masks), _p(errs), _p(out))
    return out


def ksk_gen(p, sx, s, masks, errs):
    sx, s, masks, errs = _u64(sx), _u64(s), _u64(masks), _u64(errs)
    out = np.zeros((p.k * p.N, p.ks_t, 1 << p.ks_bits, p.n + 1), dtype=np.uint64)
    lib().or_ksk_gen(pvec(p), _p(sx), _p(s), _p(masks), _p(errs), _p(out))
    return out


def ksk_gen_rows(p, sx, s, masks, errs, i0, i1):
    """Rows i0..i1-1 of the key-switching table (same definition as ksk_gen)."""
    V = 1 << p.ks_bits
    out = np.zeros((i1 - i0, p.ks_t, V, p.n + 1), dtype=np.uint64)
    L = lib()
    s = _u64(s)
    for i in range(i0, i1):
        for j in range(p.ks_t):
            for v in range(V):
                mu = (v * int(sx[i]) << (p.q - (j + 1) * p.ks_bits)) & qmask(p.q) \
                    if p.q - (j + 1) * p.ks_bits >= 0 else 0
                m = np.ascontiguousarray(masks[i, j, v])
                L.or_lwe_encrypt(p.q, p.n, _p(s), _p(m), int(errs[i, j, v]), mu,
                                 out[i - i0, j, v].ctypes.data_as(_u64p))
    return out


def extracted_key(S):
    """s'_{jN+i} = S_j[i]: the flattened GLWE key."""
    return _u64(S).ravel().copy()


# --------------------------------------------------------- bootstrapping

def ext_product(p, ggsw, glwe):
    ggsw, glwe = _u64(ggsw), _u64(glwe)
    out = np.zeros((p.k + 1) * p.N, dtype=np.uint64)
    lib().or_ext_product(pvec(p), _p(ggsw), _p(glwe), _p(out))
    return out


def blind_rotate(p, bsk, lwe, testv):
    bsk, lwe, testv = _u64(bsk), _u64(lwe), _u64(testv)
    out = np.zeros((p.k + 1) * p.N, dtype=np.uint64)
    lib().or_blind_rotate(pvec(p), _p(bsk), _p(lwe), _p(testv), _p(out))
    return out


def sample_extract(p, glwe):
    glwe = _u64(glwe)
    out = np.zeros(p.k * p.N + 1, dtype=np.uint64)
    lib().or_sample_extract(pvec(p), _p(glwe), _p(out))
    return out


def keyswitch(p, ksk, big):
    ksk, big = _u64(ksk), _u64(big)
    out = np.zeros(p.n + 1, dtype=np.uint64)
    lib().or_keyswitch(pvec(p), _p(ksk), _p(big), _p(out))
    return out


def gate_testv(p):
    out = np.zeros(p.N, dtype=np.uint64)
    lib().or_gate_testv(p.q, p.N, _p(out))
    return out


def lut_testv(p, plain_mod, table, delta_out):
    f = _u64(table)
    assert f.size == plain_mod
    out = np.zeros(p.N, dtype=np.uint64)
    lib().or_lut_testv(p.q, p.N, plain_mod, _p(f), int(delta_out) & qmask(p.q), _p(out))
    return out


def bootstrap(p, bsk, lwe, testv):
    bsk, lwe, testv = _u64(bsk), _u64(lwe), _u64(testv)
    out = np.zeros(p.k * p.N + 1, dtype=np.uint64)
    lib().or_bootstrap(pvec(p), _p(bsk), _p(lwe), _p(testv), _p(out))
    return out


def pbs(p, bsk, ksk, lwe, testv):
    bsk, ksk, lwe, testv = _u64(bsk), _u64(ksk), _u64(lwe), _u64(testv)
    out = np.zeros(p.n + 1, dtype=np.uint64)
    lib().or_pbs(pvec(p), _p(bsk), _p(ksk), _p(lwe), _p(testv), _p(out))
    return out


def gate_bootstrap(p, bsk, ksk, lwe):
    bsk, ksk, lwe = _u64(bsk), _u64(ksk), _u64(lwe)
    out = np.zeros(p.n + 1, dtype=np.uint64)
    lib().or_gate_bootstrap(pvec(p), _p(bsk), _p(ksk), _p(lwe), _p(out))
    return out


def lincomb(p, ins, weights, const):
    ins = _u64(ins).reshape(len(weights), p.n + 1)
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.int64))
    out = np.zeros(p.n + 1, dtype=np.uint64)
    lib().or_lincomb(p.q, p.n, len(weights), _p(ins), w.ctypes.data_as(_i64p),
                     int(const) & qmask(p.q), _p(out))
    return out


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def parallel_map(fn, items, threads=None):
    """Run fn over items on a thread pool (the C calls release the GIL)."""
    items = list(items)
    threads = threads or default_threads()
    if threads <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))


class Keys:
    """Oracle key material generated from seeded randomness."""

    def __init__(self, p, seed):
        import seeded_inputs as si
        self.p = p
        self.seed = seed
        self.s, self.S = si.secret_keys(p, seed)
        self.sx = extracted_key(self.S)
        bm, be = si.bsk_randomness(p, seed)
        # BSK_i = GGSW_S(s_i) for each i, generated independently on threads.
        self.bsk = np.stack(parallel_map(
            lambda i: ggsw_encrypt(p, self.S, self.s[i], bm[i], be[i]), range(p.n)))
        km, ke = si.ksk_randomness(p, seed)
        V = 1 << p.ks_bits
        self.ksk = np.zeros((p.k * p.N, p.ks_t, V, p.n + 1), dtype=np.uint64)

        def ks_rows(i0):
            i1 = min(i0 + 64, p.k * p.N)
            sub = ksk_gen_rows(p, self.sx, self.s, km, ke, i0, i1)
            self.ksk[i0:i1] = sub
        parallel_map(ks_rows, range(0, p.k * p.N, 64))
