"""ctypes binding of libfhesql.so (the gfx950 HIP library).

Argument marshalling only: every computation runs in the library's kernels.
Device buffers are torch tensors (int32 storage for 32-bit torus words,
int64 for 64-bit words); the HIP stream is torch's current stream unless one
is given.  Every call checks the library's return code and raises
``FheError`` with ``tfhe_last_error`` on failure.  The library must have been
built (``paper_2510_15413_amd.build``); importing this module on a machine
where it is missing raises immediately.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfhesql.so")

TFHE_KERNEL_MFMA = 0
TFHE_KERNEL_PLAIN = 1
SQL_OP_EQ, SQL_OP_LT, SQL_OP_GT, SQL_OP_BETWEEN = 0, 1, 2, 3
SQL_OPS = {"eq": SQL_OP_EQ, "lt": SQL_OP_LT, "gt": SQL_OP_GT, "between": SQL_OP_BETWEEN}
GATE_OPS = {"AND": 0, "NAND": 1, "OR": 2, "NOR": 3, "XOR": 4, "XNOR": 5, "ANDNY": 6, "MAJ": 7}

# Tags of the seeded streams (same numbering as the seeded input recipe).
TAG_CT_MASK = 7
TAG_CT_NOISE = 8

EXPORTS = [
    "tfhe_bsk_words", "tfhe_ksk_words", "tfhe_ctx_create", "tfhe_ctx_destroy",
    "tfhe_last_error", "tfhe_set_kernel", "tfhe_ctx_sync", "tfhe_bootstrap_batch",
    "tfhe_keyswitch_batch", "tfhe_gate_batch", "sql_mask_scan", "sql_masked_select",
    "sql_masked_sum", "sql_scan_batch", "tfhe_rng_fill", "tfhe_keygen",
    "tfhe_lwe_encrypt", "tfhe_lwe_phase", "tfhe_timing_enable", "tfhe_timing_read",
    "tfhe_set_tuning", "sql_server_create", "sql_server_destroy", "sql_server_submit",
    "sql_server_step", "sql_server_done", "sql_server_bytes_in_use",
    "sql_radix_mask_scan", "sql_radix_masked_select", "sql_radix_sum", "sql_expr_eval", "tfhe_timing_log", "sql_server_submit_expr",
    "tfhe_graph_stats", "tfhe_bootstrap_batch_noalloc", "tfhe_noalloc_scratch_bytes", "tfhe_get_tuning",
]
# Expression-tree node kinds and comparison operators (sql_expr).
SQL_EXPR_KINDS = {"column": 0, "const": 1, "literal": 2, "cmp": 3, "and": 4, "or": 5, "xor": 6, "not": 7,
                  "max": 8, "min": 9, "ite": 10}
SQL_CMP_OPS = {"eq": 0, "ne": 1, "lt": 2, "le": 3, "gt": 4, "ge": 5}
TFHE_TUNE_MAX_BATCH = 1
TFHE_TUNE_ROW_PASS = 2
TFHE_TUNE_DIGIT_BLOCKS = 3
TFHE_TUNE_SPLIT_GROUPS = 4


class FheError(RuntimeError):
    pass


class TfheParams(ctypes.Structure):
    _fields_ = [("torus_bits", ctypes.c_uint32), ("n", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("N", ctypes.c_uint32), ("bg_bits", ctypes.c_uint32), ("l", ctypes.c_uint32),
                ("ks_base_bits", ctypes.c_uint32), ("ks_t", ctypes.c_uint32)]


class SqlSumQuery(ctypes.Structure):
    _fields_ = [("d_col", ctypes.c_void_p), ("d_sum_col", ctypes.c_void_p), ("rows", ctypes.c_uint32),
                ("w", ctypes.c_uint32), ("op", ctypes.c_int), ("d_lit_a", ctypes.c_void_p),
                ("d_lit_b", ctypes.c_void_p), ("d_sum", ctypes.c_void_p)]


class SqlTableQuery(ctypes.Structure):
    _fields_ = [("d_col", ctypes.c_void_p), ("d_sel_col", ctypes.c_void_p), ("rows", ctypes.c_uint32),
                ("w", ctypes.c_uint32), ("op", ctypes.c_int), ("d_lit_a", ctypes.c_void_p),
                ("d_lit_b", ctypes.c_void_p), ("d_mask", ctypes.c_void_p), ("d_sel_out", ctypes.c_void_p)]


class SqlExpr(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("op", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("c", ctypes.c_int32), ("col", ctypes.c_int32), ("value", ctypes.c_uint64),
                ("d_lit", ctypes.c_void_p)]


_lib = None


def load():
    """Load libfhesql.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FheError(f"{LIB_PATH} is missing: build it with paper_2510_15413_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
    P = ctypes.POINTER(TfheParams)
    sig = {
        "tfhe_bsk_words": (sz, [P]),
        "tfhe_ksk_words": (sz, [P]),
        "tfhe_ctx_create": (i32, [P, vp, sz, vp, sz, i32, ctypes.POINTER(vp)]),
        "tfhe_ctx_destroy": (None, [vp]),
        "tfhe_last_error": (ctypes.c_char_p, [vp]),
        "tfhe_set_kernel": (i32, [vp, i32]),
        "tfhe_ctx_sync": (i32, [vp, vp]),
        "tfhe_bootstrap_batch": (i32, [vp, vp, vp, vp, u32, vp]),
        "tfhe_keyswitch_batch": (i32, [vp, vp, vp, u32, vp]),
        "tfhe_gate_batch": (i32, [vp, i32, vp, vp, vp, vp, u32, vp]),
        "sql_mask_scan": (i32, [vp, vp, u32, u32, i32, vp, vp, vp, vp]),
        "sql_masked_select": (i32, [vp, vp, vp, u32, u32, vp, vp]),
        "sql_masked_sum": (i32, [vp, vp, vp, u32, u32, vp, ctypes.POINTER(u32), vp]),
        "sql_scan_batch": (i32, [vp, ctypes.POINTER(SqlTableQuery), u32, i32, vp]),
        "tfhe_rng_fill": (i32, [u64, u64, u64, u64, vp, vp]),
        "tfhe_keygen": (i32, [P, u64, u32, u32, vp, vp, vp, vp, vp]),
        "tfhe_lwe_encrypt": (i32, [P, u64, u64, u64, u32, u64, vp, vp, vp, u64, u32, vp]),
        "tfhe_lwe_phase": (i32, [P, vp, vp, vp, u64, u32, vp]),
        "tfhe_timing_enable": (i32, [vp, i32]),
        "tfhe_set_tuning": (i32, [vp, i32, ctypes.c_int64]),
        "sql_server_create": (i32, [vp, sz, u32, ctypes.POINTER(vp)]),
        "sql_server_destroy": (None, [vp]),
        "sql_server_submit": (i32, [vp, ctypes.POINTER(SqlSumQuery), ctypes.POINTER(u64)]),
        "sql_server_step": (i32, [vp, vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]),
        "sql_server_done": (i32, [vp, u64]),
        "sql_server_bytes_in_use": (sz, [vp]),
        "sql_radix_mask_scan": (i32, [vp, vp, u32, u32, i32, vp, vp, vp]),
        "sql_radix_masked_select": (i32, [vp, vp, vp, u32, u32, vp, vp]),
        "sql_radix_sum": (i32, [vp, vp, u32, u32, vp, vp]),
        "tfhe_timing_log": (i32, [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), u64, ctypes.POINTER(u64)]),
        "sql_server_submit_expr": (i32, [vp, ctypes.POINTER(vp), u32, u32, u32, ctypes.POINTER(SqlExpr), u32, vp, vp,
                                         ctypes.POINTER(u64)]),
        "sql_expr_eval": (i32, [vp, ctypes.POINTER(vp), u32, u32, u32, ctypes.POINTER(SqlExpr), u32, vp, vp]),
        "tfhe_timing_read": (i32, [vp, i32, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(u64)]),
        "tfhe_graph_stats": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        "tfhe_bootstrap_batch_noalloc": (i32, [vp, vp, vp, vp, u32, vp]),
        "tfhe_noalloc_scratch_bytes": (sz, []),
        "tfhe_get_tuning": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def params_struct(p) -> TfheParams:
    return TfheParams(p.q, p.n, p.k, p.N, p.bg_bits, p.l, p.ks_bits, p.ks_t)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def torch_dtype(q):
    import torch
    return torch.int32 if q == 32 else torch.int64


def _check_dev(t, name):
    if t is None:
        return
    if not t.is_cuda or not t.is_contiguous():
        raise FheError(f"{name} must be a contiguous device tensor")


class Context:
    """A TFHE evaluation context holding device keys (tfhe_ctx)."""

    def __init__(self, p, bsk, ksk):
        """bsk/ksk: torch tensors on the device or numpy arrays (uint64 words)."""
        import numpy as np
        import torch
        L = load()
        self.p = p
        self._ps = params_struct(p)
        self.dtype = torch_dtype(p.q)
        self.wb = 4 if p.q == 32 else 8
        nb, nk = L.tfhe_bsk_words(ctypes.byref(self._ps)), L.tfhe_ksk_words(ctypes.byref(self._ps))
        if nb == 0:
            raise FheError("invalid parameter set")
        self._h = ctypes.c_void_p()
        if isinstance(bsk, np.ndarray):
            hb = np.ascontiguousarray(bsk.astype(np.uint32 if p.q == 32 else np.uint64).ravel())
            hk = np.ascontiguousarray(ksk.astype(np.uint32 if p.q == 32 else np.uint64).ravel())
            rc = L.tfhe_ctx_create(ctypes.byref(self._ps), hb.ctypes.data_as(ctypes.c_void_p), hb.nbytes,
                                   hk.ctypes.data_as(ctypes.c_void_p), hk.nbytes, 0, ctypes.byref(self._h))
        else:
            _check_dev(bsk, "bsk")
            _check_dev(ksk, "ksk")
            torch.cuda.synchronize()
            rc = L.tfhe_ctx_create(ctypes.byref(self._ps), _ptr(bsk), bsk.numel() * bsk.element_size(),
                                   _ptr(ksk), ksk.numel() * ksk.element_size(), 1, ctypes.byref(self._h))
        if rc != 0:
            raise FheError(f"tfhe_ctx_create failed ({rc})")
        del nk

    def close(self):
        if getattr(self, "_h", None):
            load().tfhe_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rc(self, rc, what):
        if rc != 0:
            msg = load().tfhe_last_error(self._h)
            raise FheError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    # -- kernel timing ----------------------------------------------------
    def timing_enable(self, on=True):
        self._rc(load().tfhe_timing_enable(self._h, 1 if on else 0), "tfhe_timing_enable")

    def timing_read(self, kind):
        """(launches, total_ms, cts) of kind 'br' (blind rotation) or 'ks'."""
        n, ms, cts = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_uint64()
        self._rc(load().tfhe_timing_read(self._h, 0 if kind == "br" else 1, ctypes.byref(n), ctypes.byref(ms),
                                         ctypes.byref(cts)), "tfhe_timing_read")
        return n.value, ms.value, cts.value

    def timing_log(self):
        """[(kind, ciphertexts)] of every launch since timing was enabled, in
        order; kind is 'br' or 'ks'."""
        L = load()
        cnt = ctypes.c_uint64()
        self._rc(L.tfhe_timing_log(self._h, None, None, 0, ctypes.byref(cnt)), "tfhe_timing_log")
        n = cnt.value
        k = (ctypes.c_uint32 * max(1, n))()
        z = (ctypes.c_uint32 * max(1, n))()
        self._rc(L.tfhe_timing_log(self._h, k, z, n, ctypes.byref(cnt)), "tfhe_timing_log")
        return [("br" if k[i] == 0 else "ks", int(z[i])) for i in range(n)]

    def graph_stats(self):
        """(captures, graph launches, graphs kept) of sql_scan_batch's graph cache."""
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        self._rc(load().tfhe_graph_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
                 "tfhe_graph_stats")
        return a.value, b.value, c.value

    def get_tuning(self):
        """Current knob values: {max_batch, row_pass, digit_blocks, split_groups}."""
        out = {}
        for name, key in (("max_batch", TFHE_TUNE_MAX_BATCH), ("row_pass", TFHE_TUNE_ROW_PASS),
                          ("digit_blocks", TFHE_TUNE_DIGIT_BLOCKS), ("split_groups", TFHE_TUNE_SPLIT_GROUPS)):
            v = ctypes.c_int64()
            self._rc(load().tfhe_get_tuning(self._h, key, ctypes.byref(v)), "tfhe_get_tuning")
            out[name] = v.value
        return out

    def set_tuning(self, max_batch=None, row_pass=None, digit_blocks=None, split_groups=None):
        L = load()
        if split_groups is not None:
            self._rc(L.tfhe_set_tuning(self._h, TFHE_TUNE_SPLIT_GROUPS, int(split_groups)), "tfhe_set_tuning")
        if digit_blocks is not None:
            self._rc(L.tfhe_set_tuning(self._h, TFHE_TUNE_DIGIT_BLOCKS, int(digit_blocks)), "tfhe_set_tuning")
        if max_batch is not None:
            self._rc(L.tfhe_set_tuning(self._h, TFHE_TUNE_MAX_BATCH, int(max_batch)), "tfhe_set_tuning")
        if row_pass is not None:
            self._rc(L.tfhe_set_tuning(self._h, TFHE_TUNE_ROW_PASS, int(row_pass)), "tfhe_set_tuning")

    # -- evaluation -------------------------------------------------------
    def set_kernel(self, kind):
        self._rc(load().tfhe_set_kernel(self._h, TFHE_KERNEL_PLAIN if kind == "plain" else TFHE_KERNEL_MFMA),
                 "tfhe_set_kernel")

    def sync(self, stream=None):
        self._rc(load().tfhe_ctx_sync(self._h, _stream(stream)), "tfhe_ctx_sync")

    def tfhe_bootstrap_batch(self, lwe_in, out, testv=None, B=None, stream=None):
        _check_dev(lwe_in, "lwe_in"); _check_dev(out, "out"); _check_dev(testv, "testv")
        B = lwe_in.shape[0] if B is None else B
        self._rc(load().tfhe_bootstrap_batch(self._h, _ptr(lwe_in), _ptr(testv), _ptr(out), B, _stream(stream)),
                 "tfhe_bootstrap_batch")

    def tfhe_bootstrap_batch_noalloc(self, lwe_in, out, testv=None, B=None, stream=None):
        """tfhe_bootstrap_batch on the library's static scratch array (no allocation)."""
        _check_dev(lwe_in, "lwe_in"); _check_dev(out, "out"); _check_dev(testv, "testv")
        B = lwe_in.shape[0] if B is None else B
        self._rc(load().tfhe_bootstrap_batch_noalloc(self._h, _ptr(lwe_in), _ptr(testv), _ptr(out), B,
                                                     _stream(stream)), "tfhe_bootstrap_batch_noalloc")

    def tfhe_keyswitch_batch(self, big_in, out, B=None, stream=None):
        _check_dev(big_in, "big_in"); _check_dev(out, "out")
        B = big_in.shape[0] if B is None else B
        self._rc(load().tfhe_keyswitch_batch(self._h, _ptr(big_in), _ptr(out), B, _stream(stream)),
                 "tfhe_keyswitch_batch")

    def tfhe_gate_batch(self, op, x, y, out, z=None, stream=None):
        for t, nm in ((x, "x"), (y, "y"), (z, "z"), (out, "out")):
            _check_dev(t, nm)
        self._rc(load().tfhe_gate_batch(self._h, GATE_OPS[op], _ptr(x), _ptr(y), _ptr(z), _ptr(out),
                                        x.shape[0], _stream(stream)), "tfhe_gate_batch")

    def sql_mask_scan(self, col, rows, w, op, lit_a, mask, lit_b=None, stream=None):
        for t, nm in ((col, "col"), (lit_a, "lit_a"), (lit_b, "lit_b"), (mask, "mask")):
            _check_dev(t, nm)
        self._rc(load().sql_mask_scan(self._h, _ptr(col), rows, w, SQL_OPS.get(op, op), _ptr(lit_a),
                                      _ptr(lit_b), _ptr(mask), _stream(stream)), "sql_mask_scan")

    def sql_masked_select(self, mask, col, rows, w, out, stream=None):
        for t, nm in ((mask, "mask"), (col, "col"), (out, "out")):
            _check_dev(t, nm)
        self._rc(load().sql_masked_select(self._h, _ptr(mask), _ptr(col), rows, w, _ptr(out), _stream(stream)),
                 "sql_masked_select")

    def sql_masked_sum(self, mask, col, rows, w, out, stream=None):
        for t, nm in ((mask, "mask"), (col, "col"), (out, "out")):
            _check_dev(t, nm)
        width = ctypes.c_uint32()
        self._rc(load().sql_masked_sum(self._h, _ptr(mask), _ptr(col), rows, w, _ptr(out), ctypes.byref(width),
                                       _stream(stream)), "sql_masked_sum")
        return width.value

    def sql_radix_mask_scan(self, col, rows, nb, op, lit, mask, stream=None):
        for t, nm in ((col, "col"), (lit, "lit"), (mask, "mask")):
            _check_dev(t, nm)
        self._rc(load().sql_radix_mask_scan(self._h, _ptr(col), rows, nb, SQL_OPS.get(op, op), _ptr(lit), _ptr(mask),
                                            _stream(stream)), "sql_radix_mask_scan")

    def sql_radix_masked_select(self, mask, col, rows, nb, out, stream=None):
        for t, nm in ((mask, "mask"), (col, "col"), (out, "out")):
            _check_dev(t, nm)
        self._rc(load().sql_radix_masked_select(self._h, _ptr(mask), _ptr(col), rows, nb, _ptr(out), _stream(stream)),
                 "sql_radix_masked_select")

    def sql_radix_sum(self, vals, rows, nb, out, stream=None):
        for t, nm in ((vals, "vals"), (out, "out")):
            _check_dev(t, nm)
        self._rc(load().sql_radix_sum(self._h, _ptr(vals), rows, nb, _ptr(out), _stream(stream)), "sql_radix_sum")

    def sql_expr_eval(self, nodes, cols, rows, w, out, lits=(), stream=None):
        """Evaluate an expression tree for every row.  nodes: list of dicts
        {"kind": column|const|literal|cmp|and|or|xor|not|max|min|ite, "col",
        "value", "lit" (index into lits), "op" (eq ne lt le gt ge), "a", "b",
        "c"}; cols, lits: device tensors [rows][w][n+1] and [w][n+1]; out:
        [rows][n+1] (boolean root) or [rows][w][n+1] (value root)."""
        for i, t in enumerate(cols):
            _check_dev(t, f"cols[{i}]")
        for i, t in enumerate(lits):
            _check_dev(t, f"lits[{i}]")
        _check_dev(out, "out")
        arr, colp = _expr_arrays(nodes, cols, lits)
        self._rc(load().sql_expr_eval(self._h, colp, len(cols), rows, w, arr, len(nodes), _ptr(out),
                                      _stream(stream)), "sql_expr_eval")

    def sql_scan_batch(self, queries, use_graph=False, stream=None):
        """queries: list of dicts with col, rows, w, op, lit_a, lit_b, mask, sel_col, sel_out."""
        arr = (SqlTableQuery * len(queries))()
        for i, q in enumerate(queries):
            for key in ("col", "lit_a", "lit_b", "mask", "sel_col", "sel_out"):
                _check_dev(q.get(key), key)
            arr[i] = SqlTableQuery(q["col"].data_ptr(), q["sel_col"].data_ptr() if q.get("sel_col") is not None else None,
                                   q["rows"], q["w"], SQL_OPS.get(q["op"], q["op"]), q["lit_a"].data_ptr(),
                                   q["lit_b"].data_ptr() if q.get("lit_b") is not None else None,
                                   q["mask"].data_ptr(),
                                   q["sel_out"].data_ptr() if q.get("sel_out") is not None else None)
        self._rc(load().sql_scan_batch(self._h, arr, len(queries), 1 if use_graph else 0, _stream(stream)),
                 "sql_scan_batch")


def _expr_arrays(nodes, cols, lits):
    """ctypes arrays of an expression node list (dicts) and its columns."""
    arr = (SqlExpr * max(1, len(nodes)))()
    for i, nd in enumerate(nodes):
        kind = nd["kind"]
        e = SqlExpr()
        e.kind = SQL_EXPR_KINDS.get(kind, -1) if isinstance(kind, str) else int(kind)
        e.op = SQL_CMP_OPS.get(nd.get("op"), -1) if isinstance(nd.get("op"), str) else int(nd.get("op", 0))
        e.a, e.b, e.c = int(nd.get("a", -1)), int(nd.get("b", -1)), int(nd.get("c", -1))
        e.col = int(nd.get("col", -1))
        e.value = int(nd.get("value", 0)) & 0xFFFFFFFFFFFFFFFF
        if kind == "literal":
            e.d_lit = lits[nd["lit"]].data_ptr()
        arr[i] = e
    colp = (ctypes.c_void_p * max(1, len(cols)))(*[t.data_ptr() for t in cols])
    return arr, colp


class Server:
    """Continuous-batching query server (sql_server_*) on a context."""

    def __init__(self, ctx, hbm_budget_bytes, max_batch=65536):
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        rc = load().sql_server_create(ctx._h, int(hbm_budget_bytes), int(max_batch), ctypes.byref(self._h))
        ctx._rc(rc, "sql_server_create")
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            load().sql_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, col, sum_col, rows, w, op, lit_a, out, lit_b=None):
        """Queue SELECT SUM(sum_col) WHERE col op lit; returns the query id."""
        for t, nm in ((col, "col"), (sum_col, "sum_col"), (lit_a, "lit_a"), (lit_b, "lit_b"), (out, "out")):
            _check_dev(t, nm)
        q = SqlSumQuery(col.data_ptr(), sum_col.data_ptr(), rows, w, SQL_OPS.get(op, op), lit_a.data_ptr(),
                        lit_b.data_ptr() if lit_b is not None else None, out.data_ptr())
        qid = ctypes.c_uint64()
        self.ctx._rc(load().sql_server_submit(self._h, ctypes.byref(q), ctypes.byref(qid)), "sql_server_submit")
        self._keep[qid.value] = (col, sum_col, lit_a, lit_b, out)
        return qid.value

    def submit_expr(self, nodes, cols, rows, w, sum_col, out, lits=()):
        """Queue SELECT SUM(sum_col) WHERE <expression tree> (nodes as in
        Context.sql_expr_eval); returns the query id."""
        for i, t in enumerate(list(cols) + list(lits) + [sum_col, out]):
            _check_dev(t, f"tensor {i}")
        arr, colp = _expr_arrays(nodes, cols, lits)
        qid = ctypes.c_uint64()
        self.ctx._rc(load().sql_server_submit_expr(self._h, colp, len(cols), rows, w, arr, len(nodes),
                                                   sum_col.data_ptr(), out.data_ptr(), ctypes.byref(qid)),
                     "sql_server_submit_expr")
        self._keep[qid.value] = (tuple(cols), tuple(lits), sum_col, out)
        return qid.value

    def step(self, stream=None):
        """One tick; returns (gates run, active, queued)."""
        g, a, q = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        self.ctx._rc(load().sql_server_step(self._h, _stream(stream), ctypes.byref(g), ctypes.byref(a),
                                            ctypes.byref(q)), "sql_server_step")
        return g.value, a.value, q.value

    def done(self, qid):
        rc = load().sql_server_done(self._h, qid)
        if rc < 0:
            raise FheError(f"unknown query id {qid}")
        if rc == 1:
            self._keep.pop(qid, None)
        return rc == 1

    def bytes_in_use(self):
        return load().sql_server_bytes_in_use(self._h)


def sum_width(w, rows):
    width = w
    r = rows
    while r > 1:
        width += 1
        r = (r + 1) // 2
    return width


# -- client-side device helpers ---------------------------------------------

def tfhe_keygen(p, seed, stream=None):
    """Seeded key generation on the device: returns (s, S, bsk, ksk) tensors."""
    import torch
    L = load()
    ps = params_struct(p)
    dt = torch_dtype(p.q)
    dev = torch.device("cuda")
    s = torch.empty(p.n, dtype=dt, device=dev)
    S = torch.empty(p.k * p.N, dtype=dt, device=dev)
    bsk = torch.empty(L.tfhe_bsk_words(ctypes.byref(ps)), dtype=dt, device=dev)
    ksk = torch.empty(L.tfhe_ksk_words(ctypes.byref(ps)), dtype=dt, device=dev)
    rc = L.tfhe_keygen(ctypes.byref(ps), seed, p.lwe_sigma_log2, p.glwe_sigma_log2, _ptr(s), _ptr(S), _ptr(bsk),
                       _ptr(ksk), _stream(stream))
    if rc != 0:
        raise FheError(f"tfhe_keygen failed ({rc})")
    return s, S, bsk, ksk


def tfhe_lwe_encrypt(p, seed, key, mu, dim=None, start=0, tag_hi=0, sigma_log2=None, stream=None):
    """Encrypt mu (device tensor of torus words) with seeded masks and noise."""
    import torch
    L = load()
    ps = params_struct(p)
    dim = p.n if dim is None else dim
    sigma = p.lwe_sigma_log2 if sigma_log2 is None else sigma_log2
    out = torch.empty((mu.numel(), dim + 1), dtype=torch_dtype(p.q), device=mu.device)
    rc = L.tfhe_lwe_encrypt(ctypes.byref(ps), seed, TAG_CT_MASK | (tag_hi << 32), TAG_CT_NOISE | (tag_hi << 32),
                            sigma, start, _ptr(key), _ptr(mu), _ptr(out), mu.numel(), dim, _stream(stream))
    if rc != 0:
        raise FheError(f"tfhe_lwe_encrypt failed ({rc})")
    return out


def tfhe_lwe_phase(p, key, cts, dim=None, stream=None):
    import torch
    L = load()
    ps = params_struct(p)
    dim = p.n if dim is None else dim
    cts2 = cts.reshape(-1, dim + 1)
    out = torch.empty(cts2.shape[0], dtype=torch_dtype(p.q), device=cts.device)
    rc = L.tfhe_lwe_phase(ctypes.byref(ps), _ptr(key), _ptr(cts2), _ptr(out), cts2.shape[0], dim, _stream(stream))
    if rc != 0:
        raise FheError(f"tfhe_lwe_phase failed ({rc})")
    return out.reshape(cts.shape[:-1])


def tfhe_rng_fill(seed, tag, count, start=0, stream=None):
    import torch
    out = torch.empty(count, dtype=torch.int64, device="cuda")
    rc = load().tfhe_rng_fill(seed, tag, start, count, _ptr(out), _stream(stream))
    if rc != 0:
        raise FheError(f"tfhe_rng_fill failed ({rc})")
    return out
