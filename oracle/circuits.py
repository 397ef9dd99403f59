"""Gate and SQL circuits of the oracle (test infrastructure only).

The FHE-SQL server (Algorithm 2, Section 4.3) builds a boolean mask per row by
evaluating the WHERE expression homomorphically and then selects
If-Then-Else(mask, value, enc(0)) (Eqs. 2-3), optionally summing the selected
values (the aggregation equations that follow them).  With TFHE gate
bootstrapping these become boolean circuits over bit-wise encrypted integers
(least significant bit first).  The gates are the TFHE paper's bootstrapped
gates (ePrint 2018/421, Sec. 4.2): a linear combination of the input
ciphertexts plus a constant, followed by a sign bootstrap that outputs
+-1/8.  A bit b is the torus value (2b - 1)/8.

Circuits are written once over a ``backend`` so the same netlist runs on
plaintext booleans (to pin its logic exhaustively) and on ciphertexts
(``CipherBackend``, built on the C oracle).

Readings of points the paper leaves open:
* equality: XNOR per bit, then a balanced AND tree pairing (0,1), (2,3), ...,
  an odd element passing up unchanged;
* a < c: borrow chain b_j = MAJ(not a_j, c_j, b_{j-1}), b_{-1} = FALSE;
* a > c is c < a; BETWEEN lo AND hi is NOR(a < lo, hi < a);
* select: AND(mask, v_j) per bit (If-Then-Else with an encrypted zero);
* SUM: pairwise adder tree in row order, ripple-carry adders whose carry-out
  becomes the new top bit; an odd operand is zero-extended by one FALSE bit;
* expression trees (the Homomorphic Expression Tree of Section 4.3 B): NOT is
  the exact negation of a ciphertext (no bootstrap); a != b, a <= b, a >= b
  are NOT(a == b), NOT(b < a), NOT(a < b); a plaintext constant is its
  trivial encryption (0, +-1/8) per bit; If-Then-Else(c, x, y) per bit is
  AND(c, x) + ANDNY(c, y) + 1/8 (a linear step: the two terms are never both
  TRUE); max(a, b) = ITE(a < b, b, a) and min(a, b) = ITE(a < b, a, b).
"""
from __future__ import annotations

import numpy as np

from . import (gate_bootstrap, lincomb, parallel_map, qmask)

# op -> (constant in units of 1/8, input weights)
GATES = {
    "AND": (-1, (1, 1)),
    "NAND": (1, (-1, -1)),
    "OR": (1, (1, 1)),
    "NOR": (-1, (-1, -1)),
    "XOR": (2, (2, 2)),
    "XNOR": (-2, (-2, -2)),
    "ANDNY": (-1, (-1, 1)),   # (not x) and y
    "MAJ": (0, (1, 1, 1)),
}


class PlainBackend:
    """Boolean reference semantics of each gate."""
    TRUE, FALSE = True, False

    def gate(self, op, *xs):
        x = [bool(v) for v in xs]
        if op == "AND": return x[0] and x[1]
        if op == "NAND": return not (x[0] and x[1])
        if op == "OR": return x[0] or x[1]
        if op == "NOR": return not (x[0] or x[1])
        if op == "XOR": return x[0] != x[1]
        if op == "XNOR": return x[0] == x[1]
        if op == "ANDNY": return (not x[0]) and x[1]
        if op == "MAJ": return (x[0] + x[1] + x[2]) >= 2
        raise ValueError(op)

    def neg(self, x):
        return not x

    def lin(self, xs, weights, c8):
        """Linear step on bits (+-1 in units of 1/8); the result must again
        be a valid bit encoding."""
        v = c8 + sum(w * (1 if x else -1) for w, x in zip(weights, xs))
        if v not in (-1, 1):
            raise ValueError(f"linear step leaves the bit encoding: {v}/8")
        return v == 1


class CipherBackend:
    """Bootstrapped gates on LWE ciphertexts (uint64 arrays of n+1 words)."""

    def __init__(self, p, keys):
        self.p = p
        self.keys = keys
        eighth = 1 << (p.q - 3)
        self.TRUE = np.zeros(p.n + 1, dtype=np.uint64)
        self.TRUE[p.n] = eighth
        self.FALSE = np.zeros(p.n + 1, dtype=np.uint64)
        self.FALSE[p.n] = (-eighth) & qmask(p.q)
        self.count = 0

    def combine(self, op, *xs):
        c8, w = GATES[op]
        const = (c8 * (1 << (self.p.q - 3))) & qmask(self.p.q)
        return lincomb(self.p, np.stack(xs), w, const)

    def gate(self, op, *xs):
        self.count += 1
        return gate_bootstrap(self.p, self.keys.bsk, self.keys.ksk, self.combine(op, *xs))

    def neg(self, x):
        out = (np.uint64(0) - np.asarray(x, dtype=np.uint64))
        return out & np.uint64(qmask(self.p.q))

    def lin(self, xs, weights, c8):
        const = (c8 * (1 << (self.p.q - 3))) & qmask(self.p.q)
        return lincomb(self.p, np.stack(xs), list(weights), const)


def eq(be, a, c):
    xs = [be.gate("XNOR", a[j], c[j]) for j in range(len(a))]
    while len(xs) > 1:
        nxt = [be.gate("AND", xs[2 * i], xs[2 * i + 1]) for i in range(len(xs) // 2)]
        if len(xs) % 2:
            nxt.append(xs[-1])
        xs = nxt
    return xs[0]


def lt(be, a, c):
    b = be.gate("MAJ", be.neg(a[0]), c[0], be.FALSE)
    for j in range(1, len(a)):
        b = be.gate("MAJ", be.neg(a[j]), c[j], b)
    return b


def gt(be, a, c):
    return lt(be, c, a)


def between(be, a, lo, hi):
    return be.gate("NOR", lt(be, a, lo), lt(be, hi, a))


def predicate(be, op, a, lit_a, lit_b=None):
    if op == "eq": return eq(be, a, lit_a)
    if op == "lt": return lt(be, a, lit_a)
    if op == "gt": return gt(be, a, lit_a)
    if op == "between": return between(be, a, lit_a, lit_b)
    raise ValueError(op)


def select(be, m, v):
    return [be.gate("AND", m, v[j]) for j in range(len(v))]


def add(be, x, y):
    """Ripple-carry sum of two equal-width operands; width grows by one."""
    s = [be.gate("XOR", x[0], y[0])]
    c = be.gate("AND", x[0], y[0])
    for j in range(1, len(x)):
        t = be.gate("XOR", x[j], y[j])
        s.append(be.gate("XOR", t, c))
        c = be.gate("MAJ", x[j], y[j], c)
    s.append(c)
    return s


def sum_tree(be, operands):
    """Pairwise adder tree over rows (0,1), (2,3), ...; odd leftover is
    zero-extended by one FALSE bit so every operand of a level has one width."""
    level = [list(o) for o in operands]
    while len(level) > 1:
        nxt = [add(be, level[2 * i], level[2 * i + 1]) for i in range(len(level) // 2)]
        if len(level) % 2:
            nxt.append(level[-1] + [be.FALSE])
        level = nxt
    return level[0]


# ---------------------------------------------------------- expression trees
#
# A WHERE expression (Section 4.3 B) is given as a list of nodes in
# topological order (every operand index smaller than the node's own); the
# last node is the root.  Node dicts:
#   {"kind": "column", "col": i}           value: encrypted column i
#   {"kind": "const", "value": v}          value: plaintext v (trivial encryption)
#   {"kind": "literal", "lit": i}          value: encrypted literal i
#   {"kind": "cmp", "op": o, "a": i, "b": j}   bool, o in eq ne lt le gt ge
#   {"kind": "and" | "or" | "xor", "a": i, "b": j}   bool
#   {"kind": "not", "a": i}                bool
#   {"kind": "max" | "min", "a": i, "b": j}   value
#   {"kind": "ite", "c": k, "a": i, "b": j}   value: c ? a : b
VALUE_KINDS = ("column", "const", "literal", "max", "min", "ite")
BOOL_KINDS = ("cmp", "and", "or", "xor", "not")


def compare(be, op, a, b):
    if op == "eq": return eq(be, a, b)
    if op == "ne": return be.neg(eq(be, a, b))
    if op == "lt": return lt(be, a, b)
    if op == "gt": return lt(be, b, a)
    if op == "le": return be.neg(lt(be, b, a))
    if op == "ge": return be.neg(lt(be, a, b))
    raise ValueError(op)


def mux(be, c, x, y):
    """c ? x : y on one bit: the AND terms are never both TRUE, so their sum
    plus 1/8 is again a bit."""
    return be.lin([be.gate("AND", c, x), be.gate("ANDNY", c, y)], [1, 1], 1)


def ite(be, c, x, y):
    return [mux(be, c, x[j], y[j]) for j in range(len(x))]


def expr_eval(be, nodes, cols, literals, w):
    """Value of the root of `nodes` for one row: a bit for a boolean root, a
    list of w bits for a value root.  cols[i] and literals[i] are lists of w
    bits of this backend."""
    vals, kinds = [], []
    for k, nd in enumerate(nodes):
        kind = nd["kind"]
        ops = [nd[x] for x in ("a", "b", "c") if x in nd]
        if any(not (0 <= i < k) for i in ops):
            raise ValueError(f"node {k}: operands must precede the node")
        if kind == "column":
            v = list(cols[nd["col"]])
        elif kind == "const":
            v = [be.TRUE if (int(nd["value"]) >> j) & 1 else be.FALSE for j in range(w)]
        elif kind == "literal":
            v = list(literals[nd["lit"]])
        elif kind in ("cmp", "max", "min"):
            if kinds[nd["a"]] != "value" or kinds[nd["b"]] != "value":
                raise ValueError(f"node {k}: {kind} takes values")
            a, b = vals[nd["a"]], vals[nd["b"]]
            if kind == "cmp":
                v = compare(be, nd["op"], a, b)
            else:
                m = lt(be, a, b)
                v = ite(be, m, b, a) if kind == "max" else ite(be, m, a, b)
        elif kind in ("and", "or", "xor"):
            if kinds[nd["a"]] != "bool" or kinds[nd["b"]] != "bool":
                raise ValueError(f"node {k}: {kind} takes booleans")
            v = be.gate(kind.upper(), vals[nd["a"]], vals[nd["b"]])
        elif kind == "not":
            if kinds[nd["a"]] != "bool":
                raise ValueError(f"node {k}: not takes a boolean")
            v = be.neg(vals[nd["a"]])
        elif kind == "ite":
            if kinds[nd["c"]] != "bool" or kinds[nd["a"]] != "value" or kinds[nd["b"]] != "value":
                raise ValueError(f"node {k}: ite takes a boolean and two values")
            v = ite(be, vals[nd["c"]], vals[nd["a"]], vals[nd["b"]])
        else:
            raise ValueError(f"node {k}: unknown kind {kind}")
        vals.append(v)
        kinds.append("value" if kind in VALUE_KINDS else "bool")
    return vals[-1]


def expr_plain(nodes, cols, literals, w):
    """Integer semantics of an expression tree (the pin of expr_eval)."""
    mask = (1 << w) - 1
    vals = []
    for nd in nodes:
        kind = nd["kind"]
        if kind == "column": v = cols[nd["col"]] & mask
        elif kind == "const": v = int(nd["value"]) & mask
        elif kind == "literal": v = literals[nd["lit"]] & mask
        elif kind == "cmp":
            a, b = vals[nd["a"]], vals[nd["b"]]
            v = {"eq": a == b, "ne": a != b, "lt": a < b, "le": a <= b, "gt": a > b, "ge": a >= b}[nd["op"]]
        elif kind == "and": v = vals[nd["a"]] and vals[nd["b"]]
        elif kind == "or": v = vals[nd["a"]] or vals[nd["b"]]
        elif kind == "xor": v = vals[nd["a"]] != vals[nd["b"]]
        elif kind == "not": v = not vals[nd["a"]]
        elif kind == "max": v = max(vals[nd["a"]], vals[nd["b"]])
        elif kind == "min": v = min(vals[nd["a"]], vals[nd["b"]])
        elif kind == "ite": v = vals[nd["a"]] if vals[nd["c"]] else vals[nd["b"]]
        else: raise ValueError(kind)
        vals.append(v)
    return vals[-1]


def expr_rows(p, keys, nodes, col_cts, lit_cts, w, threads=None):
    """Oracle evaluation of an expression tree for every row.
    col_cts: list of [rows][w][n+1] arrays; lit_cts: list of [w][n+1] arrays.
    Returns [rows][n+1] (boolean root) or [rows][w][n+1] (value root)."""
    rows = len(col_cts[0]) if col_cts else 1

    def one(r):
        be = CipherBackend(p, keys)
        out = expr_eval(be, nodes, [list(c[r]) for c in col_cts], [list(x) for x in lit_cts], w)
        return np.stack(out) if isinstance(out, list) else np.asarray(out, dtype=np.uint64)
    return np.stack(parallel_map(one, range(rows), threads))


# ------------------------------------------------------------------ drivers

def mask_rows(p, keys, op, col_cts, lit_a, lit_b=None, threads=None):
    """Oracle WHERE mask for every row: col_cts [rows][w][n+1] -> [rows][n+1]."""
    def one(r):
        be = CipherBackend(p, keys)
        return predicate(be, op, list(col_cts[r]), list(lit_a),
                         list(lit_b) if lit_b is not None else None)
    return np.stack(parallel_map(one, range(len(col_cts)), threads))


def select_rows(p, keys, masks, col_cts, threads=None):
    """Oracle masked select: AND(mask_r, bit) -> [rows][w][n+1]."""
    def one(r):
        be = CipherBackend(p, keys)
        return np.stack(select(be, masks[r], list(col_cts[r])))
    return np.stack(parallel_map(one, range(len(col_cts)), threads))


def gate_batch(p, keys, op, ins, threads=None):
    """One bootstrapped gate per row of ins ([B][nin][n+1])."""
    def one(i):
        be = CipherBackend(p, keys)
        return be.gate(op, *ins[i])
    return np.stack(parallel_map(one, range(len(ins)), threads))


# ------------------------------------------------- level-parallel evaluation

class _Node:
    __slots__ = ("op", "ins", "depth", "val")

    def __init__(self, op, ins, depth):
        self.op, self.ins, self.depth, self.val = op, ins, depth, None


class _Neg:
    __slots__ = ("x", "depth")

    def __init__(self, x, depth):
        self.x, self.depth = x, depth


class LazyBackend:
    """Records the netlist of a circuit instead of evaluating it, so that all
    gates of one depth (over many rows) can be bootstrapped in parallel.
    Leaves are ciphertext arrays; constants are the trivial ciphertexts."""

    def __init__(self, p):
        self.p = p
        eighth = 1 << (p.q - 3)
        self.TRUE = np.zeros(p.n + 1, dtype=np.uint64)
        self.TRUE[p.n] = eighth
        self.FALSE = np.zeros(p.n + 1, dtype=np.uint64)
        self.FALSE[p.n] = (-eighth) & qmask(p.q)
        self.nodes = []

    @staticmethod
    def _depth(x):
        return x.depth if isinstance(x, (_Node, _Neg)) else 0

    def gate(self, op, *xs):
        nd = _Node(op, xs, 1 + max(self._depth(x) for x in xs))
        self.nodes.append(nd)
        return nd

    def neg(self, x):
        return _Neg(x, self._depth(x))


def _value(p, x):
    if isinstance(x, _Node):
        return x.val
    if isinstance(x, _Neg):
        return (np.uint64(0) - _value(p, x.x)) & np.uint64(qmask(p.q))
    return np.asarray(x, dtype=np.uint64)


def evaluate(p, keys, lazy: LazyBackend, threads=None, progress=None):
    """Bootstrap every recorded gate, depth by depth, on a thread pool;
    progress(depth_done, depths, gates_done, gates) is called after each depth."""
    by_depth = {}
    for nd in lazy.nodes:
        by_depth.setdefault(nd.depth, []).append(nd)
    cb = CipherBackend(p, keys)

    def run(nd):
        nd.val = cb.gate(nd.op, *[_value(p, x) for x in nd.ins])

    depths = sorted(by_depth)
    total, done = len(lazy.nodes), 0
    for i, d in enumerate(depths):
        parallel_map(run, by_depth[d], threads)
        done += len(by_depth[d])
        if progress:
            progress(i + 1, len(depths), done, total)


def resolve(p, x):
    """Value of a recorded node (after evaluate) or of a leaf."""
    if isinstance(x, list):
        return np.stack([resolve(p, v) for v in x])
    return _value(p, x)


# ------------------------------------------------------------ radix circuits
#
# Programmable bootstrapping over radix integers (the reading used for the
# 64-bit workload): an integer is nb blocks of 4-bit messages, least
# significant block first; a block value x in [0, 32) (4 message bits plus
# one carry bit) is encrypted as x * delta with delta = 2^q / 64, the top bit
# of the torus left as padding.  A bootstrap with a table f over Z_32 maps an
# encryption of x to an encryption of f(x) * delta.
#   compare a vs c : x_i = a_i - c_i + 16 in [1, 31], r_i = CMP(x_i) with
#                    CMP = {<16: 0 (lt), 16: 1 (eq), >16: 2 (gt)};
#                    tree over blocks pairing (0,1),(2,3),...: 2*hi + lo -> COMB
#                    {0,1,2: 0; 3: 1; 4,5,6: 2}; the root uses ROOT_op, which
#                    outputs 16 when the relation holds and 0 otherwise.
#   select         : s_i = SEL(v_i + root), SEL(x) = x - 16 if x >= 16 else 0.
#   add            : z_i = x_i + y_i + carry_{i-1}; block MSG(z) = z mod 16 and,
#                    below the top block, carry CARRY(z) = z div 16 (wraps mod 2^(4 nb)).
#   SUM            : pairwise tree over rows, an odd operand passes up unchanged.

RADIX_P = 32       # plaintext modulus of a block (4 message bits + 1 carry bit)
RADIX_MSG = 16


def radix_tables():
    """Tables over Z_32 of the radix circuits."""
    P = RADIX_P
    cmp_ = [0 if x < 16 else (1 if x == 16 else 2) for x in range(P)]
    comb = [0 if x <= 2 else (1 if x == 3 else 2) if x <= 6 else 0 for x in range(P)]
    root = {
        "lt": [16 if x <= 2 else 0 for x in range(P)],
        "eq": [16 if x == 3 else 0 for x in range(P)],
        "gt": [16 if 4 <= x <= 6 else 0 for x in range(P)],
    }
    sel = [x - 16 if x >= 16 else 0 for x in range(P)]
    msg = [x % 16 for x in range(P)]
    carry = [x // 16 for x in range(P)]
    return {"cmp": cmp_, "comb": comb, "root_lt": root["lt"], "root_eq": root["eq"], "root_gt": root["gt"],
            "sel": sel, "msg": msg, "carry": carry}


class RadixPlainBackend:
    """Plaintext semantics: blocks are ints, lin() is the integer combination."""

    def __init__(self):
        self.t = radix_tables()

    def lin(self, ins, weights, const):
        return sum(w * x for w, x in zip(weights, ins)) + const

    def pbs(self, x, table):
        assert 0 <= x < RADIX_P, x
        return self.t[table][x]


class RadixCipherBackend:
    """Encrypted blocks: lin() is the LWE linear combination, pbs() the
    programmable bootstrap (blind rotation, extraction, key switch)."""

    def __init__(self, p, keys):
        from . import lut_testv
        self.p, self.keys = p, keys
        self.delta = 1 << (p.q - 6)
        self.tv = {name: lut_testv(p, RADIX_P, np.array(tab, dtype=np.uint64), self.delta)
                   for name, tab in radix_tables().items()}
        self.count = 0

    def lin(self, ins, weights, const):
        return lincomb(self.p, np.stack(ins), list(weights), (const * self.delta) & qmask(self.p.q))

    def pbs(self, x, table):
        from . import pbs
        self.count += 1
        return pbs(self.p, self.keys.bsk, self.keys.ksk, x, self.tv[table])


def radix_compare(be, op, a, c):
    """Encrypted 16 * [a op c] (op in lt, eq, gt) from block lists a, c."""
    r = [be.pbs(be.lin([a[i], c[i]], [1, -1], 16), "cmp") for i in range(len(a))]
    assert len(r) >= 2
    while len(r) > 1:
        root = len(r) == 2
        nxt = [be.pbs(be.lin([r[2 * i + 1], r[2 * i]], [2, 1], 0), f"root_{op}" if root else "comb")
               for i in range(len(r) // 2)]
        if len(r) % 2:
            nxt.append(r[-1])
        r = nxt
    return r[0]


def radix_select(be, m, v):
    return [be.pbs(be.lin([v[i], m], [1, 1], 0), "sel") for i in range(len(v))]


def radix_add(be, x, y):
    out, carry = [], None
    for i in range(len(x)):
        ins, ws = ([x[i], y[i]], [1, 1]) if carry is None else ([x[i], y[i], carry], [1, 1, 1])
        z = be.lin(ins, ws, 0)
        out.append(be.pbs(z, "msg"))
        if i + 1 < len(x):
            carry = be.pbs(z, "carry")
    return out


def radix_sum(be, operands):
    level = [list(o) for o in operands]
    while len(level) > 1:
        nxt = [radix_add(be, level[2 * i], level[2 * i + 1]) for i in range(len(level) // 2)]
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return level[0]


# ------------------------------------------- level-parallel radix evaluation

class _RLin:
    __slots__ = ("ins", "weights", "const", "depth")

    def __init__(self, ins, weights, const, depth):
        self.ins, self.weights, self.const, self.depth = ins, weights, const, depth


class _RPbs:
    __slots__ = ("x", "table", "depth", "val")

    def __init__(self, x, table, depth):
        self.x, self.table, self.depth, self.val = x, table, depth, None


class LazyRadixBackend:
    """Records a radix circuit (the same lin/pbs calls RadixCipherBackend
    takes) instead of evaluating it, so that the bootstraps of one depth over
    many rows run in parallel (``evaluate_radix``).  Leaves are ciphertext
    arrays.  The results are those of RadixCipherBackend: the same linear
    combinations and bootstraps, only in another order across independent
    gates."""

    def __init__(self, p):
        self.p = p
        self.nodes = []

    @staticmethod
    def _depth(x):
        return x.depth if isinstance(x, (_RLin, _RPbs)) else 0

    def lin(self, ins, weights, const):
        return _RLin(list(ins), list(weights), const, max(self._depth(x) for x in ins))

    def pbs(self, x, table):
        nd = _RPbs(x, table, 1 + self._depth(x))
        self.nodes.append(nd)
        return nd


def _rvalue(cb, x):
    if isinstance(x, _RPbs):
        return x.val
    if isinstance(x, _RLin):
        return cb.lin([_rvalue(cb, y) for y in x.ins], x.weights, x.const)
    return np.asarray(x, dtype=np.uint64)


def evaluate_radix(p, keys, lazy: LazyRadixBackend, threads=None, progress=None):
    """Run every recorded programmable bootstrap, depth by depth, on a thread
    pool; progress(depth_done, depths) is called after each depth."""
    cb = RadixCipherBackend(p, keys)
    by_depth = {}
    for nd in lazy.nodes:
        by_depth.setdefault(nd.depth, []).append(nd)

    def run(nd):
        nd.val = cb.pbs(_rvalue(cb, nd.x), nd.table)

    depths = sorted(by_depth)
    for i, d in enumerate(depths):
        parallel_map(run, by_depth[d], threads)
        if progress:
            progress(i + 1, len(depths))


def resolve_radix(p, keys, x):
    """Ciphertext of a recorded radix value (after evaluate_radix) or leaf."""
    if isinstance(x, list):
        return np.stack([resolve_radix(p, keys, v) for v in x])
    return _rvalue(RadixCipherBackend(p, keys), x)
