// Host-side netlists of the gate circuits: the circuit builders (mask
// predicates, select, SUM, radix circuits, expression trees), the cutting of
// a netlist's levels into launches, and the continuous-batching server's
// bookkeeping.  Plain C++17 with no HIP dependency, so that a host compiler
// can build and check it on its own (under AddressSanitizer and
// UndefinedBehaviorSanitizer); the kernels and launches live in sql.hip.
//
// The circuits follow Algorithm 2's mask per row, If-Then-Else(mask, value,
// enc(0)) of Eqs. 2-3 and the aggregation after Eq. 3, evaluated with TFHE
// gate bootstrapping over bit-wise encrypted integers (least significant bit
// first):
//   equality  : XNOR per bit, balanced AND tree (pairs (0,1),(2,3),...; an
//               odd element passes up);
//   a < c     : borrow chain b_j = MAJ(not a_j, c_j, b_{j-1}), b_{-1} = FALSE;
//   a > c     : c < a;   BETWEEN lo AND hi: NOR(a < lo, hi < a);
//   select    : AND(mask, v_j) per bit;
//   SUM       : pairwise ripple-carry adder tree over rows in row order, the
//               carry-out as new top bit, an odd operand zero-extended;
// and with programmable bootstrapping over radix blocks for 64-bit tori.
// A netlist is a list of levels; a level is a list of strided segments (one
// gate per row of a group) plus device copies and linear steps that run
// before its gates.
#pragma once

#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <deque>
#include <string>
#include <unordered_set>
#include <utility>
#include <vector>

#include "../../include/fhesql.h"

// ------------------------------------------------------------------ gates

// Bootstrapped gates (TFHE gate bootstrapping): constant in units of 1/8 and
// input weights of the linear combination that precedes the sign bootstrap.
enum GateOp { G_AND = 0, G_NAND, G_OR, G_NOR, G_XOR, G_XNOR, G_ANDNY, G_MAJ, G_LUT };

struct GateForm {
    int c8;
    int nin;
    int w[3];
};
inline GateForm gate_form(int op) {
    switch (op) {
        case G_AND: return {-1, 2, {1, 1, 0}};
        case G_NAND: return {1, 2, {-1, -1, 0}};
        case G_OR: return {1, 2, {1, 1, 0}};
        case G_NOR: return {-1, 2, {-1, -1, 0}};
        case G_XOR: return {2, 2, {2, 2, 0}};
        case G_XNOR: return {-2, 2, {-2, -2, 0}};
        case G_ANDNY: return {-1, 2, {-1, 1, 0}};
        case G_MAJ: return {0, 3, {1, 1, 1}};
        default: return {0, 0, {0, 0, 0}};
    }
}

// One strided group of gates of a level: gate r (0 <= r < rows) combines
// in[j] + r*in_stride[j] (word addresses) with weights w[j] and a constant,
// and writes its bootstrapped output to out + r*out_stride.  Constant
// (trivial) operands are folded into `cst` by the host, so the nin inputs
// are real ciphertexts.
struct Segment {
    uint64_t in[3];
    int64_t in_stride[3];
    uint64_t out;
    int64_t out_stride;
    uint64_t cst;     // constant body term (torus word)
    int32_t w[3];
    int32_t nin;
    uint32_t rows;
    int32_t lut;      // test polynomial index, -1 = gate test polynomial
};

// ------------------------------------------------------------- netlists

struct Ref {  // a ciphertext operand: word address + row stride in words
    uint64_t addr;
    int64_t stride;
};

struct Copy {  // device-to-device copy done before a level's gates
    uint64_t src, dst, bytes;
};

struct Level {
    std::vector<Segment> segs;    // bootstrapped gates
    std::vector<Copy> copies;     // run first
    std::vector<Segment> lins;    // linear steps, run after the copies, before the gates
};

struct Netlist {
    std::vector<Level> levels;
    size_t tmp_words = 0;  // words of temporaries used (relative addresses)
    const void* lut_table = nullptr;  // test polynomials indexed by Segment::lut
};

// Temporaries are addressed relative to a base chosen at execution time:
// the high bit marks a relative address, resolved when segments are uploaded.
constexpr uint64_t REL = 1ull << 63;

struct Builder {
    int q;      // torus bits (32 or 64)
    size_t wb;  // bytes per torus word
    size_t lw;  // words per small LWE
    Netlist net;

    Builder(int q_, uint32_t n) : q(q_), wb(q_ == 32 ? 4 : 8), lw((size_t)n + 1) {}

    uint64_t eighth() const { return q == 32 ? (1ull << 29) : (1ull << 61); }
    uint64_t wrap(int64_t v) const {
        uint64_t u = (uint64_t)v;
        return q == 32 ? (u & 0xFFFFFFFFull) : u;
    }
    Ref tmp(uint32_t rows) {
        Ref r{REL | (net.tmp_words * wb), (int64_t)lw};
        net.tmp_words += (size_t)rows * lw;
        return r;
    }
    void level_push(size_t lev, const Segment& s) {
        if (net.levels.size() <= lev) net.levels.resize(lev + 1);
        net.levels[lev].segs.push_back(s);
    }
    void lin_push(size_t lev, const Segment& s) {
        if (net.levels.size() <= lev) net.levels.resize(lev + 1);
        net.levels[lev].lins.push_back(s);
    }
    void copy_push(size_t lev, uint64_t src, uint64_t dst, uint64_t bytes) {
        if (net.levels.size() <= lev) net.levels.resize(lev + 1);
        net.levels[lev].copies.push_back(Copy{src, dst, bytes});
    }
    // Gate on `rows` rows; operands given as refs (nullptr entries = FALSE constant).
    void gate(size_t lev, int op, uint32_t rows, std::vector<const Ref*> ins, Ref out) {
        GateForm f = gate_form(op);
        Segment s{};
        int64_t cst = (int64_t)f.c8;  // units of 1/8
        int k = 0;
        for (int j = 0; j < f.nin; j++) {
            const Ref* r = ins[j];
            if (!r) {  // trivial FALSE = (0, -1/8) contributes -w_j/8
                cst -= f.w[j];
                continue;
            }
            s.in[k] = r->addr;
            s.in_stride[k] = r->stride;
            s.w[k] = f.w[j];
            k++;
        }
        s.nin = k;
        s.cst = wrap(cst * (int64_t)eighth());
        s.out = out.addr;
        s.out_stride = out.stride;
        s.rows = rows;
        s.lut = -1;
        level_push(lev, s);
    }
    void gate_w(size_t lev, uint32_t rows, std::vector<std::pair<const Ref*, int>> ins, int64_t cst8, Ref out) {
        Segment s{};
        int64_t cst = cst8;
        int k = 0;
        for (auto& pr : ins) {
            if (!pr.first) { cst -= pr.second; continue; }
            s.in[k] = pr.first->addr;
            s.in_stride[k] = pr.first->stride;
            s.w[k] = pr.second;
            k++;
        }
        s.nin = k;
        s.cst = wrap(cst * (int64_t)eighth());
        s.out = out.addr;
        s.out_stride = out.stride;
        s.rows = rows;
        s.lut = -1;
        level_push(lev, s);
    }

    // Linear combination (constant in torus words) followed by a bootstrap
    // with test polynomial `lut` of the netlist's table.
    void lin(size_t lev, uint32_t rows, std::vector<std::pair<const Ref*, int>> ins, uint64_t cst, Ref out, int lut) {
        Segment s{};
        int k = 0;
        for (auto& pr : ins) {
            s.in[k] = pr.first->addr;
            s.in_stride[k] = pr.first->stride;
            s.w[k] = pr.second;
            k++;
        }
        s.nin = k;
        s.cst = wrap((int64_t)cst);
        s.out = out.addr;
        s.out_stride = out.stride;
        s.rows = rows;
        s.lut = lut;
        level_push(lev, s);
    }

    // ---- radix circuits (blocks of 4-bit messages + 1 carry bit, delta = 2^q/64)
    enum { L_CMP = 0, L_COMB, L_ROOT_LT, L_ROOT_EQ, L_ROOT_GT, L_SEL, L_MSG, L_CARRY, L_COUNT };
    uint64_t delta() const { return 1ull << ((q == 32 ? 32 : 64) - 6); }

    size_t radix_compare(size_t lev, uint32_t rows, uint32_t nb, int op, const Ref& col, const Ref& lit, Ref out) {
        std::vector<Ref> r;
        for (uint32_t i = 0; i < nb; i++) {
            Ref a = bit(col, i, lw, wb), ci = bit(lit, i, lw, wb);
            Ref o = tmp(rows);
            lin(lev, rows, {{&a, 1}, {&ci, -1}}, 16 * delta(), o, L_CMP);
            r.push_back(o);
        }
        lev++;
        const int root = op == SQL_OP_LT ? L_ROOT_LT : op == SQL_OP_EQ ? L_ROOT_EQ : L_ROOT_GT;
        while (r.size() > 1) {
            std::vector<Ref> nxt;
            const bool last = r.size() == 2;
            for (size_t i = 0; i < r.size() / 2; i++) {
                Ref o = last ? out : tmp(rows);
                lin(lev, rows, {{&r[2 * i + 1], 2}, {&r[2 * i], 1}}, 0, o, last ? root : L_COMB);
                nxt.push_back(o);
            }
            if (r.size() % 2) nxt.push_back(r.back());
            r.swap(nxt);
            lev++;
        }
        return lev;
    }
    size_t radix_select(size_t lev, uint32_t rows, uint32_t nb, const Ref& mask, const Ref& col, Ref out) {
        for (uint32_t i = 0; i < nb; i++) {
            Ref v = bit(col, i, lw, wb), o = bit(out, i, lw, wb);
            lin(lev, rows, {{&v, 1}, {&mask, 1}}, 0, o, L_SEL);
        }
        return lev + 1;
    }
    // Pairwise row tree of ripple-carry additions; operands [rows][nb] at `vals`.
    size_t radix_sum(size_t lev, uint32_t rows, uint32_t nb, Ref vals, uint64_t sum) {
        Ref cur = vals;
        uint32_t cnt = rows;
        auto at = [&](const Ref& base, uint32_t opd, uint32_t i, int64_t stride) -> Ref {
            return Ref{base.addr + ((uint64_t)opd * base.stride + (uint64_t)i * lw) * wb, stride};
        };
        if (rows == 1) {
            copy_push(lev, cur.addr, sum, (uint64_t)nb * lw * wb);
            return lev + 1;
        }
        while (cnt > 1) {
            const uint32_t pairs = cnt / 2;
            const bool odd = cnt & 1;
            const bool last = pairs + (odd ? 1 : 0) == 1;
            Ref res;
            if (last) res = Ref{sum, (int64_t)(nb * lw)};
            else { res = tmp((pairs + (odd ? 1 : 0)) * nb); res.stride = (int64_t)(nb * lw); }
            const int64_t xs = 2 * cur.stride;
            Ref carry{};
            for (uint32_t i = 0; i < nb; i++) {
                Ref x = at(cur, 0, i, xs), y = at(cur, 1, i, xs);
                std::vector<std::pair<const Ref*, int>> ins = {{&x, 1}, {&y, 1}};
                if (i) ins.push_back({&carry, 1});
                lin(lev + i, pairs, ins, 0, at(res, 0, i, res.stride), L_MSG);
                if (i + 1 < nb) {
                    Ref nc = tmp(pairs);
                    lin(lev + i, pairs, ins, 0, nc, L_CARRY);
                    carry = nc;
                }
            }
            if (odd) copy_push(lev, at(cur, cnt - 1, 0, 0).addr, at(res, pairs, 0, 0).addr, (uint64_t)nb * lw * wb);
            lev += nb;
            cnt = pairs + (odd ? 1 : 0);
            cur = res;
        }
        return lev;
    }

    static Ref bit(const Ref& base, uint32_t j, size_t lw_, size_t wb_) {
        return Ref{base.addr + (uint64_t)j * lw_ * wb_, base.stride};
    }

    // Returns the level after the last one used; the root output goes to `out`.
    size_t eq(size_t lev, uint32_t rows, uint32_t w, const Ref& col, const Ref& lit, Ref out) {
        std::vector<Ref> nodes;
        for (uint32_t j = 0; j < w; j++) {
            Ref a = bit(col, j, lw, wb), cj = bit(lit, j, lw, wb);
            Ref o = w == 1 ? out : tmp(rows);
            gate(lev, G_XNOR, rows, {&a, &cj}, o);
            nodes.push_back(o);
        }
        lev++;
        while (nodes.size() > 1) {
            std::vector<Ref> nxt;
            const size_t pairs = nodes.size() / 2;
            for (size_t i = 0; i < pairs; i++) {
                const bool root = nodes.size() == 2;
                Ref o = root ? out : tmp(rows);
                gate(lev, G_AND, rows, {&nodes[2 * i], &nodes[2 * i + 1]}, o);
                nxt.push_back(o);
            }
            if (nodes.size() % 2) nxt.push_back(nodes.back());
            nodes.swap(nxt);
            lev++;
        }
        return lev;
    }
    // a < c as a borrow chain; swap = true computes c < a.
    size_t lt(size_t lev, uint32_t rows, uint32_t w, const Ref& a, const Ref& cc, Ref out, bool swap) {
        Ref prev{};
        for (uint32_t j = 0; j < w; j++) {
            Ref x = bit(swap ? cc : a, j, lw, wb), y = bit(swap ? a : cc, j, lw, wb);
            Ref o = j + 1 == w ? out : tmp(rows);
            // MAJ(not x, y, b) = -x + y + b; b_{-1} = FALSE
            gate_w(lev + j, rows, {{&x, -1}, {&y, 1}, {j ? &prev : nullptr, 1}}, 0, o);
            prev = o;
        }
        return lev + w;
    }
    size_t predicate(size_t lev, uint32_t rows, uint32_t w, int op, const Ref& col, const Ref& la,
                     const Ref* lb, Ref out) {
        switch (op) {
            case SQL_OP_EQ: return eq(lev, rows, w, col, la, out);
            case SQL_OP_LT: return lt(lev, rows, w, col, la, out, false);
            case SQL_OP_GT: return lt(lev, rows, w, col, la, out, true);
            case SQL_OP_BETWEEN: {
                Ref b1 = tmp(rows), b2 = tmp(rows);
                lt(lev, rows, w, col, la, b1, false);   // col < lo
                lt(lev, rows, w, col, *lb, b2, true);   // hi < col
                gate(lev + w, G_NOR, rows, {&b1, &b2}, out);
                return lev + w + 1;
            }
        }
        return lev;
    }
    size_t select(size_t lev, uint32_t rows, uint32_t w, const Ref& mask, const Ref& col, Ref out) {
        for (uint32_t j = 0; j < w; j++) {
            Ref cj = bit(col, j, lw, wb), oj = bit(out, j, lw, wb);
            gate(lev, G_AND, rows, {&mask, &cj}, oj);
        }
        return lev + 1;
    }

    // Masked SUM: select into a [rows][w] operand buffer, then a pairwise
    // ripple-carry adder tree over rows (pairs (0,1),(2,3),...; an odd last
    // operand passes up unchanged with a trivial FALSE top bit).  Result bits
    // (w + ceil(log2 rows) of them) go to `sum` (stride n+1 words per bit).
    size_t masked_sum(size_t lev, uint32_t rows, uint32_t w, const Ref& mask, const Ref& col, uint64_t sum,
                      uint64_t false_ct) {
        Ref cur = tmp(rows * w);
        cur.stride = (int64_t)(w * lw);
        lev = select(lev, rows, w, mask, col, cur);
        uint32_t cnt = rows, width = w;
        auto at = [&](const Ref& base, uint32_t op, uint32_t j, int64_t stride) -> Ref {
            return Ref{base.addr + ((uint64_t)op * base.stride + (uint64_t)j * lw) * wb, stride};
        };
        while (cnt > 1) {
            const uint32_t pairs = cnt / 2;
            const bool odd = cnt & 1;
            const uint32_t nw = width + 1;
            const bool last = (pairs + (odd ? 1 : 0)) == 1;
            Ref res;
            if (last) res = Ref{sum, (int64_t)(nw * lw)};
            else { res = tmp((pairs + (odd ? 1 : 0)) * nw); res.stride = (int64_t)(nw * lw); }
            const int64_t xs = 2 * cur.stride;  // operand-pair stride
            Ref x0 = at(cur, 0, 0, xs), y0 = at(cur, 1, 0, xs);
            Ref carry = width == 1 ? at(res, 0, 1, res.stride) : tmp(pairs);
            gate(lev, G_XOR, pairs, {&x0, &y0}, at(res, 0, 0, res.stride));
            gate(lev, G_AND, pairs, {&x0, &y0}, carry);
            Ref tb = tmp(pairs * width);
            tb.stride = (int64_t)(width * lw);
            for (uint32_t j = 1; j < width; j++) {
                Ref xj = at(cur, 0, j, xs), yj = at(cur, 1, j, xs);
                gate(lev, G_XOR, pairs, {&xj, &yj}, at(tb, 0, j, tb.stride));
            }
            for (uint32_t j = 1; j < width; j++) {
                Ref xj = at(cur, 0, j, xs), yj = at(cur, 1, j, xs);
                Ref tj = at(tb, 0, j, tb.stride);
                Ref nc = j + 1 == width ? at(res, 0, width, res.stride) : tmp(pairs);
                gate(lev + j, G_XOR, pairs, {&tj, &carry}, at(res, 0, j, res.stride));
                gate(lev + j, G_MAJ, pairs, {&xj, &yj, &carry}, nc);
                carry = nc;
            }
            if (odd) {
                const Ref src = at(cur, cnt - 1, 0, 0), dst = at(res, pairs, 0, 0);
                copy_push(lev, src.addr, dst.addr, (uint64_t)width * lw * wb);
                copy_push(lev, false_ct, at(res, pairs, width, 0).addr, lw * wb);
            }
            lev += width;
            cnt = pairs + (odd ? 1 : 0);
            width = nw;
            cur = res;
        }
        if (rows == 1) copy_push(lev, cur.addr, sum, (uint64_t)w * lw * wb);
        return lev + (rows == 1 ? 1 : 0);
    }
};

// ---------------------------------------------------- expression trees

// A wire is one encrypted bit for every row: a ciphertext reference whose
// sign carries folded NOTs (w * (-x) = (-w) * x exactly mod 2^q), or a
// plaintext constant (its trivial encryption (0, +-1/8) folded into the
// consuming step's constant).  rg / rl: first level whose gates / linear
// steps may read the wire (a linear step's output is read by the gates of its
// own level, by linear steps only from the next level on).
struct Wire {
    bool is_const = false;
    bool val = false;
    Ref r{};
    int sign = 1;
    size_t rg = 0, rl = 0;
};

struct ExprVal {
    bool is_bool = false;
    std::vector<Wire> bits;  // 1 for a boolean, w for a value
};

struct ExprCompiler {
    Builder& b;
    uint32_t rows;

    static Wire constant(bool v) {
        Wire x;
        x.is_const = true;
        x.val = v;
        return x;
    }
    static Wire neg(Wire x) {
        if (x.is_const) x.val = !x.val;
        else x.sign = -x.sign;
        return x;
    }
    // Fills a segment's operands from (wire, weight) pairs; returns the
    // constant in units of 1/8 after folding constant wires.
    static int64_t operands(Segment& s, const std::vector<std::pair<const Wire*, int>>& ins, int64_t cst8) {
        int k = 0;
        for (auto& pr : ins) {
            const Wire& x = *pr.first;
            if (x.is_const) { cst8 += x.val ? pr.second : -pr.second; continue; }
            s.in[k] = x.r.addr;
            s.in_stride[k] = x.r.stride;
            s.w[k] = pr.second * x.sign;
            k++;
        }
        s.nin = k;
        return cst8;
    }
    // Bootstrapped gate; placed at the first level where every operand exists.
    Wire gate(int op, std::vector<const Wire*> ins) {
        const GateForm f = gate_form(op);
        size_t lev = 0;
        std::vector<std::pair<const Wire*, int>> wi;
        for (int j = 0; j < f.nin; j++) {
            if (!ins[j]->is_const) lev = std::max(lev, ins[j]->rg);
            wi.push_back({ins[j], f.w[j]});
        }
        Segment s{};
        const int64_t cst8 = operands(s, wi, f.c8);
        Wire o;
        o.r = b.tmp(rows);
        s.cst = b.wrap(cst8 * (int64_t)b.eighth());
        s.out = o.r.addr;
        s.out_stride = o.r.stride;
        s.rows = rows;
        s.lut = -1;
        b.level_push(lev, s);
        o.rg = o.rl = lev + 1;
        return o;
    }
    // Linear step (no bootstrap) into `out` (a fresh temporary when null).
    Wire lin(const std::vector<std::pair<const Wire*, int>>& ins, int64_t cst8, const Ref* out) {
        size_t lev = 0;
        for (auto& pr : ins)
            if (!pr.first->is_const) lev = std::max(lev, pr.first->rl);
        Segment s{};
        cst8 = operands(s, ins, cst8);
        Wire o;
        o.r = out ? *out : b.tmp(rows);
        s.cst = b.wrap(cst8 * (int64_t)b.eighth());
        s.out = o.r.addr;
        s.out_stride = o.r.stride;
        s.rows = rows;
        s.lut = -1;
        b.lin_push(lev, s);
        o.rg = lev;
        o.rl = lev + 1;
        return o;
    }

    Wire eq(const ExprVal& a, const ExprVal& c) {
        std::vector<Wire> xs;
        for (size_t j = 0; j < a.bits.size(); j++) xs.push_back(gate(G_XNOR, {&a.bits[j], &c.bits[j]}));
        while (xs.size() > 1) {  // pairs (0,1),(2,3),...; an odd last element passes up
            std::vector<Wire> nxt;
            for (size_t i = 0; i + 1 < xs.size(); i += 2) nxt.push_back(gate(G_AND, {&xs[i], &xs[i + 1]}));
            if (xs.size() % 2) nxt.push_back(xs.back());
            xs.swap(nxt);
        }
        return xs[0];
    }
    Wire lt(const ExprVal& a, const ExprVal& c) {  // borrow chain, b_{-1} = FALSE
        Wire bw = constant(false);
        for (size_t j = 0; j < a.bits.size(); j++) {
            const Wire na = neg(a.bits[j]);
            bw = gate(G_MAJ, {&na, &c.bits[j], &bw});
        }
        return bw;
    }
    Wire compare(int op, const ExprVal& a, const ExprVal& c) {
        switch (op) {
            case SQL_CMP_EQ: return eq(a, c);
            case SQL_CMP_NE: return neg(eq(a, c));
            case SQL_CMP_LT: return lt(a, c);
            case SQL_CMP_GT: return lt(c, a);
            case SQL_CMP_LE: return neg(lt(c, a));
            default: return neg(lt(a, c));  // SQL_CMP_GE
        }
    }
    // c ? x : y per bit: AND(c, x) + ANDNY(c, y) + 1/8 (never both TRUE).
    ExprVal ite(const Wire& cw, const ExprVal& x, const ExprVal& y) {
        ExprVal o;
        for (size_t j = 0; j < x.bits.size(); j++) {
            const Wire u1 = gate(G_AND, {&cw, &x.bits[j]});
            const Wire u2 = gate(G_ANDNY, {&cw, &y.bits[j]});
            o.bits.push_back(lin({{&u1, 1}, {&u2, 1}}, 1, nullptr));
        }
        return o;
    }
};

inline Ref dev(const void* p, size_t stride_words) { return Ref{(uint64_t)(uintptr_t)p, (int64_t)stride_words}; }

// Checks an expression node list (operands precede their node, kinds and
// types match, pointers present); isb[k] receives whether node k is boolean.
// On failure *err receives the reason.
inline int check_expr(const void* const* d_cols, uint32_t ncols, uint32_t w, const sql_expr* nodes, uint32_t nnodes,
                      std::vector<char>& isb, std::string* err) {
    auto fail = [&](int code, const std::string& m) {
        if (err) *err = m;
        return code;
    };
    if (!nodes || !nnodes) return fail(TFHE_EINVAL, "empty expression");
    if (w < 1 || w > 64) return fail(TFHE_ESHAPE, "value width must be 1..64 bits");
    if (ncols && !d_cols) return fail(TFHE_EINVAL, "null column array");
    isb.assign(nnodes, 0);
    for (uint32_t k = 0; k < nnodes; k++) {
        const sql_expr& e = nodes[k];
        auto opnd = [&](int32_t i, bool want_bool) {
            return i >= 0 && (uint32_t)i < k && (isb[i] != 0) == want_bool;
        };
        bool ok = true;
        switch (e.kind) {
            case SQL_EXPR_COLUMN: ok = e.col >= 0 && (uint32_t)e.col < ncols && d_cols[e.col]; break;
            case SQL_EXPR_CONST: break;
            case SQL_EXPR_LITERAL: ok = e.d_lit != nullptr; break;
            case SQL_EXPR_CMP: ok = e.op >= SQL_CMP_EQ && e.op <= SQL_CMP_GE && opnd(e.a, false) && opnd(e.b, false); break;
            case SQL_EXPR_AND: case SQL_EXPR_OR: case SQL_EXPR_XOR: ok = opnd(e.a, true) && opnd(e.b, true); break;
            case SQL_EXPR_NOT: ok = opnd(e.a, true); break;
            case SQL_EXPR_MAX: case SQL_EXPR_MIN: ok = opnd(e.a, false) && opnd(e.b, false); break;
            case SQL_EXPR_ITE: ok = opnd(e.c, true) && opnd(e.a, false) && opnd(e.b, false); break;
            default: ok = false;
        }
        if (!ok) {
            char msg[96];
            snprintf(msg, sizeof msg, "expression node %u: bad kind, operator, operand or pointer", k);
            return fail(TFHE_EINVAL, msg);
        }
        isb[k] = e.kind == SQL_EXPR_CMP || e.kind == SQL_EXPR_AND || e.kind == SQL_EXPR_OR ||
                 e.kind == SQL_EXPR_XOR || e.kind == SQL_EXPR_NOT;
    }
    return TFHE_OK;
}

// Adds the circuits of a checked node list to b's netlist and returns the
// root's wires (not yet materialized).
inline ExprVal compile_expr(Builder& b, const void* const* d_cols, uint32_t rows, uint32_t w, const sql_expr* nodes,
                     uint32_t nnodes, const std::vector<char>& isb) {
    ExprCompiler ec{b, rows};
    const size_t lw = b.lw, wb = b.wb;
    std::vector<ExprVal> v(nnodes);
    for (uint32_t k = 0; k < nnodes; k++) {
        const sql_expr& e = nodes[k];
        ExprVal& o = v[k];
        o.is_bool = isb[k] != 0;
        switch (e.kind) {
            case SQL_EXPR_COLUMN:
            case SQL_EXPR_LITERAL: {
                const Ref base = e.kind == SQL_EXPR_COLUMN ? dev(d_cols[e.col], (size_t)w * lw) : dev(e.d_lit, 0);
                for (uint32_t j = 0; j < w; j++) {
                    Wire x;
                    x.r = Builder::bit(base, j, lw, wb);
                    o.bits.push_back(x);
                }
                break;
            }
            case SQL_EXPR_CONST:
                for (uint32_t j = 0; j < w; j++) o.bits.push_back(ExprCompiler::constant((e.value >> j) & 1));
                break;
            case SQL_EXPR_CMP: o.bits.push_back(ec.compare(e.op, v[e.a], v[e.b])); break;
            case SQL_EXPR_AND: o.bits.push_back(ec.gate(G_AND, {&v[e.a].bits[0], &v[e.b].bits[0]})); break;
            case SQL_EXPR_OR: o.bits.push_back(ec.gate(G_OR, {&v[e.a].bits[0], &v[e.b].bits[0]})); break;
            case SQL_EXPR_XOR: o.bits.push_back(ec.gate(G_XOR, {&v[e.a].bits[0], &v[e.b].bits[0]})); break;
            case SQL_EXPR_NOT: o.bits.push_back(ExprCompiler::neg(v[e.a].bits[0])); break;
            case SQL_EXPR_MAX:
            case SQL_EXPR_MIN: {
                const Wire m = ec.lt(v[e.a], v[e.b]);
                o.bits = e.kind == SQL_EXPR_MAX ? ec.ite(m, v[e.b], v[e.a]).bits : ec.ite(m, v[e.a], v[e.b]).bits;
                break;
            }
            case SQL_EXPR_ITE: o.bits = ec.ite(v[e.c].bits[0], v[e.a], v[e.b]).bits; break;
        }
    }
    return v[nnodes - 1];
}

// ------------------------------------------------------------ schedules

// One launch of the level executor: gates of one level (a piece of it when
// the level holds more gates than the launch size), with the level's copies
// and linear steps attached to its first piece.
struct Piece {
    size_t seg_off;
    int nseg;
    uint32_t total;      // gates of the launch
    size_t copy_off;
    int ncopy;
    size_t lin_off;
    int nlin;
    uint32_t lin_total;  // rows of the linear steps
};

struct Schedule {
    uint32_t chunk = 0;            // gates of the largest launch
    std::vector<Segment> flat;     // each level's linear steps, then its pieces' gate segments
    std::vector<uint32_t> starts;  // first row of each flat segment within its launch
    std::vector<Piece> pieces;
    std::vector<Copy> copies;
};

// Cuts every level of net into launches of at most min(max_batch, widest
// level) gates.  A segment cut between two launches continues in the next
// one at the row where the first stopped (its addresses moved by that many
// rows, wb bytes per word).  Addresses stay as the builder made them
// (temporaries relative).
inline Schedule plan_schedule(const Netlist& net, uint32_t max_batch, size_t wb) {
    Schedule sc;
    size_t max_gates = 0, nlinear = 0;
    for (auto& lv : net.levels) {
        size_t g = 0;
        for (auto& sg : lv.segs) g += sg.rows;
        max_gates = std::max(max_gates, g);
        nlinear += lv.copies.size() + lv.lins.size();
    }
    if (!max_gates && !nlinear) return sc;
    const uint32_t chunk = (uint32_t)std::max<size_t>(1, std::min<size_t>(max_gates, std::max<uint32_t>(1, max_batch)));
    sc.chunk = chunk;
    for (auto& L : net.levels) {
        auto& lv = L.segs;
        const size_t c0 = sc.copies.size();
        sc.copies.insert(sc.copies.end(), L.copies.begin(), L.copies.end());
        const size_t l0 = sc.flat.size();
        uint32_t lin_total = 0;
        for (const Segment& sg : L.lins) {
            sc.flat.push_back(sg);
            sc.starts.push_back(lin_total);
            lin_total += sg.rows;
        }
        if (lv.empty() && (!L.copies.empty() || lin_total))
            sc.pieces.push_back(Piece{sc.flat.size(), 0, 0, c0, (int)L.copies.size(), l0, (int)L.lins.size(), lin_total});
        bool first = true;
        size_t i = 0;
        uint32_t carried = 0;  // rows of segment i already emitted
        while (i < lv.size()) {
            Piece pc{sc.flat.size(), 0, 0, c0, first ? (int)L.copies.size() : 0,
                     l0, first ? (int)L.lins.size() : 0, first ? lin_total : 0u};
            first = false;
            while (i < lv.size() && pc.total < chunk) {
                if (lv[i].rows == 0) { i++; continue; }
                Segment sg = lv[i];
                const uint32_t take = std::min<uint32_t>(sg.rows - carried, chunk - pc.total);
                for (int j = 0; j < sg.nin; j++) sg.in[j] += (uint64_t)((int64_t)carried * sg.in_stride[j]) * wb;
                sg.out += (uint64_t)((int64_t)carried * sg.out_stride) * wb;
                sg.rows = take;
                sc.flat.push_back(sg);
                sc.starts.push_back(pc.total);
                pc.total += take;
                pc.nseg++;
                carried += take;
                if (carried == lv[i].rows) { i++; carried = 0; }
            }
            if (pc.total || pc.ncopy || pc.nlin) sc.pieces.push_back(pc);
        }
    }
    return sc;
}

// ------------------------------------------------- server bookkeeping

// A query of the continuous-batching server: its netlist, its temporaries
// (device base address once admitted) and how far its levels have been
// issued.
struct ServerQuery {
    uint64_t id = 0;
    Netlist net;
    size_t tmp_bytes = 0;
    uint64_t tmp = 0;
    size_t level = 0;   // next level to issue
    size_t seg = 0;     // next segment of that level
    uint32_t row = 0;   // rows of that segment already issued
    bool copies_done = false;
    uint64_t last_tick = ~0ull;  // the tick that issued its last level
};

// What one server tick runs: copies, then linear steps, then the gates
// (segments with their start rows within the tick's launch).
struct Tick {
    std::vector<Segment> segs;
    std::vector<uint32_t> starts;
    std::vector<Segment> lins;
    std::vector<uint32_t> lin_starts;
    std::vector<Copy> copies;
    uint32_t total = 0;      // gates
    uint32_t lin_total = 0;  // linear-step rows
};

// Admission (device memory budget), level-by-level issue of every active
// query's gates into ticks of at most max_batch gates and seg_cap segments
// (a level may span ticks; a query's next level is issued only after the
// tick that issues the last gates of the current one; ticks run in order on
// the device, so a tick may be issued before the previous one finished), and
// retirement once the tick that ran a query's last level has finished.
struct ServerBook {
    size_t budget = 0;       // device bytes the server may account for
    size_t fixed = 0;        // keys and staging, accounted from creation
    size_t in_use = 0;       // fixed + admitted queries' temporaries
    uint32_t max_batch = 0;
    size_t seg_cap = 1 << 15;
    uint32_t max_active = 256;
    uint64_t next_id = 1;
    uint64_t ticks = 0;      // ticks issued so far (the next tick's number)
    std::deque<ServerQuery*> queue;
    std::vector<ServerQuery*> active;
    std::unordered_set<uint64_t> done, known;

    static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

    // Takes ownership of q; fails (deleting it) if it could never fit.
    int enqueue(ServerQuery* q, size_t wb, uint64_t* id, std::string* err) {
        q->tmp_bytes = al256(q->net.tmp_words * wb);
        if (fixed + q->tmp_bytes > budget) {
            delete q;
            if (err) *err = "query working set exceeds the HBM budget";
            return TFHE_ENOMEM;
        }
        q->id = next_id++;
        known.insert(q->id);
        queue.push_back(q);
        *id = q->id;
        return TFHE_OK;
    }

    // Admits queued queries in arrival order while their temporaries fit the
    // budget.  alloc(bytes) returns the device base of a query's
    // temporaries, 0 on failure (which stops admission with TFHE_ENOMEM).
    template <class Alloc>
    int admit(Alloc alloc, std::string* err) {
        while (!queue.empty() && active.size() < max_active) {
            ServerQuery* q = queue.front();
            if (in_use + q->tmp_bytes > budget) break;  // wait for memory to free
            const uint64_t base = alloc(q->tmp_bytes ? q->tmp_bytes : 256);
            if (!base) {
                if (err) *err = "query temporaries";
                return TFHE_ENOMEM;
            }
            q->tmp = base;
            auto res = [&](uint64_t a) { return (a & REL) ? base + (a & ~REL) : a; };
            for (auto& L : q->net.levels) {
                for (auto* group : {&L.segs, &L.lins})
                    for (auto& sg : *group) {
                        for (int j = 0; j < sg.nin; j++) sg.in[j] = res(sg.in[j]);
                        sg.out = res(sg.out);
                    }
                for (auto& cp : L.copies) { cp.src = res(cp.src); cp.dst = res(cp.dst); }
            }
            in_use += q->tmp_bytes;
            active.push_back(q);
            queue.pop_front();
        }
        return TFHE_OK;
    }

    // Issues tick number `ticks`: every active query in admission order adds
    // its current level's copies and linear steps (when that level starts)
    // and as many of its gates as fit.
    void next_tick(Tick& t, size_t wb) {
        t = Tick();
        size_t nlin = 0;
        for (auto* q : active) {
            if (q->level >= q->net.levels.size()) {
                if (q->last_tick == ~0ull) q->last_tick = ticks;  // (a netlist without levels)
                continue;
            }
            if (t.total >= max_batch || t.segs.size() + nlin >= seg_cap) break;
            Level& L = q->net.levels[q->level];
            if (!q->copies_done) {
                if (t.segs.size() + nlin + L.lins.size() >= seg_cap) break;  // the next tick takes this level
                t.copies.insert(t.copies.end(), L.copies.begin(), L.copies.end());
                for (const Segment& sg : L.lins) {
                    t.lins.push_back(sg);
                    t.lin_starts.push_back(t.lin_total);
                    t.lin_total += sg.rows;
                }
                nlin += L.lins.size();
                q->copies_done = true;
            }
            while (q->seg < L.segs.size() && t.total < max_batch && t.segs.size() + nlin < seg_cap) {
                Segment sg = L.segs[q->seg];
                const uint32_t take = std::min<uint32_t>(sg.rows - q->row, max_batch - t.total);
                for (int j = 0; j < sg.nin; j++) sg.in[j] += (uint64_t)((int64_t)q->row * sg.in_stride[j]) * wb;
                sg.out += (uint64_t)((int64_t)q->row * sg.out_stride) * wb;
                sg.rows = take;
                if (take) {
                    t.segs.push_back(sg);
                    t.starts.push_back(t.total);
                    t.total += take;
                }
                q->row += take;
                if (q->row == L.segs[q->seg].rows) { q->seg++; q->row = 0; }
            }
            if (q->seg == L.segs.size()) {  // level fully issued; the next tick runs the next one
                q->level++;
                q->seg = 0;
                q->copies_done = false;
                if (q->level >= q->net.levels.size()) q->last_tick = ticks;
            }
        }
        ticks++;
    }

    // Retires the queries whose last level ran in a tick before `completed`
    // (every tick numbered below it has finished on the device);
    // release(base) frees a query's temporaries.
    template <class Release>
    void retire(Release release, uint64_t completed) {
        std::vector<ServerQuery*> keep;
        for (auto* q : active) {
            if (q->level >= q->net.levels.size() && q->last_tick < completed) {
                done.insert(q->id);
                release(q->tmp);
                in_use -= q->tmp_bytes;
                delete q;
            } else {
                keep.push_back(q);
            }
        }
        active.swap(keep);
    }

    // Frees every query still held (release for admitted ones).
    template <class Release>
    void clear(Release release) {
        for (auto* q : active) {
            release(q->tmp);
            delete q;
        }
        for (auto* q : queue) delete q;
        active.clear();
        queue.clear();
    }
};
