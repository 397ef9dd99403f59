// Gate circuits of the FHE-SQL server path on the GPU.
//
// Algorithm 2 of the paper computes a mask bit per row by evaluating the
// WHERE expression tree homomorphically, then If-Then-Else(mask, value,
// enc(0)) on the selected columns (Eqs. 2-3), optionally summing the selected
// values.  With TFHE gate bootstrapping each operation is a boolean circuit
// over bit-wise encrypted integers (LSB first):
//   equality  : XNOR per bit, balanced AND tree (pairs (0,1),(2,3),...; an
//               odd element passes up);
//   a < c     : borrow chain b_j = MAJ(not a_j, c_j, b_{j-1}), b_{-1} = FALSE;
//   a > c     : c < a;   BETWEEN lo AND hi: NOR(a < lo, hi < a);
//   select    : AND(mask, v_j) per bit;
//   SUM       : pairwise ripple-carry adder tree over rows in row order, the
//               carry-out as new top bit, an odd operand zero-extended.
// A netlist is a list of levels; a level is a list of strided segments
// (one gate per row of a group).  Each level runs device copies, then linear
// steps without a bootstrap (expression trees' If-Then-Else sums and root
// outputs), then three kernels over the gates of every segment: linear
// combination, blind rotation + sample extraction (MFMA or plain), key
// switching into the gate outputs.
#include <algorithm>
#include <cstdio>
#include <cstring>

#include "fhesql_internal.h"

// ------------------------------------------------------------- combine

namespace {

template <typename T>
__global__ __launch_bounds__(256) void combine_kernel(const Segment* __restrict__ segs, const uint32_t* __restrict__ start,
                                                      int nseg, uint32_t total, T* out, uint64_t* out_ptrs,
                                                      int32_t* tv_index, int n) {
    const uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= total) return;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {  // last segment with start <= g
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const Segment& sg = segs[lo];
    const int64_t r = (int64_t)(g - start[lo]);
    const T* in0 = (const T*)(uintptr_t)sg.in[0] + r * sg.in_stride[0];
    const T* in1 = (const T*)(uintptr_t)sg.in[1] + r * sg.in_stride[1];
    const T* in2 = (const T*)(uintptr_t)sg.in[2] + r * sg.in_stride[2];
    const T w0 = (T)(int64_t)sg.w[0], w1 = (T)(int64_t)sg.w[1], w2 = (T)(int64_t)sg.w[2];
    T* o = out + (size_t)g * (n + 1);
    for (int w = lane; w <= n; w += 64) {
        T acc = w == n ? (T)sg.cst : (T)0;
        if (sg.nin > 0) acc += w0 * in0[w];
        if (sg.nin > 1) acc += w1 * in1[w];
        if (sg.nin > 2) acc += w2 * in2[w];
        o[w] = acc;
    }
    if (lane == 0) {
        out_ptrs[g] = sg.out + (uint64_t)(r * sg.out_stride) * sizeof(T);
        tv_index[g] = sg.lut < 0 ? 0 : sg.lut;
    }
}

}  // namespace

int launch_combine(tfhe_ctx* c, const Segment* d_segs, const uint32_t* d_start, int nseg, uint32_t total,
                   void* lwe_out, uint64_t* out_ptrs, int32_t* tv_index, hipStream_t s) {
    if (!total) return TFHE_OK;
    const unsigned grid = (total + 3) / 4;
    if (c->q == 32)
        hipLaunchKernelGGL(combine_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, d_segs, d_start, nseg, total,
                           (uint32_t*)lwe_out, out_ptrs, tv_index, (int)c->p.n);
    else
        hipLaunchKernelGGL(combine_kernel<uint64_t>, dim3(grid), dim3(256), 0, s, d_segs, d_start, nseg, total,
                           (uint64_t*)lwe_out, out_ptrs, tv_index, (int)c->p.n);
    return hip_check(c, hipGetLastError(), "launch combine");
}

// Linear steps without a bootstrap (exact negation, the If-Then-Else sum,
// copies of an expression's result): out[r] = cst*e_n + sum_j w_j in_j[r],
// written straight to each segment's output rows.
namespace {

template <typename T>
__global__ __launch_bounds__(256) void lin_kernel(const Segment* __restrict__ segs, const uint32_t* __restrict__ start,
                                                  int nseg, uint32_t total, int n) {
    const uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= total) return;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const Segment& sg = segs[lo];
    const int64_t r = (int64_t)(g - start[lo]);
    const T* in0 = (const T*)(uintptr_t)sg.in[0] + r * sg.in_stride[0];
    const T* in1 = (const T*)(uintptr_t)sg.in[1] + r * sg.in_stride[1];
    const T* in2 = (const T*)(uintptr_t)sg.in[2] + r * sg.in_stride[2];
    const T w0 = (T)(int64_t)sg.w[0], w1 = (T)(int64_t)sg.w[1], w2 = (T)(int64_t)sg.w[2];
    T* o = (T*)(uintptr_t)sg.out + r * sg.out_stride;
    for (int w = lane; w <= n; w += 64) {
        T acc = w == n ? (T)sg.cst : (T)0;
        if (sg.nin > 0) acc += w0 * in0[w];
        if (sg.nin > 1) acc += w1 * in1[w];
        if (sg.nin > 2) acc += w2 * in2[w];
        o[w] = acc;
    }
}

int launch_lin(tfhe_ctx* c, const Segment* d_segs, const uint32_t* d_start, int nseg, uint32_t total, hipStream_t s) {
    if (!total) return TFHE_OK;
    const unsigned grid = (total + 3) / 4;
    if (c->q == 32)
        hipLaunchKernelGGL(lin_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, d_segs, d_start, nseg, total, (int)c->p.n);
    else
        hipLaunchKernelGGL(lin_kernel<uint64_t>, dim3(grid), dim3(256), 0, s, d_segs, d_start, nseg, total, (int)c->p.n);
    return hip_check(c, hipGetLastError(), "launch lin");
}

}  // namespace

// ------------------------------------------------------------- netlists

namespace {

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
    tfhe_ctx* c;
    size_t wb;
    size_t lw;  // words per small LWE
    Netlist net;

    explicit Builder(tfhe_ctx* cc) : c(cc), wb(word_bytes(cc)), lw(cc->p.n + 1) {}

    uint64_t eighth() const { return c->q == 32 ? (1ull << 29) : (1ull << 61); }
    uint64_t wrap(int64_t v) const {
        uint64_t u = (uint64_t)v;
        return c->q == 32 ? (u & 0xFFFFFFFFull) : u;
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
    uint64_t delta() const { return 1ull << ((c->q == 32 ? 32 : 64) - 6); }

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

// ---------------------------------------------------------- execution
// ---------------------------------------------------------- execution

struct Exec {
    tfhe_ctx* c;
    hipStream_t s;
    size_t wb, lw, bw;
    uint32_t max_batch;

    Exec(tfhe_ctx* cc, hipStream_t ss) : c(cc), s(ss), wb(word_bytes(cc)), lw(cc->p.n + 1),
                                          bw((size_t)cc->p.k * cc->p.N + 1), max_batch(cc->max_batch) {}

    // Lay out the workspace: temporaries, then per-level staging.
    int run(Netlist& net, bool use_graph) {
        size_t max_gates = 0, nseg_total = 0;
        for (auto& lv : net.levels) {
            size_t g = 0;
            for (auto& sg : lv.segs) g += sg.rows;
            max_gates = std::max(max_gates, g);
            nseg_total += lv.segs.size();
        }
        size_t ncopies = 0;
        for (auto& lv : net.levels) ncopies += lv.copies.size() + lv.lins.size();
        if (!max_gates && !ncopies) return TFHE_OK;
        const uint32_t chunk = (uint32_t)std::max<size_t>(1, std::min<size_t>(max_gates, max_batch));
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        const size_t tmp_b = al(net.tmp_words * wb);
        const size_t lwe_b = al((size_t)chunk * lw * wb);
        const size_t big_b = al((size_t)chunk * bw * wb);
        const size_t ptr_b = al((size_t)chunk * 8);
        const size_t tvi_b = al((size_t)chunk * 4);
        // pieces of a level can be smaller than the chunk (and then take the
        // multi-workgroup blind rotation), so size for any batch up to it
        const size_t br_b = al(blind_rotate_ws_bytes_upto(c, chunk));
        // segments split into chunks: upper bound of pieces
        std::vector<Segment> flat;
        std::vector<uint32_t> starts;
        // A level's first piece also carries its copies and linear steps.
        struct Piece {
            size_t seg_off; int nseg; uint32_t total; size_t copy_off; int ncopy;
            size_t lin_off; int nlin; uint32_t lin_total;
        };
        std::vector<Piece> pieces;
        std::vector<Copy> copies;
        for (auto& L : net.levels) {
            auto& lv = L.segs;
            const size_t c0 = copies.size();
            copies.insert(copies.end(), L.copies.begin(), L.copies.end());
            const size_t l0 = flat.size();
            uint32_t lin_total = 0;
            for (const Segment& sg : L.lins) {
                flat.push_back(sg);
                starts.push_back(lin_total);
                lin_total += sg.rows;
            }
            bool first = true;
            // split the level into chunks of at most `chunk` gates
            size_t i = 0;
            uint32_t carried = 0;  // rows of segment i already emitted
            if (lv.empty() && (!L.copies.empty() || lin_total))
                pieces.push_back(Piece{flat.size(), 0, 0, c0, (int)L.copies.size(), l0, (int)L.lins.size(), lin_total});
            while (i < lv.size()) {
                Piece pc{flat.size(), 0, 0, c0, first ? (int)L.copies.size() : 0,
                         l0, first ? (int)L.lins.size() : 0, first ? lin_total : 0u};
                first = false;
                while (i < lv.size() && pc.total < chunk) {
                    Segment sg = lv[i];
                    const uint32_t take = std::min<uint32_t>(sg.rows - carried, chunk - pc.total);
                    for (int j = 0; j < sg.nin; j++) sg.in[j] += (uint64_t)(carried * sg.in_stride[j]) * wb;
                    sg.out += (uint64_t)(carried * sg.out_stride) * wb;
                    sg.rows = take;
                    flat.push_back(sg);
                    starts.push_back(pc.total);
                    pc.total += take;
                    pc.nseg++;
                    carried += take;
                    if (carried == lv[i].rows) { i++; carried = 0; }
                }
                pieces.push_back(pc);
            }
        }
        const size_t seg_b = al(flat.size() * sizeof(Segment));
        const size_t st_b = al(starts.size() * 4);
        const size_t total = tmp_b + lwe_b + big_b + ptr_b + tvi_b + br_b + seg_b + st_b;
        int rc = ws_acquire(c, s, total);
        if (rc) return rc;
        uint8_t* base = (uint8_t*)c->ws;
        uint8_t* tmp = base;
        uint8_t* lwe = tmp + tmp_b;
        uint8_t* big = lwe + lwe_b;
        uint64_t* ptrs = (uint64_t*)(big + big_b);
        int32_t* tvi = (int32_t*)((uint8_t*)ptrs + ptr_b);
        uint8_t* brws = (uint8_t*)tvi + tvi_b;
        Segment* dsegs = (Segment*)(brws + br_b);
        uint32_t* dstart = (uint32_t*)((uint8_t*)dsegs + seg_b);
        auto resolve = [&](uint64_t a) -> uint64_t { return (a & REL) ? (uint64_t)(uintptr_t)tmp + (a & ~REL) : a; };
        for (auto& sg : flat) {
            for (int j = 0; j < 3; j++) sg.in[j] = j < sg.nin ? resolve(sg.in[j]) : 0;
            sg.out = resolve(sg.out);
        }
        for (auto& cp : copies) {
            cp.src = resolve(cp.src);
            cp.dst = resolve(cp.dst);
        }
        // the segment table and the piece starts, uploaded as one block
        std::vector<uint8_t> host(seg_b + st_b, 0);
        memcpy(host.data(), flat.data(), flat.size() * sizeof(Segment));
        memcpy(host.data() + seg_b, starts.data(), starts.size() * 4);
        if ((rc = stage_upload(c, s, dsegs, host.data(), host.size()))) return rc;

        auto enqueue = [&](hipStream_t rs) -> int {
            int e = TFHE_OK;
            for (auto& pc : pieces) {
                for (int k = 0; k < pc.ncopy && !e; k++) {
                    const Copy& cp = copies[pc.copy_off + k];
                    e = hip_check(c, hipMemcpyAsync((void*)(uintptr_t)cp.dst, (const void*)(uintptr_t)cp.src,
                                                    cp.bytes, hipMemcpyDeviceToDevice, rs), "level copy");
                }
                if (e) break;
                if (pc.nlin && (e = launch_lin(c, dsegs + pc.lin_off, dstart + pc.lin_off, pc.nlin, pc.lin_total, rs)))
                    break;
                if (!pc.total) continue;
                if ((e = launch_combine(c, dsegs + pc.seg_off, dstart + pc.seg_off, pc.nseg, pc.total, lwe, ptrs, tvi,
                                        rs)))
                    break;
                if ((e = launch_blind_rotate(c, lwe, net.lut_table, net.lut_table ? tvi : nullptr, big, pc.total,
                                             brws, br_b, rs)))
                    break;
                if ((e = launch_keyswitch(c, big, nullptr, ptrs, pc.total, rs))) break;
            }
            return e;
        };
        if (!use_graph) {
            rc = enqueue(s);
        } else {
            // A graph is keyed by everything that fixes its launches: the
            // uploaded table (resolved addresses), the pieces, the copies,
            // the tuning and the workspace; a schedule seen before relaunches
            // its instantiated graph.
            std::vector<uint8_t> key(host);
            auto put = [&](const void* p, size_t n) {
                const uint8_t* b = (const uint8_t*)p;
                key.insert(key.end(), b, b + n);
            };
            for (const Piece& pc : pieces) {  // field by field (no padding bytes in the key)
                const uint64_t f[8] = {pc.seg_off, (uint64_t)pc.nseg, pc.total, pc.copy_off, (uint64_t)pc.ncopy,
                                       pc.lin_off, (uint64_t)pc.nlin, pc.lin_total};
                put(f, sizeof f);
            }
            put(copies.data(), copies.size() * sizeof(Copy));
            const uint64_t meta[8] = {(uint64_t)(uintptr_t)net.lut_table, (uint64_t)c->kernel, c->max_batch,
                                      (uint64_t)c->row_pass, (uint64_t)c->digit_blocks,
                                      (uint64_t)(uintptr_t)c->ws, (uint64_t)c->ws_bytes, (uint64_t)br_b};
            put(meta, sizeof meta);
            hipGraphExec_t exec = nullptr;
            for (auto& g : c->graphs)
                if (g.key == key) { exec = g.exec; g.last_use = ++c->graph_clock; break; }
            if (!exec) {
                hipStream_t cap = nullptr;
                hipGraph_t graph = nullptr;
                if ((rc = hip_check(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "create capture stream")))
                    return rc;
                rc = hip_check(c, hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
                if (!rc) {
                    rc = enqueue(cap);
                    hipError_t e = hipStreamEndCapture(cap, &graph);
                    if (!rc) rc = hip_check(c, e, "end capture");
                }
                if (!rc) rc = hip_check(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
                if (graph) hipGraphDestroy(graph);
                hipStreamDestroy(cap);
                if (rc) {
                    ws_release(c, s);
                    return rc;
                }
                constexpr size_t kMaxGraphs = 8;
                if (c->graphs.size() >= kMaxGraphs) {
                    // evict the least recently used graph once nothing that
                    // used the workspace (every graph does) is in flight
                    auto lru = std::min_element(c->graphs.begin(), c->graphs.end(),
                                                [](const tfhe_ctx::GraphEntry& a, const tfhe_ctx::GraphEntry& b) {
                                                    return a.last_use < b.last_use;
                                                });
                    if (c->ws_used && (rc = hip_check(c, hipEventSynchronize(c->ws_event), "graph eviction")))
                        return rc;
                    hipGraphExecDestroy(lru->exec);
                    c->graphs.erase(lru);
                }
                c->graphs.push_back(tfhe_ctx::GraphEntry{std::move(key), exec, ++c->graph_clock});
                c->graph_captures++;
            }
            rc = hip_check(c, hipGraphLaunch(exec, s), "graph launch");
            c->graph_launches++;
        }
        const int rr = ws_release(c, s);
        return rc ? rc : rr;
    }
};

Ref dev(const void* p, size_t stride_words) { return Ref{(uint64_t)(uintptr_t)p, (int64_t)stride_words}; }

}  // namespace

// ------------------------------------------------------------ C ABI

extern "C" int tfhe_gate_batch(tfhe_ctx* c, int op, const void* d_x, const void* d_y, const void* d_z, void* d_out,
                               uint32_t B, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (op < G_AND || op > G_MAJ) return ctx_fail(c, TFHE_EINVAL, "unknown gate");
    if (!B) return TFHE_OK;
    if (!d_x || !d_y || !d_out || (op == G_MAJ && !d_z)) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    Builder b(c);
    const size_t lw = b.lw;
    Ref x = dev(d_x, lw), y = dev(d_y, lw), z = dev(d_z, lw), o = dev(d_out, lw);
    if (op == G_MAJ) b.gate(0, op, B, {&x, &y, &z}, o);
    else b.gate(0, op, B, {&x, &y}, o);
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}

static int check_scan(tfhe_ctx* c, const void* col, uint32_t w, int op, const void* la, const void* lb, const void* mask) {
    if (!col || !la || !mask) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    if (w < 1 || w > 64) return ctx_fail(c, TFHE_ESHAPE, "column width must be 1..64 bits");
    if (op < SQL_OP_EQ || op > SQL_OP_BETWEEN) return ctx_fail(c, TFHE_EINVAL, "unknown SQL operator");
    if (op == SQL_OP_BETWEEN && !lb) return ctx_fail(c, TFHE_EINVAL, "BETWEEN needs an upper literal");
    return TFHE_OK;
}

extern "C" int sql_mask_scan(tfhe_ctx* c, const void* d_col, uint32_t rows, uint32_t w, int op, const void* d_lit_a,
                             const void* d_lit_b, void* d_mask, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!rows) return TFHE_OK;
    int rc = check_scan(c, d_col, w, op, d_lit_a, d_lit_b, d_mask);
    if (rc) return rc;
    Builder b(c);
    const size_t lw = b.lw;
    Ref col = dev(d_col, (size_t)w * lw), la = dev(d_lit_a, 0), lb = dev(d_lit_b, 0), m = dev(d_mask, lw);
    b.predicate(0, rows, w, op, col, la, d_lit_b ? &lb : nullptr, m);
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}

extern "C" int sql_masked_select(tfhe_ctx* c, const void* d_mask, const void* d_col, uint32_t rows, uint32_t w,
                                 void* d_out, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!rows) return TFHE_OK;
    if (!d_mask || !d_col || !d_out) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    if (w < 1 || w > 64) return ctx_fail(c, TFHE_ESHAPE, "column width must be 1..64 bits");
    Builder b(c);
    const size_t lw = b.lw;
    b.select(0, rows, w, dev(d_mask, lw), dev(d_col, (size_t)w * lw), dev(d_out, (size_t)w * lw));
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}

extern "C" int sql_scan_batch(tfhe_ctx* c, const sql_table_query* q, uint32_t count, int use_graph, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!count) return TFHE_OK;
    if (!q) return ctx_fail(c, TFHE_EINVAL, "null query array");
    Builder b(c);
    const size_t lw = b.lw;
    for (uint32_t t = 0; t < count; t++) {
        const sql_table_query& Q = q[t];
        if (!Q.rows) continue;
        int rc = check_scan(c, Q.d_col, Q.w, Q.op, Q.d_lit_a, Q.d_lit_b, Q.d_mask);
        if (rc) return rc;
        Ref col = dev(Q.d_col, (size_t)Q.w * lw), la = dev(Q.d_lit_a, 0), lb = dev(Q.d_lit_b, 0), m = dev(Q.d_mask, lw);
        const size_t lev = b.predicate(0, Q.rows, Q.w, Q.op, col, la, Q.d_lit_b ? &lb : nullptr, m);
        if (Q.d_sel_col && Q.d_sel_out)
            b.select(lev, Q.rows, Q.w, m, dev(Q.d_sel_col, (size_t)Q.w * lw), dev(Q.d_sel_out, (size_t)Q.w * lw));
    }
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, use_graph != 0);
}

extern "C" int sql_masked_sum(tfhe_ctx* c, const void* d_mask, const void* d_col, uint32_t rows, uint32_t w,
                              void* d_sum, uint32_t* width_out, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!d_mask || !d_col || !d_sum) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    if (w < 1 || w > 32) return ctx_fail(c, TFHE_ESHAPE, "column width must be 1..32 bits");
    if (!rows) return ctx_fail(c, TFHE_ESHAPE, "SUM needs at least one row");
    uint32_t final_w = w;
    for (uint32_t r = rows; r > 1; r = (r + 1) / 2) final_w++;
    if (width_out) *width_out = final_w;
    Builder b(c);
    const size_t lw = b.lw;
    b.masked_sum(0, rows, w, dev(d_mask, lw), dev(d_col, (size_t)w * lw), (uint64_t)(uintptr_t)d_sum,
                 (uint64_t)(uintptr_t)c->d_false);
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}

namespace {

// Checks an expression node list (operands precede their node, kinds and
// types match, pointers present); isb[k] receives whether node k is boolean.
int check_expr(tfhe_ctx* c, const void* const* d_cols, uint32_t ncols, uint32_t w, const sql_expr* nodes,
               uint32_t nnodes, std::vector<char>& isb) {
    if (!nodes || !nnodes) return ctx_fail(c, TFHE_EINVAL, "empty expression");
    if (w < 1 || w > 64) return ctx_fail(c, TFHE_ESHAPE, "value width must be 1..64 bits");
    if (ncols && !d_cols) return ctx_fail(c, TFHE_EINVAL, "null column array");
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
            return ctx_fail(c, TFHE_EINVAL, msg);
        }
        isb[k] = e.kind == SQL_EXPR_CMP || e.kind == SQL_EXPR_AND || e.kind == SQL_EXPR_OR ||
                 e.kind == SQL_EXPR_XOR || e.kind == SQL_EXPR_NOT;
    }
    return TFHE_OK;
}

// Adds the circuits of a checked node list to b's netlist and returns the
// root's wires (not yet materialized).
ExprVal compile_expr(Builder& b, const void* const* d_cols, uint32_t rows, uint32_t w, const sql_expr* nodes,
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

}  // namespace

// Homomorphic expression tree (Section 4.3 B) over a table's columns.
extern "C" int sql_expr_eval(tfhe_ctx* c, const void* const* d_cols, uint32_t ncols, uint32_t rows, uint32_t w,
                             const sql_expr* nodes, uint32_t nnodes, void* d_out, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!d_out) return ctx_fail(c, TFHE_EINVAL, "null output pointer");
    std::vector<char> isb;
    int rc = check_expr(c, d_cols, ncols, w, nodes, nnodes, isb);
    if (rc) return rc;
    if (!rows) return TFHE_OK;
    Builder b(c);
    const ExprVal root = compile_expr(b, d_cols, rows, w, nodes, nnodes, isb);
    // the root's bits are written to d_out by linear steps (exact copies,
    // negations or trivial encryptions)
    ExprCompiler ec{b, rows};
    const size_t lw = b.lw, wb = b.wb;
    for (size_t j = 0; j < root.bits.size(); j++) {
        const Ref o = root.is_bool ? dev(d_out, lw)
                                   : Ref{(uint64_t)(uintptr_t)d_out + (uint64_t)j * lw * wb, (int64_t)((size_t)w * lw)};
        ec.lin({{&root.bits[j], 1}}, 0, &o);
    }
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}

// ------------------------------------------------- continuous-batching server

#include <deque>
#include <unordered_set>

namespace {

struct ServerQuery {
    uint64_t id = 0;
    Netlist net;
    size_t tmp_bytes = 0;
    void* tmp = nullptr;
    size_t level = 0;   // next level to run
    size_t seg = 0;     // next segment of that level
    uint32_t row = 0;   // rows of that segment already run
    bool copies_done = false;
};

constexpr uint32_t kMaxActive = 256;
constexpr size_t kSegCap = 1 << 15;

}  // namespace

struct sql_server {
    tfhe_ctx* c = nullptr;
    size_t budget = 0, fixed = 0, in_use = 0;
    uint32_t max_batch = 0;
    uint64_t next_id = 1;
    std::deque<ServerQuery*> queue;
    std::vector<ServerQuery*> active;
    std::unordered_set<uint64_t> done, known;
    void* stage = nullptr;
    uint8_t *lwe = nullptr, *big = nullptr, *brws = nullptr;
    size_t brws_bytes = 0;
    uint64_t* ptrs = nullptr;
    int32_t* tvi = nullptr;
    Segment* dsegs = nullptr;
    uint32_t* dstart = nullptr;
    Segment* hsegs = nullptr;
    uint32_t* hstart = nullptr;
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" int sql_server_create(tfhe_ctx* c, size_t budget, uint32_t max_batch, sql_server** out) {
    if (!c || !out || max_batch < 16) return TFHE_EINVAL;
    *out = nullptr;
    sql_server* sv = new sql_server();
    sv->c = c;
    sv->budget = budget;
    sv->max_batch = max_batch;
    const size_t wb = word_bytes(c), lw = c->p.n + 1, bw = (size_t)c->p.k * c->p.N + 1;
    const size_t NL = c->q == 32 ? 4 : 8;
    const size_t keys = (tfhe_bsk_words(&c->p) + tfhe_ksk_words(&c->p)) * wb +
                        (size_t)c->p.n * 2 * c->p.l * 2 * NL * 2 * c->p.N;
    const size_t lwe_b = al256((size_t)max_batch * lw * wb), big_b = al256((size_t)max_batch * bw * wb);
    const size_t ptr_b = al256((size_t)max_batch * 8), tvi_b = al256((size_t)max_batch * 4);
    const size_t br_b = al256(blind_rotate_ws_bytes_upto(c, max_batch));
    const size_t seg_b = al256(kSegCap * sizeof(Segment)), st_b = al256(kSegCap * 4);
    const size_t stage_b = lwe_b + big_b + ptr_b + tvi_b + br_b + seg_b + st_b;
    sv->fixed = keys + stage_b;
    if (sv->fixed > budget) {
        delete sv;
        return ctx_fail(c, TFHE_ENOMEM, "HBM budget smaller than keys + server staging");
    }
    int rc = hip_check(c, hipMalloc(&sv->stage, stage_b), "server staging");
    if (!rc) rc = hip_check(c, hipHostMalloc((void**)&sv->hsegs, kSegCap * sizeof(Segment)), "server pinned segments");
    if (!rc) rc = hip_check(c, hipHostMalloc((void**)&sv->hstart, kSegCap * 4), "server pinned starts");
    if (rc) {
        sql_server_destroy(sv);
        return rc;
    }
    uint8_t* p = (uint8_t*)sv->stage;
    sv->lwe = p; p += lwe_b;
    sv->big = p; p += big_b;
    sv->ptrs = (uint64_t*)p; p += ptr_b;
    sv->tvi = (int32_t*)p; p += tvi_b;
    sv->brws = p; p += br_b;
    sv->brws_bytes = br_b;
    sv->dsegs = (Segment*)p; p += seg_b;
    sv->dstart = (uint32_t*)p;
    sv->in_use = sv->fixed;
    *out = sv;
    return TFHE_OK;
}

extern "C" void sql_server_destroy(sql_server* sv) {
    if (!sv) return;
    hipDeviceSynchronize();
    for (auto* q : sv->active) { if (q->tmp) hipFree(q->tmp); delete q; }
    for (auto* q : sv->queue) delete q;
    if (sv->stage) hipFree(sv->stage);
    if (sv->hsegs) hipHostFree(sv->hsegs);
    if (sv->hstart) hipHostFree(sv->hstart);
    delete sv;
}

extern "C" size_t sql_server_bytes_in_use(const sql_server* sv) { return sv ? sv->in_use : 0; }

static int server_enqueue(sql_server* sv, ServerQuery* sq, size_t wb, uint64_t* id) {
    sq->tmp_bytes = al256(sq->net.tmp_words * wb);
    if (sv->fixed + sq->tmp_bytes > sv->budget) {
        delete sq;
        return ctx_fail(sv->c, TFHE_ENOMEM, "query working set exceeds the HBM budget");
    }
    sq->id = sv->next_id++;
    sv->known.insert(sq->id);
    sv->queue.push_back(sq);
    *id = sq->id;
    return TFHE_OK;
}

extern "C" int sql_server_submit(sql_server* sv, const sql_sum_query* q, uint64_t* id) {
    if (!sv || !q || !id) return TFHE_EINVAL;
    tfhe_ctx* c = sv->c;
    int rc = check_scan(c, q->d_col, q->w, q->op, q->d_lit_a, q->d_lit_b, q->d_sum);
    if (rc) return rc;
    if (!q->d_sum_col || !q->rows || q->w > 32) return ctx_fail(c, TFHE_EINVAL, "bad SUM query");
    auto* sq = new ServerQuery();
    Builder b(c);
    const size_t lw = b.lw;
    Ref col = dev(q->d_col, (size_t)q->w * lw), la = dev(q->d_lit_a, 0), lb = dev(q->d_lit_b, 0);
    Ref mask = b.tmp(q->rows);
    const size_t lev = b.predicate(0, q->rows, q->w, q->op, col, la, q->d_lit_b ? &lb : nullptr, mask);
    b.masked_sum(lev, q->rows, q->w, mask, dev(q->d_sum_col, (size_t)q->w * lw), (uint64_t)(uintptr_t)q->d_sum,
                 (uint64_t)(uintptr_t)c->d_false);
    sq->net = std::move(b.net);
    return server_enqueue(sv, sq, b.wb, id);
}

// SELECT SUM(sum_col) WHERE <expression tree>: the tree's boolean root is
// the mask of the same masked SUM circuit.
extern "C" int sql_server_submit_expr(sql_server* sv, const void* const* d_cols, uint32_t ncols, uint32_t rows,
                                      uint32_t w, const sql_expr* nodes, uint32_t nnodes, const void* d_sum_col,
                                      void* d_sum, uint64_t* id) {
    if (!sv || !id) return TFHE_EINVAL;
    tfhe_ctx* c = sv->c;
    if (!d_sum_col || !d_sum || !rows || w > 32) return ctx_fail(c, TFHE_EINVAL, "bad SUM query");
    std::vector<char> isb;
    int rc = check_expr(c, d_cols, ncols, w, nodes, nnodes, isb);
    if (rc) return rc;
    if (!isb[nnodes - 1]) return ctx_fail(c, TFHE_EINVAL, "the WHERE expression must be a condition");
    Builder b(c);
    const ExprVal root = compile_expr(b, d_cols, rows, w, nodes, nnodes, isb);
    ExprCompiler ec{b, rows};
    const Ref mask = b.tmp(rows);
    const Wire m = ec.lin({{&root.bits[0], 1}}, 0, &mask);
    b.masked_sum(m.rg, rows, w, mask, dev(d_sum_col, (size_t)w * b.lw), (uint64_t)(uintptr_t)d_sum,
                 (uint64_t)(uintptr_t)c->d_false);
    auto* sq = new ServerQuery();
    sq->net = std::move(b.net);
    return server_enqueue(sv, sq, b.wb, id);
}

static int server_admit(sql_server* sv) {
    while (!sv->queue.empty() && sv->active.size() < kMaxActive) {
        ServerQuery* q = sv->queue.front();
        if (sv->in_use + q->tmp_bytes > sv->budget) break;  // wait for memory to free
        int rc = hip_check(sv->c, hipMalloc(&q->tmp, q->tmp_bytes ? q->tmp_bytes : 256), "query temporaries");
        if (rc) return rc;
        const uint64_t base = (uint64_t)(uintptr_t)q->tmp;
        auto res = [&](uint64_t a) { return (a & REL) ? base + (a & ~REL) : a; };
        for (auto& L : q->net.levels) {
            for (auto* group : {&L.segs, &L.lins})
                for (auto& sg : *group) {
                    for (int j = 0; j < sg.nin; j++) sg.in[j] = res(sg.in[j]);
                    sg.out = res(sg.out);
                }
            for (auto& cp : L.copies) { cp.src = res(cp.src); cp.dst = res(cp.dst); }
        }
        sv->in_use += q->tmp_bytes;
        sv->active.push_back(q);
        sv->queue.pop_front();
    }
    return TFHE_OK;
}

extern "C" int sql_server_step(sql_server* sv, void* stream, uint32_t* gates, uint32_t* active, uint32_t* queued) {
    if (!sv) return TFHE_EINVAL;
    tfhe_ctx* c = sv->c;
    hipStream_t s = (hipStream_t)stream;
    int rc = server_admit(sv);
    if (rc) return rc;
    const size_t wb = word_bytes(c);
    size_t nseg = 0;
    uint32_t total = 0;
    std::vector<Copy> copies;
    std::vector<Segment> lins;  // run after the copies, before the gates
    for (auto* q : sv->active) {
        if (total >= sv->max_batch || nseg + lins.size() >= kSegCap) break;
        if (q->level >= q->net.levels.size()) continue;
        Level& L = q->net.levels[q->level];
        if (!q->copies_done) {
            if (nseg + lins.size() + L.lins.size() >= kSegCap) break;  // the next tick takes this query's level
            copies.insert(copies.end(), L.copies.begin(), L.copies.end());
            lins.insert(lins.end(), L.lins.begin(), L.lins.end());
            q->copies_done = true;
        }
        while (q->seg < L.segs.size() && total < sv->max_batch && nseg + lins.size() < kSegCap) {
            Segment sg = L.segs[q->seg];
            const uint32_t take = std::min<uint32_t>(sg.rows - q->row, sv->max_batch - total);
            for (int j = 0; j < sg.nin; j++) sg.in[j] += (uint64_t)(q->row * sg.in_stride[j]) * wb;
            sg.out += (uint64_t)(q->row * sg.out_stride) * wb;
            sg.rows = take;
            sv->hsegs[nseg] = sg;
            sv->hstart[nseg] = total;
            nseg++;
            total += take;
            q->row += take;
            if (q->row == L.segs[q->seg].rows) { q->seg++; q->row = 0; }
        }
        if (q->seg == L.segs.size()) {  // level fully issued; the next tick runs the next one
            q->level++;
            q->seg = 0;
            q->copies_done = false;
        }
    }
    for (auto& cp : copies) {
        rc = hip_check(c, hipMemcpyAsync((void*)(uintptr_t)cp.dst, (const void*)(uintptr_t)cp.src, cp.bytes,
                                         hipMemcpyDeviceToDevice, s), "server copy");
        if (rc) return rc;
    }
    if (!lins.empty()) {  // linear steps go after the gate segments in the staging arrays
        uint32_t lt = 0;
        for (size_t k = 0; k < lins.size(); k++) {
            sv->hsegs[nseg + k] = lins[k];
            sv->hstart[nseg + k] = lt;
            lt += lins[k].rows;
        }
        const size_t nl = lins.size();
        if ((rc = hip_check(c, hipMemcpyAsync(sv->dsegs + nseg, sv->hsegs + nseg, nl * sizeof(Segment),
                                              hipMemcpyHostToDevice, s), "server linear steps")) ||
            (rc = hip_check(c, hipMemcpyAsync(sv->dstart + nseg, sv->hstart + nseg, nl * 4, hipMemcpyHostToDevice, s),
                            "server linear starts")) ||
            (rc = launch_lin(c, sv->dsegs + nseg, sv->dstart + nseg, (int)nl, lt, s)))
            return rc;
    }
    if (total) {
        if ((rc = hip_check(c, hipMemcpyAsync(sv->dsegs, sv->hsegs, nseg * sizeof(Segment), hipMemcpyHostToDevice, s),
                            "server segments")) ||
            (rc = hip_check(c, hipMemcpyAsync(sv->dstart, sv->hstart, nseg * 4, hipMemcpyHostToDevice, s),
                            "server starts")) ||
            (rc = launch_combine(c, sv->dsegs, sv->dstart, (int)nseg, total, sv->lwe, sv->ptrs, sv->tvi, s)) ||
            (rc = launch_blind_rotate(c, sv->lwe, nullptr, nullptr, sv->big, total, sv->brws, sv->brws_bytes, s)) ||
            (rc = launch_keyswitch(c, sv->big, nullptr, sv->ptrs, total, s)))
            return rc;
    }
    if ((rc = hip_check(c, hipStreamSynchronize(s), "server tick"))) return rc;
    // retire finished queries
    std::vector<ServerQuery*> keep;
    for (auto* q : sv->active) {
        if (q->level >= q->net.levels.size()) {
            sv->done.insert(q->id);
            hipFree(q->tmp);
            sv->in_use -= q->tmp_bytes;
            delete q;
        } else {
            keep.push_back(q);
        }
    }
    sv->active.swap(keep);
    if (gates) *gates = total;
    if (active) *active = (uint32_t)sv->active.size();
    if (queued) *queued = (uint32_t)sv->queue.size();
    return TFHE_OK;
}

extern "C" int sql_server_done(sql_server* sv, uint64_t id) {
    if (!sv) return TFHE_EINVAL;
    if (!sv->known.count(id)) return TFHE_EINVAL;
    return sv->done.count(id) ? 1 : 0;
}

// ------------------------------------------------------------ radix C ABI

// Test polynomial of a table f over Z_p (p = 32 boxes on the half torus):
// coefficient j encodes f(m(j)), m(j) = floor((j p + N/2) / N); the last
// half-box (m(j) = p) holds -f(0) so phases just below 0 return f(0).
template <typename T>
static void lut_poly(int N, const int* f, int p, T delta, T* out) {
    for (int j = 0; j < N; j++) {
        const int64_t m = ((int64_t)j * p + N / 2) / N;
        out[j] = m >= p ? (T)(0 - delta * (T)f[0]) : (T)(delta * (T)f[m]);
    }
}

static int radix_tables_ready(tfhe_ctx* c) {
    if (c->d_radix_tv) return TFHE_OK;
    const int P = 32, N = (int)c->p.N;
    int tab[8][32];
    for (int x = 0; x < P; x++) {
        tab[0][x] = x < 16 ? 0 : (x == 16 ? 1 : 2);            // cmp
        tab[1][x] = x <= 2 ? 0 : (x == 3 ? 1 : (x <= 6 ? 2 : 0));  // comb
        tab[2][x] = x <= 2 ? 16 : 0;                           // root lt
        tab[3][x] = x == 3 ? 16 : 0;                           // root eq
        tab[4][x] = (x >= 4 && x <= 6) ? 16 : 0;               // root gt
        tab[5][x] = x >= 16 ? x - 16 : 0;                      // select
        tab[6][x] = x % 16;                                    // message
        tab[7][x] = x / 16;                                    // carry
    }
    const size_t wb = word_bytes(c);
    std::vector<uint8_t> host(8 * (size_t)N * wb);
    for (int t = 0; t < 8; t++) {
        if (c->q == 32) lut_poly<uint32_t>(N, tab[t], P, (uint32_t)1u << 26, (uint32_t*)host.data() + (size_t)t * N);
        else lut_poly<uint64_t>(N, tab[t], P, (uint64_t)1ull << 58, (uint64_t*)host.data() + (size_t)t * N);
    }
    int rc = hip_check(c, hipMalloc(&c->d_radix_tv, host.size()), "radix tables");
    if (rc) return rc;
    return hip_check(c, hipMemcpy(c->d_radix_tv, host.data(), host.size(), hipMemcpyHostToDevice), "radix tables");
}

extern "C" int sql_radix_mask_scan(tfhe_ctx* c, const void* d_col, uint32_t rows, uint32_t nb, int op,
                                   const void* d_lit, void* d_mask, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!rows) return TFHE_OK;
    if (!d_col || !d_lit || !d_mask) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    if (nb < 2 || nb > 32) return ctx_fail(c, TFHE_ESHAPE, "radix integers need 2..32 blocks");
    if (op != SQL_OP_LT && op != SQL_OP_EQ && op != SQL_OP_GT) return ctx_fail(c, TFHE_EINVAL, "radix op must be EQ, LT or GT");
    int rc = radix_tables_ready(c);
    if (rc) return rc;
    Builder b(c);
    const size_t lw = b.lw;
    b.net.lut_table = c->d_radix_tv;
    b.radix_compare(0, rows, nb, op, dev(d_col, (size_t)nb * lw), dev(d_lit, 0), dev(d_mask, lw));
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}

extern "C" int sql_radix_masked_select(tfhe_ctx* c, const void* d_mask, const void* d_col, uint32_t rows, uint32_t nb,
                                       void* d_out, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!rows) return TFHE_OK;
    if (!d_mask || !d_col || !d_out) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    if (nb < 1 || nb > 32) return ctx_fail(c, TFHE_ESHAPE, "radix integers need 1..32 blocks");
    int rc = radix_tables_ready(c);
    if (rc) return rc;
    Builder b(c);
    const size_t lw = b.lw;
    b.net.lut_table = c->d_radix_tv;
    b.radix_select(0, rows, nb, dev(d_mask, lw), dev(d_col, (size_t)nb * lw), dev(d_out, (size_t)nb * lw));
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}

extern "C" int sql_radix_sum(tfhe_ctx* c, const void* d_vals, uint32_t rows, uint32_t nb, void* d_sum, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!d_vals || !d_sum) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    if (!rows) return ctx_fail(c, TFHE_ESHAPE, "SUM needs at least one row");
    if (nb < 1 || nb > 32) return ctx_fail(c, TFHE_ESHAPE, "radix integers need 1..32 blocks");
    int rc = radix_tables_ready(c);
    if (rc) return rc;
    Builder b(c);
    const size_t lw = b.lw;
    b.net.lut_table = c->d_radix_tv;
    b.radix_sum(0, rows, nb, dev(d_vals, (size_t)nb * lw), (uint64_t)(uintptr_t)d_sum);
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}
