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

namespace {

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
        Schedule sc = plan_schedule(net, max_batch, wb);
        if (sc.pieces.empty()) return TFHE_OK;
        const uint32_t chunk = sc.chunk;
        std::vector<Segment>& flat = sc.flat;
        std::vector<uint32_t>& starts = sc.starts;
        std::vector<Piece>& pieces = sc.pieces;
        std::vector<Copy>& copies = sc.copies;
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        const size_t tmp_b = al(net.tmp_words * wb);
        const size_t lwe_b = al((size_t)chunk * lw * wb);
        const size_t big_b = al((size_t)chunk * bw * wb);
        const size_t ptr_b = al((size_t)chunk * 8);
        const size_t tvi_b = al((size_t)chunk * 4);
        // pieces of a level can be smaller than the chunk (and then take the
        // multi-workgroup blind rotation), so size for any batch up to it;
        // the key switch's digits reuse the region once the blind rotation
        // that precedes it in the stream has finished with it
        const size_t br_b = std::max(al(blind_rotate_ws_bytes_upto(c, chunk)), al(ks_digits_bytes(c, chunk)));
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
                if ((e = launch_keyswitch(c, big, nullptr, ptrs, pc.total, brws, br_b, rs))) break;
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

}  // namespace

// ------------------------------------------------------------ C ABI

extern "C" int tfhe_gate_batch(tfhe_ctx* c, int op, const void* d_x, const void* d_y, const void* d_z, void* d_out,
                               uint32_t B, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (op < G_AND || op > G_MAJ) return ctx_fail(c, TFHE_EINVAL, "unknown gate");
    if (!B) return TFHE_OK;
    if (!d_x || !d_y || !d_out || (op == G_MAJ && !d_z)) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    Builder b(c->q, c->p.n);
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
    Builder b(c->q, c->p.n);
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
    Builder b(c->q, c->p.n);
    const size_t lw = b.lw;
    b.select(0, rows, w, dev(d_mask, lw), dev(d_col, (size_t)w * lw), dev(d_out, (size_t)w * lw));
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}

extern "C" int sql_scan_batch(tfhe_ctx* c, const sql_table_query* q, uint32_t count, int use_graph, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!count) return TFHE_OK;
    if (!q) return ctx_fail(c, TFHE_EINVAL, "null query array");
    Builder b(c->q, c->p.n);
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
    Builder b(c->q, c->p.n);
    const size_t lw = b.lw;
    b.masked_sum(0, rows, w, dev(d_mask, lw), dev(d_col, (size_t)w * lw), (uint64_t)(uintptr_t)d_sum,
                 (uint64_t)(uintptr_t)c->d_false);
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}

// Homomorphic expression tree (Section 4.3 B) over a table's columns.
extern "C" int sql_expr_eval(tfhe_ctx* c, const void* const* d_cols, uint32_t ncols, uint32_t rows, uint32_t w,
                             const sql_expr* nodes, uint32_t nnodes, void* d_out, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (!d_out) return ctx_fail(c, TFHE_EINVAL, "null output pointer");
    std::vector<char> isb;
    std::string why;
    int rc = check_expr(d_cols, ncols, w, nodes, nnodes, isb, &why);
    if (rc) return ctx_fail(c, rc, why);
    if (!rows) return TFHE_OK;
    Builder b(c->q, c->p.n);
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

// The server's device side: two staging sets (each sized for max_batch
// gates and ServerBook's seg_cap segments, with pinned host copies of its
// segment tables) used by alternate ticks, so that a tick is enqueued while
// the previous one runs; the bookkeeping (admission, ticks, retirement) is
// ServerBook's.
struct ServerStage {
    uint8_t *lwe = nullptr, *big = nullptr, *brws = nullptr;
    uint64_t* ptrs = nullptr;
    int32_t* tvi = nullptr;
    Segment* dsegs = nullptr;
    uint32_t* dstart = nullptr;
    Segment* hsegs = nullptr;
    uint32_t* hstart = nullptr;
    hipEvent_t ev = nullptr;   // recorded after the tick that last used this set
    bool busy = false;
    uint64_t tick = 0;         // that tick's number
};

struct sql_server {
    tfhe_ctx* c = nullptr;
    ServerBook book;
    void* stage = nullptr;
    size_t brws_bytes = 0;
    ServerStage st[2];
    uint64_t completed = 0;            // every tick numbered below has finished
    hipStream_t last_stream = nullptr; // stream of the last tick enqueued
    int last_set = -1;
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" int sql_server_create(tfhe_ctx* c, size_t budget, uint32_t max_batch, sql_server** out) {
    if (!c || !out || max_batch < 16) return TFHE_EINVAL;
    *out = nullptr;
    sql_server* sv = new sql_server();
    sv->c = c;
    sv->book.budget = budget;
    sv->book.max_batch = max_batch;
    const size_t cap = sv->book.seg_cap;
    const size_t wb = word_bytes(c), lw = c->p.n + 1, bw = (size_t)c->p.k * c->p.N + 1;
    const size_t NL = c->q == 32 ? 4 : 8;
    const size_t keys = (tfhe_bsk_words(&c->p) + tfhe_ksk_words(&c->p)) * wb +
                        (size_t)c->p.n * 2 * c->p.l * 2 * NL * 2 * c->p.N + c->win_bytes + c->ksk8_bytes;
    const size_t lwe_b = al256((size_t)max_batch * lw * wb), big_b = al256((size_t)max_batch * bw * wb);
    const size_t ptr_b = al256((size_t)max_batch * 8), tvi_b = al256((size_t)max_batch * 4);
    // blind-rotation workspace, reused by the key switch's digits
    const size_t br_b = std::max(al256(blind_rotate_ws_bytes_upto(c, max_batch)), al256(ks_digits_bytes(c, max_batch)));
    const size_t seg_b = al256(cap * sizeof(Segment)), st_b = al256(cap * 4);
    const size_t set_b = lwe_b + big_b + ptr_b + tvi_b + br_b + seg_b + st_b;
    sv->book.fixed = keys + 2 * set_b;
    if (sv->book.fixed > budget) {
        delete sv;
        return ctx_fail(c, TFHE_ENOMEM, "HBM budget smaller than keys + server staging");
    }
    int rc = hip_check(c, hipMalloc(&sv->stage, 2 * set_b), "server staging");
    for (int k = 0; k < 2 && !rc; k++) {
        ServerStage& S = sv->st[k];
        rc = hip_check(c, hipHostMalloc((void**)&S.hsegs, cap * sizeof(Segment)), "server pinned segments");
        if (!rc) rc = hip_check(c, hipHostMalloc((void**)&S.hstart, cap * 4), "server pinned starts");
        if (!rc) rc = hip_check(c, hipEventCreateWithFlags(&S.ev, hipEventDisableTiming), "server tick event");
        if (rc) break;
        uint8_t* p = (uint8_t*)sv->stage + k * set_b;
        S.lwe = p; p += lwe_b;
        S.big = p; p += big_b;
        S.ptrs = (uint64_t*)p; p += ptr_b;
        S.tvi = (int32_t*)p; p += tvi_b;
        S.brws = p; p += br_b;
        S.dsegs = (Segment*)p; p += seg_b;
        S.dstart = (uint32_t*)p;
    }
    if (rc) {
        sql_server_destroy(sv);
        return rc;
    }
    sv->brws_bytes = br_b;
    sv->book.in_use = sv->book.fixed;
    *out = sv;
    return TFHE_OK;
}

extern "C" void sql_server_destroy(sql_server* sv) {
    if (!sv) return;
    hipDeviceSynchronize();
    sv->book.clear([](uint64_t base) { if (base) hipFreeAsync((void*)(uintptr_t)base, nullptr); });
    hipDeviceSynchronize();
    if (sv->stage) hipFree(sv->stage);
    for (auto& S : sv->st) {
        if (S.hsegs) hipHostFree(S.hsegs);
        if (S.hstart) hipHostFree(S.hstart);
        if (S.ev) hipEventDestroy(S.ev);
    }
    delete sv;
}

extern "C" size_t sql_server_bytes_in_use(const sql_server* sv) { return sv ? sv->book.in_use : 0; }

static int server_enqueue(sql_server* sv, ServerQuery* sq, size_t wb, uint64_t* id) {
    std::string why;
    const int rc = sv->book.enqueue(sq, wb, id, &why);
    return rc ? ctx_fail(sv->c, rc, why) : TFHE_OK;
}

extern "C" int sql_server_submit(sql_server* sv, const sql_sum_query* q, uint64_t* id) {
    if (!sv || !q || !id) return TFHE_EINVAL;
    tfhe_ctx* c = sv->c;
    int rc = check_scan(c, q->d_col, q->w, q->op, q->d_lit_a, q->d_lit_b, q->d_sum);
    if (rc) return rc;
    if (!q->d_sum_col || !q->rows || q->w > 32) return ctx_fail(c, TFHE_EINVAL, "bad SUM query");
    auto* sq = new ServerQuery();
    Builder b(c->q, c->p.n);
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
    std::string why;
    int rc = check_expr(d_cols, ncols, w, nodes, nnodes, isb, &why);
    if (rc) return ctx_fail(c, rc, why);
    if (!isb[nnodes - 1]) return ctx_fail(c, TFHE_EINVAL, "the WHERE expression must be a condition");
    Builder b(c->q, c->p.n);
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

// Marks the tick of set k finished once its event has completed (waiting
// for it when `wait`).
static int server_poll(sql_server* sv, int k, bool wait) {
    ServerStage& S = sv->st[k];
    if (!S.busy) return TFHE_OK;
    const hipError_t e = wait ? hipEventSynchronize(S.ev) : hipEventQuery(S.ev);
    if (e == hipErrorNotReady) return TFHE_OK;
    if (e != hipSuccess) return hip_check(sv->c, e, "server tick");
    S.busy = false;
    sv->completed = std::max(sv->completed, S.tick + 1);
    return TFHE_OK;
}

extern "C" int sql_server_step(sql_server* sv, void* stream, uint32_t* gates, uint32_t* active, uint32_t* queued) {
    if (!sv) return TFHE_EINVAL;
    tfhe_ctx* c = sv->c;
    hipStream_t s = (hipStream_t)stream;
    ServerBook& bk = sv->book;
    // this tick's staging set was last used two ticks ago: wait for that one
    const int k = (int)(bk.ticks & 1);
    int rc = server_poll(sv, k, true);
    if (!rc) rc = server_poll(sv, 1 - k, false);
    if (rc) return rc;
    if (!sv->st[0].busy && !sv->st[1].busy) sv->completed = bk.ticks;  // nothing in flight
    // temporaries go back to the stream-ordered pool after the ticks that used them
    bk.retire([&](uint64_t base) { hipFreeAsync((void*)(uintptr_t)base, s); }, sv->completed);
    std::string why;
    rc = bk.admit(
        [&](size_t bytes) -> uint64_t {
            void* p = nullptr;
            return hipMallocAsync(&p, bytes, s) == hipSuccess ? (uint64_t)(uintptr_t)p : 0;
        },
        &why);
    if (rc) return ctx_fail(c, rc, why);
    const size_t wb = word_bytes(c);
    Tick t;
    const uint64_t tick_no = bk.ticks;
    bk.next_tick(t, wb);
    const size_t nseg = t.segs.size();
    const bool work = t.total || !t.lins.empty() || !t.copies.empty();
    if (work) {
        ServerStage& S = sv->st[k];
        // a tick reads the outputs of the previous one: order the streams
        if (sv->last_set >= 0 && sv->last_stream != s && sv->st[sv->last_set].busy &&
            (rc = hip_check(c, hipStreamWaitEvent(s, sv->st[sv->last_set].ev, 0), "server tick order")))
            return rc;
        for (auto& cp : t.copies) {
            rc = hip_check(c, hipMemcpyAsync((void*)(uintptr_t)cp.dst, (const void*)(uintptr_t)cp.src, cp.bytes,
                                             hipMemcpyDeviceToDevice, s), "server copy");
            if (rc) return rc;
        }
        // gate segments first, then the linear steps, in the staging arrays
        for (size_t i = 0; i < nseg; i++) {
            S.hsegs[i] = t.segs[i];
            S.hstart[i] = t.starts[i];
        }
        for (size_t i = 0; i < t.lins.size(); i++) {
            S.hsegs[nseg + i] = t.lins[i];
            S.hstart[nseg + i] = t.lin_starts[i];
        }
        const size_t nall = nseg + t.lins.size();
        if ((rc = hip_check(c, hipMemcpyAsync(S.dsegs, S.hsegs, nall * sizeof(Segment), hipMemcpyHostToDevice, s),
                            "server segments")) ||
            (rc = hip_check(c, hipMemcpyAsync(S.dstart, S.hstart, nall * 4, hipMemcpyHostToDevice, s),
                            "server starts")))
            return rc;
        if (!t.lins.empty() &&
            (rc = launch_lin(c, S.dsegs + nseg, S.dstart + nseg, (int)t.lins.size(), t.lin_total, s)))
            return rc;
        if (t.total) {
            if ((rc = launch_combine(c, S.dsegs, S.dstart, (int)nseg, t.total, S.lwe, S.ptrs, S.tvi, s)) ||
                (rc = launch_blind_rotate(c, S.lwe, nullptr, nullptr, S.big, t.total, S.brws, sv->brws_bytes, s)) ||
                (rc = launch_keyswitch(c, S.big, nullptr, S.ptrs, t.total, S.brws, sv->brws_bytes, s)))
                return rc;
        }
        if ((rc = hip_check(c, hipEventRecord(S.ev, s), "server tick event"))) return rc;
        S.busy = true;
        S.tick = tick_no;
        sv->last_stream = s;
        sv->last_set = k;
    } else {
        // nothing to issue: let the ticks in flight finish so that finished
        // queries retire and the caller's loop makes progress
        if ((rc = server_poll(sv, 0, true)) || (rc = server_poll(sv, 1, true))) return rc;
        sv->completed = bk.ticks;
        bk.retire([&](uint64_t base) { hipFreeAsync((void*)(uintptr_t)base, s); }, sv->completed);
    }
    if (gates) *gates = t.total;
    if (active) *active = (uint32_t)bk.active.size();
    if (queued) *queued = (uint32_t)bk.queue.size();
    return TFHE_OK;
}

extern "C" int sql_server_done(sql_server* sv, uint64_t id) {
    if (!sv) return TFHE_EINVAL;
    if (!sv->book.known.count(id)) return TFHE_EINVAL;
    return sv->book.done.count(id) ? 1 : 0;
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
    Builder b(c->q, c->p.n);
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
    Builder b(c->q, c->p.n);
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
    Builder b(c->q, c->p.n);
    const size_t lw = b.lw;
    b.net.lut_table = c->d_radix_tv;
    b.radix_sum(0, rows, nb, dev(d_vals, (size_t)nb * lw), (uint64_t)(uintptr_t)d_sum);
    Exec ex(c, (hipStream_t)stream);
    return ex.run(b.net, false);
}
