// Host-only checks of the circuit netlists, the launch schedule and the
// server's bookkeeping (built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py).
//
// A plaintext model of the device runs the schedules: every ciphertext is
// named by its byte address and holds its phase in units of the encoding --
// eighths of the torus for gate bits (a bit b is 2b - 1), Delta = 2^q/64 for
// radix blocks.  A bootstrapped gate maps the linear combination (mod 8
// eighths) to +1 when it lies in (0, 1/2) and -1 when in (-1/2, 0); a
// look-up bootstrap maps a block value x in [0, 32) to its table entry.
// Results are compared with integer arithmetic on the same plaintexts.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <random>
#include <string>
#include <unordered_map>
#include <vector>

#include "../paper_2510_15413_amd/csrc/netlist.h"

static int g_checks = 0;
#define CHECK(cond, ...)                                              \
    do {                                                              \
        g_checks++;                                                   \
        if (!(cond)) {                                                \
            fprintf(stderr, "%s:%d: check failed: %s: ", __FILE__, __LINE__, #cond); \
            fprintf(stderr, __VA_ARGS__);                             \
            fprintf(stderr, "\n");                                    \
            exit(1);                                                  \
        }                                                             \
    } while (0)

// Radix tables over Z_32 of the 64-bit circuits, in Builder's L_* order.
static int radix_table(int t, int x) {
    switch (t) {
        case 0: return x < 16 ? 0 : (x == 16 ? 1 : 2);               // compare
        case 1: return x <= 2 ? 0 : (x == 3 ? 1 : (x <= 6 ? 2 : 0));  // combine
        case 2: return x <= 2 ? 16 : 0;                               // root lt
        case 3: return x == 3 ? 16 : 0;                               // root eq
        case 4: return (x >= 4 && x <= 6) ? 16 : 0;                   // root gt
        case 5: return x >= 16 ? x - 16 : 0;                          // select
        case 6: return x % 16;                                        // message
        case 7: return x / 16;                                        // carry
    }
    return -1;
}

struct Machine {
    int q;
    size_t lw, wb;
    std::unordered_map<uint64_t, int64_t> mem;
    uint64_t next = 1ull << 40;  // fake device addresses

    Machine(int q_, uint32_t n) : q(q_), lw((size_t)n + 1), wb(q_ == 32 ? 4 : 8) {}
    uint64_t alloc(size_t cts) {  // cts ciphertexts, 256-byte aligned
        const uint64_t a = next;
        next += ((cts * lw * wb + 255) / 256 + 1) * 256;
        return a;
    }
    int64_t get(uint64_t a) const {
        auto it = mem.find(a);
        CHECK(it != mem.end(), "read of an unwritten ciphertext at %llx", (unsigned long long)a);
        return it->second;
    }
    int64_t signed_word(uint64_t w) const {
        if (q == 32) return (int64_t)(int32_t)(uint32_t)w;
        return (int64_t)w;
    }
    uint64_t unit(bool radix) const { return radix ? (1ull << (q - 6)) : (1ull << (q - 3)); }
    int64_t cst_units(const Segment& s, bool radix) const {
        const int64_t c = signed_word(s.cst);
        const int64_t u = (int64_t)unit(radix);
        CHECK(c % u == 0, "constant %lld not a multiple of the unit", (long long)c);
        return c / u;
    }
    uint64_t at(uint64_t base, int64_t stride, uint32_t r) const {
        return base + (uint64_t)((int64_t)r * stride * (int64_t)wb);
    }
    static int64_t mod(int64_t x, int64_t m) { return ((x % m) + m) % m; }
    // value of one gate or linear step (no write)
    int64_t eval(const Segment& s, uint32_t r, bool bootstrap) const {
        const bool radix = s.lut >= 0;
        int64_t x = cst_units(s, radix);
        for (int j = 0; j < s.nin; j++) x += (int64_t)s.w[j] * get(at(s.in[j], s.in_stride[j], r));
        if (!bootstrap) {
            const int64_t m = mod(x, 8);
            return m >= 4 ? m - 8 : m;
        }
        if (radix) {
            const int64_t v = mod(x, 64);
            CHECK(v < 32, "radix bootstrap input %lld outside [0, 32)", (long long)v);
            return radix_table(s.lut, (int)v);
        }
        const int64_t m = mod(x, 8);
        CHECK(m != 0 && m != 4, "gate input on the decision boundary (%lld eighths)", (long long)m);
        return m < 4 ? 1 : -1;
    }
    void copy(const Copy& cp) {
        const size_t cts = cp.bytes / (lw * wb);
        CHECK(cts * lw * wb == cp.bytes, "copy of a partial ciphertext");
        for (size_t k = 0; k < cts; k++) mem[cp.dst + k * lw * wb] = get(cp.src + k * lw * wb);
    }
    // gates of a launch: every input is read before any output is written
    void gates(const Segment* segs, size_t n) {
        std::vector<std::pair<uint64_t, int64_t>> outs;
        for (size_t i = 0; i < n; i++)
            for (uint32_t r = 0; r < segs[i].rows; r++)
                outs.push_back({at(segs[i].out, segs[i].out_stride, r), eval(segs[i], r, true)});
        for (auto& o : outs) mem[o.first] = o.second;
    }
    void lins(const Segment* segs, size_t n) {
        for (size_t i = 0; i < n; i++)
            for (uint32_t r = 0; r < segs[i].rows; r++)
                mem[at(segs[i].out, segs[i].out_stride, r)] = eval(segs[i], r, false);
    }
};

// Runs a netlist through plan_schedule with temporaries at a fresh base.
static void run_net(Machine& m, Netlist net, uint32_t max_batch) {
    size_t gates_in = 0;
    for (auto& L : net.levels)
        for (auto& s : L.segs) gates_in += s.rows;
    Schedule sc = plan_schedule(net, max_batch, m.wb);
    const uint64_t tmp = m.alloc(net.tmp_words / m.lw + 1);
    auto res = [&](uint64_t a) { return (a & REL) ? tmp + (a & ~REL) : a; };
    for (auto& s : sc.flat) {
        for (int j = 0; j < s.nin; j++) s.in[j] = res(s.in[j]);
        s.out = res(s.out);
    }
    for (auto& cp : sc.copies) { cp.src = res(cp.src); cp.dst = res(cp.dst); }
    CHECK(sc.flat.size() == sc.starts.size(), "flat/starts sizes");
    size_t gates_out = 0;
    for (const Piece& pc : sc.pieces) {
        CHECK(pc.total <= sc.chunk, "launch of %u gates above the chunk %u", pc.total, sc.chunk);
        CHECK(pc.seg_off + pc.nseg <= sc.flat.size() && pc.lin_off + pc.nlin <= sc.flat.size(), "piece range");
        CHECK(pc.copy_off + pc.ncopy <= sc.copies.size(), "copy range");
        uint32_t at = 0;
        for (int k = 0; k < pc.nseg; k++) {
            CHECK(sc.starts[pc.seg_off + k] == at, "start of segment %d is %u, not %u", k, sc.starts[pc.seg_off + k], at);
            CHECK(sc.flat[pc.seg_off + k].rows > 0, "empty segment in a launch");
            at += sc.flat[pc.seg_off + k].rows;
        }
        CHECK(at == pc.total, "segments of a launch sum to %u, not %u", at, pc.total);
        uint32_t lt = 0;
        for (int k = 0; k < pc.nlin; k++) {
            CHECK(sc.starts[pc.lin_off + k] == lt, "linear start");
            lt += sc.flat[pc.lin_off + k].rows;
        }
        CHECK(lt == pc.lin_total, "linear rows");
        gates_out += pc.total;
        for (int k = 0; k < pc.ncopy; k++) m.copy(sc.copies[pc.copy_off + k]);
        m.lins(sc.flat.data() + pc.lin_off, pc.nlin);
        m.gates(sc.flat.data() + pc.seg_off, pc.nseg);
    }
    CHECK(gates_out == gates_in, "schedule runs %zu gates, netlist has %zu", gates_out, gates_in);
}

static const uint32_t kBatches[] = {1, 3, 16, 37, 1000, 65536};

// bit-wise encrypted column [rows][w] at a fresh address
static Ref column(Machine& m, const std::vector<uint64_t>& vals, uint32_t w) {
    const uint64_t base = m.alloc(vals.size() * w);
    for (size_t r = 0; r < vals.size(); r++)
        for (uint32_t j = 0; j < w; j++) m.mem[base + (r * w + j) * m.lw * m.wb] = ((vals[r] >> j) & 1) ? 1 : -1;
    return Ref{base, (int64_t)(w * m.lw)};
}

static uint64_t read_bits(const Machine& m, uint64_t base, uint32_t w) {
    uint64_t v = 0;
    for (uint32_t j = 0; j < w; j++) {
        const int64_t b = m.get(base + j * m.lw * m.wb);
        CHECK(b == 1 || b == -1, "not a bit: %lld", (long long)b);
        if (b == 1) v |= 1ull << j;
    }
    return v;
}

static void test_predicates(int q) {
    const uint32_t w = 4;
    for (int op = SQL_OP_EQ; op <= SQL_OP_BETWEEN; op++) {
        for (uint64_t lo = 0; lo < 16; lo++) {
            for (uint64_t hi = (op == SQL_OP_BETWEEN ? lo : 0); hi < (op == SQL_OP_BETWEEN ? 16u : 1u); hi++) {
                for (uint32_t mb : {1u, 16u, 65536u}) {
                    Machine m(q, 7);
                    std::vector<uint64_t> a(16);
                    for (int i = 0; i < 16; i++) a[i] = (uint64_t)i;
                    Ref col = column(m, a, w), la = column(m, {lo}, w), lb = column(m, {hi}, w);
                    la.stride = lb.stride = 0;
                    const uint64_t mask = m.alloc(16);
                    Builder b(q, 7);
                    b.predicate(0, 16, w, op, col, la, &lb, Ref{mask, (int64_t)m.lw});
                    run_net(m, b.net, mb);
                    for (uint64_t r = 0; r < 16; r++) {
                        const bool want = op == SQL_OP_EQ ? r == lo : op == SQL_OP_LT ? r < lo
                                        : op == SQL_OP_GT ? r > lo : (r >= lo && r <= hi);
                        CHECK(read_bits(m, mask + r * m.lw * m.wb, 1) == (want ? 1u : 0u), "op %d a %llu lit %llu/%llu",
                              op, (unsigned long long)r, (unsigned long long)lo, (unsigned long long)hi);
                    }
                }
            }
        }
    }
}

static void test_select_and_sum(int q, std::mt19937_64& rng) {
    for (uint32_t w : {1u, 3u, 8u}) {
        for (uint32_t rows : {1u, 2u, 3u, 5u, 8u, 13u, 40u}) {
            for (uint32_t mb : kBatches) {
                Machine m(q, 5);
                std::vector<uint64_t> vals(rows), mk(rows);
                uint64_t want = 0;
                for (uint32_t r = 0; r < rows; r++) {
                    vals[r] = rng() & ((1ull << w) - 1);
                    mk[r] = rng() & 1;
                    want += vals[r] * mk[r];
                }
                Ref col = column(m, vals, w), mask = column(m, mk, 1);
                const uint64_t fl = m.alloc(1);
                m.mem[fl] = -1;  // trivial FALSE
                uint32_t width = w;
                for (uint32_t r = rows; r > 1; r = (r + 1) / 2) width++;
                const uint64_t sum = m.alloc(width), sel = m.alloc((size_t)rows * w);
                Builder b(q, 5);
                b.masked_sum(0, rows, w, mask, col, sum, fl);
                run_net(m, b.net, mb);
                CHECK(read_bits(m, sum, width) == want, "sum rows %u w %u batch %u", rows, w, mb);
                Builder b2(q, 5);
                b2.select(0, rows, w, mask, col, Ref{sel, (int64_t)(w * m.lw)});
                run_net(m, b2.net, mb);
                for (uint32_t r = 0; r < rows; r++)
                    CHECK(read_bits(m, sel + (size_t)r * w * m.lw * m.wb, w) == vals[r] * mk[r], "select");
            }
        }
    }
}

// radix-encoded integer [rows][nb] of block values
static Ref blocks(Machine& m, const std::vector<uint64_t>& vals, uint32_t nb) {
    const uint64_t base = m.alloc(vals.size() * nb);
    for (size_t r = 0; r < vals.size(); r++)
        for (uint32_t i = 0; i < nb; i++) m.mem[base + (r * nb + i) * m.lw * m.wb] = (int64_t)((vals[r] >> (4 * i)) & 15);
    return Ref{base, (int64_t)(nb * m.lw)};
}

static uint64_t read_blocks(const Machine& m, uint64_t base, uint32_t nb) {
    uint64_t v = 0;
    for (uint32_t i = 0; i < nb; i++) {
        const int64_t b = m.get(base + i * m.lw * m.wb);
        CHECK(b >= 0 && b < 16, "block out of range: %lld", (long long)b);
        v |= (uint64_t)b << (4 * i);
    }
    return v;
}

static void test_radix(std::mt19937_64& rng) {
    const int q = 64;
    for (uint32_t nb : {2u, 3u, 8u}) {
        const uint64_t M = nb >= 16 ? ~0ull : (1ull << (4 * nb));
        for (int op : {SQL_OP_LT, SQL_OP_EQ, SQL_OP_GT}) {
            for (uint32_t mb : {1u, 7u, 65536u}) {
                const uint32_t rows = 9;
                Machine m(q, 4);
                std::vector<uint64_t> a(rows), v(rows);
                const uint64_t c = rng() % M;
                for (uint32_t r = 0; r < rows; r++) {
                    a[r] = (r % 3 == 0) ? c : rng() % M;
                    v[r] = rng() % M;
                }
                Ref col = blocks(m, a, nb), val = blocks(m, v, nb), lit = blocks(m, {c}, nb);
                lit.stride = 0;
                const uint64_t mask = m.alloc(rows), sel = m.alloc((size_t)rows * nb), sum = m.alloc(nb);
                Builder b(q, 4);
                const size_t lev = b.radix_compare(0, rows, nb, op, col, lit, Ref{mask, (int64_t)m.lw});
                b.radix_select(lev, rows, nb, Ref{mask, (int64_t)m.lw}, val, Ref{sel, (int64_t)(nb * m.lw)});
                run_net(m, b.net, mb);
                Builder b2(q, 4);
                b2.radix_sum(0, rows, nb, Ref{sel, (int64_t)(nb * m.lw)}, sum);
                run_net(m, b2.net, mb);
                uint64_t want = 0;
                for (uint32_t r = 0; r < rows; r++) {
                    const bool f = op == SQL_OP_LT ? a[r] < c : op == SQL_OP_EQ ? a[r] == c : a[r] > c;
                    CHECK(m.get(mask + r * m.lw * m.wb) == (f ? 16 : 0), "radix compare nb %u op %d", nb, op);
                    CHECK(read_blocks(m, sel + (size_t)r * nb * m.lw * m.wb, nb) == (f ? v[r] : 0), "radix select");
                    if (f) want = (want + v[r]) % M;
                }
                CHECK(read_blocks(m, sum, nb) == want, "radix sum nb %u", nb);
            }
        }
    }
}

// Expression trees: the paper's example (age > 18 AND salary < 1000) and a
// tree with MAX, MIN, ITE, NOT and XOR over two columns and a literal.
static uint64_t expr_plain(const std::vector<sql_expr>& nd, const std::vector<uint64_t>& cols, uint64_t lit,
                           uint32_t w, size_t k, std::vector<char>& isb) {
    const sql_expr& e = nd[k];
    const uint64_t M = (1ull << w) - 1;
    auto val = [&](int i) { return expr_plain(nd, cols, lit, w, (size_t)i, isb); };
    switch (e.kind) {
        case SQL_EXPR_COLUMN: return cols[e.col];
        case SQL_EXPR_CONST: return e.value & M;
        case SQL_EXPR_LITERAL: return lit;
        case SQL_EXPR_CMP: {
            const uint64_t a = val(e.a), b = val(e.b);
            switch (e.op) {
                case SQL_CMP_EQ: return a == b;
                case SQL_CMP_NE: return a != b;
                case SQL_CMP_LT: return a < b;
                case SQL_CMP_LE: return a <= b;
                case SQL_CMP_GT: return a > b;
                default: return a >= b;
            }
        }
        case SQL_EXPR_AND: return val(e.a) & val(e.b);
        case SQL_EXPR_OR: return val(e.a) | val(e.b);
        case SQL_EXPR_XOR: return val(e.a) ^ val(e.b);
        case SQL_EXPR_NOT: return !val(e.a);
        case SQL_EXPR_MAX: return std::max(val(e.a), val(e.b));
        case SQL_EXPR_MIN: return std::min(val(e.a), val(e.b));
        case SQL_EXPR_ITE: return val(e.c) ? val(e.a) : val(e.b);
    }
    return 0;
}

static sql_expr node(int kind, int op = 0, int a = -1, int b = -1, int c = -1, int col = -1, uint64_t value = 0,
                     const void* lit = nullptr) {
    sql_expr e;
    e.kind = kind;
    e.op = op;
    e.a = a;
    e.b = b;
    e.c = c;
    e.col = col;
    e.value = value;
    e.d_lit = lit;
    return e;
}

static void test_expressions(std::mt19937_64& rng) {
    const int q = 32;
    const uint32_t w = 6, rows = 23;
    for (int which = 0; which < 2; which++) {
        for (uint32_t mb : {1u, 9u, 65536u}) {
            Machine m(q, 6);
            std::vector<uint64_t> c0(rows), c1(rows);
            for (uint32_t r = 0; r < rows; r++) { c0[r] = rng() % 64; c1[r] = rng() % 64; }
            const uint64_t litv = 33;
            Ref col0 = column(m, c0, w), col1 = column(m, c1, w), lit = column(m, {litv}, w);
            const void* cols[2] = {(const void*)(uintptr_t)col0.addr, (const void*)(uintptr_t)col1.addr};
            const void* lp = (const void*)(uintptr_t)lit.addr;
            std::vector<sql_expr> nd;
            if (which == 0) {  // age > 18 AND salary < 40
                nd = {node(SQL_EXPR_COLUMN, 0, -1, -1, -1, 0), node(SQL_EXPR_CONST, 0, -1, -1, -1, -1, 18),
                      node(SQL_EXPR_CMP, SQL_CMP_GT, 0, 1), node(SQL_EXPR_COLUMN, 0, -1, -1, -1, 1),
                      node(SQL_EXPR_CONST, 0, -1, -1, -1, -1, 40), node(SQL_EXPR_CMP, SQL_CMP_LT, 3, 4),
                      node(SQL_EXPR_AND, 0, 2, 5)};
            } else {  // ITE(NOT(c0 <= lit) XOR (c1 != 7), MAX(c0, c1), MIN(c1, lit))
                nd = {node(SQL_EXPR_COLUMN, 0, -1, -1, -1, 0), node(SQL_EXPR_COLUMN, 0, -1, -1, -1, 1),
                      node(SQL_EXPR_LITERAL, 0, -1, -1, -1, -1, 0, lp), node(SQL_EXPR_CMP, SQL_CMP_LE, 0, 2),
                      node(SQL_EXPR_NOT, 0, 3), node(SQL_EXPR_CONST, 0, -1, -1, -1, -1, 7),
                      node(SQL_EXPR_CMP, SQL_CMP_NE, 1, 5), node(SQL_EXPR_XOR, 0, 4, 6),
                      node(SQL_EXPR_MAX, 0, 0, 1), node(SQL_EXPR_MIN, 0, 1, 2), node(SQL_EXPR_ITE, 0, 8, 9, 7)};
            }
            std::vector<char> isb;
            std::string err;
            CHECK(check_expr(cols, 2, w, nd.data(), (uint32_t)nd.size(), isb, &err) == TFHE_OK, "%s", err.c_str());
            Builder b(q, 6);
            const ExprVal root = compile_expr(b, cols, rows, w, nd.data(), (uint32_t)nd.size(), isb);
            ExprCompiler ec{b, rows};
            const uint32_t ow = root.is_bool ? 1 : w;
            const uint64_t out = m.alloc((size_t)rows * ow);
            for (size_t j = 0; j < root.bits.size(); j++) {
                const Ref o{out + j * m.lw * m.wb, (int64_t)(ow * m.lw)};
                ec.lin({{&root.bits[j], 1}}, 0, &o);
            }
            run_net(m, b.net, mb);
            for (uint32_t r = 0; r < rows; r++) {
                const uint64_t want = expr_plain(nd, {c0[r], c1[r]}, litv, w, nd.size() - 1, isb);
                CHECK(read_bits(m, out + (size_t)r * ow * m.lw * m.wb, ow) == want, "expression %d row %u", which, r);
            }
        }
    }
    // malformed node lists are rejected
    std::vector<char> isb;
    std::string err;
    const void* cols[1] = {(const void*)0x1000};
    std::vector<sql_expr> bad = {node(SQL_EXPR_COLUMN, 0, -1, -1, -1, 0), node(SQL_EXPR_AND, 0, 0, 0)};
    CHECK(check_expr(cols, 1, 4, bad.data(), 2, isb, &err) == TFHE_EINVAL && !err.empty(), "value as AND operand");
    bad = {node(SQL_EXPR_COLUMN, 0, -1, -1, -1, 3)};
    CHECK(check_expr(cols, 1, 4, bad.data(), 1, isb, &err) == TFHE_EINVAL, "column index out of range");
    bad = {node(SQL_EXPR_CMP, SQL_CMP_LT, 0, 0)};
    CHECK(check_expr(cols, 1, 4, bad.data(), 1, isb, &err) == TFHE_EINVAL, "operand not before its node");
    CHECK(check_expr(cols, 1, 65, bad.data(), 1, isb, &err) == TFHE_ESHAPE, "width");
}

// The server: queries of several sizes with a budget that holds two at a
// time and ticks smaller than a level, run until all are done.
static void test_server(std::mt19937_64& rng) {
    const int q = 32;
    const uint32_t n = 5, w = 4;
    for (uint32_t mb : {16u, 50u, 4096u}) {
      for (uint64_t lag : {0ull, 1ull}) {
        Machine m(q, n);
        ServerBook book;
        book.max_batch = mb;
        book.fixed = 1000;
        const uint64_t fl = m.alloc(1);
        m.mem[fl] = -1;
        struct Q { uint64_t id, sum; uint32_t width; uint64_t want; };
        std::vector<Q> qs;
        size_t biggest = 0;
        std::vector<std::pair<ServerQuery*, Q>> pending;
        for (int k = 0; k < 7; k++) {
            const uint32_t rows = 1 + (uint32_t)(rng() % 30);
            std::vector<uint64_t> a(rows), v(rows);
            for (uint32_t r = 0; r < rows; r++) { a[r] = rng() % 16; v[r] = rng() % 16; }
            const uint64_t lit = rng() % 16;
            const int op = (int)(rng() % 4);
            const uint64_t lit2 = std::max<uint64_t>(lit, rng() % 16);
            Ref col = column(m, a, w), vc = column(m, v, w), la = column(m, {lit}, w), lb = column(m, {lit2}, w);
            la.stride = lb.stride = 0;
            uint32_t width = w;
            for (uint32_t r = rows; r > 1; r = (r + 1) / 2) width++;
            const uint64_t sum = m.alloc(width);
            Builder b(q, n);
            const Ref mask = b.tmp(rows);
            const size_t lev = b.predicate(0, rows, w, op, col, la, &lb, mask);
            b.masked_sum(lev, rows, w, mask, vc, sum, fl);
            uint64_t want = 0;
            for (uint32_t r = 0; r < rows; r++) {
                const bool f = op == SQL_OP_EQ ? a[r] == lit : op == SQL_OP_LT ? a[r] < lit
                             : op == SQL_OP_GT ? a[r] > lit : (a[r] >= lit && a[r] <= lit2);
                if (f) want += v[r];
            }
            auto* sq = new ServerQuery();
            sq->net = std::move(b.net);
            biggest = std::max(biggest, ServerBook::al256(sq->net.tmp_words * m.wb));
            pending.push_back({sq, Q{0, sum, width, want}});
        }
        // room for the two largest working sets, not three of them
        book.budget = book.fixed + 2 * biggest + 255;
        book.in_use = book.fixed;
        std::string err;
        for (auto& pq : pending) {
            uint64_t id = 0;
            CHECK(book.enqueue(pq.first, m.wb, &id, &err) == TFHE_OK, "%s", err.c_str());
            pq.second.id = id;
            qs.push_back(pq.second);
        }
        // a query that can never fit is refused
        {
            auto* huge = new ServerQuery();
            huge->net.tmp_words = book.budget;  // bytes > budget
            uint64_t id = 0;
            CHECK(book.enqueue(huge, m.wb, &id, &err) == TFHE_ENOMEM, "oversized query accepted");
        }
        std::map<uint64_t, size_t> allocs;
        size_t ticks = 0;
        while (!book.queue.empty() || !book.active.empty()) {
            CHECK(++ticks < 100000, "server does not finish");
            CHECK(book.admit([&](size_t bytes) { const uint64_t a = m.alloc(bytes / m.wb / m.lw + 1); allocs[a] = bytes; return a; },
                             &err) == TFHE_OK, "admit");
            CHECK(book.in_use <= book.budget, "budget exceeded: %zu > %zu", book.in_use, book.budget);
            CHECK(!book.active.empty(), "nothing admitted");
            Tick t;
            book.next_tick(t, m.wb);
            CHECK(t.total <= mb, "tick of %u gates above %u", t.total, mb);
            CHECK(t.segs.size() + t.lins.size() <= book.seg_cap, "segment cap");
            uint32_t at = 0;
            for (size_t k = 0; k < t.segs.size(); k++) {
                CHECK(t.starts[k] == at, "tick start");
                at += t.segs[k].rows;
            }
            CHECK(at == t.total, "tick total");
            for (auto& cp : t.copies) m.copy(cp);
            m.lins(t.lins.data(), t.lins.size());
            m.gates(t.segs.data(), t.segs.size());
            // the device finishes ticks in order; with `lag` ticks in flight
            // only the ticks before the last `lag` have completed
            const uint64_t completed = book.ticks > lag ? book.ticks - lag : 0;
            for (auto* q : book.active)
                CHECK(!(q->level >= q->net.levels.size() && q->last_tick >= book.ticks), "last tick not recorded");
            book.retire([&](uint64_t base) { CHECK(allocs.erase(base) == 1, "release of an unknown base"); },
                        completed);
        }
        book.retire([&](uint64_t base) { CHECK(allocs.erase(base) == 1, "release of an unknown base"); }, book.ticks);
        CHECK(book.in_use == book.fixed, "in use %zu after the last query, fixed %zu", book.in_use, book.fixed);
        CHECK(allocs.empty(), "temporaries not released");
        for (auto& x : qs) {
            CHECK(book.done.count(x.id) == 1, "query %llu not done", (unsigned long long)x.id);
            CHECK(read_bits(m, x.sum, x.width) == x.want, "server sum (batch %u)", mb);
        }
      }
    }
}

int main() {
    std::mt19937_64 rng(12345);
    test_predicates(32);
    test_predicates(64);
    test_select_and_sum(32, rng);
    test_select_and_sum(64, rng);
    test_radix(rng);
    test_expressions(rng);
    test_server(rng);
    printf("host netlist checks passed: %d\n", g_checks);
    return 0;
}
