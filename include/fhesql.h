/*
 * fhesql.h -- C ABI of the MI355X (gfx950) TFHE oblivious-selection library.
 *
 * What it computes.  The FHE-SQL paper's server loop (Algorithm 2, Section 4)
 * evaluates the WHERE expression of a query homomorphically for every row,
 * producing one encrypted boolean per row (the selection mask M_enc,
 * Section 4.3), and then applies If-Then-Else(mask, value, enc(0)) to the
 * selected columns (Eqs. 2-3 of Section 6.D), optionally summing the
 * selected values (the aggregation equations after Eq. 3).  Its
 * homomorphic operations are TFHE's (the paper's Section 2.2 cites the TFHE
 * paper, ePrint 2018/421, and uses its boolean gates).  This library
 * implements that server path on one GPU with TFHE gate bootstrapping:
 *   bootstrap = blind rotation (gadget decomposition + GGSW x GLWE external
 *   products) -> sample extraction -> LWE key switching,
 * and boolean circuits of bootstrapped gates for =, <, >, BETWEEN, whole
 * WHERE expression trees (Section 4.3 B), the masked select and the masked
 * SUM; programmable bootstrapping with look-up tables over radix-encoded
 * 64-bit-torus integers; and a continuous-batching server for SUM queries.
 *
 * Conventions (all calls).
 *  - Torus values are uint32_t words when torus_bits = 32 and uint64_t words
 *    when torus_bits = 64 ("words" below).  Arithmetic is mod 2^torus_bits.
 *  - LWE ciphertext of dimension d: d mask words then the body (d+1 words).
 *    "small" LWE: d = n (under the LWE key s); "big" LWE: d = k*N (under the
 *    extracted GLWE key).  A batch of B ciphertexts is B*(d+1) contiguous words.
 *  - Bits are encoded as (2b-1)/8 on the torus; integers are given bit-wise,
 *    least significant bit first: a column of `rows` w-bit values is
 *    rows*w*(n+1) words, bit j of row r at ((r*w)+j)*(n+1).
 *  - Pointers named d_* are device pointers (HIP global memory) owned by the
 *    caller; they must stay valid until the stream has finished the call.
 *    Outputs must not alias inputs.  h_* pointers are host memory.
 *  - Calls are stream-ordered on the given HIP stream (NULL = default
 *    stream): they enqueue their work and return without waiting for the
 *    device, and their inputs are read and outputs written in stream order.
 *    The calls of one context share one device workspace; a call on another
 *    stream than the previous user of the workspace first makes its stream
 *    wait (hipStreamWaitEvent) for that earlier call, so calls on different
 *    streams are serialized on the device but never race.  The host blocks
 *    only when a call must grow the workspace (it then waits for the earlier
 *    calls that used it), when all pinned staging buffers of level schedules
 *    are still in flight, in sql_server_step (documented there) and in the
 *    setup calls (context creation and destruction, tfhe_ctx_sync).  Calls
 *    are not thread-safe for one context.  Results are a pure function of
 *    the keys and inputs: batching and scheduling never change an output bit.
 *  - Return value: 0 on success, else a negative error code (below);
 *    tfhe_last_error() gives a message.  No C++ exception crosses the ABI.
 */
#ifndef FHESQL_H
#define FHESQL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TFHE_OK 0
#define TFHE_EINVAL (-1)   /* bad argument or parameter set */
#define TFHE_ESHAPE (-2)   /* size or shape mismatch */
#define TFHE_ENOMEM (-3)   /* device workspace allocation failed */
#define TFHE_EHIP (-4)     /* HIP runtime error (including an earlier async fault) */

/* TFHE parameters.  k must be 1; N a power of two in [64, 2048];
 * 1 <= l, l*bg_bits <= torus_bits; ks_t*ks_base_bits <= torus_bits. */
typedef struct tfhe_params {
    uint32_t torus_bits;   /* 32 or 64 */
    uint32_t n;            /* LWE dimension */
    uint32_t k;            /* GLWE dimension */
    uint32_t N;            /* GLWE polynomial size */
    uint32_t bg_bits;      /* log2 of the gadget base Bg */
    uint32_t l;            /* gadget levels */
    uint32_t ks_base_bits; /* log2 of the key-switching base */
    uint32_t ks_t;         /* key-switching levels */
} tfhe_params;

typedef struct tfhe_ctx tfhe_ctx;

/* Blind-rotation kernel selection: the exact limb-split int8 MFMA external
 * product (default) or the plain scalar-integer one.  Both give identical bits. */
#define TFHE_KERNEL_MFMA 0
#define TFHE_KERNEL_PLAIN 1

/* SQL comparison operators (operators are plaintext metadata, Section 4.3 B). */
#define SQL_OP_EQ 0
#define SQL_OP_LT 1
#define SQL_OP_GT 2
#define SQL_OP_BETWEEN 3

/* Sizes in words of the key material for a parameter set:
 * BSK [n][(k+1)l][k+1][N] (GGSW encryptions of the LWE key bits) and
 * KSK [kN][ks_t][2^ks_base_bits][n+1] (LWE encryptions of v*s'_i/B^j).
 * Returns 0 for invalid parameters. */
size_t tfhe_bsk_words(const tfhe_params* p);
size_t tfhe_ksk_words(const tfhe_params* p);

/* Create a context on the current device: validates p, copies the keys to
 * the device (bsk/ksk are host pointers if keys_on_device == 0, device
 * pointers otherwise -- keys generated on the device need no host round trip;
 * sizes in bytes must match tfhe_bsk_words/tfhe_ksk_words), builds the
 * device-only limb-planar Toeplitz form of the BSK and allocates workspace
 * lazily.  With torus_bits = 32 and N = 1024 it also builds, when the device
 * has room, the BSK's 16-byte key windows (16 bytes per byte of the limb
 * form: 968 MB at n = 630, l = 3), from which the blind rotation reads its
 * A fragments directly; without room it stages the key in LDS instead (same
 * output bits).  With torus_bits = 32 it also keeps the key-switching table
 * as int8 limbs (4 bytes per word, 84 MB at the standard set) for the MFMA
 * key switch; without room the key switch reads the word table.  Blocks
 * until the keys are on the device.  The context owns its copies; the
 * caller keeps ownership of bsk/ksk. */
int tfhe_ctx_create(const tfhe_params* p, const void* bsk, size_t bsk_bytes,
                    const void* ksk, size_t ksk_bytes, int keys_on_device,
                    tfhe_ctx** out);
void tfhe_ctx_destroy(tfhe_ctx* ctx);
const char* tfhe_last_error(const tfhe_ctx* ctx);
/* Select TFHE_KERNEL_MFMA or TFHE_KERNEL_PLAIN for later blind rotations. */
int tfhe_set_kernel(tfhe_ctx* ctx, int kind);
/* Tuning knobs (none changes an output bit):
 *   TFHE_TUNE_MAX_BATCH  maximum ciphertexts per blind-rotation launch when a
 *                        circuit level is split into launches (default 65536);
 *   TFHE_TUNE_ROW_PASS   MFMA kernel row tiles per pass (0 = default for N,
 *                        otherwise an instantiated variant -- q = 32: 1 at
 *                        N = 64, N/64 or N/128 for N = 256..1024, 8 at
 *                        N = 2048; q = 64: 1 at N = 64, 4 for N = 256..1024,
 *                        8 or 4 at N = 2048).
 * Returns TFHE_EINVAL for an unknown key or unsupported value. */
#define TFHE_TUNE_MAX_BATCH 1
#define TFHE_TUNE_ROW_PASS 2
/*   TFHE_TUNE_DIGIT_BLOCKS 0 = the best digit grouping that fits in LDS
 *                        (default): with one MFMA row pass, when both
 *                        accumulator components fit in LDS (small N),
 *                        l <= 4 and the batch loses no occupancy by it (at
 *                        N = 256: up to 16 ciphertexts per CU), all key and
 *                        digit blocks of a CMux step staged together (three
 *                        barriers per step, the second component's digits
 *                        formed while the first component's blocks run);
 *                        else one component's
 *                        blocks at a time with accumulator component 0 held
 *                        in LDS; else all blocks of a CMux step at once, else
 *                        pairs of levels of one component (l even), else one
 *                        (u,p) block at a time; 1 = one block at a time;
 *                        2 = pairs when l is even and they fit, else one;
 *                        3 = all blocks of a step, accumulator in global
 *                        memory, when they fit; 4 = one component's blocks
 *                        at a time with component 0 in LDS and the key
 *                        staged in LDS, when it fits.  With the key windows
 *                        of a 1024-coefficient 32-bit context (see
 *                        tfhe_ctx_create) and one row pass, 0 reads the key
 *                        from them instead (no key staging, the second
 *                        component's digits formed while the first
 *                        component's blocks run).
 *                        Every grouping gives the same output bits.
 * The blind-rotation workspace depends on the row pass and digit grouping
 * (several passes with per-group digits add a digit cache).  Direct calls and
 * the level executor size it per call; a server sizes it at creation, and a
 * later tuning that needs more makes sql_server_step return TFHE_EINVAL
 * without launching (restore the tuning, or create a new server). */
#define TFHE_TUNE_DIGIT_BLOCKS 3
/*   TFHE_TUNE_SPLIT_GROUPS for N >= 256, a blind rotation of at most this
 *                        many groups of 16 ciphertexts runs each step as two
 *                        launches that spread every group's digits and
 *                        output rows over many workgroups (latency of small
 *                        batches: SUM-tree levels, server ticks) instead of
 *                        one workgroup per group for all n steps; -1 (the
 *                        default) = half the device's CUs for N >= 512 and
 *                        never for N = 256, 0 = never. */
#define TFHE_TUNE_SPLIT_GROUPS 4
int tfhe_set_tuning(tfhe_ctx* ctx, int key, int64_t value);
/* Current value of a tuning knob (as set, 0 or -1 for the defaults). */
int tfhe_get_tuning(tfhe_ctx* ctx, int key, int64_t* value);

/* Waits for the stream and reports any asynchronous fault. */
int tfhe_ctx_sync(tfhe_ctx* ctx, void* hip_stream);

/* Blind rotation + sample extraction (TFHE bootstrapping without the key
 * switch) of B small LWE ciphertexts d_lwe_in [B][n+1].  d_testv: N words of
 * the test polynomial, or NULL for the gate test polynomial (all 1/8).
 * d_out [B][kN+1]: big LWE ciphertexts under the extracted key. */
int tfhe_bootstrap_batch(tfhe_ctx* ctx, const void* d_lwe_in, const void* d_testv,
                         void* d_out, uint32_t B, void* hip_stream);

/* tfhe_bootstrap_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments and output bits, but the blind-rotation
 * workspace is a static device array of tfhe_noalloc_scratch_bytes() bytes
 * (32 MiB; one copy per device, held until the process ends) and the call
 * allocates nothing and records no timing events.  A batch whose workspace
 * would exceed the array fails with TFHE_ESHAPE before any launch (at the
 * standard 32-bit set up to 4096 ciphertexts fit; parameter sets whose
 * accumulators stay in LDS need none).  The context's device must be
 * current.  Every call on a device shares that device's array: calls that
 * overlap on one GPU (different streams, threads or contexts) race, calls
 * in one stream are ordered. */
int tfhe_bootstrap_batch_noalloc(tfhe_ctx* ctx, const void* d_lwe_in, const void* d_testv,
                                 void* d_out, uint32_t B, void* hip_stream);
size_t tfhe_noalloc_scratch_bytes(void);

/* LWE key switching of B big ciphertexts d_in [B][kN+1] to d_out [B][n+1].
 * The batch's rounded digits (B*kN 16-bit values, 32-bit when
 * ks_t*ks_base_bits > 16) are staged in the context's workspace. */
int tfhe_keyswitch_batch(tfhe_ctx* ctx, const void* d_in, void* d_out, uint32_t B,
                         void* hip_stream);

/* Bootstrapped boolean gates on B independent input tuples: d_x, d_y (and
 * d_z for MAJ) [B][n+1]; d_out [B][n+1].  op: 0 AND, 1 NAND, 2 OR, 3 NOR,
 * 4 XOR, 5 XNOR, 6 ANDNY (not x and y), 7 MAJ. */
int tfhe_gate_batch(tfhe_ctx* ctx, int op, const void* d_x, const void* d_y,
                    const void* d_z, void* d_out, uint32_t B, void* hip_stream);

/* WHERE mask of a column scan (Algorithm 2's mask loop; Eq. 1 for equality):
 * d_mask[r] = enc(col[r] op lit) for every row.  d_col [rows][w][n+1];
 * d_lit_a [w][n+1] (encrypted literal bits); d_lit_b: upper literal for
 * BETWEEN (lit_a <= col <= lit_b), else NULL; d_mask [rows][n+1]. */
int sql_mask_scan(tfhe_ctx* ctx, const void* d_col, uint32_t rows, uint32_t w, int op,
                  const void* d_lit_a, const void* d_lit_b, void* d_mask, void* hip_stream);

/* Masked select (If-Then-Else with an encrypted zero, Eqs. 2-3):
 * d_out[r][j] = AND(mask[r], col[r][j]).  d_out [rows][w][n+1]. */
int sql_masked_select(tfhe_ctx* ctx, const void* d_mask, const void* d_col, uint32_t rows,
                      uint32_t w, void* d_out, void* hip_stream);

/* Masked SUM (the aggregation of the selected entries): d_sum receives the
 * encrypted bits of sum_r mask[r]*col[r], width w + ceil(log2 rows),
 * [width][n+1].  *width_out returns that width. */
int sql_masked_sum(tfhe_ctx* ctx, const void* d_mask, const void* d_col, uint32_t rows,
                   uint32_t w, void* d_sum, uint32_t* width_out, void* hip_stream);

/* One table scan of a batch: mask (and optionally the masked select). */
typedef struct sql_table_query {
    const void* d_col;     /* [rows][w][n+1] predicate column */
    const void* d_sel_col; /* [rows][w][n+1] selected column or NULL (mask only) */
    uint32_t rows;
    uint32_t w;
    int op;
    const void* d_lit_a;   /* [w][n+1] */
    const void* d_lit_b;   /* [w][n+1] for BETWEEN else NULL */
    void* d_mask;          /* [rows][n+1] */
    void* d_sel_out;       /* [rows][w][n+1] or NULL */
} sql_table_query;

/* Many tables with uneven row counts and mixed predicates in one level-batched
 * schedule: every level's gates of all tables go into one launch sequence.
 * use_graph != 0 captures the whole schedule into one HIP graph and launches
 * it. */
int sql_scan_batch(tfhe_ctx* ctx, const sql_table_query* q, uint32_t count, int use_graph,
                   void* hip_stream);
/* With use_graph, the instantiated graph is kept (up to 8 per context, least
 * recently used evicted) keyed by everything that fixes its launches: the
 * tables' device addresses and sizes, predicates, the tuning and the
 * workspace address; repeating a batch relaunches it without a new capture.
 * A workspace reallocation drops every kept graph.  tfhe_graph_stats reports
 * the captures and graph launches so far and the graphs kept (any pointer may
 * be NULL). */
int tfhe_graph_stats(tfhe_ctx* ctx, uint64_t* captures, uint64_t* launches, uint64_t* cached);

/* ---- Homomorphic expression trees (Section 4.3 B: leaves are operands,
 * inner nodes are operators given as plaintext metadata).
 *
 * Value nodes are w-bit integers (bit-wise encrypted, LSB first); boolean
 * nodes are single encrypted bits.  Circuits, per row:
 *   EQ: XNOR per bit + balanced AND tree; LT: borrow chain
 *   b_j = MAJ(not a_j, c_j, b_{j-1}), b_{-1} = FALSE; GT(a,b) = LT(b,a);
 *   NE = NOT EQ; LE(a,b) = NOT LT(b,a); GE(a,b) = NOT LT(a,b);
 *   AND, OR, XOR: one bootstrapped gate; NOT: exact negation (no bootstrap);
 *   ITE(c, x, y) per bit: AND(c, x_j) + ANDNY(c, y_j) + 1/8 (linear, exact);
 *   MAX(a,b) = ITE(LT(a,b), b, a); MIN(a,b) = ITE(LT(a,b), a, b);
 *   CONST: the trivial encryption (0, +-1/8) of each bit of `value`. */
#define SQL_EXPR_COLUMN 0   /* value: column `col` of d_cols */
#define SQL_EXPR_CONST 1    /* value: plaintext `value` (low w bits) */
#define SQL_EXPR_LITERAL 2  /* value: encrypted literal at d_lit, [w][n+1] */
#define SQL_EXPR_CMP 3      /* bool: `op` (SQL_CMP_*) of values a, b */
#define SQL_EXPR_AND 4      /* bool: a AND b */
#define SQL_EXPR_OR 5       /* bool: a OR b */
#define SQL_EXPR_XOR 6      /* bool: a XOR b */
#define SQL_EXPR_NOT 7      /* bool: NOT a */
#define SQL_EXPR_MAX 8      /* value: max(a, b) */
#define SQL_EXPR_MIN 9      /* value: min(a, b) */
#define SQL_EXPR_ITE 10     /* value: c ? a : b (c bool) */

#define SQL_CMP_EQ 0
#define SQL_CMP_NE 1
#define SQL_CMP_LT 2
#define SQL_CMP_LE 3
#define SQL_CMP_GT 4
#define SQL_CMP_GE 5

typedef struct sql_expr {
    int32_t kind;         /* SQL_EXPR_* */
    int32_t op;           /* SQL_EXPR_CMP: SQL_CMP_* */
    int32_t a, b, c;      /* operand node indices, each smaller than this node's */
    int32_t col;          /* SQL_EXPR_COLUMN: index into d_cols */
    uint64_t value;       /* SQL_EXPR_CONST */
    const void* d_lit;    /* SQL_EXPR_LITERAL: device [w][n+1] */
} sql_expr;

/* Evaluates nodes[0..nnodes-1] (topological order; the last node is the root)
 * for every row.  d_cols: host array of ncols device pointers, each
 * [rows][w][n+1].  d_out: [rows][n+1] for a boolean root, [rows][w][n+1] for
 * a value root; it must not alias an input.  Every gate of the netlist is
 * bootstrapped whatever its inputs (no constant folding), so the output bits
 * are a function of the node list and the inputs alone.  Errors: TFHE_EINVAL
 * for an unknown kind or operator, an operand index out of order, a boolean
 * where a value is expected (or the reverse), a column index >= ncols or a
 * null pointer; TFHE_ESHAPE for w outside 1..64. */
int sql_expr_eval(tfhe_ctx* ctx, const void* const* d_cols, uint32_t ncols, uint32_t rows,
                  uint32_t w, const sql_expr* nodes, uint32_t nnodes, void* d_out,
                  void* hip_stream);

/* Kernel timing.  While enabled (on != 0), every blind-rotation and
 * key-switching kernel launched by this context is bracketed by HIP events
 * recorded on the stream it runs on (not during graph capture).  Enabling
 * clears the counters.  tfhe_timing_read synchronizes the events and returns,
 * per kernel kind (0 = blind rotation, 1 = key switching), the number of
 * launches, the summed kernel time in milliseconds and the summed batch size
 * (ciphertexts).  Any pointer may be NULL. */
int tfhe_timing_enable(tfhe_ctx* ctx, int on);
int tfhe_timing_read(tfhe_ctx* ctx, int kind, uint64_t* launches, double* total_ms,
                     uint64_t* cts);

/* Ordered launch log since timing was enabled (not during graph capture):
 * for launch i, kinds[i] (0 blind rotation, 1 key switching) and sizes[i]
 * (ciphertexts).  Copies min(max, count) entries (either array may be NULL);
 * *count receives the number recorded (at most 2^22).  The schedule is a
 * function of the query's structure and row counts only -- what the ideal
 * functionality of Section 5 leaks (the AST with literals redacted and the
 * table size) -- never of the encrypted data or literals. */
int tfhe_timing_log(tfhe_ctx* ctx, uint32_t* kinds, uint32_t* sizes, uint64_t max, uint64_t* count);

/* ---- radix integers (programmable bootstrapping with look-up tables) ----
 * An integer is nb blocks of 4-bit messages, least significant block first; a
 * block value x in [0, 32) (4 message bits + 1 carry bit) is the LWE
 * encryption of x * 2^q / 64 (the top torus bit is padding).  Each gate is a
 * linear combination followed by a programmable bootstrap whose test
 * polynomial encodes a table over Z_32.  Columns are [rows][nb][n+1] words. */

/* d_mask[r] = 16 * [col[r] op lit] as one block (op: SQL_OP_EQ/LT/GT):
 * block-wise x_i = a_i - c_i + 16 -> {lt, eq, gt}, tree-combined 2*hi + lo.
 * nb >= 2.  d_lit [nb][n+1]. */
int sql_radix_mask_scan(tfhe_ctx* ctx, const void* d_col, uint32_t rows, uint32_t nb, int op,
                        const void* d_lit, void* d_mask, void* hip_stream);
/* d_out[r][i] = col[r][i] if mask[r] encrypts 16, else 0 (If-Then-Else). */
int sql_radix_masked_select(tfhe_ctx* ctx, const void* d_mask, const void* d_col, uint32_t rows,
                            uint32_t nb, void* d_out, void* hip_stream);
/* d_sum [nb][n+1] = sum of the rows of d_vals [rows][nb][n+1] mod 2^(4 nb):
 * pairwise row tree of ripple-carry radix additions. */
int sql_radix_sum(tfhe_ctx* ctx, const void* d_vals, uint32_t rows, uint32_t nb, void* d_sum,
                  void* hip_stream);

/* ---- continuous-batching query server ----
 * Serves SELECT SUM(col2) WHERE col1 op literal queries (Algorithm 2's mask,
 * the If-Then-Else of Eqs. 2-3 and the aggregation after Eq. 3).  Queries
 * are admitted while the device memory they need (circuit temporaries) fits
 * in the budget next to the resident keys and the server's staging buffers;
 * each tick runs the next circuit level of every active query -- up to
 * max_batch gates, a level may span ticks -- as one batched combine / blind
 * rotation / key switch, so queries that arrive while others run share the
 * same launches.  A query's result bits do not depend on what it is batched
 * with. */
typedef struct sql_server sql_server;

typedef struct sql_sum_query {
    const void* d_col;      /* [rows][w][n+1] predicate column */
    const void* d_sum_col;  /* [rows][w][n+1] summed column */
    uint32_t rows;
    uint32_t w;
    int op;                 /* SQL_OP_EQ, SQL_OP_LT, SQL_OP_GT or SQL_OP_BETWEEN */
    const void* d_lit_a;    /* [w][n+1] */
    const void* d_lit_b;    /* [w][n+1] for BETWEEN, else NULL */
    void* d_sum;            /* [w + ceil(log2 rows)][n+1] result */
} sql_sum_query;

/* hbm_budget_bytes: total device memory the server may account for (keys,
 * two staging sets, temporaries); max_batch: gates per tick. */
int sql_server_create(tfhe_ctx* ctx, size_t hbm_budget_bytes, uint32_t max_batch,
                      sql_server** out);
void sql_server_destroy(sql_server* srv);
/* Queue a query; its buffers must stay valid until it is done.  *id receives
 * its identifier.  Fails with TFHE_ENOMEM if it could never fit the budget. */
int sql_server_submit(sql_server* srv, const sql_sum_query* q, uint64_t* id);
/* Queue SELECT SUM(d_sum_col) WHERE <expression tree> over `rows` rows: the
 * nodes (as in sql_expr_eval; the root must be a condition) are compiled at
 * submission, so the node array may be freed on return, while the columns,
 * literals, d_sum_col [rows][w][n+1] and d_sum (sum width of
 * sql_masked_sum, [width][n+1]) must stay valid until the query is done.
 * Errors as sql_expr_eval, TFHE_ENOMEM as sql_server_submit. */
int sql_server_submit_expr(sql_server* srv, const void* const* d_cols, uint32_t ncols, uint32_t rows,
                           uint32_t w, const sql_expr* nodes, uint32_t nnodes, const void* d_sum_col,
                           void* d_sum, uint64_t* id);
/* Enqueues one tick on the stream and returns while it runs: two ticks may
 * be in flight (the server alternates two staging sets), so the call blocks
 * only until the tick before the previous one has finished.  Queries whose
 * last level ran in a finished tick are retired (sql_server_done turns 1 and
 * their temporaries go back to the stream-ordered pool), queued queries are
 * admitted, and the next tick's copies, linear steps and gates are issued.
 * A tick with nothing to issue waits for the ticks in flight instead, so a
 * loop that steps until every query is done ends.  Consecutive ticks on
 * different streams are ordered by an event.  Outputs (any may be NULL):
 * gates issued, active and queued query counts. */
int sql_server_step(sql_server* srv, void* hip_stream, uint32_t* gates, uint32_t* active,
                    uint32_t* queued);
/* 1 when query id has completed (its d_sum holds the result), 0 otherwise,
 * negative for an unknown id. */
int sql_server_done(sql_server* srv, uint64_t id);
/* Device bytes the server currently accounts for. */
size_t sql_server_bytes_in_use(const sql_server* srv);

/* ---- client-side helpers on the device (synthetic data and checks) ---- */

/* Counter-based SplitMix64 stream: value i of (seed, tag) is
 * mix64(K + (i+1)*0x9E3779B97F4A7C15), K = mix64(seed ^ mix64(tag + 0x9E3779B97F4A7C15)).
 * Fills d_out[count] (uint64_t) with values start .. start+count-1. */
int tfhe_rng_fill(uint64_t seed, uint64_t tag, uint64_t start, uint64_t count, void* d_out,
                  void* hip_stream);

/* Key generation on the device from seeded streams (the tags of the seeded
 * input recipe): binary keys s (n words) and S (kN words) written to
 * d_lwe_key / d_glwe_key (words holding 0/1), BSK and KSK to d_bsk / d_ksk
 * (tfhe_bsk_words / tfhe_ksk_words words).  sigma_log2 values give the
 * noise standard deviations 2^-lwe_sigma_log2 and 2^-glwe_sigma_log2. */
int tfhe_keygen(const tfhe_params* p, uint64_t seed, uint32_t lwe_sigma_log2,
                uint32_t glwe_sigma_log2, void* d_lwe_key, void* d_glwe_key, void* d_bsk,
                void* d_ksk, void* hip_stream);

/* Encrypt `count` plaintext torus values d_mu[count] (words) under the LWE
 * key d_key (n words of 0/1) with seeded masks/noise: ciphertext i uses mask
 * values (start+i)*n .. and noise sample start+i of the (seed, tag) streams.
 * d_out [count][n+1]. */
int tfhe_lwe_encrypt(const tfhe_params* p, uint64_t seed, uint64_t mask_tag,
                     uint64_t noise_tag, uint32_t sigma_log2, uint64_t start,
                     const void* d_key, const void* d_mu, void* d_out, uint64_t count,
                     uint32_t dim, void* hip_stream);

/* Phases b - <a, s> of count LWE ciphertexts of dimension dim: d_out[count] words. */
int tfhe_lwe_phase(const tfhe_params* p, const void* d_key, const void* d_cts, void* d_out,
                   uint64_t count, uint32_t dim, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* FHESQL_H */
