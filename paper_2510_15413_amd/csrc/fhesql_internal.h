// Internal definitions of the gfx950 TFHE library: context, device helpers
// and kernel launchers shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/fhesql.h"

#define FHE_DEV __device__ __forceinline__

// ------------------------------------------------------------------ torus

template <typename T> struct Torus;
template <> struct Torus<uint32_t> {
    static constexpr int Q = 32;
    static constexpr int LIMBS = 4;  // balanced int8 limbs of a key word
};
template <> struct Torus<uint64_t> {
    static constexpr int Q = 64;
    static constexpr int LIMBS = 8;
};

// Round x to its top `bits` bits, ties up: floor((x + 2^(Q-bits-1)) / 2^(Q-bits)).
template <typename T>
FHE_DEV T round_top(T x, int bits) {
    constexpr int Q = Torus<T>::Q;
    if (bits >= Q) return x;
    const int sh = Q - bits;
    return (T)((x + ((T)1 << (sh - 1))) >> sh);
}

// Modulus switch to Z_2N (log2(2N) = lg2n bits).
template <typename T>
FHE_DEV uint32_t mod_switch(T x, int lg2n) { return (uint32_t)round_top<T>(x, lg2n); }

// Coefficient j of X^e * P (e in [0, 2N)) read through an accessor p(idx).
template <typename T, typename F>
FHE_DEV T monomial_coef(F p, int N, int e, int j) {
    int neg = e >= N;
    int es = neg ? e - N : e;
    int s = j - es;
    T v = s >= 0 ? p(s) : (T)(0 - p(s + N));
    return neg ? (T)(0 - v) : v;
}

// ------------------------------------------------------- SplitMix64 stream

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t tag) {
    return mix64(seed ^ mix64(tag + kGamma));
}
// Value `idx` of the stream with key K.
__host__ __device__ __forceinline__ uint64_t stream_at(uint64_t K, uint64_t idx) {
    return mix64(K + (idx + 1) * kGamma);
}
// Uniform q-bit torus value (top bits).
template <typename T>
__host__ __device__ __forceinline__ T stream_torus(uint64_t K, uint64_t idx) {
    uint64_t v = stream_at(K, idx);
    return Torus<T>::Q == 64 ? (T)v : (T)(v >> 32);
}
// Centred Irwin-Hall error (12 uniform 32-bit halves of values 6s..6s+5),
// scaled to std 2^(Q - sigma_log2), ties rounded up.
template <typename T>
__host__ __device__ __forceinline__ T stream_noise(uint64_t K, uint64_t s, int sigma_log2) {
    int64_t acc = -((int64_t)6 << 32);
    for (int t = 0; t < 6; t++) {
        uint64_t v = stream_at(K, 6 * s + t);
        acc += (int64_t)(v >> 32) + (int64_t)(v & 0xFFFFFFFFull);
    }
    const int shift = 32 - Torus<T>::Q + sigma_log2;
    int64_t e = shift > 0 ? ((acc + ((int64_t)1 << (shift - 1))) >> shift) : (int64_t)((uint64_t)acc << (-shift));
    return (T)(uint64_t)e;
}

// Gates, segments and netlists (host-only code shared with the host tests).
#include "netlist.h"

// ---------------------------------------------------------------- context

struct tfhe_ctx {
    tfhe_params p{};
    int q = 32;
    int kernel = TFHE_KERNEL_MFMA;
    uint32_t max_batch = 65536;  // ciphertexts per blind-rotation launch in circuits
    int row_pass = 0;            // MFMA row tiles per pass (0 = default)
    int digit_blocks = 0;        // 0 auto, 1 one digit block at a time, 2 pairs of levels
    int64_t split_groups = -1;   // batches of at most this many 16-ciphertext groups take the
                                 // multi-workgroup blind rotation (-1 = half the CUs)
    void* d_radix_tv = nullptr;  // radix look-up test polynomials [8][N] words
    void* d_bsk = nullptr;     // [n][(k+1)l][k+1][N] words
    int8_t* d_bsk8 = nullptr;  // [n][(k+1)l][k+1][LIMBS][2N] Toeplitz limb form
    void* d_win = nullptr;     // [n][(k+1)l][k+1][LIMBS][2N] 16-byte windows of bsk8 (N = 1024, q = 32), or null
    size_t win_bytes = 0;
    void* d_ksk = nullptr;     // [kN][t][2^b][ks_row] words (rows padded to whole 128-byte lines)
    size_t ks_row = 0;         // words per KSK row on the device: n+1 rounded up to 128 bytes
    int8_t* d_ksk8 = nullptr;  // q = 32: [4 limbs][ks_wp][kN*t*2^b] balanced int8 limbs of the KSK, row-transposed
    int ks_wp = 0;             // n+1 rounded up to 16 (rows of d_ksk8 past n are zero)
    size_t ksk8_bytes = 0;
    void* d_gate_tv = nullptr; // N words of 1/8
    void* d_false = nullptr;   // trivial FALSE ciphertext (0^n, -1/8)
    // workspace (grown on demand), shared by the calls on this context.  A
    // call on stream s first makes s wait for the event recorded after the
    // last call that used it (if that was another stream), so calls stay
    // stream-ordered without host synchronization.
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipEvent_t ws_event = nullptr;
    hipStream_t ws_stream = nullptr;
    bool ws_used = false;
    // pinned host buffers for uploads of level schedules; a buffer is reused
    // once the copy that last read it has completed
    struct HostStage {
        void* p;
        size_t cap;
        hipEvent_t ev;
        bool used;
    };
    std::vector<HostStage> stages;
    // instantiated graphs of level schedules, keyed by everything that
    // determines their launches (resolved segments, launch sizes, copies,
    // tuning, workspace address)
    struct GraphEntry {
        std::vector<uint8_t> key;
        hipGraphExec_t exec;
        uint64_t last_use;
    };
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0, graph_captures = 0, graph_launches = 0;
    int device = 0;  // the device current at creation, which holds every buffer
    std::string err;
    hipDeviceProp_t prop{};
    // kernel timing (per kind: 0 blind rotation, 1 key switching)
    bool timing = false;
    struct Timed {
        hipEvent_t a, b;
        int kind;
        uint32_t cts;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;
    uint64_t t_launch[2] = {0, 0}, t_cts[2] = {0, 0};
    std::vector<uint64_t> t_log;  // (kind << 32) | ciphertexts, per launch in order
    double t_ms[2] = {0, 0};
};

// Records an event pair around one launch when timing is enabled.
struct TimedLaunch {
    tfhe_ctx* c;
    hipStream_t s;
    int kind;
    uint32_t cts;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(tfhe_ctx* cc, hipStream_t ss, int k, uint32_t n);
    ~TimedLaunch();
};

int ctx_fail(tfhe_ctx* c, int code, const std::string& msg);
int hip_check(tfhe_ctx* c, hipError_t e, const char* what);
// Workspace of at least `bytes` for a call on stream s: grows it if needed
// (waiting for earlier calls that used the old buffer) and otherwise makes s
// wait for the last call that used it on another stream.
int ws_acquire(tfhe_ctx* c, hipStream_t s, size_t bytes);
// Records that the calls just enqueued on s use the workspace.
int ws_release(tfhe_ctx* c, hipStream_t s);
// Enqueues a host-to-device copy of `bytes` from host memory `src` on s
// through a pinned staging buffer (src may be reused on return).
int stage_upload(tfhe_ctx* c, hipStream_t s, void* d_dst, const void* src, size_t bytes);
void graphs_clear(tfhe_ctx* c);

size_t word_bytes(const tfhe_ctx* c);

// kernel launchers (each returns a TFHE_* code)
int launch_bsk_limbs(tfhe_ctx* c, hipStream_t s);
// ws: blind-rotation workspace of ws_cap bytes (at least blind_rotate_ws_bytes(c, B)
// under the current tuning, else the launch fails with TFHE_EINVAL).
int launch_blind_rotate(tfhe_ctx* c, const void* lwe_in, const void* testv_table,
                        const int32_t* tv_index, void* big_out, uint32_t B, void* ws,
                        size_t ws_cap, hipStream_t s);
size_t blind_rotate_ws_bytes(const tfhe_ctx* c, uint32_t B);
// Largest blind-rotation workspace of any batch of at most Bmax ciphertexts.
size_t blind_rotate_ws_bytes_upto(const tfhe_ctx* c, uint32_t Bmax);
// dig: device buffer of at least ks_digits_bytes(c, B) bytes that the key
// switch fills with the batch's rounded digits before it reads them.
int launch_keyswitch(tfhe_ctx* c, const void* big_in, void* out, const uint64_t* out_ptrs,
                     uint32_t B, void* dig, size_t dig_cap, hipStream_t s);
size_t ks_digits_bytes(const tfhe_ctx* c, uint32_t B);
int launch_combine(tfhe_ctx* c, const Segment* d_segs, const uint32_t* d_seg_start,
                   int nseg, uint32_t total, void* lwe_out, uint64_t* out_ptrs,
                   int32_t* tv_index, hipStream_t s);
