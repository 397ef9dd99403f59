// Context management, key preprocessing, device key generation, encryption
// and the bootstrap / key-switch entry points of the C ABI.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "fhesql_internal.h"

int launch_br_mfma(tfhe_ctx* c, const void* lwe_in, const void* tv, const int32_t* tv_index,
                   void* big_out, uint32_t B, void* ws, size_t ws_cap, hipStream_t s);
int launch_br_plain(tfhe_ctx* c, const void* lwe_in, const void* tv, const int32_t* tv_index,
                    void* big_out, uint32_t B, hipStream_t s);
size_t mfma_ws_bytes(const tfhe_ctx* c, uint32_t B);
size_t mfma_ws_bytes_upto(const tfhe_ctx* c, uint32_t Bmax);
static int timing_drain(tfhe_ctx* c);

int ctx_fail(tfhe_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_check(tfhe_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return TFHE_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return ctx_fail(c, e == hipErrorOutOfMemory ? TFHE_ENOMEM : TFHE_EHIP, m);
}

size_t word_bytes(const tfhe_ctx* c) { return c->q == 32 ? 4 : 8; }

int ws_acquire(tfhe_ctx* c, hipStream_t s, size_t bytes) {
    if (bytes <= c->ws_bytes) {
        if (c->ws_used && c->ws_stream != s)
            return hip_check(c, hipStreamWaitEvent(s, c->ws_event, 0), "wait for the workspace");
        return TFHE_OK;
    }
    if (c->ws) {
        // earlier calls may still read the old buffer, and captured graphs
        // refer to its address
        if (c->ws_used) {
            hipError_t e = hipEventSynchronize(c->ws_event);
            if (e != hipSuccess) return hip_check(c, e, "wait before workspace growth");
        }
        graphs_clear(c);
        hipFree(c->ws);
        c->ws = nullptr;
        c->ws_bytes = 0;
        c->ws_used = false;
    }
    size_t want = bytes + bytes / 4;
    hipError_t e = hipMalloc(&c->ws, want);
    if (e != hipSuccess) {
        c->ws = nullptr;
        return hip_check(c, e, "workspace hipMalloc");
    }
    c->ws_bytes = want;
    return TFHE_OK;
}

int ws_release(tfhe_ctx* c, hipStream_t s) {
    if (!c->ws_event) {
        int rc = hip_check(c, hipEventCreateWithFlags(&c->ws_event, hipEventDisableTiming), "workspace event");
        if (rc) return rc;
    }
    c->ws_stream = s;
    c->ws_used = true;
    return hip_check(c, hipEventRecord(c->ws_event, s), "workspace event record");
}

int stage_upload(tfhe_ctx* c, hipStream_t s, void* d_dst, const void* src, size_t bytes) {
    if (!bytes) return TFHE_OK;
    constexpr size_t kMaxStages = 16;
    // a free buffer: never used or its last copy has completed
    auto is_free = [](const tfhe_ctx::HostStage& h) { return !h.used || hipEventQuery(h.ev) == hipSuccess; };
    tfhe_ctx::HostStage* pick = nullptr;
    for (auto& h : c->stages)
        if (h.cap >= bytes && is_free(h)) { pick = &h; break; }
    if (!pick) {
        tfhe_ctx::HostStage* spare = nullptr;  // a free buffer that is too small
        for (auto& h : c->stages)
            if (is_free(h)) { spare = &h; break; }
        if (!spare && c->stages.size() >= kMaxStages) {
            // every buffer is in flight: wait for the first one
            spare = &c->stages[0];
            int rc = hip_check(c, hipEventSynchronize(spare->ev), "wait for a staging buffer");
            if (rc) return rc;
        }
        if (!spare) {
            c->stages.push_back(tfhe_ctx::HostStage{nullptr, 0, nullptr, false});
            spare = &c->stages.back();
            int rc = hip_check(c, hipEventCreateWithFlags(&spare->ev, hipEventDisableTiming), "staging event");
            if (rc) { c->stages.pop_back(); return rc; }
        }
        if (spare->cap < bytes) {
            if (spare->p) hipHostFree(spare->p);
            spare->p = nullptr;
            spare->cap = 0;
            const size_t cap = std::max<size_t>(bytes + bytes / 4, 1 << 16);
            int rc = hip_check(c, hipHostMalloc(&spare->p, cap), "pinned staging buffer");
            if (rc) return rc;
            spare->cap = cap;
        }
        pick = spare;
    }
    memcpy(pick->p, src, bytes);
    int rc = hip_check(c, hipMemcpyAsync(d_dst, pick->p, bytes, hipMemcpyHostToDevice, s), "upload");
    if (rc) return rc;
    pick->used = true;
    return hip_check(c, hipEventRecord(pick->ev, s), "staging event record");
}

void graphs_clear(tfhe_ctx* c) {
    for (auto& g : c->graphs) hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

static bool valid_params(const tfhe_params* p, std::string* why) {
    auto bad = [&](const char* m) { if (why) *why = m; return false; };
    if (!p) return bad("null parameters");
    if (p->torus_bits != 32 && p->torus_bits != 64) return bad("torus_bits must be 32 or 64");
    if (p->k != 1) return bad("only k = 1 is supported");
    if (p->N < 64 || p->N > 2048 || (p->N & (p->N - 1))) return bad("N must be a power of two in [64, 2048]");
    if (p->n < 1 || p->n > 4096) return bad("n out of range");
    if (p->l < 1 || p->bg_bits < 1 || p->l * p->bg_bits > 31 || p->bg_bits > 8)
        return bad("gadget needs 1 <= bg_bits <= 8 and l*bg_bits <= 31");
    if (p->ks_t < 1 || p->ks_base_bits < 1 || p->ks_base_bits > 4 || p->ks_t * p->ks_base_bits > 32)
        return bad("key switching needs 1 <= ks_base_bits <= 4 and ks_t*ks_base_bits <= 32");
    return true;
}

extern "C" size_t tfhe_bsk_words(const tfhe_params* p) {
    if (!valid_params(p, nullptr)) return 0;
    return (size_t)p->n * (p->k + 1) * p->l * (p->k + 1) * p->N;
}

extern "C" size_t tfhe_ksk_words(const tfhe_params* p) {
    if (!valid_params(p, nullptr)) return 0;
    return (size_t)p->k * p->N * p->ks_t * ((size_t)1 << p->ks_base_bits) * (p->n + 1);
}

// ------------------------------------------------------------- key limbs

// bsk8[i][r][v][m][x] = limb m of Kext[N-1-x], K = BSK[i][r][v], with
// Kext[t] = K[t] (t >= 0), -K[t+N] (t < 0); balanced limbs in [-128, 127]
// with sum_m limb_m 2^{8m} = Kext mod 2^q.
template <typename T>
__global__ void bsk_limbs_kernel(const T* bsk, int8_t* bsk8, size_t polys, int N) {
    constexpr int NL = Torus<T>::LIMBS;
    const size_t total = polys * 2 * N;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t poly = idx / (2 * N);
        const int x = (int)(idx % (2 * N));
        const int t = N - 1 - x;
        const T* K = bsk + poly * N;
        T val = t >= 0 ? K[t] : (T)(0 - K[t + N]);
        int carry = 0;
        int8_t* dst = bsk8 + poly * NL * 2 * N + x;
#pragma unroll
        for (int m = 0; m < NL; m++) {
            int r = (int)((val >> (8 * m)) & 0xFF) + carry;
            carry = r >= 128;
            dst[(size_t)m * 2 * N] = (int8_t)(r - (carry << 8));
        }
    }
}

// win[row][x] = bytes x .. x+15 of limb row `row` of bsk8 (zero past its
// 2N bytes): the 16-byte-aligned A fragments of the windowed-key blind
// rotation, one per byte offset.
__global__ void key_windows_kernel(const int8_t* bsk8, uint4* win, size_t rows, int N2) {
    const size_t total = rows * N2;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t row = idx / N2;
        const int x = (int)(idx % N2);
        const uint8_t* S = (const uint8_t*)bsk8 + row * N2;
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 16; j++)
            if (x + j < N2) w[j >> 2] |= (uint32_t)S[x + j] << (8 * (j & 3));
        win[idx] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// ksk8[m][w][k] = limb m of KSK row k, word w (zero for w > n): the
// balanced int8 limbs (sum_m limb_m 2^{8m} = word mod 2^32) of the 32-bit
// key-switching table, each word's K = kN*t*2^b limbs contiguous, for the
// MFMA key switch.
__global__ void ksk_limbs_kernel(const uint32_t* ksk, int8_t* ksk8, size_t ks_row, int n, int Wp, size_t K) {
    const size_t total = (size_t)Wp * K;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int w = (int)(idx / K);
        const size_t k = idx % K;
        const uint32_t val = w <= n ? ksk[k * ks_row + w] : 0u;
        int carry = 0;
#pragma unroll
        for (int m = 0; m < 4; m++) {
            int r = (int)((val >> (8 * m)) & 0xFF) + carry;
            carry = r >= 128;
            ksk8[(size_t)m * total + idx] = (int8_t)(r - (carry << 8));
        }
    }
}

template <typename T>
__global__ void fill_kernel(T* dst, size_t count, T value) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = value;
}

int launch_bsk_limbs(tfhe_ctx* c, hipStream_t s) {
    const size_t polys = (size_t)c->p.n * (c->p.k + 1) * c->p.l * (c->p.k + 1);
    if (c->q == 32)
        hipLaunchKernelGGL(bsk_limbs_kernel<uint32_t>, dim3(2048), dim3(256), 0, s, (const uint32_t*)c->d_bsk,
                           c->d_bsk8, polys, (int)c->p.N);
    else
        hipLaunchKernelGGL(bsk_limbs_kernel<uint64_t>, dim3(2048), dim3(256), 0, s, (const uint64_t*)c->d_bsk,
                           c->d_bsk8, polys, (int)c->p.N);
    return hip_check(c, hipGetLastError(), "launch bsk_limbs");
}

extern "C" int tfhe_ctx_create(const tfhe_params* p, const void* bsk, size_t bsk_bytes, const void* ksk,
                               size_t ksk_bytes, int keys_on_device, tfhe_ctx** out) {
    if (!out) return TFHE_EINVAL;
    *out = nullptr;
    std::string why;
    if (!valid_params(p, &why)) return TFHE_EINVAL;
    if (!bsk || !ksk) return TFHE_EINVAL;
    tfhe_ctx* c = new tfhe_ctx();
    c->p = *p;
    c->q = (int)p->torus_bits;
    const size_t wb = word_bytes(c);
    if (bsk_bytes != tfhe_bsk_words(p) * wb || ksk_bytes != tfhe_ksk_words(p) * wb) {
        delete c;
        return TFHE_ESHAPE;
    }
    int dev = 0;
    hipGetDevice(&dev);
    c->device = dev;
    hipGetDeviceProperties(&c->prop, dev);
    const int NL = c->q == 32 ? 4 : 8;
    const size_t polys = (size_t)p->n * (p->k + 1) * p->l * (p->k + 1);
    int rc = TFHE_OK;
    const hipMemcpyKind kind = keys_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    // KSK rows start on 128-byte lines, so that a key-switch workgroup's
    // 16-word slice of a row touches whole lines of its own
    c->ks_row = ((p->n + 1) * wb + 127) / 128 * 128 / wb;
    const size_t ks_rows = (size_t)p->k * p->N * p->ks_t * ((size_t)1 << p->ks_base_bits);
    if ((rc = hip_check(c, hipMalloc(&c->d_bsk, bsk_bytes), "hipMalloc bsk")) ||
        (rc = hip_check(c, hipMalloc(&c->d_ksk, ks_rows * c->ks_row * wb), "hipMalloc ksk")) ||
        (rc = hip_check(c, hipMalloc((void**)&c->d_bsk8, polys * NL * 2 * p->N), "hipMalloc bsk8")) ||
        (rc = hip_check(c, hipMalloc(&c->d_gate_tv, p->N * wb), "hipMalloc testv")) ||
        (rc = hip_check(c, hipMalloc(&c->d_false, (p->n + 1) * wb), "hipMalloc false")) ||
        (rc = hip_check(c, hipMemcpy(c->d_bsk, bsk, bsk_bytes, kind), "copy bsk")) ||
        (rc = hip_check(c, hipMemset(c->d_ksk, 0, ks_rows * c->ks_row * wb), "clear ksk")) ||
        (rc = hip_check(c, hipMemcpy2D(c->d_ksk, c->ks_row * wb, ksk, (p->n + 1) * wb, (p->n + 1) * wb, ks_rows, kind),
                        "copy ksk"))) {
        tfhe_ctx_destroy(c);
        return rc;
    }
    if ((rc = launch_bsk_limbs(c, 0))) { tfhe_ctx_destroy(c); return rc; }
    if (c->q == 32) {
        // the MFMA key switch's limb table (4 bytes per word: 84 MB at the
        // standard set); without room the key switch reads the word table
        c->ks_wp = (int)((p->n + 1 + 15) / 16 * 16);
        const size_t K = ks_rows;
        if (hipMalloc((void**)&c->d_ksk8, 4 * (size_t)c->ks_wp * K) != hipSuccess) {
            (void)hipGetLastError();
            c->d_ksk8 = nullptr;
        } else {
            c->ksk8_bytes = 4 * (size_t)c->ks_wp * K;
            hipLaunchKernelGGL(ksk_limbs_kernel, dim3(4096), dim3(256), 0, 0, (const uint32_t*)c->d_ksk, c->d_ksk8,
                               c->ks_row, (int)p->n, c->ks_wp, K);
            if ((rc = hip_check(c, hipGetLastError(), "launch ksk_limbs"))) { tfhe_ctx_destroy(c); return rc; }
        }
    }
    if (c->q == 32 && p->N == 1024) {
        // the windowed-key blind rotation's fragments (16 bytes per byte of
        // bsk8: 968 MB at n = 630, l = 3); without room for them the kernel
        // stages the key in LDS instead
        const size_t rows = polys * NL;
        c->win_bytes = rows * 2 * p->N * 16;
        if (hipMalloc(&c->d_win, c->win_bytes) != hipSuccess) {
            (void)hipGetLastError();
            c->d_win = nullptr;
            c->win_bytes = 0;
        } else {
            hipLaunchKernelGGL(key_windows_kernel, dim3(4096), dim3(256), 0, 0, (const int8_t*)c->d_bsk8,
                               (uint4*)c->d_win, rows, 2 * (int)p->N);
            if ((rc = hip_check(c, hipGetLastError(), "launch key_windows"))) { tfhe_ctx_destroy(c); return rc; }
        }
    }
    if (c->q == 32)
        hipLaunchKernelGGL(fill_kernel<uint32_t>, dim3(8), dim3(256), 0, 0, (uint32_t*)c->d_gate_tv, (size_t)p->N,
                           (uint32_t)1u << 29);
    else
        hipLaunchKernelGGL(fill_kernel<uint64_t>, dim3(8), dim3(256), 0, 0, (uint64_t*)c->d_gate_tv, (size_t)p->N,
                           (uint64_t)1ull << 61);
    {
        std::vector<uint8_t> f((p->n + 1) * wb, 0);
        if (c->q == 32) ((uint32_t*)f.data())[p->n] = (uint32_t)(0u - (1u << 29));
        else ((uint64_t*)f.data())[p->n] = (uint64_t)(0ull - (1ull << 61));
        if ((rc = hip_check(c, hipMemcpy(c->d_false, f.data(), f.size(), hipMemcpyHostToDevice), "copy false"))) {
            tfhe_ctx_destroy(c);
            return rc;
        }
    }
    if ((rc = hip_check(c, hipDeviceSynchronize(), "context setup"))) { tfhe_ctx_destroy(c); return rc; }
    *out = c;
    return TFHE_OK;
}

extern "C" void tfhe_ctx_destroy(tfhe_ctx* c) {
    if (!c) return;
    hipDeviceSynchronize();
    timing_drain(c);
    for (auto e : c->event_pool) hipEventDestroy(e);
    graphs_clear(c);
    for (auto& h : c->stages) {
        if (h.p) hipHostFree(h.p);
        if (h.ev) hipEventDestroy(h.ev);
    }
    if (c->ws_event) hipEventDestroy(c->ws_event);
    if (c->d_bsk) hipFree(c->d_bsk);
    if (c->d_bsk8) hipFree(c->d_bsk8);
    if (c->d_win) hipFree(c->d_win);
    if (c->d_ksk) hipFree(c->d_ksk);
    if (c->d_ksk8) hipFree(c->d_ksk8);
    if (c->d_gate_tv) hipFree(c->d_gate_tv);
    if (c->d_false) hipFree(c->d_false);
    if (c->d_radix_tv) hipFree(c->d_radix_tv);
    if (c->ws) hipFree(c->ws);
    delete c;
}

extern "C" const char* tfhe_last_error(const tfhe_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" int tfhe_set_kernel(tfhe_ctx* c, int kind) {
    if (!c) return TFHE_EINVAL;
    if (kind != TFHE_KERNEL_MFMA && kind != TFHE_KERNEL_PLAIN) return ctx_fail(c, TFHE_EINVAL, "unknown kernel kind");
    c->kernel = kind;
    return TFHE_OK;
}

bool mfma_row_pass_supported(const tfhe_ctx* c, int rp);

extern "C" int tfhe_set_tuning(tfhe_ctx* c, int key, int64_t value) {
    if (!c) return TFHE_EINVAL;
    if (key == TFHE_TUNE_MAX_BATCH) {
        if (value < 16 || value > (1 << 22)) return ctx_fail(c, TFHE_EINVAL, "max batch must be in [16, 2^22]");
        c->max_batch = (uint32_t)value;
        return TFHE_OK;
    }
    if (key == TFHE_TUNE_DIGIT_BLOCKS) {
        if (value < 0 || value > 4) return ctx_fail(c, TFHE_EINVAL, "digit blocks must be 0, 1, 2, 3 or 4");
        c->digit_blocks = (int)value;
        return TFHE_OK;
    }
    if (key == TFHE_TUNE_SPLIT_GROUPS) {
        if (value < -1 || value > (1 << 20)) return ctx_fail(c, TFHE_EINVAL, "split groups must be in [-1, 2^20]");
        c->split_groups = value;
        return TFHE_OK;
    }
    if (key == TFHE_TUNE_ROW_PASS) {
        if (value != 0 && !mfma_row_pass_supported(c, (int)value))
            return ctx_fail(c, TFHE_EINVAL, "row tiles per pass not instantiated for this N");
        c->row_pass = (int)value;
        return TFHE_OK;
    }
    return ctx_fail(c, TFHE_EINVAL, "unknown tuning key");
}

extern "C" int tfhe_get_tuning(tfhe_ctx* c, int key, int64_t* value) {
    if (!c || !value) return TFHE_EINVAL;
    switch (key) {
        case TFHE_TUNE_MAX_BATCH: *value = c->max_batch; return TFHE_OK;
        case TFHE_TUNE_ROW_PASS: *value = c->row_pass; return TFHE_OK;
        case TFHE_TUNE_DIGIT_BLOCKS: *value = c->digit_blocks; return TFHE_OK;
        case TFHE_TUNE_SPLIT_GROUPS: *value = c->split_groups; return TFHE_OK;
    }
    return ctx_fail(c, TFHE_EINVAL, "unknown tuning key");
}

extern "C" int tfhe_ctx_sync(tfhe_ctx* c, void* stream) {
    if (!c) return TFHE_EINVAL;
    return hip_check(c, hipStreamSynchronize((hipStream_t)stream), "stream synchronize");
}

// ---------------------------------------------------------------- timing

static hipEvent_t pool_get(tfhe_ctx* c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

TimedLaunch::TimedLaunch(tfhe_ctx* cc, hipStream_t ss, int k, uint32_t n) : c(cc), s(ss), kind(k), cts(n) {
    if (!c->timing || capturing(s)) return;
    a = pool_get(c);
    b = pool_get(c);
    if (a && b) hipEventRecord(a, s);
}

TimedLaunch::~TimedLaunch() {
    if (!a || !b) return;
    hipEventRecord(b, s);
    c->timed.push_back(tfhe_ctx::Timed{a, b, kind, cts});
}

static int timing_drain(tfhe_ctx* c) {
    for (auto& t : c->timed) {
        float ms = 0;
        hipError_t e = hipEventSynchronize(t.b);
        if (e != hipSuccess) return hip_check(c, e, "timing event");
        hipEventElapsedTime(&ms, t.a, t.b);
        c->t_launch[t.kind]++;
        c->t_ms[t.kind] += ms;
        c->t_cts[t.kind] += t.cts;
        if (c->t_log.size() < (1u << 22)) c->t_log.push_back(((uint64_t)t.kind << 32) | t.cts);
        c->event_pool.push_back(t.a);
        c->event_pool.push_back(t.b);
    }
    c->timed.clear();
    return TFHE_OK;
}

extern "C" int tfhe_timing_enable(tfhe_ctx* c, int on) {
    if (!c) return TFHE_EINVAL;
    int rc = timing_drain(c);
    if (rc) return rc;
    c->timing = on != 0;
    for (int k = 0; k < 2; k++) { c->t_launch[k] = 0; c->t_ms[k] = 0; c->t_cts[k] = 0; }
    c->t_log.clear();
    return TFHE_OK;
}

extern "C" int tfhe_timing_log(tfhe_ctx* c, uint32_t* kinds, uint32_t* sizes, uint64_t max, uint64_t* count) {
    if (!c) return TFHE_EINVAL;
    int rc = timing_drain(c);
    if (rc) return rc;
    const uint64_t n = c->t_log.size();
    if (count) *count = n;
    for (uint64_t i = 0; i < n && i < max; i++) {
        if (kinds) kinds[i] = (uint32_t)(c->t_log[i] >> 32);
        if (sizes) sizes[i] = (uint32_t)c->t_log[i];
    }
    return TFHE_OK;
}

extern "C" int tfhe_timing_read(tfhe_ctx* c, int kind, uint64_t* launches, double* total_ms, uint64_t* cts) {
    if (!c || kind < 0 || kind > 1) return TFHE_EINVAL;
    int rc = timing_drain(c);
    if (rc) return rc;
    if (launches) *launches = c->t_launch[kind];
    if (total_ms) *total_ms = c->t_ms[kind];
    if (cts) *cts = c->t_cts[kind];
    return TFHE_OK;
}

size_t blind_rotate_ws_bytes(const tfhe_ctx* c, uint32_t B) {
    return c->kernel == TFHE_KERNEL_MFMA ? mfma_ws_bytes(c, B) : 0;
}

size_t blind_rotate_ws_bytes_upto(const tfhe_ctx* c, uint32_t Bmax) {
    return c->kernel == TFHE_KERNEL_MFMA ? mfma_ws_bytes_upto(c, Bmax) : 0;
}

int launch_blind_rotate(tfhe_ctx* c, const void* lwe_in, const void* testv_table, const int32_t* tv_index,
                        void* big_out, uint32_t B, void* ws, size_t ws_cap, hipStream_t s) {
    if (B == 0) return TFHE_OK;
    const void* tv = testv_table ? testv_table : c->d_gate_tv;
    TimedLaunch tl(c, s, 0, B);
    if (c->kernel == TFHE_KERNEL_PLAIN) return launch_br_plain(c, lwe_in, tv, tv_index, big_out, B, s);
    return launch_br_mfma(c, lwe_in, tv, tv_index, big_out, B, ws, ws_cap, s);
}

extern "C" int tfhe_bootstrap_batch(tfhe_ctx* c, const void* d_lwe_in, const void* d_testv, void* d_out,
                                    uint32_t B, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (B == 0) return TFHE_OK;
    if (!d_lwe_in || !d_out) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    hipStream_t s = (hipStream_t)stream;
    const size_t need = blind_rotate_ws_bytes(c, B);
    if (!need) return launch_blind_rotate(c, d_lwe_in, d_testv, nullptr, d_out, B, nullptr, 0, s);
    int rc = ws_acquire(c, s, need);
    if (rc) return rc;
    rc = launch_blind_rotate(c, d_lwe_in, d_testv, nullptr, d_out, B, c->ws, c->ws_bytes, s);
    const int rr = ws_release(c, s);
    return rc ? rc : rr;
}

extern "C" int tfhe_graph_stats(tfhe_ctx* c, uint64_t* captures, uint64_t* launches, uint64_t* cached) {
    if (!c) return TFHE_EINVAL;
    if (captures) *captures = c->graph_captures;
    if (launches) *launches = c->graph_launches;
    if (cached) *cached = c->graphs.size();
    return TFHE_OK;
}

extern "C" int tfhe_keyswitch_batch(tfhe_ctx* c, const void* d_in, void* d_out, uint32_t B, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (B == 0) return TFHE_OK;
    if (!d_in || !d_out) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    hipStream_t s = (hipStream_t)stream;
    int rc = ws_acquire(c, s, ks_digits_bytes(c, B));
    if (rc) return rc;
    rc = launch_keyswitch(c, d_in, d_out, nullptr, B, c->ws, c->ws_bytes, s);
    const int rr = ws_release(c, s);
    return rc ? rc : rr;
}

// ------------------------------------------------------- seeded streams

namespace {
enum { TAG_LWE_KEY = 1, TAG_GLWE_KEY = 2, TAG_BSK_MASK = 3, TAG_BSK_NOISE = 4, TAG_KSK_MASK = 5, TAG_KSK_NOISE = 6 };

__global__ void rng_fill_kernel(uint64_t K, uint64_t start, uint64_t count, uint64_t* out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = stream_at(K, start + i);
}

template <typename T>
__global__ void key_bits_kernel(uint64_t K, T* out, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        out[i] = (T)(stream_at(K, i) >> 63);
}

// GGSW rows of BSK_i = GGSW_S(s_i): row r = u*l + (p-1) is a GLWE encryption
// of zero (A = mask stream, B = A*S + e) plus s_i 2^{q - p*bg} at coefficient 0
// of component u.  Pass 1 writes masks, pass 2 bodies and the gadget term.
template <typename T>
__global__ void bsk_mask_kernel(uint64_t K, T* bsk, size_t rows_total, int N) {
    // k = 1: component 0 of each row is the mask
    const size_t total = rows_total * N;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const size_t row = idx / N;
        const int j = (int)(idx % N);
        bsk[row * 2 * N + j] = stream_torus<T>(K, idx);
    }
}

template <typename T>
__global__ void bsk_body_kernel(uint64_t Kn, T* bsk, const T* S, const T* s, size_t rows_total, int N, int l,
                                int bgb, int sigma) {
    constexpr int Q = Torus<T>::Q;
    const size_t total = rows_total * N;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const size_t row = idx / N;
        const int j = (int)(idx % N);
        const T* A = bsk + row * 2 * N;
        // (A * S)[j] = sum_{x<=j} A[x] S[j-x] - sum_{x>j} A[x] S[N+j-x]
        T acc = stream_noise<T>(Kn, idx, sigma);
        for (int x = 0; x <= j; x++) acc += S[j - x] ? A[x] : (T)0;
        for (int x = j + 1; x < N; x++) acc -= S[N + j - x] ? A[x] : (T)0;
        bsk[row * 2 * N + N + j] = acc;
    }
}

template <typename T>
__global__ void bsk_gadget_kernel(T* bsk, const T* s, int n, int l, int N, int bgb) {
    constexpr int Q = Torus<T>::Q;
    const int total = n * 2 * l;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int i = idx / (2 * l), r = idx % (2 * l);
        const int u = r / l, p = r % l + 1;
        const int e = Q - p * bgb;
        const T g = e >= Q ? (T)0 : (T)((T)1 << e);
        // component u of row r, coefficient 0 (added after the body was formed)
        bsk[((size_t)i * 2 * l + r) * 2 * N + (size_t)u * N] += s[i] * g;
    }
}

// KSK[i][j][v] = LWE_s(v s'_i 2^{q-(j+1)b}); every entry is a fresh encryption.
template <typename T>
__global__ void ksk_kernel(uint64_t Km, uint64_t Kn, T* ksk, const T* sx, const T* s, int kN, int t, int bb, int n,
                           int sigma) {
    constexpr int Q = Torus<T>::Q;
    const int V = 1 << bb;
    const size_t total = (size_t)kN * t * V;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int v = (int)(e % V);
        const int j = (int)((e / V) % t);
        const size_t i = e / ((size_t)V * t);
        T* row = ksk + e * (n + 1);
        const int sh = Q - (j + 1) * bb;
        T mu = sh >= 0 && sh < Q ? (T)((T)v * sx[i] << sh) : (T)0;
        T b = stream_noise<T>(Kn, e, sigma) + mu;
        for (int w = 0; w < n; w++) {
            T a = stream_torus<T>(Km, e * n + w);
            row[w] = a;
            b += a * s[w];
        }
        row[n] = b;
    }
}

template <typename T>
__global__ void lwe_encrypt_kernel(uint64_t Km, uint64_t Kn, int sigma, uint64_t start, const T* key, const T* mu,
                                   T* out, uint64_t count, int dim) {
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < count; c += (uint64_t)gridDim.x * blockDim.x) {
        T* ct = out + c * (dim + 1);
        T b = stream_noise<T>(Kn, start + c, sigma) + mu[c];
        const uint64_t base = (start + c) * dim;
        for (int w = 0; w < dim; w++) {
            T a = stream_torus<T>(Km, base + w);
            ct[w] = a;
            b += a * key[w];
        }
        ct[dim] = b;
    }
}

// One wave per ciphertext: phase = b - <a, key>.
template <typename T>
__global__ void lwe_phase_kernel(const T* key, const T* cts, T* out, uint64_t count, int dim) {
    const uint64_t c = blockIdx.x * 4ull + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= count) return;
    const T* ct = cts + c * (dim + 1);
    T acc = 0;
    for (int w = lane; w < dim; w += 64) acc += ct[w] * key[w];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) out[c] = ct[dim] - acc;
}
}  // namespace

extern "C" int tfhe_rng_fill(uint64_t seed, uint64_t tag, uint64_t start, uint64_t count, void* d_out, void* stream) {
    if (!d_out && count) return TFHE_EINVAL;
    if (!count) return TFHE_OK;
    hipLaunchKernelGGL(rng_fill_kernel, dim3(1024), dim3(256), 0, (hipStream_t)stream, stream_key(seed, tag), start,
                       count, (uint64_t*)d_out);
    return hipGetLastError() == hipSuccess ? TFHE_OK : TFHE_EHIP;
}

template <typename T>
static int keygen_t(const tfhe_params* p, uint64_t seed, int ls, int gs, T* s, T* S, T* bsk, T* ksk, hipStream_t st) {
    const int n = p->n, N = p->N, l = p->l;
    hipLaunchKernelGGL(key_bits_kernel<T>, dim3(64), dim3(256), 0, st, stream_key(seed, TAG_LWE_KEY), s, n);
    hipLaunchKernelGGL(key_bits_kernel<T>, dim3(64), dim3(256), 0, st, stream_key(seed, TAG_GLWE_KEY), S, N);
    const size_t rows = (size_t)n * 2 * l;
    hipLaunchKernelGGL(bsk_mask_kernel<T>, dim3(2048), dim3(256), 0, st, stream_key(seed, TAG_BSK_MASK), bsk, rows, N);
    hipLaunchKernelGGL(bsk_body_kernel<T>, dim3(4096), dim3(256), 0, st, stream_key(seed, TAG_BSK_NOISE), bsk,
                       (const T*)S, (const T*)s, rows, N, l, (int)p->bg_bits, gs);
    hipLaunchKernelGGL(bsk_gadget_kernel<T>, dim3(64), dim3(256), 0, st, bsk, (const T*)s, n, l, N, (int)p->bg_bits);
    hipLaunchKernelGGL(ksk_kernel<T>, dim3(4096), dim3(64), 0, st, stream_key(seed, TAG_KSK_MASK),
                       stream_key(seed, TAG_KSK_NOISE), ksk, (const T*)S, (const T*)s, (int)(p->k * N), (int)p->ks_t,
                       (int)p->ks_base_bits, n, ls);
    return hipGetLastError() == hipSuccess ? TFHE_OK : TFHE_EHIP;
}

extern "C" int tfhe_keygen(const tfhe_params* p, uint64_t seed, uint32_t lwe_sigma_log2, uint32_t glwe_sigma_log2,
                           void* d_lwe_key, void* d_glwe_key, void* d_bsk, void* d_ksk, void* stream) {
    if (!valid_params(p, nullptr) || !d_lwe_key || !d_glwe_key || !d_bsk || !d_ksk) return TFHE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (p->torus_bits == 32)
        return keygen_t<uint32_t>(p, seed, lwe_sigma_log2, glwe_sigma_log2, (uint32_t*)d_lwe_key,
                                  (uint32_t*)d_glwe_key, (uint32_t*)d_bsk, (uint32_t*)d_ksk, st);
    return keygen_t<uint64_t>(p, seed, lwe_sigma_log2, glwe_sigma_log2, (uint64_t*)d_lwe_key, (uint64_t*)d_glwe_key,
                              (uint64_t*)d_bsk, (uint64_t*)d_ksk, st);
}

extern "C" int tfhe_lwe_encrypt(const tfhe_params* p, uint64_t seed, uint64_t mask_tag, uint64_t noise_tag,
                                uint32_t sigma_log2, uint64_t start, const void* d_key, const void* d_mu, void* d_out,
                                uint64_t count, uint32_t dim, void* stream) {
    if (!p || (p->torus_bits != 32 && p->torus_bits != 64) || !d_key || !d_mu || !d_out) return TFHE_EINVAL;
    if (!count) return TFHE_OK;
    hipStream_t st = (hipStream_t)stream;
    const uint64_t Km = stream_key(seed, mask_tag), Kn = stream_key(seed, noise_tag);
    if (p->torus_bits == 32)
        hipLaunchKernelGGL(lwe_encrypt_kernel<uint32_t>, dim3(2048), dim3(128), 0, st, Km, Kn, (int)sigma_log2, start,
                           (const uint32_t*)d_key, (const uint32_t*)d_mu, (uint32_t*)d_out, count, (int)dim);
    else
        hipLaunchKernelGGL(lwe_encrypt_kernel<uint64_t>, dim3(2048), dim3(128), 0, st, Km, Kn, (int)sigma_log2, start,
                           (const uint64_t*)d_key, (const uint64_t*)d_mu, (uint64_t*)d_out, count, (int)dim);
    return hipGetLastError() == hipSuccess ? TFHE_OK : TFHE_EHIP;
}

extern "C" int tfhe_lwe_phase(const tfhe_params* p, const void* d_key, const void* d_cts, void* d_out, uint64_t count,
                              uint32_t dim, void* stream) {
    if (!p || (p->torus_bits != 32 && p->torus_bits != 64) || !d_key || !d_cts || !d_out) return TFHE_EINVAL;
    if (!count) return TFHE_OK;
    hipStream_t st = (hipStream_t)stream;
    const unsigned grid = (unsigned)((count + 3) / 4);
    if (p->torus_bits == 32)
        hipLaunchKernelGGL(lwe_phase_kernel<uint32_t>, dim3(grid), dim3(256), 0, st, (const uint32_t*)d_key,
                           (const uint32_t*)d_cts, (uint32_t*)d_out, count, (int)dim);
    else
        hipLaunchKernelGGL(lwe_phase_kernel<uint64_t>, dim3(grid), dim3(256), 0, st, (const uint64_t*)d_key,
                           (const uint64_t*)d_cts, (uint64_t*)d_out, count, (int)dim);
    return hipGetLastError() == hipSuccess ? TFHE_OK : TFHE_EHIP;
}
