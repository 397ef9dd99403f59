// Blind rotation + sample extraction without any device allocation, for
// callers that cannot allocate (code under HIP graph capture, serving loops
// or harnesses that forbid hipMalloc): the blind-rotation workspace is a
// file-scope device array instead of the context's allocated workspace.
#include <cstdio>
#include <mutex>

#include "fhesql_internal.h"

int launch_br_mfma(tfhe_ctx* c, const void* lwe_in, const void* tv, const int32_t* tv_index,
                   void* big_out, uint32_t B, void* ws, size_t ws_cap, hipStream_t s);
int launch_br_plain(tfhe_ctx* c, const void* lwe_in, const void* tv, const int32_t* tv_index,
                    void* big_out, uint32_t B, hipStream_t s);

namespace {

// One copy per device, held by each device the library runs on until the
// process ends.  On the host the array's name is only a stand-in: the device
// address of each device's copy comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is passed to
// kernels.  No kernel needs the scratch cleared: the blind rotation writes
// every accumulator word it reads (its prologue) and the digit cache is
// written by a step's first row pass before the later passes read it.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

// This device's scratch address (taken on its first call), or null.
void* scratch_address(tfhe_ctx* c, int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            hip_check(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" size_t tfhe_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int tfhe_bootstrap_batch_noalloc(tfhe_ctx* c, const void* d_lwe_in, const void* d_testv, void* d_out,
                                            uint32_t B, void* stream) {
    if (!c) return TFHE_EINVAL;
    if (B == 0) return TFHE_OK;
    if (!d_lwe_in || !d_out) return ctx_fail(c, TFHE_EINVAL, "null ciphertext pointer");
    int dev = -1;
    int rc = hip_check(c, hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev != c->device || dev < 0 || dev >= kMaxDevices)
        return ctx_fail(c, TFHE_EINVAL, "the context's device must be the current device");
    const size_t need = blind_rotate_ws_bytes(c, B);
    if (need > kScratchBytes) {
        char msg[160];
        snprintf(msg, sizeof msg, "a batch of %u needs %zu bytes of scratch, more than the %zu-byte static array", B,
                 need, kScratchBytes);
        return ctx_fail(c, TFHE_ESHAPE, msg);
    }
    void* ptr = scratch_address(c, dev);
    if (!ptr) return TFHE_EHIP;
    // no timing events: creating them could allocate
    const void* tv = d_testv ? d_testv : c->d_gate_tv;
    hipStream_t s = (hipStream_t)stream;
    if (c->kernel == TFHE_KERNEL_PLAIN) return launch_br_plain(c, d_lwe_in, tv, nullptr, d_out, B, s);
    return launch_br_mfma(c, d_lwe_in, tv, nullptr, d_out, B, ptr, kScratchBytes, s);
}
