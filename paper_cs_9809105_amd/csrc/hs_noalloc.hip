// hs_noalloc.hip -- hs_gemm_noalloc: C = A . B through the same kernels as
// hs_gemm, with the workspace (the packed operands) taken from a scratch
// array that the library's code object holds on every device, so that the
// call needs no device allocation by anyone (for callers that cannot
// allocate: code under stream capture, tight serving loops).
//
// The array `scratch` below is a device symbol.  Its name in host code is
// only a host-side stand-in, never a device address: the device address is
// looked up once per device with hipGetSymbolAddress, on that device's first
// call, and only that address is handed to kernels.  Each device holds its
// own copy of the array for the life of the process.  All calls on one
// device share that copy: calls that overlap in time on one device (two
// streams, two threads) race on it and must be ordered by the caller.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hs.h"

namespace {

const int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[HS_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device), or nullptr if the runtime cannot give it.
void *scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" hs_status hs_gemm_noalloc(int64_t m, int64_t n, int64_t k, int dtype, hs_schedule s,
                                     const void *A, int64_t lda, const void *B, int64_t ldb,
                                     void *C, int64_t ldc, void *stream) {
    // hs_gemm's own argument checks first: with no workspace it returns
    // HS_ERR_WORKSPACE_TOO_SMALL, before any launch, exactly when the
    // arguments are valid and a workspace is needed; any other status
    // (an error, or HS_OK for a call that needs no workspace) is final
    const hs_status st = hs_gemm(m, n, k, dtype, s, A, lda, B, ldb, C, ldc, nullptr, 0, stream);
    if (st != HS_ERR_WORKSPACE_TOO_SMALL) return st;
    const size_t need = hs_workspace_size(HS_OP_GEMM, m, n, k, dtype, s);
    if (need > (size_t)HS_NOALLOC_SCRATCH_BYTES) return HS_ERR_EXCEEDS_SCRATCH;
    void *ws = scratch_on_current_device();
    if (!ws) return HS_ERR_LAUNCH_FAILED;
    // every byte of the workspace that the kernels read is written first by
    // the same call (packed operands, padding and FP8 exponents included),
    // so nothing left by an earlier call needs clearing
    return hs_gemm(m, n, k, dtype, s, A, lda, B, ldb, C, ldc, ws, (size_t)HS_NOALLOC_SCRATCH_BYTES, stream);
}
