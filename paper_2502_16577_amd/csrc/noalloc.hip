// perm_dense_f64_noalloc: the dense real permanent for callers that cannot
// allocate device memory (code under graph capture, serving loops, harnesses
// that forbid hipMalloc).  The workspace of perm_dense_f64 (column copies,
// start vector, block partials) lives in a fixed array in the library's
// device memory, one copy per GPU, instead of a caller-provided buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "perm.h"
#include "perm_internal.h"

namespace {

// 256 KiB holds perm_dense_f64's workspace for every n <= 53 (the block
// partials grow with the lane count above n = 50).
constexpr size_t kScratchBytes = size_t(256) << 10;
constexpr int kMaxDevices = 64;

// The array itself.  In host code its name only stands in for the symbol:
// the device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is ever passed to kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (looked up on the first
// call on the device, with it current).
int scratch_for_current_device(void **ptr)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PERM_EHIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PERM_EHIP;
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    return PERM_OK;
}

}  // namespace

extern "C" {

size_t perm_noalloc_scratch_bytes(void) { return kScratchBytes; }

int perm_dense_f64_noalloc(int n, const double *A, int64_t lda, double *out, void *stream)
{
    if (n < 0 || n > PERM_MAX_N || !out) return PERM_EINVAL;
    if (n > 0 && (!A || lda < n)) return PERM_EINVAL;
    const size_t need = perm_workspace_bytes(PERM_KIND_DENSE_F64, n, 0);
    if (need > kScratchBytes) return PERM_ESCRATCH;
    void *ws = nullptr;
    const int rc = scratch_for_current_device(&ws);
    if (rc != PERM_OK) return rc;
    // every launch of the sweep stores its block partials before the
    // finalize reads them, so nothing in the array has to start at zero
    return perm_dense_f64(n, A, lda, out, ws, kScratchBytes, stream);
}

}  // extern "C"
