// C ABI of libperm_mi355x.so: argument validation, workspace sizing, launch
// planning and dispatch to the HIP kernels.  Every check happens before any
// GPU work is queued; no function here allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "perm.h"
#include "perm_internal.h"

namespace perm {

// Lanes x chunk = 2^(n-1) exactly (Section 3.2: with power-of-two chunks every
// lane of a wave flips the same column at the same local step, and no
// remainder kernel is needed).  About 2^18 lanes fill the 256 CUs with four
// waves per SIMD; smaller problems use fewer lanes but at least one block and
// at least 64 steps per lane where the problem allows it.
SweepPlan plan_sweep(int n, int /*steps_per_op_hint*/)
{
    SweepPlan p;
    p.n = n;
    if (n <= 12) {
        p.log2_chunk = n > 0 ? n - 1 : 0;
        p.log2_reseed = p.log2_chunk;
        p.lanes = 1;
        p.blocks = 1;
        return p;
    }
    const int total = n - 1;                 // log2 of the number of steps
    const int cmin = std::min(6, total - 8);  // keep >= 256 lanes (one block)
    const int c = std::max(cmin, total - 18);
    p.log2_chunk = c;
    p.log2_reseed = std::min(9, c);
    p.lanes = int64_t(1) << (total - c);
    p.blocks = p.lanes / kBlock;
    return p;
}

DenseWs dense_ws_layout(int n, int components, int64_t blocks)
{
    DenseWs L;
    size_t off = 0;
    const size_t nn = size_t(n) * size_t(n) * size_t(components) * sizeof(double);
    L.acol = off;
    off += align256(nn);
    L.aneg = off;
    off += align256(nn);
    L.x0 = off;
    off += align256(size_t(n) * size_t(components) * sizeof(double));
    L.partials = off;
    off += align256(size_t(std::max<int64_t>(blocks, 1)) * size_t(components) * sizeof(dd));
    L.total = off;
    return L;
}

}  // namespace perm

using namespace perm;

namespace {

bool valid_n(int n) { return n >= 0 && n <= PERM_MAX_N; }

int check_ws(const void *ws, size_t ws_bytes, size_t need)
{
    if (need == 0) return PERM_OK;
    if (!ws || ws_bytes < need) return PERM_EWORKSPACE;
    return PERM_OK;
}

}  // namespace

extern "C" {

const char *perm_strerror(int status)
{
    switch (status) {
    case PERM_OK: return "success";
    case PERM_EINVAL: return "invalid argument";
    case PERM_ERANGE: return "result exceeds the representable range";
    case PERM_EWORKSPACE: return "workspace missing or too small";
    case PERM_EHIP: return "HIP runtime error";
    case PERM_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

int perm_version(void) { return 100; }

size_t perm_workspace_bytes(int kind, int n, int64_t m)
{
    (void)m;
    if (!valid_n(n)) return 0;
    switch (kind) {
    case PERM_KIND_DENSE_F64: {
        const SweepPlan p = plan_sweep(n, 0);
        return dense_ws_layout(n, 1, p.blocks).total;
    }
    case PERM_KIND_DENSE_C128: {
        const SweepPlan p = plan_sweep(n, 0);
        return dense_ws_layout(n, 2, p.blocks).total;
    }
    default: return 0;
    }
}

int perm_dense_f64(int n, const double *A, int64_t lda, double *out, void *ws, size_t ws_bytes,
                   void *stream)
{
    if (!valid_n(n) || !out) return PERM_EINVAL;
    if (n > 0 && (!A || lda < n)) return PERM_EINVAL;
    const int w = check_ws(ws, ws_bytes, perm_workspace_bytes(PERM_KIND_DENSE_F64, n, 0));
    if (w != PERM_OK) return w;
    return launch_dense_f64(n, A, lda, out, static_cast<char *>(ws),
                            static_cast<hipStream_t>(stream));
}

int perm_dense_c128(int n, const perm_c128 *A, int64_t lda, perm_c128 *out, void *ws,
                    size_t ws_bytes, void *stream)
{
    if (!valid_n(n) || !out) return PERM_EINVAL;
    if (n > 0 && (!A || lda < n)) return PERM_EINVAL;
    const int w = check_ws(ws, ws_bytes, perm_workspace_bytes(PERM_KIND_DENSE_C128, n, 0));
    if (w != PERM_OK) return w;
    return launch_dense_c128(n, A, lda, out, static_cast<char *>(ws),
                             static_cast<hipStream_t>(stream));
}

int perm_sparse_f64(int, const int32_t *, const int32_t *, const double *, int32_t, double *,
                    void *, size_t, void *)
{
    return PERM_EUNSUPPORTED;
}

int perm_binary_exact(int, const int32_t *, const int32_t *, int32_t, int, uint64_t *, uint64_t *,
                      void *, size_t, void *)
{
    return PERM_EUNSUPPORTED;
}

uint64_t perm_binary_prime(int) { return 0; }

}  // extern "C"
