// Device-side descriptors of a batched launch (shared by the host planner and
// the batched kernels).
#pragma once

#include "perm_internal.h"

namespace perm {

constexpr int kBatchMaxK = 32;
constexpr int kBatchThreads = kGradSlices * kWave;  // one grad_item per block

// Staged rows per column of an order-k matrix (grad_item's padding).
__host__ __device__ inline int batch_rows(int k) { return grad_rows(k); }

// One matrix of the batch.
struct BatchMatDev {
    int32_t k;         // order
    int32_t c;         // log2 of the Gray steps per lane
    int32_t r;         // log2 of the exact re-seed interval (r <= c - 1)
    int32_t waves;     // items (64 subsets each) covering its 2^(k-1) steps
    int64_t data_off;  // element offset of the matrix in the packed data (and grad)
    int64_t stage;     // double offset of its staged column copies
    int64_t item0;     // index of its first item among all items (matrix-major)
    int64_t gbase;     // dd offset of its first item's gradient partial
};

// One work item: subsets 64 w .. 64 w + 63 of matrix m.
struct BatchItemDev {
    int32_t m;
    int32_t w;
};

// Orders are split into groups with their own persistent kernel (each
// kernel's register allocation covers only its own orders):
// group 0: k <= 16 (one 16x16 MFMA tile), 1: 17..24, 2: 25..32.
constexpr int kBatchGroups = 3;
inline int batch_group(int k) { return k <= 16 ? 0 : (k <= 24 ? 1 : 2); }

struct BatchLaunch {
    int64_t count = 0;
    const BatchMatDev *mats = nullptr;
    const BatchItemDev *items[kBatchGroups] = {nullptr, nullptr, nullptr};  // execution order
    int64_t n_items[kBatchGroups] = {0, 0, 0};
    int64_t grid[kBatchGroups] = {0, 0, 0};
    uint32_t *counters = nullptr;               // one work counter per group
    double *stage = nullptr;
    dd *perm_parts = nullptr;
    dd *g_parts = nullptr;
    const double *data = nullptr;  // packed matrices: (re, im) pairs, or reals if `real`
    double *out = nullptr;
    double *grad = nullptr;
    int want_grad = 0;
    int real = 0;
};

// Enqueues reset, staging, the persistent kernels (largest orders first) and
// the finalize on `stream`.
int launch_batched(const BatchLaunch &L, hipStream_t stream);
// The same with the persistent kernels of the groups on `side` streams
// (fork / join through events) so they run concurrently; used under graph
// capture.  side[g] may equal stream.
int launch_batched_forked(const BatchLaunch &L, hipStream_t stream,
                          const hipStream_t side[kBatchGroups], hipEvent_t fork,
                          const hipEvent_t join[kBatchGroups]);

// out = sum_m wts[m] * perms[m] (double-double, fixed order); perms and out
// are complex (re, im) pairs, or reals if `real`.
int launch_weighted_sum(int count, const double *wts, const double *perms, double *out, bool real,
                        hipStream_t stream);

}  // namespace perm
