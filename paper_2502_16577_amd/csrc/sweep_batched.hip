// Batched permanents (and gradients) of many small complex or real matrices
// of uneven order in one persistent launch.
//
// The batch is cut into work items: item (m, w) covers subsets 64 w ..
// 64 w + 63 of matrix m, each walking 2^c Gray steps (subset K walks g in
// [K 2^c, (K+1) 2^c)).  A persistent grid of two-wave blocks (one item at a
// time, the waves splitting the rows) pulls items from an atomic counter,
// largest matrices first, and dispatches on the (block-uniform) order k to a
// sweep compiled for that k.  Each item writes
// its own double-double partials (permanent, and G if requested); a
// segmented finalize sums the items of every matrix in a fixed order, so the
// result does not depend on which wave ran which item.
//
// Per item the arithmetic is grad_item (grad_item.h), the same as for a
// single matrix: x in VGPRs, the flipped column read with scalar loads, an
// exact re-seed of x every 2^r steps, leave-one-out products, and the
// gradient contraction organised by Gray-code windows with FP64 MFMA.
#include "batched_internal.h"
#include "grad_item.h"

namespace perm {

// Stages every matrix in grad_item's layout: acol[W (j kp + i) + comp] with
// kp = batch_rows(k) rows per column (rows >= k zero), then x0[W i + comp]
// for i < kp (1 for rows >= k), at stage + mats[m].stage (doubles); W = 2
// (re, im) for complex matrices, 1 for real ones.  One block per matrix.
template <bool CPLX>
__global__ __launch_bounds__(kBlock) void batched_prep(const BatchMatDev *__restrict__ mats,
                                                       const double *__restrict__ data,
                                                       double *__restrict__ stage)
{
    constexpr int W = CPLX ? 2 : 1;
    const BatchMatDev M = mats[blockIdx.x];
    const int k = M.k;
    const int kp = batch_rows(k);
    const double *A = data + W * M.data_off;
    double *acol = stage + M.stage;
    double *x0 = acol + W * k * kp;
    for (int idx = threadIdx.x; idx < k * kp; idx += blockDim.x) {
        const int j = idx / kp, i = idx - j * kp;
#pragma unroll
        for (int q = 0; q < W; ++q) acol[W * idx + q] = i < k ? A[W * (i * k + j) + q] : 0.0;
    }
    for (int i = k + int(threadIdx.x); i < kp; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < W; ++q) x0[W * i + q] = q == 0 ? 1.0 : 0.0;
    }
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < W; ++q) {
            double s = 0.0, e = 0.0;  // compensated row sum
            for (int j = 0; j < k; ++j) acc_add(s, e, A[W * (i * k + j) + q]);
            x0[W * i + q] = (A[W * (i * k + k - 1) + q] - 0.5 * s) - 0.5 * e;
        }
    }
}

__global__ void batched_reset(uint32_t *counters, int n)
{
    if (int(threadIdx.x) < n) counters[threadIdx.x] = 0u;
}

template <int K, bool CPLX>
__device__ __forceinline__ void batched_item(const BatchMatDev &M, int w,
                                             const double *__restrict__ stage,
                                             dd *__restrict__ perm_out, dd *__restrict__ g_out,
                                             bool want_grad, double *__restrict__ lds)
{
    constexpr int W = CPLX ? 2 : 1;
    const double *acol = stage + M.stage;
    if constexpr (K == 1) {  // one subset: perm = a, G = [1]
        if ((threadIdx.x & 63u) == 0) {
            perm_out[0] = dd{0.5 * acol[0], 0.0};  // the finalize multiplies by 2
            perm_out[1] = dd{CPLX ? 0.5 * acol[1] : 0.0, 0.0};
            if (want_grad) {
                g_out[0] = dd{1.0, 0.0};
                if (CPLX) g_out[1] = dd{0.0, 0.0};
            }
        }
    } else {
        constexpr int KP = GradItemShape<K, CPLX>::NP;
        const double *x0 = acol + W * K * KP;
        const uint64_t lanes_active = (uint64_t(1) << (K - 1)) >> M.c;
        grad_item<K, CPLX>(acol, x0, uint64_t(w), M.c, M.r, lanes_active, perm_out, g_out,
                           want_grad, lds);
    }
}

template <int K0, int K1, bool CPLX>
struct BatchDispatch {
    __device__ __forceinline__ static void run(int k, const BatchMatDev &M, int w, const double *stage,
                                               dd *pp, dd *gp, bool want_grad, double *lds)
    {
        if (k == K0) batched_item<K0, CPLX>(M, w, stage, pp, gp, want_grad, lds);
        else if constexpr (K0 < K1)
            BatchDispatch<K0 + 1, K1, CPLX>::run(k, M, w, stage, pp, gp, want_grad, lds);
    }
};

// Persistent loop for the items of orders in [K0, K1]: blocks of
// kBatchThreads (the waves of one grad_item) take items from the counter.
template <int K0, int K1, bool CPLX>
__device__ __forceinline__ void persistent_items(
    const BatchMatDev *__restrict__ mats, const BatchItemDev *__restrict__ items, int64_t n_items,
    uint32_t *__restrict__ counter, const double *__restrict__ stage,
    dd *__restrict__ perm_parts, dd *__restrict__ g_parts, int want_grad, double *lds,
    uint32_t *next)
{
    constexpr int W = CPLX ? 2 : 1;
    for (;;) {
        if (threadIdx.x == 0) *next = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(*next);
        __syncthreads();  // every wave has read `next` before it is overwritten
        if (int64_t(it) >= n_items) break;
        const BatchItemDev I = items[it];
        const BatchMatDev M = mats[I.m];
        dd *pp = perm_parts + 2 * (M.item0 + I.w);
        dd *gp = g_parts + M.gbase + int64_t(I.w) * W * M.k * M.k;
        BatchDispatch<K0, K1, CPLX>::run(M.k, M, I.w, stage, pp, gp, want_grad != 0, lds);
    }
}

// Orders up to 24 fit two waves per SIMD (at most 256 registers per lane)
// without spilling; the compiler is held to that.
template <int K0, int K1, bool CPLX>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(2))) void
batched_persistent(const BatchMatDev *__restrict__ mats, const BatchItemDev *__restrict__ items,
                   int64_t n_items, uint32_t *__restrict__ counter,
                   const double *__restrict__ stage, dd *__restrict__ perm_parts,
                   dd *__restrict__ g_parts, int want_grad)
{
    static_assert(GradItemShape<K1, CPLX>::THREADS == kBatchThreads, "block shape");
    __shared__ double lds[GradItemShape<K1, CPLX>::LDS_DOUBLES];
    __shared__ uint32_t next;
    persistent_items<K0, K1, CPLX>(mats, items, n_items, counter, stage, perm_parts, g_parts,
                                   want_grad, lds, &next);
}

// Orders 25..32 need more registers: one wave per SIMD.
template <int K0, int K1, bool CPLX>
__global__ __launch_bounds__(kBatchThreads) void batched_persistent_large(
    const BatchMatDev *__restrict__ mats, const BatchItemDev *__restrict__ items, int64_t n_items,
    uint32_t *__restrict__ counter, const double *__restrict__ stage,
    dd *__restrict__ perm_parts, dd *__restrict__ g_parts, int want_grad)
{
    static_assert(GradItemShape<K1, CPLX>::THREADS == kBatchThreads, "block shape");
    __shared__ double lds[GradItemShape<K1, CPLX>::LDS_DOUBLES];
    __shared__ uint32_t next;
    persistent_items<K0, K1, CPLX>(mats, items, n_items, counter, stage, perm_parts, g_parts,
                                   want_grad, lds, &next);
}

// One block per matrix: perm[m] = 2 (-1)^(k-1) sum of item partials, and
// G[m] = (-1)^(k-1) sum of item G partials, in item order.  out holds W
// doubles per matrix and grad W doubles per entry, packed like the data.
template <bool CPLX>
__global__ __launch_bounds__(kBlock) void batched_finalize(const BatchMatDev *__restrict__ mats,
                                                           const dd *__restrict__ perm_parts,
                                                           const dd *__restrict__ g_parts,
                                                           double *__restrict__ out,
                                                           double *__restrict__ grad)
{
    constexpr int W = CPLX ? 2 : 1;
    __shared__ dd red[kWavesPerBlock];
    const BatchMatDev M = mats[blockIdx.x];
    const int k = M.k;
    const double sgn = (k & 1) ? 1.0 : -1.0;
    for (int q = 0; q < W; ++q) {
        dd acc = dd{0.0, 0.0};
        for (int w = threadIdx.x; w < M.waves; w += kBlock)
            acc = dd_add(acc, perm_parts[2 * (M.item0 + w) + q]);
        const dd t = block_reduce_dd(acc, red);
        if (threadIdx.x == 0) out[W * blockIdx.x + q] = 2.0 * sgn * (t.hi + t.lo);
    }
    if (!grad) return;
    double *gout = grad + W * M.data_off;
    for (int e = threadIdx.x; e < W * k * k; e += kBlock) {
        dd acc = dd{0.0, 0.0};
        for (int w = 0; w < M.waves; ++w)
            acc = dd_add(acc, g_parts[M.gbase + int64_t(w) * W * k * k + e]);
        gout[e] = sgn * (acc.hi + acc.lo);
    }
}

// sum_m w_m perm_m in double-double, fixed order, one block; perms and out
// hold W doubles per value (2: complex, 1: real).
template <int W>
__global__ __launch_bounds__(kBlock) void weighted_sum(int count, const double *__restrict__ wts,
                                                       const double *__restrict__ perms,
                                                       double *__restrict__ out)
{
    __shared__ dd red[kWavesPerBlock];
    for (int q = 0; q < W; ++q) {
        dd acc = dd{0.0, 0.0};
        for (int m = threadIdx.x; m < count; m += kBlock) {
#pragma clang fp contract(off)
            // (no contraction: fused into the sum below, p would enter as the
            // exact product, whose rounding error e already carries)
            const double v = perms[W * m + q];
            const double p = wts[m] * v;
            const double e = __builtin_fma(wts[m], v, -p);  // exact product error
            acc = dd_add(acc, dd{p, e});
        }
        const dd t = block_reduce_dd(acc, red);
        if (threadIdx.x == 0) out[q] = t.hi + t.lo;
    }
}

int launch_weighted_sum(int count, const double *wts, const double *perms, double *out, bool real,
                        hipStream_t stream)
{
    if (real)
        hipLaunchKernelGGL(weighted_sum<1>, dim3(1), dim3(kBlock), 0, stream, count, wts, perms, out);
    else
        hipLaunchKernelGGL(weighted_sum<2>, dim3(1), dim3(kBlock), 0, stream, count, wts, perms, out);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

template <bool CPLX>
static void launch_persistent_t(const BatchLaunch &L, int g, hipStream_t stream)
{
    const dim3 grid(unsigned(L.grid[g])), block(kBatchThreads);
    const int64_t n = L.n_items[g];
    if (g == 0)
        hipLaunchKernelGGL((batched_persistent<1, 16, CPLX>), grid, block, 0, stream, L.mats,
                           L.items[0], n, L.counters + 0, L.stage, L.perm_parts, L.g_parts,
                           L.want_grad);
    else if (g == 1)
        hipLaunchKernelGGL((batched_persistent<17, 24, CPLX>), grid, block, 0, stream, L.mats,
                           L.items[1], n, L.counters + 1, L.stage, L.perm_parts, L.g_parts,
                           L.want_grad);
    else
        hipLaunchKernelGGL((batched_persistent_large<25, 32, CPLX>), grid, block, 0, stream, L.mats,
                           L.items[2], n, L.counters + 2, L.stage, L.perm_parts, L.g_parts,
                           L.want_grad);
}

static void launch_persistent(const BatchLaunch &L, int g, hipStream_t stream)
{
    if (L.n_items[g] <= 0) return;
    if (L.real) launch_persistent_t<false>(L, g, stream);
    else launch_persistent_t<true>(L, g, stream);
}

static void launch_prep(const BatchLaunch &L, hipStream_t stream)
{
    hipLaunchKernelGGL(batched_reset, dim3(1), dim3(64), 0, stream, L.counters, kBatchGroups);
    if (L.real)
        hipLaunchKernelGGL(batched_prep<false>, dim3(unsigned(L.count)), dim3(kBlock), 0, stream,
                           L.mats, L.data, L.stage);
    else
        hipLaunchKernelGGL(batched_prep<true>, dim3(unsigned(L.count)), dim3(kBlock), 0, stream,
                           L.mats, L.data, L.stage);
}

static void launch_finalize(const BatchLaunch &L, hipStream_t stream)
{
    double *grad = L.want_grad ? L.grad : nullptr;
    if (L.real)
        hipLaunchKernelGGL(batched_finalize<false>, dim3(unsigned(L.count)), dim3(kBlock), 0, stream,
                           L.mats, L.perm_parts, L.g_parts, L.out, grad);
    else
        hipLaunchKernelGGL(batched_finalize<true>, dim3(unsigned(L.count)), dim3(kBlock), 0, stream,
                           L.mats, L.perm_parts, L.g_parts, L.out, grad);
}

int launch_batched(const BatchLaunch &L, hipStream_t stream)
{
    launch_prep(L, stream);
    for (int g = kBatchGroups - 1; g >= 0; --g) launch_persistent(L, g, stream);
    launch_finalize(L, stream);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

int launch_batched_forked(const BatchLaunch &L, hipStream_t stream,
                          const hipStream_t side[kBatchGroups], hipEvent_t fork,
                          const hipEvent_t join[kBatchGroups])
{
    launch_prep(L, stream);
    if (hipEventRecord(fork, stream) != hipSuccess) return PERM_EHIP;
    for (int g = kBatchGroups - 1; g >= 0; --g) {
        if (L.n_items[g] <= 0) continue;
        if (side[g] != stream && hipStreamWaitEvent(side[g], fork, 0) != hipSuccess) return PERM_EHIP;
        launch_persistent(L, g, side[g]);
        if (side[g] != stream) {
            if (hipEventRecord(join[g], side[g]) != hipSuccess) return PERM_EHIP;
            if (hipStreamWaitEvent(stream, join[g], 0) != hipSuccess) return PERM_EHIP;
        }
    }
    launch_finalize(L, stream);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
