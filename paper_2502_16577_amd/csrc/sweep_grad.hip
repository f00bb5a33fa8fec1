// Permanent and its gradient dperm/dA in one Gray-walk sweep.
//
// With tau_j(g) = +1 when column j is in S_g or j = n-1 and -1 otherwise,
// x_i(g) = (1/2) sum_j tau_j(g) a_ij, so differentiating the Nijenhuis-Wilf
// sum of Algorithm 1 term by term gives
//     dperm/da_kl = (-1)^(n-1) sum_g (-1)^g L_k(g) tau_l(g),
//     L_k(g) = prod_{i != k} x_i(g)  (leave-one-out products).
// Per subset the kernel forms L by prefix and suffix product passes (no
// division, so zeros in x are harmless) and contracts V = (-1)^g L with tau
// on FP64 MFMA, organised by Gray-code windows (grad_item.h).  Each block of
// two waves covers 64 subsets; the waves split the rows.  The MFMA
// accumulators are folded at the end of every window (at most 512 steps)
// into per-item double-double accumulators in global memory.
#include "grad_item.h"

namespace perm {

constexpr int kGradBlock = kGradSlices * kWave;  // one grad_item per block

// Staging for grad_item: column-major A with np rows per column (rows >= n
// zero) and x0 with np entries (1 for rows >= n).  A is row-major with W
// doubles per entry and a row stride of lda entries.
template <bool CPLX>
__global__ __launch_bounds__(kBlock) void prep_grad(int n, int np, const double *__restrict__ A,
                                                    int64_t lda, double *__restrict__ acol,
                                                    double *__restrict__ x0)
{
    constexpr int W = CPLX ? 2 : 1;
    for (int idx = threadIdx.x; idx < n * np; idx += blockDim.x) {
        const int j = idx / np, i = idx - j * np;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const double v = i < n ? A[(int64_t(i) * lda + j) * W + q] : 0.0;
            acol[W * idx + q] = v;
        }
    }
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < W; ++q) {
            if (i >= n) {
                x0[W * i + q] = q == 0 ? 1.0 : 0.0;
                continue;
            }
            double s = 0.0, e = 0.0;  // compensated row sum
            for (int j = 0; j < n; ++j) acc_add(s, e, A[(int64_t(i) * lda + j) * W + q]);
            x0[W * i + q] = (A[(int64_t(i) * lda + n - 1) * W + q] - 0.5 * s) - 0.5 * e;
        }
    }
}

// Permanent (and, if asked, gradient) of one matrix: item w = blockIdx.x
// (subsets 64 w .. 64 w + 63).  perm_part[2w..2w+1] and g_part[w * W*N*N ...]
// receive the item's shares.
template <int N, bool CPLX>
__device__ __forceinline__ void sweep_grad_body(const double *__restrict__ acol,
                                                const double *__restrict__ x0,
                                                dd *__restrict__ perm_part, dd *__restrict__ g_part,
                                                int c, int r, int64_t lanes_active, int want_grad)
{
    using S = GradItemShape<N, CPLX>;
    static_assert(S::THREADS == kGradBlock, "block shape");
    __shared__ double lds[S::LDS_DOUBLES];
    const uint64_t w = blockIdx.x;
    grad_item<N, CPLX>(acol, x0, w, c, r, uint64_t(lanes_active), perm_part + 2 * w,
                       g_part + w * uint64_t(S::W * N * N), want_grad != 0, lds);
}

// Orders up to 24 fit two waves per SIMD (at most 256 registers per lane,
// as in the batched kernel of orders 17..24); the compiler is held to that.
template <int N, bool CPLX>
__global__ __launch_bounds__(kGradBlock) __attribute__((amdgpu_waves_per_eu(2))) void
sweep_grad(const double *__restrict__ acol, const double *__restrict__ x0, dd *__restrict__ perm_part, dd *__restrict__ g_part, int c,
           int r, int64_t lanes_active, int want_grad)
{
    sweep_grad_body<N, CPLX>(acol, x0, perm_part, g_part, c, r, lanes_active, want_grad);
}

// Orders 25..32: one wave per SIMD.
template <int N, bool CPLX>
__global__ __launch_bounds__(kGradBlock) void sweep_grad_large(
    const double *__restrict__ acol, const double *__restrict__ x0, dd *__restrict__ perm_part, dd *__restrict__ g_part, int c, int r, int64_t lanes_active,
    int want_grad)
{
    sweep_grad_body<N, CPLX>(acol, x0, perm_part, g_part, c, r, lanes_active, want_grad);
}

// n = 1: perm = a, dperm/da = 1.
__global__ void grad_order1(const double *__restrict__ a, int cplx, double *__restrict__ out_perm,
                            double *__restrict__ out_grad)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    out_perm[0] = a[0];
    if (cplx) out_perm[1] = a[1];
    if (out_grad) {
        out_grad[0] = 1.0;
        if (cplx) out_grad[1] = 0.0;
    }
}

// First pass over the items' G partials, read coalesced: block (t, s) takes
// the entries 64 t .. 64 t + 63 (one per lane) and the items of slice s, wave
// w every fourth item from the slice's w-th, then adds its waves in order.
template <int N, bool CPLX>
__global__ __launch_bounds__(kBlock) void grad_slice_sums(const dd *__restrict__ g_part,
                                                          int64_t items, int slices,
                                                          dd *__restrict__ g_sum)
{
    constexpr int E = (CPLX ? 2 : 1) * N * N;
    __shared__ dd red[kWavesPerBlock][kWave];
    const int lane = int(threadIdx.x) & (kWave - 1);
    const int w = int(threadIdx.x) / kWave;
    const int e = int(blockIdx.x) * kWave + lane;
    const int64_t per = (items + slices - 1) / slices;
    const int64_t v0 = int64_t(blockIdx.y) * per;
    const int64_t v1 = v0 + per < items ? v0 + per : items;
    dd acc = dd{0.0, 0.0};
    if (e < E)
        for (int64_t v = v0 + w; v < v1; v += kWavesPerBlock) acc = dd_add(acc, g_part[v * E + e]);
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0 && e < E) {
        dd t = red[0][lane];
        for (int q = 1; q < kWavesPerBlock; ++q) t = dd_add(t, red[q][lane]);
        g_sum[int64_t(blockIdx.y) * E + e] = t;
    }
}

// Second pass: G = (-1)^(n-1) times the sum of the slices' sums, one wave per
// entry (lane s reads slice s's sum; at most 64 slices) combined by a fixed
// shuffle tree; block 0 also writes 2 (-1)^(n-1) times the sum of the items'
// permanent shares.
template <int N, bool CPLX>
__global__ __launch_bounds__(kBlock) void finalize_grad(const dd *__restrict__ perm_part,
                                                        const dd *__restrict__ g_sum,
                                                        int64_t items, int slices,
                                                        double *__restrict__ out_perm,
                                                        double *__restrict__ out_grad)
{
    constexpr int W = CPLX ? 2 : 1;
    constexpr int E = W * N * N;
    __shared__ dd red[kWavesPerBlock];
    const double sgn = (N & 1) ? 1.0 : -1.0;
    const int lane = int(threadIdx.x) & (kWave - 1);
    const int e = int(blockIdx.x) * kWavesPerBlock + int(threadIdx.x) / kWave;
    dd t = dd{0.0, 0.0};
    if (e < E && lane < slices) t = g_sum[int64_t(lane) * E + e];
    t = wave_reduce_dd(t);
    if (e < E && lane == 0) out_grad[e] = sgn * (t.hi + t.lo);
    if (blockIdx.x == 0) {
        for (int q = 0; q < W; ++q) {
            dd pacc = dd{0.0, 0.0};
            for (int64_t v = threadIdx.x; v < items; v += kBlock)
                pacc = dd_add(pacc, perm_part[v * 2 + q]);
            const dd pt = block_reduce_dd(pacc, red);
            if (threadIdx.x == 0) out_perm[q] = 2.0 * sgn * (pt.hi + pt.lo);
        }
    }
}

// Forward only: 2 (-1)^(n-1) times the sum of the waves' shares (fixed order).
template <bool CPLX>
__global__ __launch_bounds__(kBlock) void finalize_perm_only(const dd *__restrict__ perm_part,
                                                             int64_t waves, double scale,
                                                             double *__restrict__ out_perm)
{
    __shared__ dd red[kWavesPerBlock];
    for (int q = 0; q < (CPLX ? 2 : 1); ++q) {
        dd acc = dd{0.0, 0.0};
        for (int64_t v = threadIdx.x; v < waves; v += kBlock) acc = dd_add(acc, perm_part[v * 2 + q]);
        const dd t = block_reduce_dd(acc, red);
        if (threadIdx.x == 0) out_perm[q] = scale * (t.hi + t.lo);
    }
}

template <int N, bool CPLX>
static void launch_grad_n(const GradPlan &p, const double *acol, const double *x0, dd *pp, dd *gp,
                          dd *gs, bool want_grad, double *out_perm, double *out_grad,
                          hipStream_t stream)
{
    if constexpr (N <= 24)
        hipLaunchKernelGGL((sweep_grad<N, CPLX>), dim3(unsigned(p.waves)), dim3(kGradBlock), 0,
                           stream, acol, x0, pp, gp, p.log2_chunk, p.log2_reseed,
                           p.lanes_active, int(want_grad));
    else
        hipLaunchKernelGGL((sweep_grad_large<N, CPLX>), dim3(unsigned(p.waves)), dim3(kGradBlock),
                           0, stream, acol, x0, pp, gp, p.log2_chunk, p.log2_reseed,
                           p.lanes_active, int(want_grad));
    if (want_grad) {
        constexpr int E = N * N * (CPLX ? 2 : 1);
        const int slices = grad_sum_slices(p.waves);
        hipLaunchKernelGGL((grad_slice_sums<N, CPLX>),
                           dim3(unsigned((E + kWave - 1) / kWave), unsigned(slices)), dim3(kBlock),
                           0, stream, gp, p.waves, slices, gs);
        hipLaunchKernelGGL((finalize_grad<N, CPLX>),
                           dim3(unsigned((E + kWavesPerBlock - 1) / kWavesPerBlock)), dim3(kBlock),
                           0, stream, pp, gs, p.waves, slices, out_perm, out_grad);
    } else
        hipLaunchKernelGGL(finalize_perm_only<CPLX>, dim3(1), dim3(kBlock), 0, stream, pp, p.waves,
                           (N & 1) ? 2.0 : -2.0, out_perm);
}

using GradLauncher = void (*)(const GradPlan &, const double *, const double *, dd *, dd *, dd *,
                              bool, double *, double *, hipStream_t);

template <bool CPLX, int... Ns>
struct GradTable {
    static GradLauncher get(int n)
    {
        GradLauncher f = nullptr;
        ((n == Ns ? (f = &launch_grad_n<Ns, CPLX>, 0) : 0), ...);
        return f;
    }
};

using GradF64Table = GradTable<false, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18,
                               19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32>;
using GradC128Table = GradTable<true, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18,
                                19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32>;

// Gray-walk decomposition of one matrix for grad_item: lanes * 2^c = 2^(n-1)
// with c >= 1, at most 2^16 lanes (1024 two-wave items: two waves per SIMD),
// r <= c - 1.  Below that cap the lanes are as many as keep 2^4 steps per
// lane: more, shorter items fill the chip at small n, which outweighs their
// per-item set-up (measured per perm_grad call: n = 16 complex 0.123 ->
// 0.034 ms, n = 20 complex 0.146 -> 0.068 ms, n = 22 real 0.092 -> 0.064 ms
// against the earlier minimum of 2^7 steps; n >= 24 sits at the cap).
GradPlan plan_grad(int n)
{
    GradPlan p;
    p.n = n;
    if (n <= 1) {
        p.waves = 1;
        return p;
    }
    const int total = n - 1;
    int lanes_log = total - 1;
    if (lanes_log > 16) lanes_log = 16;
    if (total >= 12 && lanes_log > total - 4) lanes_log = total - 4;  // >= 16 steps per lane
    if (lanes_log < 0) lanes_log = 0;
    p.log2_chunk = total - lanes_log;
    p.log2_reseed = p.log2_chunk - 1 < 9 ? p.log2_chunk - 1 : 9;
    p.lanes_active = int64_t(1) << lanes_log;
    p.waves = p.lanes_active >= kWave ? p.lanes_active / kWave : 1;
    return p;
}

static int launch_stage(int n, bool cplx, const void *A, int64_t lda, double *acol, double *x0,
                        hipStream_t stream)
{
    const int np = grad_rows(n);
    if (cplx)
        hipLaunchKernelGGL(prep_grad<true>, dim3(1), dim3(kBlock), 0, stream, n, np,
                           static_cast<const double *>(A), lda, acol, x0);
    else
        hipLaunchKernelGGL(prep_grad<false>, dim3(1), dim3(kBlock), 0, stream, n, np,
                           static_cast<const double *>(A), lda, acol, x0);
    return PERM_OK;
}

int launch_grad(int n, bool cplx, const void *A, int64_t lda, void *out_perm, void *out_grad,
                char *ws, hipStream_t stream)
{
    return launch_grad_or_small(n, cplx, A, lda, out_perm, out_grad, true, ws, stream);
}

int launch_grad_or_small(int n, bool cplx, const void *A, int64_t lda, void *out_perm,
                         void *out_grad, bool want_grad, char *ws, hipStream_t stream)
{
    const GradPlan p = plan_grad(n);
    const GradWs L = grad_ws_layout(n, cplx ? 2 : 1, p.waves);
    if (n == 1) {
        // a[0] is read straight from the caller's matrix
        hipLaunchKernelGGL(grad_order1, dim3(1), dim3(1), 0, stream, static_cast<const double *>(A),
                           int(cplx), static_cast<double *>(out_perm),
                           want_grad ? static_cast<double *>(out_grad) : nullptr);
        return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
    }
    double *acol = reinterpret_cast<double *>(ws + L.acol);
    double *x0 = reinterpret_cast<double *>(ws + L.x0);
    dd *pp = reinterpret_cast<dd *>(ws + L.perm_partials);
    dd *gp = reinterpret_cast<dd *>(ws + L.grad_partials);
    dd *gs = reinterpret_cast<dd *>(ws + L.grad_sums);
    launch_stage(n, cplx, A, lda, acol, x0, stream);
    GradLauncher f = cplx ? GradC128Table::get(n) : GradF64Table::get(n);
    if (!f) return PERM_EUNSUPPORTED;
    f(p, acol, x0, pp, gp, gs, want_grad, static_cast<double *>(out_perm),
      static_cast<double *>(out_grad), stream);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
