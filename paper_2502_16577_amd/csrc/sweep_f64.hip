// Dense real FP64 permanent: the Gray-code Ryser / Nijenhuis-Wilf sweep
// (Algorithm 1 of arXiv 2502.16577, chunked as in Algorithm 3 with the
// power-of-two chunks of Section 3.1.1).
//
// Data layout in HBM (all inside the caller's workspace):
//   acol[j*N + i] = a_ij   (column-major, so one Gray step reads one
//   aneg[j*N + i] = -a_ij   contiguous column; the sign picks the copy)
//   x0[i] = a_{i,n-1} - r_i/2
//   partials[b] = double-double sum of block b
//
// Per lane: x[N] lives in VGPRs (N is a template parameter, the analogue of
// the paper's per-matrix rebuild of Section 3.2).  Because the chunk length is
// a power of two and bit 0 of the chunk index is shared by the whole wave,
// the flipped column j = ctz(l) and its sign are wave-uniform at every step,
// so the column is fetched with scalar loads into SGPRs and feeds v_add_f64
// directly: no LDS traffic and no per-lane addressing in the hot loop.
#include <algorithm>
#include <cmath>

#include "sweep_common.h"

namespace perm {

__global__ __launch_bounds__(kBlock) void prep_dense_f64(int n, const double *__restrict__ A,
                                                         int64_t lda, double *__restrict__ acol,
                                                         double *__restrict__ aneg,
                                                         double *__restrict__ x0)
{
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int j = idx / n;
        const int i = idx - j * n;
        const double v = A[int64_t(i) * lda + j];
        acol[idx] = v;
        aneg[idx] = -v;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double s = 0.0, e = 0.0;  // compensated row sum r_i = s + e
        for (int j = 0; j < n; ++j) acc_add(s, e, A[int64_t(i) * lda + j]);
        x0[i] = (A[int64_t(i) * lda + n - 1] - 0.5 * s) - 0.5 * e;
    }
}

template <int N>
__device__ __forceinline__ double product4(const double (&x)[N])
{
    static_assert(N >= 4, "product4 needs N >= 4");
    double p0 = x[0], p1 = x[1], p2 = x[2], p3 = x[3];
#pragma unroll
    for (int i = 4; i < N; i += 4) {
        p0 *= x[i];
        if (i + 1 < N) p1 *= x[i + 1];
        if (i + 2 < N) p2 *= x[i + 2];
        if (i + 3 < N) p3 *= x[i + 3];
    }
    return (p0 * p1) * (p2 * p3);
}

template <int N>
__device__ __forceinline__ void add_column(double (&x)[N], const double *__restrict__ a)
{
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] += a[i];
}

// x = x0 + sum of the columns in the Gray code of step l of this lane's
// chunk: the lane-specific columns j >= c (bits `hbits`) and the
// wave-uniform columns j < c (bits `low`).
template <int N>
__device__ __forceinline__ void reseed(double (&x)[N], const double *__restrict__ acol,
                                       const double *__restrict__ x0, uint64_t hbits,
                                       uint32_t low, int c)
{
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = x0[i];
    for (int j = c; j < N - 1; ++j) {
        const double f = ((hbits >> (j - c)) & 1u) ? 1.0 : 0.0;
        const double *a = acol + j * N;
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] = __builtin_fma(f, a[i], x[i]);
    }
    while (low) {
        const int j = __builtin_ctz(low);
        low &= low - 1u;
        add_column<N>(x, acol + j * N);
    }
}

// One lane walks its chunk in blocks of 2^U steps.  In a block starting at
// l (a multiple of 2^U) only step l flips a column chosen at run time (ctz(l),
// or an exact re-seed); step l + m, 0 < m < 2^U, flips column ctz(m), and its
// sign -- bit ctz(m) of the Gray code after the step, i.e. bit ctz(m) + 1 of
// l + m inverted -- is fixed by m alone, except for m = 2^(U-1) where it is
// bit U of l.  So 2^U - 1 of every 2^U flips read a column at a constant
// address with a constant sign, and the 2^U signed terms are summed in a
// short tree before one compensated update of the lane partial.
// Requires c > U (so bit U of g lies inside the chunk); re-seeds happen at
// block starts, so the effective re-seed interval is at least 2^U.  U = 4
// (16-step blocks) where the plan's chunks allow it (n >= 14), else 3.
template <int N>
constexpr int dense_unroll() { return N >= 14 ? 4 : 3; }

// ACC: how a lane accumulates the block sums -- kAccTwoSum (two-sum: the lane
// partial is a double-double, the paper's "DQ" of Table 3), kAccKahan (Kahan
// compensation, the paper's "Kahan"), kAccPlain (plain doubles, the paper's
// "DD").  A launch walks steps [l_begin, l_end) of every lane's chunk (both
// multiples of the re-seed interval and of 2^U), so a long sweep runs as
// several full-grid launches; `accumulate` adds this launch's block sums to
// the partials of the previous ones (in launch order) instead of storing.
template <int N, int ACC>
__global__ __launch_bounds__(kBlock) void sweep_dense_f64(const double *__restrict__ acol,
                                                          const double *__restrict__ aneg,
                                                          const double *__restrict__ x0,
                                                          dd *__restrict__ partials, int c, int r,
                                                          uint32_t l_begin, uint32_t l_end,
                                                          int accumulate)
{
    constexpr int U = dense_unroll<N>();
    constexpr uint32_t B = 1u << U;
    __shared__ dd red[kWavesPerBlock];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = uniform_wave_index();
    const uint64_t K = lane_chunk_index(wave, lane);
    const uint32_t kb = uint32_t(wave & 1u);
    const uint64_t g0 = K << c;
    const uint64_t hbits = (g0 ^ (g0 >> 1)) >> c;
    const uint32_t rmask = (1u << r) - 1u;

    double x[N];
    double s = 0.0, e = 0.0;
    for (uint32_t l = l_begin; l < l_end; l += B) {
        // step l: re-seed exactly (always at l_begin), or flip column ctz(l)
        if ((l & rmask) == 0) {
            reseed<N>(x, acol, x0, hbits, gray_low(l, kb, c), c);
        } else {
            const int j = __builtin_ctz(l);
            const bool add = (gray_low(l, kb, c) >> j) & 1u;
            add_column<N>(x, (add ? acol : aneg) + j * N);
        }
        double t[B];
        t[0] = product4<N>(x);
#pragma unroll
        for (uint32_t m = 1; m < B; ++m) {
            const int j = __builtin_ctz(m);
            const bool neg = (j + 1 < U) ? ((m >> (j + 1)) & 1u) : ((l >> U) & 1u);
            // An offset the compiler cannot see through, fresh at every step:
            // otherwise it merges or hoists these constant-address column
            // loads and keeps whole columns live in SGPRs, which spills.
            uint32_t zero = 0;
            asm volatile("" : "+s"(zero));
            add_column<N>(x, (neg ? aneg : acol) + j * N + zero);
            t[m] = product4<N>(x);
        }
        // (-1)^g = (-1)^m since l is even
#pragma unroll
        for (uint32_t m = 0; m < B; m += 2) t[m] -= t[m + 1];
#pragma unroll
        for (uint32_t w = 4; w <= B; w *= 2)
#pragma unroll
            for (uint32_t m = 0; m < B; m += w) t[m] += t[m + w / 2];
        const double v = t[0];
        if constexpr (ACC == kAccTwoSum) {
            acc_add(s, e, v);
        } else if constexpr (ACC == kAccKahan) {
            const double y = v - e;  // e holds the running compensation
            const double u = s + y;
            e = (u - s) - y;
            s = u;
        } else {
            s += v;
        }
    }
    // Kahan's e is the negated lost low part
    const dd t = block_reduce_dd(ACC == kAccKahan ? dd{s, -e} : dd{s, e}, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = accumulate ? dd_add(partials[blockIdx.x], t) : t;
}

int64_t dense_launch_span(int n, const SweepPlan &p, const SweepOptions &o)
{
    const int64_t C = int64_t(1) << p.log2_chunk;
    int64_t span = o.max_steps_per_launch / p.lanes;
    const int64_t unit = std::max<int64_t>(int64_t(1) << o.log2_reseed, 1 << (n >= 14 ? 4 : 3));
    span = std::max(unit, span - span % unit);
    int64_t pow2 = unit;
    while (pow2 * 2 <= span && pow2 * 2 <= C) pow2 *= 2;
    return std::min(pow2, C);
}

// Launches [o.first_launch, o.first_launch + o.launch_count) of the sweep
// (all of them for launch_count 0); launch i covers steps [i span, (i+1) span)
// of every lane's chunk and adds to the partials of launches before it.
template <int N>
static void launch_sweep_n(const SweepPlan &p, const SweepOptions &o, const double *acol,
                           const double *aneg, const double *x0, dd *partials,
                           hipStream_t stream)
{
    const int64_t C = int64_t(1) << p.log2_chunk;
    const int64_t span = dense_launch_span(N, p, o);
    const int64_t nl = C / span;
    const int64_t first = std::min(o.first_launch, nl);
    const int64_t end = o.launch_count > 0 ? std::min(nl, first + o.launch_count) : nl;
    for (int64_t i = first; i < end; ++i) {
        const int64_t l0 = i * span;
        const uint32_t lb = uint32_t(l0), le = uint32_t(l0 + span);
        const int accumulate = l0 > 0;
        if (o.accumulation == kAccTwoSum)
            hipLaunchKernelGGL((sweep_dense_f64<N, kAccTwoSum>), dim3(unsigned(p.blocks)),
                               dim3(kBlock), 0, stream, acol, aneg, x0, partials, p.log2_chunk,
                               o.log2_reseed, lb, le, accumulate);
        else if (o.accumulation == kAccKahan)
            hipLaunchKernelGGL((sweep_dense_f64<N, kAccKahan>), dim3(unsigned(p.blocks)),
                               dim3(kBlock), 0, stream, acol, aneg, x0, partials, p.log2_chunk,
                               o.log2_reseed, lb, le, accumulate);
        else
            hipLaunchKernelGGL((sweep_dense_f64<N, kAccPlain>), dim3(unsigned(p.blocks)),
                               dim3(kBlock), 0, stream, acol, aneg, x0, partials, p.log2_chunk,
                               o.log2_reseed, lb, le, accumulate);
    }
}

using SweepLauncher = void (*)(const SweepPlan &, const SweepOptions &, const double *,
                               const double *, const double *, dd *, hipStream_t);

template <int... Ns>
struct SweepTable {
    static SweepLauncher get(int n)
    {
        SweepLauncher f = nullptr;
        ((n == Ns ? (f = &launch_sweep_n<Ns>, 0) : 0), ...);
        return f;
    }
};

using DenseF64Table =
    SweepTable<13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32, 33,
               34, 35, 36, 37, 38, 39, 40, 41, 42, 43, 44, 45, 46, 47, 48, 49, 50, 51, 52, 53, 54,
               55, 56, 57, 58, 59, 60, 61, 62, 63>;

__global__ void write_one_f64(double *out) { out[0] = 1.0; }

int launch_dense_f64(int n, const double *A, int64_t lda, double *out, char *ws,
                     hipStream_t stream)
{
    return launch_dense_f64_opt(n, A, lda, out, default_sweep_options(n), ws, stream);
}

// The dense sweep's plan under the options: plan_sweep's, or the lane count
// of o.log2_lanes clamped to [2^8, max(2^18, default)], to chunks longer than
// the block (c > U) and to chunks of at most 2^31 steps.
SweepPlan dense_plan(int n, const SweepOptions &o)
{
    SweepPlan p = plan_sweep(n, 0);
    if (o.log2_lanes > 0 && n > kSmallN) {
        const int total = n - 1;
        int ll = o.log2_lanes;
        const int unroll = n >= 14 ? 4 : 3;                    // dense_unroll<n>()
        const int max_ll = std::max(total - 1 - unroll, 8);   // c > U
        if (ll > max_ll) ll = max_ll;
        if (ll < 8) ll = 8;                       // one full block of 256 lanes
        const int def_ll = int(std::log2(double(p.lanes)));
        if (ll > std::max(18, def_ll)) ll = std::max(18, def_ll);
        if (ll < total - 31) ll = total - 31;     // chunks of at most 2^31 steps
        p.log2_chunk = total - ll;
        p.lanes = int64_t(1) << ll;
        p.blocks = p.lanes / kBlock;
        if (p.log2_reseed > p.log2_chunk) p.log2_reseed = p.log2_chunk;
    }
    return p;
}

int64_t dense_f64_launches(int n, const SweepOptions &o)
{
    if (n <= kSmallN) return 1;
    const SweepPlan p = dense_plan(n, o);
    SweepOptions oo = o;
    if (oo.log2_reseed < 1 || oo.log2_reseed > p.log2_chunk) oo.log2_reseed = p.log2_chunk;
    return (int64_t(1) << p.log2_chunk) / dense_launch_span(n, p, oo);
}

int launch_dense_f64_opt(int n, const double *A, int64_t lda, double *out, const SweepOptions &o,
                         char *ws, hipStream_t stream)
{
    // The workspace holds block partials for max(default, 2^18 lanes); other
    // lane counts are clamped to that.
    if (n == 0) {
        hipLaunchKernelGGL(write_one_f64, dim3(1), dim3(1), 0, stream, out);
        return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
    }
    if (o.accumulation == kAccExtended) return launch_dense_ext(n, A, lda, out, o, ws, stream);
    const SweepPlan p = dense_plan(n, o);
    const DenseWs L = dense_ws_layout(n, 1, dense_ws_blocks(n));
    double *acol = reinterpret_cast<double *>(ws + L.acol);
    double *aneg = reinterpret_cast<double *>(ws + L.aneg);
    double *x0 = reinterpret_cast<double *>(ws + L.x0);
    dd *partials = reinterpret_cast<dd *>(ws + L.partials);
    if (n <= kSmallN)  // one or a few waves: the gradient sweep's kernel without the gradient
        return launch_grad_or_small(n, false, A, lda, out, nullptr, false, ws, stream);
    hipLaunchKernelGGL(prep_dense_f64, dim3(1), dim3(kBlock), 0, stream, n, A, lda, acol, aneg, x0);
    const int64_t nparts = p.blocks;
    {
        SweepLauncher f = DenseF64Table::get(n);
        if (!f) return PERM_EUNSUPPORTED;
        if (p.log2_chunk <= (n >= 14 ? 4 : 3)) return PERM_EUNSUPPORTED;  // the block walk needs c > U
        SweepOptions oo = o;
        if (oo.log2_reseed < 1 || oo.log2_reseed > p.log2_chunk) oo.log2_reseed = p.log2_chunk;
        f(p, oo, acol, aneg, x0, partials, stream);
    }
    const double scale = (n & 1) ? 2.0 : -2.0;  // 2 (-1)^(n-1)
    hipLaunchKernelGGL(finalize_partials, dim3(1), dim3(kBlock), 0, stream, partials, nparts, 1,
                       scale, out);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
