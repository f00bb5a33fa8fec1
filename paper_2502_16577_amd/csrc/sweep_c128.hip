// Dense complex permanent: the same Gray-code Ryser / Nijenhuis-Wilf sweep
// as sweep_f64.hip with complex x and complex products (the paper lists
// complex matrices among its inputs, Section 1; the algorithm is unchanged).
//
// Layout: acol[2*(j*N + i) + {0,1}] = (Re, Im) a_ij, aneg its negation,
// x0[2*i + {0,1}] the start vector.  x lives in 2N VGPR pairs; the column of
// each step is wave-uniform and read with scalar loads.
#include <algorithm>

#include "sweep_common.h"

namespace perm {

__global__ __launch_bounds__(kBlock) void prep_dense_c128(int n, const perm_c128 *__restrict__ A,
                                                          int64_t lda, double *__restrict__ acol,
                                                          double *__restrict__ aneg,
                                                          double *__restrict__ x0)
{
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int j = idx / n;
        const int i = idx - j * n;
        const perm_c128 v = A[int64_t(i) * lda + j];
        acol[2 * idx] = v.re;
        acol[2 * idx + 1] = v.im;
        aneg[2 * idx] = -v.re;
        aneg[2 * idx + 1] = -v.im;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double sr = 0.0, er = 0.0, si = 0.0, ei = 0.0;
        for (int j = 0; j < n; ++j) {
            const perm_c128 v = A[int64_t(i) * lda + j];
            acc_add(sr, er, v.re);
            acc_add(si, ei, v.im);
        }
        const perm_c128 last = A[int64_t(i) * lda + n - 1];
        x0[2 * i] = (last.re - 0.5 * sr) - 0.5 * er;
        x0[2 * i + 1] = (last.im - 0.5 * si) - 0.5 * ei;
    }
}

__device__ __forceinline__ void cmul(double &ar, double &ai, double br, double bi)
{
    const double r = ar * br - ai * bi;
    const double i = ar * bi + ai * br;
    ar = r;
    ai = i;
}

// Eight interleaved chains (more independent work per step) where the
// registers allow it (n <= 30); four above.
template <int N>
__device__ __forceinline__ void cproduct8(const double (&xr)[N], const double (&xi)[N],
                                          double &outr, double &outi)
{
    static_assert(N >= 8, "cproduct8 needs N >= 8");
    double r[8], im[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        r[c] = xr[c];
        im[c] = xi[c];
    }
#pragma unroll
    for (int i = 8; i < N; ++i) cmul(r[i & 7], im[i & 7], xr[i], xi[i]);
    cmul(r[0], im[0], r[1], im[1]);
    cmul(r[2], im[2], r[3], im[3]);
    cmul(r[4], im[4], r[5], im[5]);
    cmul(r[6], im[6], r[7], im[7]);
    cmul(r[0], im[0], r[2], im[2]);
    cmul(r[4], im[4], r[6], im[6]);
    cmul(r[0], im[0], r[4], im[4]);
    outr = r[0];
    outi = im[0];
}

template <int N>
__device__ __forceinline__ void cproduct4(const double (&xr)[N], const double (&xi)[N],
                                          double &outr, double &outi)
{
    static_assert(N >= 4, "cproduct4 needs N >= 4");
    double r0 = xr[0], i0 = xi[0], r1 = xr[1], i1 = xi[1];
    double r2 = xr[2], i2 = xi[2], r3 = xr[3], i3 = xi[3];
#pragma unroll
    for (int i = 4; i < N; i += 4) {
        cmul(r0, i0, xr[i], xi[i]);
        if (i + 1 < N) cmul(r1, i1, xr[i + 1], xi[i + 1]);
        if (i + 2 < N) cmul(r2, i2, xr[i + 2], xi[i + 2]);
        if (i + 3 < N) cmul(r3, i3, xr[i + 3], xi[i + 3]);
    }
    cmul(r0, i0, r1, i1);
    cmul(r2, i2, r3, i3);
    cmul(r0, i0, r2, i2);
    outr = r0;
    outi = i0;
}

template <int N>
__device__ __forceinline__ void cproduct(const double (&xr)[N], const double (&xi)[N],
                                         double &outr, double &outi)
{
    if constexpr (N <= 30) cproduct8<N>(xr, xi, outr, outi);
    else cproduct4<N>(xr, xi, outr, outi);
}

template <int N>
__device__ __forceinline__ void add_ccolumn(double (&xr)[N], double (&xi)[N],
                                            const double *__restrict__ a)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xr[i] += a[2 * i];
        xi[i] += a[2 * i + 1];
    }
}

template <int N>
__device__ __forceinline__ void creseed(double (&xr)[N], double (&xi)[N],
                                        const double *__restrict__ acol,
                                        const double *__restrict__ x0, uint64_t hbits, uint32_t low,
                                        int c)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xr[i] = x0[2 * i];
        xi[i] = x0[2 * i + 1];
    }
    for (int j = c; j < N - 1; ++j) {
        const double f = ((hbits >> (j - c)) & 1u) ? 1.0 : 0.0;
        const double *a = acol + 2 * j * N;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            xr[i] = __builtin_fma(f, a[2 * i], xr[i]);
            xi[i] = __builtin_fma(f, a[2 * i + 1], xi[i]);
        }
    }
    while (low) {
        const int j = __builtin_ctz(low);
        low &= low - 1u;
        add_ccolumn<N>(xr, xi, acol + 2 * j * N);
    }
}

// The lane walks its chunk in blocks of 2^U steps exactly as the real sweep
// does: only the first step of a block flips a column chosen at run time;
// steps l + m flip column ctz(m) with a sign fixed by m (by bit U of l for
// m = 2^(U-1)).  The block's signed terms are summed in a chain before one
// compensated update of each lane partial.  Requires c > U.
template <int N>
constexpr int cdense_unroll() { return N >= 14 ? 4 : 3; }

template <int N>
__global__ __launch_bounds__(kBlock) void sweep_dense_c128(const double *__restrict__ acol,
                                                           const double *__restrict__ aneg,
                                                           const double *__restrict__ x0,
                                                           dd *__restrict__ partials, int c,
                                                           int r, uint32_t l_begin,
                                                           uint32_t l_end, int accumulate)
{
    constexpr int U = cdense_unroll<N>();
    constexpr uint32_t B = 1u << U;
    __shared__ dd red[kWavesPerBlock];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = uniform_wave_index();
    const uint64_t K = lane_chunk_index(wave, lane);
    const uint32_t kb = uint32_t(wave & 1u);
    const uint64_t g0 = K << c;
    const uint64_t hbits = (g0 ^ (g0 >> 1)) >> c;
    const uint32_t rmask = (1u << r) - 1u;

    double xr[N], xi[N];
    double sr = 0.0, er = 0.0, si = 0.0, ei = 0.0;
    for (uint32_t l = l_begin; l < l_end; l += B) {
        if ((l & rmask) == 0) {  // always at l_begin, a re-seed boundary
            creseed<N>(xr, xi, acol, x0, hbits, gray_low(l, kb, c), c);
        } else {
            const int j = __builtin_ctz(l);
            const bool add = (gray_low(l, kb, c) >> j) & 1u;
            add_ccolumn<N>(xr, xi, (add ? acol : aneg) + 2 * j * N);
        }
        double br, bi;
        cproduct<N>(xr, xi, br, bi);
#pragma unroll
        for (uint32_t m = 1; m < B; ++m) {
            const int j = __builtin_ctz(m);
            const bool neg = (j + 1 < U) ? ((m >> (j + 1)) & 1u) : ((l >> U) & 1u);
            // a fresh opaque offset per step keeps the compiler from merging
            // or hoisting these constant-address column loads (whole columns
            // held in SGPRs would spill)
            uint32_t zero = 0;
            asm volatile("" : "+s"(zero));
            add_ccolumn<N>(xr, xi, (neg ? aneg : acol) + 2 * j * N + zero);
            double tr, ti;
            cproduct<N>(xr, xi, tr, ti);
            if (m & 1u) {  // (-1)^g = (-1)^m since l is even
                br -= tr;
                bi -= ti;
            } else {
                br += tr;
                bi += ti;
            }
        }
        acc_add(sr, er, br);
        acc_add(si, ei, bi);
    }
    const dd tr = block_reduce_dd(dd{sr, er}, red);
    const dd ti = block_reduce_dd(dd{si, ei}, red);
    if (threadIdx.x == 0) {
        dd *pp = partials + 2 * blockIdx.x;
        pp[0] = accumulate ? dd_add(pp[0], tr) : tr;
        pp[1] = accumulate ? dd_add(pp[1], ti) : ti;
    }
}

template <int N>
static void launch_csweep_n(const SweepPlan &p, const double *acol, const double *aneg,
                            const double *x0, dd *partials, hipStream_t stream)
{
    // long sweeps: full-grid launches over consecutive ranges of every lane's
    // chunk, each of at most 2^40 subset-steps and starting on a re-seed
    // boundary; later launches add to the partials of earlier ones
    const int64_t C = int64_t(1) << p.log2_chunk;
    int64_t span = std::max<int64_t>((int64_t(1) << 40) / p.lanes,
                                     std::max<int64_t>(int64_t(1) << p.log2_reseed,
                                                       1 << cdense_unroll<N>()));
    int64_t pow2 = 1;
    while (pow2 * 2 <= span) pow2 *= 2;
    span = std::min(pow2, C);
    for (int64_t l0 = 0; l0 < C; l0 += span)
        hipLaunchKernelGGL(sweep_dense_c128<N>, dim3(unsigned(p.blocks)), dim3(kBlock), 0, stream,
                           acol, aneg, x0, partials, p.log2_chunk, p.log2_reseed, uint32_t(l0),
                           uint32_t(l0 + span), int(l0 > 0));
}

using CSweepLauncher = void (*)(const SweepPlan &, const double *, const double *,
                                const double *, dd *, hipStream_t);

template <int... Ns>
struct CSweepTable {
    static CSweepLauncher get(int n)
    {
        CSweepLauncher f = nullptr;
        ((n == Ns ? (f = &launch_csweep_n<Ns>, 0) : 0), ...);
        return f;
    }
};

using DenseC128Table =
    CSweepTable<13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32,
                33, 34, 35, 36, 37, 38, 39, 40, 41, 42, 43, 44, 45, 46, 47, 48, 49, 50, 51, 52, 53,
                54, 55, 56, 57, 58, 59, 60, 61, 62, 63>;

__global__ void write_one_c128(perm_c128 *out) { out[0] = perm_c128{1.0, 0.0}; }

int launch_dense_c128(int n, const perm_c128 *A, int64_t lda, perm_c128 *out, char *ws,
                      hipStream_t stream)
{
    if (n == 0) {
        hipLaunchKernelGGL(write_one_c128, dim3(1), dim3(1), 0, stream, out);
        return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
    }
    const SweepPlan p = plan_sweep(n, 0);
    const DenseWs L = dense_ws_layout(n, 2, dense_ws_blocks(n));
    double *acol = reinterpret_cast<double *>(ws + L.acol);
    double *aneg = reinterpret_cast<double *>(ws + L.aneg);
    double *x0 = reinterpret_cast<double *>(ws + L.x0);
    dd *partials = reinterpret_cast<dd *>(ws + L.partials);
    if (n <= kSmallN)  // one or a few waves: the gradient sweep's kernel without the gradient
        return launch_grad_or_small(n, true, A, lda, out, nullptr, false, ws, stream);
    hipLaunchKernelGGL(prep_dense_c128, dim3(1), dim3(kBlock), 0, stream, n, A, lda, acol, aneg,
                       x0);
    const int64_t nparts = p.blocks;
    {
        CSweepLauncher f = DenseC128Table::get(n);
        if (!f) return PERM_EUNSUPPORTED;
        f(p, acol, aneg, x0, partials, stream);
    }
    const double scale = (n & 1) ? 2.0 : -2.0;
    hipLaunchKernelGGL(finalize_partials, dim3(1), dim3(kBlock), 0, stream, partials, nparts, 2,
                       scale, reinterpret_cast<double *>(out));
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
