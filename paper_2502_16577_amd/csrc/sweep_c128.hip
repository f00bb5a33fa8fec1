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

// ---------------------------------------------------------------------------
// Extended-precision complex walk (accumulation mode kAccExtended): the real
// and imaginary parts of every x_i are pairs exact in their high parts (the
// entries are split error-free, below),
// every factor of the product a complex double-double product (each real
// product the rounded product of the high parts plus, as the low part, its
// FMA rounding error and the cross terms; the two real sums by two-sum), and
// the lane partial a complex double-double.  Each operation is then exact to
// about 2^-104 of its operands.  One step per loop iteration; the lane
// partitioning and re-seeds are those of the FP64 walk.

// Error-free split of the entries (both components) for the extended walk,
// row by row: a_ij = ah_ij + al_ij with ah_ij a multiple of a power of two q_i
// and |al_ij| <= q_i / 2 in each component, q_i chosen from the row's sum
// m_i = sum_j (|re a_ij| + |im a_ij|) so that m_i / q_i < 2^50; then both high
// parts of x_i (sums of multiples of q_i / 2 below 2^51 of them) are exact in
// FP64 with one addition per flip.  The grid is per row as in the real walk:
// a shared grid would leave rows of much smaller scale in their low parts,
// whose products with each other the double-double product does not keep.
// `split` holds four arrays of n x n interleaved (re, im) pairs,
// column-major like the column copies: ah, al, -ah, -al (a flip adds the pair
// of the sign it needs).
__global__ __launch_bounds__(kBlock) void prep_dense_c128_ext(int n, const perm_c128 *__restrict__ A,
                                                              int64_t lda, double *__restrict__ split)
{
    __shared__ double grid[kBlock];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double m = 0.0;
        for (int j = 0; j < n; ++j) {
            const perm_c128 v = A[int64_t(i) * lda + j];
            m += __builtin_fabs(v.re) + __builtin_fabs(v.im);
        }
        int e = 0;
        frexp(m > 0.0 ? m : 1.0, &e);  // m < 2^e
        grid[i] = ldexp(1.0, e - 50 > -1074 ? e - 50 : -1074);  // no grid below the least double
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int j = idx / n;
        const int i = idx - j * n;
        const double q = grid[i];
        const perm_c128 v = A[int64_t(i) * lda + j];
        const double hr = rint(v.re / q) * q, hi = rint(v.im / q) * q;  // exact
        const double lr = v.re - hr, li = v.im - hi;  // exact: the bits below q
        const int64_t nn2 = 2 * int64_t(n) * n;
        split[2 * idx] = hr;
        split[2 * idx + 1] = hi;
        split[nn2 + 2 * idx] = lr;
        split[nn2 + 2 * idx + 1] = li;
        split[2 * nn2 + 2 * idx] = -hr;
        split[2 * nn2 + 2 * idx + 1] = -hi;
        split[3 * nn2 + 2 * idx] = -lr;
        split[3 * nn2 + 2 * idx + 1] = -li;
    }
}

// a b as a double-double (rounded product of the high parts; its FMA
// rounding error and the cross terms as the low part).  Contraction is off:
// fused into a later sum, the rounded product would enter as the exact
// product, whose rounding error the low part already carries.
__device__ __forceinline__ void cext_prod(double ah, double al, double bh, double bl, double &h,
                                          double &l)
{
#pragma clang fp contract(off)
    h = ah * bh;
    double e = __builtin_fma(ah, bh, -h);
    e = __builtin_fma(ah, bl, e);
    l = __builtin_fma(al, bh, e);
}

// (ar, ai) *= (br, bi), every component a double-double (high, low).  The
// two sums are two-sums written out with contraction off and without
// negating a product: a negated product in a contracting scope becomes a
// new, contractible multiply that the compiler fuses into the sum, which
// counts the product's rounding error twice.
__device__ __forceinline__ void cext_mul(double &arh, double &arl, double &aih, double &ail,
                                         double brh, double brl, double bih, double bil)
{
#pragma clang fp contract(off)
    double p1h, p1l, p2h, p2l, p3h, p3l, p4h, p4l;
    cext_prod(arh, arl, brh, brl, p1h, p1l);
    cext_prod(aih, ail, bih, bil, p2h, p2l);
    cext_prod(arh, arl, bih, bil, p3h, p3l);
    cext_prod(aih, ail, brh, brl, p4h, p4l);
    // re = p1 - p2
    double s = p1h - p2h;
    double bb = s - p1h;
    double t = (p1h - (s - bb)) - (p2h + bb);
    arh = s;
    arl = t + (p1l - p2l);
    // im = p3 + p4
    s = p3h + p4h;
    bb = s - p3h;
    t = (p3h - (s - bb)) + (p4h - bb);
    aih = s;
    ail = t + (p3l + p4l);
}

// x_i += f a_ij for both components of the split column (f = +-1/2 in a
// re-seed): exact in the high parts, one rounded addition in each low part.
template <int N>
__device__ __forceinline__ void cext_add_column(double (&xrh)[N], double (&xrl)[N],
                                                double (&xih)[N], double (&xil)[N],
                                                const double *__restrict__ ah,
                                                const double *__restrict__ al, double f)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xrh[i] = __builtin_fma(f, ah[2 * i], xrh[i]);
        xrl[i] = __builtin_fma(f, al[2 * i], xrl[i]);
        xih[i] = __builtin_fma(f, ah[2 * i + 1], xih[i]);
        xil[i] = __builtin_fma(f, al[2 * i + 1], xil[i]);
    }
}

// A flip, x_i +-= a_ij, from the split pair of the flip's sign (high and low
// parts 2 N * N apart): one add per part, with the column entry read from
// scalar registers as its only scalar operand.
template <int N>
__device__ __forceinline__ void cext_flip_column(double (&xrh)[N], double (&xrl)[N],
                                                 double (&xih)[N], double (&xil)[N],
                                                 const double *__restrict__ col)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xrh[i] += col[2 * i];
        xrl[i] += col[2 * N * N + 2 * i];
        xih[i] += col[2 * i + 1];
        xil[i] += col[2 * N * N + 2 * i + 1];
    }
}

template <int N>
__global__ __launch_bounds__(kBlock) void sweep_dense_c128_ext(const double *__restrict__ split,
                                                               dd *__restrict__ partials, int c,
                                                               int r, uint32_t l_begin,
                                                               uint32_t l_end, int accumulate)
{
    __shared__ dd red[kWavesPerBlock];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = uniform_wave_index();
    const uint64_t K = lane_chunk_index(wave, lane);
    const uint32_t kb = uint32_t(wave & 1u);
    const uint64_t g0 = K << c;
    const uint64_t hbits = (g0 ^ (g0 >> 1)) >> c;
    const uint32_t rmask = (1u << r) - 1u;

    const double *__restrict__ ahi = split;
    const double *__restrict__ alo = split + 2 * N * N;
    double xrh[N], xrl[N], xih[N], xil[N];
    double srh = 0.0, srl = 0.0, sih = 0.0, sil = 0.0;  // lane partial
    for (uint32_t l = l_begin; l < l_end; ++l) {
        if ((l & rmask) == 0) {
            // x = (a_{n-1} + sum_{j<n-1} s_j a_j) / 2, s_j = +1 for the columns
            // in this step's Gray code, else -1
            const uint32_t low = gray_low(l, kb, c);
#pragma unroll
            for (int i = 0; i < N; ++i) {
                xrh[i] = 0.5 * ahi[2 * ((N - 1) * N + i)];
                xrl[i] = 0.5 * alo[2 * ((N - 1) * N + i)];
                xih[i] = 0.5 * ahi[2 * ((N - 1) * N + i) + 1];
                xil[i] = 0.5 * alo[2 * ((N - 1) * N + i) + 1];
            }
            for (int j = 0; j < N - 1; ++j) {
                const bool in = j < c ? ((low >> j) & 1u) != 0u : ((hbits >> (j - c)) & 1u) != 0u;
                cext_add_column<N>(xrh, xrl, xih, xil, ahi + 2 * j * N, alo + 2 * j * N,
                                   in ? 0.5 : -0.5);
            }
        } else {
            const int j = __builtin_ctz(l);
            const bool add = (gray_low(l, kb, c) >> j) & 1u;
            cext_flip_column<N>(xrh, xrl, xih, xil, split + (add ? 0 : 4 * N * N) + 2 * j * N);
        }
        // the product as two interleaved chains
        double prh[2], prl[2], pih[2], pil[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            prh[q] = xrh[q];
            prl[q] = xrl[q];
            pih[q] = xih[q];
            pil[q] = xil[q];
        }
#pragma unroll
        for (int i = 2; i < N; ++i)
            cext_mul(prh[i & 1], prl[i & 1], pih[i & 1], pil[i & 1], xrh[i], xrl[i], xih[i], xil[i]);
        cext_mul(prh[0], prl[0], pih[0], pil[0], prh[1], prl[1], pih[1], pil[1]);
        double th = prh[0], tl = prl[0], uh = pih[0], ul = pil[0];
        if (l & 1u) {  // (-1)^g: g = K 2^c + l with c >= 1
            th = -th;
            tl = -tl;
            uh = -uh;
            ul = -ul;
        }
        double s, t;
        two_sum(srh, th, s, t);
        two_sum(s, t + (srl + tl), srh, srl);
        two_sum(sih, uh, s, t);
        two_sum(s, t + (sil + ul), sih, sil);
    }
    const dd tr = block_reduce_dd(dd{srh, srl}, red);
    const dd ti = block_reduce_dd(dd{sih, sil}, red);
    if (threadIdx.x == 0) {
        dd *pp = partials + 2 * blockIdx.x;
        pp[0] = accumulate ? dd_add(pp[0], tr) : tr;
        pp[1] = accumulate ? dd_add(pp[1], ti) : ti;
    }
}

template <int N>
static void launch_csweep_ext_n(const SweepPlan &p, int log2_reseed, const double *split,
                                dd *partials, hipStream_t stream)
{
    // launches of at most 2^37 subset-steps (the walk is about 8 times slower
    // than the FP64 one), each over a consecutive range of every lane's chunk
    // starting on a re-seed boundary
    const int64_t C = int64_t(1) << p.log2_chunk;
    int64_t span = std::max<int64_t>((int64_t(1) << 37) / p.lanes, int64_t(1) << log2_reseed);
    int64_t pow2 = 1;
    while (pow2 * 2 <= span) pow2 *= 2;
    span = std::min(pow2, C);
    for (int64_t l0 = 0; l0 < C; l0 += span)
        hipLaunchKernelGGL(sweep_dense_c128_ext<N>, dim3(unsigned(p.blocks)), dim3(kBlock), 0,
                           stream, split, partials, p.log2_chunk, log2_reseed, uint32_t(l0),
                           uint32_t(l0 + span), int(l0 > 0));
}

using CExtLauncher = void (*)(const SweepPlan &, int, const double *, dd *, hipStream_t);

template <int... Ns>
struct CExtTable {
    static CExtLauncher get(int n)
    {
        CExtLauncher f = nullptr;
        ((n == Ns ? (f = &launch_csweep_ext_n<Ns>, 0) : 0), ...);
        return f;
    }
};

using DenseC128ExtTable = CExtTable<13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28,
                                    29, 30, 31, 32>;

__global__ void write_one_c128(perm_c128 *out) { out[0] = perm_c128{1.0, 0.0}; }

int launch_dense_c128_ext(int n, const perm_c128 *A, int64_t lda, perm_c128 *out,
                          int log2_reseed, char *ws, hipStream_t stream)
{
    if (n == 0) {
        hipLaunchKernelGGL(write_one_c128, dim3(1), dim3(1), 0, stream, out);
        return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
    }
    CExtLauncher f = DenseC128ExtTable::get(n);
    if (!f) return PERM_EUNSUPPORTED;
    const SweepPlan p = plan_sweep(n, 0);
    if (p.log2_chunk < 1) return PERM_EUNSUPPORTED;
    int r = log2_reseed > 0 ? log2_reseed : p.log2_reseed;
    if (r > p.log2_chunk) r = p.log2_chunk;
    const DenseWs L = dense_ws_layout(n, 2, dense_ws_blocks(n));
    double *split = reinterpret_cast<double *>(ws + L.ext);
    dd *partials = reinterpret_cast<dd *>(ws + L.partials);
    hipLaunchKernelGGL(prep_dense_c128_ext, dim3(1), dim3(kBlock), 0, stream, n, A, lda, split);
    f(p, r, split, partials, stream);
    hipLaunchKernelGGL(finalize_partials, dim3(1), dim3(kBlock), 0, stream, partials, p.blocks, 2,
                       (n & 1) ? 2.0 : -2.0, reinterpret_cast<double *>(out));
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

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
