// Dense real permanent in extended precision (accumulation mode
// PERM_ACC_EXTENDED): the Gray-code Ryser / Nijenhuis-Wilf walk of Algorithm 1
// with x, the products and the lane partials in double-double, beyond the
// paper's precision modes of Section 5.  Launch shapes, re-seeds and split
// launches are those of the FP64 walk (dense_plan, dense_launch_span).
#include <algorithm>
#include <cmath>

#include "sweep_common.h"

namespace perm {

// Extended-precision walk (accumulation mode kAccExtended).  The FP64 walk
// rounds every x_i and every product to 2^-53; where the alternating sum
// cancels deeply (R(A) / |perm(A)| about 1e6 for U[0,1) entries at n = 40)
// those roundings, which are correlated along the Gray walk, leave a
// relative error near 1e-10 even when x is rebuilt exactly every 16 steps.
// Here every x_i is a pair (hi, lo) kept exactly in its high part (the
// entries are split error-free, below), every product a double-double formed
// with FMA, and the lane partial a double-double, so each operation is exact
// to about 2^-104 of its operands.  Two steps per loop iteration; the lane
// partitioning, re-seeds and split launches are those of the FP64 walk.

// Error-free split of the entries for the extended walk, row by row: a_ij =
// ah_ij + al_ij with ah_ij a multiple of a power of two q_i and |al_ij| <=
// q_i / 2, q_i chosen from the row's absolute sum m_i = sum_j |a_ij| so that
// m_i / q_i < 2^50.  Every x_i of the walk is (a_{i,n-1} + sum_{j<n-1} s_j
// a_ij) / 2 with s_j = +-1, so its high part, a sum of multiples of q_i / 2
// below 2^51 of them, is exact in FP64 with one addition per flip, and its
// low part stays below n q_i / 4.  The grid is per row because each x_i uses
// only its own row: a grid shared by rows of very different scale would put
// a small row wholly in its low part, and the product, which keeps the cross
// terms of high and low parts but not low times low, would lose every term
// with two such rows.  `split` holds four n x n column-major arrays: ah, al,
// -ah, -al (a flip adds the pair of the sign it needs, as the FP64 walk
// picks between its column and its negation).
__global__ __launch_bounds__(kBlock) void prep_dense_ext(int n, const double *__restrict__ A,
                                                         int64_t lda, double *__restrict__ split)
{
    __shared__ double grid[kBlock];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double m = 0.0;
        for (int j = 0; j < n; ++j) m += __builtin_fabs(A[int64_t(i) * lda + j]);
        int e = 0;
        frexp(m > 0.0 ? m : 1.0, &e);  // m < 2^e (a rounded row sum is within 2^-45 of its value)
        grid[i] = ldexp(1.0, e - 50 > -1074 ? e - 50 : -1074);  // no grid below the least double
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int j = idx / n;
        const int i = idx - j * n;
        const double q = grid[i];
        const double a = A[int64_t(i) * lda + j];
        const double h = rint(a / q) * q;  // exact: q is a power of two
        const double l = a - h;            // exact: the bits of a below q
        split[idx] = h;
        split[n * n + idx] = l;
        split[2 * n * n + idx] = -h;
        split[3 * n * n + idx] = -l;
    }
}

// (ah, al) *= (bh, bl): the rounded product of the high parts, and as the
// low part its exact rounding error (FMA) plus the two cross terms.  The low
// part is formed afresh at every factor, so it stays within a few ulps of
// the high part and needs no renormalising sum; the pair holds the product
// to about 2^-104 of the operands even where a high part has cancelled below
// its low part.  Contraction is off: fused into a later sum, the rounded
// product p would enter as the exact product, whose rounding error the low
// part already carries, so that error would count twice.
__device__ __forceinline__ void ext_mul(double &ah, double &al, double bh, double bl)
{
#pragma clang fp contract(off)
    const double p = ah * bh;
    double e = __builtin_fma(ah, bh, -p);
    e = __builtin_fma(ah, bl, e);
    e = __builtin_fma(al, bh, e);
    ah = p;
    al = e;
}

// x_i += f a_ij for the split column (f = +-1/2 in a re-seed):
// exact in the high part, one rounded addition in the low part.
template <int N>
__device__ __forceinline__ void ext_add_column(double (&xh)[N], double (&xl)[N],
                                               const double *__restrict__ ah,
                                               const double *__restrict__ al, double f)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xh[i] = __builtin_fma(f, ah[i], xh[i]);
        xl[i] = __builtin_fma(f, al[i], xl[i]);
    }
}

// A flip, x_i +-= a_ij, from the split pair of the flip's sign (ah and al,
// or their negations, at a distance of N * N): one add per part, with the
// column entry read from scalar registers as its only scalar operand.
template <int N>
__device__ __forceinline__ void ext_flip_column(double (&xh)[N], double (&xl)[N],
                                                const double *__restrict__ col)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xh[i] += col[i];
        xl[i] += col[N * N + i];
    }
}

// x = (a_{n-1} + sum_{j<n-1} s_j a_j) / 2 with s_j = +1 for the columns in the
// Gray code of this lane's step (bits below c wave-uniform in `low`, the
// others the lane's `hbits`), else -1.
template <int N>
__device__ __forceinline__ void ext_reseed(double (&xh)[N], double (&xl)[N],
                                           const double *__restrict__ ahi, uint64_t hbits,
                                           uint32_t low, int c)
{
    const double *__restrict__ alo = ahi + N * N;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xh[i] = 0.5 * ahi[(N - 1) * N + i];
        xl[i] = 0.5 * alo[(N - 1) * N + i];
    }
    for (int j = 0; j < N - 1; ++j) {
        const bool in = j < c ? ((low >> j) & 1u) != 0u : ((hbits >> (j - c)) & 1u) != 0u;
        ext_add_column<N>(xh, xl, ahi + j * N, alo + j * N, in ? 0.5 : -0.5);
    }
}

// prod_i x_i as four interleaved double-double chains.
template <int N>
__device__ __forceinline__ void ext_product(const double (&xh)[N], const double (&xl)[N],
                                            double &ph, double &pl)
{
    static_assert(N >= 4, "ext_product needs N >= 4");
    double h[4], l[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = xh[q];
        l[q] = xl[q];
    }
#pragma unroll
    for (int i = 4; i < N; ++i) ext_mul(h[i & 3], l[i & 3], xh[i], xl[i]);
    ext_mul(h[0], l[0], h[1], l[1]);
    ext_mul(h[2], l[2], h[3], l[3]);
    ext_mul(h[0], l[0], h[2], l[2]);
    ph = h[0];
    pl = l[0];
}

// Adds prod_i x_i (NEG: subtracts it), a double-double, to the lane partial
// (sh, sl): a two-sum of the high parts, then the low parts and a second
// two-sum.  Contraction is off and the product is never negated: a negated
// product in a contracting scope can be rebuilt as a new multiply and fused
// into the add, which would count its rounding error (already in pl) twice.
template <int N, bool NEG>
__device__ __forceinline__ void ext_term(const double (&xh)[N], const double (&xl)[N],
                                         double &sh, double &sl)
{
#pragma clang fp contract(off)
    double ph, pl;
    ext_product<N>(xh, xl, ph, pl);
    const double s = NEG ? sh - ph : sh + ph;
    const double bb = s - sh;
    const double t = NEG ? (sh - (s - bb)) - (ph + bb) : (sh - (s - bb)) + (ph - bb);
    const double u = NEG ? t + (sl - pl) : t + (sl + pl);
    const double s2 = s + u;
    const double bb2 = s2 - s;
    sl = (s - (s2 - bb2)) + (u - bb2);
    sh = s2;
}

template <int N>
__global__ __launch_bounds__(kBlock) void sweep_dense_ext(const double *__restrict__ split,
                                                          dd *__restrict__ partials, int c, int r,
                                                          uint32_t l_begin, uint32_t l_end,
                                                          int accumulate)
{
    __shared__ dd red[kWavesPerBlock];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = uniform_wave_index();
    const uint64_t K = lane_chunk_index(wave, lane);
    const uint32_t kb = uint32_t(wave & 1u);
    const uint64_t g0 = K << c;
    const uint64_t hbits = (g0 ^ (g0 >> 1)) >> c;
    const uint32_t rmask = (1u << r) - 1u;

    double xh[N], xl[N];
    double sh = 0.0, sl = 0.0;  // lane partial, double-double
    // Two steps per trip (launch ranges and re-seed intervals are even): the
    // even step l re-seeds or flips column ctz(l) >= 1 and adds its term, the
    // odd step flips column 0, at a fixed address whose loads can be issued
    // during the even step, and subtracts its term ((-1)^g = (-1)^l, c >= 1).
    for (uint32_t l = l_begin; l < l_end; l += 2u) {
        if ((l & rmask) == 0) {
            ext_reseed<N>(xh, xl, split, hbits, gray_low(l, kb, c), c);
        } else {
            const int j = __builtin_ctz(l);
            const bool add = (gray_low(l, kb, c) >> j) & 1u;
            ext_flip_column<N>(xh, xl, split + (add ? 0 : 2 * N * N) + j * N);
        }
        ext_term<N, false>(xh, xl, sh, sl);
        const bool add0 = gray_low(l + 1u, kb, c) & 1u;
        ext_flip_column<N>(xh, xl, split + (add0 ? 0 : 2 * N * N));
        ext_term<N, true>(xh, xl, sh, sl);
    }
    const dd tot = block_reduce_dd(dd{sh, sl}, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = accumulate ? dd_add(partials[blockIdx.x], tot) : tot;
}

template <int N>
static void launch_ext_n(const SweepPlan &p, const SweepOptions &o, const double *split,
                         dd *partials, hipStream_t stream)
{
    const int64_t C = int64_t(1) << p.log2_chunk;
    const int64_t span = dense_launch_span(N, p, o);
    const int64_t nl = C / span;
    const int64_t first = std::min(o.first_launch, nl);
    const int64_t end = o.launch_count > 0 ? std::min(nl, first + o.launch_count) : nl;
    for (int64_t i = first; i < end; ++i) {
        const int64_t l0 = i * span;
        hipLaunchKernelGGL((sweep_dense_ext<N>), dim3(unsigned(p.blocks)), dim3(kBlock), 0, stream,
                           split, partials, p.log2_chunk, o.log2_reseed, uint32_t(l0),
                           uint32_t(l0 + span), int(l0 > 0));
    }
}

using ExtLauncher = void (*)(const SweepPlan &, const SweepOptions &, const double *, dd *,
                             hipStream_t);

template <int... Ns>
struct ExtTable {
    static ExtLauncher get(int n)
    {
        ExtLauncher f = nullptr;
        ((n == Ns ? (f = &launch_ext_n<Ns>, 0) : 0), ...);
        return f;
    }
};

using DenseExtTable =
    ExtTable<13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32, 33,
             34, 35, 36, 37, 38, 39, 40, 41, 42, 43, 44, 45, 46, 47, 48>;

// Chunk steps per launch: the sweep runs over the full grid as consecutive
// ranges of each lane's chunk of at most max_steps_per_launch subset-steps
// per launch (one launch for the usual sizes); a power-of-two number of
// re-seed intervals (and blocks), so every range is whole and starts on a
// re-seed boundary.

int launch_dense_ext(int n, const double *A, int64_t lda, double *out, const SweepOptions &o,
                     char *ws, hipStream_t stream)
{
    const SweepPlan p = dense_plan(n, o);
    if (n < kExtMinN || n > kExtMaxN || p.log2_chunk < 1) return PERM_EUNSUPPORTED;
    ExtLauncher f = DenseExtTable::get(n);
    if (!f) return PERM_EUNSUPPORTED;
    const DenseWs L = dense_ws_layout(n, 1, dense_ws_blocks(n));
    double *split = reinterpret_cast<double *>(ws + L.ext);
    dd *partials = reinterpret_cast<dd *>(ws + L.partials);
    hipLaunchKernelGGL(prep_dense_ext, dim3(1), dim3(kBlock), 0, stream, n, A, lda, split);
    SweepOptions oo = o;
    if (oo.log2_reseed < 1 || oo.log2_reseed > p.log2_chunk) oo.log2_reseed = p.log2_chunk;
    f(p, oo, split, partials, stream);
    hipLaunchKernelGGL(finalize_partials, dim3(1), dim3(kBlock), 0, stream, partials, p.blocks, 1,
                       (n & 1) ? 2.0 : -2.0, out);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
