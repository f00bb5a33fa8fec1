// Exact permanent of a 0/1 matrix: the Gray-code Ryser / Nijenhuis-Wilf
// sweep on y = 2x (integral: y_i = 2 a_{i,n-1} - r_i, each flip adds +-2 to
// the rows of column j), reduced modulo several primes p_k just above 2^50.
//
// Per step every lane forms the exact product of its y_i in FP64: rows are
// grouped so that a group's product is at most 2^50 < p_k for any
// |y_i| <= n, so each group product is an exact integer, already a residue,
// and the term is zero exactly when one group product is.  Terms that are
// zero are dropped (for random 0/1 matrices most are: about 91 % at n = 32,
// Bernoulli(1/2)).  Lanes with a nonzero term append their group products to
// a per-wave queue in LDS; when the queue holds 64 entries the whole wave
// drains it, one entry per lane, multiplying the group products modulo every
// prime with all lanes busy.  The modular products are FP64 operations
// (mulmod50): residues are kept as signed integers in doubles.  Residues are
// reduced across lanes, blocks and the grid by modular addition (exact, so
// the order does not matter).
#include "sweep_common.h"

namespace perm {

// a * b mod p as a signed residue of magnitude <= 0.875 p, for integers
// |a|, |b| <= p held in doubles, p in (2^50, 2^50 + 2^40), pinv = fl(1/p).
// a b = h + l exactly (error-free product); q = rint(h pinv) is within 0.875
// of a b / p (three roundings of relative size 2^-53 on a quotient below
// 2^50, plus the rounding to an integer); q p = qh + ql exactly; every
// difference below is an integer of magnitude < 2^52, hence exact, and
// (h - qh) + (l - ql) = a b - q p.  Contraction is off so the compiler keeps
// exactly these operations.
__device__ __forceinline__ double mulmod50(double a, double b, double p, double pinv)
{
#pragma clang fp contract(off)
    const double h = a * b;
    const double l = __builtin_fma(a, b, -h);
    const double q = __builtin_rint(h * pinv);
    const double qh = q * p;
    const double ql = __builtin_fma(q, p, -qh);
    return (h - qh) + (l - ql);
}

// (acc + t) mod p, signed, magnitude <= p / 2 + 1, for |acc|, |t| <= p.
__device__ __forceinline__ double addmod50(double acc, double t, double p, double pinv)
{
#pragma clang fp contract(off)
    const double s = acc + t;  // integers below 2^52: exact
    return __builtin_fma(-__builtin_rint(s * pinv), p, s);
}

// A signed residue |v| < p as the representative in [0, p).
__device__ __forceinline__ uint64_t residue_u64(double v, double p)
{
    return uint64_t(v < 0.0 ? v + p : v);
}

__device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t p)
{
    const uint64_t s = a + b;  // a, b < p < 2^51: no overflow
    return s >= p ? s - p : s;
}

// Number of bits of the largest possible |y_i| (<= n) and rows per exact group.
template <int N>
struct BinGroups {
    static constexpr int bits = (N <= 2) ? 1 : (N <= 4) ? 2 : (N <= 8) ? 3 : (N <= 16) ? 4
                               : (N <= 32) ? 5 : 6;
    static constexpr int G = 50 / bits;                 // |group product| <= 2^50 < p
    static constexpr int M = (N + G - 1) / G;           // number of groups
};

// Stages the matrix: ycol[j*n + i] = 2 a_ij, yneg = -2 a_ij, y0[i] = 2 a_{i,n-1} - r_i.
__global__ __launch_bounds__(kBlock) void prep_binary(int n, const double *__restrict__ dense01,
                                                      double *__restrict__ ycol,
                                                      double *__restrict__ yneg,
                                                      double *__restrict__ y0)
{
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int j = idx / n;
        const int i = idx - j * n;
        const double v = 2.0 * dense01[int64_t(i) * n + j];
        ycol[idx] = v;
        yneg[idx] = -v;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += dense01[int64_t(i) * n + j];
        y0[i] = 2.0 * dense01[int64_t(i) * n + n - 1] - r;
    }
}

// n <= 12: one lane; the whole alternating sum R is below 2^11 * 12! < 2^40,
// so it is accumulated exactly in int64 and reduced once per prime.
__global__ void serial_binary(int n, const double *__restrict__ ycol,
                              const double *__restrict__ yneg, const double *__restrict__ y0,
                              int nprimes, BinaryPrimes P, uint64_t *__restrict__ partials)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double y[12];
    for (int i = 0; i < n; ++i) y[i] = y0[i];
    double p = 1.0;
    for (int i = 0; i < n; ++i) p *= y[i];
    int64_t R = int64_t(p);
    const uint32_t steps = 1u << (n - 1);
    for (uint32_t g = 1; g < steps; ++g) {
        const int j = __builtin_ctz(g);
        const bool add = ((g ^ (g >> 1)) >> j) & 1u;
        const double *a = (add ? ycol : yneg) + j * n;
        p = 1.0;
        for (int i = 0; i < n; ++i) {
            y[i] += a[i];
            p *= y[i];
        }
        R += (g & 1u) ? -int64_t(p) : int64_t(p);
    }
    for (int k = 0; k < nprimes; ++k) {
        const uint64_t pk = uint64_t(P.p[k]);
        const int64_t m = R % int64_t(pk);
        partials[k] = m < 0 ? uint64_t(m + int64_t(pk)) : uint64_t(m);
    }
}

constexpr int kQueueCap = 128;  // entries per wave; at most 63 wait between drains

// Steps per block of the walk: 2^U (requires c > U, as the plan gives).
template <int N>
constexpr int binary_unroll() { return N >= 14 ? 4 : 3; }

template <int N>
__device__ __forceinline__ void group_products(const double (&y)[N],
                                               double (&gp)[BinGroups<N>::M])
{
    constexpr int G = BinGroups<N>::G;
    constexpr int M = BinGroups<N>::M;
#pragma unroll
    for (int m = 0; m < M; ++m) gp[m] = y[m * G];
#pragma unroll
    for (int t = 1; t < G; ++t) {
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (m * G + t < N) gp[m] *= y[m * G + t];
    }
}

// One queue entry: the signed group products of one nonzero term, multiplied
// modulo every prime into the lane's residues.
template <int M>
__device__ __forceinline__ void drain_entry(const double *__restrict__ q, int slot, int nprimes,
                                            const BinaryPrimes &P, double (&acc)[kMaxPrimes])
{
    double g[M];
#pragma unroll
    for (int m = 0; m < M; ++m) g[m] = q[m * kQueueCap + slot];
#pragma unroll
    for (int k = 0; k < kMaxPrimes; ++k) {
        if (k < nprimes) {
            double t = g[0];  // |g| <= 2^50 < p: already a residue
#pragma unroll
            for (int m = 1; m < M; ++m) t = mulmod50(t, g[m], P.p[k], P.pinv[k]);
            acc[k] = addmod50(acc[k], t, P.p[k], P.pinv[k]);
        }
    }
}

// Exact zero-block skipping (skip_b > 0): inside an aligned block of 2^b
// local steps only columns < b flip, so the first `nfrozen` rows (the host
// orders rows so that these have no nonzero in columns < b) keep their y for
// the whole block.  If one of them is zero for every lane of the wave, all
// 2^b terms of the block are zero and the block reduces to its net effect, a
// single flip of column b - 1.
template <int N>
__global__ __launch_bounds__(kBlock) void sweep_binary(const double *__restrict__ ycol,
                                                       const double *__restrict__ yneg,
                                                       const double *__restrict__ y0, int c,
                                                       int nprimes, int skip_b, int nfrozen,
                                                       const BinaryPrimes P,
                                                       uint64_t *__restrict__ partials)
{
    constexpr int M = BinGroups<N>::M;
    __shared__ double queue[kWavesPerBlock][M * kQueueCap];
    __shared__ uint64_t red[kWavesPerBlock][kMaxPrimes];

    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + wib;
    const uint64_t K = lane_chunk_index(wave, lane);
    const uint32_t kb = uint32_t(wave & 1u);
    const uint64_t g0 = K << c;
    const uint64_t hbits = (g0 ^ (g0 >> 1)) >> c;
    const uint32_t C = 1u << c;
    double *q = queue[wib];

    // Exact seed (integers: no drift, no re-seeding needed).
    double y[N];
#pragma unroll
    for (int i = 0; i < N; ++i) y[i] = y0[i];
    for (int j = c; j < N - 1; ++j) {
        const double f = ((hbits >> (j - c)) & 1u) ? 1.0 : 0.0;
        const double *a = ycol + j * N;
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] = __builtin_fma(f, a[i], y[i]);
    }
    {
        uint32_t low = gray_low(0, kb, c);
        while (low) {
            const int j = __builtin_ctz(low);
            low &= low - 1u;
            const double *a = ycol + j * N;
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] += a[i];
        }
    }

    double acc[kMaxPrimes];  // signed residues, |acc| <= p / 2 + 1
#pragma unroll
    for (int k = 0; k < kMaxPrimes; ++k) acc[k] = 0.0;
    uint32_t count = 0;  // wave-uniform queue length

    auto push_term = [&](bool negative) {
        double gp[M];
        group_products<N>(y, gp);
        // the term is nonzero iff the smallest |group product| is (FP64
        // minima: no lane-mask logic on the scalar unit)
        double mn = __builtin_fabs(gp[0]);
#pragma unroll
        for (int m = 1; m < M; ++m) mn = __builtin_fmin(mn, __builtin_fabs(gp[m]));
        const bool nz = mn != 0.0;
        if (negative) gp[0] = -gp[0];
        const uint64_t ballot = __ballot(nz);
        if (ballot == 0) return;
        const uint32_t before = __builtin_amdgcn_mbcnt_hi(uint32_t(ballot >> 32),
                                                          __builtin_amdgcn_mbcnt_lo(uint32_t(ballot), 0u));
        const uint32_t pc = uint32_t(__builtin_popcountll(ballot));
        // Every lane stores, without a branch: nonzero terms to the next
        // free slots, the others past them (slot <= count + 63 < kQueueCap,
        // as count < 64 here), where a later push overwrites them before a
        // drain reads that far.
        const uint32_t slot = nz ? count + before : count + pc + (lane - before);
#pragma unroll
        for (int m = 0; m < M; ++m) q[m * kQueueCap + slot] = gp[m];
        count += pc;
        if (count >= 64) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            drain_entry<M>(q, int(count - 64 + lane), nprimes, P, acc);
            count -= 64;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    };

    // Blocks of 2^U steps as in the real sweep: only the block's first step
    // flips a column chosen at run time; step l + m flips column ctz(m) with
    // a sign fixed by m (by bit U of l for m = 2^(U-1)), read from a constant
    // address.  Zero-block skipping works on aligned blocks of 2^skip_b >= 2^U
    // steps, tested at block starts.
    constexpr int U = binary_unroll<N>();
    constexpr uint32_t B = 1u << U;
    const uint32_t bmask = skip_b > 0 ? (1u << skip_b) - 1u : 0u;
    for (uint32_t l = 0; l < C; l += B) {
        if (l != 0) {
            const int j = __builtin_ctz(l);
            const bool add = (gray_low(l, kb, c) >> j) & 1u;
            const double *a = (add ? ycol : yneg) + j * N;
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] += a[i];
        }
        if (skip_b > 0 && (l & bmask) == 0) {
            double pf = 1.0;
#pragma unroll
            for (int i = 0; i < N; ++i)
                if (i < nfrozen) pf *= y[i];
            if (__ballot(pf != 0.0) == 0) {
                // net effect of the block: column b - 1 flips once (at l + 2^(b-1))
                const uint32_t lh = l + (1u << (skip_b - 1));
                const bool add = (gray_low(lh, kb, c) >> (skip_b - 1)) & 1u;
                const double *a = (add ? ycol : yneg) + (skip_b - 1) * N;
#pragma unroll
                for (int i = 0; i < N; ++i) y[i] += a[i];
                l += bmask + 1u - B;  // the loop adds B: next step is the next block's start
                continue;
            }
        }
        push_term(false);  // (-1)^g = (-1)^m, l even
#pragma unroll
        for (uint32_t m = 1; m < B; ++m) {
            const int j = __builtin_ctz(m);
            const bool neg = (j + 1 < U) ? ((m >> (j + 1)) & 1u) : ((l >> U) & 1u);
            // a fresh opaque offset per step keeps the compiler from hoisting
            // these constant-address column loads into long-lived SGPRs
            uint32_t zero = 0;
            asm volatile("" : "+s"(zero));
            const double *a = (neg ? yneg : ycol) + j * N + zero;
#pragma unroll
            for (int i = 0; i < N; ++i) y[i] += a[i];
            push_term((m & 1u) != 0u);
        }
    }
    // drain what is left (fewer than 64 entries)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < count) drain_entry<M>(q, int(lane), nprimes, P, acc);

    // wave reduction by modular addition, then across the block
#pragma unroll
    for (int k = 0; k < kMaxPrimes; ++k) {
        if (k < nprimes) {
            const uint64_t p = uint64_t(P.p[k]);
            uint64_t v = residue_u64(acc[k], P.p[k]);
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const uint64_t o = __shfl_xor(v, off, 64);
                v = addmod(v, o, p);
            }
            if (lane == 0) red[wib][k] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < uint32_t(nprimes)) {
        const int k = int(threadIdx.x);
        const uint64_t p = uint64_t(P.p[k]);
        uint64_t v = 0;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) v = addmod(v, red[w][k], p);
        partials[uint64_t(blockIdx.x) * nprimes + k] = v;
    }
}

__global__ __launch_bounds__(kBlock) void finalize_residues(const uint64_t *__restrict__ partials,
                                                            int64_t count, int nprimes,
                                                            BinaryPrimes P,
                                                            uint64_t *__restrict__ out)
{
    __shared__ uint64_t red[kBlock];
    for (int k = 0; k < nprimes; ++k) {
        const uint64_t p = uint64_t(P.p[k]);
        uint64_t v = 0;
        for (int64_t b = threadIdx.x; b < count; b += kBlock) v = addmod(v, partials[b * nprimes + k], p);
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = kBlock / 2; s > 0; s >>= 1) {
            if (int(threadIdx.x) < s) red[threadIdx.x] = addmod(red[threadIdx.x], red[threadIdx.x + s], p);
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

template <int N>
static void launch_bin_n(const SweepPlan &p, const double *ycol, const double *yneg,
                         const double *y0, int nprimes, int skip_b, int nfrozen,
                         const BinaryPrimes &P, uint64_t *partials, hipStream_t stream)
{
    hipLaunchKernelGGL(sweep_binary<N>, dim3(unsigned(p.blocks)), dim3(kBlock), 0, stream, ycol,
                       yneg, y0, p.log2_chunk, nprimes, skip_b, nfrozen, P, partials);
}

using BinLauncher = void (*)(const SweepPlan &, const double *, const double *, const double *,
                             int, int, int, const BinaryPrimes &, uint64_t *, hipStream_t);

template <int... Ns>
struct BinTable {
    static BinLauncher get(int n)
    {
        BinLauncher f = nullptr;
        ((n == Ns ? (f = &launch_bin_n<Ns>, 0) : 0), ...);
        return f;
    }
};

using BinaryTable =
    BinTable<13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32, 33,
             34, 35, 36, 37, 38, 39, 40, 41, 42, 43, 44, 45, 46, 47, 48, 49, 50, 51, 52, 53, 54,
             55, 56, 57, 58, 59, 60, 61, 62, 63>;

int launch_binary_residues(int n, const double *dense01, int nprimes, int skip_b, int nfrozen,
                           uint64_t *residues_dev, char *ws, hipStream_t stream)
{
    const SweepPlan p = plan_sweep_fine(n);
    const BinaryWs L = binary_ws_layout(n, p.blocks);
    const BinaryPrimes P = binary_primes();
    double *ycol = reinterpret_cast<double *>(ws + L.ycol);
    double *yneg = reinterpret_cast<double *>(ws + L.yneg);
    double *y0 = reinterpret_cast<double *>(ws + L.y0);
    uint64_t *partials = reinterpret_cast<uint64_t *>(ws + L.partials);
    hipLaunchKernelGGL(prep_binary, dim3(1), dim3(kBlock), 0, stream, n, dense01, ycol, yneg, y0);
    int64_t nparts = 1;
    if (n <= 12) {
        hipLaunchKernelGGL(serial_binary, dim3(1), dim3(64), 0, stream, n, ycol, yneg, y0, nprimes,
                           P, partials);
    } else {
        BinLauncher f = BinaryTable::get(n);
        if (!f) return PERM_EUNSUPPORTED;
        f(p, ycol, yneg, y0, nprimes, skip_b > p.log2_chunk ? 0 : skip_b, nfrozen, P, partials,
          stream);
        nparts = p.blocks;
    }
    hipLaunchKernelGGL(finalize_residues, dim3(1), dim3(kBlock), 0, stream, partials, nparts,
                       nprimes, P, residues_dev);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
