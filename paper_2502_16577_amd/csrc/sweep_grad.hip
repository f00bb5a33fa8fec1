// Permanent and its gradient dperm/dA in one Gray-walk sweep.
//
// With tau_j(g) = +1 when column j is in S_g or j = n-1 and -1 otherwise,
// x_i(g) = (1/2) sum_j tau_j(g) a_ij, so differentiating the Nijenhuis-Wilf
// sum of Algorithm 1 term by term gives
//     dperm/da_kl = (-1)^(n-1) sum_g (-1)^g L_k(g) tau_l(g),
//     L_k(g) = prod_{i != k} x_i(g)  (leave-one-out products).
// Per subset the kernel forms L by a prefix and a suffix product pass (no
// division, so zeros in x are harmless), and the rank-1 updates L tau^T of
// the 64 subsets a wave holds at one step are one FP64 MFMA contraction:
//     G (n x n) += V (n x 64) * T (64 x n),   V = L^T, T = (-1)^g tau,
// as 16 x v_mfma_f64_16x16x4f64 per 16x16 output tile.  V goes through LDS
// to get from lane-per-subset to the MFMA operand layout; T is computed in
// registers from the Gray code of the subset each lane stands for.
//
// MFMA operand layout (gfx950, 64 lanes): A[i][k] at lane i + 16k,
// B[k][j] at lane j + 16k, D[i][j] at lane j + 16 (i mod 4), register i / 4.
// The MFMA accumulators are folded every 32 steps into per-wave double-double
// accumulators in global memory, so plain FP64 accumulation never spans more
// than 2048 terms.
#include "sweep_common.h"

namespace perm {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kGradBlock = 64;  // one wave per block
constexpr int kFlushPairs = 16;  // fold MFMA accumulators every 16 step pairs

// Complex or real scalar helpers (CPLX selects; imaginary parts unused if real).
template <bool CPLX>
struct Num {
    __device__ __forceinline__ static void mul(double &ar, double &ai, double br, double bi)
    {
        if constexpr (CPLX) {
            const double r = ar * br - ai * bi;
            const double i = ar * bi + ai * br;
            ar = r;
            ai = i;
        } else {
            ar *= br;
        }
    }
};

// One lane, n <= 10: Algorithm 1 with the gradient formula above, directly.
__global__ void serial_grad(int n, int cplx, const double *__restrict__ acol,
                            const double *__restrict__ aneg, const double *__restrict__ x0,
                            dd *__restrict__ perm_part, double *__restrict__ grad_out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int w = cplx ? 2 : 1;
    double xr[10], xi[10];
    double gr[100], gi[100];
    for (int i = 0; i < n; ++i) {
        xr[i] = x0[w * i];
        xi[i] = cplx ? x0[w * i + 1] : 0.0;
    }
    for (int q = 0; q < n * n; ++q) gr[q] = gi[q] = 0.0;
    double sr = 0.0, er = 0.0, si = 0.0, ei = 0.0;
    const uint32_t steps = 1u << (n - 1);
    for (uint32_t g = 0; g < steps; ++g) {
        if (g) {
            const int j = __builtin_ctz(g);
            const bool add = ((g ^ (g >> 1)) >> j) & 1u;
            const double *a = (add ? acol : aneg) + w * j * n;
            for (int i = 0; i < n; ++i) {
                xr[i] += a[w * i];
                if (cplx) xi[i] += a[w * i + 1];
            }
        }
        const uint32_t gray = g ^ (g >> 1);
        const double sg = (g & 1u) ? -1.0 : 1.0;
        double pr = 1.0, pi = 0.0;
        for (int i = 0; i < n; ++i) {
            if (cplx) Num<true>::mul(pr, pi, xr[i], xi[i]);
            else pr *= xr[i];
        }
        acc_add(sr, er, sg * pr);
        acc_add(si, ei, sg * pi);
        for (int k = 0; k < n; ++k) {
            double lr = 1.0, li = 0.0;
            for (int i = 0; i < n; ++i)
                if (i != k) {
                    if (cplx) Num<true>::mul(lr, li, xr[i], xi[i]);
                    else lr *= xr[i];
                }
            for (int l = 0; l < n; ++l) {
                const double tau = (l == n - 1 || ((gray >> l) & 1u)) ? 1.0 : -1.0;
                gr[k * n + l] += sg * tau * lr;
                gi[k * n + l] += sg * tau * li;
            }
        }
    }
    perm_part[0] = dd{sr, er};
    perm_part[1] = dd{si, ei};
    const double sgn = (n & 1) ? 1.0 : -1.0;  // (-1)^(n-1)
    for (int q = 0; q < n * n; ++q) {
        grad_out[w * q] = sgn * gr[q];
        if (cplx) grad_out[w * q + 1] = sgn * gi[q];
    }
}

template <int N, bool CPLX>
struct GradShape {
    static constexpr int MT = (N + 15) / 16;     // 16-row tiles of G
    static constexpr int NP = 16 * MT;           // padded order
    static constexpr int LDS_STRIDE = NP + 1;    // doubles per lane row in LDS
    static constexpr int COMPS = CPLX ? 2 : 1;
};


// Per-wave accumulator buffer (double-double, lane-contiguous for coalescing):
// acc[wave][slot][lane], slot = ((w * MT + a) * MT + b) * 4 + e holds
// G[16a + lane/16 + 4e][16b + lane%16] of component w.
template <int N, bool CPLX>
__global__ __launch_bounds__(kGradBlock) void sweep_grad(const double *__restrict__ acol,
                                                         const double *__restrict__ aneg,
                                                         const double *__restrict__ x0,
                                                         dd *__restrict__ perm_part,
                                                         dd *__restrict__ grad_acc, int c, int r)
{
    using S = GradShape<N, CPLX>;
    constexpr int MT = S::MT;
    constexpr int W = S::COMPS;  // doubles per matrix entry
    constexpr int SLOTS = W * MT * MT * 4;
    __shared__ double vs[W][kWave * S::LDS_STRIDE];

    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = uint64_t(blockIdx.x);  // one wave per block
    const uint64_t K = lane_chunk_index(wave, lane);
    const uint32_t kb = uint32_t(wave & 1u);
    const uint64_t g0 = K << c;
    const uint64_t hbits = (g0 ^ (g0 >> 1)) >> c;
    const uint32_t C = 1u << c;
    const uint32_t rmask = (1u << r) - 1u;
    const int jcol0 = int(lane & 15u);
    dd *gacc = grad_acc + wave * size_t(SLOTS) * kWave + lane;

    double xr[N], xi[N];
    v4d accm[W][MT][MT];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int b = 0; b < MT; ++b) accm[w][a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < SLOTS; ++t) gacc[size_t(t) * kWave] = dd{0.0, 0.0};
    double sr = 0.0, er = 0.0, si = 0.0, ei = 0.0;

    auto reseed_x = [&](uint32_t l) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            xr[i] = x0[W * i];
            xi[i] = CPLX ? x0[W * i + 1] : 0.0;
        }
        for (int j = c; j < N - 1; ++j) {
            const double f = ((hbits >> (j - c)) & 1u) ? 1.0 : 0.0;
            const double *a = acol + W * j * N;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                xr[i] = __builtin_fma(f, a[W * i], xr[i]);
                if (CPLX) xi[i] = __builtin_fma(f, a[W * i + 1], xi[i]);
            }
        }
        uint32_t low = gray_low(l, kb, c);
        while (low) {
            const int j = __builtin_ctz(low);
            low &= low - 1u;
            const double *a = acol + W * j * N;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                xr[i] += a[W * i];
                if (CPLX) xi[i] += a[W * i + 1];
            }
        }
    };
    auto flip = [&](int j, bool add) {
        const double *a = (add ? acol : aneg) + W * j * N;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            xr[i] += a[W * i];
            if (CPLX) xi[i] += a[W * i + 1];
        }
    };

    // One subset per lane at local step l: the term, the leave-one-out
    // products into LDS (the prefix pass writes, the suffix pass finishes in
    // place), then the MFMA contraction of the wave's 64 rank-1 updates.
    auto step = [&](uint32_t l) {
        const bool neg = l & 1u;  // (-1)^g = (-1)^l
        double *vr = &vs[0][lane * S::LDS_STRIDE];
        double *vi = &vs[W - 1][lane * S::LDS_STRIDE];
        double pr = 1.0, pi = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            vr[i] = pr;
            if (CPLX) vi[i] = pi;
            Num<CPLX>::mul(pr, pi, xr[i], xi[i]);
        }
        acc_add(sr, er, neg ? -pr : pr);
        if (CPLX) acc_add(si, ei, neg ? -pi : pi);
        double sufr = 1.0, sufi = 0.0;
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
            double lr = vr[i], li = CPLX ? vi[i] : 0.0;
            Num<CPLX>::mul(lr, li, sufr, sufi);
            vr[i] = lr;
            if (CPLX) vi[i] = li;
            Num<CPLX>::mul(sufr, sufi, xr[i], xi[i]);
        }

        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        const uint64_t glow = gray_low(l, kb, c);
        const double sg = neg ? -1.0 : 1.0;
#pragma unroll 2
        for (int q = 0; q < 16; ++q) {
            const uint32_t kl = uint32_t(4 * q) + (lane >> 4);  // subset lane of this K row
            const uint64_t gq = lane_chunk_index(wave, kl) << c;
            const uint64_t gray = (((gq ^ (gq >> 1)) >> c) << c) | glow;
            double bop[MT];
#pragma unroll
            for (int b = 0; b < MT; ++b) {
                const int j = 16 * b + jcol0;
                double t = ((gray >> j) & 1u) ? sg : -sg;
                if (j == N - 1) t = sg;
                if (j >= N) t = 0.0;
                bop[b] = t;
            }
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const int i = 16 * a + jcol0;  // A row = lane % 16
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const double aop = (i < N) ? vs[w][kl * S::LDS_STRIDE + i] : 0.0;
#pragma unroll
                    for (int b = 0; b < MT; ++b)
                        accm[w][a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[b],
                                                                             accm[w][a][b], 0, 0, 0);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };

    auto fold = [&]() {
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
            for (int a = 0; a < MT; ++a)
#pragma unroll
                for (int b = 0; b < MT; ++b) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        dd *p = gacc + size_t(((w * MT + a) * MT + b) * 4 + e) * kWave;
                        const dd v = *p;
                        double s, t;
                        two_sum(v.hi, accm[w][a][b][e], s, t);
                        *p = dd{s, v.lo + t};
                    }
                    accm[w][a][b] = v4d{0.0, 0.0, 0.0, 0.0};
                }
    };

    uint32_t pairs = 0;
    for (uint32_t l = 0; l < C; l += 2) {
        if ((l & rmask) == 0) {
            reseed_x(l);
        } else {
            const int j = __builtin_ctz(l);
            flip(j, (gray_low(l, kb, c) >> j) & 1u);
        }
        step(l);
        flip(0, gray_low(l + 1, kb, c) & 1u);
        step(l + 1);
        if (++pairs == kFlushPairs) {
            fold();
            pairs = 0;
        }
    }
    fold();

    const dd pr = wave_reduce_dd(dd{sr, er});
    const dd pim = wave_reduce_dd(dd{si, ei});
    if (lane == 0) {
        perm_part[wave * 2] = pr;
        perm_part[wave * 2 + 1] = pim;
    }
}

// Sums the per-wave accumulators in a fixed order.  One block per entry
// (i, j, component); its threads stride over the waves, then reduce in LDS.
// Writes (-1)^(n-1) G row-major (interleaved re, im if complex); block 0
// also writes the permanent.
template <int N, bool CPLX>
__global__ __launch_bounds__(kBlock) void finalize_grad(const dd *__restrict__ perm_part,
                                                        const dd *__restrict__ grad_acc,
                                                        int64_t waves,
                                                        double *__restrict__ out_perm,
                                                        double *__restrict__ out_grad)
{
    using S = GradShape<N, CPLX>;
    constexpr int MT = S::MT;
    constexpr int W = S::COMPS;
    constexpr int SLOTS = W * MT * MT * 4;
    __shared__ dd red[kWavesPerBlock];
    const int e_id = int(blockIdx.x);  // entry = (i * N + j) * W + w
    const int w = e_id % W;
    const int ij = e_id / W;
    const int i = ij / N, j = ij % N;
    const int a = i / 16, b = j / 16;
    const int ii = i % 16, jj = j % 16;
    const int lane = jj + 16 * (ii % 4);
    const int e = ii / 4;
    const int slot = ((w * MT + a) * MT + b) * 4 + e;
    dd acc = dd{0.0, 0.0};
    for (int64_t v = threadIdx.x; v < waves; v += kBlock)
        acc = dd_add(acc, grad_acc[(v * SLOTS + slot) * kWave + lane]);
    const dd t = block_reduce_dd(acc, red);
    const double sgn = (N & 1) ? 1.0 : -1.0;
    if (threadIdx.x == 0) out_grad[e_id] = sgn * (t.hi + t.lo);
    if (blockIdx.x == 0) {
        for (int q = 0; q < W; ++q) {
            dd pacc = dd{0.0, 0.0};
            for (int64_t v = threadIdx.x; v < waves; v += kBlock)
                pacc = dd_add(pacc, perm_part[v * 2 + q]);
            const dd pt = block_reduce_dd(pacc, red);
            if (threadIdx.x == 0) out_perm[q] = 2.0 * sgn * (pt.hi + pt.lo);
        }
    }
}

template <int N, bool CPLX>
static void launch_grad_n(int64_t waves, const double *acol, const double *aneg, const double *x0,
                          dd *pp, dd *gp, int c, int r, double *out_perm, double *out_grad,
                          hipStream_t stream)
{
    hipLaunchKernelGGL((sweep_grad<N, CPLX>), dim3(unsigned(waves)), dim3(kGradBlock), 0, stream,
                       acol, aneg, x0, pp, gp, c, r);
    hipLaunchKernelGGL((finalize_grad<N, CPLX>), dim3(unsigned(N * N * (CPLX ? 2 : 1))),
                       dim3(kBlock), 0, stream, pp, gp, waves, out_perm, out_grad);
}

using GradLauncher = void (*)(int64_t, const double *, const double *, const double *, dd *, dd *,
                              int, int, double *, double *, hipStream_t);

template <bool CPLX, int... Ns>
struct GradTable {
    static GradLauncher get(int n)
    {
        GradLauncher f = nullptr;
        ((n == Ns ? (f = &launch_grad_n<Ns, CPLX>, 0) : 0), ...);
        return f;
    }
};

using GradF64Table = GradTable<false, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25,
                               26, 27, 28, 29, 30, 31, 32>;
using GradC128Table = GradTable<true, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25,
                                26, 27, 28, 29, 30, 31, 32>;

GradPlan plan_grad(int n)
{
    GradPlan p;
    p.n = n;
    if (n <= kGradSerialMaxN) {
        p.waves = 1;
        p.log2_chunk = n > 0 ? n - 1 : 0;
        p.log2_reseed = p.log2_chunk;
        return p;
    }
    const int total = n - 1;
    int lanes_log = total - 2;
    if (lanes_log > 16) lanes_log = 16;
    if (lanes_log < 7) lanes_log = 7;
    p.log2_chunk = total - lanes_log;
    p.log2_reseed = p.log2_chunk < 9 ? p.log2_chunk : 9;
    p.waves = (int64_t(1) << lanes_log) / kWave;
    return p;
}

int launch_grad(int n, bool cplx, const void *A, int64_t lda, void *out_perm, void *out_grad,
                char *ws, hipStream_t stream)
{
    const GradPlan p = plan_grad(n);
    const GradWs L = grad_ws_layout(n, cplx ? 2 : 1, p.waves);
    double *acol = reinterpret_cast<double *>(ws + L.acol);
    double *aneg = reinterpret_cast<double *>(ws + L.aneg);
    double *x0 = reinterpret_cast<double *>(ws + L.x0);
    dd *pp = reinterpret_cast<dd *>(ws + L.perm_partials);
    dd *gp = reinterpret_cast<dd *>(ws + L.grad_partials);
    if (cplx)
        hipLaunchKernelGGL(prep_dense_c128, dim3(1), dim3(kBlock), 0, stream, n,
                           static_cast<const perm_c128 *>(A), lda, acol, aneg, x0);
    else
        hipLaunchKernelGGL(prep_dense_f64, dim3(1), dim3(kBlock), 0, stream, n,
                           static_cast<const double *>(A), lda, acol, aneg, x0);
    if (n <= kGradSerialMaxN) {
        hipLaunchKernelGGL(serial_grad, dim3(1), dim3(64), 0, stream, n, int(cplx), acol, aneg, x0,
                           pp, static_cast<double *>(out_grad));
        hipLaunchKernelGGL(finalize_partials, dim3(1), dim3(kBlock), 0, stream, pp, int64_t(1),
                           cplx ? 2 : 1, (n & 1) ? 2.0 : -2.0, static_cast<double *>(out_perm));
        return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
    }
    GradLauncher f = cplx ? GradC128Table::get(n) : GradF64Table::get(n);
    if (!f) return PERM_EUNSUPPORTED;
    f(p.waves, acol, aneg, x0, pp, gp, p.log2_chunk, p.log2_reseed,
      static_cast<double *>(out_perm), static_cast<double *>(out_grad), stream);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
