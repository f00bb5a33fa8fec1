// Batched permanents (and gradients) of many small complex matrices of
// uneven order in one persistent launch.
//
// The batch is cut into work items: item (m, w) is wave w of matrix m, and
// covers 64 lanes x 2^c Gray steps of that matrix (lane K = 64 w + lane
// walks g in [K 2^c, (K+1) 2^c)).  A persistent grid of one-wave blocks pulls
// items from an atomic counter, largest matrices first, and dispatches on
// the (wave-uniform) order k to a sweep compiled for that k.  Each item writes
// its own double-double partials (permanent, and G if requested); a
// segmented finalize sums the items of every matrix in a fixed order, so the
// result does not depend on which wave ran which item.
//
// Per item the arithmetic is the one of sweep_grad.hip: x in VGPRs, the
// flipped column read with scalar loads, an exact re-seed of x every 2^r
// steps, leave-one-out products into LDS, and the rank-1 updates of the 64
// subsets of one step contracted with v_mfma_f64_16x16x4f64.  Because the
// lane index enters the Gray code from bit c upwards, the only flip whose sign
// depends on the lane is the one at l = 2^(c-1); r <= c - 1 makes that step a
// re-seed, so every incremental flip is wave-uniform.
#include "batched_internal.h"
#include "sweep_common.h"

namespace perm {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void cmulb(double &ar, double &ai, double br, double bi)
{
    const double r = ar * br - ai * bi;
    const double i = ar * bi + ai * br;
    ar = r;
    ai = i;
}

// Stages every matrix: acol[2(j k + i) + {re,im}], aneg = -acol, x0[2 i + {re,im}]
// at stage + mats[m].stage (doubles).  One block per matrix.
__global__ __launch_bounds__(kBlock) void batched_prep(const BatchMatDev *__restrict__ mats,
                                                       const perm_c128 *__restrict__ data,
                                                       double *__restrict__ stage)
{
    const BatchMatDev M = mats[blockIdx.x];
    const int k = M.k;
    const perm_c128 *A = data + M.data_off;
    double *acol = stage + M.stage;
    double *aneg = acol + 2 * k * k;
    double *x0 = aneg + 2 * k * k;
    for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
        const int j = idx / k, i = idx - j * k;
        const perm_c128 v = A[i * k + j];
        acol[2 * idx] = v.re;
        acol[2 * idx + 1] = v.im;
        aneg[2 * idx] = -v.re;
        aneg[2 * idx + 1] = -v.im;
    }
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        double sr = 0.0, er = 0.0, si = 0.0, ei = 0.0;
        for (int j = 0; j < k; ++j) {
            acc_add(sr, er, A[i * k + j].re);
            acc_add(si, ei, A[i * k + j].im);
        }
        x0[2 * i] = (A[i * k + k - 1].re - 0.5 * sr) - 0.5 * er;
        x0[2 * i + 1] = (A[i * k + k - 1].im - 0.5 * si) - 0.5 * ei;
    }
}

__global__ void batched_reset(uint32_t *counters, int n)
{
    if (int(threadIdx.x) < n) counters[threadIdx.x] = 0u;
}

constexpr int kBatchFoldPairs = 16;

template <int K>
__device__ __forceinline__ void batched_item(const BatchMatDev &M, int w,
                                             const double *__restrict__ stage,
                                             dd *__restrict__ perm_out, dd *__restrict__ g_out,
                                             bool want_grad, double *__restrict__ lds)
{
    constexpr int MT = (K + 15) / 16;
    constexpr int STRIDE = 16 * MT + 1;
    const uint32_t lane = threadIdx.x & 63u;
    const double *acol = stage + M.stage;
    const double *aneg = acol + 2 * K * K;
    const double *x0 = aneg + 2 * K * K;
    const int c = M.c;
    const uint32_t C = 1u << c;
    const uint32_t rmask = (1u << M.r) - 1u;
    const uint64_t lanes_active = (uint64_t(1) << (K - 1)) >> c;
    const uint64_t Kl = uint64_t(w) * kWave + lane;
    const double act = Kl < lanes_active ? 1.0 : 0.0;
    const int jcol0 = int(lane & 15u);

    if (K == 1) {  // one subset: perm = a, G = [1]
        if (lane == 0) {
            perm_out[0] = dd{0.5 * acol[0], 0.0};  // finalize multiplies by 2
            perm_out[1] = dd{0.5 * acol[1], 0.0};
            if (want_grad) {
                g_out[0] = dd{1.0, 0.0};
                g_out[1] = dd{0.0, 0.0};
            }
        }
        return;
    }

    double xr[K], xi[K];
    v4d accm[2][MT][MT];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int b = 0; b < MT; ++b) accm[q][a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    if (want_grad)
        for (int e = int(lane); e < 2 * K * K; e += kWave) g_out[e] = dd{0.0, 0.0};
    double sr = 0.0, er = 0.0, si = 0.0, ei = 0.0;

    auto reseed = [&](uint32_t l) {
        const uint64_t g = (Kl << c) | l;
        const uint64_t gray = g ^ (g >> 1);
#pragma unroll
        for (int i = 0; i < K; ++i) {
            xr[i] = act * x0[2 * i];
            xi[i] = act * x0[2 * i + 1];
        }
        for (int j = 0; j < K - 1; ++j) {
            const double f = ((gray >> j) & 1u) ? act : 0.0;
            const double *a = acol + 2 * j * K;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                xr[i] = __builtin_fma(f, a[2 * i], xr[i]);
                xi[i] = __builtin_fma(f, a[2 * i + 1], xi[i]);
            }
        }
    };
    auto flip = [&](int j, bool add) {
        const double *a = (add ? acol : aneg) + 2 * j * K;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            xr[i] = __builtin_fma(act, a[2 * i], xr[i]);
            xi[i] = __builtin_fma(act, a[2 * i + 1], xi[i]);
        }
    };
    auto step = [&](uint32_t l) {
        const bool neg = l & 1u;
        double *vr = lds + lane * STRIDE;
        double *vi = lds + kWave * STRIDE + lane * STRIDE;
        double pr = 1.0, pi = 0.0;
        if (want_grad) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                vr[i] = pr;
                vi[i] = pi;
                cmulb(pr, pi, xr[i], xi[i]);
            }
        } else {
            double r0 = xr[0], i0 = xi[0], r1 = 1.0, i1 = 0.0;
#pragma unroll
            for (int i = 1; i < K; i += 2) {
                cmulb(r1, i1, xr[i], xi[i]);
                if (i + 1 < K) cmulb(r0, i0, xr[i + 1], xi[i + 1]);
            }
            cmulb(r0, i0, r1, i1);
            pr = r0;
            pi = i0;
        }
        acc_add(sr, er, neg ? -pr : pr);
        acc_add(si, ei, neg ? -pi : pi);
        if (!want_grad) return;
        double sufr = 1.0, sufi = 0.0;
#pragma unroll
        for (int i = K - 1; i >= 0; --i) {
            double lr = vr[i], li = vi[i];
            cmulb(lr, li, sufr, sufi);
            vr[i] = lr;
            vi[i] = li;
            cmulb(sufr, sufi, xr[i], xi[i]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double sg = neg ? -1.0 : 1.0;
#pragma unroll 2
        for (int q = 0; q < 16; ++q) {
            const uint32_t kl = uint32_t(4 * q) + (lane >> 4);
            const uint64_t Kq = uint64_t(w) * kWave + kl;
            const uint64_t g = (Kq << c) | l;
            const uint64_t gray = g ^ (g >> 1);
            const double sq = Kq < lanes_active ? sg : 0.0;
            double bop[MT];
#pragma unroll
            for (int b = 0; b < MT; ++b) {
                const int j = 16 * b + jcol0;
                double t = ((gray >> j) & 1u) ? sq : -sq;
                if (j == K - 1) t = sq;
                if (j >= K) t = 0.0;
                bop[b] = t;
            }
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const int i = 16 * a + jcol0;
                const double are = (i < K) ? lds[kl * STRIDE + i] : 0.0;
                const double aim = (i < K) ? lds[kWave * STRIDE + kl * STRIDE + i] : 0.0;
#pragma unroll
                for (int b = 0; b < MT; ++b) {
                    accm[0][a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(are, bop[b], accm[0][a][b], 0, 0, 0);
                    accm[1][a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim, bop[b], accm[1][a][b], 0, 0, 0);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    auto fold = [&]() {
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int a = 0; a < MT; ++a)
#pragma unroll
                for (int b = 0; b < MT; ++b) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int i = 16 * a + int(lane >> 4) + 4 * e;
                        const int j = 16 * b + jcol0;
                        if (i < K && j < K) {
                            dd *p = g_out + (i * K + j) * 2 + q;
                            const dd v = *p;
                            double s, t;
                            two_sum(v.hi, accm[q][a][b][e], s, t);
                            *p = dd{s, v.lo + t};
                        }
                    }
                    accm[q][a][b] = v4d{0.0, 0.0, 0.0, 0.0};
                }
    };

    uint32_t pairs = 0;
    for (uint32_t l = 0; l < C; l += 2) {
        if ((l & rmask) == 0) {
            reseed(l);
        } else {
            const int j = __builtin_ctz(l);
            flip(j, (((l ^ (l >> 1)) >> j) & 1u) != 0u);
        }
        step(l);
        if (c == 1) {
            reseed(l + 1);  // the column-0 sign depends on the lane when c == 1
        } else {
            const uint32_t l1 = l + 1;
            flip(0, ((l1 ^ (l1 >> 1)) & 1u) != 0u);
        }
        step(l + 1);
        if (want_grad && ++pairs == kBatchFoldPairs) {
            fold();
            pairs = 0;
        }
    }
    if (want_grad) fold();
    const dd pr = wave_reduce_dd(dd{sr, er});
    const dd pim = wave_reduce_dd(dd{si, ei});
    if (lane == 0) {
        perm_out[0] = pr;
        perm_out[1] = pim;
    }
}

template <int K0, int K1>
struct BatchDispatch {
    __device__ static void run(int k, const BatchMatDev &M, int w, const double *stage, dd *pp,
                               dd *gp, bool want_grad, double *lds)
    {
        if (k == K0) batched_item<K0>(M, w, stage, pp, gp, want_grad, lds);
        else if constexpr (K0 < K1) BatchDispatch<K0 + 1, K1>::run(k, M, w, stage, pp, gp, want_grad, lds);
    }
};

// Persistent kernel for the items of orders in [K0, K1].
template <int K0, int K1>
__global__ __launch_bounds__(kWave) void batched_persistent(
    const BatchMatDev *__restrict__ mats, const BatchItemDev *__restrict__ items, int64_t n_items,
    uint32_t *__restrict__ counter, const double *__restrict__ stage,
    dd *__restrict__ perm_parts, dd *__restrict__ g_parts, int want_grad)
{
    constexpr int MT = (K1 + 15) / 16;
    __shared__ double lds[2 * kWave * (16 * MT + 1)];
    for (;;) {
        uint32_t it = 0;
        if (threadIdx.x == 0) it = atomicAdd(counter, 1u);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0, 64));
        if (int64_t(it) >= n_items) break;
        const BatchItemDev I = items[it];
        const BatchMatDev M = mats[I.m];
        dd *pp = perm_parts + 2 * (M.item0 + I.w);
        dd *gp = g_parts + M.gbase + int64_t(I.w) * 2 * M.k * M.k;
        BatchDispatch<K0, K1>::run(M.k, M, I.w, stage, pp, gp, want_grad != 0, lds);
    }
}

// One block per matrix: perm[m] = 2 (-1)^(k-1) sum of item partials, and
// G[m] = (-1)^(k-1) sum of item G partials, in item order.
__global__ __launch_bounds__(kBlock) void batched_finalize(const BatchMatDev *__restrict__ mats,
                                                           const dd *__restrict__ perm_parts,
                                                           const dd *__restrict__ g_parts,
                                                           perm_c128 *__restrict__ out,
                                                           perm_c128 *__restrict__ grad)
{
    __shared__ dd red[kWavesPerBlock];
    const BatchMatDev M = mats[blockIdx.x];
    const int k = M.k;
    const double sgn = (k & 1) ? 1.0 : -1.0;
    for (int q = 0; q < 2; ++q) {
        dd acc = dd{0.0, 0.0};
        for (int w = threadIdx.x; w < M.waves; w += kBlock)
            acc = dd_add(acc, perm_parts[2 * (M.item0 + w) + q]);
        const dd t = block_reduce_dd(acc, red);
        if (threadIdx.x == 0) {
            const double v = 2.0 * sgn * (t.hi + t.lo);
            if (q == 0) out[blockIdx.x].re = v;
            else out[blockIdx.x].im = v;
        }
    }
    if (!grad) return;
    double *gout = reinterpret_cast<double *>(grad + M.data_off);
    for (int e = threadIdx.x; e < 2 * k * k; e += kBlock) {
        dd acc = dd{0.0, 0.0};
        for (int w = 0; w < M.waves; ++w) acc = dd_add(acc, g_parts[M.gbase + int64_t(w) * 2 * k * k + e]);
        gout[e] = sgn * (acc.hi + acc.lo);
    }
}

static void launch_persistent(const BatchLaunch &L, int g, hipStream_t stream)
{
    if (L.n_items[g] <= 0) return;
    const dim3 grid(unsigned(L.grid[g])), block(kWave);
    const int64_t n = L.n_items[g];
    if (g == 0)
        hipLaunchKernelGGL((batched_persistent<1, 16>), grid, block, 0, stream, L.mats, L.items[0], n,
                           L.counters + 0, L.stage, L.perm_parts, L.g_parts, L.want_grad);
    else if (g == 1)
        hipLaunchKernelGGL((batched_persistent<17, 24>), grid, block, 0, stream, L.mats, L.items[1], n,
                           L.counters + 1, L.stage, L.perm_parts, L.g_parts, L.want_grad);
    else
        hipLaunchKernelGGL((batched_persistent<25, 32>), grid, block, 0, stream, L.mats, L.items[2], n,
                           L.counters + 2, L.stage, L.perm_parts, L.g_parts, L.want_grad);
}

int launch_batched(const BatchLaunch &L, hipStream_t stream)
{
    hipLaunchKernelGGL(batched_reset, dim3(1), dim3(64), 0, stream, L.counters, kBatchGroups);
    hipLaunchKernelGGL(batched_prep, dim3(unsigned(L.count)), dim3(kBlock), 0, stream, L.mats, L.data,
                       L.stage);
    for (int g = kBatchGroups - 1; g >= 0; --g) launch_persistent(L, g, stream);
    hipLaunchKernelGGL(batched_finalize, dim3(unsigned(L.count)), dim3(kBlock), 0, stream, L.mats,
                       L.perm_parts, L.g_parts, L.out, L.want_grad ? L.grad : nullptr);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

int launch_batched_forked(const BatchLaunch &L, hipStream_t stream,
                          const hipStream_t side[kBatchGroups], hipEvent_t fork,
                          const hipEvent_t join[kBatchGroups])
{
    hipLaunchKernelGGL(batched_reset, dim3(1), dim3(64), 0, stream, L.counters, kBatchGroups);
    hipLaunchKernelGGL(batched_prep, dim3(unsigned(L.count)), dim3(kBlock), 0, stream, L.mats, L.data,
                       L.stage);
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
    hipLaunchKernelGGL(batched_finalize, dim3(unsigned(L.count)), dim3(kBlock), 0, stream, L.mats,
                       L.perm_parts, L.g_parts, L.out, L.want_grad ? L.grad : nullptr);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
