// One work item of the permanent-and-gradient sweep: 64 subsets (lane K =
// 64 w + lane walks the Gray steps g in [K 2^c, (K+1) 2^c) of one matrix),
// processed by a block of NS waves that split the matrix's rows: wave h
// holds rows [h R, (h+1) R) of every subset's x, window sum and
// leave-one-out products, so each wave keeps 1/NS of the state in
// registers.  Once per step the waves swap the products of their slices
// through LDS.
// Shared by the single-matrix kernel (sweep_grad.hip) and the batched
// persistent kernels (sweep_batched.hip).
//
// Gradient formula: with tau_j(g) = +1 if column j is in S_g or j = n-1, else
// -1, and L_i(g) = prod_{k != i} x_k(g),
//     dperm/da_ij = (-1)^(n-1) sum_g (-1)^g L_i(g) tau_j(g)
// i.e. G = sum over subsets of the rank-1 updates V tau^T, V = (-1)^g L.
//
// The contraction is organised by the Gray code.  Split the local steps of
// a lane into aligned windows of F = 2^f steps (f <= c - 1).  Inside a window
// the bits of g from f upwards do not change, so tau_j is constant for every
// column j >= f:
//   * columns j >= f: the rank-1 updates of a window add up to W tau^T with
//     W = sum of V over the window (one vector per lane); at the end of each
//     window the 64 lanes' W are contracted with their tau as one FP64 MFMA
//     product, G (rows x n) += W (rows x 64) T (64 x n), K running over lanes.
//   * columns j < f: tau_j depends only on the step (the same for every lane
//     of the wave), so per step G[:, j] += tau_j U with U = sum over lanes of
//     V; each lane sums 16 lanes' V from LDS (the reads of one step overlap
//     the next step's flip and product).  For j >= 1, tau_j is the same at
//     both steps of an aligned pair, so one MFMA per pair, with the B operand
//     tau_j repeated down K, adds the four partial sums of the pair and forms
//     the outer product with tau; column 0 is summed per lane with its sign
//     and contracted at the end of the window.
// MFMA operand layout (gfx950): A[i][k] at lane i + 16k, B[k][j] at lane
// j + 16k, D[i][j] at lane j + 16 (i mod 4), register i / 4.
// Accumulators fold into the item's double-double partial G in global memory
// at the end of every window (2^9 steps at most, so plain FP64 accumulation
// never spans more than 512 steps of 64 subsets).
//
// Staged layout: acol holds column j at [W (j NP + i)] with NP = NS R rows
// (rows >= n are zero) and x0 has NP entries (1 for rows >= n), so a padding
// row keeps x = 1 and changes no product.  A flip's sign goes into the FMA
// multiplier, so no negated copy is staged.
#pragma once

#include <type_traits>

#include "sweep_common.h"

namespace perm {

typedef double v4d __attribute__((ext_vector_type(4)));

template <bool CPLX>
__device__ __forceinline__ void gmul(double &ar, double &ai, double br, double bi)
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

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N, bool CPLX>
struct GradItemShape {
    static constexpr int NS = kGradSlices;        // waves (row slices) per item
    static constexpr int R = (N + NS - 1) / NS;   // rows per slice (<= 16 for N <= 32)
    static constexpr int NP = NS * R;             // staged rows per column
    static constexpr int MT = (N + 15) / 16;      // 16-column tiles of G
    static constexpr int STRIDE = R + 1;          // doubles per lane row in LDS
    static constexpr int W = CPLX ? 2 : 1;        // components
    static constexpr int VBUF = W * kWave * STRIDE;   // per-wave transposition buffer
    static constexpr int XBUF = 2 * NS * kWave * W;   // product exchange, two step parities
    static constexpr int LDS_DOUBLES = NS * VBUF + XBUF;
    static constexpr int THREADS = NS * kWave;
    static_assert(R <= 16, "a slice must fit one 16-row MFMA tile");
};

// Called by all NS waves of a block (each must make the call: it
// synchronises the block once per step).
// Inputs: staged acol / x0 (layout above); the item's index w (its
// subsets are 64 w .. 64 w + 63); log2 chunk c >= 1; log2 re-seed interval
// r <= c - 1; lanes_active (subsets K >= lanes_active idle with x = 0).
// Outputs: perm_out[0..1] (double-double re, im of the item's share of
// sum_g (-1)^g prod x; im is 0 for real matrices), and, if want_grad,
// g_out[(i*N + j)*W + comp] for i < N (double-double share of
// sum_g (-1)^g L_i tau_j; each wave zeroes and fills its own rows).
template <int N, bool CPLX>
__device__ __forceinline__ void grad_item(const double *__restrict__ acol,
                                          const double *__restrict__ x0, uint64_t w, int c, int r,
                                          uint64_t lanes_active, dd *__restrict__ perm_out,
                                          dd *__restrict__ g_out, bool want_grad,
                                          double *__restrict__ lds)
{
    using S = GradItemShape<N, CPLX>;
    constexpr int NS = S::NS;
    constexpr int R = S::R;
    constexpr int NP = S::NP;
    constexpr int MT = S::MT;
    constexpr int W = S::W;
    constexpr int STRIDE = S::STRIDE;
    const uint32_t lane = threadIdx.x & 63u;
    const int h = int(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));  // row slice
    const int row0 = h * R;
    double *vbuf = lds + h * S::VBUF;
    double *xbuf = lds + NS * S::VBUF;
    const uint32_t C = 1u << c;
    const uint32_t rmask = (1u << r) - 1u;
    const int f = c - 1 < 9 ? c - 1 : 9;  // window = 2^f steps
    const uint32_t fmask = (1u << f) - 1u;
    const uint64_t Kl = w * kWave + lane;
    const double act = Kl < lanes_active ? 1.0 : 0.0;
    const int jj = int(lane & 15u);      // B column / A row within a tile
    const int kq = int(lane >> 4);       // K index within an MFMA (0..3)

    double xr[R], xi[R];
    double wr[R], wi[R];                 // window sums of V (this slice's rows)
    v4d acc_lo[W];                       // low columns (j < f)
#pragma unroll
    for (int q = 0; q < W; ++q) acc_lo[q] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < R; ++t) {
        wr[t] = 0.0;
        wi[t] = 0.0;
    }
    if (want_grad) {
        const int rows = N - row0 < R ? N - row0 : R;
        for (int e = int(lane); e < rows * N * W; e += kWave) g_out[row0 * N * W + e] = dd{0.0, 0.0};
    }
    double sr = 0.0, er = 0.0;  // this wave's compensated share of the permanent's sum

    auto reseed = [&](uint32_t l) {
        const uint64_t g = (Kl << c) | l;
        const uint64_t gray = g ^ (g >> 1);
        const double *xs = x0 + W * row0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            xr[t] = act * xs[W * t];
            xi[t] = CPLX ? act * xs[W * t + 1] : 0.0;
        }
        for (int j = 0; j < N - 1; ++j) {
            const double fj = ((gray >> j) & 1u) ? act : 0.0;
            const double *a = acol + W * (j * NP + row0);
#pragma unroll
            for (int t = 0; t < R; ++t) {
                xr[t] = __builtin_fma(fj, a[W * t], xr[t]);
                if (CPLX) xi[t] = __builtin_fma(fj, a[W * t + 1], xi[t]);
            }
        }
    };
    // The sign of the flip goes into the multiplier (one staged copy, half
    // the scalar-cache footprint of two).
    const double nact = -act;
    auto flip = [&](int j, bool add) {
        const double *a = acol + W * (j * NP + row0);
        const double sa = add ? act : nact;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            xr[t] = __builtin_fma(sa, a[W * t], xr[t]);
            if (CPLX) xi[t] = __builtin_fma(sa, a[W * t + 1], xi[t]);
        }
    };

    // tau_j of the subset of lane `lk` at local step l (0 for padding columns).
    auto tau = [&](uint64_t lk, uint32_t l, int j) -> double {
        if (j >= N) return 0.0;
        if (j == N - 1) return 1.0;
        const uint64_t g = ((w * kWave + lk) << c) | l;
        return (((g ^ (g >> 1)) >> j) & 1u) ? 1.0 : -1.0;
    };

    // The low columns' share of the step before (its V is in vbuf, written by
    // this wave before these reads in program order; a wave's LDS accesses
    // complete in order): lane (jj, kq) adds 16 lanes' V of slice row jj
    // (lanes 16 kq .. 16 kq + 15), and the MFMA adds the four kq partial
    // sums and multiplies by tau_j(l) for the columns j < f.  The reads of a
    // component are issued by lo_read and consumed by lo_add, with other
    // work of the current step in between to hide the LDS latency.
    double lv[16];
    double lsum[W];
    const int jr = jj < R ? jj : 0;      // lanes jj >= R read row 0 and drop it
    auto lo_read = [&](int q) {
        const double *col = vbuf + q * kWave * STRIDE + jr + 16 * kq * STRIDE;
#pragma unroll
        for (int m = 0; m < 16; ++m) lv[m] = col[m * STRIDE];
    };
    auto lo_add = [&](int q) {
#pragma unroll
        for (int span = 8; span >= 1; span /= 2)
#pragma unroll
            for (int m = 0; m < span; ++m) lv[m] += lv[m + span];
        lsum[q] = (jj < R) ? lv[0] : 0.0;
    };
    // The MFMA runs once per aligned pair of steps (l even, l + 1): tau_j for
    // j >= 1 is the same at both (only bit 0 of the step changes), so the
    // pair's partial sums gs are multiplied once; column 0, whose tau flips
    // inside the pair, is accumulated per lane (y0) and contracted at the end
    // of the window.  Called only with f >= 1 (windows of whole pairs).
    double gs[W], y0[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        gs[q] = 0.0;
        y0[q] = 0.0;
    }
    auto lo_apply = [&](uint32_t l) {
        // tau_0 of step l: bit 0 of its Gray code (bits 0 and 1 are local)
        const double t0 = ((l ^ (l >> 1)) & 1u) ? 1.0 : -1.0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            gs[q] += lsum[q];
            y0[q] = __builtin_fma(t0, lsum[q], y0[q]);
        }
        if ((l & 1u) == 1u) {
            const double bl = (jj >= 1 && jj < f) ? tau(0, l, jj) : 0.0;
#pragma unroll
            for (int q = 0; q < W; ++q) {
                acc_lo[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(gs[q], bl, acc_lo[q], 0, 0, 0);
                gs[q] = 0.0;
            }
        }
    };
    // end of a window: column 0 from the per-lane sums (B = e_0 adds the
    // four kq partial sums of each row into column 0)
    auto lo_fold0 = [&]() {
        const double b0 = (jj == 0) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            acc_lo[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0[q], b0, acc_lo[q], 0, 0, 0);
            y0[q] = 0.0;
        }
    };

    // One step of the walk: the leave-one-out products of this slice's rows,
    // their window sums, and the low columns' contribution.  NEG is the sign
    // (-1)^g of the step (the walk takes steps in pairs, even then odd, so
    // it is known at compile time).
    //
    // With pre_i = x_0 ... x_{i-1} (the earlier rows of the slice), F the
    // slice product and O the other slice's product, L_i = (-1)^g O pre_i
    // (prod of the later rows), formed from the last row down; the empty
    // products (pre_0, the later rows of the last row) are never multiplied
    // in: 3 (R - 1) complex products per lane and step.  One dependency
    // chain: cutting the rows into independent chains (2, 3 or 4 of them)
    // measured slower, as the extra partial products cost more in register
    // pressure than the parallelism gains at two waves per SIMD.
    auto step = [&](uint32_t l, auto neg_tag) {
        constexpr bool NEG = decltype(neg_tag)::value;
        // the previous step's low-column values (written by this wave, in
        // order before these reads), unless this step opens a window
        const bool pend = want_grad && f > 0 && (l & fmask) != 0u;
        double pr[R], pim[R];      // pre_i (i >= 1)
        double fr = xr[0], fi = xi[0];
#pragma unroll
        for (int t = 1; t < R; ++t) {
            pr[t] = fr;
            pim[t] = fi;
            gmul<CPLX>(fr, fi, xr[t], xi[t]);
        }
        // keeps the adds of the low-column reads after the product above
        __builtin_amdgcn_sched_barrier(0);
        if (pend) {
            lo_add(0);
            if (CPLX) lo_read(1);
        }
        // the other slices' products, through LDS (the buffer alternates
        // with the step parity, so one barrier per step suffices)
        double *xb = xbuf + int(l & 1u) * NS * kWave * W;
        xb[(h * kWave + lane) * W] = fr;
        if (CPLX) xb[(h * kWave + lane) * W + 1] = fi;
        __syncthreads();
        double orr, oii;
        if constexpr (NS == 2) {
            orr = xb[((1 - h) * kWave + lane) * W];
            oii = CPLX ? xb[((1 - h) * kWave + lane) * W + 1] : 0.0;
        } else {
            orr = 1.0;
            oii = 0.0;
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) {
                if (s2 == h) continue;
                const double *xo = xb + (s2 * kWave + lane) * W;
                gmul<CPLX>(orr, oii, xo[0], CPLX ? xo[1] : 0.0);
            }
        }
        if (NEG) {
            orr = -orr;
            oii = -oii;
        }
        // the whole signed product, shared between the waves: for complex
        // matrices wave 0 accumulates its real part and wave 1 its imaginary
        // part; for real ones wave 0 takes the even steps and wave 1 the odd
        if constexpr (CPLX) {
            if (h == 0) acc_add(sr, er, fr * orr - fi * oii);
            else acc_add(sr, er, fr * oii + fi * orr);
        } else {
            if (h == (NEG ? 1 : 0)) acc_add(sr, er, fr * orr);
        }
        if (!want_grad) return;
        if (pend) {
            if (CPLX) lo_add(1);
            lo_apply(l - 1);
        }
        // from the last row down: s = (-1)^g O (prod of the later rows),
        // L_i = pre_i s; V goes to this wave's transposition buffer for the
        // low columns
        double sufr = orr, sufi = oii;
        double *vr = vbuf + lane * STRIDE;
        double *vi = vbuf + (W - 1) * kWave * STRIDE + lane * STRIDE;
#pragma unroll
        for (int t = R - 1; t >= 0; --t) {
            double lr = sufr, li = sufi;
            if (t > 0) {
                gmul<CPLX>(lr, li, pr[t], pim[t]);
                gmul<CPLX>(sufr, sufi, xr[t], xi[t]);
            }
            wr[t] += lr;
            if (CPLX) wi[t] += li;
            vr[t] = lr;
            if (CPLX) vi[t] = li;
        }
    };

    auto close_window = [&](uint32_t l0) {
        if (f > 0) {  // the window's last step
#pragma unroll
            for (int q = 0; q < W; ++q) {
                lo_read(q);
                lo_add(q);
            }
            lo_apply(l0 + fmask);
            lo_fold0();
        }
        v4d acc_hi[W][MT];  // the window's contraction (slice rows x all columns)
#pragma unroll
        for (int q = 0; q < W; ++q)
#pragma unroll
            for (int b = 0; b < MT; ++b) acc_hi[q][b] = v4d{0.0, 0.0, 0.0, 0.0};
        double *vr = vbuf + lane * STRIDE;
        double *vi = vbuf + (W - 1) * kWave * STRIDE + lane * STRIDE;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            vr[t] = wr[t];
            if (CPLX) vi[t] = wi[t];
            wr[t] = 0.0;
            wi[t] = 0.0;
        }
        wave_sync_lds();
#pragma unroll 2
        for (int q4 = 0; q4 < 16; ++q4) {
            const uint64_t lk = uint64_t(4 * q4 + kq);  // lane (subset) of this K row
            double bop[MT];
#pragma unroll
            for (int b = 0; b < MT; ++b) {
                const int j = 16 * b + jj;
                bop[b] = (j >= f) ? tau(lk, l0, j) * (w * kWave + lk < lanes_active ? 1.0 : 0.0)
                                  : 0.0;
            }
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const double av = (jj < R) ? vbuf[q * kWave * STRIDE + lk * STRIDE + jj] : 0.0;
#pragma unroll
                for (int b = 0; b < MT; ++b)
                    acc_hi[q][b] =
                        __builtin_amdgcn_mfma_f64_16x16x4f64(av, bop[b], acc_hi[q][b], 0, 0, 0);
            }
        }
        wave_sync_lds();
        // fold into the item's partial G (this slice's rows)
#pragma unroll
        for (int q = 0; q < W; ++q)
#pragma unroll
            for (int b = 0; b < MT; ++b) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int t = kq + 4 * e;  // slice row
                    const int i = row0 + t;
                    const int j = 16 * b + jj;
                    double v = acc_hi[q][b][e];
                    if (b == 0) v += acc_lo[q][e];
                    if (t < R && i < N && j < N) {
                        dd *p = g_out + (i * N + j) * W + q;
                        const dd o = *p;
                        double s, u;
                        two_sum(o.hi, v, s, u);
                        *p = dd{s, o.lo + u};
                    }
                }
            }
#pragma unroll
        for (int q = 0; q < W; ++q) acc_lo[q] = v4d{0.0, 0.0, 0.0, 0.0};
    };

    for (uint32_t l = 0; l < C; l += 2) {
        // the previous step's low-column reads go out before the flip
        if (want_grad && f > 0 && (l & fmask) != 0u) lo_read(0);
        if ((l & rmask) == 0) {
            reseed(l);
        } else {
            const int j = __builtin_ctz(l);
            flip(j, (((l ^ (l >> 1)) >> j) & 1u) != 0u);
        }
        step(l, std::false_type{});
        if (want_grad && f == 0) close_window(l);
        if (want_grad && f > 0) lo_read(0);
        if (c == 1) {
            reseed(l + 1);  // the column-0 sign depends on the lane when c == 1
        } else {
            const uint32_t l1 = l + 1;
            flip(0, ((l1 ^ (l1 >> 1)) & 1u) != 0u);
        }
        step(l + 1, std::true_type{});
        if (want_grad && ((l + 2) & fmask) == 0) close_window((l + 1) & ~fmask);
    }
    // the item's share of sum_g (-1)^g prod x: for complex matrices each
    // wave holds one component; for real ones both hold parts of the real
    // sum, combined through LDS
    const dd part = wave_reduce_dd(dd{sr, er});
    if constexpr (CPLX) {
        if (lane == 0) perm_out[h] = part;
    } else {
        __syncthreads();  // every wave is done with the exchange buffers
        if (h == 1 && lane == 0) {
            xbuf[0] = part.hi;
            xbuf[1] = part.lo;
        }
        __syncthreads();
        if (h == 0 && lane == 0) {
            perm_out[0] = dd_add(part, dd{xbuf[0], xbuf[1]});
            perm_out[1] = dd{0.0, 0.0};
        }
    }
}

}  // namespace perm
