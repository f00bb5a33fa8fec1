// Device-side building blocks shared by the Gray-walk sweep kernels.
#pragma once

#include "perm_internal.h"

namespace perm {

// Low c bits of Gray(g) for g = K * 2^c + l, where kb = bit 0 of K is the
// only bit of K that reaches below bit c (through g >> 1).
__device__ inline uint32_t gray_low(uint32_t l, uint32_t kb, int c)
{
    uint32_t gl = l ^ (l >> 1) ^ (kb << (c - 1));
    return gl & ((1u << c) - 1u);
}

// Chunk index of this lane.  Bit 0 of K comes from the wave index, so it is
// the same for all 64 lanes of a wave: then the column flipped at each step
// and its sign are wave-uniform at every step (bits below c of g are the
// local step index, bit c is K's bit 0), which keeps A in scalar registers.
__device__ inline uint64_t lane_chunk_index(uint64_t wave, uint32_t lane)
{
    return (wave & 1u) | (uint64_t(lane) << 1) | ((wave >> 1) << 7);
}

// Global index of this thread's wave, in a scalar register: the compiler
// cannot see that threadIdx.x >> 6 is the same for a whole wave, so without
// readfirstlane everything derived from it would be treated as divergent.
__device__ inline uint64_t uniform_wave_index()
{
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    return uint64_t(blockIdx.x) * kWavesPerBlock + w;
}

// Wave-wide double-double sum; every lane ends with the total.
__device__ inline dd wave_reduce_dd(dd v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        dd o;
        o.hi = __shfl_xor(v.hi, off, 64);
        o.lo = __shfl_xor(v.lo, off, 64);
        v = dd_add(v, o);
    }
    return v;
}

// Block-wide (kBlock threads) double-double sum; the result is valid in
// thread 0.  Order is fixed, so the result is bitwise reproducible.
__device__ inline dd block_reduce_dd(dd v, dd *lds /* kWavesPerBlock */)
{
    v = wave_reduce_dd(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[wave] = v;
    __syncthreads();
    dd t = dd{0.0, 0.0};
    if (threadIdx.x == 0) {
        t = lds[0];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) t = dd_add(t, lds[w]);
    }
    __syncthreads();
    return t;
}

// Compensated accumulation of one term into (s, e): Sum2 of Ogita, Rump and
// Oishi (the error of every addition is collected exactly by two_sum).
__device__ inline void acc_add(double &s, double &e, double v)
{
    double t, err;
    two_sum(s, v, t, err);
    s = t;
    e += err;
}

// Staging kernels (sweep_f64.hip, sweep_c128.hip): column-major +-A and x0.
__global__ void prep_dense_f64(int n, const double *__restrict__ A, int64_t lda,
                               double *__restrict__ acol, double *__restrict__ aneg,
                               double *__restrict__ x0);
__global__ void prep_dense_c128(int n, const perm_c128 *__restrict__ A, int64_t lda,
                                double *__restrict__ acol, double *__restrict__ aneg,
                                double *__restrict__ x0);

// Binary path staging and the modular sum of per-block residues
// (sweep_binary.hip).
__global__ void prep_binary(int n, const double *__restrict__ dense01, double *__restrict__ ycol,
                            double *__restrict__ yneg, double *__restrict__ y0);
__global__ void finalize_residues(const uint64_t *__restrict__ partials, int64_t count,
                                  int nprimes, BinaryPrimes P, uint64_t *__restrict__ out);

// Sums `count` double-double partials (components interleaved: partial b of
// component q is at p[b * comps + q]) in a fixed order with one block, and
// writes scale * total (rounded to double) to out[q].
__global__ void finalize_partials(const dd *__restrict__ p, int64_t count, int comps,
                                  double scale, double *__restrict__ out);

}  // namespace perm
