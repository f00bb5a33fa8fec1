// Fixed-order reduction of per-block double-double partials.
#include "sweep_common.h"

namespace perm {

__global__ __launch_bounds__(kBlock) void finalize_partials(const dd *__restrict__ p,
                                                            int64_t count, int comps,
                                                            double scale,
                                                            double *__restrict__ out)
{
    __shared__ dd red[kWavesPerBlock];
    for (int q = 0; q < comps; ++q) {
        dd acc = dd{0.0, 0.0};
        for (int64_t b = threadIdx.x; b < count; b += kBlock) acc = dd_add(acc, p[b * comps + q]);
        const dd t = block_reduce_dd(acc, red);
        // scale is +-2 (or +-1), so this product is exact.
        if (threadIdx.x == 0) out[q] = scale * (t.hi + t.lo);
    }
}

__global__ void write_f64(double v, double *__restrict__ out) { out[0] = v; }

// Sparse staging: zero the n x n row-major copy, then scatter the nonzeros.
// The entries travel inside the kernel arguments (at most kScatterChunk per
// launch), so the caller's host arrays are no longer needed once the launch
// has been queued: no host buffer has to outlive an asynchronous copy.
__global__ __launch_bounds__(kBlock) void zero_f64(double *__restrict__ p, int64_t count)
{
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < count;
         i += int64_t(gridDim.x) * kBlock)
        p[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void scatter_f64(ScatterChunk c, double *__restrict__ dense)
{
    for (int t = threadIdx.x; t < c.count; t += kBlock) dense[c.pos[t]] = c.val[t];
}

int launch_stage_sparse(int n, const int32_t *pos, const double *val, int64_t count,
                        double *dense, hipStream_t stream)
{
    const int64_t nn = int64_t(n) * n;
    hipLaunchKernelGGL(zero_f64, dim3(unsigned((nn + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       stream, dense, nn);
    for (int64_t b = 0; b < count; b += kScatterChunk) {
        ScatterChunk c;
        c.count = int(count - b < kScatterChunk ? count - b : kScatterChunk);
        for (int t = 0; t < c.count; ++t) {
            c.pos[t] = pos[b + t];
            c.val[t] = val[b + t];
        }
        hipLaunchKernelGGL(scatter_f64, dim3(1), dim3(kBlock), 0, stream, c, dense);
    }
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

int launch_write_f64(double v, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(write_f64, dim3(1), dim3(1), 0, stream, v, out);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
