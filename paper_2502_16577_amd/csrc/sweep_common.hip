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

int launch_write_f64(double v, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(write_f64, dim3(1), dim3(1), 0, stream, v, out);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
