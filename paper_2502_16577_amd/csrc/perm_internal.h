// Internal declarations shared by the host ABI layer and the HIP kernels of
// libperm_mi355x.so.  Not part of the public ABI (that is include/perm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "perm.h"

namespace perm {

// ---------------------------------------------------------------------------
// Launch shape
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;          // threads per block: 4 waves of 64
constexpr int kWave = 64;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxPrimes = 6;        // binary path: at most 6 primes of 51 bits
constexpr int kSmallN = 12;          // n <= 12: forward sweeps run on the one-wave gradient kernel

// Gray-walk decomposition of the 2^(n-1) steps of one matrix:
//   lanes * 2^log2_chunk == 2^(n-1), every lane walks one contiguous chunk,
//   and x is rebuilt exactly from the Gray code every 2^log2_reseed steps.
struct SweepPlan {
    int n = 0;
    int log2_chunk = 0;      // c: steps per lane = 2^c (c >= 2)
    int log2_reseed = 0;     // r: exact re-seed every 2^r steps (1 <= r <= c)
    int64_t lanes = 0;       // 2^(n-1-c), a multiple of 128 (whole wave pairs)
    int64_t blocks = 0;      // lanes / kBlock (rounded up)
};

SweepPlan plan_sweep(int n, int steps_per_op_hint);
// The same walk with 4x more, shorter chunks (n > 12), for sweeps whose work
// per lane depends on the data (the exact binary sweeps: nonzero terms and
// skipped blocks): waves that finish early are replaced by new ones.
SweepPlan plan_sweep_fine(int n);

// Primes of the exact binary path: the six smallest primes above 2^50.  A
// residue, and the product of two residues divided by p, fit the 53-bit
// significand, so the kernels multiply modulo p in FP64 arithmetic: two
// error-free products and a rounded quotient (no 64-bit integer multiplies).
constexpr uint64_t kBinaryPrimes[kMaxPrimes] = {
    1125899906842679ull, 1125899906842723ull, 1125899906842769ull,
    1125899906842783ull, 1125899906842817ull, 1125899906842829ull};

// The primes as kernel arguments: p exactly, and 1/p rounded to nearest.
struct BinaryPrimes {
    double p[kMaxPrimes];
    double pinv[kMaxPrimes];
};

inline BinaryPrimes binary_primes()
{
    BinaryPrimes P;
    for (int k = 0; k < kMaxPrimes; ++k) {
        P.p[k] = double(kBinaryPrimes[k]);
        P.pinv[k] = 1.0 / P.p[k];
    }
    return P;
}

// Run-time options of the dense real sweep.
constexpr int kAccTwoSum = 0, kAccPlain = 1, kAccKahan = 2;  // lane accumulation modes
constexpr int kAccExtended = 3;  // x, products and lane partial in double-double
constexpr int kExtMinN = 13, kExtMaxN = 48;  // orders of the extended-precision walk

struct SweepOptions {
    int accumulation = kAccTwoSum;                  // kAcc* (same values as PERM_ACC_*)
    int log2_reseed = 9;                            // exact re-seed every 2^r steps (<= c)
    int64_t max_steps_per_launch = int64_t(1) << 40;  // split longer sweeps into launches
    int log2_lanes = 0;                             // 0 = plan_sweep's choice
    int64_t first_launch = 0;                       // run launches [first, first + count)
    int64_t launch_count = 0;                       // 0 = through the last one
};

inline SweepOptions default_sweep_options(int n)
{
    SweepOptions o;
    const SweepPlan p = plan_sweep(n, 0);
    o.log2_reseed = p.log2_reseed;
    return o;
}

// ---------------------------------------------------------------------------
// Double-double helpers (error-free transformations; require IEEE
// round-to-nearest and no reassociation, which hipcc gives without
// -ffast-math).
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
};

__host__ __device__ inline void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Sum of two double-double values (accurate to about 2^-104 relative).
__host__ __device__ inline dd dd_add(dd a, dd b)
{
    double s, e;
    two_sum(a.hi, b.hi, s, e);
    double t, f;
    two_sum(a.lo, b.lo, t, f);
    e += t;
    double hi = s + e;
    double lo = e - (hi - s);
    lo += f;
    double hi2 = hi + lo;
    return dd{hi2, lo - (hi2 - hi)};
}

// ---------------------------------------------------------------------------
// Workspace layouts (byte offsets into the caller's device workspace)
// ---------------------------------------------------------------------------
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct DenseWs {
    size_t acol = 0;      // n*n scalars, column-major copy of A
    size_t aneg = 0;      // n*n scalars, its negation
    size_t x0 = 0;        // n scalars, Nijenhuis-Wilf start vector
    size_t partials = 0;  // one dd (per component) per block
    size_t ext = 0;       // 4 n*n scalars for the extended walk's split entries
                          // and their negations (orders it supports only)
    size_t total = 0;
};

DenseWs dense_ws_layout(int n, int components, int64_t blocks);

// Block partials a dense workspace holds: the default plan's blocks, and at
// least 1024 (2^18 lanes) so perm_dense_f64_ex may choose other lane counts.
inline int64_t dense_ws_blocks(int n)
{
    const int64_t b = plan_sweep(n, 0).blocks;
    return b > 1024 ? b : 1024;
}

struct BinaryWs {
    size_t dense01 = 0;   // n*n doubles, the 0/1 pattern row-major (staged from the host CSC)
    size_t ycol = 0;      // n*n doubles, 2 a_ij column-major
    size_t yneg = 0;      // n*n doubles, -2 a_ij
    size_t y0 = 0;        // n doubles, 2 a_{i,n-1} - r_i
    size_t partials = 0;  // blocks * kMaxPrimes uint64 residues
    size_t residues = 0;  // kMaxPrimes uint64 residues of the whole sum
    size_t total = 0;
};

BinaryWs binary_ws_layout(int n, int64_t blocks);

// Gradient sweep (and the forward sweep of small n): one wave per block.
constexpr int kGradMaxN = 32;        // MFMA tiles of G up to 2 x 2

struct GradPlan {
    int n = 0;
    int log2_chunk = 0;       // c >= 1 (n >= 2)
    int log2_reseed = 0;      // r <= c - 1
    int64_t lanes_active = 0; // 2^(n-1-c); lanes beyond it idle (small n)
    int64_t waves = 0;
};

GradPlan plan_grad(int n);

struct GradWs {
    size_t acol = 0, x0 = 0;            // staged columns (grad_rows(n) rows each), start vector
    size_t perm_partials = 0;           // waves * 2 dd
    size_t grad_partials = 0;           // waves * components * n * n dd
    size_t grad_sums = 0;               // grad_sum_slices(waves) * components * n * n dd
    size_t total = 0;
};

// The items' G partials are summed in two fixed-order passes: over slices of
// the items (about 16 items a slice, at most 64 slices), then over the slices.
inline int grad_sum_slices(int64_t items)
{
    const int64_t s = items / 16;
    return int(s < 1 ? 1 : s > 64 ? 64 : s);
}

GradWs grad_ws_layout(int n, int components, int64_t waves);
// Waves per gradient work item; they split the matrix's rows (grad_item.h).
constexpr int kGradSlices = 2;
// Staged rows per column for grad_item: padded to a multiple of the slices.
__host__ __device__ inline int grad_rows(int n)
{
    return (n + kGradSlices - 1) / kGradSlices * kGradSlices;
}

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).  All return PERM_OK or
// PERM_EHIP and only enqueue work on `stream`.
// ---------------------------------------------------------------------------
// Matrix-specific sparse sweep (sparse_codegen.cpp): `rows[j]` lists the
// nonzero rows of column j of the staged matrix `dense_dev` (row-major,
// lda = n, on the device).  Compiles and caches one kernel per device and
// pattern.
constexpr int kSparseGenMinN = 14;
int launch_sparse_gen(int n, const std::vector<std::vector<int>> &rows, const double *dense_dev,
                      double *out, char *ws, hipStream_t stream);
std::string sparse_gen_source(int n, const std::vector<std::vector<int>> &rows);
// Exact binary sweep through a kernel generated for the pattern: rows are
// ordered with the n_cold rows that columns 0..3 do not touch first, `rows`
// as above; writes the nprimes residues of sum_g (-1)^g prod y to
// residues_dev (binary workspace layout).
int launch_binary_gen(int n, int n_cold, const std::vector<std::vector<int>> &rows,
                      const double *dense01_dev, int nprimes, uint64_t *residues_dev, char *ws,
                      hipStream_t stream);
std::string binary_gen_source(int n, int n_cold, const std::vector<std::vector<int>> &rows);

// out[0] = v (a kernel, so it can sit in a captured graph).
int launch_write_f64(double v, double *out, hipStream_t stream);
// Stages count entries into the row-major n x n copy `dense` (device):
// zeroes it, then dense[pos[t]] = val[t].  pos / val are host arrays whose
// contents are copied into the kernel arguments, so they may be released as
// soon as the call returns (no synchronisation).
constexpr int kScatterChunk = 256;
struct ScatterChunk {
    int count;
    int32_t pos[kScatterChunk];
    double val[kScatterChunk];
};
int launch_stage_sparse(int n, const int32_t *pos, const double *val, int64_t count,
                        double *dense, hipStream_t stream);
int launch_dense_f64(int n, const double *A, int64_t lda, double *out, char *ws,
                     hipStream_t stream);
int launch_dense_f64_opt(int n, const double *A, int64_t lda, double *out, const SweepOptions &o,
                         char *ws, hipStream_t stream);
// The dense sweep's plan under the options, and the number of launches the
// sweep is split into (1 for n <= 12).
SweepPlan dense_plan(int n, const SweepOptions &o);
// Steps of every lane's chunk per launch of the dense walks (a power of two,
// a multiple of the re-seed interval).
int64_t dense_launch_span(int n, const SweepPlan &p, const SweepOptions &o);
// The extended-precision dense walk (sweep_ext.hip), n >= 1.
int launch_dense_ext(int n, const double *A, int64_t lda, double *out, const SweepOptions &o,
                     char *ws, hipStream_t stream);
int64_t dense_f64_launches(int n, const SweepOptions &o);
int launch_dense_c128_ext(int n, const perm_c128 *A, int64_t lda, perm_c128 *out,
                          int log2_reseed, char *ws, hipStream_t stream);
constexpr int kExtMaxNComplex = 32;  // orders of the complex extended-precision walk
int launch_dense_c128(int n, const perm_c128 *A, int64_t lda, perm_c128 *out, char *ws,
                      hipStream_t stream);
// Permanent and dperm/dA (row-major n x n, interleaved if complex).
int launch_grad(int n, bool cplx, const void *A, int64_t lda, void *out_perm, void *out_grad,
                char *ws, hipStream_t stream);
// The same sweep without the gradient (used for the forward path of n <= 12).
int launch_grad_or_small(int n, bool cplx, const void *A, int64_t lda, void *out_perm,
                         void *out_grad, bool want_grad, char *ws, hipStream_t stream);
// Residues R_k = sum_g (-1)^g prod_i y_i(g) mod p_k (k < nprimes) into residues_dev.
// skip_b > 0 enables exact zero-block skipping with blocks of 2^skip_b steps;
// rows 0 .. nfrozen-1 must then have no nonzero in columns 0 .. skip_b-1.
int launch_binary_residues(int n, const double *dense01, int nprimes, int skip_b, int nfrozen,
                           uint64_t *residues_dev, char *ws, hipStream_t stream);

}  // namespace perm
