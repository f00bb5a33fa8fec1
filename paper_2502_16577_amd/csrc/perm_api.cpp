// C ABI of libperm_mi355x.so: argument validation, workspace sizing, launch
// planning and dispatch to the HIP kernels.  Every check happens before any
// GPU work is queued; no function here allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "perm.h"
#include "perm_internal.h"

namespace perm {

// Lanes x chunk = 2^(n-1) exactly (Section 3.1.1: with power-of-two chunks every
// lane of a wave flips the same column at the same local step, and no
// remainder kernel is needed).  About 2^18 lanes fill the 256 CUs with four
// waves per SIMD; smaller problems use fewer lanes but at least one block and
// at least 64 steps per lane where the problem allows it.
SweepPlan plan_sweep(int n, int /*steps_per_op_hint*/)
{
    SweepPlan p;
    p.n = n;
    if (n <= 12) {
        p.log2_chunk = n > 0 ? n - 1 : 0;
        p.log2_reseed = p.log2_chunk;
        p.lanes = 1;
        p.blocks = 1;
        return p;
    }
    const int total = n - 1;                 // log2 of the number of steps
    const int cmin = std::min(6, total - 8);  // keep >= 256 lanes (one block)
    // at most 2^31 steps per lane (32-bit local step index): above n = 50
    // the lane count grows instead
    const int c = std::min(31, std::max(cmin, total - 18));
    p.log2_chunk = c;
    p.log2_reseed = std::min(9, c);
    p.lanes = int64_t(1) << (total - c);
    p.blocks = p.lanes / kBlock;
    return p;
}

SweepPlan plan_sweep_fine(int n)
{
    SweepPlan p = plan_sweep(n, 0);
    if (n <= 12) return p;
    // 2^20 lanes (16384 waves, 16 per SIMD) instead of 2^18: a lane's work
    // depends on the data (nonzero terms, skipped blocks), and with more,
    // shorter chunks the waves that finish early are replaced by new ones
    const int total = n - 1;
    const int cmin = std::min(6, total - 8);
    const int c = std::max(cmin, total - 20);
    if (c >= p.log2_chunk || c > 31) return p;
    p.log2_chunk = c;
    p.log2_reseed = std::min(9, c);
    p.lanes = int64_t(1) << (total - c);
    p.blocks = p.lanes / kBlock;
    return p;
}

DenseWs dense_ws_layout(int n, int components, int64_t blocks)
{
    DenseWs L;
    size_t off = 0;
    const size_t nn = size_t(n) * size_t(n) * size_t(components) * sizeof(double);
    L.acol = off;
    off += align256(nn);
    L.aneg = off;
    off += align256(nn);
    L.x0 = off;
    off += align256(size_t(n) * size_t(components) * sizeof(double));
    L.partials = off;
    off += align256(size_t(std::max<int64_t>(blocks, 1)) * size_t(components) * sizeof(dd));
    if (n <= (components == 1 ? kExtMaxN : kExtMaxNComplex)) {
        L.ext = off;
        off += align256(4 * nn);
    }
    L.total = off;
    return L;
}

BinaryWs binary_ws_layout(int n, int64_t blocks)
{
    BinaryWs L;
    size_t off = 0;
    const size_t nn = size_t(n) * size_t(n) * sizeof(double);
    L.dense01 = off;
    off += align256(nn);
    L.ycol = off;
    off += align256(nn);
    L.yneg = off;
    off += align256(nn);
    L.y0 = off;
    off += align256(size_t(n) * sizeof(double));
    L.partials = off;
    off += align256(size_t(std::max<int64_t>(blocks, 1)) * kMaxPrimes * sizeof(uint64_t));
    L.residues = off;
    off += align256(kMaxPrimes * sizeof(uint64_t));
    L.total = off;
    return L;
}

GradWs grad_ws_layout(int n, int components, int64_t waves)
{
    GradWs L;
    size_t off = 0;
    const size_t np = size_t(grad_rows(n));
    const size_t nn = size_t(n) * np * size_t(components) * sizeof(double);
    L.acol = off;
    off += align256(nn);
    L.x0 = off;
    off += align256(np * size_t(components) * sizeof(double));
    L.perm_partials = off;
    off += align256(size_t(std::max<int64_t>(waves, 1)) * 2 * sizeof(dd));
    L.grad_partials = off;
    off += align256(size_t(std::max<int64_t>(waves, 1)) * size_t(components) * size_t(n) *
                    size_t(n) * sizeof(dd));
    L.grad_sums = off;
    off += align256(size_t(grad_sum_slices(waves)) * size_t(components) * size_t(n) * size_t(n) *
                    sizeof(dd));
    L.total = off;
    return L;
}

uint64_t host_prime(int k) { return kBinaryPrimes[k]; }

}  // namespace perm

using namespace perm;

static_assert(kAccTwoSum == PERM_ACC_TWOSUM && kAccPlain == PERM_ACC_PLAIN && kAccKahan == PERM_ACC_KAHAN &&
                  kAccExtended == PERM_ACC_EXTENDED,
              "accumulation modes must match the ABI");

namespace {

bool valid_n(int n) { return n >= 0 && n <= PERM_MAX_N; }

// CSC pattern checks: col_ptr[0] = 0, nondecreasing, col_ptr[n] = nnz, row
// indices in [0, n) and strictly increasing inside each column.
bool valid_csc(int n, const int32_t *col_ptr, const int32_t *row_idx, int32_t nnz)
{
    if (!col_ptr || nnz < 0 || (nnz > 0 && !row_idx)) return false;
    if (int64_t(nnz) > int64_t(n) * n) return false;
    if (col_ptr[0] != 0 || col_ptr[n] != nnz) return false;
    for (int j = 0; j < n; ++j) {
        if (col_ptr[j + 1] < col_ptr[j]) return false;
        for (int32_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) {
            if (row_idx[p] < 0 || row_idx[p] >= n) return false;
            if (p > col_ptr[j] && row_idx[p] <= row_idx[p - 1]) return false;
        }
    }
    return true;
}

uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t p)
{
    return uint64_t((unsigned __int128)a * b % p);
}

uint64_t powmod_host(uint64_t a, uint64_t e, uint64_t p)
{
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = mulmod_host(r, a, p);
        a = mulmod_host(a, a, p);
        e >>= 1;
    }
    return r;
}

// log2 of the Bregman-Minc bound prod_i (r_i!)^(1/r_i) on the permanent of a
// 0/1 matrix with row sums r_i (all r_i >= 1).
double bregman_log2(const std::vector<int> &r)
{
    double b = 0.0;
    for (int ri : r) b += std::lgamma(double(ri) + 1.0) / std::log(2.0) / double(ri);
    return b;
}

int check_ws(const void *ws, size_t ws_bytes, size_t need)
{
    if (need == 0) return PERM_OK;
    if (!ws || ws_bytes < need) return PERM_EWORKSPACE;
    return PERM_OK;
}

}  // namespace

extern "C" {

const char *perm_strerror(int status)
{
    switch (status) {
    case PERM_OK: return "success";
    case PERM_EINVAL: return "invalid argument";
    case PERM_ERANGE: return "result exceeds the representable range";
    case PERM_EWORKSPACE: return "workspace missing or too small";
    case PERM_EHIP: return "HIP runtime error";
    case PERM_EUNSUPPORTED: return "unsupported request";
    case PERM_ECOMPILE: return "run-time compilation of a generated kernel failed";
    case PERM_ESCRATCH: return "request exceeds the fixed scratch of an allocation-free entry point";
    default: return "unknown status";
    }
}

int perm_version(void) { return 100; }

size_t perm_workspace_bytes(int kind, int n, int64_t m)
{
    (void)m;
    if (!valid_n(n)) return 0;
    switch (kind) {
    case PERM_KIND_DENSE_F64:
    case PERM_KIND_DENSE_C128: {
        const int comps = kind == PERM_KIND_DENSE_C128 ? 2 : 1;
        if (n <= kSmallN) return grad_ws_layout(n, comps, plan_grad(n).waves).total;
        return dense_ws_layout(n, comps, dense_ws_blocks(n)).total;
    }
    case PERM_KIND_SPARSE_F64: {
        return perm_workspace_bytes(PERM_KIND_DENSE_F64, n, 0) +
               align256(size_t(n) * n * sizeof(double));
    }
    case PERM_KIND_GRAD_F64:
    case PERM_KIND_GRAD_C128: {
        if (n > kGradMaxN) return 0;
        const GradPlan p = plan_grad(n);
        return grad_ws_layout(n, kind == PERM_KIND_GRAD_C128 ? 2 : 1, p.waves).total;
    }
    case PERM_KIND_BINARY: {
        const SweepPlan p = plan_sweep_fine(n);
        return binary_ws_layout(n, p.blocks).total;
    }
    default: return 0;
    }
}

int perm_dense_f64(int n, const double *A, int64_t lda, double *out, void *ws, size_t ws_bytes,
                   void *stream)
{
    if (!valid_n(n) || !out) return PERM_EINVAL;
    if (n > 0 && (!A || lda < n)) return PERM_EINVAL;
    const int w = check_ws(ws, ws_bytes, perm_workspace_bytes(PERM_KIND_DENSE_F64, n, 0));
    if (w != PERM_OK) return w;
    return launch_dense_f64(n, A, lda, out, static_cast<char *>(ws),
                            static_cast<hipStream_t>(stream));
}

// perm_options -> SweepOptions; false for invalid options.
static bool sweep_options(int n, const perm_options *opt, SweepOptions &o)
{
    o = default_sweep_options(n);
    if (!opt) return true;
    if (opt->accumulation != PERM_ACC_TWOSUM && opt->accumulation != PERM_ACC_PLAIN &&
        opt->accumulation != PERM_ACC_KAHAN && opt->accumulation != PERM_ACC_EXTENDED)
        return false;
    if (opt->log2_reseed < 0 || opt->log2_reseed > 62 || opt->max_steps_per_launch < 0 ||
        opt->log2_lanes < 0 || opt->log2_lanes > 40 || opt->first_launch < 0 ||
        opt->launch_count < 0)
        return false;
    o.log2_lanes = opt->log2_lanes;
    o.accumulation = opt->accumulation;
    if (opt->log2_reseed > 0) o.log2_reseed = opt->log2_reseed;
    if (opt->max_steps_per_launch > 0) o.max_steps_per_launch = opt->max_steps_per_launch;
    o.first_launch = opt->first_launch;
    o.launch_count = opt->launch_count;
    return true;
}

int64_t perm_dense_f64_launches(int n, const perm_options *opt)
{
    if (!valid_n(n)) return PERM_EINVAL;
    SweepOptions o;
    if (!sweep_options(n, opt, o)) return PERM_EINVAL;
    return n == 0 ? 1 : dense_f64_launches(n, o);
}

int perm_dense_f64_ex(int n, const double *A, int64_t lda, const perm_options *opt, double *out,
                      void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_n(n) || !out) return PERM_EINVAL;
    if (n > 0 && (!A || lda < n)) return PERM_EINVAL;
    SweepOptions o;
    if (!sweep_options(n, opt, o)) return PERM_EINVAL;
    if (o.accumulation == kAccExtended && n > 0 && (n < kExtMinN || n > kExtMaxN))
        return PERM_EUNSUPPORTED;
    if (o.first_launch >= (n == 0 ? 1 : dense_f64_launches(n, o))) return PERM_EINVAL;
    const int w = check_ws(ws, ws_bytes, perm_workspace_bytes(PERM_KIND_DENSE_F64, n, 0));
    if (w != PERM_OK) return w;
    return launch_dense_f64_opt(n, A, lda, out, o, static_cast<char *>(ws),
                                static_cast<hipStream_t>(stream));
}

int perm_dense_c128(int n, const perm_c128 *A, int64_t lda, perm_c128 *out, void *ws,
                    size_t ws_bytes, void *stream)
{
    if (!valid_n(n) || !out) return PERM_EINVAL;
    if (n > 0 && (!A || lda < n)) return PERM_EINVAL;
    const int w = check_ws(ws, ws_bytes, perm_workspace_bytes(PERM_KIND_DENSE_C128, n, 0));
    if (w != PERM_OK) return w;
    return launch_dense_c128(n, A, lda, out, static_cast<char *>(ws),
                             static_cast<hipStream_t>(stream));
}

int perm_dense_c128_ex(int n, const perm_c128 *A, int64_t lda, const perm_options *opt,
                       perm_c128 *out, void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_n(n) || !out) return PERM_EINVAL;
    if (n > 0 && (!A || lda < n)) return PERM_EINVAL;
    int acc = PERM_ACC_TWOSUM, reseed = 0;
    if (opt) {
        if (opt->accumulation != PERM_ACC_TWOSUM && opt->accumulation != PERM_ACC_PLAIN &&
            opt->accumulation != PERM_ACC_KAHAN && opt->accumulation != PERM_ACC_EXTENDED)
            return PERM_EINVAL;
        if (opt->log2_reseed < 0 || opt->log2_reseed > 62 || opt->max_steps_per_launch < 0 ||
            opt->log2_lanes < 0 || opt->first_launch < 0 || opt->launch_count < 0)
            return PERM_EINVAL;
        acc = opt->accumulation;
        reseed = opt->log2_reseed;
        if (acc == PERM_ACC_PLAIN || acc == PERM_ACC_KAHAN) return PERM_EUNSUPPORTED;
        if (acc == PERM_ACC_TWOSUM && reseed != 0) return PERM_EUNSUPPORTED;
        if (opt->max_steps_per_launch != 0 || opt->log2_lanes != 0 || opt->first_launch != 0 ||
            opt->launch_count != 0)
            return PERM_EUNSUPPORTED;
    }
    if (acc == PERM_ACC_EXTENDED && n > 0 && (n < kExtMinN || n > kExtMaxNComplex))
        return PERM_EUNSUPPORTED;
    const int w = check_ws(ws, ws_bytes, perm_workspace_bytes(PERM_KIND_DENSE_C128, n, 0));
    if (w != PERM_OK) return w;
    if (acc == PERM_ACC_EXTENDED)
        return launch_dense_c128_ext(n, A, lda, out, reseed, static_cast<char *>(ws),
                                     static_cast<hipStream_t>(stream));
    return launch_dense_c128(n, A, lda, out, static_cast<char *>(ws),
                             static_cast<hipStream_t>(stream));
}

// A row or column without a nonzero value meets every permutation, so the
// permanent is exactly 0 (the sweep's terms would cancel only to rounding).
static bool has_empty_line(int n, const int32_t *col_ptr, const int32_t *row_idx,
                           const double *vals)
{
    std::vector<char> row_hit(n, 0);
    for (int j = 0; j < n; ++j) {
        bool col_hit = false;
        for (int32_t q = col_ptr[j]; q < col_ptr[j + 1]; ++q)
            if (vals[q] != 0.0) {
                col_hit = true;
                row_hit[row_idx[q]] = 1;
            }
        if (!col_hit) return true;
    }
    for (int i = 0; i < n; ++i)
        if (!row_hit[i]) return true;
    return false;
}

// Validation shared by the sparse real entry points; PERM_OK to go on.
static int sparse_args(int n, const int32_t *col_ptr, const int32_t *row_idx, const double *vals,
                       int32_t nnz, double *out, void *ws, size_t ws_bytes)
{
    if (!valid_n(n) || !out) return PERM_EINVAL;
    if (n > 0 && (!valid_csc(n, col_ptr, row_idx, nnz) || (nnz > 0 && !vals))) return PERM_EINVAL;
    return check_ws(ws, ws_bytes, perm_workspace_bytes(PERM_KIND_SPARSE_F64, n, nnz));
}

// Columns of a CSC matrix by ascending nonzero count (stable): new column jn
// is old column order[jn].  The permanent is invariant under column
// permutations; in the Gray walk the low columns flip most often (column 0
// every other step) and the last column never, so with the sparsest columns
// lowest each step updates, and rounds, the fewest entries of x.  On the
// 40 x 40 six-per-row pattern with scaled values this takes the dense sweep's
// relative error from 3.5e-10 (given order) to 7e-11 (descending: 1e-8).
static std::vector<int> columns_by_count(int n, const int32_t *col_ptr)
{
    std::vector<int> order(n);
    for (int j = 0; j < n; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return col_ptr[x + 1] - col_ptr[x] < col_ptr[y + 1] - col_ptr[y];
    });
    return order;
}

// Staged-column sweep: the matrix is scattered into a row-major copy behind
// the dense workspace, its columns by ascending count, and swept like a
// dense matrix (every step adds a whole column, zeros included).  Used for
// n < kSparseGenMinN (at most 2^12 steps) and by perm_sparse_f64_staged.
static int sparse_staged(int n, const int32_t *col_ptr, const int32_t *row_idx,
                         const double *vals, char *base, double *out, hipStream_t st)
{
    const size_t off = perm_workspace_bytes(PERM_KIND_DENSE_F64, n, 0);
    double *dense = reinterpret_cast<double *>(base + off);
    const int32_t nnz = col_ptr[n];
    const std::vector<int> order = columns_by_count(n, col_ptr);
    std::vector<int32_t> pos(nnz);
    for (int jn = 0; jn < n; ++jn) {
        const int j = order[jn];
        for (int32_t q = col_ptr[j]; q < col_ptr[j + 1]; ++q) pos[q] = row_idx[q] * n + jn;
    }
    int rc = launch_stage_sparse(n, pos.data(), vals, nnz, dense, st);
    if (rc != PERM_OK) return rc;
    return launch_dense_f64(n, dense, n, out, base, st);
}

int perm_sparse_f64(int n, const int32_t *col_ptr, const int32_t *row_idx, const double *vals,
                    int32_t nnz, double *out, void *ws, size_t ws_bytes, void *stream)
{
    int rc = sparse_args(n, col_ptr, row_idx, vals, nnz, out, ws, ws_bytes);
    if (rc != PERM_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    if (n == 0) return launch_dense_f64(0, nullptr, 0, out, base, st);
    if (has_empty_line(n, col_ptr, row_idx, vals)) return launch_write_f64(0.0, out, st);
    if (n < kSparseGenMinN) return sparse_staged(n, col_ptr, row_idx, vals, base, out, st);
    // Algorithm 2's update: a step adds only the flipped column's nonzeros.
    // With x in registers a run-time row index cannot name a register, so
    // the update lists are compiled into a kernel for this pattern.
    // Columns by ascending count: the low columns, flipped at 15 of every
    // 16 steps, then cost the fewest updates (and round the fewest entries
    // of x), and the densest column is the never-flipped last one.
    const std::vector<int> order = columns_by_count(n, col_ptr);
    // Rows (also free to permute): those with a nonzero in the four lowest
    // columns go last.  Steps inside a 16-step block change only these rows,
    // and the generated product evaluates rows in a fixed order, so the
    // compiler computes the product of the other rows once per block.
    std::vector<char> hot(n, 0);
    for (int jn = 0; jn < std::min(n, 4); ++jn)
        for (int32_t q = col_ptr[order[jn]]; q < col_ptr[order[jn] + 1]; ++q) hot[row_idx[q]] = 1;
    std::vector<int> new_row(n);
    {
        int k = 0;
        for (int i = 0; i < n; ++i)
            if (!hot[i]) new_row[i] = k++;
        for (int i = 0; i < n; ++i)
            if (hot[i]) new_row[i] = k++;
    }
    std::vector<int32_t> pos;
    std::vector<double> val;
    pos.reserve(nnz);
    val.reserve(nnz);
    std::vector<std::vector<int>> rows(n);
    for (int jn = 0; jn < n; ++jn) {
        const int j = order[jn];
        for (int32_t q = col_ptr[j]; q < col_ptr[j + 1]; ++q) {
            const int i = new_row[row_idx[q]];
            pos.push_back(i * n + jn);
            val.push_back(vals[q]);
            rows[jn].push_back(i);
        }
        std::sort(rows[jn].begin(), rows[jn].end());
    }
    const size_t off = perm_workspace_bytes(PERM_KIND_DENSE_F64, n, 0);
    double *dense = reinterpret_cast<double *>(base + off);
    rc = launch_stage_sparse(n, pos.data(), val.data(), int64_t(pos.size()), dense, st);
    if (rc != PERM_OK) return rc;
    return launch_sparse_gen(n, rows, dense, out, base, st);
}

int perm_sparse_f64_staged(int n, const int32_t *col_ptr, const int32_t *row_idx,
                           const double *vals, int32_t nnz, double *out, void *ws,
                           size_t ws_bytes, void *stream)
{
    int rc = sparse_args(n, col_ptr, row_idx, vals, nnz, out, ws, ws_bytes);
    if (rc != PERM_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    if (n == 0) return launch_dense_f64(0, nullptr, 0, out, base, st);
    if (has_empty_line(n, col_ptr, row_idx, vals)) return launch_write_f64(0.0, out, st);
    return sparse_staged(n, col_ptr, row_idx, vals, base, out, st);
}

// The exact binary path; `generated` selects the kernel generated for the
// pattern (n >= kSparseGenMinN) instead of the staged one.
static int binary_exact(int n, const int32_t *col_ptr, const int32_t *row_idx, int32_t nnz,
                        int n_primes, uint64_t out_limbs[5], uint64_t *out_residues,
                        int *out_nprimes, void *ws, size_t ws_bytes, void *stream,
                        bool generated)
{
    if (!valid_n(n) || !out_limbs || n_primes < 0 || n_primes > kMaxPrimes) return PERM_EINVAL;
    if (n > 0 && !valid_csc(n, col_ptr, row_idx, nnz)) return PERM_EINVAL;
    for (int k = 0; k < 5; ++k) out_limbs[k] = 0;
    if (out_residues)
        for (int k = 0; k < kMaxPrimes; ++k) out_residues[k] = 0;
    if (n == 0) {
        const int np0 = n_primes ? n_primes : 3;
        out_limbs[0] = 1;
        if (out_residues)
            for (int k = 0; k < np0; ++k) out_residues[k] = 1;
        if (out_nprimes) *out_nprimes = np0;
        return PERM_OK;
    }
    // Dense 0/1 pattern, row sums, and the number of primes from the bound.
    std::vector<double> dense(size_t(n) * n, 0.0);
    std::vector<int> rsum(n, 0), csum(n, 0);
    for (int j = 0; j < n; ++j)
        for (int32_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) {
            dense[size_t(row_idx[p]) * n + j] = 1.0;
            rsum[row_idx[p]]++;
            csum[j]++;
        }
    bool empty_line = false;
    for (int i = 0; i < n; ++i) empty_line = empty_line || rsum[i] == 0 || csum[i] == 0;
    int needed = 3;
    if (!empty_line) {
        const double bits = bregman_log2(rsum) + 1.0;  // +1: margin for rounding of the bound
        // every prime exceeds 2^50, so `needed` primes hold 50 * needed bits
        while (needed < kMaxPrimes && double(needed) * 50.0 < bits) ++needed;
        if (double(needed) * 50.0 < bits) return PERM_ERANGE;
    }
    const int np = n_primes == 0 ? needed : n_primes;
    if (np < needed && !empty_line) return PERM_ERANGE;
    if (out_nprimes) *out_nprimes = np;
    if (empty_line) return PERM_OK;  // an empty row or column: no perfect matching
    const SweepPlan plan = plan_sweep_fine(n);
    const BinaryWs L = binary_ws_layout(n, plan.blocks);
    const int w = check_ws(ws, ws_bytes, L.total);
    if (w != PERM_OK) return w;

    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    uint64_t *res_dev = reinterpret_cast<uint64_t *>(base + L.residues);
    int rc = PERM_OK;
    if (generated && n >= kSparseGenMinN) {
        // Columns by ascending count (the low columns flip most often and the
        // densest is the never-flipped last one); rows that columns 0..3 do
        // not touch first ("cold": constant inside a 16-step block).
        std::vector<int> col(n);
        for (int j = 0; j < n; ++j) col[j] = j;
        std::stable_sort(col.begin(), col.end(), [&](int x, int y) { return csum[x] < csum[y]; });
        std::vector<char> hot(n, 0);
        for (int jn = 0; jn < 4; ++jn)
            for (int i = 0; i < n; ++i) hot[i] = hot[i] || dense[size_t(i) * n + col[jn]] != 0.0;
        std::vector<int> row;
        for (int i = 0; i < n; ++i)
            if (!hot[i]) row.push_back(i);
        const int n_cold = int(row.size());
        for (int i = 0; i < n; ++i)
            if (hot[i]) row.push_back(i);
        std::vector<double> pd(size_t(n) * n);
        std::vector<std::vector<int>> rows(n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                pd[size_t(i) * n + j] = dense[size_t(row[i]) * n + col[j]];
                if (pd[size_t(i) * n + j] != 0.0) rows[j].push_back(i);
            }
        if (hipMemcpyAsync(base + L.dense01, pd.data(), pd.size() * sizeof(double),
                           hipMemcpyHostToDevice, st) != hipSuccess)
            return PERM_EHIP;
        rc = launch_binary_gen(n, n_cold, rows, reinterpret_cast<const double *>(base + L.dense01),
                               np, res_dev, base, st);
        if (rc != PERM_OK) {
            hipStreamSynchronize(st);  // the staging buffer must outlive the copy
            return rc;
        }
        if (hipStreamSynchronize(st) != hipSuccess) return PERM_EHIP;
    } else {
    // Zero-block skipping plan (the permanent is invariant under row and
    // column permutations): columns by ascending count, so the fast-flipping
    // low columns touch few rows and the densest column is the never-flipped
    // last one; then rows with no nonzero in columns < b first.
    int skip_b = 0, nfrozen = 0;
    if (n > 12) {
        std::vector<int> col(n);
        for (int j = 0; j < n; ++j) col[j] = j;
        std::stable_sort(col.begin(), col.end(), [&](int x, int y) { return csum[x] < csum[y]; });
        // probability that y_i = 0 for a random subset (binomial count of the
        // row's flippable nonzeros hitting exactly half the row count)
        std::vector<double> q(n, 0.0);
        for (int i = 0; i < n; ++i) {
            const int last = dense[size_t(i) * n + col[n - 1]] != 0.0;
            const int rr = rsum[i] - last;
            const int t = rsum[i] / 2 - last;
            if (rsum[i] % 2 == 0 && t >= 0 && t <= rr)
                q[i] = std::exp(std::lgamma(rr + 1.0) - std::lgamma(t + 1.0) - std::lgamma(rr - t + 1.0) -
                                rr * std::log(2.0));
        }
        const double step_cost = 2.0 * n + 5.0;
        double best = step_cost;
        // skipped blocks are whole blocks of the kernel's walk (2^U steps)
        const int bmin = n >= 14 ? 4 : 3;
        for (int b = bmin; b <= std::min(plan.log2_chunk, 10); ++b) {
            double alive = 1.0;  // P(a lane's block is not provably zero)
            for (int i = 0; i < n; ++i) {
                bool frozen = true;
                for (int j = 0; j < b && frozen; ++j) frozen = dense[size_t(i) * n + col[j]] == 0.0;
                if (frozen) alive *= 1.0 - q[i];
            }
            const double p_skip = std::pow(1.0 - alive, 64.0);
            const double B = double(1 << b);
            const double cost = (1.5 * n + p_skip * 2.0 * n + (1.0 - p_skip) * B * step_cost) / B;
            if (cost < 0.8 * best) {
                best = cost;
                skip_b = b;
            }
        }
        std::vector<int> row(n);
        for (int i = 0; i < n; ++i) row[i] = i;
        if (skip_b > 0) {
            auto frozen = [&](int i) {
                for (int j = 0; j < skip_b; ++j)
                    if (dense[size_t(i) * n + col[j]] != 0.0) return false;
                return true;
            };
            std::stable_partition(row.begin(), row.end(), frozen);
            for (int i = 0; i < n; ++i) nfrozen += frozen(i);
        }
        std::vector<double> perm_dense(size_t(n) * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) perm_dense[size_t(i) * n + j] = dense[size_t(row[i]) * n + col[j]];
        dense.swap(perm_dense);
    }

    if (hipMemcpyAsync(base + L.dense01, dense.data(), dense.size() * sizeof(double),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return PERM_EHIP;
    rc = launch_binary_residues(n, reinterpret_cast<const double *>(base + L.dense01), np, skip_b,
                                nfrozen, res_dev, base, st);
    if (rc != PERM_OK) {
        hipStreamSynchronize(st);  // the staging buffer must outlive the copy
        return rc;
    }
    }
    uint64_t R[kMaxPrimes] = {};
    if (hipMemcpyAsync(R, res_dev, sizeof(uint64_t) * np, hipMemcpyDeviceToHost, st) != hipSuccess)
        return PERM_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return PERM_EHIP;

    // R_k = (-1)^(n-1) 2^(n-1) perm  (mod p_k)
    uint64_t res[kMaxPrimes];
    for (int k = 0; k < np; ++k) {
        const uint64_t p = host_prime(k);
        const uint64_t inv2 = (p + 1) / 2;
        uint64_t v = mulmod_host(R[k] % p, powmod_host(inv2, uint64_t(n - 1), p), p);
        if (!(n & 1) && v) v = p - v;
        res[k] = v;
        if (out_residues) out_residues[k] = v;
    }
    // Garner: perm = t_0 + p_0 (t_1 + p_1 (t_2 + ...)), 0 <= perm < prod p_k.
    uint64_t t[kMaxPrimes];
    for (int k = 0; k < np; ++k) {
        const uint64_t pk = host_prime(k);
        uint64_t v = res[k];
        for (int j = 0; j < k; ++j) {
            const uint64_t pj = host_prime(j) % pk;
            const uint64_t inv = powmod_host(pj, pk - 2, pk);
            v = mulmod_host((v + pk - t[j] % pk) % pk, inv, pk);
        }
        t[k] = v;
    }
    uint64_t limbs[6] = {0, 0, 0, 0, 0, 0};
    limbs[0] = t[np - 1];
    for (int k = np - 2; k >= 0; --k) {
        // limbs = limbs * p_k + t_k
        unsigned __int128 carry = t[k];
        const uint64_t pk = host_prime(k);
        for (int q = 0; q < 6; ++q) {
            const unsigned __int128 v = (unsigned __int128)limbs[q] * pk + carry;
            limbs[q] = uint64_t(v);
            carry = v >> 64;
        }
    }
    for (int q = 0; q < 5; ++q) out_limbs[q] = limbs[q];
    return PERM_OK;
}

int perm_binary_exact(int n, const int32_t *col_ptr, const int32_t *row_idx, int32_t nnz,
                      int n_primes, uint64_t out_limbs[5], uint64_t *out_residues,
                      int *out_nprimes, void *ws, size_t ws_bytes, void *stream)
{
    return binary_exact(n, col_ptr, row_idx, nnz, n_primes, out_limbs, out_residues, out_nprimes,
                        ws, ws_bytes, stream, false);
}

int perm_binary_exact_gen(int n, const int32_t *col_ptr, const int32_t *row_idx, int32_t nnz,
                          int n_primes, uint64_t out_limbs[5], uint64_t *out_residues,
                          int *out_nprimes, void *ws, size_t ws_bytes, void *stream)
{
    return binary_exact(n, col_ptr, row_idx, nnz, n_primes, out_limbs, out_residues, out_nprimes,
                        ws, ws_bytes, stream, true);
}

int perm_grad(int n, int dtype, const void *A, int64_t lda, void *out_perm, void *out_grad,
              void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_n(n) || !out_perm || (n > 0 && (!out_grad || !A || lda < n))) return PERM_EINVAL;
    if (dtype != PERM_DTYPE_F64 && dtype != PERM_DTYPE_C128) return PERM_EINVAL;
    if (n > kGradMaxN) return PERM_EUNSUPPORTED;
    const bool cplx = dtype == PERM_DTYPE_C128;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0) {
        return cplx ? launch_dense_c128(0, nullptr, 0, static_cast<perm_c128 *>(out_perm), nullptr, st)
                    : launch_dense_f64(0, nullptr, 0, static_cast<double *>(out_perm), nullptr, st);
    }
    const int kind = cplx ? PERM_KIND_GRAD_C128 : PERM_KIND_GRAD_F64;
    const int w = check_ws(ws, ws_bytes, perm_workspace_bytes(kind, n, 0));
    if (w != PERM_OK) return w;
    return launch_grad(n, cplx, A, lda, out_perm, out_grad, static_cast<char *>(ws), st);
}

uint64_t perm_binary_prime(int k)
{
    if (k < 0 || k >= kMaxPrimes) return 0;
    return host_prime(k);
}

}  // extern "C"
