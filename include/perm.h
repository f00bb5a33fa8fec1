/*
 * perm.h -- C ABI of libperm_mi355x.so: matrix permanents on AMD MI355X
 * (gfx950) by the Gray-code-ordered Ryser / Nijenhuis-Wilf sweep.
 *
 * Method (arXiv 2502.16577, Section 2, Algorithm 1): with row sums r_i and the
 * start vector x_i = a_{i,n-1} - r_i / 2, the 2^(n-1) subsets S of the first
 * n-1 columns are visited in binary-reflected Gray-code order; step g flips
 * column j = ctz(g), updates x += s * A[:, j] (s = +1 when the column enters
 * S, -1 when it leaves), and accumulates (-1)^g * prod_i x_i.  The permanent
 * is 2 (-1)^(n-1) times that sum.  The iteration space is split into
 * power-of-two chunks, one per GPU lane, each seeded in closed form from its
 * Gray code (Algorithm 3 with the chunking of Section 3.1.1).
 *
 * General conventions (all entry points):
 *   - Dense matrices are DEVICE pointers, row-major: entry (i, j) is at
 *     A[i * lda + j], lda >= n.  Complex entries are perm_c128 (re, im).
 *   - Sparse patterns (CSC: col_ptr[n+1], row_idx[nnz], vals[nnz]) are HOST
 *     pointers: the library validates them and derives the launch plan from
 *     them before any GPU work, then stages them into the workspace.
 *   - ws is a DEVICE workspace of at least perm_workspace_bytes(kind, n, m)
 *     bytes, owned by the caller; the library allocates no device memory for
 *     data (perm_sparse_f64 and the *_gen entry points load code modules
 *     compiled for a sparsity pattern, which stay loaded) and keeps no
 *     pointer to caller memory after a call returns.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  All
 *     calls are asynchronous on that stream except perm_binary_exact(_gen),
 *     which synchronise it to finish the Chinese remaindering on the host.
 *     Sparse real inputs travel to the device inside kernel arguments, so
 *     the host arrays may be reused as soon as the call returns.
 *   - Results are deterministic for fixed inputs and sizes: partial sums are
 *     combined in a fixed order and no result goes through atomics.
 *   - perm_dense_f64(_ex), perm_dense_c128, perm_grad and perm_weighted_sum
 *     only enqueue kernels (no allocation, copy, memset or synchronisation),
 *     so they can be captured into a hipGraph; the binary entry points copy
 *     host data and synchronise, so they cannot.
 *   - n == 0 yields 1 (the empty product); n < 0 or n > PERM_MAX_N is
 *     PERM_EINVAL.  Errors are reported as negative return values before any
 *     GPU work is queued, except PERM_EHIP which reports a HIP runtime error.
 *   - No C++ exceptions cross the ABI.
 */
#ifndef PERM_MI355X_H
#define PERM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PERM_MAX_N 63

typedef struct {
    double re, im;
} perm_c128;

/* Status codes. */
#define PERM_OK            0
#define PERM_EINVAL       -1  /* bad argument: n out of range, NULL, lda < n, malformed CSC */
#define PERM_ERANGE       -2  /* result would not fit (binary: bound above the CRT modulus) */
#define PERM_EWORKSPACE   -3  /* ws NULL or ws_bytes below perm_workspace_bytes() */
#define PERM_EHIP         -4  /* a HIP runtime call failed */
#define PERM_EUNSUPPORTED -5  /* valid request the library does not implement */
#define PERM_ECOMPILE     -6  /* run-time compilation of a generated kernel failed */
#define PERM_ESCRATCH     -7  /* request exceeds the fixed scratch of an allocation-free entry point */

/* Workspace kinds for perm_workspace_bytes(). */
#define PERM_KIND_DENSE_F64   1
#define PERM_KIND_DENSE_C128  2
#define PERM_KIND_SPARSE_F64  3
#define PERM_KIND_BINARY      4
#define PERM_KIND_GRAD_F64    5
#define PERM_KIND_GRAD_C128   6
#define PERM_KIND_BATCHED     7

/* Human-readable text of a status code (static storage). */
const char *perm_strerror(int status);

/* Library version as 10000*major + 100*minor + patch. */
int perm_version(void);

/*
 * Bytes of device workspace a call needs.  kind is one of PERM_KIND_*; n is
 * the matrix order (for PERM_KIND_BATCHED: the largest order in the batch);
 * m is nnz for the sparse kinds, the number of matrices for the batched kind,
 * and ignored otherwise.  Returns 0 for an invalid request.
 */
size_t perm_workspace_bytes(int kind, int n, int64_t m);

/*
 * Permanent of a dense real n x n matrix (Algorithm 1 over 2^(n-1) subsets,
 * Section 2; chunked as in Algorithm 3).  All arithmetic is FP64; each lane
 * keeps its x in registers, re-derives it exactly from the Gray code at fixed
 * intervals, and accumulates its terms with two-sum compensation; lane, block
 * and grid partials are combined as double-double in a fixed order.
 *   A    device, row-major, lda >= n
 *   out  device, one double
 */
int perm_dense_f64(int n, const double *A, int64_t lda, double *out,
                   void *ws, size_t ws_bytes, void *stream);

/*
 * perm_dense_f64 for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the workspace lives in a fixed array of perm_noalloc_scratch_bytes() bytes
 * inside the library's device memory, one copy per GPU, held until the
 * process ends.  The caller passes only the input and the output.  Same
 * kernels and result as perm_dense_f64 with a caller workspace.
 *   A, lda, out, stream  as for perm_dense_f64 (the current device's array
 *                        is used; the stream must belong to that device)
 * PERM_ESCRATCH when the order needs more workspace than the array holds
 * (n > 53).  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (on different streams, or from several threads) race and must
 * be ordered by the caller.  The array keeps the last call's contents; no
 * call relies on it starting at zero.  The first call on a device looks up
 * the array's address there (no allocation).
 */
int perm_dense_f64_noalloc(int n, const double *A, int64_t lda, double *out, void *stream);

/* Size in bytes of each GPU's fixed array used by perm_dense_f64_noalloc. */
size_t perm_noalloc_scratch_bytes(void);

/* Options of perm_dense_f64_ex (zero-initialise for the defaults). */
/* Lane accumulation modes (Section 5, Table 3); block and grid partials are
 * always combined in double-double (the paper's "quad" outer sum). */
#define PERM_ACC_TWOSUM 0  /* two-sum: the lane partial is a double-double ("DQ"); the default */
#define PERM_ACC_PLAIN  1  /* plain double lane partial ("DD") */
#define PERM_ACC_KAHAN  2  /* Kahan-compensated lane partial ("Kahan") */
/* Extended precision, beyond the paper's modes: x, every product and the lane
 * partial in double-double, about 2^-104 per operation instead of 2^-53, and
 * about three times the time of the FP64 walk.  The entries are split
 * error-free on a power-of-two grid per row so that the high part of x is exact;
 * every product is formed by FMA.  For deep cancellation, where
 * R(A) / |perm(A)| is large (about 1e6 for U[0,1) entries at n = 40).  Orders
 * 13..48 (PERM_EUNSUPPORTED otherwise; n = 0 gives 1).  log2_lanes,
 * log2_reseed and the split launches apply as in the other modes.  The
 * workspace is the one perm_workspace_bytes gives for the order, which holds
 * the split entries for the orders this mode supports. */
#define PERM_ACC_EXTENDED 3

typedef struct {
    int accumulation;              /* PERM_ACC_TWOSUM, PERM_ACC_PLAIN, PERM_ACC_KAHAN or
                                      PERM_ACC_EXTENDED */
    int log2_reseed;               /* exact re-seed of x every 2^r steps; 0 = default (2^9),
                                      values above the lane's chunk mean once per chunk;
                                      steps are walked in blocks of 16 (8 for n = 13), so
                                      shorter intervals act as the block length */
    int64_t max_steps_per_launch;  /* 0 = default (2^40): longer sweeps run as several
                                      full-grid launches, each over a consecutive range of
                                      every lane's chunk (a power-of-two number of re-seed
                                      intervals) */
    int log2_lanes;                /* 0 = default (about 2^18 lanes); else the number of
                                      lanes (one Gray chunk each) as a power of two, clamped
                                      to [2^8, 2^18] (or the default if larger), to chunks
                                      longer than the 16-step block, and to chunks of at
                                      most 2^31 steps */
    int64_t first_launch;          /* the first launch of the split sweep to run */
    int64_t launch_count;          /* how many to run; 0 = through the last (see
                                      perm_dense_f64_ex) */
} perm_options;

/* perm_dense_f64 with options (opt may be NULL).  PERM_EINVAL for an unknown
 * accumulation mode, negative fields, or first_launch at or beyond the number
 * of launches; PERM_EUNSUPPORTED for PERM_ACC_EXTENDED outside orders 13..48
 * (n = 0 gives 1).  A long sweep can be run as several calls, each over a range
 * of its launches (perm_dense_f64_launches gives their number), in order,
 * with the same A, options (apart from the range), workspace and stream: a
 * call adds its launches' block sums to the partials the earlier calls left
 * in the workspace and writes the running total to out, so out holds the
 * permanent after the call that runs the last launch. */
int perm_dense_f64_ex(int n, const double *A, int64_t lda, const perm_options *opt,
                      double *out, void *ws, size_t ws_bytes, void *stream);

/* Number of launches perm_dense_f64_ex splits the sweep of order n into under
 * these options (opt may be NULL); negative (PERM_EINVAL) for invalid options. */
int64_t perm_dense_f64_launches(int n, const perm_options *opt);

/*
 * Permanent of a dense complex n x n matrix: the same sweep with complex x
 * and complex products (Section 1 lists complex matrices among the supported
 * inputs).
 *   A    device, row-major perm_c128, lda >= n
 *   out  device, one perm_c128
 */
int perm_dense_c128(int n, const perm_c128 *A, int64_t lda, perm_c128 *out,
                    void *ws, size_t ws_bytes, void *stream);

/* perm_dense_c128 with options (opt may be NULL for the default).  The
 * complex sweep has two accumulation modes: PERM_ACC_TWOSUM (the default,
 * as perm_dense_c128) and PERM_ACC_EXTENDED (real and imaginary parts of x,
 * every product and the lane partial in double-double; orders 13..32, n = 0
 * gives 1; log2_reseed applies).  PERM_ACC_PLAIN and PERM_ACC_KAHAN,
 * log2_reseed in the default mode, and nonzero max_steps_per_launch,
 * log2_lanes, first_launch or launch_count are PERM_EUNSUPPORTED; negative
 * fields or an unknown mode PERM_EINVAL.  Same workspace as perm_dense_c128. */
int perm_dense_c128_ex(int n, const perm_c128 *A, int64_t lda, const perm_options *opt,
                       perm_c128 *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Permanent of a sparse real n x n matrix in CSC (Algorithm 2, SpaRyser,
 * Section 2.1): the same Gray walk as the dense sweep, but a step adds to x
 * only the nonzeros of the flipped column; the product still runs over all
 * n rows.  With x held in registers a run-time row index cannot address a
 * register, so for n >= 14 the nonzero lists of the pattern are compiled
 * into a kernel (the per-matrix code generation of Section 3.2): the first
 * call for a pattern on a device compiles it with hiprtc (about a second)
 * and keeps the module loaded until the process ends; later calls with the
 * same pattern, whatever the values, reuse it.  Columns are reordered by
 * ascending count and rows touched by the four lowest columns are moved
 * last (the permanent is invariant under both), so inside a 16-step block
 * the product of the untouched rows is formed once.  For n < 14 (at most
 * 2^12 steps) the matrix is staged as dense columns instead.
 *   col_ptr  host int32[n+1], col_ptr[0] = 0, nondecreasing, col_ptr[n] = nnz
 *   row_idx  host int32[nnz], strictly increasing within a column, in [0, n)
 *   vals     host double[nnz]
 *   out      device, one double
 * Asynchronous: the nonzeros are copied into kernel arguments, and nothing
 * waits for the stream.  A row or column without a nonzero value gives
 * exactly 0 (written by a one-thread kernel, no sweep).  PERM_ECOMPILE if the
 * run-time compilation fails (perm_sparse_f64_staged needs none).
 */
int perm_sparse_f64(int n, const int32_t *col_ptr, const int32_t *row_idx,
                    const double *vals, int32_t nnz, double *out,
                    void *ws, size_t ws_bytes, void *stream);

/* The same permanent without run-time compilation: the matrix is staged as
 * dense columns and swept by the dense kernel, so every step adds a whole
 * column (zeros included).  Same arguments, workspace (PERM_KIND_SPARSE_F64)
 * and asynchrony as perm_sparse_f64. */
int perm_sparse_f64_staged(int n, const int32_t *col_ptr, const int32_t *row_idx,
                           const double *vals, int32_t nnz, double *out, void *ws,
                           size_t ws_bytes, void *stream);

/*
 * Exact permanent of a 0/1 matrix given by its nonzero pattern in CSC (the
 * number of perfect matchings of its bipartite graph, Section 1).  The sweep
 * runs on y = 2x, which is integral, modulo n_primes primes just above 2^50
 * (perm_binary_prime), with the modular products done in FP64 arithmetic;
 * the residues are combined by Chinese remaindering on the host.
 *   col_ptr, row_idx  host CSC pattern as for perm_sparse_f64
 *   n_primes          0 = choose from the Bregman bound (at least 3), else 1..6
 *   out_limbs         host uint64[5]: perm as unsigned little-endian 320 bits
 *   out_residues      host uint64[6] or NULL: perm mod p_k for the primes
 *                     used, zero in the unused slots
 *   out_nprimes       host int or NULL: number of primes used
 * Synchronises `stream`.  PERM_ERANGE if the bound exceeds the modulus of
 * the requested primes.  A matrix with an empty row or column has permanent
 * 0 and launches nothing.
 */
int perm_binary_exact(int n, const int32_t *col_ptr, const int32_t *row_idx,
                      int32_t nnz, int n_primes, uint64_t out_limbs[5],
                      uint64_t *out_residues, int *out_nprimes, void *ws,
                      size_t ws_bytes, void *stream);

/* perm_binary_exact through a kernel generated for this 0/1 pattern (the
 * per-matrix code generation of Section 3.2 applied to the exact path):
 * columns are reordered by ascending count and the rows the four lowest
 * columns touch are moved last; each flip is a fixed list of +-2 updates on
 * the column's rows; inside a 16-step block the products of the other rows
 * ("cold" rows) are computed once, and a block in which a cold row is zero
 * for all 64 subsets of a wave is skipped whole (only its net flip of column
 * 3 is applied).  The first call for a pattern on a device compiles the
 * kernel with hiprtc and keeps it loaded until the process ends.  Same
 * arguments, results, workspace (PERM_KIND_BINARY) and synchronisation as
 * perm_binary_exact; n < 14 runs perm_binary_exact's own kernel.
 * PERM_ECOMPILE if the compilation fails. */
int perm_binary_exact_gen(int n, const int32_t *col_ptr, const int32_t *row_idx, int32_t nnz,
                          int n_primes, uint64_t out_limbs[5], uint64_t *out_residues,
                          int *out_nprimes, void *ws, size_t ws_bytes, void *stream);

/* Element types for perm_grad. */
#define PERM_DTYPE_F64  1
#define PERM_DTYPE_C128 2

/*
 * Permanent and its gradient G_ij = dperm/da_ij in the same sweep.  The
 * permanent is multilinear in the entries, and with tau_j(g) = +1 if column
 * j is in the Gray subset S_g or j = n-1, else -1, differentiating the sum of
 * Algorithm 1 term by term gives G = (-1)^(n-1) sum_g (-1)^g L(g) tau(g)^T,
 * L_i(g) = prod_{k != i} x_k(g).  L comes from prefix / suffix products (no
 * division); the rank-1 updates of 64 subsets at a time are one FP64 MFMA
 * contraction.  For complex A, G is the complex (holomorphic) derivative.
 *   dtype     PERM_DTYPE_F64 (A, out_perm, out_grad are double) or
 *             PERM_DTYPE_C128 (perm_c128)
 *   A         device, row-major, lda >= n
 *   out_perm  device, one element
 *   out_grad  device, n x n row-major elements
 * n <= 32 (PERM_EUNSUPPORTED above).
 */
int perm_grad(int n, int dtype, const void *A, int64_t lda, void *out_perm,
              void *out_grad, void *ws, size_t ws_bytes, void *stream);

/*
 * Batched permanents (and gradients) of many small complex or real matrices
 * of uneven order, e.g. the amplitudes of photon-counting distributions
 * (Section 1) or the leaves of a Section 4 decomposition:
 * one persistent launch in which waves pull (matrix, chunk) work items,
 * largest orders first, and per-item partials are summed per matrix in a
 * fixed order.
 *
 * A plan holds the work list and launch shapes for one set of orders; it is
 * host memory owned by the caller (create / destroy), not thread-safe, and
 * caches the hipGraph of the launch for the last (data, out, grad, ws).
 *   count      number of matrices (>= 1)
 *   k          host int32[count], orders 1..32
 *   offset     host int64[count], element offset of matrix m in `data`
 *              (row-major k x k perm_c128; the same packing is used for grad)
 *   want_grad  nonzero: also compute dperm/dA of every matrix
 */
typedef struct perm_plan perm_plan;

int perm_batched_plan_create(int count, const int32_t *k, const int64_t *offset,
                             int want_grad, perm_plan **plan);
/* The same for real matrices: offsets count doubles, data / out / grad are
 * double, and the plan runs through the *_f64 entry points below (the
 * complex ones return PERM_EINVAL for it, and the _f64 ones for a complex
 * plan).  Each item is the real form of the same sweep (one component). */
int perm_batched_plan_create_f64(int count, const int32_t *k, const int64_t *offset,
                                 int want_grad, perm_plan **plan);
void perm_plan_destroy(perm_plan *plan);

/* Device workspace bytes for any launch (and any autotuning) of this plan. */
size_t perm_batched_workspace_bytes(const perm_plan *plan);

/*
 * Runs the batch.  data, out (perm_c128[count]) and grad (same packing as
 * data; required if the plan wants gradients) are device pointers.  The plan
 * is copied into `ws` on first use with this ws (a synchronous copy); with
 * use_graph != 0 the launch is captured once into a hipGraph (reset, staging,
 * persistent kernels on forked streams, finalize) and replayed with
 * hipGraphLaunch on `stream`.
 */
int perm_batched(perm_plan *plan, const perm_c128 *data, perm_c128 *out, perm_c128 *grad,
                 int use_graph, void *ws, size_t ws_bytes, void *stream);
/* perm_batched for a plan made by perm_batched_plan_create_f64: data and
 * grad row-major k x k doubles at the plan's offsets, out double[count]. */
int perm_batched_f64(perm_plan *plan, const double *data, double *out, double *grad,
                     int use_graph, void *ws, size_t ws_bytes, void *stream);

/*
 * Autotuner: times the batch on this device as the graph runs it (each
 * group's persistent kernel on its own stream, concurrently) and keeps the
 * fastest configuration in the plan, searching one knob at a time from the
 * defaults: the Gray steps per lane (2^8, 2^10, 2^12), then the persistent
 * grid of each group that has work (orders 1..16: 512 / 1024 / 2048 blocks;
 * 17..24: 512 / 768 / 1024, i.e. 1, 1.5 or 2 waves per SIMD; 25..32: 256 /
 * 384 / 512).  The result is kept for the rest of the process, keyed by
 * (device, want_grad, histogram of the orders): a plan created later with
 * the same key starts from it, and autotuning such a plan returns the
 * stored configuration and time without running anything.  Otherwise it
 * synchronises `stream` and writes the outputs as a side effect.  best_ms
 * (nullable) receives the time of the chosen configuration.
 */
int perm_batched_autotune(perm_plan *plan, const perm_c128 *data, perm_c128 *out,
                          perm_c128 *grad, void *ws, size_t ws_bytes, void *stream,
                          double *best_ms);
/* perm_batched_autotune for a real plan (the kept tunings of real and
 * complex plans are separate). */
int perm_batched_autotune_f64(perm_plan *plan, const double *data, double *out, double *grad,
                              void *ws, size_t ws_bytes, void *stream, double *best_ms);

/* Plan introspection (any output may be NULL): number of work items, log2
 * steps per lane, grid[3] = persistent blocks of the groups of orders 1..16,
 * 17..24 and 25..32, and whether the configuration came from the tuning
 * kept by an earlier perm_batched_autotune in this process. */
int perm_batched_plan_info(const perm_plan *plan, int64_t *n_items, int *log2_chunk,
                           int64_t *grid, int *tuned_from_cache);

/* out = sum_m weights[m] * perms[m] over count >= 1 complex device values
 * (each product split exactly by FMA), in double-double and a fixed order.
 * Asynchronous on `stream`. */
int perm_weighted_sum(int count, const double *weights, const perm_c128 *perms, perm_c128 *out,
                      void *stream);
/* The same over real values (double perms[count], double out[1]); combines
 * the leaves of a Section 4 decomposition, perm(A) = sum_l w_l perm(leaf_l). */
int perm_weighted_sum_f64(int count, const double *weights, const double *perms, double *out,
                          void *stream);

/*
 * Sparse preprocessing of Section 4 (host only, no GPU work).
 *   PERM_DECOMP_DM  fine-grain Dulmage-Mendelsohn pruning (Section 4.1):
 *                   find a perfect matching, orient matching edges row ->
 *                   column and the others column -> row, and delete every
 *                   nonzero whose row and column lie in different strongly
 *                   connected components (it lies on no perfect matching);
 *                   no perfect matching means perm = 0 (no leaves).
 *   PERM_DECOMP_FM  Algorithm 4 (DecompRyser): while a row or column has at
 *                   most 4 nonzeros, remove it by the Forbert-Marx expansion
 *                   (Eq. (expand)): 1 nonzero -> alpha * perm(minor), 2 -> the
 *                   merged (n-1) x (n-1) matrix, 3 or 4 -> two matrices
 *                   (at most 2^16 such two-way splits per call; after that
 *                   the remaining matrices are leaves).
 * The result is a list of leaves (k_m, weight_m, k_m x k_m row-major matrix)
 * with perm(A) = sum_m weight_m perm(leaf_m); a leaf of order 0 is stored as
 * the 1 x 1 matrix [1].  min_leaf stops decomposing matrices of that order or
 * less.  PERM_ERANGE if more than 2^22 leaves would be produced.
 *   PERM_DECOMP_FOLD (with PERM_DECOMP_FM) keeps no leaf of order 0, 1 or 2:
 *                   their weighted permanents (w, w a, w (ad + bc)) are summed
 *                   on the host in double-double, and perm_decomp_folded
 *                   returns that sum, so perm(A) = folded + sum_m weight_m
 *                   perm(leaf_m).  Without the flag folded is 0.
 */
#define PERM_DECOMP_DM 1
#define PERM_DECOMP_FM 2
#define PERM_DECOMP_FOLD 4

typedef struct perm_decomp perm_decomp;

int perm_decompose(int n, const int32_t *col_ptr, const int32_t *row_idx, const double *vals,
                   int32_t nnz, int flags, int min_leaf, perm_decomp **out);
int perm_decomp_info(const perm_decomp *d, int *count, int *max_order, int64_t *total_elements,
                     int64_t *removed_nonzeros);
/* Leaf idx: order, weight and (if data is non-NULL) its k*k entries. */
int perm_decomp_leaf(const perm_decomp *d, int idx, int *k, double *weight, double *data);
/* All leaves at once (host arrays of perm_decomp_info's count, any may be
 * NULL): k[i], weight[i], offset[i] = element offset of leaf i in data, and
 * data = the leaves' row-major entries back to back (total_elements). */
int perm_decomp_leaves(const perm_decomp *d, int32_t *k, double *weight, int64_t *offset,
                       double *data);
/* The folded leaves' sum as a (hi, lo) double-double (host array of 2). */
int perm_decomp_folded(const perm_decomp *d, double out[2]);
void perm_decomp_destroy(perm_decomp *d);

/* The k-th prime used by perm_binary_exact (k = 0..5; the six smallest
 * primes above 2^50), 0 if out of range. */
uint64_t perm_binary_prime(int k);

#ifdef __cplusplus
}
#endif

#endif /* PERM_MI355X_H */
