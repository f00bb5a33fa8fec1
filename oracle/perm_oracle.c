/*
 * perm_oracle.c -- CPU oracle for matrix permanents.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * Everything here is deliberately plain: no blocking, no fusion, no
 * vectorisation tricks.  Floating-point work is done in x87 long double
 * (64-bit mantissa) with Kahan-compensated sums, i.e. with more precision
 * than the double-precision method under test; binary matrices are done in
 * exact multi-word integer arithmetic.
 *
 * Functions and the passage of the paper (arXiv 2502.16577, "SUperman") each
 * one follows:
 *
 *   orc_brute_real / orc_brute_cplx       Eq. (1): sum over all permutations
 *                                         of prod_i a[i][sigma(i)].
 *   orc_inclexcl_real / orc_inclexcl_cplx Eq. (2): Ryser inclusion-exclusion
 *                                         over all 2^n column subsets, no
 *                                         Gray code, no Nijenhuis-Wilf halving.
 *   orc_ryser_real / orc_ryser_cplx       Algorithm 1 (Gray-code Ryser with
 *                                         the Nijenhuis-Wilf start vector),
 *                                         split into chunks as in Algorithm 3
 *                                         (each chunk re-derives x from the
 *                                         Gray code of the step before it).
 *                                         Also returns R(A) = 2 * sum_g |term_g|.
 *   orc_ryser_csc_real                    Algorithm 2 (SpaRyser): the same walk
 *                                         on a matrix given by its columns in
 *                                         CSC form, where a step adds only the
 *                                         nonzeros of the flipped column to x
 *                                         (Section 2.1; the printed algorithm
 *                                         leaves this update out).
 *   orc_ryser_binary                      Algorithm 2 on a 0/1 matrix in exact
 *                                         integers: y = 2x is integral, every
 *                                         term is an exact 384-bit integer, and
 *                                         a term is skipped when some y_i == 0
 *                                         (its product is exactly zero).
 *   orc_matchings_dp                      Number of perfect matchings of the
 *                                         bipartite graph of a 0/1 matrix by a
 *                                         row-by-row DP over used-column masks;
 *                                         equals perm for 0/1 matrices
 *                                         (Section 1).  An independent
 *                                         algorithm, used to pin the above.
 *   orc_gray, orc_flip_col, orc_flip_sign Section 2 / Table 1: Gray_g =
 *                                         g xor (g >> 1), the changed bit, and
 *                                         whether it is added or removed.
 *
 * Conventions: real matrices are row-major double[n*n]; complex matrices are
 * row-major interleaved (re, im) double[2*n*n].  Results in long double are
 * returned as an unevaluated pair (hi, lo) of doubles with hi = (double)v and
 * lo = (double)(v - hi).  Column indices are 0-based; bit j of a Gray code
 * selects column j, and column n-1 is the one fixed by the Nijenhuis-Wilf
 * extension (never flipped).
 *
 * Return value of every entry point: 0 on success, -1 for a bad argument.
 *
 * Mutation hooks (ORC_MUTANT): the test suite rebuilds this file with
 * -DORC_MUTANT=k to plant one plausible mistake at a time and checks that the
 * pins catch each one.  The default build (ORC_MUTANT undefined or 0) has no
 * mutation.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <unistd.h>

#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

typedef long double ld;

/* ------------------------------------------------------------------------ */
/* Small helpers                                                            */
/* ------------------------------------------------------------------------ */

static void ld_split(ld v, double out[2])
{
    double hi = (double)v;
    out[0] = hi;
    out[1] = (double)(v - (ld)hi);
}

/* Kahan compensated sum (Section 5 uses it for the thread partials). */
typedef struct { ld s, c; } kahan_t;

static void kahan_add(kahan_t *k, ld v)
{
    ld y = v - k->c;
    ld t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

uint64_t orc_gray(uint64_t g) { return g ^ (g >> 1); }

/* Column flipped between Gray_{g-1} and Gray_g (g >= 1): log2 of their xor. */
int orc_flip_col(uint64_t g)
{
    uint64_t d = orc_gray(g) ^ orc_gray(g - 1);
    int j = 0;
    while ((d >> j) != 1) j++;
    return j;
}

/* +1 if column orc_flip_col(g) is added at step g, -1 if it is removed. */
int orc_flip_sign(uint64_t g)
{
    int j = orc_flip_col(g);
    return ((orc_gray(g) >> j) & 1) ? 1 : -1;
}

static int default_threads(int nthreads)
{
    if (nthreads > 0) return nthreads;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

/* ------------------------------------------------------------------------ */
/* Eq. (1): brute force over permutations                                   */
/* ------------------------------------------------------------------------ */

/* Next permutation in lexicographic order; returns 0 after the last one. */
static int next_permutation(int *p, int n)
{
    int i = n - 2;
    while (i >= 0 && p[i] >= p[i + 1]) i--;
    if (i < 0) return 0;
    int j = n - 1;
    while (p[j] <= p[i]) j--;
    int t = p[i]; p[i] = p[j]; p[j] = t;
    for (int a = i + 1, b = n - 1; a < b; a++, b--) {
        t = p[a]; p[a] = p[b]; p[b] = t;
    }
    return 1;
}

int orc_brute_real(int n, const double *a, double out[2])
{
    if (n < 0 || n > 12 || (n > 0 && !a) || !out) return -1;
    int sigma[12];
    for (int i = 0; i < n; i++) sigma[i] = i;
    kahan_t acc = {0, 0};
    do {
        ld prod = 1;
        for (int i = 0; i < n; i++) prod *= (ld)a[i * n + sigma[i]];
#if ORC_MUTANT == 1
        if (n > 1 && sigma[0] == 1) continue;   /* drops a set of permutations */
#endif
        kahan_add(&acc, prod);
    } while (n > 0 && next_permutation(sigma, n));
    ld_split(acc.s - acc.c, out);
    return 0;
}

int orc_brute_cplx(int n, const double *a, double out[4])
{
    if (n < 0 || n > 12 || (n > 0 && !a) || !out) return -1;
    int sigma[12];
    for (int i = 0; i < n; i++) sigma[i] = i;
    kahan_t re = {0, 0}, im = {0, 0};
    do {
        ld pr = 1, pi = 0;
        for (int i = 0; i < n; i++) {
            ld ar = a[2 * (i * n + sigma[i])], ai = a[2 * (i * n + sigma[i]) + 1];
            ld nr = pr * ar - pi * ai;
            ld ni = pr * ai + pi * ar;
            pr = nr; pi = ni;
        }
        kahan_add(&re, pr);
        kahan_add(&im, pi);
    } while (n > 0 && next_permutation(sigma, n));
    ld_split(re.s - re.c, out);
    ld_split(im.s - im.c, out + 2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. (2): inclusion-exclusion over all 2^n column subsets                 */
/* ------------------------------------------------------------------------ */

int orc_inclexcl_real(int n, const double *a, double out[2])
{
    if (n < 0 || n > 24 || (n > 0 && !a) || !out) return -1;
    kahan_t acc = {0, 0};
    uint64_t nsub = 1ull << n;
    for (uint64_t S = 0; S < nsub; S++) {
        ld prod = 1;
        for (int i = 0; i < n; i++) {
            ld rs = 0;
            for (int j = 0; j < n; j++)
                if ((S >> j) & 1) rs += (ld)a[i * n + j];
            prod *= rs;
        }
        int card = __builtin_popcountll(S);
        kahan_add(&acc, (card & 1) ? -prod : prod);
    }
    ld v = acc.s - acc.c;
#if ORC_MUTANT != 8
    if (n & 1) v = -v;                          /* (-1)^n */
#endif
    ld_split(v, out);
    return 0;
}

int orc_inclexcl_cplx(int n, const double *a, double out[4])
{
    if (n < 0 || n > 24 || (n > 0 && !a) || !out) return -1;
    kahan_t re = {0, 0}, im = {0, 0};
    uint64_t nsub = 1ull << n;
    for (uint64_t S = 0; S < nsub; S++) {
        ld pr = 1, pi = 0;
        for (int i = 0; i < n; i++) {
            ld sr = 0, si = 0;
            for (int j = 0; j < n; j++)
                if ((S >> j) & 1) { sr += a[2 * (i * n + j)]; si += a[2 * (i * n + j) + 1]; }
            ld nr = pr * sr - pi * si;
            ld ni = pr * si + pi * sr;
            pr = nr; pi = ni;
        }
        int neg = __builtin_popcountll(S) & 1;
        kahan_add(&re, neg ? -pr : pr);
        kahan_add(&im, neg ? -pi : pi);
    }
    ld vr = re.s - re.c, vi = im.s - im.c;
    if (n & 1) { vr = -vr; vi = -vi; }
    ld_split(vr, out);
    ld_split(vi, out + 2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 split into chunks as in Algorithm 3 (real and complex)       */
/* ------------------------------------------------------------------------ */

/* Steps g = 1 .. 2^(n-1)-1 are cut into chunks of ORC_CHUNK consecutive
 * steps; every chunk starts from x rebuilt from Gray_{start-1} (Algorithm 3)
 * so rounding drift never spans more than one chunk.  Chunks are grouped
 * into work items; item results are combined in item order, so the result
 * does not depend on the number of threads. */
#define ORC_CHUNK 4096ull

typedef struct {
    int n, cplx;
    const double *a;        /* dense row-major matrix, or NULL when csc_* is given */
    const int32_t *csc_ptr, *csc_row;   /* CSC columns (real only) */
    const double *csc_val;
    ld *x0r, *x0i;          /* Nijenhuis-Wilf start vector */
    uint64_t steps;         /* 2^(n-1) - 1 loop iterations */
    uint64_t nitems, chunks_per_item;
    ld *item_re, *item_im, *item_abs;
    uint64_t next_item;     /* atomic work counter */
    uint64_t first_chunk;   /* chunk index of item 0 (0 except for samples) */
} ryser_job_t;

/* x += sign * column j of the matrix (every row for a dense matrix, the
 * column's nonzeros for a CSC one). */
static inline void add_column(const ryser_job_t *J, int j, int sign, ld *xr, ld *xi)
{
    const int n = J->n;
    if (J->csc_ptr) {
        const int32_t q0 = J->csc_ptr[j], q1 = J->csc_ptr[j + 1];
        if (sign > 0)
            for (int32_t q = q0; q < q1; q++) xr[J->csc_row[q]] += J->csc_val[q];
        else
            for (int32_t q = q0; q < q1; q++) xr[J->csc_row[q]] -= J->csc_val[q];
#if ORC_MUTANT == 11
        if (q1 > q0)                               /* loses the column's first nonzero */
            xr[J->csc_row[q0]] -= sign * (ld)J->csc_val[q0];
#endif
        return;
    }
    if (J->cplx) {
        const double *c = J->a;
        if (sign > 0)
            for (int i = 0; i < n; i++) { xr[i] += c[2 * (i * n + j)]; xi[i] += c[2 * (i * n + j) + 1]; }
        else
            for (int i = 0; i < n; i++) { xr[i] -= c[2 * (i * n + j)]; xi[i] -= c[2 * (i * n + j) + 1]; }
        return;
    }
#if ORC_MUTANT == 4
    const int rs = 1, cs = n;                      /* transposed operand */
#else
    const int rs = n, cs = 1;                      /* a_ij at a[i * n + j] */
#endif
    if (sign > 0)
        for (int i = 0; i < n; i++) xr[i] += J->a[i * rs + j * cs];
    else
        for (int i = 0; i < n; i++) xr[i] -= J->a[i * rs + j * cs];
}

static void ryser_range(const ryser_job_t *J, uint64_t start, uint64_t end,
                        kahan_t *kre, kahan_t *kim, ld *abs_sum)
{
    /* Run steps g = start .. end (inclusive), 1 <= start <= end. */
    const int n = J->n;
    ld xr[64], xi[64];
    for (int i = 0; i < n; i++) { xr[i] = J->x0r[i]; xi[i] = J->cplx ? J->x0i[i] : 0; }
    /* x of the subset Gray_{start-1}, rebuilt from the start vector
     * (Algorithm 3: every chunk begins from a freshly derived state). */
    uint64_t gp = orc_gray(start - 1);
    for (int j = 0; j < n - 1; j++)
        if ((gp >> j) & 1) add_column(J, j, 1, xr, xi);
    for (uint64_t g = start; g <= end; g++) {
        int j = orc_flip_col(g);
        int s = orc_flip_sign(g);
#if ORC_MUTANT == 2
        s = -s;                                   /* wrong update sign */
#endif
#if ORC_MUTANT == 3
        if (j > 0) j = j - 1;                     /* wrong column index */
#endif
        add_column(J, j, s, xr, xi);
        ld pr = 1, pi = 0;
        if (J->cplx) {
            for (int i = 0; i < n; i++) {
                ld nr = pr * xr[i] - pi * xi[i];
                ld ni = pr * xi[i] + pi * xr[i];
#if ORC_MUTANT == 6
                ni = pr * xi[i] - pi * xr[i];     /* conjugation slip */
#endif
                pr = nr; pi = ni;
            }
        } else {
            for (int i = 0; i < n; i++) pr *= xr[i];
        }
        if (g & 1) { pr = -pr; pi = -pi; }         /* (-1)^g */
        kahan_add(kre, pr);
        if (J->cplx) kahan_add(kim, pi);
#if ORC_MUTANT == 10
        *abs_sum += J->cplx ? (pr < 0 ? -pr : pr) + (pi < 0 ? -pi : pi)   /* |re| + |im| */
                            : (pr < 0 ? -pr : pr);
#else
        *abs_sum += J->cplx ? __builtin_sqrtl(pr * pr + pi * pi) : (pr < 0 ? -pr : pr);
#endif
    }
}

static void *ryser_worker(void *arg)
{
    ryser_job_t *J = (ryser_job_t *)arg;
    for (;;) {
        uint64_t it = __atomic_fetch_add(&J->next_item, 1, __ATOMIC_RELAXED);
        if (it >= J->nitems) break;
        kahan_t kre = {0, 0}, kim = {0, 0};
        ld abs_sum = 0;
        uint64_t c0 = J->first_chunk + it * J->chunks_per_item;
        for (uint64_t c = c0; c < c0 + J->chunks_per_item; c++) {
            uint64_t start = c * ORC_CHUNK + 1;
            if (start > J->steps) break;
            uint64_t end = start + ORC_CHUNK - 1;
            if (end > J->steps) end = J->steps;     /* clamp to 2^(n-1)-1 */
            kahan_t cre = {0, 0}, cim = {0, 0};
            ryser_range(J, start, end, &cre, &cim, &abs_sum);
            kahan_add(&kre, cre.s - cre.c);
            kahan_add(&kim, cim.s - cim.c);
        }
        J->item_re[it] = kre.s - kre.c;
        J->item_im[it] = kim.s - kim.c;
        J->item_abs[it] = abs_sum;
    }
    return NULL;
}

/* Runs steps 1 .. 2^(n-1)-1 of the walk of job J (x0r / x0i set) over
 * nthreads threads, adds the g = 0 term prod_i x0_i, and writes
 * 2 (-1)^(n-1) times the sum (Algorithm 1's final factor 4 (n mod 2) - 2)
 * and R(A) = 2 sum_g |term_g|. */
static int walk_all(ryser_job_t *J, int nthreads, double out[4], double absum[2])
{
    const int n = J->n, cplx = J->cplx;
    /* the empty subset's term (g = 0): the product of the start vector */
    ld p0r = 1, p0i = 0;
    for (int i = 0; i < n; i++) {
        ld nr = p0r * J->x0r[i] - p0i * J->x0i[i];
        ld ni = p0r * J->x0i[i] + p0i * J->x0r[i];
        p0r = nr; p0i = ni;
    }
    J->steps = (1ull << (n - 1)) - 1;
    uint64_t nchunks = (J->steps + ORC_CHUNK - 1) / ORC_CHUNK;
    J->chunks_per_item = 1;
    while (nchunks / J->chunks_per_item > (1ull << 16)) J->chunks_per_item <<= 1;
    J->nitems = (nchunks + J->chunks_per_item - 1) / J->chunks_per_item;
    size_t nb = (J->nitems ? J->nitems : 1) * sizeof(ld);
    J->item_re = (ld *)calloc(1, nb);
    J->item_im = (ld *)calloc(1, nb);
    J->item_abs = (ld *)calloc(1, nb);
    if (!J->item_re || !J->item_im || !J->item_abs) {
        free(J->item_re); free(J->item_im); free(J->item_abs);
        return -1;
    }
    int T = default_threads(nthreads);
    if ((uint64_t)T > J->nitems) T = J->nitems ? (int)J->nitems : 1;
    if (T > 256) T = 256;
    pthread_t th[256];
    int ok[256] = {0};
    for (int t = 1; t < T; t++) ok[t] = pthread_create(&th[t], NULL, ryser_worker, J) == 0;
    ryser_worker(J);
    for (int t = 1; t < T; t++) if (ok[t]) pthread_join(th[t], NULL);

    kahan_t kre = {0, 0}, kim = {0, 0};
    kahan_add(&kre, p0r);
    kahan_add(&kim, p0i);
    ld abs_sum = cplx ? __builtin_sqrtl(p0r * p0r + p0i * p0i) : (p0r < 0 ? -p0r : p0r);
    for (uint64_t it = 0; it < J->nitems; it++) {
        kahan_add(&kre, J->item_re[it]);
        kahan_add(&kim, J->item_im[it]);
        abs_sum += J->item_abs[it];
    }
    free(J->item_re); free(J->item_im); free(J->item_abs);

    ld f = (n & 1) ? 2 : -2;                    /* 2 (-1)^(n-1) */
    ld_split(f * (kre.s - kre.c), out);
    if (cplx) ld_split(f * (kim.s - kim.c), out + 2);
#if ORC_MUTANT == 9
    if (absum) ld_split(abs_sum, absum);        /* loses the factor 2 */
#else
    if (absum) ld_split(2 * abs_sum, absum);
#endif
    return 0;
}

static int ryser_common(int n, const double *a, int cplx, int nthreads,
                        double out[4], double absum[2])
{
    if (n < 0 || n > 63 || (n > 0 && !a) || !out) return -1;
    if (n == 0) {
        double one[2] = {1.0, 0.0};
        memcpy(out, one, sizeof one);
        if (cplx) { out[2] = 0; out[3] = 0; }
        if (absum) { absum[0] = 1.0; absum[1] = 0.0; }
        return 0;
    }
    ld x0r[64], x0i[64];
    /* Algorithm 1's start vector: x_i = a_{i,n} - (row sum)/2, with a_{i,n}
     * the entry in the last (never flipped) column. */
    for (int i = 0; i < n; i++) {
        ld sr = 0, si = 0;
        for (int j = 0; j < n; j++) {
            if (cplx) { sr += a[2 * (i * n + j)]; si += a[2 * (i * n + j) + 1]; }
            else sr += a[i * n + j];
        }
        if (cplx) {
            x0r[i] = a[2 * (i * n + n - 1)] - sr / 2;
            x0i[i] = a[2 * (i * n + n - 1) + 1] - si / 2;
        } else {
#if ORC_MUTANT == 5
            x0r[i] = a[i * n + n - 1] - sr;       /* lost factor 1/2 */
#else
            x0r[i] = a[i * n + n - 1] - sr / 2;
#endif
            x0i[i] = 0;
        }
    }
    ryser_job_t J;
    memset(&J, 0, sizeof J);
    J.n = n; J.cplx = cplx; J.a = a; J.x0r = x0r; J.x0i = x0i;
    return walk_all(&J, nthreads, out, absum);
}

int orc_ryser_real(int n, const double *a, int nthreads, double out[2], double absum[2])
{
    double tmp[4];
    int rc = ryser_common(n, a, 0, nthreads, tmp, absum);
    if (rc == 0) { out[0] = tmp[0]; out[1] = tmp[1]; }
    return rc;
}

int orc_ryser_cplx(int n, const double *a, int nthreads, double out[4], double absum[2])
{
    return ryser_common(n, a, 1, nthreads, out, absum);
}

/* Partial sum of Algorithm 1 over the chunks [first_chunk, first_chunk +
 * nchunks) of ORC_CHUNK steps each (no final scaling, no g = 0 term).  Used
 * only to time the oracle on a bounded sample of a large workload. */
int orc_ryser_real_sample(int n, const double *a, int nthreads, uint64_t first_chunk,
                          uint64_t nchunks, double out[2])
{
    if (n < 2 || n > 63 || !a || !out) return -1;
    ld x0r[64], x0i[64];
    for (int i = 0; i < n; i++) {
        ld sr = 0;
        for (int j = 0; j < n; j++) sr += a[i * n + j];
        x0r[i] = a[i * n + n - 1] - sr / 2;
        x0i[i] = 0;
    }
    ryser_job_t J;
    memset(&J, 0, sizeof J);
    J.n = n; J.cplx = 0; J.a = a; J.x0r = x0r; J.x0i = x0i;
    J.steps = (1ull << (n - 1)) - 1;
    uint64_t total_chunks = (J.steps + ORC_CHUNK - 1) / ORC_CHUNK;
    if (first_chunk >= total_chunks) return -1;
    if (first_chunk + nchunks > total_chunks) nchunks = total_chunks - first_chunk;
    /* one work item per chunk of the sample, offset by first_chunk */
    J.chunks_per_item = 1;
    J.nitems = nchunks;
    J.item_re = (ld *)calloc(nchunks ? nchunks : 1, sizeof(ld));
    J.item_im = (ld *)calloc(nchunks ? nchunks : 1, sizeof(ld));
    J.item_abs = (ld *)calloc(nchunks ? nchunks : 1, sizeof(ld));
    if (!J.item_re || !J.item_im || !J.item_abs) {
        free(J.item_re); free(J.item_im); free(J.item_abs);
        return -1;
    }
    J.first_chunk = first_chunk;
    int T = default_threads(nthreads);
    if (T > 256) T = 256;
    pthread_t th[256];
    int ok[256] = {0};
    for (int t = 1; t < T; t++) ok[t] = pthread_create(&th[t], NULL, ryser_worker, &J) == 0;
    ryser_worker(&J);
    for (int t = 1; t < T; t++) if (ok[t]) pthread_join(th[t], NULL);
    kahan_t k = {0, 0};
    for (uint64_t it = 0; it < J.nitems; it++) kahan_add(&k, J.item_re[it]);
    free(J.item_re); free(J.item_im); free(J.item_abs);
    ld_split(k.s - k.c, out);
    return 0;
}

/* Part `part` of `nparts` of the unscaled sum of Algorithm 1 for a real
 * matrix, dense (a) or given by CSC columns (col_ptr, row_idx, vals; a is
 * NULL then): the chunks [part*K/nparts, (part+1)*K/nparts) of the walk's
 * K chunks, plus the g = 0 term in part 0.  Written as a (hi, lo) pair, with
 * the part's share of sum_g |term_g| in absum.  The sum of all parts times
 * 2 (-1)^(n-1) is the permanent (the whole walk, grouped differently), so a
 * long sweep can be computed piece by piece and resumed. */
int orc_ryser_real_part(int n, const double *a, const int32_t *col_ptr,
                        const int32_t *row_idx, const double *vals, int nthreads,
                        uint64_t part, uint64_t nparts, double out[2], double absum[2])
{
    if (n < 2 || n > 63 || (!a && !col_ptr) || !out || !absum || nparts == 0 || part >= nparts)
        return -1;
    ld x0r[64], x0i[64];
    for (int i = 0; i < n; i++) { x0r[i] = 0; x0i[i] = 0; }
    if (a) {
        for (int i = 0; i < n; i++) {
            ld sr = 0;
            for (int j = 0; j < n; j++) sr += a[i * n + j];
            x0r[i] = a[i * n + n - 1] - sr / 2;
        }
    } else {
        /* row sums and last-column entries from the stored nonzeros */
        ld rsum[64], last[64];
        for (int i = 0; i < n; i++) { rsum[i] = 0; last[i] = 0; }
        if (col_ptr[0] != 0) return -1;
        for (int j = 0; j < n; j++) {
            if (col_ptr[j + 1] < col_ptr[j]) return -1;
            for (int32_t q = col_ptr[j]; q < col_ptr[j + 1]; q++) {
                if (row_idx[q] < 0 || row_idx[q] >= n) return -1;
                rsum[row_idx[q]] += vals[q];
                if (j == n - 1) last[row_idx[q]] = vals[q];
            }
        }
        for (int i = 0; i < n; i++) x0r[i] = last[i] - rsum[i] / 2;
    }
    ryser_job_t J;
    memset(&J, 0, sizeof J);
    J.n = n; J.cplx = 0; J.a = a; J.x0r = x0r; J.x0i = x0i;
    if (!a) { J.csc_ptr = col_ptr; J.csc_row = row_idx; J.csc_val = vals; }
    J.steps = (1ull << (n - 1)) - 1;
    const uint64_t total_chunks = (J.steps + ORC_CHUNK - 1) / ORC_CHUNK;
    /* part boundaries by 128-bit products, so any nparts is exact */
    const uint64_t c0 = (uint64_t)(((unsigned __int128)total_chunks * part) / nparts);
    const uint64_t c1 = (uint64_t)(((unsigned __int128)total_chunks * (part + 1)) / nparts);
    const uint64_t nchunks = c1 - c0;
    J.chunks_per_item = 1;
    J.nitems = nchunks;
    J.first_chunk = c0;
    size_t nb = (nchunks ? nchunks : 1) * sizeof(ld);
    J.item_re = (ld *)calloc(1, nb);
    J.item_im = (ld *)calloc(1, nb);
    J.item_abs = (ld *)calloc(1, nb);
    if (!J.item_re || !J.item_im || !J.item_abs) {
        free(J.item_re); free(J.item_im); free(J.item_abs);
        return -1;
    }
    int T = default_threads(nthreads);
    if (T > 256) T = 256;
    pthread_t th[256];
    int ok[256] = {0};
    for (int t = 1; t < T; t++) ok[t] = pthread_create(&th[t], NULL, ryser_worker, &J) == 0;
    ryser_worker(&J);
    for (int t = 1; t < T; t++) if (ok[t]) pthread_join(th[t], NULL);
    kahan_t k = {0, 0};
    ld abs_sum = 0;
    if (part == 0) {
        ld p0 = 1;
        for (int i = 0; i < n; i++) p0 *= x0r[i];
        kahan_add(&k, p0);
        abs_sum += p0 < 0 ? -p0 : p0;
    }
    for (uint64_t it = 0; it < J.nitems; it++) {
        kahan_add(&k, J.item_re[it]);
        abs_sum += J.item_abs[it];
    }
    free(J.item_re); free(J.item_im); free(J.item_abs);
    ld_split(k.s - k.c, out);
    ld_split(abs_sum, absum);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (SpaRyser): the walk on CSC columns                          */
/* ------------------------------------------------------------------------ */

/*
 * Permanent of a real n x n matrix given by its columns in CSC form
 * (col_ptr[n+1], row_idx[nnz], vals[nnz]; duplicates are not allowed).  The
 * row sums and the entries of the last column come from the stored
 * nonzeros; each step of the Gray walk adds or subtracts only the nonzeros
 * of the flipped column, and the product still runs over every row.  The
 * result equals orc_ryser_real on the dense form of the same matrix.
 */
int orc_ryser_csc_real(int n, const int32_t *col_ptr, const int32_t *row_idx,
                       const double *vals, int nthreads, double out[2], double absum[2])
{
    if (n < 0 || n > 63 || !out || (n > 0 && !col_ptr)) return -1;
    if (n == 0) {
        out[0] = 1.0; out[1] = 0.0;
        if (absum) { absum[0] = 1.0; absum[1] = 0.0; }
        return 0;
    }
    if (col_ptr[0] != 0) return -1;
    for (int j = 0; j < n; j++) {
        if (col_ptr[j + 1] < col_ptr[j]) return -1;
        for (int32_t q = col_ptr[j]; q < col_ptr[j + 1]; q++)
            if (row_idx[q] < 0 || row_idx[q] >= n) return -1;
    }
    /* row sums and last-column entries, columns taken in ascending order
     * (the dense oracle's order of summation; absent entries are zeros) */
    ld rsum[64], last[64], x0r[64], x0i[64];
    for (int i = 0; i < n; i++) { rsum[i] = 0; last[i] = 0; x0i[i] = 0; }
    for (int j = 0; j < n; j++)
        for (int32_t q = col_ptr[j]; q < col_ptr[j + 1]; q++) {
            rsum[row_idx[q]] += vals[q];
            if (j == n - 1) last[row_idx[q]] = vals[q];
        }
    for (int i = 0; i < n; i++) x0r[i] = last[i] - rsum[i] / 2;
    ryser_job_t J;
    memset(&J, 0, sizeof J);
    J.n = n; J.cplx = 0; J.a = NULL;
    J.csc_ptr = col_ptr; J.csc_row = row_idx; J.csc_val = vals;
    J.x0r = x0r; J.x0i = x0i;
    double tmp[4];
    int rc = walk_all(&J, nthreads, tmp, absum);
    if (rc == 0) { out[0] = tmp[0]; out[1] = tmp[1]; }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Exact binary permanent: Algorithm 2 on y = 2x in 384-bit integers          */
/* ------------------------------------------------------------------------ */

#define LIMBS 6   /* 384 bits: |2^(n-1) perm| <= 2^62 * 63! < 2^352 */

typedef struct { uint64_t w[LIMBS]; } big_t;   /* two's complement, wraps mod 2^384 */

static void big_add(big_t *acc, const big_t *v)
{
    unsigned __int128 carry = 0;
    for (int k = 0; k < LIMBS; k++) {
        carry += (unsigned __int128)acc->w[k] + v->w[k];
        acc->w[k] = (uint64_t)carry;
        carry >>= 64;
    }
}

static void big_sub(big_t *acc, const big_t *v)
{
    uint64_t borrow = 0;
    for (int k = 0; k < LIMBS; k++) {
        unsigned __int128 d = (unsigned __int128)acc->w[k] - v->w[k] - borrow;
        acc->w[k] = (uint64_t)d;
        borrow = (uint64_t)(d >> 64) ? 1 : 0;
    }
}

static void big_mul_small(big_t *v, uint64_t m)
{
    unsigned __int128 carry = 0;
    for (int k = 0; k < LIMBS; k++) {
        carry += (unsigned __int128)v->w[k] * m;
        v->w[k] = (uint64_t)carry;
        carry >>= 64;
    }
}

typedef struct {
    int n;
    const int32_t *cptr, *ridx;   /* CCS of the 0/1 pattern */
    const int64_t *y0;            /* 2 * Nijenhuis-Wilf start vector */
    uint64_t steps, nitems, chunks_per_item, next_item;
    big_t *item;
    uint64_t *item_nonzero;       /* number of nonzero terms (statistics) */
} bin_job_t;

static void bin_term(const int64_t *y, int n, int negative, big_t *acc)
{
    big_t mag;
    memset(&mag, 0, sizeof mag);
    mag.w[0] = 1;
    for (int i = 0; i < n; i++) {
        int64_t v = y[i];
        if (v < 0) { negative = !negative; v = -v; }
        big_mul_small(&mag, (uint64_t)v);
    }
    if (negative) big_sub(acc, &mag); else big_add(acc, &mag);
}

static void *bin_worker(void *arg)
{
    bin_job_t *J = (bin_job_t *)arg;
    const int n = J->n;
    for (;;) {
        uint64_t it = __atomic_fetch_add(&J->next_item, 1, __ATOMIC_RELAXED);
        if (it >= J->nitems) break;
        big_t acc;
        memset(&acc, 0, sizeof acc);
        uint64_t nonzero = 0;
        uint64_t c0 = it * J->chunks_per_item;
        for (uint64_t c = c0; c < c0 + J->chunks_per_item; c++) {
            uint64_t start = c * ORC_CHUNK + 1;
            if (start > J->steps) break;
            uint64_t end = start + ORC_CHUNK - 1;
            if (end > J->steps) end = J->steps;
            int64_t y[64];
            for (int i = 0; i < n; i++) y[i] = J->y0[i];
            uint64_t gp = orc_gray(start - 1);
            for (int j = 0; j < n - 1; j++)
                if ((gp >> j) & 1)
                    for (int32_t p = J->cptr[j]; p < J->cptr[j + 1]; p++) y[J->ridx[p]] += 2;
            int zeros = 0;
            for (int i = 0; i < n; i++) zeros += (y[i] == 0);
            for (uint64_t g = start; g <= end; g++) {
                int j = orc_flip_col(g);
                int s = orc_flip_sign(g);
                for (int32_t p = J->cptr[j]; p < J->cptr[j + 1]; p++) {
                    int r = J->ridx[p];
                    zeros -= (y[r] == 0);
                    y[r] += 2 * s;
                    zeros += (y[r] == 0);
                }
                if (zeros) continue;                /* product is exactly 0 */
                nonzero++;
                bin_term(y, n, (int)(g & 1), &acc);
            }
        }
        J->item[it] = acc;
        J->item_nonzero[it] = nonzero;
    }
    return NULL;
}

/*
 * Exact permanent of a 0/1 matrix given as row-major unsigned char[n*n]
 * (entries must be 0 or 1), 1 <= n <= 63.
 * out_limbs[6]: perm as an unsigned little-endian 384-bit integer.
 * out_nonzero (nullable): number of steps whose term was nonzero.
 * Returns 0, -1 on bad input, -2 if an internal exactness check fails.
 */
int orc_ryser_binary(int n, const unsigned char *a, int nthreads, uint64_t out_limbs[6],
                     uint64_t *out_nonzero)
{
    if (n < 1 || n > 63 || !a || !out_limbs) return -1;
    for (int k = 0; k < n * n; k++) if (a[k] > 1) return -1;
    int32_t *cptr = (int32_t *)calloc(n + 1, sizeof(int32_t));
    int32_t *ridx = (int32_t *)calloc(n * n + 1, sizeof(int32_t));
    if (!cptr || !ridx) { free(cptr); free(ridx); return -1; }
    int nnz = 0;
    for (int j = 0; j < n; j++) {
        cptr[j] = nnz;
        for (int i = 0; i < n; i++) if (a[i * n + j]) ridx[nnz++] = i;
    }
    cptr[n] = nnz;
    int64_t y0[64];
    for (int i = 0; i < n; i++) {
        int64_t r = 0;
        for (int j = 0; j < n; j++) r += a[i * n + j];
#if ORC_MUTANT == 7
        y0[i] = 2 * (int64_t)a[i * n] - r;            /* wrong fixed column */
#else
        y0[i] = 2 * (int64_t)a[i * n + n - 1] - r;    /* y = 2 (a_{i,n} - r_i / 2) */
#endif
    }
    bin_job_t J;
    memset(&J, 0, sizeof J);
    J.n = n; J.cptr = cptr; J.ridx = ridx; J.y0 = y0;
    J.steps = (1ull << (n - 1)) - 1;
    uint64_t nchunks = (J.steps + ORC_CHUNK - 1) / ORC_CHUNK;
    J.chunks_per_item = 1;
    while (nchunks / J.chunks_per_item > (1ull << 16)) J.chunks_per_item <<= 1;
    J.nitems = (nchunks + J.chunks_per_item - 1) / J.chunks_per_item;
    size_t ni = J.nitems ? J.nitems : 1;
    J.item = (big_t *)calloc(ni, sizeof(big_t));
    J.item_nonzero = (uint64_t *)calloc(ni, sizeof(uint64_t));
    if (!J.item || !J.item_nonzero) {
        free(J.item); free(J.item_nonzero); free(cptr); free(ridx);
        return -1;
    }
    int T = default_threads(nthreads);
    if ((uint64_t)T > J.nitems) T = J.nitems ? (int)J.nitems : 1;
    if (T > 256) T = 256;
    pthread_t th[256];
    int ok[256] = {0};
    for (int t = 1; t < T; t++) ok[t] = pthread_create(&th[t], NULL, bin_worker, &J) == 0;
    bin_worker(&J);
    for (int t = 1; t < T; t++) if (ok[t]) pthread_join(th[t], NULL);

    big_t acc;
    memset(&acc, 0, sizeof acc);
    uint64_t nonzero = 0;
    int zeros0 = 0;
    for (int i = 0; i < n; i++) zeros0 += (y0[i] == 0);
    if (!zeros0) { nonzero++; bin_term(y0, n, 0, &acc); }   /* g = 0 */
    for (uint64_t it = 0; it < J.nitems; it++) {
        big_add(&acc, &J.item[it]);
        nonzero += J.item_nonzero[it];
    }
    free(J.item); free(J.item_nonzero); free(cptr); free(ridx);

    /* acc = (-1)^(n-1) 2^(n-1) perm.  Undo the sign, then check that the low
     * n-1 bits are zero and shift them out. */
    if (!(n & 1)) {                   /* (-1)^(n-1) = -1: negate */
        big_t z;
        memset(&z, 0, sizeof z);
        big_sub(&z, &acc);
        acc = z;
    }
    if (acc.w[LIMBS - 1] >> 63) return -2;      /* a permanent of a 0/1 matrix is >= 0 */
    int sh = n - 1;
    for (int b = 0; b < sh; b++)
        if ((acc.w[b / 64] >> (b % 64)) & 1) return -2;
    for (int k = 0; k < LIMBS; k++) {
        uint64_t lo = acc.w[k] >> sh;
        uint64_t hi = (k + 1 < LIMBS && sh) ? (acc.w[k + 1] << (64 - sh)) : 0;
        out_limbs[k] = sh ? (lo | hi) : acc.w[k];
    }
    if (out_nonzero) *out_nonzero = nonzero;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Perfect matchings of a 0/1 matrix by DP over used-column masks             */
/* ------------------------------------------------------------------------ */

/* dp[mask] = number of ways to match rows 0..popcount(mask)-1 to exactly the
 * columns in mask.  n <= 26; the count is returned as a 128-bit integer in
 * out[0] (low) / out[1] (high). */
int orc_matchings_dp(int n, const unsigned char *a, uint64_t out[2])
{
    if (n < 0 || n > 26 || (n > 0 && !a) || !out) return -1;
    if (n == 0) { out[0] = 1; out[1] = 0; return 0; }
    uint64_t nmask = 1ull << n;
    unsigned __int128 *dp = (unsigned __int128 *)calloc(nmask, sizeof(unsigned __int128));
    if (!dp) return -1;
    dp[0] = 1;
    for (uint64_t mask = 0; mask < nmask; mask++) {
        if (!dp[mask]) continue;
        int row = __builtin_popcountll(mask);
        if (row >= n) continue;
        for (int j = 0; j < n; j++)
            if (!((mask >> j) & 1) && a[row * n + j]) dp[mask | (1ull << j)] += dp[mask];
    }
    unsigned __int128 v = dp[nmask - 1];
    free(dp);
    out[0] = (uint64_t)v;
    out[1] = (uint64_t)(v >> 64);
    return 0;
}
