// Sparse preprocessing of Section 4: fine-grain Dulmage-Mendelsohn pruning
// (Section 4.1) and the Forbert-Marx decomposition driven by Algorithm 4
// (DecompRyser).  Host code: it turns one sparse matrix into a list of
// weighted smaller matrices ("leaves") whose permanents, times the weights,
// sum to the permanent of the input.  The leaves are then solved on the GPU
// (batched launch) and summed by perm_weighted_sum.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "perm.h"

namespace {

struct Mat {  // dense square matrix, row-major
    int n = 0;
    std::vector<double> a;
    double &at(int i, int j) { return a[size_t(i) * n + j]; }
    double at(int i, int j) const { return a[size_t(i) * n + j]; }
};

struct Leaf {
    double weight;
    Mat m;
};

// ---- Section 4.1: perfect matching, orientation, SCCs, pruning -------------

// Maximum bipartite matching by augmenting paths (n <= 63, so O(n^3) is
// trivial).  match_col[j] = row matched to column j, or -1.
bool perfect_matching(const Mat &A, std::vector<int> &match_row, std::vector<int> &match_col)
{
    const int n = A.n;
    match_row.assign(n, -1);
    match_col.assign(n, -1);
    std::vector<int> seen;
    // augmenting-path search; recursion depth <= n
    struct Aug {
        const Mat &A;
        std::vector<int> &mr, &mc, &seen;
        int stamp = 0;
        bool run(int i)
        {
            for (int j = 0; j < A.n; ++j) {
                if (A.at(i, j) == 0.0 || seen[j] == stamp) continue;
                seen[j] = stamp;
                if (mc[j] < 0 || run(mc[j])) {
                    mc[j] = i;
                    mr[i] = j;
                    return true;
                }
            }
            return false;
        }
    };
    seen.assign(n, -1);
    Aug aug{A, match_row, match_col, seen};
    for (int i = 0; i < n; ++i) {
        aug.stamp = i;
        if (!aug.run(i)) return false;
    }
    return true;
}

// Tarjan's strongly connected components on the directed bipartite graph
// of Section 4.1: vertices 0..n-1 rows, n..2n-1 columns; matching edges go
// row -> column, the other nonzeros column -> row.
std::vector<int> sccs(const Mat &A, const std::vector<int> &match_row)
{
    const int n = A.n, V = 2 * n;
    std::vector<std::vector<int>> adj(V);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (A.at(i, j) == 0.0) continue;
            if (match_row[i] == j) adj[i].push_back(n + j);
            else adj[n + j].push_back(i);
        }
    std::vector<int> index(V, -1), low(V, 0), comp(V, -1), stack;
    std::vector<char> on(V, 0);
    int counter = 0, ncomp = 0;
    struct Frame { int v; size_t e; };
    for (int s = 0; s < V; ++s) {
        if (index[s] >= 0) continue;
        std::vector<Frame> call{{s, 0}};
        index[s] = low[s] = counter++;
        stack.push_back(s);
        on[s] = 1;
        while (!call.empty()) {
            Frame &f = call.back();
            if (f.e < adj[f.v].size()) {
                const int w = adj[f.v][f.e++];
                if (index[w] < 0) {
                    index[w] = low[w] = counter++;
                    stack.push_back(w);
                    on[w] = 1;
                    call.push_back({w, 0});
                } else if (on[w]) {
                    low[f.v] = std::min(low[f.v], index[w]);
                }
            } else {
                const int v = f.v;
                if (low[v] == index[v]) {
                    int w;
                    do {
                        w = stack.back();
                        stack.pop_back();
                        on[w] = 0;
                        comp[w] = ncomp;
                    } while (w != v);
                    ++ncomp;
                }
                call.pop_back();
                if (!call.empty()) low[call.back().v] = std::min(low[call.back().v], low[v]);
            }
        }
    }
    return comp;
}

// Deletes the nonzeros outside the matching whose row and column lie in
// different SCCs: such an edge is on no alternating cycle, so it belongs to
// no perfect matching and multiplies zero in every term of Eq. (1).  The
// matching's own edges form a perfect matching and are always kept.
// Returns false if there is no perfect matching (perm = 0).
bool dm_prune(Mat &A, int64_t &removed)
{
    std::vector<int> mr, mc;
    if (!perfect_matching(A, mr, mc)) return false;
    const std::vector<int> comp = sccs(A, mr);
    for (int i = 0; i < A.n; ++i)
        for (int j = 0; j < A.n; ++j)
            if (A.at(i, j) != 0.0 && mr[i] != j && comp[i] != comp[A.n + j]) {
                A.at(i, j) = 0.0;
                ++removed;
            }
    return true;
}

// ---- Algorithm 4: DecompRyser ------------------------------------------------

Mat transpose(const Mat &A)
{
    Mat T;
    T.n = A.n;
    T.a.resize(A.a.size());
    for (int i = 0; i < A.n; ++i)
        for (int j = 0; j < A.n; ++j) T.at(j, i) = A.at(i, j);
    return T;
}

// The three reductions of Algorithm 4 on row r with nonzero columns c1 (and
// c2): rows are ordered r first, then the others in order; columns c1, c2
// first, then the others in order (the row and columns moved to the front,
// row 0 = (alpha, beta, c), column 0 = (alpha; d), column 1 = (beta; e)).
// Each builds its child directly from A, with one allocation.
struct Front {
    int n;
    int rows[PERM_MAX_N];  // rows[0] = r
    int cols[PERM_MAX_N];  // cols[0] = c1 (, cols[1] = c2)
    Front(const Mat &A, int r, int c1, int c2) : n(A.n)
    {
        int k = 0;
        rows[k++] = r;
        for (int i = 0; i < n; ++i)
            if (i != r) rows[k++] = i;
        k = 0;
        cols[k++] = c1;
        if (c2 >= 0) cols[k++] = c2;
        for (int j = 0; j < n; ++j)
            if (j != c1 && j != c2) cols[k++] = j;
    }
};

// The minor without row r and column c1 (d1compress).
Mat minor_of(const Mat &A, const Front &F)
{
    const int n = A.n;
    Mat M;
    M.n = n - 1;
    M.a.resize(size_t(n - 1) * (n - 1));
    for (int i = 1; i < n; ++i) {
        const double *src = &A.a[size_t(F.rows[i]) * n];
        double *dst = &M.a[size_t(i - 1) * (n - 1)];
        for (int j = 1; j < n; ++j) dst[j - 1] = src[F.cols[j]];
    }
    return M;
}

// [alpha e + beta d, B]: the (n-1) x (n-1) matrix of the second term.
Mat merged(const Mat &A, const Front &F, double alpha, double beta)
{
    const int n = A.n;
    Mat M;
    M.n = n - 1;
    M.a.resize(size_t(n - 1) * (n - 1));
    for (int i = 1; i < n; ++i) {
        const double *src = &A.a[size_t(F.rows[i]) * n];
        double *dst = &M.a[size_t(i - 1) * (n - 1)];
        dst[0] = alpha * src[F.cols[1]] + beta * src[F.cols[0]];
        for (int j = 2; j < n; ++j) dst[j - 1] = src[F.cols[j]];
    }
    return M;
}

// The first term of d34compress: the permuted matrix with alpha and beta
// replaced by zeros, [0 0 c; d e B].
Mat zeroed_front(const Mat &A, const Front &F)
{
    const int n = A.n;
    Mat Z;
    Z.n = n;
    Z.a.resize(size_t(n) * n);
    for (int i = 0; i < n; ++i) {
        const double *src = &A.a[size_t(F.rows[i]) * n];
        double *dst = &Z.a[size_t(i) * n];
        for (int j = 0; j < n; ++j) dst[j] = src[F.cols[j]];
    }
    Z.a[0] = 0.0;
    Z.a[1] = 0.0;
    return Z;
}

// Double-double accumulator for the folded leaves (two-sum of Ogita, Rump
// and Oishi; products split exactly by FMA).
struct DDSum {
    double hi = 0.0, lo = 0.0;
    void add(double v)
    {
        const double s = hi + v;
        const double bb = s - hi;
        lo += (hi - (s - bb)) + (v - bb);
        hi = s;
    }
    void add_product(double a, double b)
    {
#pragma clang fp contract(off)
        // (p must stay the rounded product: its error is added separately)
        const double p = a * b;
        add(p);
        add(std::fma(a, b, -p));
    }
};

struct Decomposer {
    int min_leaf = 0;              // stop decomposing at this order
    bool fold = false;             // sum leaves of order <= 2 into `folded`
    DDSum folded;
    int64_t split_budget = 1 << 16;  // two-way splits (minNnz 3 or 4) allowed in total
    int64_t max_leaves = 1 << 22;
    std::vector<Leaf> leaves;
    bool overflow = false;

    void rec(Mat A, double w, int depth)
    {
        if (overflow) return;
        if (fold && A.n <= 2) {  // perm of order 0, 1, 2 directly: w, w a, w (ad + bc)
            if (A.n == 0) {
                folded.add(w);
            } else if (A.n == 1) {
                folded.add_product(w, A.a[0]);
            } else {
                folded.add_product(w * A.a[0], A.a[3]);
                folded.add_product(w * A.a[1], A.a[2]);
            }
            return;
        }
        if (A.n == 0) {  // the empty product: a 1 x 1 leaf [1] carries the weight
            Mat one;
            one.n = 1;
            one.a.assign(1, 1.0);
            leaves.push_back(Leaf{w, one});
            return;
        }
        // row or column with the fewest nonzeros (Algorithm 4, getMinimumNnz):
        // all counts in one row-major pass; rows before columns, lower index
        // first among equal counts
        const int n = A.n;
        int cr[PERM_MAX_N] = {}, cc[PERM_MAX_N] = {};
        for (int i = 0; i < n; ++i) {
            const double *row = &A.a[size_t(i) * n];
            for (int j = 0; j < n; ++j) {
                const int nz = row[j] != 0.0;
                cr[i] += nz;
                cc[j] += nz;
            }
        }
        int best = n + 1, best_idx = 0;
        bool best_is_col = false;
        for (int i = 0; i < n; ++i) {
            if (cr[i] < best) { best = cr[i]; best_idx = i; best_is_col = false; }
            if (cc[i] < best) { best = cc[i]; best_idx = i; best_is_col = true; }
        }
        if (best == 0) return;  // an empty row or column: this term is 0
        // the two-way split of minNnz 3 or 4 doubles the work items; once the
        // budget is spent such matrices are solved as they are
        if (best > 4 || n <= min_leaf || (best > 2 && split_budget <= 0)) {
            if (int64_t(leaves.size()) >= max_leaves) { overflow = true; return; }
            leaves.push_back(Leaf{w, std::move(A)});
            return;
        }
        if (best_is_col) A = transpose(A);  // perm(A^T) = perm(A)
        const int r = best_idx;
        int c1 = -1, c2 = -1;
        for (int j = 0; j < n; ++j)
            if (A.at(r, j) != 0.0) {
                if (c1 < 0) c1 = j;
                else if (c2 < 0) c2 = j;
            }
        if (best == 1) {  // d1compress: perm = alpha * perm(minor)
            const Front F(A, r, c1, -1);
            const double alpha = A.at(r, c1);
            rec(minor_of(A, F), w * alpha, depth + 1);
            return;
        }
        const Front F(A, r, c1, c2);
        const double alpha = A.at(r, c1), beta = A.at(r, c2);
        if (best == 2) {  // d2compress: c = 0, only the merged term survives
            rec(merged(A, F, alpha, beta), w, depth + 1);
            return;
        }
        // d34compress: perm = perm([0 0 c; d e B]) + perm([alpha e + beta d, B])
        --split_budget;
        Mat Z = zeroed_front(A, F);
        rec(merged(A, F, alpha, beta), w, depth + 1);
        rec(std::move(Z), w, depth + 1);
    }
};

}  // namespace

struct perm_decomp {
    std::vector<Leaf> leaves;
    double folded[2] = {0.0, 0.0};  // sum of the folded leaves (hi, lo)
    int64_t removed = 0;
    int zero = 0;
};

extern "C" {

int perm_decompose(int n, const int32_t *col_ptr, const int32_t *row_idx, const double *vals,
                   int32_t nnz, int flags, int min_leaf, perm_decomp **out)
{
    if (!out) return PERM_EINVAL;
    *out = nullptr;
    if (n < 1 || n > PERM_MAX_N || !col_ptr || nnz < 0 || (nnz > 0 && (!row_idx || !vals)))
        return PERM_EINVAL;
    if (col_ptr[0] != 0 || col_ptr[n] != nnz) return PERM_EINVAL;
    Mat A;
    A.n = n;
    A.a.assign(size_t(n) * n, 0.0);
    for (int j = 0; j < n; ++j) {
        if (col_ptr[j + 1] < col_ptr[j]) return PERM_EINVAL;
        for (int32_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) {
            if (row_idx[p] < 0 || row_idx[p] >= n) return PERM_EINVAL;
            if (p > col_ptr[j] && row_idx[p] <= row_idx[p - 1]) return PERM_EINVAL;
            A.at(row_idx[p], j) = vals[p];
        }
    }
    perm_decomp *D = new (std::nothrow) perm_decomp;
    if (!D) return PERM_EINVAL;
    if ((flags & PERM_DECOMP_DM) && !dm_prune(A, D->removed)) {
        D->zero = 1;  // no perfect matching: perm = 0, no leaves
        *out = D;
        return PERM_OK;
    }
    if (flags & PERM_DECOMP_FM) {
        Decomposer dec;
        dec.min_leaf = std::max(min_leaf, 0);
        dec.fold = (flags & PERM_DECOMP_FOLD) != 0;
        dec.rec(A, 1.0, 0);
        if (dec.overflow) {
            delete D;
            return PERM_ERANGE;
        }
        D->leaves = std::move(dec.leaves);
        D->folded[0] = dec.folded.hi + dec.folded.lo;
        D->folded[1] = dec.folded.lo - (D->folded[0] - dec.folded.hi);
    } else {
        D->leaves.push_back(Leaf{1.0, A});
    }
    *out = D;
    return PERM_OK;
}

int perm_decomp_info(const perm_decomp *d, int *count, int *max_order, int64_t *total_elements,
                     int64_t *removed)
{
    if (!d) return PERM_EINVAL;
    int64_t tot = 0;
    int mx = 0;
    for (const Leaf &L : d->leaves) {
        tot += int64_t(L.m.n) * L.m.n;
        mx = std::max(mx, L.m.n);
    }
    if (count) *count = int(d->leaves.size());
    if (max_order) *max_order = mx;
    if (total_elements) *total_elements = tot;
    if (removed) *removed = d->removed;
    return PERM_OK;
}

int perm_decomp_leaf(const perm_decomp *d, int idx, int *k, double *weight, double *data)
{
    if (!d || idx < 0 || idx >= int(d->leaves.size())) return PERM_EINVAL;
    const Leaf &L = d->leaves[idx];
    if (k) *k = L.m.n;
    if (weight) *weight = L.weight;
    if (data && !L.m.a.empty()) std::memcpy(data, L.m.a.data(), L.m.a.size() * sizeof(double));
    return PERM_OK;
}

int perm_decomp_leaves(const perm_decomp *d, int32_t *k, double *weight, int64_t *offset,
                       double *data)
{
    if (!d) return PERM_EINVAL;
    int64_t off = 0;
    for (size_t i = 0; i < d->leaves.size(); ++i) {
        const Leaf &L = d->leaves[i];
        if (k) k[i] = L.m.n;
        if (weight) weight[i] = L.weight;
        if (offset) offset[i] = off;
        if (data && !L.m.a.empty())
            std::memcpy(data + off, L.m.a.data(), L.m.a.size() * sizeof(double));
        off += int64_t(L.m.n) * L.m.n;
    }
    return PERM_OK;
}

int perm_decomp_folded(const perm_decomp *d, double out[2])
{
    if (!d || !out) return PERM_EINVAL;
    out[0] = d->folded[0];
    out[1] = d->folded[1];
    return PERM_OK;
}

void perm_decomp_destroy(perm_decomp *d) { delete d; }

}  // extern "C"
