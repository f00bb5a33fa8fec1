// Matrix-specific sparse sweep (the paper's per-matrix code generation,
// Section 3.2, applied to the sparse update of Algorithm 2): the host writes
// a HIP kernel in which the update of every column is a fixed list of
// `x_r += a_rj` on named registers -- only the column's nonzeros, with
// compile-time row indices -- compiles it for gfx950 with hiprtc, and keeps
// the loaded module for the rest of the process, keyed by device and
// sparsity pattern (the values are read from the staged column-major copy,
// so matrices with the same pattern share one module).
//
// The generated kernel walks each lane's chunk in 16-step blocks exactly as
// the dense sweep does (one column chosen at run time per block, read whole
// from the staged copy; the other fifteen flips are compile-time columns
// 0..3 with signs fixed by the step within the block), re-seeds exactly
// every 2^r steps, accumulates block sums by two-sum and writes one
// double-double partial per block.  The exact binary variant below works the
// same way on y = 2x with residues modulo primes.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "perm.h"
#include "sweep_common.h"

namespace perm {
namespace {

constexpr int kGenUnroll = 4;  // 16-step blocks

// Device helpers of the generated source: double-double sums and the
// wave / block reductions, in the same fixed order as the library's own.
const char *kPrelude = R"(
typedef unsigned int u32;
typedef unsigned long long u64;
struct dd { double hi, lo; };
__device__ inline void two_sum(double a, double b, double &s, double &e)
{ s = a + b; double bb = s - a; e = (a - (s - bb)) + (b - bb); }
__device__ inline dd dd_add(dd a, dd b)
{
    double s, e; two_sum(a.hi, b.hi, s, e);
    double t, f; two_sum(a.lo, b.lo, t, f);
    e += t; double hi = s + e; double lo = e - (hi - s); lo += f;
    double hi2 = hi + lo; return dd{hi2, lo - (hi2 - hi)};
}
__device__ inline dd block_reduce_dd(dd v, dd *lds)
{
    for (int off = 32; off >= 1; off >>= 1) {
        dd o; o.hi = __shfl_xor(v.hi, off, 64); o.lo = __shfl_xor(v.lo, off, 64);
        v = dd_add(v, o);
    }
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    dd t = dd{0.0, 0.0};
    if (threadIdx.x == 0) { t = lds[0]; for (int w = 1; w < 4; ++w) t = dd_add(t, lds[w]); }
    return t;
}
__device__ inline u32 gray_low(u32 l, u32 kb, int c)
{ u32 g = l ^ (l >> 1) ^ (kb << (c - 1)); return g & ((1u << c) - 1u); }
)";

// Column j's update: op is "+=", "-=" or an FMA with the lane factor f.
std::string column_code(int n, const std::vector<std::vector<int>> &rows, int j, char op)
{
    std::ostringstream o;
    for (int r : rows[j]) {
        const int off = j * n + r;
        if (op == '+') o << "x" << r << " += a[" << off << "]; ";
        else if (op == '-') o << "x" << r << " -= a[" << off << "]; ";
        else o << "x" << r << " = __builtin_fma(f, a[" << off << "], x" << r << "); ";
    }
    return o.str();
}


// Update of every row by a run-time column `col` (wave-uniform pointer into
// the staged column-major copy): straight-line code, so no register copies
// are needed where control flow merges.  op: '+' adds, 'f' adds f * col.
std::string dense_column_code(int n, const char *var, char op)
{
    std::ostringstream o;
    for (int i = 0; i < n; ++i) {
        if (op == '+') o << var << i << " += col[" << i << "]; ";
        else o << var << i << " = __builtin_fma(f, col[" << i << "], " << var << i << "); ";
    }
    return o.str();
}

// Product of x0..x{n-1} in four interleaved chains (independent latency).
std::string product_code(int n)
{
    std::ostringstream o;
    o << "(";
    for (int ch = 0; ch < 4; ++ch) {
        if (ch == 2) o << ") * (";
        else if (ch) o << " * ";
        o << "(";
        bool first = true;
        for (int i = ch; i < n; i += 4) {
            o << (first ? "" : " * ") << "x" << i;
            first = false;
        }
        if (first) o << "1.0";
        o << ")";
    }
    o << ")";
    return o.str();
}

std::string kernel_source(int n, const std::vector<std::vector<int>> &rows)
{
    std::ostringstream o;
    o << kPrelude;
    o << "extern \"C\" __global__ __launch_bounds__(256) void perm_sparse_gen(\n"
         "    const double *__restrict__ a, const double *__restrict__ an, const double *__restrict__ xs,\n"
         "    dd *__restrict__ partials, int c, int r, u32 l_begin, u32 l_end, int accumulate)\n{\n"
         "    __shared__ dd red[4];\n"
         "    const u32 lane = threadIdx.x & 63u;\n"
         "    const u64 wave = u64(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);\n"
         "    const u64 K = (wave & 1u) | (u64(lane) << 1) | ((wave >> 1) << 7);\n"
         "    const u32 kb = u32(wave & 1u);\n"
         "    const u64 g0 = K << c;\n"
         "    const u64 hbits = (g0 ^ (g0 >> 1)) >> c;\n"
         "    const u32 rmask = (1u << r) - 1u;\n";
    o << "    double";
    for (int i = 0; i < n; ++i) o << (i ? ", " : " ") << "x" << i;
    o << ";\n    double s = 0.0, e = 0.0;\n";
    o << "    for (u32 l = l_begin; l < l_end; l += 16u) {\n"
         "        if ((l & rmask) == 0) {\n";
    for (int i = 0; i < n; ++i) o << "            x" << i << " = xs[" << i << "];\n";
    // re-seed and the block's first (run-time) flip read whole staged
    // columns; only the compile-time flips below use the nonzero lists
    o << "            for (int j = c; j < " << n - 1 << "; ++j) {\n"
         "                const double f = ((hbits >> (j - c)) & 1u) ? 1.0 : 0.0;\n"
         "                const double *col = a + j * " << n << ";\n                "
      << dense_column_code(n, "x", 'f')
      << "\n            }\n"
         "            u32 low = gray_low(l, kb, c);\n"
         "            while (low) {\n"
         "                const int j = __builtin_ctz(low);\n"
         "                low &= low - 1u;\n"
         "                const double *col = a + j * " << n << ";\n                "
      << dense_column_code(n, "x", '+')
      << "\n            }\n"
         "        } else {\n"
         "            const int j = __builtin_ctz(l);\n"
         "            const double *col = (((gray_low(l, kb, c) >> j) & 1u) ? a : an) + j * " << n << ";\n"
         "            "
      << dense_column_code(n, "x", '+') << "\n        }\n";
    const std::string prod = product_code(n);
    o << "        double t0 = " << prod << ";\n";
    const int B = 1 << kGenUnroll;
    for (int m = 1; m < B; ++m) {
        const int j = __builtin_ctz(unsigned(m));
        if (j + 1 < kGenUnroll) {
            const bool neg = (m >> (j + 1)) & 1;
            o << "        " << column_code(n, rows, j, neg ? '-' : '+') << "\n";
        } else {  // sign from bit U of l
            o << "        if ((l >> " << kGenUnroll << ") & 1u) { " << column_code(n, rows, j, '-')
              << "} else { " << column_code(n, rows, j, '+') << "}\n";
        }
        o << "        double t" << m << " = " << prod << ";\n";
    }
    // signed block sum: (-1)^m, pairwise then a tree
    o << "        const double v = ";
    o << "(((t0 - t1) + (t2 - t3)) + ((t4 - t5) + (t6 - t7))) + "
         "(((t8 - t9) + (t10 - t11)) + ((t12 - t13) + (t14 - t15)));\n";
    o << "        double tt, er; two_sum(s, v, tt, er); s = tt; e += er;\n"
         "    }\n"
         "    const dd t = block_reduce_dd(dd{s, e}, red);\n"
         "    if (threadIdx.x == 0) partials[blockIdx.x] = accumulate ? dd_add(partials[blockIdx.x], t) : t;\n"
         "}\n";
    return o.str();
}

// ---- exact binary sweep (y = 2x, residues modulo primes just above 2^50) --

// Rows per group: |y_i| <= n <= 2^bits, so a group product is at most 2^50,
// below every prime (an exact integer and already a residue).
int binary_group_rows(int n)
{
    const int bits = n <= 2 ? 1 : n <= 4 ? 2 : n <= 8 ? 3 : n <= 16 ? 4 : n <= 32 ? 5 : 6;
    return 50 / bits;
}

// Same arithmetic as the staged binary kernel: signed residues in doubles,
// a * b mod p by an error-free product and a rounded quotient (exact for
// |a|, |b| <= p, p in (2^50, 2^50 + 2^40)); contraction off so that exactly
// these operations are emitted.
const char *kBinaryPrelude = R"(
typedef unsigned int u32;
typedef unsigned long long u64;
struct BinaryPrimes { double p[6]; double pinv[6]; };
__device__ inline double mulmod50(double a, double b, double p, double pinv)
{
#pragma clang fp contract(off)
    const double h = a * b;
    const double l = __builtin_fma(a, b, -h);
    const double q = __builtin_rint(h * pinv);
    const double qh = q * p;
    const double ql = __builtin_fma(q, p, -qh);
    return (h - qh) + (l - ql);
}
__device__ inline double addmod50(double acc, double t, double p, double pinv)
{
#pragma clang fp contract(off)
    const double s = acc + t;
    return __builtin_fma(-__builtin_rint(s * pinv), p, s);
}
__device__ inline u64 residue_u64(double v, double p) { return u64(v < 0.0 ? v + p : v); }
__device__ inline u64 addmod(u64 a, u64 b, u64 p) { const u64 s = a + b; return s >= p ? s - p : s; }
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ inline u32 gray_low(u32 l, u32 kb, int c)
{ u32 g = l ^ (l >> 1) ^ (kb << (c - 1)); return g & ((1u << c) - 1u); }
)";

// Column j's update on y: +2 / -2 on its rows, or + f (a lane's 0 / 2).
std::string ycolumn_code(const std::vector<std::vector<int>> &rows, int j, char op)
{
    std::ostringstream o;
    for (int r : rows[j]) {
        if (op == '+') o << "y" << r << " += 2.0; ";
        else if (op == '-') o << "y" << r << " -= 2.0; ";
        else o << "y" << r << " += f; ";
    }
    return o.str();
}


// Group products: cold rows [0, n_cold) and hot rows [n_cold, n) are grouped
// separately (G rows per group), so the cold groups stay constant inside a
// 16-step block.  Returns the expressions; *m_cold = number of cold groups.
std::vector<std::string> group_exprs(int n, int n_cold, int *m_cold)
{
    const int G = binary_group_rows(n);
    std::vector<std::string> g;
    // a balanced product tree (short dependency chains; any order is exact)
    std::function<std::string(int, int)> tree = [&](int a, int b) -> std::string {
        if (b - a == 1) return "y" + std::to_string(a);
        const int mid = a + (b - a) / 2;
        return "(" + tree(a, mid) + " * " + tree(mid, b) + ")";
    };
    auto add_range = [&](int a, int b) {
        for (int s = a; s < b; s += G) g.push_back(tree(s, std::min(b, s + G)));
    };
    add_range(0, n_cold);
    *m_cold = int(g.size());
    add_range(n_cold, n);
    return g;
}

std::string binary_kernel_source(int n, int n_cold, const std::vector<std::vector<int>> &rows)
{
    int m_cold = 0;
    const std::vector<std::string> grp = group_exprs(n, n_cold, &m_cold);
    const int M = int(grp.size());
    std::ostringstream o;
    o << kBinaryPrelude;
    o << "#define M " << M << "\n#define QCAP 128\n";
    o << "extern \"C\" __global__ __launch_bounds__(256) void perm_binary_gen(\n"
         "    const double *__restrict__ yc, const double *__restrict__ yn, const double *__restrict__ ys,\n"
         "    u64 *__restrict__ partials, int c, int nprimes, const BinaryPrimes P)\n{\n"
         "    __shared__ double queue[4][M * QCAP];\n"
         "    __shared__ u64 red[4][6];\n"
         "    const u32 lane = threadIdx.x & 63u;\n"
         "    const u32 wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);\n"
         "    const u64 wave = u64(blockIdx.x) * 4 + wib;\n"
         "    const u64 K = (wave & 1u) | (u64(lane) << 1) | ((wave >> 1) << 7);\n"
         "    const u32 kb = u32(wave & 1u);\n"
         "    const u64 g0 = K << c;\n"
         "    const u64 hbits = (g0 ^ (g0 >> 1)) >> c;\n"
         "    const u32 C = 1u << c;\n"
         "    double *q = queue[wib];\n";
    o << "    double";
    for (int i = 0; i < n; ++i) o << (i ? ", " : " ") << "y" << i;
    o << ";\n";
    for (int i = 0; i < n; ++i) o << "    y" << i << " = ys[" << i << "];\n";
    // exact seed of the chunk start (integers: no drift, no re-seeding)
    o << "    for (int j = c; j < " << n - 1 << "; ++j) {\n"
         "        const double f = ((hbits >> (j - c)) & 1u) ? 1.0 : 0.0;\n"
         "        const double *col = yc + j * " << n << ";\n        "
      << dense_column_code(n, "y", 'f') << "\n    }\n"
      << "    {\n        u32 low = gray_low(0, kb, c);\n"
         "        while (low) {\n            const int j = __builtin_ctz(low);\n"
         "            low &= low - 1u;\n"
         "            const double *col = yc + j * " << n << ";\n            "
      << dense_column_code(n, "y", '+') << "\n        }\n    }\n";
    o << "    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};\n    u32 count = 0;\n";
    // drain one queue entry into the residues
    o << "    auto drain = [&](int slot) {\n        double g[M];\n"
         "#pragma unroll\n        for (int m = 0; m < M; ++m) g[m] = q[m * QCAP + slot];\n"
         "#pragma unroll\n        for (int k = 0; k < 6; ++k) {\n"
         "            if (k < nprimes) {\n"
         "                double t = g[0];\n"
         "#pragma unroll\n                for (int m = 1; m < M; ++m) t = mulmod50(t, g[m], P.p[k], P.pinv[k]);\n"
         "                acc[k] = addmod50(acc[k], t, P.p[k], P.pinv[k]);\n"
         "            }\n        }\n    };\n";
    // push the current term if it is nonzero
    o << "    auto push = [&](bool negative) {\n        double gp[M];\n";
    for (int m = 0; m < M; ++m) o << "        gp[" << m << "] = " << grp[m] << ";\n";
    // zero test by FP64 minima; every lane stores without a branch, lanes
    // with a zero term past the new entries (slot <= count + 63 < QCAP)
    o << "        double mn = __builtin_fabs(gp[0]);\n"
         "#pragma unroll\n        for (int m = 1; m < M; ++m) mn = __builtin_fmin(mn, __builtin_fabs(gp[m]));\n"
         "        const bool nz = mn != 0.0;\n"
         "        if (negative) gp[0] = -gp[0];\n"
         "        const u64 ballot = __ballot(nz);\n"
         "        if (ballot == 0) return;\n"
         "        const u32 before = __builtin_amdgcn_mbcnt_hi(u32(ballot >> 32), __builtin_amdgcn_mbcnt_lo(u32(ballot), 0u));\n"
         "        const u32 pc = u32(__builtin_popcountll(ballot));\n"
         "        const u32 slot = nz ? count + before : count + pc + (lane - before);\n"
         "#pragma unroll\n        for (int m = 0; m < M; ++m) q[m * QCAP + slot] = gp[m];\n"
         "        count += pc;\n"
         "        if (count >= 64) {\n            wave_sync();\n"
         "            drain(int(count - 64 + lane));\n            count -= 64;\n            wave_sync();\n"
         "        }\n    };\n";
    // the walk in 16-step blocks
    o << "    for (u32 l = 0; l < C; l += 16u) {\n"
         "        if (l != 0) {\n            const int j = __builtin_ctz(l);\n"
         "            const double *col = (((gray_low(l, kb, c) >> j) & 1u) ? yc : yn) + j * " << n << ";\n"
         "            " << dense_column_code(n, "y", '+') << "\n        }\n";
    if (m_cold > 0) {
        // cold rows do not change inside the block: if one is zero for every
        // lane, all 16 terms are zero and only the flip of column 3 remains
        // (bitwise &: no short-circuit branches)
        o << "        bool cold_nz = true;\n";
        for (int m = 0; m < m_cold; ++m) o << "        cold_nz = cold_nz & (" << grp[m] << " != 0.0);\n";
        o << "        if (__ballot(cold_nz) == 0) {\n"
             "            if ((l >> 4) & 1u) { " << ycolumn_code(rows, 3, '-') << "} else { "
          << ycolumn_code(rows, 3, '+') << "}\n            continue;\n        }\n";
    }
    // the 16 steps of the block, unrolled: each flip is its list of +-2
    // updates; the cold rows are not written inside the block, so their
    // group products are common to the sixteen pushes
    for (int m = 0; m < 16; ++m) {
        if (m > 0) {
            const int j = __builtin_ctz(unsigned(m));
            if (j + 1 < kGenUnroll) {
                const bool neg = (m >> (j + 1)) & 1;
                o << "        " << ycolumn_code(rows, j, neg ? '-' : '+') << "\n";
            } else {
                o << "        if ((l >> 4) & 1u) { " << ycolumn_code(rows, j, '-') << "} else { "
                  << ycolumn_code(rows, j, '+') << "}\n";
            }
        }
        o << "        push(" << ((m & 1) ? "true" : "false") << ");\n";
    }
    o << "    }\n";
    // what is left in the queue, then the modular reductions
    o << "    wave_sync();\n    if (lane < count) drain(int(lane));\n"
         "#pragma unroll\n    for (int k = 0; k < 6; ++k) {\n"
         "        if (k < nprimes) {\n            const u64 p = u64(P.p[k]);\n"
         "            u64 v = residue_u64(acc[k], P.p[k]);\n"
         "#pragma unroll\n            for (int off = 32; off >= 1; off >>= 1) v = addmod(v, __shfl_xor(v, off, 64), p);\n"
         "            if (lane == 0) red[wib][k] = v;\n        }\n    }\n"
         "    __syncthreads();\n"
         "    if (threadIdx.x < u32(nprimes)) {\n        const int k = int(threadIdx.x);\n"
         "        const u64 p = u64(P.p[k]);\n        u64 v = 0;\n"
         "        for (int w = 0; w < 4; ++w) v = addmod(v, red[w][k], p);\n"
         "        partials[u64(blockIdx.x) * nprimes + k] = v;\n    }\n}\n";
    return o.str();
}

struct GenModule {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
};

std::mutex g_mu;
std::unordered_map<std::string, GenModule> g_cache;

std::string cache_key(int kind, int dev, int n, int extra, const std::vector<std::vector<int>> &rows)
{
    std::string k;
    auto put = [&](int v) { k.append(reinterpret_cast<const char *>(&v), sizeof(v)); };
    put(kind);
    put(dev);
    put(n);
    put(extra);
    for (const auto &c : rows) {
        put(int(c.size()));
        for (int r : c) put(r);
    }
    return k;
}

int compile_module(const std::string &src, const char *name, GenModule &out)
{
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "perm_generated.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        return PERM_ECOMPILE;
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult cr = hiprtcCompileProgram(prog, 6, opts);
    size_t sz = 0;
    std::vector<char> code;
    if (cr == HIPRTC_SUCCESS && hiprtcGetCodeSize(prog, &sz) == HIPRTC_SUCCESS && sz > 0) {
        code.resize(sz);
        if (hiprtcGetCode(prog, code.data()) != HIPRTC_SUCCESS) code.clear();
    }
    hiprtcDestroyProgram(&prog);
    if (code.empty()) return PERM_ECOMPILE;
    if (hipModuleLoadData(&out.mod, code.data()) != hipSuccess) return PERM_EHIP;
    if (hipModuleGetFunction(&out.fn, out.mod, name) != hipSuccess) return PERM_EHIP;
    return PERM_OK;
}

// The module for (kind, device, pattern), compiled on first use.
int get_module(int kind, int n, int extra, const std::vector<std::vector<int>> &rows,
               const std::string &src_if_new, const char *name, GenModule &m)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PERM_EHIP;
    std::lock_guard<std::mutex> lock(g_mu);
    const std::string key = cache_key(kind, dev, n, extra, rows);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        m = it->second;
        return PERM_OK;
    }
    const int rc = compile_module(src_if_new, name, m);
    if (rc != PERM_OK) return rc;
    g_cache.emplace(key, m);
    return PERM_OK;
}

}  // namespace

std::string sparse_gen_source(int n, const std::vector<std::vector<int>> &rows)
{
    return kernel_source(n, rows);
}

int launch_sparse_gen(int n, const std::vector<std::vector<int>> &rows, const double *dense_dev,
                      double *out, char *ws, hipStream_t stream)
{
    if (n < kSparseGenMinN || n > PERM_MAX_N) return PERM_EUNSUPPORTED;
    GenModule m;
    {
        const int rc = get_module(0, n, 0, rows, kernel_source(n, rows), "perm_sparse_gen", m);
        if (rc != PERM_OK) return rc;
    }
    const SweepPlan p = plan_sweep(n, 0);
    const DenseWs L = dense_ws_layout(n, 1, dense_ws_blocks(n));
    double *acol = reinterpret_cast<double *>(ws + L.acol);
    double *aneg = reinterpret_cast<double *>(ws + L.aneg);
    double *x0 = reinterpret_cast<double *>(ws + L.x0);
    dd *partials = reinterpret_cast<dd *>(ws + L.partials);
    hipLaunchKernelGGL(prep_dense_f64, dim3(1), dim3(kBlock), 0, stream, n, dense_dev, int64_t(n),
                       acol, aneg, x0);
    // full-grid launches over ranges of every lane's chunk (at most 2^40
    // subset-steps each), every range starting on a re-seed boundary
    const int c = p.log2_chunk;
    const int r = std::max(p.log2_reseed, kGenUnroll);
    const int64_t C = int64_t(1) << c;
    int64_t span = std::max<int64_t>((int64_t(1) << 40) / p.lanes, int64_t(1) << r);
    int64_t pow2 = 1;
    while (pow2 * 2 <= span) pow2 *= 2;
    span = std::min(pow2, C);
    for (int64_t l0 = 0; l0 < C; l0 += span) {
        const double *a_arg = acol;
        const double *an_arg = aneg;
        const double *x_arg = x0;
        dd *p_arg = partials;
        int c_arg = c, r_arg = r;
        uint32_t lb = uint32_t(l0), le = uint32_t(l0 + span);
        int acc = l0 > 0;
        void *args[] = {&a_arg, &an_arg, &x_arg, &p_arg, &c_arg, &r_arg, &lb, &le, &acc};
        if (hipModuleLaunchKernel(m.fn, unsigned(p.blocks), 1, 1, kBlock, 1, 1, 0, stream, args,
                                  nullptr) != hipSuccess)
            return PERM_EHIP;
    }
    const double scale = (n & 1) ? 2.0 : -2.0;  // 2 (-1)^(n-1)
    hipLaunchKernelGGL(finalize_partials, dim3(1), dim3(kBlock), 0, stream, partials, p.blocks, 1,
                       scale, out);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm

namespace perm {

std::string binary_gen_source(int n, int n_cold, const std::vector<std::vector<int>> &rows)
{
    return binary_kernel_source(n, n_cold, rows);
}

int launch_binary_gen(int n, int n_cold, const std::vector<std::vector<int>> &rows,
                      const double *dense01_dev, int nprimes, uint64_t *residues_dev, char *ws,
                      hipStream_t stream)
{
    if (n < kSparseGenMinN || n > PERM_MAX_N) return PERM_EUNSUPPORTED;
    GenModule m;
    {
        const int rc = get_module(1, n, n_cold, rows, binary_kernel_source(n, n_cold, rows),
                                  "perm_binary_gen", m);
        if (rc != PERM_OK) return rc;
    }
    const SweepPlan p = plan_sweep_fine(n);
    const BinaryWs L = binary_ws_layout(n, p.blocks);
    double *ycol = reinterpret_cast<double *>(ws + L.ycol);
    double *yneg = reinterpret_cast<double *>(ws + L.yneg);
    double *y0 = reinterpret_cast<double *>(ws + L.y0);
    uint64_t *partials = reinterpret_cast<uint64_t *>(ws + L.partials);
    hipLaunchKernelGGL(prep_binary, dim3(1), dim3(kBlock), 0, stream, n, dense01_dev, ycol, yneg,
                       y0);
    {
        const double *yc_arg = ycol;
        const double *yn_arg = yneg;
        const double *y_arg = y0;
        uint64_t *p_arg = partials;
        int c_arg = p.log2_chunk, np_arg = nprimes;
        BinaryPrimes pr_arg = binary_primes();
        void *args[] = {&yc_arg, &yn_arg, &y_arg, &p_arg, &c_arg, &np_arg, &pr_arg};
        if (hipModuleLaunchKernel(m.fn, unsigned(p.blocks), 1, 1, kBlock, 1, 1, 0, stream, args,
                                  nullptr) != hipSuccess)
            return PERM_EHIP;
    }
    hipLaunchKernelGGL(finalize_residues, dim3(1), dim3(kBlock), 0, stream, partials, p.blocks,
                       nprimes, binary_primes(), residues_dev);
    return hipGetLastError() == hipSuccess ? PERM_OK : PERM_EHIP;
}

}  // namespace perm
