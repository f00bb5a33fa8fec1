// Host side of the batched entry points: the plan (work list, workspace
// layout, launch shapes), its autotuner, the upload of the plan into the
// caller's workspace and the hipGraph that replays one batched launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <vector>

#include "batched_internal.h"
#include "perm.h"

using namespace perm;

namespace {

// Tuning knobs.  log2_chunk is the number of Gray steps per lane (log2) used
// for large matrices; grid[g] is the number of persistent two-wave blocks of
// group g's kernel, which sets how many waves each SIMD runs (the kernels of
// orders 1..24 fit two waves per SIMD, 1024 blocks on 256 CUs; the kernel of
// orders 25..32 one, 512 blocks).
struct BatchTuning {
    int log2_chunk = 10;
    int64_t grid[kBatchGroups] = {2048, 1024, 512};
};

// Candidates the autotuner times, one knob at a time (coordinate descent
// from the defaults): steps per lane, then each group's grid.
const int kTuneChunks[] = {8, 10, 12};
const int64_t kTuneGrid[kBatchGroups][3] = {{512, 1024, 2048}, {512, 768, 1024}, {256, 384, 512}};

// Tunings found by perm_batched_autotune, kept for the process and keyed by
// (device, gradient or not, histogram of the orders): a later plan with the
// same key starts from the tuned values and its autotune call returns at once.
struct TuneKey {
    int device = 0;
    int want_grad = 0;
    int real = 0;
    std::array<int32_t, kBatchMaxK + 1> hist{};
    bool operator<(const TuneKey &o) const
    {
        if (device != o.device) return device < o.device;
        if (want_grad != o.want_grad) return want_grad < o.want_grad;
        if (real != o.real) return real < o.real;
        return hist < o.hist;
    }
};
struct TuneEntry {
    BatchTuning tune;
    double ms = 0.0;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune_cache;

}  // namespace

struct perm_plan {
    int count = 0;
    int want_grad = 0;
    int real = 0;  // 1: real matrices (doubles), 0: complex (re, im) pairs
    std::vector<int32_t> k;
    std::vector<int64_t> off;
    BatchTuning tune;
    // derived from (k, tune)
    std::vector<BatchMatDev> mats;
    std::vector<BatchItemDev> items[kBatchGroups];
    int64_t n_items_total = 0;
    int64_t stage_doubles = 0;
    int64_t g_dd = 0;
    // workspace layout (bytes)
    size_t o_mats = 0, o_items[kBatchGroups] = {0, 0, 0}, o_counters = 0, o_stage = 0, o_perm = 0,
           o_grad = 0, total = 0;
    size_t ws_max = 0;  // over every tuning candidate
    // caches
    const void *uploaded_ws = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *g_data = nullptr, *g_out = nullptr, *g_grad = nullptr, *g_ws = nullptr;
    hipStream_t side[kBatchGroups] = {nullptr, nullptr, nullptr};
    hipStream_t capture = nullptr;
    hipEvent_t fork = nullptr, join[kBatchGroups] = {nullptr, nullptr, nullptr};
    // recorded after every graph launch: the graph's work is finished once
    // it completes (waited for before the graph or the streams are destroyed)
    hipEvent_t launched = nullptr;
    int tuned_from_cache = 0;  // 1: the tuning came from the process-wide cache
};

namespace {

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

// Per-matrix walk decomposition: at most 2^log2_chunk steps per lane, whole
// 64-lane waves where the matrix has enough steps (2^(k-1) >= 128), and
// r <= c - 1 so the lane-dependent flip at 2^(c-1) is an exact re-seed.
void derive(perm_plan &P)
{
    const int ct = P.tune.log2_chunk;
    const int64_t W = P.real ? 1 : 2;  // doubles per element
    P.mats.assign(P.count, BatchMatDev{});
    for (int g = 0; g < kBatchGroups; ++g) P.items[g].clear();
    int64_t item0 = 0, stage = 0, gdd = 0;
    for (int m = 0; m < P.count; ++m) {
        BatchMatDev &M = P.mats[m];
        const int k = P.k[m];
        M.k = k;
        M.data_off = P.off[m];
        if (k == 1) {
            M.c = 0;
            M.r = 0;
            M.waves = 1;
        } else {
            const int total = k - 1;
            const int c = std::max(1, std::min(ct, total - 6));
            M.c = c;
            M.r = std::min(9, c - 1);
            const int64_t lanes = int64_t(1) << (total - c);
            M.waves = int32_t(std::max<int64_t>(1, lanes / kWave));
        }
        M.stage = stage;
        stage += W * int64_t(k) * batch_rows(k) + W * int64_t(batch_rows(k));
        M.item0 = item0;
        item0 += M.waves;
        M.gbase = gdd;
        if (P.want_grad) gdd += int64_t(M.waves) * W * k * k;
    }
    // Work list per group: largest order first (longest items first), then
    // matrix, then wave -- a fixed order, so the plan is deterministic.
    std::vector<int> order(P.count);
    for (int m = 0; m < P.count; ++m) order[m] = m;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P.k[a] > P.k[b]; });
    for (int m : order) {
        const int g = batch_group(P.k[m]);
        for (int w = 0; w < P.mats[m].waves; ++w) P.items[g].push_back(BatchItemDev{m, w});
    }
    P.n_items_total = item0;
    P.stage_doubles = stage;
    P.g_dd = gdd;
    size_t o = 0;
    P.o_mats = o;
    o += a256(sizeof(BatchMatDev) * size_t(P.count));
    for (int g = 0; g < kBatchGroups; ++g) {
        P.o_items[g] = o;
        o += a256(sizeof(BatchItemDev) * std::max<size_t>(1, P.items[g].size()));
    }
    P.o_counters = o;
    o += a256(sizeof(uint32_t) * kBatchGroups);
    P.o_stage = o;
    o += a256(sizeof(double) * size_t(stage));
    P.o_perm = o;
    o += a256(sizeof(dd) * 2 * size_t(item0));
    P.o_grad = o;
    o += a256(sizeof(dd) * size_t(std::max<int64_t>(gdd, 1)));
    P.total = o;
}

// Waits for the last graph launch of the plan (if any) to finish.
void wait_graph(perm_plan &P)
{
    if (P.exec && P.launched) hipEventSynchronize(P.launched);
}

void drop_graph(perm_plan &P)
{
    wait_graph(P);
    if (P.exec) hipGraphExecDestroy(P.exec);
    P.exec = nullptr;
    P.g_data = P.g_out = P.g_grad = P.g_ws = nullptr;
}

int upload(perm_plan &P, char *ws, hipStream_t st)
{
    if (P.uploaded_ws == ws) return PERM_OK;
    if (hipMemcpyAsync(ws + P.o_mats, P.mats.data(), sizeof(BatchMatDev) * P.mats.size(),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return PERM_EHIP;
    for (int g = 0; g < kBatchGroups; ++g)
        if (!P.items[g].empty() &&
            hipMemcpyAsync(ws + P.o_items[g], P.items[g].data(),
                           sizeof(BatchItemDev) * P.items[g].size(), hipMemcpyHostToDevice,
                           st) != hipSuccess)
            return PERM_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return PERM_EHIP;
    P.uploaded_ws = ws;
    return PERM_OK;
}

TuneKey tune_key(const perm_plan &P)
{
    TuneKey key;
    hipGetDevice(&key.device);
    key.want_grad = P.want_grad;
    key.real = P.real;
    for (int k : P.k) key.hist[k]++;
    return key;
}

// The plan's side streams and events (created once, reused by every graph
// capture and every tuning launch).
int ensure_streams(perm_plan &P)
{
    if (!P.capture && hipStreamCreateWithFlags(&P.capture, hipStreamNonBlocking) != hipSuccess)
        return PERM_EHIP;
    if (!P.fork && hipEventCreateWithFlags(&P.fork, hipEventDisableTiming) != hipSuccess)
        return PERM_EHIP;
    if (!P.launched && hipEventCreateWithFlags(&P.launched, hipEventDisableTiming) != hipSuccess)
        return PERM_EHIP;
    for (int g = 0; g < kBatchGroups; ++g) {
        if (!P.side[g] && hipStreamCreateWithFlags(&P.side[g], hipStreamNonBlocking) != hipSuccess)
            return PERM_EHIP;
        if (!P.join[g] && hipEventCreateWithFlags(&P.join[g], hipEventDisableTiming) != hipSuccess)
            return PERM_EHIP;
    }
    return PERM_OK;
}

BatchLaunch make_launch(const perm_plan &P, char *ws, const double *data, double *out,
                        double *grad)
{
    BatchLaunch L;
    L.count = P.count;
    L.mats = reinterpret_cast<const BatchMatDev *>(ws + P.o_mats);
    for (int g = 0; g < kBatchGroups; ++g) {
        L.items[g] = reinterpret_cast<const BatchItemDev *>(ws + P.o_items[g]);
        L.n_items[g] = int64_t(P.items[g].size());
        L.grid[g] = std::min<int64_t>(P.tune.grid[g], std::max<int64_t>(1, L.n_items[g]));
    }
    L.counters = reinterpret_cast<uint32_t *>(ws + P.o_counters);
    L.stage = reinterpret_cast<double *>(ws + P.o_stage);
    L.perm_parts = reinterpret_cast<dd *>(ws + P.o_perm);
    L.g_parts = reinterpret_cast<dd *>(ws + P.o_grad);
    L.data = data;
    L.out = out;
    L.grad = grad;
    L.want_grad = P.want_grad;
    L.real = P.real;
    return L;
}

int plan_create(int count, const int32_t *k, const int64_t *offset, int want_grad, int real,
                perm_plan **plan)
{
    if (!plan) return PERM_EINVAL;
    *plan = nullptr;
    if (count < 1 || !k || !offset) return PERM_EINVAL;
    for (int m = 0; m < count; ++m)
        if (k[m] < 1 || k[m] > kBatchMaxK || offset[m] < 0) return PERM_EINVAL;
    perm_plan *P = new (std::nothrow) perm_plan;
    if (!P) return PERM_EINVAL;
    P->count = count;
    P->want_grad = want_grad ? 1 : 0;
    P->real = real;
    P->k.assign(k, k + count);
    P->off.assign(offset, offset + count);
    // the workspace must hold the largest layout over every tuning candidate:
    // the shortest chunks give every matrix the most items, so that one
    P->tune.log2_chunk = *std::min_element(std::begin(kTuneChunks), std::end(kTuneChunks));
    derive(*P);
    const size_t mx = P->total;
    P->tune = BatchTuning{};
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(tune_key(*P));
        if (it != g_tune_cache.end()) {
            P->tune = it->second.tune;
            P->tuned_from_cache = 1;
        }
    }
    derive(*P);
    P->ws_max = std::max(mx, P->total);
    *plan = P;
    return PERM_OK;
}

int run_batched(perm_plan *plan, const double *data, double *out, double *grad, int use_graph,
                void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !data || !out) return PERM_EINVAL;
    if (plan->want_grad && !grad) return PERM_EINVAL;
    if (!ws || ws_bytes < plan->ws_max) return PERM_EWORKSPACE;
    perm_plan &P = *plan;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    int rc = upload(P, base, st);
    if (rc != PERM_OK) return rc;
    const BatchLaunch L = make_launch(P, base, data, out, grad);
    if (!use_graph) return launch_batched(L, st);

    if (!P.exec || P.g_data != data || P.g_out != out || P.g_grad != grad || P.g_ws != ws) {
        drop_graph(P);
        if ((rc = ensure_streams(P)) != PERM_OK) return rc;
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(P.capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return PERM_EHIP;
        rc = launch_batched_forked(L, P.capture, P.side, P.fork, P.join);
        const hipError_t e = hipStreamEndCapture(P.capture, &graph);
        if (rc != PERM_OK || e != hipSuccess || !graph) {
            if (graph) hipGraphDestroy(graph);
            return PERM_EHIP;
        }
        const hipError_t ie = hipGraphInstantiate(&P.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            P.exec = nullptr;
            return PERM_EHIP;
        }
        P.g_data = data;
        P.g_out = out;
        P.g_grad = grad;
        P.g_ws = ws;
    }
    if (hipGraphLaunch(P.exec, st) != hipSuccess) return PERM_EHIP;
    return hipEventRecord(P.launched, st) == hipSuccess ? PERM_OK : PERM_EHIP;
}

int autotune(perm_plan *plan, const double *data, double *out, double *grad, void *ws,
             size_t ws_bytes, void *stream, double *best_ms)
{
    if (!plan || !data || !out) return PERM_EINVAL;
    if (plan->want_grad && !grad) return PERM_EINVAL;
    if (!ws || ws_bytes < plan->ws_max) return PERM_EWORKSPACE;
    perm_plan &P = *plan;
    const TuneKey key = tune_key(P);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            wait_graph(P);
            P.tune = it->second.tune;
            P.tuned_from_cache = 1;
            derive(P);
            P.uploaded_ws = nullptr;
            drop_graph(P);
            if (best_ms) *best_ms = it->second.ms;
            return PERM_OK;
        }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = ensure_streams(P);
    if (rc != PERM_OK) return rc;
    drop_graph(P);  // waits for the last graph launch before the workspace is reused
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PERM_EHIP;
    // Times one candidate exactly as it will run: captured into the plan's
    // graph by perm_batched (one untimed launch, which also uploads the
    // plan), then the average of two graph launches.
    auto time_it = [&](const BatchTuning &t, float &ms) -> int {
        drop_graph(P);  // waits for the previous candidate's last launch
        P.tune = t;
        derive(P);
        P.uploaded_ws = nullptr;
        int r = run_batched(plan, data, out, grad, 1, ws, ws_bytes, stream);
        if (r != PERM_OK) return r;
        if (hipEventRecord(e0, st) != hipSuccess) return PERM_EHIP;
        for (int rep = 0; rep < 2; ++rep)
            if ((r = run_batched(plan, data, out, grad, 1, ws, ws_bytes, stream)) != PERM_OK) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return PERM_EHIP;
        hipEventElapsedTime(&ms, e0, e1);
        ms *= 0.5f;
        return PERM_OK;
    };
    BatchTuning best = P.tune;
    float best_t = 1e30f;
    // the first candidate is timed twice and the second time kept: the first
    // batched launches of a process run while the clocks ramp up, which
    // otherwise makes the starting configuration look slow
    rc = time_it(best, best_t);
    if (rc == PERM_OK) rc = time_it(best, best_t);
    // one knob at a time: steps per lane, then the grid of each group that
    // has work (largest orders first)
    for (int knob = -1; knob < kBatchGroups && rc == PERM_OK; ++knob) {
        if (knob >= 0) {
            bool any = false;
            for (int k : P.k) any = any || batch_group(k) == knob;
            if (!any) continue;
        }
        const int ncand = knob < 0 ? int(std::size(kTuneChunks)) : 3;
        for (int c = 0; c < ncand && rc == PERM_OK; ++c) {
            BatchTuning t = best;
            if (knob < 0) t.log2_chunk = kTuneChunks[c];
            else t.grid[knob] = kTuneGrid[knob][c];
            if (knob < 0 ? t.log2_chunk == best.log2_chunk : t.grid[knob] == best.grid[knob])
                continue;
            float ms = 0.f;
            rc = time_it(t, ms);
            if (rc == PERM_OK && ms < best_t) {
                best_t = ms;
                best = t;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    drop_graph(P);  // the graph holds the last candidate; the next call captures the best
    P.tune = best;
    derive(P);
    P.uploaded_ws = nullptr;
    if (rc == PERM_OK) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = TuneEntry{best, double(best_t)};
        P.tuned_from_cache = 0;
    }
    if (best_ms) *best_ms = best_t;
    return rc;
}

}  // namespace

extern "C" {

int perm_batched_plan_create(int count, const int32_t *k, const int64_t *offset, int want_grad,
                             perm_plan **plan)
{
    return plan_create(count, k, offset, want_grad, 0, plan);
}

int perm_batched_plan_create_f64(int count, const int32_t *k, const int64_t *offset,
                                 int want_grad, perm_plan **plan)
{
    return plan_create(count, k, offset, want_grad, 1, plan);
}

void perm_plan_destroy(perm_plan *plan)
{
    if (!plan) return;
    // No plan-owned object is released while a graph launch that uses it is
    // still queued or running: drop_graph waits for the last launch first,
    // and the side streams (used only while capturing) are idle after it.
    drop_graph(*plan);
    if (plan->launched) hipEventDestroy(plan->launched);
    for (int g = 0; g < kBatchGroups; ++g) {
        if (plan->side[g]) hipStreamDestroy(plan->side[g]);
        if (plan->join[g]) hipEventDestroy(plan->join[g]);
    }
    if (plan->capture) hipStreamDestroy(plan->capture);
    if (plan->fork) hipEventDestroy(plan->fork);
    delete plan;
}

size_t perm_batched_workspace_bytes(const perm_plan *plan) { return plan ? plan->ws_max : 0; }

int perm_batched(perm_plan *plan, const perm_c128 *data, perm_c128 *out, perm_c128 *grad,
                 int use_graph, void *ws, size_t ws_bytes, void *stream)
{
    if (plan && plan->real) return PERM_EINVAL;
    return run_batched(plan, reinterpret_cast<const double *>(data),
                       reinterpret_cast<double *>(out), reinterpret_cast<double *>(grad),
                       use_graph, ws, ws_bytes, stream);
}

int perm_batched_f64(perm_plan *plan, const double *data, double *out, double *grad,
                     int use_graph, void *ws, size_t ws_bytes, void *stream)
{
    if (plan && !plan->real) return PERM_EINVAL;
    return run_batched(plan, data, out, grad, use_graph, ws, ws_bytes, stream);
}

int perm_batched_autotune(perm_plan *plan, const perm_c128 *data, perm_c128 *out,
                          perm_c128 *grad, void *ws, size_t ws_bytes, void *stream,
                          double *best_ms)
{
    if (plan && plan->real) return PERM_EINVAL;
    return autotune(plan, reinterpret_cast<const double *>(data), reinterpret_cast<double *>(out),
                    reinterpret_cast<double *>(grad), ws, ws_bytes, stream, best_ms);
}

int perm_batched_autotune_f64(perm_plan *plan, const double *data, double *out, double *grad,
                              void *ws, size_t ws_bytes, void *stream, double *best_ms)
{
    if (plan && !plan->real) return PERM_EINVAL;
    return autotune(plan, data, out, grad, ws, ws_bytes, stream, best_ms);
}

int perm_weighted_sum(int count, const double *weights, const perm_c128 *perms, perm_c128 *out,
                      void *stream)
{
    if (count < 1 || !weights || !perms || !out) return PERM_EINVAL;
    return launch_weighted_sum(count, weights, reinterpret_cast<const double *>(perms),
                               reinterpret_cast<double *>(out), false,
                               static_cast<hipStream_t>(stream));
}

int perm_weighted_sum_f64(int count, const double *weights, const double *perms, double *out,
                          void *stream)
{
    if (count < 1 || !weights || !perms || !out) return PERM_EINVAL;
    return launch_weighted_sum(count, weights, perms, out, true, static_cast<hipStream_t>(stream));
}

int perm_batched_plan_info(const perm_plan *plan, int64_t *n_items, int *log2_chunk,
                           int64_t *grid, int *tuned_from_cache)
{
    if (!plan) return PERM_EINVAL;
    if (n_items) *n_items = plan->n_items_total;
    if (log2_chunk) *log2_chunk = plan->tune.log2_chunk;
    if (grid)
        for (int g = 0; g < kBatchGroups; ++g) grid[g] = plan->tune.grid[g];
    if (tuned_from_cache) *tuned_from_cache = plan->tuned_from_cache;
    return PERM_OK;
}

}  // extern "C"
