"""Benchmark: Ryser subset-steps/s of the dense FP64 permanent on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the dense real 32 x 32 matrix with i.i.d. U[0,1) entries (seed
16578), resident in HBM before timing.  One step is one complete
perm_dense_f64 call -- staging kernel, the Gray-walk sweep over all 2^31
column subsets, and the fixed-order reduction -- so one step processes
2^31 subset-steps.  Prints one JSON line.

roofline: the sweep is bound by the FP64 vector ALU.  Algorithmic work per
subset-step is 2n + 2 flops (n additions, n multiplications, the sign and
the accumulation; the count the paper uses for its error estimate).  None of
it is multiply-add shaped, so one FP64 lane-operation per flop: the ceiling
is 256 CUs x 64 FP64 lanes/clock x 2.4 GHz = 39.32 Tflop/s (the published
78.6 TFLOP/s counts an FMA as two flops).  The duration is the average HIP
event time of one call on the launch stream, which includes the two tiny
kernels around the sweep (under 0.5 % of it).

cpu_baseline: the CPU oracle (long double, all host threads) timed on a
bounded sample of the same matrix's Gray walk, scaled to subset-steps/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 32
PEAK_ALU_TFLOPS = 256 * 64 * 2.4e9 / 1e12      # 39.32: one add or mul per lane per clock
PEAK_FMA_TFLOPS = 78.6                           # published FP64 vector peak (FMA = 2 flops)

# HBM bytes per sweep launch from rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a
# plain 1 GiB copy (profiles/sweep_dense_f64_n32_u01.md).  Valid only for the
# kernel source they were measured on; reported as null once it changes.
COUNTERS_SRC = os.path.join(ROOT, "paper_2502_16577_amd", "csrc", "sweep_f64.hip")
COUNTERS_SRC_SHA256 = "2e9356c7e13965c121678f44cb3f3c16b6568bb55b9148af0310e214dab47f79"
TRAFFIC_BYTES_PER_LAUNCH = 188 * 1024 * 2.000 + 32 * 1024 * 1.000


def traffic_bytes():
    import hashlib
    with open(COUNTERS_SRC, "rb") as f:
        ok = hashlib.sha256(f.read()).hexdigest() == COUNTERS_SRC_SHA256
    return TRAFFIC_BYTES_PER_LAUNCH if ok else None


def cpu_baseline(a, target_seconds=12.0):
    from oracle.oracle import default
    orc = default()
    # the host's share of cores: OMP_NUM_THREADS where set, at most 16
    threads = min(int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1), 16)
    chunk = orc.CHUNK_STEPS
    nch = 256
    t0 = time.perf_counter()
    orc.ryser_sample(a, 0, nch, threads)
    dt = time.perf_counter() - t0
    # grow the sample to about target_seconds of wall time
    nch = int(min(max(nch * target_seconds / max(dt, 1e-3), nch), (1 << (N - 1)) // chunk))
    t0 = time.perf_counter()
    orc.ryser_sample(a, 1024, nch, threads)
    dt = time.perf_counter() - t0
    steps = nch * chunk
    # the same oracle on one thread, over a smaller sample (about 2 s)
    total = (1 << (N - 1)) // chunk
    n1 = min(max(1, int(nch * 2.0 / (max(dt, 1e-3) * threads))), total)
    t0 = time.perf_counter()
    orc.ryser_sample(a, 0, n1, 1)
    dt1 = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "subset-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} of the 2^31 Gray steps of the same 32x32 U[0,1) matrix "
                      f"({nch} chunks of {chunk} steps, long double), {dt:.2f} s wall",
            "single_thread": {"value": n1 * chunk / dt1, "unit": "subset-steps/s",
                              "sample": f"{n1} chunks of {chunk} steps on one thread, "
                                        f"{dt1:.2f} s wall"}}


def bench_batched(reps: int = 5, use_graph: bool = True, baselines: bool = True):
    """Batched perm + dperm/dA of the 4096-matrix photon-counting batch (one
    hipGraph launch) against per-matrix launches: of perm_grad, and of the
    plain forward solver (perm_dense_c128 on the matrix and on each of its
    k^2 minors), the latter timed on one matrix per order and extrapolated
    over the batch's order histogram."""
    import numpy as np
    import torch
    from paper_2502_16577_amd import api, workloads

    dev = torch.device("cuda:0")
    mats = workloads.batched_submatrices(4096, 8, 24)
    ks, offs, data = workloads.pack(mats)
    d = torch.from_numpy(data).to(dev)
    plan = api.BatchedPlan(ks, offs, want_grad=True)
    tuned_ms = plan.autotune(d)
    out, grad = plan.outputs(d)
    stream = torch.cuda.current_stream(dev)
    for _ in range(2):
        plan.run(d, out=out, grad=grad, use_graph=use_graph)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.run(d, out=out, grad=grad, use_graph=use_graph)
    e1.record(stream)
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1) / reps
    if not baselines:
        return {"matrices": 4096, "batch_ms": batch_ms, "value": 4096 / (batch_ms * 1e-3),
                "unit": "matrices/s (perm+grad)", "graph": use_graph,
                "autotuned": {"best_ms": tuned_ms, **plan.info()}}

    # per-matrix perm_grad launches over the whole batch
    dm = [torch.from_numpy(a).to(dev) for a in mats]
    wsg = torch.empty(max(api.workspace_bytes(6, n) for n in range(1, 25)), dtype=torch.uint8,
                      device=dev)
    po = torch.empty((), dtype=torch.complex128, device=dev)
    go = torch.empty((24, 24), dtype=torch.complex128, device=dev)
    for a in dm[:64]:
        k = a.shape[0]
        api.perm_grad(a, out_perm=po, out_grad=go[:k, :k].contiguous(), ws=wsg)
    torch.cuda.synchronize()
    gbuf = [torch.empty((a.shape[0], a.shape[0]), dtype=torch.complex128, device=dev) for a in dm]
    t0 = time.perf_counter()
    for a, g in zip(dm, gbuf):
        api.perm_grad(a, out_perm=po, out_grad=g, ws=wsg)
    torch.cuda.synchronize()
    per_grad_ms = (time.perf_counter() - t0) * 1e3

    # plain forward solver: perm + every minor, one launch each (sampled per order)
    wsp = torch.empty(max(api.workspace_bytes(2, n) for n in range(1, 25)), dtype=torch.uint8,
                      device=dev)
    per_k = {}
    for k in sorted(set(int(x) for x in ks)):
        m = int(np.nonzero(ks == k)[0][0])
        a = mats[m]
        minors = [torch.from_numpy(np.ascontiguousarray(np.delete(np.delete(a, i, 0), j, 1))).to(dev)
                  for i in range(k) for j in range(k)]
        full = dm[m]
        api.perm_dense_c128(full, out=po, ws=wsp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.perm_dense_c128(full, out=po, ws=wsp)
        for mm in minors:
            api.perm_dense_c128(mm, out=po, ws=wsp)
        torch.cuda.synchronize()
        per_k[k] = (time.perf_counter() - t0) * 1e3
    plain_ms = float(sum(per_k[int(k)] for k in ks))

    # GEMM-equivalent work of the contraction G += V tau^T: 2 real GEMMs (Re, Im
    # of V) x 2 k^2 flops per subset; the windowed kernel issues 1/16 of it on MFMA
    mfma_flops = float(sum((2 ** (int(k) - 1)) * 4 * int(k) ** 2 for k in ks))
    # FP64 slot operations of the complex sweep with its gradient, 20k + 60
    # per subset-step (as for the single-matrix adjoint)
    alu_ops = float(sum((2 ** (int(k) - 1)) * (20 * int(k) + 60) for k in ks))
    alu_tflops = alu_ops / (batch_ms * 1e-3) / 1e12
    return {
        "workload": "4096 complex128 k x k submatrices, k ~ U{8..24}, rows/cols drawn with "
                    "repetition from a 64x64 Haar unitary (seeds 16583, 16584); perm + dperm/dA",
        "matrices": 4096,
        "subset_steps": int(sum(2 ** (int(k) - 1) for k in ks)),
        "batch_ms": batch_ms,
        "value": 4096 / (batch_ms * 1e-3),
        "unit": "matrices/s (perm+grad)",
        "autotuned": {"best_ms": tuned_ms, **plan.info()},
        "per_matrix_perm_grad_ms": per_grad_ms,
        "plain_solver_ms_extrapolated": plain_ms,
        "plain_solver_sample": "one matrix per order k: perm_dense_c128 on A and on each of its "
                               "k^2 minors (1 + k^2 launches), scaled by the order histogram",
        "speedup_vs_plain_solver": plain_ms / batch_ms,
        "speedup_vs_per_matrix_perm_grad": per_grad_ms / batch_ms,
        "gemm_equivalent_tflops": mfma_flops / (batch_ms * 1e-3) / 1e12,
        "roofline": {"bound": "alu", "achieved": alu_tflops, "peak": PEAK_ALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": alu_tflops / PEAK_ALU_TFLOPS,
                     "ops_per_subset_step": "20k + 60"},
    }


def _timed(fn, reps, stream):
    """Average HIP-event milliseconds of fn() over reps calls on stream."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_rows():
    """One JSON line per hot-path row other than the headline: the complex
    sweep (30x30 Haar block), the sparse real path and the Section 4 pipeline
    (40x40, 6 per row), the exact binary path (32x32 Bernoulli, 40x40 sparse),
    and perm + dperm/dA of one matrix (24x24 real and complex)."""
    import torch
    from paper_2502_16577_amd import api, workloads

    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)

    def line(rec):
        print(json.dumps(rec), flush=True)

    # a7: complex dense sweep, priced like the real one in FP64 operations
    # that each take one instruction slot (add, mul, FMA): 2n adds, n - 1
    # complex products of 2 mul + 2 FMA, 2 accumulation adds = 6n - 2 per step
    n = 30
    A = torch.from_numpy(workloads.haar_block(120, n, workloads.SEED_HAAR120)).to(dev)
    out = torch.empty((), dtype=torch.complex128, device=dev)
    ws = torch.empty(api.workspace_bytes(2, n), dtype=torch.uint8, device=dev)
    for _ in range(10):  # untimed: the first calls run while the clocks ramp up
        api.perm_dense_c128(A, out=out, ws=ws)
    ms = _timed(lambda: api.perm_dense_c128(A, out=out, ws=ws), 10, st)
    fl = (6 * n - 2) * 2 ** (n - 1)
    line({"row": "a7 complex sweep", "workload": "30x30 block of a 120x120 Haar unitary (seed 16581)",
          "ms": ms, "subset_steps_per_s": 2 ** (n - 1) / (ms * 1e-3),
          "roofline": {"bound": "alu", "achieved": fl / (ms * 1e-3) / 1e12, "peak": PEAK_ALU_TFLOPS,
                       "unit": "TFLOP/s", "frac": fl / (ms * 1e-3) / 1e12 / PEAK_ALU_TFLOPS,
                       "ops_per_subset_step": 6 * n - 2,
                       "flops_per_subset_step_fma_as_2": 8 * n - 4}})

    # a8: sparse real (staged columns) and the Section 4 decomposition path
    n = 40
    a = workloads.sparse_rows(n, 6, workloads.SEED_SPARSE40)
    cp, ri, va = workloads.to_csc(a)
    api.perm_sparse_f64(n, cp, ri, va)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v = api.perm_sparse_f64(n, cp, ri, va).item()
    dt = time.perf_counter() - t0
    nnz_col = len(ri) / n
    fl = (n - 1 + nnz_col + 1) * 2 ** (n - 1)  # products, the column's nonzeros, accumulation
    line({"row": "a8 sparse real", "workload": "40x40 0/1 as f64, 6 per row (seed 16582)",
          "seconds": dt, "perm": v, "subset_steps_per_s": 2 ** (n - 1) / dt,
          "roofline": {"bound": "alu", "achieved": fl / dt / 1e12, "peak": PEAK_ALU_TFLOPS,
                       "unit": "TFLOP/s", "frac": fl / dt / 1e12 / PEAK_ALU_TFLOPS,
                       "flops_per_subset_step": n - 1 + nnz_col + 1,
                       "note": "staged dense columns: n adds per step are executed"}})
    # the same matrix through the kernel generated for its pattern (the first
    # call compiles it; the timed call reuses the cached module)
    t0 = time.perf_counter()
    api.perm_sparse_f64_gen(n, cp, ri, va)
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    t0 = time.perf_counter()
    v = api.perm_sparse_f64_gen(n, cp, ri, va).item()
    dt = time.perf_counter() - t0
    # (no roofline: inside a 16-step block the generated product re-uses the
    # product of the rows the block does not touch, so it executes far fewer
    # operations than the n - 1 + nnz_j per step the method is priced at)
    line({"row": "next-4 generated sparse kernel", "workload": "same 40x40 matrix, kernel "
          "generated for its pattern (hiprtc)", "seconds": dt, "first_call_seconds": first,
          "perm": v, "subset_steps_per_s": 2 ** (n - 1) / dt,
          "method_flops_per_s": fl / dt})
    api.perm_sparse_decomp(n, cp, ri, va)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v = api.perm_sparse_decomp(n, cp, ri, va).item()
    dt = time.perf_counter() - t0
    line({"row": "next-3 DecompRyser", "workload": "same 40x40 matrix, DM pruning + Forbert-Marx, "
          "leaves batched on the GPU (host decomposition included)", "seconds": dt, "perm": v})

    # a9: exact binary
    for name, a01 in (("32x32 Bernoulli(1/2) (seed 16580)",
                       workloads.bernoulli(32, workloads.SEED_BERNOULLI32)),
                      ("40x40 0/1, 6 per row (seed 16582)", a)):
        nb = a01.shape[0]
        api.perm_binary_exact(a01)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(st)
        val, res = api.perm_binary_exact(a01)
        e1.record(st)
        dt = time.perf_counter() - t0
        torch.cuda.synchronize()
        gpu_s = e0.elapsed_time(e1) * 1e-3  # staging copy + kernels, on the call's stream
        rec = {"row": "a9 binary exact", "workload": name, "seconds": dt, "gpu_seconds": gpu_s,
               "perm": str(val), "primes": len(res), "subset_steps_per_s": 2 ** (nb - 1) / dt}
        if nb == 32:
            # every subset-step of a dense pattern costs the n adds and n - 1
            # multiplies of the exact FP64 products (plus the zero test), the
            # same FP64 slot count as the real sweep; the modular products of
            # the 9 % nonzero terms come on top
            ops = 2 * nb * 2 ** (nb - 1)
            rec["roofline"] = {"bound": "alu", "achieved": ops / gpu_s / 1e12,
                               "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                               "frac": ops / gpu_s / 1e12 / PEAK_ALU_TFLOPS,
                               "ops_per_subset_step": 2 * nb}
        line(rec)
        # the same through the kernel generated for the pattern
        t0 = time.perf_counter()
        api.perm_binary_exact(a01, generated=True)
        first = time.perf_counter() - t0
        t0 = time.perf_counter()
        gval, gres = api.perm_binary_exact(a01, generated=True)
        dt = time.perf_counter() - t0
        line({"row": "a9 binary exact, generated kernel", "workload": name, "seconds": dt,
              "first_call_seconds": first, "perm": str(gval), "equal": gval == val,
              "subset_steps_per_s": 2 ** (nb - 1) / dt})

    # a10: perm + dperm/dA of one matrix
    for dtype, mat in (("f64", workloads.uniform(24, 1024)),
                       ("c128", workloads.haar_block(120, 24, workloads.SEED_HAAR120))):
        n = 24
        A = torch.from_numpy(mat).to(dev)
        po = torch.empty((), dtype=A.dtype, device=dev)
        go = torch.empty((n, n), dtype=A.dtype, device=dev)
        kind = 5 if dtype == "f64" else 6
        wsg = torch.empty(api.workspace_bytes(kind, n), dtype=torch.uint8, device=dev)
        api.perm_grad(A, out_perm=po, out_grad=go, ws=wsg)
        ms = _timed(lambda: api.perm_grad(A, out_perm=po, out_grad=go, ws=wsg), 5, st)
        cplx = dtype == "c128"
        # G = sum over subsets of V tau^T: n^2 multiply-adds per subset (x2 for complex V)
        gemm = (4 if cplx else 2) * n * n * 2 ** (n - 1)
        # FP64 slot operations per subset-step of the sweep as designed: the x
        # update, the forward product, three products per row for the
        # leave-one-out products (prefix, combine, suffix), the window sums of
        # V, and the 16-lane partial sums of V for the low columns (16 adds
        # per component in each of the two waves); a complex product is 4
        ops = (20 * n + 60) if cplx else (6 * n + 31)
        achieved = ops * 2 ** (n - 1) / (ms * 1e-3) / 1e12
        line({"row": "a10 perm + dperm/dA", "workload": f"24x24 {dtype}", "ms": ms,
              "subset_steps_per_s": 2 ** (n - 1) / (ms * 1e-3),
              "gemm_equivalent_tflops": gemm / (ms * 1e-3) / 1e12,
              "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS,
                           "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS,
                           "ops_per_subset_step": ops}})


# Best published GPU kernel (x_reg-A_shr-rebuild with CEG, Quadro GV100) of
# Table 4 and the precision study of Table 3 (GV100), in seconds / relative error.
PAPER_TABLE4_GV100_S = {30: 0.83, 32: 0.93, 35: 1.20, 40: 14.17, 45: 528.98, 48: 4326.23}
PAPER_TABLE4_CPU44_S = {30: 0.65, 32: 2.74, 35: 23.15, 40: 835.50, 45: 30323.30, 48: 256779.81}
PAPER_TABLE3_GV100 = {35: {"DD": 1.40e-9, "Kahan": 8.78e-12, "DD_s": 1.31, "Kahan_s": 1.34},
                      40: {"DD": 2.69e-7, "Kahan": 6.63e-11, "DD_s": 14.25, "Kahan_s": 14.78},
                      45: {"DD": 1.49e-4, "Kahan": 2.34e-10, "DD_s": 496.34, "Kahan_s": 526.46}}


def _perm_long(api, A, acc, label):
    """perm_dense_f64_ex of A; a sweep of more than 2^43 subset-steps runs as
    groups of its launches (about 2^44 steps, under a minute, per group), with
    one progress line per group."""
    import torch
    n = A.shape[0]
    if n <= 44:
        return api.perm_dense_f64_ex(A, accumulation=acc).item()
    nl = api.dense_f64_launches(n, accumulation=acc)
    group = max(1, nl >> (n - 1 - 44))
    ws = torch.empty(api.workspace_bytes(1, n), dtype=torch.uint8, device=A.device)
    out = torch.empty((), dtype=torch.float64, device=A.device)
    t0 = time.perf_counter()
    for first in range(0, nl, group):
        api.perm_dense_f64_ex(A, accumulation=acc, first_launch=first, launch_count=group,
                              out=out, ws=ws)
        v = out.item()
        print(json.dumps({"progress": label, "n": n, "launches_done": min(first + group, nl),
                          "launches": nl, "seconds": time.perf_counter() - t0}), flush=True)
    return v


def paper_tables(sizes):
    """Table 4 shapes (dense U[0,1), one matrix per n) and Table 3 shapes (all
    entries 0.91, perm = n! 0.91^n, where the paper lists them) on this GPU;
    one JSON line per row."""
    import fractions
    import math
    import torch
    from paper_2502_16577_amd import api, workloads

    dev = torch.device("cuda:0")
    for n in sizes:
        a = workloads.uniform(n, 1000 + n)
        A = torch.from_numpy(a).to(dev)
        if n <= 40:  # untimed first call (clocks, code loading); long sweeps need none
            api.perm_dense_f64(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        v = _perm_long(api, A, api.ACC_TWOSUM, f"table 4, n = {n}")
        dt = time.perf_counter() - t0
        print(json.dumps({"table": 4, "n": n, "workload": f"dense {n}x{n} U[0,1) seed {1000 + n}",
                          "seconds": dt, "subset_steps_per_s": 2 ** (n - 1) / dt, "perm": v,
                          "paper_gv100_s": PAPER_TABLE4_GV100_S.get(n),
                          "paper_cpu44_s": PAPER_TABLE4_CPU44_S.get(n)}), flush=True)
        if PAPER_TABLE3_GV100.get(n) is None:
            continue
        J = torch.full((n, n), 0.91, dtype=torch.float64, device=dev)
        # n! a^n in exact rational arithmetic for the stored double a = fl(0.91)
        exact = float(math.factorial(n) * fractions.Fraction(0.91) ** n)
        for name, acc in (("twosum", api.ACC_TWOSUM), ("kahan", api.ACC_KAHAN),
                          ("plain", api.ACC_PLAIN)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v = _perm_long(api, J, acc, f"table 3, n = {n}, {name}")
            dt = time.perf_counter() - t0
            print(json.dumps({"table": 3, "n": n, "accumulation": name,
                              "workload": f"all entries 0.91, {n}x{n}",
                              "rel_error": abs(v - exact) / exact, "seconds": dt,
                              "paper_gv100": PAPER_TABLE3_GV100.get(n)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched perm+grad leg")
    ap.add_argument("--paper-tables", type=str, default="",
                    help="comma-separated n: time the paper's Table 4 / Table 3 shapes and exit")
    ap.add_argument("--rows", action="store_true",
                    help="time the other hot-path rows (complex, sparse, binary, gradient) and exit")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched perm+grad leg (prints its JSON object)")
    ap.add_argument("--batched-eager", action="store_true",
                    help="launch the batched leg's kernels directly instead of as a hipGraph "
                         "(for counter collection, which does not follow graph launches)")
    ap.add_argument("--batched-quick", action="store_true",
                    help="batched leg without the per-matrix baselines (profiling runs)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (3 times) and exit; "
                         "used to scale FETCH_SIZE / WRITE_SIZE counters to bytes")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": nbytes,
                          "copy_bytes_written_per_launch": nbytes, "launches": 3}))
        return
    if args.paper_tables:
        paper_tables([int(x) for x in args.paper_tables.split(",")])
        return
    if args.rows:
        bench_rows()
        return
    if args.only_batched:
        print(json.dumps(bench_batched(use_graph=not args.batched_eager,
                                       baselines=not args.batched_quick)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: one GPU only (the library has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_16577_amd import api, workloads

    dev = torch.device("cuda:0")
    a = workloads.uniform(N, workloads.SEED_U32)
    A = torch.from_numpy(a).to(dev)
    out = torch.empty((), dtype=torch.float64, device=dev)
    ws = torch.empty(api.workspace_bytes(1, N), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        api.perm_dense_f64(A, out=out, ws=ws)
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s, e in evs:
        s.record(stream)
        api.perm_dense_f64(A, out=out, ws=ws)
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [s.elapsed_time(e) for s, e in evs]
    avg_ms = sum(ev_ms) / len(ev_ms)

    steps_per_call = 2 ** (N - 1)
    value = steps_per_call * args.steps / wall
    flops_per_call = (2 * N + 2) * steps_per_call
    achieved = flops_per_call / (avg_ms * 1e-3) / 1e12

    rec = {
        "metric": "Ryser subset-steps/s & % FP64 peak; batched perm+grad/s vs plain at 1e-10",
        "value": value,
        "unit": "subset-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dense real 32x32, entries U[0,1) (seed 16578), "
                               "one perm_dense_f64 call = 2^31 subset-steps",
                   "n": N, "subset_steps_per_step": steps_per_call},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS, "traffic": traffic_bytes(),
                     "kernel": "sweep_dense_f64<32>", "event_ms_per_launch": avg_ms,
                     "flops_per_subset_step": 2 * N + 2,
                     "frac_of_published_fp64_peak_78.6": achieved / PEAK_FMA_TFLOPS},
        "result": float(out.item()),
    }
    if not args.no_batched:
        rec["batched"] = bench_batched()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(a)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
