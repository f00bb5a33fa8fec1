"""Benchmark: Ryser subset-steps/s of the dense FP64 permanent on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the dense real 32 x 32 matrix with i.i.d. U[0,1) entries (seed
16578), resident in HBM before timing.  One step is one complete
perm_dense_f64 call -- staging kernel, the Gray-walk sweep over all 2^31
column subsets, and the fixed-order reduction -- so one step processes
2^31 subset-steps.  Prints one JSON line.

roofline: the sweep is bound by the FP64 vector ALU.  Algorithmic work per
subset-step is 2n + 2 flops (n additions, n multiplications, the sign and
the accumulation; the count the paper uses for its error estimate).  `peak`
is the published FP64 vector peak, 78.6 TFLOP/s, which counts a multiply-add
as two flops; none of this loop's work is multiply-add shaped, so `frac`
cannot exceed 0.5.  `issue_slot_utilisation` is the same work counted as
FP64 lane-operations (one add or multiply each) over the issue rate of
256 CUs x 64 lanes x 2.4 GHz = 3.93e13 per second, whose ceiling is 1.  The
duration is the average HIP event time of one call on the launch stream,
which includes the two tiny kernels around the sweep (under 0.5 % of it).

rows: the other hot-path rows measured in the same run (complex 30 x 30,
exact binary 32 x 32 and 40 x 40, sparse real 40 x 40, perm + gradient of a
24 x 24 matrix), each with its time and its difference from the stored
oracle value (tests/golden/) against the tolerance used in the tests.

batched: one hipGraph launch of perm + dperm/dA for the 4096-matrix batch,
against per-matrix launches captured in graphs (so the device time is
compared, not the Python launch loop), with the accuracy of both checked.

cpu_baseline: the CPU oracle (long double) timed on a bounded sample of the
same matrix's Gray walk, on the cores this process may use.
"""
from __future__ import annotations

import argparse
import fractions
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 32
PEAK_FP64_TFLOPS = 78.6                          # published FP64 vector peak (FMA = 2 flops)
LANE_OPS_PER_S = 256 * 64 * 2.4e9                # FP64 lane-operations issued per second
GOLDEN = os.path.join(ROOT, "tests", "golden")

# HBM bytes per sweep launch from rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a
# plain 1 GiB copy (profiles/sweep_dense_f64_n32_u01.md).  Valid only for the
# kernel source they were measured on; reported as null once it changes.
COUNTERS_SRC = os.path.join(ROOT, "paper_2502_16577_amd", "csrc", "sweep_f64.hip")
COUNTERS_SRC_SHA256 = "bb41e5ba510883f728a454befe2ef0f1682db634e86eec74dda9464e9ddee02a"
TRAFFIC_BYTES_PER_LAUNCH = 188.0 * 1024 * 2.000 + 32 * 1024 * 1.000


def traffic_bytes():
    import hashlib
    with open(COUNTERS_SRC, "rb") as f:
        ok = hashlib.sha256(f.read()).hexdigest() == COUNTERS_SRC_SHA256
    return TRAFFIC_BYTES_PER_LAUNCH if ok else None


def _json(rec) -> str:
    """One JSON line; numpy scalars become plain numbers and booleans."""
    return json.dumps(rec, default=lambda o: o.item() if hasattr(o, "item") else str(o))


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def host_cpu():
    """Cores this process may use: its affinity set, capped by the cgroup CPU
    quota where one is set; with nproc and the CPU model."""
    nproc = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = nproc
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()[:2]
            if q != "max":
                quota = max(1, int(int(q) / int(per)))
    except (OSError, ValueError):
        pass
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = min(affinity, quota) if quota else affinity
    return {"threads": threads, "nproc": nproc, "affinity": affinity, "cgroup_quota_cpus": quota,
            "cpu_model": model}


def cpu_baseline(a, target_seconds=12.0):
    from oracle.oracle import default
    orc = default()
    cpu = host_cpu()
    threads = cpu["threads"]
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
            "host": cpu,
            "single_thread": {"value": n1 * chunk / dt1, "unit": "subset-steps/s",
                              "sample": f"{n1} chunks of {chunk} steps on one thread, "
                                        f"{dt1:.2f} s wall"}}


def _graph_ms(fn, reps=3):
    """Captures the launches fn() makes on the current stream into one graph,
    replays it (once untimed) and returns the average HIP-event milliseconds
    of a replay: the device time of the launches without the host's Python
    loop between them."""
    import torch
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    g.replay()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        g.replay()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del g
    return ms


def bench_batched(reps: int = 5, use_graph: bool = True, baselines: bool = True,
                  autotune: bool = True):
    """Batched perm + dperm/dA of the 4096-matrix photon-counting batch (one
    hipGraph launch) against per-matrix launches, each side's device time:
    perm_grad on every matrix (all 4096 calls captured in one graph), and the
    plain forward solver -- perm_dense_c128 on the matrix and on each of its
    k^2 minors -- captured per order for one matrix of every order and scaled
    by the batch's order histogram.  Accuracy: the batch against the stored
    oracle sample, and every per-matrix result against the batch."""
    import numpy as np
    import torch
    from paper_2502_16577_amd import api, workloads

    dev = torch.device("cuda:0")
    mats = workloads.batched_submatrices(4096, 8, 24)
    ks, offs, data = workloads.pack(mats)
    d = torch.from_numpy(data).to(dev)
    plan = api.BatchedPlan(ks, offs, want_grad=True)
    try:
        tuned_ms = plan.autotune(d) if autotune else None
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
        info = plan.info()
    finally:
        plan.close()
    rec = {"workload": "4096 complex128 k x k submatrices, k ~ U{8..24}, rows/cols drawn with "
                       "repetition from a 64x64 Haar unitary (seeds 16583, 16584); perm + dperm/dA",
           "matrices": 4096, "subset_steps": int(sum(2 ** (int(k) - 1) for k in ks)),
           "batch_ms": batch_ms, "value": 4096 / (batch_ms * 1e-3),
           "unit": "matrices/s (perm+grad)", "graph": use_graph,
           "autotuned": {"best_ms": tuned_ms, **info}}
    # FP64 slot operations of the complex sweep with its gradient, 20k + 60
    # per subset-step (as for the single-matrix adjoint)
    alu_ops = float(sum((2 ** (int(k) - 1)) * (20 * int(k) + 60) for k in ks))
    lane_ops_per_s = alu_ops / (batch_ms * 1e-3)
    rec["roofline"] = {"bound": "alu", "achieved": lane_ops_per_s / 1e12, "peak": LANE_OPS_PER_S / 1e12,
                       "unit": "T lane-ops/s", "frac": lane_ops_per_s / LANE_OPS_PER_S,
                       "ops_per_subset_step": "20k + 60",
                       "note": "FP64 lane-operations (add, mul, FMA one each) over the issue "
                               "rate 256 x 64 x 2.4e9"}
    if not baselines:
        return rec

    oh = out.cpu().numpy()
    gh = grad.cpu().numpy()
    G = [gh[o:o + k * k].reshape(k, k) for k, o in zip(ks, offs)]
    # accuracy of the batch against the stored oracle sample
    smp = _golden("samples.json")["batched"]
    assert smp["digest"] == workloads.digest(data), "batched sample input drifted"
    worst = {"perm": 0.0, "minor": 0.0, "fd": 0.0}
    for e in smp["perms"]:
        want = complex(*e["value"])
        worst["perm"] = max(worst["perm"], abs(oh[e["m"]] - want) / (1e-13 * e["abs_sum"]))
    for e in smp["minors"]:
        want = complex(*e["value"])
        worst["minor"] = max(worst["minor"], abs(G[e["m"]][e["i"], e["j"]] - want) / (1e-10 * e["abs_perm"]))
    for e in smp["fd"]:
        want = complex(*e["value"])
        worst["fd"] = max(worst["fd"], abs(G[e["m"]][e["i"], e["j"]] - want) / (1e-6 * abs(want)))
    rec["accuracy_vs_oracle"] = {
        "sample": f"{len(smp['perms'])} permanents, {len(smp['minors'])} minors, "
                  f"{len(smp['fd'])} central differences (tests/golden/samples.json)",
        "worst_over_tolerance": worst,
        "tolerances": "perm 1e-13 R(A); minor 1e-10 perm(|minor|); FD 1e-6 |FD|"}

    # per-matrix perm_grad: every call captured into one graph
    dm = [torch.from_numpy(a).to(dev) for a in mats]
    wsg = torch.empty(max(api.workspace_bytes(6, n) for n in range(1, 25)), dtype=torch.uint8,
                      device=dev)
    pbuf = torch.empty(4096, dtype=torch.complex128, device=dev)
    gbuf = [torch.empty((a.shape[0], a.shape[0]), dtype=torch.complex128, device=dev) for a in dm]

    def per_matrix():
        for m, (a, g) in enumerate(zip(dm, gbuf)):
            api.perm_grad(a, out_perm=pbuf[m], out_grad=g, ws=wsg)

    t0 = time.perf_counter()
    per_matrix()
    torch.cuda.synchronize()
    per_wall_ms = (time.perf_counter() - t0) * 1e3
    per_grad_ms = _graph_ms(per_matrix)
    pb = pbuf.cpu().numpy()
    diff_p = max(abs(pb[m] - oh[m]) / max(abs(oh[m]), 1e-300) for m in range(4096))
    diff_g = max(float(np.max(np.abs(gbuf[m].cpu().numpy() - G[m])) / np.max(np.abs(G[m])))
                 for m in range(4096))

    # plain forward solver: perm + every minor, 1 + k^2 launches per matrix,
    # captured per order for one matrix of that order
    wsp = torch.empty(max(api.workspace_bytes(2, n) for n in range(1, 25)), dtype=torch.uint8,
                      device=dev)
    per_k, plain_diff = {}, 0.0
    for k in sorted(set(int(x) for x in ks)):
        m = int(np.nonzero(ks == k)[0][0])
        a = mats[m]
        minors = [torch.from_numpy(np.ascontiguousarray(np.delete(np.delete(a, i, 0), j, 1))).to(dev)
                  for i in range(k) for j in range(k)]
        res = torch.empty(1 + k * k, dtype=torch.complex128, device=dev)

        def plain():
            api.perm_dense_c128(dm[m], out=res[0], ws=wsp)
            for t, mm in enumerate(minors):
                api.perm_dense_c128(mm, out=res[1 + t], ws=wsp)

        per_k[k] = _graph_ms(plain, reps=1)
        rh = res.cpu().numpy()
        plain_diff = max(plain_diff, float(np.max(np.abs(rh[1:].reshape(k, k) - G[m])) / np.max(np.abs(G[m]))))
    plain_ms = float(sum(per_k[int(k)] for k in ks))
    rec.update({
        "per_matrix_perm_grad_ms": per_grad_ms,
        "per_matrix_perm_grad_python_loop_ms": per_wall_ms,
        "speedup_vs_per_matrix_perm_grad": per_grad_ms / batch_ms,
        "per_matrix_vs_batch_max_rel_diff": {"perm": diff_p, "grad": diff_g},
        "plain_solver_ms_extrapolated": plain_ms,
        "plain_solver_sample": "one matrix per order k: perm_dense_c128 on A and on each of its "
                               "k^2 minors (1 + k^2 launches, one graph per order), scaled by the "
                               "order histogram",
        "plain_solver_vs_batch_max_rel_diff_grad": plain_diff,
        "speedup_vs_plain_solver": plain_ms / batch_ms,
    })
    return rec


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


def measure_rows():
    """The hot-path rows other than the headline, each timed and checked
    against the stored oracle value: the complex sweep (30x30 Haar block),
    the exact binary path (32x32 Bernoulli; the 40x40 sparse pattern, staged
    and generated kernels), the sparse real path (the 40x40 pattern), and
    perm + dperm/dA of one 24x24 matrix (complex and real).  Returns
    {name: record}."""
    import numpy as np
    import torch
    from paper_2502_16577_amd import api, workloads

    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    full = _golden("full_size.json")
    smp = _golden("samples.json")
    rows = {}

    # a7: complex dense sweep.  FP64 lane-operations per subset-step: 2n
    # adds, n - 1 complex products of 2 mul + 2 FMA, 2 accumulation adds
    n = 30
    a = workloads.haar_block(120, n, workloads.SEED_HAAR120)
    g = full["haar30"]
    assert workloads.digest(a) == g["digest"]
    A = torch.from_numpy(a).to(dev)
    out = torch.empty((), dtype=torch.complex128, device=dev)
    ws = torch.empty(api.workspace_bytes(2, n), dtype=torch.uint8, device=dev)
    for _ in range(10):  # untimed: the first calls run while the clocks ramp up
        api.perm_dense_c128(A, out=out, ws=ws)
    ms = _timed(lambda: api.perm_dense_c128(A, out=out, ws=ws), 10, st)
    want = complex(sum(g["re"]), sum(g["im"]))
    err = abs(complex(out.item()) - want)
    ops = (6 * n - 2) * 2 ** (n - 1)
    rows["a7_complex30"] = {
        "workload": "30x30 block of a 120x120 Haar unitary (seed 16581)", "ms": ms,
        "subset_steps_per_s": 2 ** (n - 1) / (ms * 1e-3),
        "issue_slot_utilisation": ops / (ms * 1e-3) / LANE_OPS_PER_S,
        "abs_err": err, "tol": min(1e-13 * g["abs_sum"], 1e-10 * g["abs_perm"]),
        "ok": bool(err <= 1e-13 * g["abs_sum"] and err <= 1e-10 * g["abs_perm"])}
    # the same matrix in the extended-precision walk (double-double x,
    # products and lane sums), against the same stored value
    api.perm_dense_c128_ex(A, accumulation=api.ACC_EXTENDED, out=out, ws=ws)
    ms_ext = _timed(lambda: api.perm_dense_c128_ex(A, accumulation=api.ACC_EXTENDED, out=out,
                                                   ws=ws), 3, st)
    err_ext = abs(complex(out.item()) - want)
    rows["a7_complex30"].update({"extended_ms": ms_ext, "extended_abs_err": err_ext,
                                 "extended_ok": bool(err_ext <= 1e-10 * g["abs_perm"])})

    # a9: exact binary, 32x32 Bernoulli and the 40x40 sparse pattern
    for name, key, a01 in (("a9_binary32", "bernoulli32", workloads.bernoulli(32, workloads.SEED_BERNOULLI32)),
                           ("a9_binary40", "sparse40", workloads.sparse_rows(40, 6, workloads.SEED_SPARSE40))):
        g = full[key]
        assert workloads.digest(a01) == g["digest"]
        rec = {"workload": {"bernoulli32": "32x32 Bernoulli(1/2) (seed 16580)",
                            "sparse40": "40x40 0/1, 6 per row (seed 16582)"}[key]}
        for label, gen in (("staged", False), ("generated", True)):
            t0 = time.perf_counter()
            api.perm_binary_exact(a01, generated=gen)  # the generated path compiles here
            first = time.perf_counter() - t0
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(st)
            val, res = api.perm_binary_exact(a01, generated=gen)
            e1.record(st)
            dt = time.perf_counter() - t0
            torch.cuda.synchronize()
            rec[label] = {"seconds": dt, "gpu_seconds": e0.elapsed_time(e1) * 1e-3,
                          "first_call_seconds": first, "exact": bool(str(val) == g["value"])}
        rows[name] = rec

    # a8: sparse real, the 40x40 pattern with entries d_i e_j (d, e uniform in
    # [0.5, 1.5), seed 7040): perm = prod d prod e times the pattern's exact
    # permanent; and, once its oracle value is stored, the same pattern with
    # U[0,1) values (Algorithm 2's CSC walk in long double)
    n = 40
    pat = workloads.sparse_rows(n, 6, workloads.SEED_SPARSE40)
    assert workloads.digest(pat) == full["sparse40"]["digest"]
    d, e = workloads.scaling_vectors(n, 7040)
    exact = fractions.Fraction(int(full["sparse40"]["value"]))
    for v in list(d) + list(e):
        exact *= fractions.Fraction(float(v))
    cp, ri, va = workloads.to_csc(pat * np.outer(d, e))
    out = torch.empty((), dtype=torch.float64, device=dev)
    wss = torch.empty(api.workspace_bytes(3, n, len(ri)), dtype=torch.uint8, device=dev)
    t0 = time.perf_counter()
    api.perm_sparse_f64(n, cp, ri, va, out=out, ws=wss)
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    ms = _timed(lambda: api.perm_sparse_f64(n, cp, ri, va, out=out, ws=wss), 3, st)
    want = float(exact)
    rel = abs(out.item() - want) / abs(want)
    ms_staged = _timed(lambda: api.perm_sparse_f64_staged(n, cp, ri, va, out=out, ws=wss), 1, st)
    rel_staged = abs(out.item() - want) / abs(want)
    rows["a8_sparse40"] = {
        "workload": "40x40 pattern with 6 per row (seed 16582), values d_i e_j, d and e uniform "
                    "in [0.5, 1.5) (seed 7040); perm_sparse_f64 (kernel generated for the pattern)",
        "ms": ms, "first_call_seconds": first, "subset_steps_per_s": 2 ** (n - 1) / (ms * 1e-3),
        "rel_err": rel, "tol": 1e-10, "ok": bool(rel <= 1e-10),
        "staged_ms": ms_staged, "staged_rel_err": rel_staged}
    if "sparse40u" in full:
        g = full["sparse40u"]
        a = pat * workloads.uniform(n, workloads.SEED_SPARSE40_VALUES)
        assert workloads.digest(a) == g["digest"]
        cp, ri, va = workloads.to_csc(a)
        want = g["value"][0] + g["value"][1]
        api.perm_sparse_f64(n, cp, ri, va, out=out, ws=wss)
        rel_u = abs(out.item() - want) / abs(want)
        api.perm_sparse_f64_staged(n, cp, ri, va, out=out, ws=wss)
        rel_us = abs(out.item() - want) / abs(want)
        rel_ud = abs(api.perm_sparse_decomp(n, cp, ri, va).item() - want) / abs(want)
        rows["a8_sparse40"]["u_values"] = {
            "workload": "the same pattern with U[0,1) values (seed 16585)",
            "rel_err": rel_u, "staged_rel_err": rel_us, "decomposition_rel_err": rel_ud,
            "forward_error_scale": n * 2.0 ** -53 * g["abs_sum"] / abs(want),
            "r_over_perm": g["abs_sum"] / abs(want), "tol": 1e-10,
            "ok": bool(max(rel_u, rel_us, rel_ud) <= 1e-10)}

    # a10: perm + dperm/dA of one 24x24 matrix (complex and real)
    for name, key, mat in (("a10_grad24c", "grad24c", workloads.haar_block(120, 24, workloads.SEED_HAAR120)),
                           ("a10_grad24r", "grad24r", workloads.uniform(24, 1024))):
        n = 24
        g = smp[key]
        assert workloads.digest(mat) == g["digest"]
        A = torch.from_numpy(mat).to(dev)
        po = torch.empty((), dtype=A.dtype, device=dev)
        go = torch.empty((n, n), dtype=A.dtype, device=dev)
        cplx = key.endswith("c")
        wsg = torch.empty(api.workspace_bytes(6 if cplx else 5, n), dtype=torch.uint8, device=dev)
        for _ in range(3):
            api.perm_grad(A, out_perm=po, out_grad=go, ws=wsg)
        ms = _timed(lambda: api.perm_grad(A, out_perm=po, out_grad=go, ws=wsg), 5, st)
        pv = complex(po.item())
        gh = go.cpu().numpy()
        perr = abs(pv - complex(*g["perm"])) / (1e-13 * g["abs_sum"])
        merr = max(abs(gh[e["i"], e["j"]] - complex(*e["value"])) / (1e-10 * e["abs_perm"])
                   for e in g["minors"])
        # FP64 lane-operations per subset-step as designed: x update, forward
        # product, three products per row for the leave-one-out products, the
        # window sums of V and the 16-lane partial sums for the low columns
        ops = (20 * n + 60) if cplx else (6 * n + 31)
        rows[name] = {"workload": f"24x24 {'Haar block (seed 16581)' if cplx else 'U[0,1) (seed 1024)'}",
                      "ms": ms, "subset_steps_per_s": 2 ** (n - 1) / (ms * 1e-3),
                      "issue_slot_utilisation": ops * 2 ** (n - 1) / (ms * 1e-3) / LANE_OPS_PER_S,
                      "perm_err_over_tol": perr, "minor_err_over_tol": merr,
                      "tol": "perm 1e-13 R(A); minors 1e-10 perm(|minor|)",
                      "ok": bool(perr <= 1.0 and merr <= 1.0)}

    # next-1: the paper's Table 4 shape at n = 40 (2^39 subset-steps) against
    # the stored oracle value, in the default FP64 walk and the
    # extended-precision walk (double-double x and products)
    if "u40" in full:
        n = 40
        g = full["u40"]
        a = workloads.uniform(n, 1000 + n)
        assert workloads.digest(a) == g["digest"]
        want = g["value"][0] + g["value"][1]
        A = torch.from_numpy(a).to(dev)
        out = torch.empty((), dtype=torch.float64, device=dev)
        ws = torch.empty(api.workspace_bytes(1, n), dtype=torch.uint8, device=dev)
        api.perm_dense_f64(A, out=out, ws=ws)
        ms = _timed(lambda: api.perm_dense_f64(A, out=out, ws=ws), 1, st)
        rel = abs(out.item() - want) / abs(want)
        ms_ext = _timed(lambda: api.perm_dense_f64_ex(A, accumulation=api.ACC_EXTENDED, out=out,
                                                      ws=ws), 1, st)
        rel_ext = abs(out.item() - want) / abs(want)
        fwd = n * 2.0 ** -53 * g["abs_sum"] / abs(want)
        rows["next1_table4_n40"] = {
            "workload": "dense 40x40 U[0,1) (seed 1040), 2^39 subset-steps",
            "ms": ms, "rel_err": rel, "forward_error_scale": fwd, "ok_fp64": bool(rel <= fwd),
            "extended_ms": ms_ext, "extended_rel_err": rel_ext, "tol": 1e-10,
            "ok": bool(rel_ext <= 1e-10),
            "paper_gv100_s": PAPER_TABLE4_GV100_S.get(n)}
    return rows


def bench_rows():
    """One JSON line per hot-path row other than the headline (measure_rows),
    and the Section 4 pipeline on the 40x40 sparse matrix."""
    import torch
    from paper_2502_16577_amd import api, workloads

    for name, rec in measure_rows().items():
        print(_json({"row": name, **rec}), flush=True)
    n = 40
    a = workloads.sparse_rows(n, 6, workloads.SEED_SPARSE40)
    g = _golden("full_size.json")["sparse40"]
    assert workloads.digest(a) == g["digest"]
    cp, ri, va = workloads.to_csc(a)
    api.perm_sparse_decomp(n, cp, ri, va)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v = api.perm_sparse_decomp(n, cp, ri, va).item()
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    ks = api._decompose_arrays(n, cp, ri, va, api.DECOMP_DM | api.DECOMP_FM | api.DECOMP_FOLD, 0)[0]
    host = time.perf_counter() - t0
    print(_json({"row": "next-3 DecompRyser", "workload": "40x40 0/1, 6 per row (seed 16582): "
                      "DM pruning + Forbert-Marx (leaves of order <= 2 folded on the host), "
                      "large leaves as real sweeps, the rest batched (host decomposition "
                      "included)", "seconds": dt, "host_decomposition_seconds": host,
                 "leaves": int(len(ks)), "leaf_subset_steps": int(sum(2 ** (int(k) - 1) for k in ks)),
                 "plain_sweep_subset_steps": 2 ** (n - 1), "perm": v,
                 "rel_err": abs(v - int(g["value"])) / int(g["value"])}), flush=True)


# Best published GPU kernel (x_reg-A_shr-rebuild with CEG, Quadro GV100) of
# Table 4 and the precision study of Table 3 (GV100), in seconds / relative error.
PAPER_TABLE4_GV100_S = {30: 0.83, 32: 0.93, 35: 1.20, 40: 14.17, 45: 528.98, 48: 4326.23}
PAPER_TABLE4_CPU44_S = {30: 0.65, 32: 2.74, 35: 23.15, 40: 835.50, 45: 30323.30, 48: 256779.81}
PAPER_TABLE3_GV100 = {35: {"DD": 1.40e-9, "Kahan": 8.78e-12, "DD_s": 1.31, "Kahan_s": 1.34},
                      40: {"DD": 2.69e-7, "Kahan": 6.63e-11, "DD_s": 14.25, "Kahan_s": 14.78},
                      45: {"DD": 1.49e-4, "Kahan": 2.34e-10, "DD_s": 496.34, "Kahan_s": 526.46}}


def _perm_long(api, A, acc, label):
    """perm_dense_f64_ex of A; a sweep of more than 2^43 subset-steps (2^40 in
    the extended-precision walk, about eight times slower) runs as groups of
    its launches (under a minute per group), with one progress line per
    group."""
    import torch
    n = A.shape[0]
    top = 41 if acc == api.ACC_EXTENDED else 44
    if n <= top:
        return api.perm_dense_f64_ex(A, accumulation=acc).item()
    nl = api.dense_f64_launches(n, accumulation=acc)
    group = max(1, nl >> (n - 1 - top))
    ws = torch.empty(api.workspace_bytes(1, n), dtype=torch.uint8, device=A.device)
    out = torch.empty((), dtype=torch.float64, device=A.device)
    t0 = time.perf_counter()
    for first in range(0, nl, group):
        api.perm_dense_f64_ex(A, accumulation=acc, first_launch=first, launch_count=group,
                              out=out, ws=ws)
        v = out.item()
        print(_json({"progress": label, "n": n, "launches_done": min(first + group, nl),
                          "launches": nl, "seconds": time.perf_counter() - t0}), flush=True)
    return v


def paper_tables(sizes, tables=(3, 4), modes=None):
    """Table 4 shapes (dense U[0,1), one matrix per n) and Table 3 shapes (all
    entries 0.91, perm = n! 0.91^n, where the paper lists them) on this GPU;
    one JSON line per row.  `tables` selects the tables and `modes` (names:
    twosum, kahan, plain, extended; None for all) the accumulation modes."""
    import fractions
    import math
    import torch
    from paper_2502_16577_amd import api, workloads

    dev = torch.device("cuda:0")
    all_modes = [("twosum", api.ACC_TWOSUM), ("kahan", api.ACC_KAHAN), ("plain", api.ACC_PLAIN),
                 ("extended", api.ACC_EXTENDED)]
    full = _golden("full_size.json")
    for n in sizes:
        chosen = [(name, acc) for name, acc in all_modes
                  if (modes is None or name in modes)
                  and (acc != api.ACC_EXTENDED or 13 <= n <= 48)]
        if 4 in tables:
            a = workloads.uniform(n, 1000 + n)
            A = torch.from_numpy(a).to(dev)
            g = full.get(f"u{n}")
            want = g["value"][0] + g["value"][1] if g and g.get("digest") == workloads.digest(a) else None
            if n <= 40:  # untimed first call (clocks, code loading); long sweeps need none
                api.perm_dense_f64(A)
            for name, acc in chosen:
                if acc in (api.ACC_KAHAN, api.ACC_PLAIN):
                    continue  # Table 4 reports the default and the extended walk
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                v = _perm_long(api, A, acc, f"table 4, n = {n}, {name}")
                dt = time.perf_counter() - t0
                print(_json({"table": 4, "n": n, "accumulation": name,
                                  "workload": f"dense {n}x{n} U[0,1) seed {1000 + n}",
                                  "seconds": dt, "subset_steps_per_s": 2 ** (n - 1) / dt, "perm": v,
                                  "rel_error_vs_oracle": abs(v - want) / abs(want) if want else None,
                                  "paper_gv100_s": PAPER_TABLE4_GV100_S.get(n),
                                  "paper_cpu44_s": PAPER_TABLE4_CPU44_S.get(n)}), flush=True)
        if 3 not in tables or PAPER_TABLE3_GV100.get(n) is None:
            continue
        J = torch.full((n, n), 0.91, dtype=torch.float64, device=dev)
        # n! a^n in exact rational arithmetic for the stored double a = fl(0.91)
        exact = float(math.factorial(n) * fractions.Fraction(0.91) ** n)
        for name, acc in chosen:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v = _perm_long(api, J, acc, f"table 3, n = {n}, {name}")
            dt = time.perf_counter() - t0
            print(_json({"table": 3, "n": n, "accumulation": name,
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
    ap.add_argument("--no-rows", action="store_true", help="skip the other hot-path rows")
    ap.add_argument("--paper-tables", type=str, default="",
                    help="comma-separated n: time the paper's Table 4 / Table 3 shapes and exit")
    ap.add_argument("--tables", type=str, default="3,4",
                    help="with --paper-tables: which tables (comma-separated: 3, 4)")
    ap.add_argument("--modes", type=str, default="",
                    help="with --paper-tables: accumulation modes (twosum, kahan, plain, "
                         "extended; default all)")
    ap.add_argument("--rows", action="store_true",
                    help="time the other hot-path rows (complex, sparse, binary, gradient) and exit")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched perm+grad leg (prints its JSON object)")
    ap.add_argument("--batched-eager", action="store_true",
                    help="launch the batched leg's kernels directly instead of as a hipGraph "
                         "(for counter collection, which does not follow graph launches)")
    ap.add_argument("--batched-no-tune", action="store_true",
                    help="batched leg with the default plan (no autotuning; profiling runs)")
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
        print(_json({"copy_bytes_read_per_launch": nbytes,
                          "copy_bytes_written_per_launch": nbytes, "launches": 3}))
        return
    if args.paper_tables:
        paper_tables([int(x) for x in args.paper_tables.split(",")],
                     tables=tuple(int(x) for x in args.tables.split(",")),
                     modes=args.modes.split(",") if args.modes else None)
        return
    if args.rows:
        bench_rows()
        return
    if args.only_batched:
        print(_json(bench_batched(use_graph=not args.batched_eager,
                                       baselines=not args.batched_quick,
                                       autotune=not args.batched_no_tune)), flush=True)
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic_bytes(),
                     "kernel": "sweep_dense_f64<32, 0>", "event_ms_per_launch": avg_ms,
                     "flops_per_subset_step": 2 * N + 2,
                     "frac_ceiling": 0.5,
                     "issue_slot_utilisation": achieved * 1e12 / LANE_OPS_PER_S},
        "result": float(out.item()),
    }
    g = _golden("full_size.json")["u32"]
    want = sum(g["value"])
    rec["result_rel_err"] = abs(rec["result"] - want) / want
    if not args.no_rows:
        rec["rows"] = measure_rows()
    if not args.no_batched:
        rec["batched"] = bench_batched()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(a)
    print(_json(rec), flush=True)


if __name__ == "__main__":
    main()
