"""Python binding of libperm_mi355x.so.

Argument marshalling only: torch supplies device memory (inputs, outputs,
workspaces) and the current HIP stream; every step of the computation runs in
the library's HIP kernels.  Function names follow the C ABI in
include/perm.h.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import torch

from . import _native as N


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def workspace_bytes(kind: int, n: int, m: int = 0) -> int:
    return int(N.lib().perm_workspace_bytes(kind, n, m))


def _workspace(kind: int, n: int, m: int, device, ws=None):
    need = workspace_bytes(kind, n, m)
    if ws is not None:
        if ws.numel() * ws.element_size() < need:
            raise ValueError(f"workspace of {need} bytes needed")
        return ws, need
    return torch.empty(max(need, 1), dtype=torch.uint8, device=device), need


def _check_square(A: torch.Tensor):
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    if A.device.type != "cuda":
        raise ValueError("device tensor expected")
    if A.shape[0] > 0 and A.stride(1) != 1:
        raise ValueError("rows must be contiguous (stride(1) == 1)")


def perm_dense_f64(A: torch.Tensor, out: torch.Tensor | None = None, ws=None) -> torch.Tensor:
    """Permanent of a dense float64 CUDA matrix; returns a 0-d device tensor."""
    _check_square(A)
    if A.dtype != torch.float64:
        raise TypeError("float64 expected")
    n = A.shape[0]
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=A.device)
    ws, need = _workspace(N.KIND_DENSE_F64, n, 0, A.device, ws)
    st = N.lib().perm_dense_f64(n, A.data_ptr() if n else None, A.stride(0) if n else 0,
                                out.data_ptr(), ws.data_ptr(), need, _stream(A.device))
    N.check(st, "perm_dense_f64")
    return out


class PermOptions(ctypes.Structure):
    """perm_options of include/perm.h."""
    _fields_ = [("accumulation", ctypes.c_int), ("log2_reseed", ctypes.c_int),
                ("max_steps_per_launch", ctypes.c_int64), ("log2_lanes", ctypes.c_int),
                ("first_launch", ctypes.c_int64), ("launch_count", ctypes.c_int64)]


ACC_TWOSUM = 0
ACC_PLAIN = 1
ACC_KAHAN = 2
ACC_EXTENDED = 3  # x, products and lane sums in double-double (orders 13..48)


def perm_dense_f64_ex(A: torch.Tensor, accumulation: int = ACC_TWOSUM, log2_reseed: int = 0,
                      max_steps_per_launch: int = 0, log2_lanes: int = 0,
                      first_launch: int = 0, launch_count: int = 0,
                      out: torch.Tensor | None = None, ws=None):
    """perm_dense_f64 with options: accumulation ACC_TWOSUM (default) or
    ACC_PLAIN (the paper's plain-double "DD" variant), the exact re-seed
    interval 2^log2_reseed (0 = default) and the longest single launch.
    ACC_KAHAN selects Kahan-compensated lane sums (the paper's "Kahan");
    ACC_EXTENDED walks x and forms the products in double-double.
    first_launch / launch_count run part of a split sweep: calls over
    consecutive ranges of its launches (dense_f64_launches), in order and with
    the same ws, leave the permanent in out after the last one."""
    _check_square(A)
    if A.dtype != torch.float64:
        raise TypeError("float64 expected")
    n = A.shape[0]
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=A.device)
    ws, need = _workspace(N.KIND_DENSE_F64, n, 0, A.device, ws)
    opt = PermOptions(accumulation, log2_reseed, max_steps_per_launch, log2_lanes, first_launch,
                      launch_count)
    st = N.lib().perm_dense_f64_ex(n, A.data_ptr() if n else None, A.stride(0) if n else 0,
                                   ctypes.byref(opt), out.data_ptr(), ws.data_ptr(), need,
                                   _stream(A.device))
    N.check(st, "perm_dense_f64_ex")
    return out


def dense_f64_launches(n: int, accumulation: int = ACC_TWOSUM, log2_reseed: int = 0,
                       max_steps_per_launch: int = 0, log2_lanes: int = 0) -> int:
    """Number of launches perm_dense_f64_ex splits the sweep of order n into."""
    opt = PermOptions(accumulation, log2_reseed, max_steps_per_launch, log2_lanes, 0, 0)
    r = int(N.lib().perm_dense_f64_launches(n, ctypes.byref(opt)))
    N.check(r if r < 0 else 0, "perm_dense_f64_launches")
    return r


def perm_dense_c128(A: torch.Tensor, out: torch.Tensor | None = None, ws=None) -> torch.Tensor:
    """Permanent of a dense complex128 CUDA matrix; returns a 0-d device tensor."""
    _check_square(A)
    if A.dtype != torch.complex128:
        raise TypeError("complex128 expected")
    n = A.shape[0]
    if out is None:
        out = torch.empty((), dtype=torch.complex128, device=A.device)
    ws, need = _workspace(N.KIND_DENSE_C128, n, 0, A.device, ws)
    st = N.lib().perm_dense_c128(n, A.data_ptr() if n else None, A.stride(0) if n else 0,
                                 out.data_ptr(), ws.data_ptr(), need, _stream(A.device))
    N.check(st, "perm_dense_c128")
    return out


def perm_dense_c128_ex(A: torch.Tensor, accumulation: int = ACC_TWOSUM, log2_reseed: int = 0,
                       out: torch.Tensor | None = None, ws=None) -> torch.Tensor:
    """perm_dense_c128 with an accumulation mode: ACC_TWOSUM (default) or
    ACC_EXTENDED (x, products and lane sums in double-double; orders 13..32,
    where log2_reseed sets the exact re-seed interval)."""
    _check_square(A)
    if A.dtype != torch.complex128:
        raise TypeError("complex128 expected")
    n = A.shape[0]
    if out is None:
        out = torch.empty((), dtype=torch.complex128, device=A.device)
    ws, need = _workspace(N.KIND_DENSE_C128, n, 0, A.device, ws)
    opt = PermOptions(accumulation, log2_reseed, 0, 0, 0, 0)
    st = N.lib().perm_dense_c128_ex(n, A.data_ptr() if n else None, A.stride(0) if n else 0,
                                    ctypes.byref(opt), out.data_ptr(), ws.data_ptr(), need,
                                    _stream(A.device))
    N.check(st, "perm_dense_c128_ex")
    return out


def _sparse_call(fn_name, n, col_ptr, row_idx, vals, device, out, ws):
    col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int32)
    row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    device = torch.device(device)
    nnz = int(row_idx.size)
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=device)
    ws, need = _workspace(N.KIND_SPARSE_F64, n, nnz, device, ws)
    st = getattr(N.lib(), fn_name)(n, col_ptr.ctypes.data if n else None,
                                   row_idx.ctypes.data if nnz else None,
                                   vals.ctypes.data if nnz else None, nnz, out.data_ptr(),
                                   ws.data_ptr(), need, _stream(device))
    N.check(st, fn_name)
    return out


def perm_sparse_f64(n: int, col_ptr, row_idx, vals, device="cuda:0", out=None, ws=None):
    """Permanent of a sparse real matrix given in CSC on the host (Algorithm
    2: a step updates x by the flipped column's nonzeros only, through a
    kernel compiled for the pattern; the module is cached per device and
    pattern)."""
    return _sparse_call("perm_sparse_f64", n, col_ptr, row_idx, vals, device, out, ws)


def perm_sparse_f64_staged(n: int, col_ptr, row_idx, vals, device="cuda:0", out=None, ws=None):
    """perm_sparse_f64 without run-time compilation (dense column copies)."""
    return _sparse_call("perm_sparse_f64_staged", n, col_ptr, row_idx, vals, device, out, ws)


def perm(A: torch.Tensor) -> torch.Tensor:
    """Permanent of a dense float64 or complex128 CUDA matrix."""
    if A.dtype == torch.complex128:
        return perm_dense_c128(A)
    return perm_dense_f64(A)


def _csc_of(a01):
    """CSC pattern (col_ptr, row_idx) of a square 0/1 matrix (host)."""
    a = np.asarray(a01.cpu() if isinstance(a01, torch.Tensor) else a01)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("square matrix expected")
    if not np.all((a == 0) | (a == 1)):
        raise ValueError("0/1 entries expected")
    n = a.shape[0]
    col_ptr = np.zeros(n + 1, np.int32)
    rows = []
    for j in range(n):
        nz = np.nonzero(a[:, j])[0]
        rows.extend(int(r) for r in nz)
        col_ptr[j + 1] = len(rows)
    return n, col_ptr, np.array(rows, np.int32)


def perm_binary_exact(a01=None, *, csc=None, n_primes: int = 0, device="cuda:0", ws=None,
                      generated: bool = False):
    """Exact permanent of a 0/1 matrix (dense 0/1 array or csc=(n, col_ptr, row_idx)).

    generated=True runs perm_binary_exact_gen (a kernel compiled for the
    pattern).  Returns (value as Python int, list of residues perm mod p_k)."""
    if csc is None:
        n, col_ptr, row_idx = _csc_of(a01)
    else:
        n, col_ptr, row_idx = csc
        col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int32)
        row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
    device = torch.device(device)
    ws, need = _workspace(N.KIND_BINARY, n, 0, device, ws)
    limbs = np.zeros(5, np.uint64)
    res = np.zeros(6, np.uint64)
    used = ctypes.c_int(0)
    nnz = int(row_idx.size)
    fn = N.lib().perm_binary_exact_gen if generated else N.lib().perm_binary_exact
    st = fn(
        n, col_ptr.ctypes.data if n else None,
        row_idx.ctypes.data if nnz else None, nnz, n_primes,
        limbs.ctypes.data, res.ctypes.data, ctypes.byref(used), ws.data_ptr(), need,
        _stream(device))
    N.check(st, "perm_binary_exact_gen" if generated else "perm_binary_exact")
    value = 0
    for k in range(4, -1, -1):
        value = (value << 64) | int(limbs[k])
    return value, [int(r) for r in res[:used.value]]


def binary_prime(k: int) -> int:
    return int(N.lib().perm_binary_prime(k))


DTYPE_F64 = 1
DTYPE_C128 = 2


def perm_grad(A: torch.Tensor, out_perm=None, out_grad=None, ws=None):
    """Permanent and dperm/dA of a dense float64 / complex128 CUDA matrix (n <= 32).

    Returns (perm as a 0-d tensor, G as an n x n tensor); for complex A, G is
    the complex derivative dperm/da_ij."""
    _check_square(A)
    if A.dtype == torch.float64:
        dt, kind = DTYPE_F64, N.KIND_GRAD_F64
    elif A.dtype == torch.complex128:
        dt, kind = DTYPE_C128, N.KIND_GRAD_C128
    else:
        raise TypeError("float64 or complex128 expected")
    n = A.shape[0]
    if out_perm is None:
        out_perm = torch.empty((), dtype=A.dtype, device=A.device)
    if out_grad is None:
        out_grad = torch.empty((n, n), dtype=A.dtype, device=A.device)
    ws, need = _workspace(kind, n, 0, A.device, ws)
    st = N.lib().perm_grad(n, dt, A.data_ptr() if n else None, A.stride(0) if n else 0,
                           out_perm.data_ptr(), out_grad.data_ptr() if n else None,
                           ws.data_ptr(), need, _stream(A.device))
    N.check(st, "perm_grad")
    return out_perm, out_grad


class Perm(torch.autograd.Function):
    """perm(A) with a hand-written adjoint: forward runs perm_grad when A
    needs a gradient (the gradient comes from the same sweep), backward
    returns grad_out * G (real) or grad_out * conj(G) (complex, PyTorch's
    convention for holomorphic functions)."""

    @staticmethod
    def forward(ctx, A):
        if ctx.needs_input_grad[0]:
            p, g = perm_grad(A)
            ctx.save_for_backward(g)
            return p
        return perm(A)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        if g.is_complex():
            return grad_out * g.conj()
        return grad_out * g


def permanent(A: torch.Tensor) -> torch.Tensor:
    """Differentiable permanent of a dense float64 / complex128 CUDA matrix."""
    return Perm.apply(A)


class BatchedPlan:
    """Plan of a batched permanent (+ gradient) launch over packed complex
    (``real=False``, complex128 data) or real (``real=True``, float64 data)
    matrices.

    ``ks``: orders (1..32); ``offsets``: element offsets into the packed data
    (``workloads.pack`` produces both).  Owns the C plan and a workspace."""

    def __init__(self, ks, offsets, want_grad: bool = True, device="cuda:0", real: bool = False):
        self.ks = np.ascontiguousarray(ks, dtype=np.int32)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.count = int(self.ks.size)
        self.want_grad = bool(want_grad)
        self.device = torch.device(device)
        self.real = bool(real)
        self.dtype = torch.float64 if self.real else torch.complex128
        sfx = "_f64" if self.real else ""
        self._run = getattr(N.lib(), "perm_batched" + sfx)
        self._tune = getattr(N.lib(), "perm_batched_autotune" + sfx)
        h = ctypes.c_void_p()
        N.check(getattr(N.lib(), "perm_batched_plan_create" + sfx)(
            self.count, self.ks.ctypes.data, self.offsets.ctypes.data, int(want_grad),
            ctypes.byref(h)), "perm_batched_plan_create" + sfx)
        self._h = h
        nb = int(N.lib().perm_batched_workspace_bytes(h))
        self.ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=self.device)
        self.ws_bytes = nb

    def close(self):
        """Destroys the C plan (it waits for the plan's last graph launch
        first) and releases the workspace.  Idempotent."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            N.lib().perm_plan_destroy(h)
        self._h = None
        self.ws = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # At interpreter exit the HIP runtime may already be shutting down:
        # then the plan is left to the process teardown instead of calling
        # into HIP (close() is the deterministic way to release it).
        if sys.is_finalizing() or N is None:
            return
        self.close()

    def outputs(self, data: torch.Tensor):
        out = torch.empty(self.count, dtype=self.dtype, device=self.device)
        grad = torch.empty_like(data) if self.want_grad else None
        return out, grad

    def run(self, data: torch.Tensor, out=None, grad=None, use_graph: bool = True):
        if data.dtype != self.dtype or data.device != self.device or not data.is_contiguous():
            raise ValueError(f"contiguous {self.dtype} data on the plan's device expected")
        if out is None:
            out, g2 = self.outputs(data)
            grad = g2 if grad is None else grad
        st = self._run(self._h, data.data_ptr(), out.data_ptr(),
                                  grad.data_ptr() if grad is not None else None, int(use_graph),
                                  self.ws.data_ptr(), self.ws_bytes, _stream(self.device))
        N.check(st, "perm_batched")
        return out, grad

    def autotune(self, data: torch.Tensor):
        out, grad = self.outputs(data)
        best = ctypes.c_double(0.0)
        if data.dtype != self.dtype or data.device != self.device or not data.is_contiguous():
            raise ValueError(f"contiguous {self.dtype} data on the plan's device expected")
        N.check(self._tune(self._h, data.data_ptr(), out.data_ptr(),
                                              grad.data_ptr() if grad is not None else None,
                                              self.ws.data_ptr(), self.ws_bytes,
                                              _stream(self.device), ctypes.byref(best)),
                "perm_batched_autotune")
        return best.value

    def info(self):
        """Work items, log2 steps per lane, persistent grid per group of
        orders (1..16, 17..24, 25..32) and whether the tuning came from an
        earlier autotune in this process."""
        ni, lc, fc = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        grid = np.zeros(3, np.int64)
        N.check(N.lib().perm_batched_plan_info(self._h, ctypes.byref(ni), ctypes.byref(lc),
                                               grid.ctypes.data, ctypes.byref(fc)),
                "perm_batched_plan_info")
        return {"items": ni.value, "log2_chunk": lc.value,
                "grid": {"k1_16": int(grid[0]), "k17_24": int(grid[1]), "k25_32": int(grid[2])},
                "tuned_from_cache": bool(fc.value)}


DECOMP_DM = 1
DECOMP_FM = 2
DECOMP_FOLD = 4


def _decompose_arrays(n: int, col_ptr, row_idx, vals, flags: int, min_leaf: int):
    """perm_decompose + perm_decomp_leaves: (k int32[L], weight float64[L],
    offset int64[L], data float64[total], removed, folded (hi, lo))."""
    col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int32)
    row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    h = ctypes.c_void_p()
    L = N.lib()
    N.check(L.perm_decompose(n, col_ptr.ctypes.data, row_idx.ctypes.data if row_idx.size else None,
                             vals.ctypes.data if vals.size else None, int(row_idx.size), flags,
                             min_leaf, ctypes.byref(h)), "perm_decompose")
    try:
        cnt, mx = ctypes.c_int(), ctypes.c_int()
        tot, rem = ctypes.c_int64(), ctypes.c_int64()
        N.check(L.perm_decomp_info(h, ctypes.byref(cnt), ctypes.byref(mx), ctypes.byref(tot),
                                   ctypes.byref(rem)), "perm_decomp_info")
        ks = np.zeros(cnt.value, np.int32)
        ws = np.zeros(cnt.value, np.float64)
        offs = np.zeros(cnt.value, np.int64)
        data = np.zeros(max(tot.value, 1), np.float64)
        if cnt.value:
            N.check(L.perm_decomp_leaves(h, ks.ctypes.data, ws.ctypes.data, offs.ctypes.data,
                                         data.ctypes.data), "perm_decomp_leaves")
        folded = np.zeros(2, np.float64)
        N.check(L.perm_decomp_folded(h, folded.ctypes.data), "perm_decomp_folded")
        return ks, ws, offs, data, rem.value, folded
    finally:
        L.perm_decomp_destroy(h)


def decompose(n: int, col_ptr, row_idx, vals, flags: int = DECOMP_DM | DECOMP_FM,
              min_leaf: int = 0):
    """Section 4 preprocessing on the host (no GPU work).

    Returns (leaves, removed) with leaves = [(weight, k x k float64 array)]:
    perm(A) = sum weight * perm(leaf); an empty list means perm = 0.  With
    DECOMP_FOLD the leaves of order <= 2 are summed on the host and returned
    as one leaf of order 0 per component of the double-double sum (weight
    hi, then lo), so the identity still reads sum weight * perm(leaf)."""
    ks, ws, offs, data, removed, folded = _decompose_arrays(n, col_ptr, row_idx, vals, flags,
                                                            min_leaf)
    leaves = [(float(ws[i]), data[offs[i]:offs[i] + ks[i] * ks[i]].reshape(ks[i], ks[i]))
              for i in range(len(ks))]
    if flags & DECOMP_FOLD:
        leaves += [(float(f), np.zeros((0, 0))) for f in folded if f != 0.0]
    return leaves, removed


def perm_sparse_decomp(n: int, col_ptr, row_idx, vals,
                       flags: int = DECOMP_DM | DECOMP_FM | DECOMP_FOLD, device="cuda:0",
                       dense_min: int = 20):
    """perm of a sparse real matrix by the Section 4 pipeline: host
    decomposition into weighted leaves (those of order <= 2 summed on the
    host with DECOMP_FOLD); leaves of order >= dense_min each as one real
    full-chip sweep (perm_dense_f64), the smaller ones in one batched launch;
    then a double-double weighted sum on the GPU.  Returns a 0-d float64
    device tensor."""
    device = torch.device(device)
    ks, ws, offs, data, _, folded = _decompose_arrays(n, col_ptr, row_idx, vals, flags, 0)
    out = torch.zeros((), dtype=torch.float64, device=device)
    # the folded sum enters the weighted sum as two order-0 leaves (perm 1)
    fw = [float(f) for f in folded if f != 0.0]
    if len(ks) == 0 and not fw:
        return out
    dense_min = max(2, min(int(dense_min), 33))
    small = np.nonzero(ks < dense_min)[0]
    big = np.nonzero(ks >= dense_min)[0]
    order = np.concatenate([small, big])
    perms = torch.zeros(len(ks) + len(fw), dtype=torch.float64, device=device)
    perms[len(ks):] = 1.0
    dev = torch.from_numpy(data).to(device)  # every leaf, one copy
    keep = [dev]
    if len(small):  # the small leaves in one batched launch, in place
        plan = BatchedPlan(ks[small], offs[small], want_grad=False, device=device, real=True)
        plan.run(dev, out=perms[:len(small)], use_graph=False)
        keep.append(plan)
    for t, i in enumerate(big):  # one real sweep over the whole chip per large leaf
        k = int(ks[i])
        perm_dense_f64(dev[offs[i]:offs[i] + k * k].view(k, k), out=perms[len(small) + t])
    w = torch.from_numpy(np.ascontiguousarray(np.concatenate([ws[order], fw]))).to(device)
    N.check(N.lib().perm_weighted_sum_f64(len(ks) + len(fw), w.data_ptr(), perms.data_ptr(),
                                          out.data_ptr(), _stream(device)),
            "perm_weighted_sum_f64")
    torch.cuda.current_stream(device).synchronize()  # keep plan / weights alive until done
    for obj in keep:
        if isinstance(obj, BatchedPlan):
            obj.close()
    return out
