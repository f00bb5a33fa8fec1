"""Python binding of libperm_mi355x.so.

Argument marshalling only: torch supplies device memory (inputs, outputs,
workspaces) and the current HIP stream; every step of the computation runs in
the library's HIP kernels.  Function names follow the C ABI in
include/perm.h.
"""
from __future__ import annotations

import ctypes

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


def perm(A: torch.Tensor) -> torch.Tensor:
    """Permanent of a dense float64 or complex128 CUDA matrix."""
    if A.dtype == torch.complex128:
        return perm_dense_c128(A)
    return perm_dense_f64(A)
