"""ctypes loader of libperm_mi355x.so (argument marshalling only).

The library is the product: if it is missing this module raises, it never
falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libperm_mi355x.so")

PERM_OK = 0
PERM_EINVAL = -1
PERM_ERANGE = -2
PERM_EWORKSPACE = -3
PERM_EHIP = -4
PERM_EUNSUPPORTED = -5
PERM_ECOMPILE = -6
PERM_ESCRATCH = -7

KIND_DENSE_F64 = 1
KIND_DENSE_C128 = 2
KIND_SPARSE_F64 = 3
KIND_BINARY = 4
KIND_GRAD_F64 = 5
KIND_GRAD_C128 = 6
KIND_BATCHED = 7

# (name, restype, argtypes) of every symbol include/perm.h declares.
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_int = ctypes.c_int
_sz = ctypes.c_size_t
_u64 = ctypes.c_uint64
SIGNATURES = [
    ("perm_strerror", ctypes.c_char_p, [_int]),
    ("perm_version", _int, []),
    ("perm_workspace_bytes", _sz, [_int, _int, _i64]),
    ("perm_dense_f64", _int, [_int, _vp, _i64, _vp, _vp, _sz, _vp]),
    ("perm_dense_f64_ex", _int, [_int, _vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    ("perm_dense_f64_noalloc", _int, [_int, _vp, _i64, _vp, _vp]),
    ("perm_noalloc_scratch_bytes", _sz, []),
    ("perm_dense_f64_launches", _i64, [_int, _vp]),
    ("perm_dense_c128", _int, [_int, _vp, _i64, _vp, _vp, _sz, _vp]),
    ("perm_sparse_f64", _int, [_int, _vp, _vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    ("perm_sparse_f64_staged", _int, [_int, _vp, _vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    ("perm_binary_exact", _int, [_int, _vp, _vp, _i32, _int, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("perm_binary_exact_gen", _int, [_int, _vp, _vp, _i32, _int, _vp, _vp, _vp, _vp, _sz, _vp]),
    ("perm_binary_prime", _u64, [_int]),
    ("perm_grad", _int, [_int, _int, _vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    ("perm_batched_plan_create", _int, [_int, _vp, _vp, _int, ctypes.POINTER(_vp)]),
    ("perm_plan_destroy", None, [_vp]),
    ("perm_batched_workspace_bytes", _sz, [_vp]),
    ("perm_batched", _int, [_vp, _vp, _vp, _vp, _int, _vp, _sz, _vp]),
    ("perm_batched_autotune", _int, [_vp, _vp, _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(ctypes.c_double)]),
    ("perm_weighted_sum", _int, [_int, _vp, _vp, _vp, _vp]),
    ("perm_dense_c128_ex", _int, [_int, _vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    ("perm_batched_plan_create_f64", _int, [_int, _vp, _vp, _int, ctypes.POINTER(_vp)]),
    ("perm_batched_f64", _int, [_vp, _vp, _vp, _vp, _int, _vp, _sz, _vp]),
    ("perm_batched_autotune_f64", _int, [_vp, _vp, _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(ctypes.c_double)]),
    ("perm_weighted_sum_f64", _int, [_int, _vp, _vp, _vp, _vp]),
    ("perm_decompose", _int, [_int, _vp, _vp, _vp, _i32, _int, _int, ctypes.POINTER(_vp)]),
    ("perm_decomp_info", _int, [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_i64),
                                ctypes.POINTER(_i64)]),
    ("perm_decomp_leaf", _int, [_vp, _int, ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double), _vp]),
    ("perm_decomp_leaves", _int, [_vp, _vp, _vp, _vp, _vp]),
    ("perm_decomp_folded", _int, [_vp, _vp]),
    ("perm_decomp_destroy", None, [_vp]),
    ("perm_batched_plan_info", _int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_int), _vp,
                                      ctypes.POINTER(_int)]),
]

_lock = threading.Lock()
_lib = None


class PermError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().perm_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with "
                    "`python -m paper_2502_16577_amd.build` (no fallback exists)")
            L = ctypes.CDLL(LIB_PATH)
            for name, res, args in SIGNATURES:
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def check(status: int, where: str):
    if status != PERM_OK:
        raise PermError(status, where)
