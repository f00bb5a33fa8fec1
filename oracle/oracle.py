"""Python front end of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this module.  The product library never does: it shares no
code with the oracle, and the oracle never imports the product package.

The arithmetic lives in ``perm_oracle.c`` (plain C, long double and exact
integers); this module compiles it with gcc, loads it with ctypes and adds the
few steps that are plain definitions rather than arithmetic of the method:

* ``grad_minors``: dperm/da_ij is the permanent of A with row i and column j
  deleted (the permanent is linear in each entry, and expanding Eq. (1) along
  row i gives the coefficient of a_ij).
* ``grad_fd``: central finite differences; because the permanent is affine in
  each single entry they are exact in exact arithmetic for any step h.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(out_path: str = _LIB_PATH, mutant: int = 0) -> str:
    """Compile perm_oracle.c into a shared library (gcc, -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall",
           "-fno-fast-math", "-ffp-contract=off",
           f"-DORC_MUTANT={int(mutant)}", "-o", out_path, _SRC, "-lpthread"]
    subprocess.run(cmd, check=True)
    return out_path


def _declare(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    u8p = ctypes.POINTER(ctypes.c_ubyte)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    c_int = ctypes.c_int
    lib.orc_gray.restype = ctypes.c_uint64
    lib.orc_gray.argtypes = [ctypes.c_uint64]
    lib.orc_flip_col.restype = c_int
    lib.orc_flip_col.argtypes = [ctypes.c_uint64]
    lib.orc_flip_sign.restype = c_int
    lib.orc_flip_sign.argtypes = [ctypes.c_uint64]
    for name in ("orc_brute_real", "orc_brute_cplx", "orc_inclexcl_real", "orc_inclexcl_cplx"):
        f = getattr(lib, name)
        f.restype = c_int
        f.argtypes = [c_int, dp, dp]
    for name in ("orc_ryser_real", "orc_ryser_cplx"):
        f = getattr(lib, name)
        f.restype = c_int
        f.argtypes = [c_int, dp, c_int, dp, dp]
    lib.orc_ryser_real_sample.restype = c_int
    lib.orc_ryser_real_sample.argtypes = [c_int, dp, c_int, ctypes.c_uint64, ctypes.c_uint64, dp]
    lib.orc_ryser_real_part.restype = c_int
    lib.orc_ryser_real_part.argtypes = [c_int, dp, i32p, i32p, dp, c_int, ctypes.c_uint64,
                                        ctypes.c_uint64, dp, dp]
    lib.orc_ryser_csc_real.restype = c_int
    lib.orc_ryser_csc_real.argtypes = [c_int, i32p, i32p, dp, c_int, dp, dp]
    lib.orc_ryser_binary.restype = c_int
    lib.orc_ryser_binary.argtypes = [c_int, u8p, c_int, u64p, u64p]
    lib.orc_matchings_dp.restype = c_int
    lib.orc_matchings_dp.argtypes = [c_int, u8p, u64p]
    return lib


def load(path: str | None = None):
    """Load the oracle library, building it first if it is missing."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build()
            _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _real(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("square matrix expected")
    return a


def _cplx(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("square matrix expected")
    return a.view(np.float64).reshape(a.shape[0], 2 * a.shape[0])


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with status {rc}")


class Oracle:
    """Thin object wrapper so tests can also load a mutated build."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # -- Section 2 / Table 1 ------------------------------------------------
    def gray(self, g: int) -> int:
        return int(self.lib.orc_gray(g))

    def flip_col(self, g: int) -> int:
        return int(self.lib.orc_flip_col(g))

    def flip_sign(self, g: int) -> int:
        return int(self.lib.orc_flip_sign(g))

    # -- Eq. (1) ------------------------------------------------------------
    def brute(self, a):
        if np.iscomplexobj(a):
            c = _cplx(a)
            out = np.zeros(4)
            _check(self.lib.orc_brute_cplx(c.shape[0], _dptr(c), _dptr(out)), "brute_cplx")
            return complex(out[0] + out[1], out[2] + out[3])
        r = _real(a)
        out = np.zeros(2)
        _check(self.lib.orc_brute_real(r.shape[0], _dptr(r), _dptr(out)), "brute_real")
        return float(out[0] + out[1])

    # -- Eq. (2) ------------------------------------------------------------
    def inclexcl(self, a):
        if np.iscomplexobj(a):
            c = _cplx(a)
            out = np.zeros(4)
            _check(self.lib.orc_inclexcl_cplx(c.shape[0], _dptr(c), _dptr(out)), "inclexcl_cplx")
            return complex(out[0] + out[1], out[2] + out[3])
        r = _real(a)
        out = np.zeros(2)
        _check(self.lib.orc_inclexcl_real(r.shape[0], _dptr(r), _dptr(out)), "inclexcl_real")
        return float(out[0] + out[1])

    # -- Algorithm 1 chunked as Algorithm 3 ---------------------------------
    def ryser(self, a, threads: int = 0, with_abs: bool = False, split: bool = False):
        """perm(A) by Gray-code Ryser in long double.

        Returns the value (float or complex); with ``with_abs`` also
        R(A) = 2 * sum_g |term_g|, the Ryser absolute sum; with ``split``
        the value is returned as the (hi, lo) double pair(s) instead.
        """
        absum = np.zeros(2)
        if np.iscomplexobj(a):
            c = _cplx(a)
            out = np.zeros(4)
            _check(self.lib.orc_ryser_cplx(c.shape[0], _dptr(c), threads, _dptr(out), _dptr(absum)),
                   "ryser_cplx")
            val = (out[0], out[1], out[2], out[3]) if split else complex(out[0] + out[1], out[2] + out[3])
        else:
            r = _real(a)
            out = np.zeros(2)
            _check(self.lib.orc_ryser_real(r.shape[0], _dptr(r), threads, _dptr(out), _dptr(absum)),
                   "ryser_real")
            val = (out[0], out[1]) if split else float(out[0] + out[1])
        if with_abs:
            return val, float(absum[0] + absum[1])
        return val

    def ryser_sample(self, a, first_chunk: int, nchunks: int, threads: int = 0) -> float:
        """Unscaled partial sum of Algorithm 1 over chunks of 4096 steps
        [first_chunk, first_chunk + nchunks) -- for timing samples only."""
        r = _real(a)
        out = np.zeros(2)
        _check(self.lib.orc_ryser_real_sample(r.shape[0], _dptr(r), threads, first_chunk, nchunks,
                                              _dptr(out)), "ryser_real_sample")
        return float(out[0] + out[1])

    CHUNK_STEPS = 4096

    def ryser_part(self, a, part: int, nparts: int, threads: int = 0, csc=None):
        """Part ``part`` of ``nparts`` of Algorithm 1's unscaled sum for a
        real matrix (dense ``a``, or ``csc = (col_ptr, row_idx, vals)`` with
        ``a`` the order n): the walk's chunks split into equal consecutive
        ranges, the g = 0 term in part 0.  Returns ((hi, lo), (abs_hi, abs_lo));
        the permanent is 2 (-1)^(n-1) times the sum over all parts."""
        out = np.zeros(2)
        absum = np.zeros(2)
        i32 = ctypes.POINTER(ctypes.c_int32)
        if csc is None:
            r = _real(a)
            n = r.shape[0]
            rc = self.lib.orc_ryser_real_part(n, _dptr(r), None, None, None, threads, part, nparts,
                                              _dptr(out), _dptr(absum))
        else:
            n = int(a)
            cp = np.ascontiguousarray(csc[0], dtype=np.int32)
            ri = np.ascontiguousarray(csc[1], dtype=np.int32)
            v = np.ascontiguousarray(csc[2], dtype=np.float64)
            if cp.size != n + 1 or ri.size != v.size:
                raise ValueError("malformed CSC")
            rc = self.lib.orc_ryser_real_part(n, None, cp.ctypes.data_as(i32), ri.ctypes.data_as(i32),
                                              _dptr(v), threads, part, nparts, _dptr(out), _dptr(absum))
        _check(rc, "ryser_real_part")
        return (float(out[0]), float(out[1])), (float(absum[0]), float(absum[1]))

    # -- Algorithm 2 ----------------------------------------------------------
    def ryser_csc(self, n: int, col_ptr, row_idx, vals, threads: int = 0,
                  with_abs: bool = False, split: bool = False):
        """perm of a real matrix given by CSC columns (Algorithm 2: a step
        updates x by the flipped column's nonzeros only), long double."""
        col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int32)
        row_idx = np.ascontiguousarray(row_idx, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        if col_ptr.size != n + 1 or row_idx.size != vals.size:
            raise ValueError("malformed CSC")
        i32 = ctypes.POINTER(ctypes.c_int32)
        out = np.zeros(2)
        absum = np.zeros(2)
        _check(self.lib.orc_ryser_csc_real(
            n, col_ptr.ctypes.data_as(i32), row_idx.ctypes.data_as(i32), _dptr(vals), threads,
            _dptr(out), _dptr(absum)), "ryser_csc_real")
        v = (out[0], out[1]) if split else float(out[0] + out[1])
        return (v, float(absum[0] + absum[1])) if with_abs else v

    def sparse(self, a, threads: int = 0, with_abs: bool = False, split: bool = False):
        """ryser_csc of the nonzeros of a dense real matrix."""
        r = _real(a)
        n = r.shape[0]
        col_ptr = np.zeros(n + 1, np.int32)
        rows, vals = [], []
        for j in range(n):
            nz = np.nonzero(r[:, j])[0]
            rows.extend(nz.tolist())
            vals.extend(r[nz, j].tolist())
            col_ptr[j + 1] = len(rows)
        return self.ryser_csc(n, col_ptr, rows, vals, threads, with_abs, split)

    # -- exact binary ---------------------------------------------------------
    def binary(self, a01, threads: int = 0, with_nonzero: bool = False):
        """Exact permanent (Python int) of a 0/1 matrix."""
        b = np.ascontiguousarray(np.asarray(a01, dtype=np.uint8))
        if b.ndim != 2 or b.shape[0] != b.shape[1] or b.max(initial=0) > 1:
            raise ValueError("square 0/1 matrix expected")
        n = b.shape[0]
        if n == 0:
            return (1, 0) if with_nonzero else 1
        limbs = np.zeros(6, np.uint64)
        nz = np.zeros(1, np.uint64)
        u8 = ctypes.POINTER(ctypes.c_ubyte)
        u64 = ctypes.POINTER(ctypes.c_uint64)
        _check(self.lib.orc_ryser_binary(n, b.ctypes.data_as(u8), threads, limbs.ctypes.data_as(u64),
                                         nz.ctypes.data_as(u64)), "ryser_binary")
        v = 0
        for k in range(5, -1, -1):
            v = (v << 64) | int(limbs[k])
        return (v, int(nz[0])) if with_nonzero else v

    def matchings(self, a01) -> int:
        b = np.ascontiguousarray(np.asarray(a01, dtype=np.uint8))
        n = b.shape[0]
        out = np.zeros(2, np.uint64)
        _check(self.lib.orc_matchings_dp(n, b.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
               "matchings_dp")
        return int(out[0]) | (int(out[1]) << 64)

    # -- gradient -------------------------------------------------------------
    def perm(self, a, threads: int = 0):
        """Best oracle value: Eq. (1) for n <= 8, else Algorithm 1."""
        n = np.asarray(a).shape[0]
        if n <= 8:
            return self.brute(a)
        return self.ryser(a, threads=threads)

    def minor(self, a, i: int, j: int, threads: int = 0):
        a = np.asarray(a)
        m = np.delete(np.delete(a, i, axis=0), j, axis=1)
        if m.shape[0] == 0:
            return 1.0 + 0j if np.iscomplexobj(a) else 1.0
        return self.perm(m, threads=threads)

    def grad_minors(self, a, threads: int = 0, entries=None):
        """dperm/da_ij = perm(A without row i and column j)."""
        a = np.asarray(a)
        n = a.shape[0]
        dt = np.complex128 if np.iscomplexobj(a) else np.float64
        if entries is None:
            g = np.zeros((n, n), dt)
            for i in range(n):
                for j in range(n):
                    g[i, j] = self.minor(a, i, j, threads)
            return g
        return np.array([self.minor(a, i, j, threads) for (i, j) in entries], dt)

    def grad_fd(self, a, i: int, j: int, h: float = 0.125, threads: int = 0):
        """(perm(A + h E_ij) - perm(A - h E_ij)) / (2h); exact for affine maps."""
        a = np.array(a, copy=True)
        ap = a.copy()
        am = a.copy()
        ap[i, j] += h
        am[i, j] -= h
        return (self.perm(ap, threads) - self.perm(am, threads)) / (2 * h)


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
