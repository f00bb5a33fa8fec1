"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and arranges them into matrices; it
holds none of the permanent method's arithmetic.  All draws use
``numpy.random.default_rng(seed)`` (PCG64), and the unitary generator uses
its own Householder QR written with element-wise numpy operations and
numpy's own reductions (no BLAS/LAPACK), so the same seed gives bit-identical
matrices on every x86-64 host with this numpy.

Workload families (the paper benchmarks "randomly generated" dense matrices,
Section 6, and SuiteSparse matrices; the synthetic families below stand in for
them):

* ``uniform(n, seed)``      entries i.i.d. U[0, 1)
* ``rademacher(n, seed)``   entries i.i.d. +-1
* ``bernoulli(n, seed)``    0/1 entries, P(1) = 1/2
* ``haar_unitary(m, seed)`` Haar-random m x m unitary: complex Gaussian
  Z = (X + iY)/sqrt(2), Z = QR, U = Q diag(R_ii / |R_ii|)
* ``haar_block(m, k, seed)`` top-left k x k block of such a unitary
* ``sparse_rows(n, per_row, seed)`` 0/1 matrix with exactly ``per_row``
  distinct random columns per row; the whole matrix is redrawn from the same
  stream until no column is empty
* ``batched_submatrices(...)`` ``count`` complex k x k matrices, k uniform in
  [kmin, kmax], each made of k rows and k columns (drawn with repetition) of
  one Haar unitary -- the shape of photon-counting amplitudes
* ``all_ones(n)``, ``ones_minus_identity(n)``, ``tridiagonal_ones(n)``,
  ``block_ones(n, b)``: closed-form families.
"""
from __future__ import annotations

import hashlib

import numpy as np

# Seeds of the benchmark configurations.
SEED_U20 = 16577
SEED_U32 = 16578
SEED_RADEMACHER32 = 16579
SEED_BERNOULLI32 = 16580
SEED_HAAR120 = 16581
SEED_SPARSE40 = 16582
SEED_HAAR64 = 16583
SEED_BATCH = 16584
# values of the sparse 40 x 40 pattern when it is run as a real matrix
SEED_SPARSE40_VALUES = 16585


def uniform(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random((n, n))


def rademacher(n: int, seed: int) -> np.ndarray:
    r = np.random.default_rng(seed).integers(0, 2, size=(n, n))
    return (2 * r - 1).astype(np.float64)


def bernoulli(n: int, seed: int, p: float = 0.5) -> np.ndarray:
    return (np.random.default_rng(seed).random((n, n)) < p).astype(np.uint8)


def _householder_qr(z: np.ndarray):
    """Plain Householder QR of a square complex matrix.  Returns (Q, R)."""
    a = np.array(z, dtype=np.complex128, copy=True)
    m = a.shape[0]
    vs = []
    for k in range(m):
        x = a[k:, k].copy()
        nx = np.sqrt(np.sum(x.real * x.real + x.imag * x.imag))
        if nx == 0.0:
            vs.append(None)
            continue
        x0 = x[0]
        phase = x0 / abs(x0) if x0 != 0 else 1.0 + 0j
        v = x.copy()
        v[0] = x0 + phase * nx
        nv = np.sqrt(np.sum(v.real * v.real + v.imag * v.imag))
        v = v / nv
        # a[k:, k:] -= 2 v (v^H a[k:, k:])
        w = np.sum(np.conj(v)[:, None] * a[k:, k:], axis=0)
        a[k:, k:] = a[k:, k:] - 2.0 * v[:, None] * w[None, :]
        vs.append(v)
    r = np.triu(a)
    q = np.eye(m, dtype=np.complex128)
    for k in range(m - 1, -1, -1):
        v = vs[k]
        if v is None:
            continue
        w = np.sum(np.conj(v)[:, None] * q[k:, :], axis=0)
        q[k:, :] = q[k:, :] - 2.0 * v[:, None] * w[None, :]
    return q, r


def haar_unitary(m: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((m, m))
    y = rng.standard_normal((m, m))
    z = (x + 1j * y) / np.sqrt(2.0)
    q, r = _householder_qr(z)
    d = np.diag(r)
    ph = d / np.abs(d)
    return q * ph[None, :]


def haar_block(m: int, k: int, seed: int) -> np.ndarray:
    return np.ascontiguousarray(haar_unitary(m, seed)[:k, :k])


def sparse_rows(n: int, per_row: int, seed: int, max_draws: int = 10000) -> np.ndarray:
    rng = np.random.default_rng(seed)
    for _ in range(max_draws):
        a = np.zeros((n, n), np.uint8)
        for i in range(n):
            a[i, rng.choice(n, size=per_row, replace=False)] = 1
        if a.sum(axis=0).min() >= 1:
            return a
    raise RuntimeError("could not draw a matrix without empty columns")


def batched_submatrices(count: int = 4096, kmin: int = 8, kmax: int = 24, m: int = 64,
                        seed_unitary: int = SEED_HAAR64, seed_select: int = SEED_BATCH):
    """Returns a list of ``count`` complex k x k matrices (k in [kmin, kmax])."""
    u = haar_unitary(m, seed_unitary)
    rng = np.random.default_rng(seed_select)
    mats = []
    for _ in range(count):
        k = int(rng.integers(kmin, kmax + 1))
        rows = rng.integers(0, m, size=k)
        cols = rng.integers(0, m, size=k)
        mats.append(np.ascontiguousarray(u[rows][:, cols]))
    return mats


def pack(mats):
    """Packs square matrices into (k int32[count], offset int64[count], data)."""
    ks = np.array([a.shape[0] for a in mats], np.int32)
    offs = np.zeros(len(mats), np.int64)
    if len(mats) > 1:
        offs[1:] = np.cumsum((ks.astype(np.int64) ** 2))[:-1]
    dt = np.complex128 if any(np.iscomplexobj(a) for a in mats) else np.float64
    data = np.concatenate([np.asarray(a, dt).ravel() for a in mats]) if mats else np.zeros(0, dt)
    return ks, offs, data


def all_ones(n: int) -> np.ndarray:
    return np.ones((n, n))


def ones_minus_identity(n: int) -> np.ndarray:
    return np.ones((n, n)) - np.eye(n)


def tridiagonal_ones(n: int) -> np.ndarray:
    a = np.eye(n)
    for i in range(n - 1):
        a[i, i + 1] = 1.0
        a[i + 1, i] = 1.0
    return a


def block_ones(n: int, b: int) -> np.ndarray:
    a = np.zeros((n, n))
    for s in range(0, n, b):
        a[s:s + b, s:s + b] = 1.0
    return a


def scaling_vectors(n: int, seed: int):
    """Two vectors d, e of n entries uniform in [0.5, 1.5) (row and column
    scalings of a test pattern)."""
    rng = np.random.default_rng(seed)
    return rng.random(n) + 0.5, rng.random(n) + 0.5


def to_csc(a):
    """CSC (col_ptr int32[n+1], row_idx int32[nnz], vals float64[nnz]) of a dense matrix."""
    a = np.asarray(a)
    n = a.shape[0]
    col_ptr = np.zeros(n + 1, np.int32)
    rows, vals = [], []
    for j in range(n):
        nz = np.nonzero(a[:, j])[0]
        rows.extend(nz.tolist())
        vals.extend(a[nz, j].tolist())
        col_ptr[j + 1] = len(rows)
    return col_ptr, np.array(rows, np.int32), np.array(vals, np.float64)


def digest(a) -> str:
    """sha256 of the matrix bytes (dtype and shape included)."""
    a = np.ascontiguousarray(a)
    h = hashlib.sha256()
    h.update(str(a.dtype).encode())
    h.update(str(a.shape).encode())
    h.update(a.tobytes())
    return h.hexdigest()
