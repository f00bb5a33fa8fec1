"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments before any GPU work (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_2502_16577_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(perm_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = N.lib()
    decl = declared_symbols()
    assert decl, "no declarations found"
    for name in decl:
        assert hasattr(lib, name), name
    assert {s[0] for s in N.SIGNATURES} >= decl


def test_strerror_and_version():
    lib = N.lib()
    assert lib.perm_strerror(0) == b"success"
    assert lib.perm_strerror(N.PERM_EINVAL) == b"invalid argument"
    assert b"compilation" in lib.perm_strerror(N.PERM_ECOMPILE)
    assert lib.perm_version() >= 100


def test_workspace_query():
    lib = N.lib()
    assert lib.perm_workspace_bytes(N.KIND_DENSE_F64, 32, 0) > 0
    assert lib.perm_workspace_bytes(N.KIND_DENSE_C128, 30, 0) > lib.perm_workspace_bytes(
        N.KIND_DENSE_F64, 30, 0)
    assert lib.perm_workspace_bytes(N.KIND_DENSE_F64, 64, 0) == 0
    assert lib.perm_workspace_bytes(N.KIND_DENSE_F64, -1, 0) == 0
    assert lib.perm_workspace_bytes(999, 10, 0) == 0


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation


@pytest.mark.parametrize("fn", ["perm_dense_f64", "perm_dense_c128"])
def test_dense_argument_errors(fn):
    lib = N.lib()
    f = getattr(lib, fn)
    ws_big = 1 << 30
    assert f(-1, FAKE, 4, FAKE, FAKE, ws_big, None) == N.PERM_EINVAL
    assert f(64, FAKE, 64, FAKE, FAKE, ws_big, None) == N.PERM_EINVAL
    assert f(4, None, 4, FAKE, FAKE, ws_big, None) == N.PERM_EINVAL
    assert f(4, FAKE, 3, FAKE, FAKE, ws_big, None) == N.PERM_EINVAL
    assert f(4, FAKE, 4, None, FAKE, ws_big, None) == N.PERM_EINVAL
    assert f(20, FAKE, 20, FAKE, None, ws_big, None) == N.PERM_EWORKSPACE
    assert f(20, FAKE, 20, FAKE, FAKE, 16, None) == N.PERM_EWORKSPACE


def test_binary_argument_errors():
    import numpy as np
    lib = N.lib()
    limbs = np.zeros(5, np.uint64)
    cp = np.array([0, 1, 2], np.int32)
    ri = np.array([0, 1], np.int32)
    big = 1 << 30
    f = lib.perm_binary_exact
    assert f(-1, cp.ctypes.data, ri.ctypes.data, 2, 0, limbs.ctypes.data, None, None, FAKE, big, None) == N.PERM_EINVAL
    assert f(2, cp.ctypes.data, ri.ctypes.data, 2, 0, None, None, None, FAKE, big, None) == N.PERM_EINVAL
    assert f(2, cp.ctypes.data, ri.ctypes.data, 2, 7, limbs.ctypes.data, None, None, FAKE, big, None) == N.PERM_EINVAL
    bad_ptr = np.array([0, 2, 1], np.int32)      # not monotone / wrong end
    assert f(2, bad_ptr.ctypes.data, ri.ctypes.data, 2, 0, limbs.ctypes.data, None, None, FAKE, big, None) == N.PERM_EINVAL
    bad_rows = np.array([1, 0], np.int32)
    cp1 = np.array([0, 2, 2], np.int32)          # column 0 holds rows 1, 0: unsorted
    assert f(2, cp1.ctypes.data, bad_rows.ctypes.data, 2, 0, limbs.ctypes.data, None, None, FAKE, big, None) == N.PERM_EINVAL
    oob = np.array([0, 5], np.int32)
    assert f(2, cp.ctypes.data, oob.ctypes.data, 2, 0, limbs.ctypes.data, None, None, FAKE, big, None) == N.PERM_EINVAL
    # a full 2x2 pattern needs the workspace
    cpf = np.array([0, 2, 4], np.int32)
    rif = np.array([0, 1, 0, 1], np.int32)
    assert f(2, cpf.ctypes.data, rif.ctypes.data, 4, 0, limbs.ctypes.data, None, None, None, 0, None) == N.PERM_EWORKSPACE
    # too few primes for the bound of J_32 (32! > 2^117) -> ERANGE before any GPU work
    n = 32
    cpj = np.arange(0, n * n + 1, n, dtype=np.int32)
    rij = np.tile(np.arange(n, dtype=np.int32), n)
    assert f(n, cpj.ctypes.data, rij.ctypes.data, n * n, 1, limbs.ctypes.data, None, None, FAKE, big, None) == N.PERM_ERANGE


@pytest.mark.parametrize("n,enough", [(40, 4), (57, 6), (63, 6)])
def test_binary_prime_count_follows_the_bound(n, enough):
    # J_n: the Bregman-Minc bound is n! itself; with 50 bits per prime,
    # `enough - 1` primes are refused before any GPU work (40! ~ 2^159.2,
    # 57! ~ 2^255.9, 63! ~ 2^279.3)
    import math
    import numpy as np
    assert (enough - 1) * 50 < math.log2(math.factorial(n)) + 1 <= enough * 50
    lib = N.lib()
    limbs = np.zeros(5, np.uint64)
    used = ctypes.c_int(0)
    cp = np.arange(0, n * n + 1, n, dtype=np.int32)
    ri = np.tile(np.arange(n, dtype=np.int32), n)
    rc = lib.perm_binary_exact(n, cp.ctypes.data, ri.ctypes.data, n * n, enough - 1,
                               limbs.ctypes.data, None, ctypes.byref(used), FAKE, 1 << 30, None)
    assert rc == N.PERM_ERANGE


def test_binary_primes_are_primes_above_2_50():
    def is_prime(m):
        d, s = m - 1, 0
        while d % 2 == 0:
            d //= 2
            s += 1
        for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
            x = pow(a, d, m)
            if x in (1, m - 1):
                continue
            for _ in range(s - 1):
                x = x * x % m
                if x == m - 1:
                    break
            else:
                return False
        return True
    lib = N.lib()
    ps = [lib.perm_binary_prime(k) for k in range(6)]
    # the FP64 modular products need 2^50 < p < 2^50 + 2^40
    assert len(set(ps)) == 6 and all(2 ** 50 < p < 2 ** 50 + 2 ** 40 and is_prime(p) for p in ps)
    assert lib.perm_binary_prime(6) == 0 and lib.perm_binary_prime(-1) == 0


@pytest.mark.parametrize("name", ["perm_sparse_f64", "perm_sparse_f64_staged"])
def test_sparse_argument_errors(name):
    import numpy as np
    lib = N.lib()
    f = getattr(lib, name)
    cp = np.array([0, 1, 2], np.int32)
    ri = np.array([0, 1], np.int32)
    v = np.array([1.0, 2.0])
    big = 1 << 30
    assert f(-1, cp.ctypes.data, ri.ctypes.data, v.ctypes.data, 2, FAKE, FAKE, big, None) == N.PERM_EINVAL
    assert f(2, cp.ctypes.data, ri.ctypes.data, None, 2, FAKE, FAKE, big, None) == N.PERM_EINVAL
    assert f(2, cp.ctypes.data, ri.ctypes.data, v.ctypes.data, 3, FAKE, FAKE, big, None) == N.PERM_EINVAL
    assert f(2, cp.ctypes.data, ri.ctypes.data, v.ctypes.data, 2, None, FAKE, big, None) == N.PERM_EINVAL
    assert f(2, cp.ctypes.data, ri.ctypes.data, v.ctypes.data, 2, FAKE, None, 0, None) == N.PERM_EWORKSPACE


def test_batched_plan_errors_and_workspace():
    import ctypes
    import numpy as np
    lib = N.lib()
    h = ctypes.c_void_p()
    k = np.array([3, 33], np.int32)
    off = np.array([0, 9], np.int64)
    assert lib.perm_batched_plan_create(2, k.ctypes.data, off.ctypes.data, 1, ctypes.byref(h)) == N.PERM_EINVAL
    k = np.array([3, 0], np.int32)
    assert lib.perm_batched_plan_create(2, k.ctypes.data, off.ctypes.data, 1, ctypes.byref(h)) == N.PERM_EINVAL
    assert lib.perm_batched_plan_create(0, k.ctypes.data, off.ctypes.data, 1, ctypes.byref(h)) == N.PERM_EINVAL
    k = np.array([3, 24], np.int32)
    assert lib.perm_batched_plan_create(2, k.ctypes.data, off.ctypes.data, 1, ctypes.byref(h)) == 0
    nb = lib.perm_batched_workspace_bytes(h)
    assert nb > 0
    # too small a workspace, or a missing gradient buffer: refused before any GPU work
    assert lib.perm_batched(h, FAKE, FAKE, FAKE, 1, FAKE, nb - 1, None) == N.PERM_EWORKSPACE
    assert lib.perm_batched(h, FAKE, FAKE, None, 1, FAKE, nb, None) == N.PERM_EINVAL
    lib.perm_plan_destroy(h)


def test_real_batched_plan_errors_and_workspace():
    import ctypes
    import numpy as np
    lib = N.lib()
    k = np.array([3, 24, 32], np.int32)
    off = np.array([0, 9, 585], np.int64)
    hc, hr = ctypes.c_void_p(), ctypes.c_void_p()
    assert lib.perm_batched_plan_create(3, k.ctypes.data, off.ctypes.data, 1, ctypes.byref(hc)) == 0
    assert lib.perm_batched_plan_create_f64(3, k.ctypes.data, off.ctypes.data, 1, ctypes.byref(hr)) == 0
    nc, nr = lib.perm_batched_workspace_bytes(hc), lib.perm_batched_workspace_bytes(hr)
    # one component instead of two: about half the staging and gradient partials
    assert 0 < nr < nc
    # each plan runs only through the entry points of its own element type
    assert lib.perm_batched(hr, FAKE, FAKE, FAKE, 1, FAKE, nr, None) == N.PERM_EINVAL
    assert lib.perm_batched_autotune(hr, FAKE, FAKE, FAKE, FAKE, nr, None, None) == N.PERM_EINVAL
    assert lib.perm_batched_f64(hc, FAKE, FAKE, FAKE, 1, FAKE, nc, None) == N.PERM_EINVAL
    assert lib.perm_batched_autotune_f64(hc, FAKE, FAKE, FAKE, FAKE, nc, None, None) == N.PERM_EINVAL
    assert lib.perm_batched_f64(hr, FAKE, FAKE, FAKE, 1, FAKE, nr - 1, None) == N.PERM_EWORKSPACE
    assert lib.perm_batched_f64(hr, FAKE, FAKE, None, 1, FAKE, nr, None) == N.PERM_EINVAL
    k[1] = 33
    h = ctypes.c_void_p()
    assert lib.perm_batched_plan_create_f64(3, k.ctypes.data, off.ctypes.data, 0, ctypes.byref(h)) == N.PERM_EINVAL
    assert lib.perm_weighted_sum_f64(0, FAKE, FAKE, FAKE, None) == N.PERM_EINVAL
    assert lib.perm_weighted_sum_f64(2, FAKE, None, FAKE, None) == N.PERM_EINVAL
    lib.perm_plan_destroy(hc)
    lib.perm_plan_destroy(hr)


def test_dense_ex_option_errors():
    import ctypes
    from paper_2502_16577_amd.api import PermOptions
    lib = N.lib()
    big = 1 << 30
    bad = PermOptions(7, 0, 0, 0)
    assert lib.perm_dense_f64_ex(20, FAKE, 20, ctypes.byref(bad), FAKE, FAKE, big, None) == N.PERM_EINVAL
    bad = PermOptions(0, -1, 0, 0)
    assert lib.perm_dense_f64_ex(20, FAKE, 20, ctypes.byref(bad), FAKE, FAKE, big, None) == N.PERM_EINVAL
    bad = PermOptions(0, 0, -5, 0)
    assert lib.perm_dense_f64_ex(20, FAKE, 20, ctypes.byref(bad), FAKE, FAKE, big, None) == N.PERM_EINVAL
    bad = PermOptions(0, 0, 0, -1)
    assert lib.perm_dense_f64_ex(20, FAKE, 20, ctypes.byref(bad), FAKE, FAKE, big, None) == N.PERM_EINVAL
    ok = PermOptions(1, 4, 1 << 20, 12)
    assert lib.perm_dense_f64_ex(20, FAKE, 20, ctypes.byref(ok), FAKE, None, 0, None) == N.PERM_EWORKSPACE
    # the extended-precision walk: orders 13..48 only (checked before the
    # workspace), n = 0 is the empty product as in every mode
    ext = PermOptions(3, 0, 0, 0)
    for n in (12, 49, 63):
        assert lib.perm_dense_f64_ex(n, FAKE, n, ctypes.byref(ext), FAKE, FAKE, big, None) == N.PERM_EUNSUPPORTED
    for n in (13, 48):
        assert lib.perm_dense_f64_ex(n, FAKE, n, ctypes.byref(ext), FAKE, None, 0, None) == N.PERM_EWORKSPACE
    assert lib.perm_dense_f64_launches(40, ctypes.byref(ext)) == 1
    bad = PermOptions(4, 0, 0, 0)
    assert lib.perm_dense_f64_ex(20, FAKE, 20, ctypes.byref(bad), FAKE, FAKE, big, None) == N.PERM_EINVAL
    # the complex sweep: two-sum (default) and extended (orders 13..32) only
    f = lib.perm_dense_c128_ex
    for opt, want in ((PermOptions(1, 0, 0, 0), N.PERM_EUNSUPPORTED),
                      (PermOptions(2, 0, 0, 0), N.PERM_EUNSUPPORTED),
                      (PermOptions(0, 5, 0, 0), N.PERM_EUNSUPPORTED),
                      (PermOptions(3, 0, 1 << 20, 0), N.PERM_EUNSUPPORTED),
                      (PermOptions(3, 0, 0, 12), N.PERM_EUNSUPPORTED),
                      (PermOptions(5, 0, 0, 0), N.PERM_EINVAL),
                      (PermOptions(3, -1, 0, 0), N.PERM_EINVAL)):
        assert f(20, FAKE, 20, ctypes.byref(opt), FAKE, FAKE, big, None) == want, (opt.accumulation,)
    for n in (12, 33):
        assert f(n, FAKE, n, ctypes.byref(ext), FAKE, FAKE, big, None) == N.PERM_EUNSUPPORTED
    for n in (13, 32):
        assert f(n, FAKE, n, ctypes.byref(ext), FAKE, None, 0, None) == N.PERM_EWORKSPACE
    assert f(20, FAKE, 20, None, FAKE, None, 0, None) == N.PERM_EWORKSPACE
    assert f(20, FAKE, 19, ctypes.byref(ext), FAKE, FAKE, big, None) == N.PERM_EINVAL
    # launch ranges: n = 26 (2^18 lanes of 128 steps) with 16-step re-seeds and
    # at most 2^22 subset-steps per launch is 8 launches; a range starting at
    # or beyond the last, or a negative field, is refused before any GPU work
    split = PermOptions(0, 4, 1 << 22, 0)
    assert lib.perm_dense_f64_launches(26, ctypes.byref(split)) == 8
    assert lib.perm_dense_f64_launches(26, None) == 1
    assert lib.perm_dense_f64_launches(8, ctypes.byref(split)) == 1
    assert lib.perm_dense_f64_launches(-1, None) == N.PERM_EINVAL
    beyond = PermOptions(0, 4, 1 << 22, 0, 8, 1)
    assert lib.perm_dense_f64_ex(26, FAKE, 26, ctypes.byref(beyond), FAKE, FAKE, big, None) == N.PERM_EINVAL
    for neg in (PermOptions(0, 4, 1 << 22, 0, -1, 0), PermOptions(0, 4, 1 << 22, 0, 0, -1)):
        assert lib.perm_dense_f64_ex(26, FAKE, 26, ctypes.byref(neg), FAKE, FAKE, big, None) == N.PERM_EINVAL
        assert lib.perm_dense_f64_launches(26, ctypes.byref(neg)) == N.PERM_EINVAL


def test_binary_empty_matrix_on_the_host():
    # n = 0: permanent 1 (the empty product), decided before any GPU work
    import numpy as np
    lib = N.lib()
    limbs = np.zeros(5, np.uint64)
    res = np.zeros(6, np.uint64)
    used = ctypes.c_int(0)
    cp = np.zeros(1, np.int32)
    assert lib.perm_binary_exact(0, cp.ctypes.data, None, 0, 0, limbs.ctypes.data, res.ctypes.data,
                                 ctypes.byref(used), None, 0, None) == N.PERM_OK
    assert list(limbs) == [1, 0, 0, 0, 0] and used.value == 3 and list(res[:3]) == [1, 1, 1]
