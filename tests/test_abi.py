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
