"""perm_dense_f64_noalloc (the allocation-free entry point) against
perm_dense_f64 through the C ABI: two calls in a row on the same GPU, the
second on a smaller matrix, each bit for bit equal to the entry point that
takes a caller workspace (same kernels, same launch plan), and the n = 20
result against the stored oracle value."""
import ctypes
import json
import os

import numpy as np
import pytest
import torch

from paper_2502_16577_amd import _native as N
from paper_2502_16577_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_size.json")


def _noalloc(A, out):
    st = torch.cuda.current_stream(DEV).cuda_stream
    return N.lib().perm_dense_f64_noalloc(A.shape[0], A.data_ptr(), A.stride(0), out.data_ptr(), st)


def _with_ws(A, out):
    n = A.shape[0]
    need = N.lib().perm_workspace_bytes(N.KIND_DENSE_F64, n, 0)
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    st = torch.cuda.current_stream(DEV).cuda_stream
    rc = N.lib().perm_dense_f64(n, A.data_ptr(), A.stride(0), out.data_ptr(), ws.data_ptr(), need, st)
    torch.cuda.synchronize()
    return rc


def test_noalloc_matches_workspace_entry_point_twice():
    with open(GOLDEN) as f:
        golden = json.load(f)
    cases = [("u32", W.uniform(32, W.SEED_U32)), ("u20", W.uniform(20, W.SEED_U20))]
    for name, a in cases:  # the second call is the smaller input
        assert W.digest(a) == golden[name]["digest"]
        A = torch.from_numpy(a).to(DEV)
        got = torch.full((), -1.0, dtype=torch.float64, device=DEV)
        ref = torch.full((), -2.0, dtype=torch.float64, device=DEV)
        assert _noalloc(A, got) == N.PERM_OK
        torch.cuda.synchronize()
        assert _with_ws(A, ref) == N.PERM_OK
        assert got.item() == ref.item(), (name, got.item(), ref.item())
        want = sum(golden[name]["value"])
        assert abs(got.item() - want) <= 1e-10 * abs(want), (name, got.item(), want)


def test_noalloc_rejects_orders_beyond_its_scratch():
    A = torch.zeros((1, 1), dtype=torch.float64, device=DEV)
    out = torch.empty((), dtype=torch.float64, device=DEV)
    limit = N.lib().perm_noalloc_scratch_bytes()
    for n in (54, 63):
        assert N.lib().perm_workspace_bytes(N.KIND_DENSE_F64, n, 0) > limit
        st = N.lib().perm_dense_f64_noalloc(n, A.data_ptr(), n, out.data_ptr(), None)
        assert st == N.PERM_ESCRATCH
    assert N.lib().perm_workspace_bytes(N.KIND_DENSE_F64, 53, 0) <= limit
