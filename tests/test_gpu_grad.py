"""Parity of the adjoint (perm_grad, autograd) with the oracle's minors and
finite differences.

Gradient tolerances: |G - minors| <= 1e-10 * perm(|minor|) entrywise (the
scale used for signed / complex permanents; relative 1e-10 for positive
entries); instead of an R-based gate on each entry, Laplace's identity
sum_j a_ij G_ij = perm(A) is checked on every row and column.
Finite differences: max |G - FD| <= 1e-6 * max |FD| (FD from the oracle,
exact for an affine map up to rounding).
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_2502_16577_amd import api
from paper_2502_16577_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def gpu_grad(a):
    p, g = api.perm_grad(torch.from_numpy(np.ascontiguousarray(a)).to(DEV))
    return p.cpu().numpy().item(), g.cpu().numpy()


def minor_scale(oracle, a, i, j):
    m = np.delete(np.delete(np.abs(a), i, 0), j, 1)
    return oracle.perm(m) if m.size else 1.0


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10, 11, 12, 13, 14])
def test_real_full_minors(oracle, n):
    a = W.uniform(n, 1200 + n)
    p, g = gpu_grad(a)
    want = oracle.grad_minors(a)
    assert abs(p - oracle.perm(a)) <= 1e-10 * abs(oracle.perm(a))
    assert np.all(np.abs(g - want) <= 1e-10 * np.abs(want) + 1e-300), (n, np.max(np.abs(g - want) / np.abs(want)))


@pytest.mark.parametrize("n", [1, 4, 9, 11, 13, 16])
def test_complex_full_minors(oracle, n):
    a = W.haar_block(2 * n + 2, n, 1300 + n)
    p, g = gpu_grad(a)
    want = oracle.grad_minors(a)
    for i in range(n):
        for j in range(n):
            assert abs(g[i, j] - want[i, j]) <= 1e-10 * minor_scale(oracle, a, i, j), (i, j)
    assert abs(p - oracle.perm(a)) <= 1e-10 * oracle.perm(np.abs(a))


@pytest.mark.parametrize("n,cplx", [(20, False), (24, False), (22, True), (24, True)])
def test_sampled_minors_and_laplace(oracle, n, cplx):
    a = W.haar_block(2 * n, n, 1400 + n) if cplx else np.random.default_rng(1400 + n).standard_normal((n, n))
    p, g = gpu_grad(a)
    rng = np.random.default_rng(n)
    for _ in range(3):
        i, j = int(rng.integers(n)), int(rng.integers(n))
        want = oracle.minor(a, i, j)
        assert abs(g[i, j] - want) <= 1e-10 * minor_scale(oracle, a, i, j), (i, j, g[i, j], want)
    pref, rsum = oracle.ryser(a, with_abs=True)
    # Laplace expansion along every row and column reproduces the permanent
    for i in range(n):
        assert abs(np.dot(a[i], g[i]) - pref) <= 1e-12 * rsum
        assert abs(np.dot(a[:, i], g[:, i]) - pref) <= 1e-12 * rsum
    assert abs(np.sum(a * g) - n * pref) <= 1e-11 * rsum


def test_fd(oracle):
    n = 12
    a = W.haar_block(30, n, 1500)
    _, g = gpu_grad(a)
    fd = np.array([[oracle.grad_fd(a, i, j) for j in range(n)] for i in range(n)])
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_perm_matches_forward_kernel():
    a = W.uniform(22, 3)
    A = torch.from_numpy(a).to(DEV)
    p, _ = api.perm_grad(A)
    q = api.perm_dense_f64(A)
    assert abs(p.item() - q.item()) <= 1e-12 * abs(q.item())


@pytest.mark.parametrize("dtype", [torch.float64, torch.complex128])
@pytest.mark.parametrize("n", [4, 12])
def test_autograd_gradcheck(dtype, n):
    g = torch.Generator().manual_seed(n)
    A = torch.randn(n, n, dtype=dtype, generator=g).to(DEV).requires_grad_(True)
    assert torch.autograd.gradcheck(api.permanent, (A,), eps=1e-6, atol=1e-7, rtol=1e-6)


def test_autograd_backward_value():
    a = W.uniform(13, 7)
    A = torch.from_numpy(a).to(DEV).requires_grad_(True)
    p = api.permanent(A)
    (3.0 * p).backward()
    _, g = api.perm_grad(A.detach())
    assert torch.allclose(A.grad, 3.0 * g, rtol=0, atol=0)


def test_largest_order_real(oracle):
    # n = 32, the largest order perm_grad takes (2^31 subsets), on the 32 x 32
    # U[0,1) input whose permanent the oracle value in tests/golden holds: the
    # permanent against it, one sampled minor from the oracle (a 31 x 31 sweep
    # on the host), and Laplace's identity on every row and column, which ties
    # all n^2 entries to the permanent
    with open(os.path.join(os.path.dirname(__file__), "golden", "full_size.json")) as f:
        gold = json.load(f)["u32"]
    n = 32
    a = W.uniform(n, W.SEED_U32)
    assert W.digest(a) == gold["digest"]
    want = gold["value"][0] + gold["value"][1]
    p, g = gpu_grad(a)
    assert abs(p - want) <= 1e-10 * want, (p, want)
    i, j = 5, 27
    m = oracle.minor(a, i, j)
    assert abs(g[i, j] - m) <= 1e-10 * m, (g[i, j], m)
    for k in range(n):
        assert abs(np.dot(a[k], g[k]) - want) <= 1e-10 * want, k
        assert abs(np.dot(a[:, k], g[:, k]) - want) <= 1e-10 * want, k


def test_empty_matrix():
    # perm of the 0 x 0 matrix is 1; its gradient has no entries
    for dtype in (torch.float64, torch.complex128):
        p, g = api.perm_grad(torch.zeros((0, 0), dtype=dtype, device=DEV))
        assert p.item() == 1 and g.shape == (0, 0)
