"""Parity of perm_sparse_f64 (CSC input) with the oracle's SpaRyser and Ryser."""
import numpy as np
import pytest

from paper_2502_16577_amd import api
from paper_2502_16577_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,per_row", [(1, 1), (5, 2), (13, 3), (17, 4), (22, 6), (26, 6)])
def test_sparse_uniform_values(oracle, n, per_row):
    pat = W.sparse_rows(n, per_row, 1000 + n).astype(np.float64)
    a = pat * W.uniform(n, 1100 + n)
    cp, ri, v = W.to_csc(a)
    got = api.perm_sparse_f64(n, cp, ri, v).item()
    want = oracle.ryser(a)
    assert abs(got - want) <= 1e-10 * abs(want), (got, want)
    if n <= 22:
        assert abs(oracle.sparse(a) - want) <= 1e-12 * abs(want)


def test_sparse_signed_values(oracle):
    n = 24
    pat = W.sparse_rows(n, 5, 77).astype(np.float64)
    a = pat * np.random.default_rng(78).standard_normal((n, n))
    cp, ri, v = W.to_csc(a)
    got = api.perm_sparse_f64(n, cp, ri, v).item()
    want, r = oracle.ryser(a, with_abs=True)
    assert abs(got - want) <= 1e-10 * oracle.ryser(np.abs(a))
    assert abs(got - want) <= 1e-13 * r


def test_sparse_matches_dense_bitwise():
    import torch
    n = 25
    a = W.sparse_rows(n, 6, 5).astype(np.float64) * W.uniform(n, 6)
    cp, ri, v = W.to_csc(a)
    s = api.perm_sparse_f64(n, cp, ri, v).item()
    d = api.perm_dense_f64(torch.from_numpy(a).to("cuda:0")).item()
    assert s == d


# Generated, pattern-specific kernels (hiprtc): parity with the oracle on
# sparse patterns of several densities, signed values, and the 40x40 input.
@pytest.mark.parametrize("n,per_row", [(14, 2), (14, 3), (17, 3), (21, 4), (24, 6)])
def test_generated_kernel_uniform_values(oracle, n, per_row):
    pat = W.sparse_rows(n, per_row, 2000 + n).astype(np.float64)
    a = pat * W.uniform(n, 2100 + n)
    cp, ri, v = W.to_csc(a)
    got = api.perm_sparse_f64_gen(n, cp, ri, v).item()
    want, r = oracle.ryser(a, with_abs=True)
    # relative 1e-10, with R(A) as the scale where the permanent cancels to 0
    assert abs(got - want) <= 1e-10 * abs(want) + 1e-13 * r, (n, got, want, r)


def test_generated_kernel_signed_values_and_pattern_reuse(oracle):
    # two matrices with one pattern: the second call reuses the compiled module
    n = 22
    pat = W.sparse_rows(n, 5, 91).astype(np.float64)
    for seed in (92, 93):
        a = pat * np.random.default_rng(seed).standard_normal((n, n))
        cp, ri, v = W.to_csc(a)
        got = api.perm_sparse_f64_gen(n, cp, ri, v).item()
        want, r = oracle.ryser(a, with_abs=True)
        assert abs(got - want) <= 1e-10 * oracle.ryser(np.abs(a))
        assert abs(got - want) <= 1e-13 * r, (seed, got, want, r)


def test_generated_kernel_small_and_dense_patterns(oracle):
    # below the generated path's minimum order the staged sweep runs; a fully
    # dense pattern is a valid (if pointless) input
    for n, a in ((9, W.uniform(9, 94)), (15, W.uniform(15, 95))):
        cp, ri, v = W.to_csc(a)
        got = api.perm_sparse_f64_gen(n, cp, ri, v).item()
        want = oracle.ryser(a)
        assert abs(got - want) <= 1e-10 * abs(want), (n, got, want)


def test_generated_kernel_full_size_sparse40():
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "full_size.json")))["sparse40"]
    a = W.sparse_rows(40, 6, W.SEED_SPARSE40)
    assert W.digest(a) == g["digest"]
    cp, ri, v = W.to_csc(a.astype(np.float64))
    got = api.perm_sparse_f64_gen(40, cp, ri, v).item()
    want = float(g["value"])
    assert abs(got - want) <= 1e-10 * want, (got, want)
