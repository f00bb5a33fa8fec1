"""The Section 4 pipeline on the GPU: host decomposition, one batched launch
over the leaves, weighted double-double sum."""
import json
import os

import numpy as np
import pytest

from paper_2502_16577_amd import api
from paper_2502_16577_amd import workloads as W

pytestmark = pytest.mark.gpu


def scaled_perm(d, e, perm_pattern):
    """perm(D P E) = prod d prod e perm(P), in exact rational arithmetic."""
    from fractions import Fraction
    s = Fraction(perm_pattern)
    for v in list(d) + list(e):
        s *= Fraction(float(v))
    return float(s)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_size.json")


@pytest.mark.parametrize("n,per_row,seed", [(16, 3, 1), (20, 4, 2), (24, 5, 3), (26, 6, 4)])
def test_sparse_decomp_matches_oracle(oracle, n, per_row, seed):
    pat = W.sparse_rows(n, per_row, seed).astype(np.float64)
    A = pat * (np.random.default_rng(seed).random((n, n)) + 0.25)
    cp, ri, v = W.to_csc(A)
    want, r = oracle.ryser(A, with_abs=True)
    got = api.perm_sparse_decomp(n, cp, ri, v).item()
    assert abs(got - want) <= 1e-10 * abs(want) + 1e-15 * r, (got, want)


@pytest.mark.parametrize("dense_min", [2, 12, 33])
@pytest.mark.parametrize("fold", [False, True])
def test_leaf_routing_and_folding(oracle, dense_min, fold):
    # every leaf on the batched launch (dense_min 33), every leaf of order >= 2
    # as its own real sweep (dense_min 2), and a mix; leaves of order <= 2
    # summed on the host or not
    n = 24
    pat = W.sparse_rows(n, 4, 41).astype(np.float64)
    A = pat * (np.random.default_rng(42).random((n, n)) - 0.2)
    cp, ri, v = W.to_csc(A)
    want, r = oracle.ryser(A, with_abs=True)
    flags = api.DECOMP_DM | api.DECOMP_FM | (api.DECOMP_FOLD if fold else 0)
    got = api.perm_sparse_decomp(n, cp, ri, v, flags=flags, dense_min=dense_min).item()
    assert abs(got - want) <= 1e-13 * r, (got, want, r)


def test_sparse40_through_decomposition():
    # the 40x40 0/1 matrix with 6 nonzeros per row: exact value from the oracle
    with open(GOLDEN) as f:
        g = json.load(f)["sparse40"]
    a = W.sparse_rows(40, 6, W.SEED_SPARSE40)
    assert W.digest(a) == g["digest"]
    cp, ri, v = W.to_csc(a.astype(np.float64))
    got = api.perm_sparse_decomp(40, cp, ri, v).item()
    want = int(g["value"])
    assert abs(got - want) <= 1e-10 * want, (got, want)


def test_sparse40_scaled_values_through_decomposition():
    # entries d_i e_j on the same pattern: perm = prod d prod e perm(pattern),
    # with the pattern's exact value from the oracle
    with open(GOLDEN) as f:
        g = json.load(f)["sparse40"]
    a = W.sparse_rows(40, 6, W.SEED_SPARSE40).astype(np.float64)
    d, e = W.scaling_vectors(40, 7040)
    cp, ri, v = W.to_csc(a * np.outer(d, e))
    got = api.perm_sparse_decomp(40, cp, ri, v).item()
    want = scaled_perm(d, e, int(g["value"]))
    assert abs(got - want) <= 1e-10 * want, (got, want)
