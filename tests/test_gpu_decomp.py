"""The Section 4 pipeline on the GPU: host decomposition, one batched launch
over the leaves, weighted double-double sum."""
import json
import os

import numpy as np
import pytest

from paper_2502_16577_amd import api
from paper_2502_16577_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_size.json")


@pytest.mark.parametrize("n,per_row,seed", [(16, 3, 1), (20, 4, 2), (24, 5, 3), (26, 6, 4)])
def test_sparse_decomp_matches_oracle(oracle, n, per_row, seed):
    pat = W.sparse_rows(n, per_row, seed).astype(np.float64)
    A = pat * (np.random.default_rng(seed).random((n, n)) + 0.25)
    cp, ri, v = W.to_csc(A)
    want, r = oracle.ryser(A, with_abs=True)
    got = api.perm_sparse_decomp(n, cp, ri, v).item()
    assert abs(got - want) <= 1e-10 * abs(want) + 1e-15 * r, (got, want)


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
