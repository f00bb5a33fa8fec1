"""Section 4 preprocessing (host): Dulmage-Mendelsohn pruning and the
Forbert-Marx decomposition of Algorithm 4, checked against the oracle."""
import numpy as np
import pytest

from paper_2502_16577_amd import api
from paper_2502_16577_amd import workloads as W


def test_forbert_marx_identity(oracle):
    # Eq. (expand): perm([a b c; d e B]) = perm([0 0 c; d e B]) + perm([a e + b d, B])
    rng = np.random.default_rng(3)
    for n in (3, 4, 6, 7):
        A = rng.standard_normal((n, n))
        Z = A.copy()
        Z[0, 0] = Z[0, 1] = 0.0
        M = np.column_stack([A[0, 0] * A[1:, 1] + A[0, 1] * A[1:, 0], A[1:, 2:]])
        assert abs(oracle.brute(A) - (oracle.brute(Z) + oracle.brute(M))) <= 1e-12 * oracle.brute(np.abs(A))


def weighted(oracle, leaves):
    return sum(w * (oracle.perm(m) if m.shape[0] else 1.0) for w, m in leaves)


def test_dm_removes_offdiagonal_of_triangular(oracle):
    # Section 4.1: for a lower-triangular matrix the pruning leaves only the diagonal
    n = 12
    rng = np.random.default_rng(4)
    A = np.tril(rng.random((n, n)) + 0.1)
    cp, ri, v = W.to_csc(A)
    leaves, removed = api.decompose(n, cp, ri, v, flags=api.DECOMP_DM)
    assert removed == int(np.count_nonzero(A)) - n
    (w, m), = leaves
    assert np.count_nonzero(m) == n
    assert abs(weighted(oracle, leaves) - np.prod(np.diag(A))) <= 1e-12 * np.prod(np.diag(A))


def test_no_perfect_matching_gives_no_leaves():
    A = np.eye(6)
    A[2, 2] = 0.0
    A[2, 3] = 1.0   # rows 2 and 3 both only in column 3
    cp, ri, v = W.to_csc(A)
    leaves, _ = api.decompose(6, cp, ri, v)
    assert leaves == []


@pytest.mark.parametrize("n,per_row,seed", [(10, 2, 1), (12, 3, 2), (14, 4, 3), (16, 3, 4),
                                            (18, 5, 5), (16, 6, 6)])
def test_decomposition_preserves_perm(oracle, n, per_row, seed):
    pat = W.sparse_rows(n, per_row, seed).astype(np.float64)
    A = pat * (np.random.default_rng(seed).random((n, n)) + 0.25)
    cp, ri, v = W.to_csc(A)
    # R(A) bounds the oracle's own rounding (some of these patterns have no
    # perfect matching: perm = 0 exactly, the oracle returns rounding noise)
    want, r = oracle.ryser(A, with_abs=True)
    for flags in (api.DECOMP_DM, api.DECOMP_FM, api.DECOMP_DM | api.DECOMP_FM):
        leaves, _ = api.decompose(n, cp, ri, v, flags=flags)
        got = weighted(oracle, leaves)
        assert abs(got - want) <= 1e-11 * abs(want) + 1e-15 * r, (flags, got, want)
        if flags & api.DECOMP_FM:
            # after the decomposition no leaf has a row or column with <= 4 nonzeros
            for _, m in leaves:
                if m.shape[0] > 1:
                    assert (np.count_nonzero(m, axis=0).min() > 4 and np.count_nonzero(m, axis=1).min() > 4)


def test_decomposition_of_signed_values(oracle):
    n = 15
    pat = W.sparse_rows(n, 4, 21).astype(np.float64)
    A = pat * np.random.default_rng(22).standard_normal((n, n))
    cp, ri, v = W.to_csc(A)
    leaves, _ = api.decompose(n, cp, ri, v)
    want, r = oracle.ryser(A, with_abs=True)
    assert abs(weighted(oracle, leaves) - want) <= 1e-12 * r


@pytest.mark.parametrize("n,per_row,seed", [(12, 3, 2), (16, 3, 4), (18, 5, 5), (24, 4, 7)])
def test_folded_leaves_preserve_perm(oracle, n, per_row, seed):
    # leaves of order 0, 1 and 2 summed on the host (two order-0 leaves carry
    # the double-double sum); no stored leaf of order <= 2 remains
    pat = W.sparse_rows(n, per_row, seed).astype(np.float64)
    A = pat * (np.random.default_rng(seed).random((n, n)) - 0.3)
    cp, ri, v = W.to_csc(A)
    want, r = oracle.ryser(A, with_abs=True)
    plain, _ = api.decompose(n, cp, ri, v)
    folded, _ = api.decompose(n, cp, ri, v, flags=api.DECOMP_DM | api.DECOMP_FM | api.DECOMP_FOLD)
    assert all(m.shape[0] > 2 for w, m in folded if m.shape[0] != 0)
    assert sum(1 for _, m in folded if m.shape[0] == 0) <= 2
    assert len(folded) <= len(plain)
    assert abs(weighted(oracle, folded) - want) <= 1e-11 * abs(want) + 1e-14 * r
    assert abs(weighted(oracle, folded) - weighted(oracle, plain)) <= 1e-14 * r


def test_folding_a_fully_reducible_matrix(oracle):
    # a tridiagonal matrix reduces completely (every row has <= 3 nonzeros):
    # with folding there are no stored leaves at all
    n = 20
    rng = np.random.default_rng(9)
    A = np.diag(rng.random(n) + 0.5) + np.diag(rng.random(n - 1), 1) + np.diag(rng.random(n - 1), -1)
    cp, ri, v = W.to_csc(A)
    leaves, _ = api.decompose(n, cp, ri, v, flags=api.DECOMP_DM | api.DECOMP_FM | api.DECOMP_FOLD)
    assert all(m.shape[0] == 0 for _, m in leaves)
    want = oracle.ryser(A)
    assert abs(weighted(oracle, leaves) - want) <= 1e-13 * abs(want)
