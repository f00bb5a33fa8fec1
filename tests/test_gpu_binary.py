"""Bit-exact parity of the binary (modular + CRT) HIP path with the oracle."""
import json
import math
import os

import numpy as np
import pytest

from paper_2502_16577_amd import api
from paper_2502_16577_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_size.json")


def derangements(n):
    d = [1, 0]
    for k in range(2, n + 1):
        d.append((k - 1) * (d[k - 1] + d[k - 2]))
    return d[n]


def fib(n):
    a, b = 0, 1
    for _ in range(n):
        a, b = b, a + b
    return a


def check_residues(value, residues):
    for k, r in enumerate(residues):
        assert r == value % api.binary_prime(k), k


@pytest.mark.parametrize("n", list(range(1, 25)))
def test_bernoulli_small(oracle, n):
    a = W.bernoulli(n, 800 + n)
    got, res = api.perm_binary_exact(a)
    assert got == oracle.binary(a), n
    check_residues(got, res)


@pytest.mark.parametrize("n,per_row", [(14, 3), (18, 4), (22, 5), (26, 6)])
def test_sparse_rows_small(oracle, n, per_row):
    a = W.sparse_rows(n, per_row, 900 + n)
    got, res = api.perm_binary_exact(a)
    assert got == oracle.binary(a)
    check_residues(got, res)


@pytest.mark.parametrize("n", [13, 20, 27, 34])
def test_closed_forms(n):
    assert api.perm_binary_exact(np.ones((n, n), np.uint8))[0] == math.factorial(n)
    assert api.perm_binary_exact(W.ones_minus_identity(n).astype(np.uint8))[0] == derangements(n)
    assert api.perm_binary_exact(W.tridiagonal_ones(n).astype(np.uint8))[0] == fib(n + 1)


def test_more_primes_than_needed_agree():
    a = W.bernoulli(20, 5)
    v3, r3 = api.perm_binary_exact(a, n_primes=3)
    v6, r6 = api.perm_binary_exact(a, n_primes=6)
    assert v3 == v6 and r3 == r6[:3]
    check_residues(v6, r6)


def test_empty_row_gives_zero():
    a = W.bernoulli(16, 2)
    a[3, :] = 0
    assert api.perm_binary_exact(a)[0] == 0


def _golden(name):
    with open(GOLDEN) as f:
        data = json.load(f)
    if name not in data:
        pytest.skip(f"no stored oracle value for {name}: run tests/golden/make_golden.py {name}")
    return data[name]


def test_full_size_bernoulli32():
    g = _golden("bernoulli32")
    a = W.bernoulli(32, W.SEED_BERNOULLI32)
    assert W.digest(a) == g["digest"]
    got, res = api.perm_binary_exact(a)
    assert got == int(g["value"])
    check_residues(got, res)


def test_full_size_sparse40():
    g = _golden("sparse40")
    a = W.sparse_rows(40, 6, W.SEED_SPARSE40)
    assert W.digest(a) == g["digest"]
    got, res = api.perm_binary_exact(a)
    assert got == int(g["value"])
    check_residues(got, res)


# Kernels generated for the pattern (perm_binary_exact_gen): the same exact
# values, on random patterns against the oracle, closed forms and both
# full-size inputs.
@pytest.mark.parametrize("n,per_row", [(14, 3), (17, 4), (21, 5), (24, 6)])
def test_generated_sparse_rows(oracle, n, per_row):
    a = W.sparse_rows(n, per_row, 1900 + n)
    got, res = api.perm_binary_exact(a, generated=True)
    assert got == oracle.binary(a), n
    check_residues(got, res)


@pytest.mark.parametrize("n", [14, 19, 24])
def test_generated_bernoulli_and_closed_forms(oracle, n):
    a = W.bernoulli(n, 1950 + n)
    assert api.perm_binary_exact(a, generated=True)[0] == oracle.binary(a)
    assert api.perm_binary_exact(np.ones((n, n), np.uint8), generated=True)[0] == math.factorial(n)
    assert api.perm_binary_exact(W.ones_minus_identity(n).astype(np.uint8),
                                 generated=True)[0] == derangements(n)
    assert api.perm_binary_exact(W.tridiagonal_ones(n).astype(np.uint8),
                                 generated=True)[0] == fib(n + 1)
    assert api.perm_binary_exact(W.block_ones(n, 2 if n % 2 == 0 else 1).astype(np.uint8),
                                 generated=True)[0] == (2 if n % 2 == 0 else 1) ** (n // (2 if n % 2 == 0 else 1))


def test_generated_small_and_empty():
    a = W.bernoulli(10, 7)  # below the generated path's minimum order: the staged kernel
    assert api.perm_binary_exact(a, generated=True)[0] == api.perm_binary_exact(a)[0]
    b = W.bernoulli(16, 2)
    b[:, 5] = 0
    assert api.perm_binary_exact(b, generated=True)[0] == 0


@pytest.mark.parametrize("name", ["bernoulli32", "sparse40"])
def test_generated_full_size(name):
    g = _golden(name)
    a = (W.bernoulli(32, W.SEED_BERNOULLI32) if name == "bernoulli32"
         else W.sparse_rows(40, 6, W.SEED_SPARSE40))
    assert W.digest(a) == g["digest"]
    got, res = api.perm_binary_exact(a, generated=True)
    assert got == int(g["value"]), name
    check_residues(got, res)
