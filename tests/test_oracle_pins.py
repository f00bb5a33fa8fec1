"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here touches the GPU path.  Each test names the passage or the
identity it checks.  ``test_mutants_are_caught`` rebuilds the oracle with one
planted mistake at a time and checks that these pins notice every one.
"""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle.oracle import Oracle, build, load
from paper_2502_16577_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fixture_rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


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


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# --- Section 2, Table 1 and the CBL recursion of Section 3.1.1 ---------------

def test_table1_gray_codes(oracle):
    for g, binary, gray, changed in _fixture_rows("paper_table1_gray3.txt"):
        g = int(g)
        assert format(g, "03b") == binary
        assert format(oracle.gray(g), "03b") == gray
        if changed != "-":
            assert oracle.flip_col(g) == int(changed)
            # the sign is +1 exactly when the changed bit is set in Gray_g
            assert oracle.flip_sign(g) == (1 if gray[::-1][int(changed)] == "1" else -1)


def test_cbl_recursion(oracle):
    cbl3 = [int(t) for t in _fixture_rows("paper_cbl3.txt")[0]]
    assert [oracle.flip_col(g) for g in range(1, 8)] == cbl3
    prev = cbl3
    for k in range(4, 12):
        cur = [oracle.flip_col(g) for g in range(1, 2 ** k)]
        assert cur == prev + [k - 1] + prev[::-1]
        assert len(cur) == 2 ** k - 1
        prev = cur


# --- Eq. (1) vs Eq. (2) vs Algorithm 1 --------------------------------------

@pytest.mark.parametrize("n", list(range(1, 10)))
def test_three_formulas_agree_real(oracle, n):
    rng = np.random.default_rng(1000 + n)
    for a in (rng.random((n, n)), rng.standard_normal((n, n))):
        b = oracle.brute(a)
        assert rel(oracle.inclexcl(a), b) < 1e-14 or abs(oracle.inclexcl(a) - b) < 1e-13
        assert abs(oracle.ryser(a) - b) <= 1e-14 * max(1.0, oracle.brute(np.abs(a)))


@pytest.mark.parametrize("n", list(range(1, 9)))
def test_three_formulas_agree_complex(oracle, n):
    rng = np.random.default_rng(2000 + n)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = oracle.brute(a)
    scale = oracle.brute(np.abs(a))
    assert abs(oracle.inclexcl(a) - b) <= 1e-14 * scale
    assert abs(oracle.ryser(a) - b) <= 1e-14 * scale


def test_ryser_vs_inclexcl_larger(oracle):
    # Eq. (2) without Gray code or halving, against Algorithm 1, n = 14..16.
    # Eq. (2) sums terms up to (row sum)^n, about 1e5 times perm for these
    # inputs, so its own long-double rounding allows ~1e-14 relative.
    for n in (14, 16):
        a = W.uniform(n, 77 + n)
        assert rel(oracle.ryser(a), oracle.inclexcl(a)) < 1e-12
        c = W.haar_block(2 * n, n, 99 + n)
        scale = oracle.ryser(np.abs(c))
        assert abs(oracle.ryser(c) - oracle.inclexcl(c)) < 1e-13 * scale


def test_thread_count_does_not_change_result(oracle):
    a = W.uniform(20, W.SEED_U20)
    v1 = oracle.ryser(a, threads=1, split=True)
    v8 = oracle.ryser(a, threads=8, split=True)
    assert v1 == v8


# --- closed forms -----------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 12, 16, 20])
def test_all_ones_is_factorial(oracle, n):
    # Section 5: all entries equal a gives n! a^n.
    assert rel(oracle.ryser(W.all_ones(n)), math.factorial(n)) < 1e-15
    a = 0.91
    assert rel(oracle.ryser(np.full((n, n), a)), math.factorial(n) * a ** n) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 6, 10, 15, 20])
def test_ones_minus_identity_is_derangements(oracle, n):
    assert rel(oracle.ryser(W.ones_minus_identity(n)), derangements(n)) < 1e-14


def test_identity_diagonal_triangular(oracle):
    rng = np.random.default_rng(5)
    for n in (1, 4, 9, 17):
        assert oracle.ryser(np.eye(n)) == pytest.approx(1.0, rel=1e-15)
        d = rng.random(n) + 0.5
        assert rel(oracle.ryser(np.diag(d)), float(np.prod(d))) < 1e-14
        t = np.tril(rng.random((n, n))) + np.diag(d)
        assert rel(oracle.ryser(t), float(np.prod(np.diag(t)))) < 1e-13


def test_rank_one(oracle):
    rng = np.random.default_rng(6)
    for n in (3, 7, 12, 18):
        u = rng.random(n) + 0.1
        v = rng.random(n) + 0.1
        exact = math.factorial(n) * float(np.prod(u)) * float(np.prod(v))
        assert rel(oracle.ryser(np.outer(u, v)), exact) < 1e-13


def test_block_diagonal_and_tridiagonal(oracle):
    rng = np.random.default_rng(7)
    b1, b2 = rng.random((5, 5)), rng.random((7, 7))
    a = np.zeros((12, 12))
    a[:5, :5] = b1
    a[5:, 5:] = b2
    assert rel(oracle.ryser(a), oracle.brute(b1) * oracle.ryser(b2)) < 1e-13
    for n in (5, 10, 19):
        # Section 1: tridiagonal all-ones (a Hessenberg family) gives Fibonacci numbers.
        assert rel(oracle.ryser(W.tridiagonal_ones(n)), fib(n + 1)) < 1e-14


def test_invariances(oracle):
    rng = np.random.default_rng(8)
    n = 13
    a = rng.standard_normal((n, n))
    p = oracle.ryser(a)
    scale = oracle.ryser(np.abs(a))
    pr, pc = rng.permutation(n), rng.permutation(n)
    assert abs(oracle.ryser(a[pr][:, pc]) - p) < 1e-13 * scale
    assert abs(oracle.ryser(a.T) - p) < 1e-13 * scale
    d = rng.random(n) + 0.5
    assert abs(oracle.ryser(d[:, None] * a) - np.prod(d) * p) < 1e-13 * scale * np.prod(d)


def test_complex_phase_construction(oracle):
    # perm(D1 B D2) = prod(D1) prod(D2) perm(B) for diagonal D1, D2.
    rng = np.random.default_rng(9)
    n = 12
    b = rng.random((n, n))
    th, ph = rng.random(n) * 2 * np.pi, rng.random(n) * 2 * np.pi
    c = np.exp(1j * th)[:, None] * b * np.exp(1j * ph)[None, :]
    want = np.exp(1j * (th.sum() + ph.sum())) * oracle.ryser(b)
    assert abs(oracle.ryser(c) - want) < 1e-14 * abs(want)


# --- Algorithm 2 on CSC columns -----------------------------------------------

def test_csc_walk_equals_dense_walk(oracle):
    # a step adds only the flipped column's nonzeros; adding the zeros as
    # well (the dense walk) changes no value, so the two agree bit for bit
    for n, per_row, seed in ((9, 3, 1), (16, 4, 3), (21, 5, 4)):
        a = W.sparse_rows(n, per_row, seed).astype(np.float64) * W.uniform(n, seed + 10)
        a[0, :] *= -1.0  # signed entries too
        assert oracle.sparse(a) == oracle.ryser(a)


def test_csc_walk_closed_forms(oracle):
    for n in (1, 2, 7, 13, 18):
        assert oracle.sparse(np.eye(n)) == 1.0
        assert rel(oracle.sparse(W.ones_minus_identity(n)), derangements(n)) < 1e-14
        assert rel(oracle.sparse(W.tridiagonal_ones(n)), fib(n + 1)) < 1e-14
        assert rel(oracle.sparse(W.block_ones(n, 3)), (
            math.factorial(3) ** (n // 3) * math.factorial(n % 3))) < 1e-14


def test_walk_in_parts_adds_up_to_the_whole(oracle):
    # the walk cut into consecutive pieces (how the 40 x 40 reference values
    # are computed) sums to the permanent: checked against Eq. (1), the
    # closed forms n! and D_n, and the undivided walk, dense and CSC
    from fractions import Fraction

    def whole(n, parts):
        tot = sum(Fraction(h) + Fraction(l) for (h, l), _ in parts) * (2 if n % 2 else -2)
        ab = 2 * sum(Fraction(h) + Fraction(l) for _, (h, l) in parts)
        return float(tot), float(ab)

    for n in (2, 5, 8):
        a = W.uniform(n, 300 + n) - 0.5
        v, _ = whole(n, [oracle.ryser_part(a, p, 3) for p in range(3)])
        assert rel(v, oracle.brute(a)) < 1e-13
    for n, k in ((12, 1), (13, 4), (16, 9)):
        v, r = whole(n, [oracle.ryser_part(W.all_ones(n), p, k) for p in range(k)])
        assert v == math.factorial(n) and rel(r, r_all_ones(n)) < 1e-14
        v, _ = whole(n, [oracle.ryser_part(W.ones_minus_identity(n), p, k) for p in range(k)])
        assert rel(v, derangements(n)) < 1e-15
    a = W.uniform(17, 317)
    want, r = oracle.ryser(a, with_abs=True)
    v, rp = whole(17, [oracle.ryser_part(a, p, 7) for p in range(7)])
    assert rel(v, want) < 1e-15 and rel(rp, r) < 1e-15
    s = W.sparse_rows(18, 4, 318).astype(np.float64) * W.uniform(18, 319)
    cp, ri, vals = W.to_csc(s)
    v, _ = whole(18, [oracle.ryser_part(18, p, 5, csc=(cp, ri, vals)) for p in range(5)])
    assert rel(v, oracle.ryser_csc(18, cp, ri, vals)) < 1e-15


# --- R(A), the Ryser absolute sum 2 sum_g |prod_i x_i(g)| ---------------------
# Closed forms that follow from Algorithm 1's start vector
# x_i(S) = a_{i,n-1} + sum_{j in S} a_ij - r_i / 2 over the subsets S of the
# first n - 1 columns:
#   * I_n: every x_i(S) is +-1/2, so each of the 2^(n-1) terms is 2^-n: R = 1.
#   * diag(d): x_i(S) = +-d_i / 2, so R = prod_i |d_i| (also for complex d).
#   * J_n: x_i(S) = |S| + 1 - n/2 in every row, so
#     R = 2 sum_k C(n-1, k) |k + 1 - n/2|^n.
#   * scaling row i by c multiplies every x_i(S) by c: R(DA) = prod|d_i| R(A).

def r_all_ones(n):
    from fractions import Fraction
    tot = sum(math.comb(n - 1, k) * abs(Fraction(2 * (k + 1) - n, 2)) ** n for k in range(n))
    return float(2 * tot)


@pytest.mark.parametrize("n", [1, 2, 3, 8, 13, 20])
def test_r_identity_is_one(oracle, n):
    _, r = oracle.ryser(np.eye(n), with_abs=True)
    assert r == 1.0


@pytest.mark.parametrize("n", [2, 5, 11, 17])
def test_r_diagonal(oracle, n):
    rng = np.random.default_rng(40 + n)
    d = rng.random(n) + 0.25
    d[rng.random(n) < 0.5] *= -1.0
    _, r = oracle.ryser(np.diag(d), with_abs=True)
    assert rel(r, float(np.prod(np.abs(d)))) < 1e-14
    # complex diagonal: the modulus of each complex term
    z = d * np.exp(1j * rng.random(n) * 2 * np.pi)
    _, rc = oracle.ryser(np.diag(z), with_abs=True)
    assert rel(rc, float(np.prod(np.abs(z)))) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 6, 9, 14, 19])
def test_r_all_ones_closed_form(oracle, n):
    _, r = oracle.ryser(W.all_ones(n), with_abs=True)
    assert rel(r, r_all_ones(n)) < 1e-14
    # all entries 0.91: every x_i(S) scales by 0.91
    _, r91 = oracle.ryser(np.full((n, n), 0.91), with_abs=True)
    assert rel(r91, r_all_ones(n) * 0.91 ** n) < 1e-13


def test_r_brute_force_subsets(oracle):
    # tiny orders: the absolute subset sum term by term, without the Gray order
    rng = np.random.default_rng(17)
    for n in range(1, 9):
        for a in (rng.standard_normal((n, n)),
                  rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))):
            x0 = a[:, n - 1] - a.sum(axis=1) / 2
            tot = 0.0
            for s in range(2 ** (n - 1)):
                cols = [j for j in range(n - 1) if (s >> j) & 1]
                tot += abs(np.prod(x0 + a[:, cols].sum(axis=1)))
            _, r = oracle.ryser(a, with_abs=True)
            assert rel(r, 2 * tot) < 1e-13, n


def test_r_invariances(oracle):
    rng = np.random.default_rng(18)
    n = 12
    a = rng.standard_normal((n, n))
    v, r = oracle.ryser(a, with_abs=True)
    assert abs(v) <= r
    pr = rng.permutation(n)                       # rows: the x_i are permuted
    assert rel(oracle.ryser(a[pr], with_abs=True)[1], r) < 1e-14
    pc = np.concatenate([rng.permutation(n - 1), [n - 1]])  # columns other than the last
    assert rel(oracle.ryser(a[:, pc], with_abs=True)[1], r) < 1e-14
    d = rng.random(n) + 0.5
    assert rel(oracle.ryser(d[:, None] * a, with_abs=True)[1], float(np.prod(d)) * r) < 1e-13
    c = a * np.exp(1j * rng.random(n) * 2 * np.pi)[:, None]  # unit phases on the rows
    assert rel(oracle.ryser(c, with_abs=True)[1], r) < 1e-13


# --- exact binary ------------------------------------------------------------

def test_matchings_dp_vs_brute(oracle):
    for n in range(1, 9):
        a = W.bernoulli(n, 300 + n)
        assert oracle.matchings(a) == round(oracle.brute(a.astype(np.float64)))


@pytest.mark.parametrize("n", [1, 2, 5, 10, 16, 20])
def test_binary_vs_matchings(oracle, n):
    a = W.bernoulli(n, 400 + n)
    assert oracle.binary(a) == oracle.matchings(a)


def test_binary_sparse_vs_matchings(oracle):
    a = W.sparse_rows(22, 5, 12)
    assert oracle.binary(a) == oracle.matchings(a)


@pytest.mark.parametrize("n", [1, 7, 20, 25])
def test_binary_closed_forms(oracle, n):
    assert oracle.binary(W.all_ones(n).astype(np.uint8)) == math.factorial(n)
    assert oracle.binary(W.ones_minus_identity(n).astype(np.uint8)) == derangements(n)
    assert oracle.binary(W.tridiagonal_ones(n).astype(np.uint8)) == fib(n + 1)


def test_binary_block_ones_beyond_64_bits(oracle):
    # 4 blocks of all-ones 5x5 -> (5!)^4; 4 blocks of 6x6 -> 720^4
    assert oracle.binary(W.block_ones(20, 5).astype(np.uint8)) == math.factorial(5) ** 4
    assert oracle.binary(W.block_ones(24, 6).astype(np.uint8)) == math.factorial(6) ** 4
    # J_26: 26! > 2^88, needs more than two 64-bit words of the accumulator
    assert oracle.binary(np.ones((26, 26), np.uint8)) == math.factorial(26)


# --- gradient ----------------------------------------------------------------

def test_grad_laplace_and_euler(oracle):
    rng = np.random.default_rng(13)
    n = 7
    a = rng.standard_normal((n, n))
    g = oracle.grad_minors(a)
    p = oracle.brute(a)
    for i in range(n):
        assert abs(np.dot(a[i], g[i]) - p) < 1e-12       # Laplace expansion along row i
        assert abs(np.dot(a[:, i], g[:, i]) - p) < 1e-12  # and along column i
    assert abs(np.sum(a * g) - n * p) < 1e-11             # Euler: homogeneous of degree n


def test_grad_fd_equals_minors(oracle):
    rng = np.random.default_rng(14)
    n = 6
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    g = oracle.grad_minors(a)
    for (i, j) in [(0, 0), (2, 5), (5, 1)]:
        assert abs(oracle.grad_fd(a, i, j) - g[i, j]) < 1e-12


# --- planted mistakes are caught ----------------------------------------------

def _pins_pass(orc: Oracle) -> bool:
    try:
        rng = np.random.default_rng(123)
        for n in (3, 5, 6):
            a = rng.standard_normal((n, n))
            b = orc.brute(a)
            scale = orc.brute(np.abs(a))
            if abs(orc.inclexcl(a) - b) > 1e-12 * scale:
                return False
            if abs(orc.ryser(a) - b) > 1e-12 * scale:
                return False
            c = a + 1j * rng.standard_normal((n, n))
            if abs(orc.ryser(c) - orc.inclexcl(c)) > 1e-12 * orc.brute(np.abs(c)):
                return False
        if round(orc.ryser(W.all_ones(6))) != 720:
            return False
        if orc.brute(W.ones_minus_identity(5)) != 44:
            return False
        a = W.bernoulli(9, 5)
        if orc.binary(a) != orc.matchings(a):
            return False
        # R(A) closed forms
        if orc.ryser(np.eye(6), with_abs=True)[1] != 1.0:
            return False
        z = np.array([0.5, 1.5, 2.0, 0.75]) * np.exp(1j * np.array([0.3, 1.1, 2.0, 4.0]))
        if abs(orc.ryser(np.diag(z), with_abs=True)[1] - np.prod(np.abs(z))) > 1e-14:
            return False
        # Algorithm 2 on CSC columns
        if round(orc.sparse(W.ones_minus_identity(6))) != 265:
            return False
        s = W.sparse_rows(8, 3, 2).astype(np.float64) * W.uniform(8, 3)
        if orc.sparse(s) != orc.ryser(s):
            return False
        return True
    except RuntimeError:
        return False


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11])
def test_mutants_are_caught(mutant):
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, f"liboracle_m{mutant}.so")
        build(path, mutant=mutant)
        assert not _pins_pass(Oracle(load(path))), f"mutant {mutant} slipped through the pins"


def test_unmutated_build_passes_the_same_pins(oracle):
    assert _pins_pass(oracle)
