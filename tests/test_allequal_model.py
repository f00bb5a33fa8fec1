"""Rounding model of the dense FP64 sweep on the all-equal matrix.

Section 5 measures precision on matrices whose entries all equal one value a
(perm = n! a^n).  With all rows equal, every row of x holds the same value,
and after an exact re-seed that value depends only on k0, the number of
columns in the subset; inside one re-seed interval of 2^9 steps the walk then
depends only on k0 and on bit 9 of the interval's first index.  Over the
intervals g0 = 512 h, popcount(Gray(g0)) = (h mod 2) + popcount(Gray(h)), the
second term takes the value k' for C(n - 10, k') of the h, and its parity is
h mod 2.  So the whole sweep of 2^(n-1) steps is a sum over n - 9 classes with
binomial weights, which these tests evaluate in exact rational arithmetic with
chosen parts rounded as FP64 would round them.

This is analysis, not parity: it explains the size of the all-equal errors
(the paper's Table 3 shapes) by splitting them into the rounding of x, of the
products and of the block sums.  The kernel-order model (x walked in FP64,
the product as four chains, the 16-term block tree with one product of each
even/odd pair fused into the subtraction, as the compiled code does) gives
relative errors 5.5e-13, -5.8e-11, -1.46e-10 and -1.03e-9 at n = 35, 38, 40
and 45, which are the errors the GPU measures in its compensated modes.
"""
import math
from fractions import Fraction

import pytest

A = 0.91           # the all-equal entry (stored double)
LOG2_RESEED = 9
BLOCK = 16


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _x0_fp64(n):
    # x_i = a_{i,n-1} - r_i / 2 with a compensated row sum (as the staging does)
    s = e = 0.0
    for _ in range(n):
        s, err = _two_sum(s, A)
        e += err
    return (A - 0.5 * s) - 0.5 * e


def _chains(x, n):
    """The product of n copies of x as four interleaved chains, halves rounded."""
    p = [x, x, x, x]
    for i in range(4, n, 4):
        for q in range(4):
            if i + q < n:
                p[q] *= x
    return p[0] * p[1], p[2] * p[3]


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _interval_x(n, k0, b9, walk):
    """x at the 512 steps of one re-seed interval of class (k0, b9): exact
    rationals, or FP64 values walked from the FP64 re-seed when walk=True."""
    aq = Fraction(A)
    x0q = aq - n * aq / 2
    xf = _x0_fp64(n)
    for _ in range(k0):
        xf = xf + A
    k = k0
    out = []
    for l in range(1 << LOG2_RESEED):
        if l:
            j = (l & -l).bit_length() - 1
            above = (l >> (j + 1)) & 1 if j + 1 < LOG2_RESEED else b9
            add = ((l >> j) & 1) ^ above      # bit j of the Gray code after the step
            k += 1 if add else -1
            xf = xf + A if add else xf - A
        out.append(xf if walk else x0q + k * aq)
    return out


def _interval_sum(n, xs, model):
    """Exact sum of the interval's block sums, each block summed as `model` says."""
    total = Fraction(0)
    for b in range(0, len(xs), BLOCK):
        blk = xs[b:b + BLOCK]
        if model == "exact":
            total += sum((-1) ** m * Fraction(x) ** n for m, x in enumerate(blk))
            continue
        if model == "chains":   # FP64 products, exact sums
            total += sum((-1) ** m * Fraction(p * q)
                         for m, (p, q) in enumerate(_chains(float(x), n) for x in blk))
            continue
        # "kernel": FP64 products, even term fused into the pair difference, tree
        v = []
        for m in range(0, BLOCK, 2):
            pe, qe = _chains(float(blk[m]), n)
            po, qo = _chains(float(blk[m + 1]), n)
            v.append(_fma(pe, qe, -(po * qo)))
        while len(v) > 1:
            v = [v[i] + v[i + 1] for i in range(0, len(v), 2)]
        total += Fraction(v[0])
    return total


def sweep_model(n, x_mode, model):
    """2 (-1)^(n-1) sum over all 2^(n-1) steps, by classes (k0, b9)."""
    m = n - 1 - LOG2_RESEED
    tot = Fraction(0)
    for kp in range(m + 1):
        b9 = kp & 1
        xs = _interval_x(n, kp + b9, b9, walk=(x_mode == "walk"))
        if x_mode == "round_once":
            xs = [float(x) for x in xs]
        tot += math.comb(m, kp) * _interval_sum(n, xs, model)
    return tot * (2 if n % 2 else -2)


def _rel(n, x_mode, model):
    exact = math.factorial(n) * Fraction(A) ** n
    return float((sweep_model(n, x_mode, model) - exact) / exact)


@pytest.mark.parametrize("n", [12, 20, 35, 40, 45])
def test_class_reduction_is_exact(n):
    # no rounding anywhere: the class sum is exactly n! a^n
    assert sweep_model(n, "exact", "exact") == math.factorial(n) * Fraction(A) ** n


def test_error_split_at_paper_sizes():
    # each rounding source alone, and the kernel's order; all well inside the
    # forward-error scale n u R(A) / perm(A) of the all-equal matrix
    rows = {}
    for n in (35, 40, 45):
        r = 2 * sum(math.comb(n - 1, k) * abs(Fraction(2 * (k + 1) - n, 2)) ** n for k in range(n))
        scale = n * 2.0 ** -53 * float(r / math.factorial(n))
        rows[n] = {
            "x rounded once": _rel(n, "round_once", "exact"),
            "x walked in FP64": _rel(n, "walk", "exact"),
            "products (x rounded once)": _rel(n, "round_once", "chains"),
            "x walk + products": _rel(n, "walk", "chains"),
            "kernel order": _rel(n, "walk", "kernel"),
        }
        for name, v in rows[n].items():
            print(f"n = {n}: {name:28s} {v: .3e}  (n u R/perm = {scale:.2e})")
            assert abs(v) < scale
    # the kernel-order model is the error the GPU measures (two-sum mode)
    assert rows[40]["kernel order"] == pytest.approx(-1.458e-10, rel=2e-3)
    # the 16-term tree adds next to nothing to the product and x errors
    for n in (35, 40, 45):
        assert abs(rows[n]["kernel order"] - rows[n]["x walk + products"]) < 0.5 * max(
            abs(rows[n]["x walk + products"]), 1e-11)
