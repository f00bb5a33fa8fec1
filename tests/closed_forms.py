"""Exact values for GPU tests that have a closed form (test helpers; no GPU,
no oracle)."""
import fractions
import math


def all_ones_first_launch(n, log2_lanes, span):
    """perm_dense_f64_ex's output after only the first launch of a split sweep
    of the all-ones matrix: 2 (-1)^(n-1) times the sum over lanes K < 2^m
    (m = log2_lanes) and steps l < span of (-1)^l x^n, x = pc + 1 - n/2 with pc
    the number of columns j < n - 1 in the Gray code of g = K 2^c + l.  For
    l < 2^(c-1), pc = popcount(Gray(K)) + (K & 1) + popcount(Gray(l)); bit 0 of
    K is the parity of popcount(Gray(K)), and popcount(Gray(K)) = k for C(m, k)
    of the K (Gray coding is a bijection).  Returns (value, sum of |terms|),
    exact as Fractions."""
    m = log2_lanes
    tot = 0
    absum = 0
    for k in range(m + 1):
        v = k + (k & 1)
        for l in range(span):
            y = 2 * (v + bin(l ^ (l >> 1)).count("1") + 1) - n  # y = 2x
            t = math.comb(m, k) * y ** n
            tot += -t if l & 1 else t
            absum += abs(t)
    scale = fractions.Fraction(2, 2 ** n)
    return (scale * tot if n % 2 else -scale * tot), scale * absum
