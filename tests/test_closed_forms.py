"""The closed forms used by the GPU tests, checked by brute force on small
cases (CPU)."""
import fractions

import pytest

from closed_forms import all_ones_first_launch


def brute_first_launch(n, m, span):
    """The same partial sum term by term: every lane K < 2^m and step l < span,
    g = K 2^(n-1-m) + l, x = (number of columns in Gray(g)) + 1 - n/2 for the
    all-ones matrix, times 2 (-1)^(n-1)."""
    c = n - 1 - m
    tot = fractions.Fraction(0)
    absum = fractions.Fraction(0)
    for K in range(1 << m):
        for l in range(span):
            g = (K << c) + l
            x = fractions.Fraction(2 * bin(g ^ (g >> 1)).count("1") + 2 - n, 2)
            t = x ** n
            tot += -t if g & 1 else t
            absum += abs(t)
    return 2 * (-1) ** (n - 1) * tot, 2 * absum


@pytest.mark.parametrize("n,m,span", [(9, 2, 2), (10, 3, 4), (11, 4, 8), (13, 5, 16), (12, 0, 16)])
def test_all_ones_first_launch_by_brute_force(n, m, span):
    assert all_ones_first_launch(n, m, span) == brute_first_launch(n, m, span)


def test_all_ones_whole_sweep_is_n_factorial():
    # with every lane's whole chunk (span = 2^c) the sum is perm(J_n) = n!;
    # the closed form needs l < 2^(c-1), so this runs the brute force only
    import math
    for n in (5, 8, 11):
        for m in (0, 2):
            assert brute_first_launch(n, m, 1 << (n - 1 - m))[0] == math.factorial(n)
