"""Pin of the LeNet-shaped stack's activation (CPU only).

The configuration asks for the degree-4 least-squares polynomial ReLU on
[-1, 1].  With uniform weight on [-1, 1] that is the L2 projection of
max(0, x) onto polynomials of degree <= 4.  The oracle stores it as the table
``RELU4``; its FP64 reference ``relu4_ref`` reuses the table, so the table is
pinned here twice, independently of how it was derived (a Legendre
projection):

1. the normal equations G c = b in the monomial basis, solved in exact
   rationals: G[i][j] = integral of x^(i+j) over [-1, 1], b[i] = integral of
   x^i max(0, x) = 1 / (i + 2);
2. numpy's own least-squares fit on a dense uniform grid of [-1, 1].
"""
from fractions import Fraction

import numpy as np

from oracle import layers as LY


def _solve_exact(G, b):
    """Gauss-Jordan elimination over the rationals."""
    n = len(b)
    A = [row[:] + [b[i]] for i, row in enumerate(G)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        piv = A[c][c]
        A[c] = [v / piv for v in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [a - f * v for a, v in zip(A[r], A[c])]
    return [A[i][n] for i in range(n)]


def _moment(k):
    """integral of x^k over [-1, 1]"""
    return Fraction(0) if k % 2 else Fraction(2, k + 1)


def exact_relu4():
    G = [[_moment(i + j) for j in range(5)] for i in range(5)]
    b = [Fraction(1, i + 2) for i in range(5)]  # integral of x^(i+1) over [0, 1]
    return _solve_exact(G, b)


def test_relu4_table_is_the_exact_least_squares_fit():
    c = exact_relu4()
    assert c[3] == 0  # max(0, x) = (x + |x|) / 2: only x is odd
    table = [LY.RELU4.get(k, 0.0) for k in range(5)]
    for k in range(5):
        assert abs(table[k] - float(c[k])) < 1e-15, (k, table[k], c[k])
    # the rationals themselves (so that a typo in either the table or the
    # solver shows up as a mismatch of small fractions)
    assert c == [Fraction(15, 256), Fraction(1, 2), Fraction(105, 128), Fraction(0), Fraction(-105, 256)]


def test_relu4_table_matches_a_dense_grid_fit():
    x = np.linspace(-1.0, 1.0, 400001)
    fit = np.polynomial.Polynomial.fit(x, np.maximum(0.0, x), 4, domain=[-1, 1], window=[-1, 1])
    table = np.array([LY.RELU4.get(k, 0.0) for k in range(5)])
    assert np.max(np.abs(fit.coef - table)) < 1e-5


def test_relu4_is_optimal_against_perturbations():
    """Any change of one coefficient raises the L2 error (first-order
    optimality checked numerically on a fine grid)."""
    x = np.linspace(-1.0, 1.0, 200001)
    f = np.maximum(0.0, x)

    def err(coef):
        return np.trapezoid((np.polynomial.polynomial.polyval(x, coef) - f) ** 2, x)

    base = np.array([LY.RELU4.get(k, 0.0) for k in range(5)])
    e0 = err(base)
    for k in range(5):
        for d in (1e-3, -1e-3):
            c = base.copy()
            c[k] += d
            assert err(c) > e0
    # the fit's known worst-case error (at x = 0)
    assert abs(np.max(np.abs(LY.relu4_ref(x) - f)) - 15.0 / 256.0) < 1e-12
