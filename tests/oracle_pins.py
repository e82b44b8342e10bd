"""Pin checks for a single-system tridiagonal solver ``solve(a, b, c, d) -> x``.

Each check compares against something other than the solver's own formula:
dense LU (numpy/LAPACK), LAPACK's banded solver, exact rational elimination,
closed forms, manufactured integer solutions, and the normwise backward-error
bound.  They are plain functions so that the same suite runs against the
oracle and against deliberately broken copies of it (the mutation test).
"""
from fractions import Fraction

import numpy as np
import scipy.linalg

EPS = np.finfo(np.float64).eps


def dense(a, b, c):
    n = len(b)
    A = np.diag(np.asarray(b, dtype=np.float64))
    for i in range(1, n):
        A[i, i - 1] = a[i]
    for i in range(n - 1):
        A[i, i + 1] = c[i]
    return A


def relerr(x, ref):
    return np.max(np.abs(np.asarray(x) - ref)) / max(np.max(np.abs(ref)), 1e-300)


def random_dominant(rs, n, margin=(0.5, 2.0)):
    a = rs.uniform(-1, 1, n)
    c = rs.uniform(-1, 1, n)
    a[0] = 0.0
    c[-1] = 0.0
    b = (np.abs(a) + np.abs(c)) + rs.uniform(*margin, n)
    b *= np.where(rs.uniform(size=n) < 0.5, -1.0, 1.0)   # mixed signs stay dominant
    d = rs.uniform(-1, 1, n)
    return a, b, c, d


def check_dense_lu(solve, seeds=range(40), tol=1e-13):
    """Against numpy.linalg.solve (LAPACK getrf/getrs with partial pivoting)."""
    for seed in seeds:
        rs = np.random.default_rng(seed)
        n = int(rs.integers(1, 65))
        a, b, c, d = random_dominant(rs, n)
        ref = np.linalg.solve(dense(a, b, c), d)
        e = relerr(solve(a, b, c, d), ref)
        assert e <= tol, (seed, n, e)


def check_banded(solve, seeds=range(40, 60), tol=1e-13):
    """Against scipy.linalg.solve_banded (LAPACK gbsv)."""
    for seed in seeds:
        rs = np.random.default_rng(seed)
        n = int(rs.integers(2, 200))
        a, b, c, d = random_dominant(rs, n, margin=(0.01, 0.1))
        ab = np.zeros((3, n))
        ab[0, 1:] = c[:-1]
        ab[1] = b
        ab[2, :-1] = a[1:]
        ref = scipy.linalg.solve_banded((1, 1), ab, d)
        e = relerr(solve(a, b, c, d), ref)
        assert e <= tol, (seed, n, e)


def exact_solve(a, b, c, d):
    """Dense Gauss-Jordan elimination in exact rationals (no rounding at all)."""
    n = len(b)
    M = [[Fraction(0)] * (n + 1) for _ in range(n)]
    for i in range(n):
        M[i][i] = Fraction(b[i])
        if i > 0:
            M[i][i - 1] = Fraction(a[i])
        if i < n - 1:
            M[i][i + 1] = Fraction(c[i])
        M[i][n] = Fraction(d[i])
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [u - f * v for u, v in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def check_exact_rational(solve, seeds=range(30), tol=4 * EPS):
    """Small integer systems: the exact rational solution, rounded, within a few ulps."""
    for seed in seeds:
        rs = np.random.default_rng(1000 + seed)
        n = int(rs.integers(1, 9))
        a = rs.integers(-4, 5, n).astype(float)
        c = rs.integers(-4, 5, n).astype(float)
        a[0] = 0.0
        c[-1] = 0.0
        b = np.abs(a) + np.abs(c) + rs.integers(1, 4, n)
        d = rs.integers(-9, 10, n).astype(float)
        ref = np.array([float(v) for v in exact_solve(a, b, c, d)])
        e = relerr(solve(a, b, c, d), ref)
        assert e <= tol * n, (seed, n, e)


def check_closed_form(solve, sizes=(1, 2, 3, 12, 64, 128)):
    """tridiag(-1, 2, -1) x = 1 has x_k = k (n + 1 - k) / 2 (k = 1..n): exact
    integers or halves.  Rounding error grows like n^2 eps (kappa ~ n^2)."""
    for n in sizes:
        a = np.full(n, -1.0); a[0] = 0.0
        c = np.full(n, -1.0); c[-1] = 0.0
        b = np.full(n, 2.0)
        k = np.arange(1, n + 1, dtype=np.float64)
        ref = k * (n + 1 - k) / 2.0
        e = relerr(solve(a, b, c, np.ones(n)), ref)
        assert e <= 2.0 * n * n * EPS, (n, e)


def check_cramer(solve):
    """n = 1: x = d/b.  n = 2: Cramer's rule."""
    rs = np.random.default_rng(7)
    for _ in range(20):
        b0 = rs.uniform(1, 2)
        d0 = rs.uniform(-1, 1)
        x = solve([0.0], [b0], [0.0], [d0])
        assert abs(x[0] - d0 / b0) <= 2 * EPS * abs(d0 / b0)
        a1, c0 = rs.uniform(-1, 1, 2)
        b0, b1 = rs.uniform(2, 3, 2)
        d0, d1 = rs.uniform(-1, 1, 2)
        det = b0 * b1 - c0 * a1
        ref = np.array([(d0 * b1 - c0 * d1) / det, (b0 * d1 - a1 * d0) / det])
        e = relerr(solve([0.0, a1], [b0, b1], [c0, 0.0], [d0, d1]), ref)
        assert e <= 8 * EPS, e


def check_manufactured(solve, seeds=range(20)):
    """Integer x and integer coefficients: d = A x is exact in FP64, so the
    solver must return x to within a few ulps."""
    for seed in seeds:
        rs = np.random.default_rng(500 + seed)
        n = int(rs.integers(2, 300))
        a = rs.integers(-3, 4, n).astype(float); a[0] = 0.0
        c = rs.integers(-3, 4, n).astype(float); c[-1] = 0.0
        b = np.abs(a) + np.abs(c) + rs.integers(1, 3, n)
        x = rs.integers(-8, 9, n).astype(float)
        d = b * x
        d[1:] += a[1:] * x[:-1]
        d[:-1] += c[:-1] * x[1:]
        e = relerr(solve(a, b, c, d), x)
        assert e <= 64 * EPS, (seed, n, e)


def check_backward_error(solve, seeds=range(20)):
    """Normwise backward error |d - A x|_inf / (|A|_inf |x|_inf + |d|_inf) <= c n eps."""
    for seed in seeds:
        rs = np.random.default_rng(900 + seed)
        n = int(rs.integers(2, 2000))
        a, b, c, d = random_dominant(rs, n, margin=(0.01, 1.0))
        x = np.asarray(solve(a, b, c, d))
        r = d - (b * x)
        r[1:] -= a[1:] * x[:-1]
        r[:-1] -= c[:-1] * x[1:]
        normA = np.max(np.abs(a) + np.abs(b) + np.abs(c))
        eta = np.max(np.abs(r)) / (normA * np.max(np.abs(x)) + np.max(np.abs(d)))
        assert eta <= 8 * EPS, (seed, n, eta)


def check_ignores_corners(solve):
    """a[0] and c[n-1] are outside the matrix and must not change x."""
    rs = np.random.default_rng(3)
    a, b, c, d = random_dominant(rs, 17)
    x0 = np.asarray(solve(a, b, c, d))
    a2, c2 = a.copy(), c.copy()
    a2[0], c2[-1] = 123.0, -77.0
    assert np.array_equal(x0, np.asarray(solve(a2, b, c2, d)))


ALL_CHECKS = [check_dense_lu, check_banded, check_exact_rational, check_closed_form,
              check_cramer, check_manufactured, check_backward_error, check_ignores_corners]
