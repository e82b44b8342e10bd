"""Pins of the oracle's complex solve (CPU only).

The paper's Poisson data are complex (Sec. 8.1): after the Fourier transform
in x and y each z-line is a tridiagonal system with a real operator and a
complex right-hand side.  The oracle solves such systems by the Thomas
recurrences in complex arithmetic.  It is checked here against dense complex
LAPACK solves, exact Gaussian-rational elimination, a closed form, the real
oracle on the real and imaginary parts (linearity, for real operators), and a
mutation test that plants typical mistakes into its complex routine.
"""
import ctypes
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import oracle_pins as pins
from workloads import configs

EPS = np.finfo(np.float64).eps


def dense_z(a, b, c):
    n = len(b)
    A = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        A[i, i] = b[i]
        if i > 0:
            A[i, i - 1] = a[i]
        if i < n - 1:
            A[i, i + 1] = c[i]
    return A


def relerr_z(x, ref):
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def random_complex_dominant(rs, n):
    z = lambda: rs.uniform(-1, 1, n) + 1j * rs.uniform(-1, 1, n)
    a, c, d = z(), z(), z()
    a[0] = 0.0
    c[-1] = 0.0
    phase = np.exp(1j * rs.uniform(0, 2 * np.pi, n))
    b = (np.abs(a) + np.abs(c) + rs.uniform(0.5, 2.0, n)) * phase
    return a, b, c, d


# Gaussian rationals as (re, im) pairs of Fractions: exact complex elimination
def _zmul(u, v):
    return (u[0] * v[0] - u[1] * v[1], u[0] * v[1] + u[1] * v[0])


def _zsub(u, v):
    return (u[0] - v[0], u[1] - v[1])


def _zdiv(u, v):
    den = v[0] * v[0] + v[1] * v[1]
    return ((u[0] * v[0] + u[1] * v[1]) / den, (u[1] * v[0] - u[0] * v[1]) / den)


def exact_solve_z(a, b, c, d):
    """Dense Gauss-Jordan elimination over the Gaussian rationals (no rounding)."""
    n = len(b)
    F = lambda z: (Fraction(float(np.real(z))), Fraction(float(np.imag(z))))
    zero = (Fraction(0), Fraction(0))
    M = [[zero] * (n + 1) for _ in range(n)]
    for i in range(n):
        M[i][i] = F(b[i])
        if i > 0:
            M[i][i - 1] = F(a[i])
        if i < n - 1:
            M[i][i + 1] = F(c[i])
        M[i][n] = F(d[i])
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != zero)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != zero:
                f = _zdiv(M[r][col], M[col][col])
                M[r] = [_zsub(u, _zmul(f, v)) for u, v in zip(M[r], M[col])]
    return [_zdiv(M[i][n], M[i][i]) for i in range(n)]


@pytest.mark.parametrize("precision", [oracle.F64, oracle.LONG_DOUBLE])
def test_complex_dense_lu(precision):
    for seed in range(40):
        rs = np.random.default_rng(5000 + seed)
        n = int(rs.integers(1, 65))
        a, b, c, d = random_complex_dominant(rs, n)
        ref = np.linalg.solve(dense_z(a, b, c), d)
        e = relerr_z(oracle.thomas_complex(a, b, c, d, precision), ref)
        assert e <= 1e-13, (seed, n, e)


def test_complex_exact_gaussian_integers():
    for seed in range(25):
        rs = np.random.default_rng(6000 + seed)
        n = int(rs.integers(1, 8))
        gi = lambda lo, hi: rs.integers(lo, hi, n) + 1j * rs.integers(lo, hi, n)
        a, c, d = gi(-3, 4), gi(-3, 4), gi(-9, 10)
        a[0] = 0.0
        c[-1] = 0.0
        b = (np.abs(a) + np.abs(c)).round() + 2 + 1j * rs.integers(-2, 3, n)
        ref = np.array([float(re) + 1j * float(im) for re, im in exact_solve_z(a, b, c, d)])
        e = relerr_z(oracle.thomas_complex(a, b, c, d), ref)
        assert e <= 8 * n * EPS, (seed, n, e)


def test_complex_closed_form():
    """tridiag(-1, 2, -1) x = w has x_k = w k (n + 1 - k) / 2; the operator
    multiplied by i with the right-hand side multiplied by i gives the same x."""
    w = 1.0 + 2.0j
    for n in (1, 2, 3, 12, 64, 128):
        a = np.full(n, -1.0 + 0j); a[0] = 0.0
        c = np.full(n, -1.0 + 0j); c[-1] = 0.0
        b = np.full(n, 2.0 + 0j)
        k = np.arange(1, n + 1, dtype=np.float64)
        ref = w * k * (n + 1 - k) / 2.0
        assert relerr_z(oracle.thomas_complex(a, b, c, np.full(n, w)), ref) <= 2.0 * n * n * EPS
        got = oracle.thomas_complex(1j * a, 1j * b, 1j * c, np.full(n, 1j * w))
        assert relerr_z(got, ref) <= 2.0 * n * n * EPS


def test_complex_real_operator_is_two_real_solves():
    """A real operator acts on the real and imaginary parts separately: the
    complex solve equals the real oracle applied to each part."""
    for seed in range(20):
        rs = np.random.default_rng(7000 + seed)
        n = int(rs.integers(2, 200))
        a, b, c, _ = pins.random_dominant(rs, n)
        d = rs.uniform(-1, 1, n) + 1j * rs.uniform(-1, 1, n)
        got = oracle.thomas_complex(a, b, c, d)
        ref = oracle.thomas(a, b, c, d.real) + 1j * oracle.thomas(a, b, c, d.imag)
        assert relerr_z(got, ref) <= 4 * EPS, seed


def test_complex_singular_pivot_reported():
    with pytest.raises(oracle.OracleError):
        oracle.thomas_complex([0, 1], [0j, 1], [1, 0], [1, 1])


def test_complex_batch_layout_matches_dense():
    """The batch routine gathers mode (i, j)'s z-line of the interleaved
    complex array, adds the mode's shift to the diagonal and scatters x back."""
    p = configs.poisson_complex(8, 4, 24)
    _, _, _, d = configs.full_arrays(p)
    dz = d[0::2] + 1j * d[1::2]
    lay = configs.complex_layout(p)
    x = oracle.solve_batch_complex(lay, p.a, p.b, p.c, dz, shift=p.shift)
    X = x.reshape(24, 4, 8)
    D = dz.reshape(24, 4, 8)
    for s in range(32):
        i, j = s % 8, s // 8
        ref = np.linalg.solve(dense_z(p.a, p.b + p.shift[s], p.c), D[:, j, i])
        assert relerr_z(X[:, j, i], ref) <= 1e-12, s
    # the generator's two right-hand sides are the real and imaginary parts
    rhs = configs.system_rhs(p, 5)
    assert np.array_equal(rhs[0], D[:, 0, 5].real) and np.array_equal(rhs[1], D[:, 0, 5].imag)
    assert d[0] == 0.0 and d[1] == 0.0


def test_complex_batch_system_range():
    p = configs.poisson_complex(4, 2, 10)
    _, _, _, d = configs.full_arrays(p)
    dz = d[0::2] + 1j * d[1::2]
    lay = configs.complex_layout(p)
    full = oracle.solve_batch_complex(lay, p.a, p.b, p.c, dz, shift=p.shift)
    part = oracle.solve_batch_complex(lay, p.a, p.b, p.c, dz, shift=p.shift, systems=(2, 5))
    for s in range(8):
        rows = lay.sys_rows(s)
        if 2 <= s < 5:
            assert np.array_equal(part[rows], full[rows])
        else:
            assert not part[rows].any()


COMPLEX_MUTANTS = {
    "dropped_term": ("m = b[i] - a[i] * cp[i - 1];", "m = b[i];"),
    "conjugated": ("m = b[i] - a[i] * cp[i - 1];", "m = b[i] - conj(a[i]) * cp[i - 1];"),
    "wrong_sign": ("dp[i] = (d[i] - a[i] * dp[i - 1]) / m;", "dp[i] = (d[i] + a[i] * dp[i - 1]) / m;"),
    "real_part_only": ("dp[0] = d[0] / m;", "dp[0] = creal(d[0]) / m;"),
    "shifted_index": ("x[i] = dp[i] - cp[i] * x[i + 1];", "x[i] = dp[i] - cp[i + 1] * x[i + 1];"),
    "transposed": ("dp[i] = (d[i] - a[i] * dp[i - 1]) / m;", "dp[i] = (d[i] - c[i - 1] * dp[i - 1]) / m;"),
}

COMPLEX_CHECKS = [test_complex_dense_lu, test_complex_exact_gaussian_integers,
                  test_complex_closed_form, test_complex_real_operator_is_two_real_solves]


@pytest.mark.parametrize("name", sorted(COMPLEX_MUTANTS))
def test_complex_pins_reject_mutant(name, tmp_path, monkeypatch):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    old, new = COMPLEX_MUTANTS[name]
    start = src.index("static int thomas_z(")
    end = src.index("static int thomas_zld(")
    body = src[start:end]
    assert old in body
    mutated = src[:start] + body.replace(old, new, 1) + src[end:]
    cfile = tmp_path / "m.c"
    cfile.write_text(mutated)
    so = tmp_path / "libmz.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(so), str(cfile), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_thomas_z.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_int]

    def thomas_complex(a, b, c, d, precision=oracle.F64):
        arrs = [np.ascontiguousarray(v, dtype=np.complex128) for v in (a, b, c, d)]
        x = np.empty(arrs[3].size, dtype=np.complex128)
        rc = lib.oracle_thomas_z(x.size, *[v.ctypes.data_as(dp) for v in arrs],
                                 x.ctypes.data_as(dp), 0)
        if rc != 0:
            raise AssertionError("mutant reported failure")
        return x

    monkeypatch.setattr(oracle, "thomas_complex", thomas_complex)
    caught = []
    for check in COMPLEX_CHECKS:
        try:
            if check is test_complex_dense_lu:
                check(oracle.F64)
            else:
                check()
        except (AssertionError, ZeroDivisionError, FloatingPointError, ValueError):
            caught.append(check.__name__)
    assert caught, f"no pin caught mutant {name}"
