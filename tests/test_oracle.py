"""Pins of the oracle against mathematics it does not share (CPU only).

The oracle is the FP64 Thomas algorithm (x = A^{-1} d per system, the problem
statement of the paper's Algorithms 1 and 2).  It is checked against dense and
banded LAPACK solves, exact rational elimination, closed forms, manufactured
integer solutions and the backward-error bound.  A mutation test plants the
typical mistakes (dropped term, wrong sign, shifted index, transposed operand)
into copies of the oracle and requires the pin suite to reject every one.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from tests import oracle_pins as pins
from workloads import configs


def _oracle_f64(a, b, c, d):
    return oracle.thomas(a, b, c, d, oracle.F64)


def _oracle_ld(a, b, c, d):
    return oracle.thomas(a, b, c, d, oracle.LONG_DOUBLE)


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_f64_pins(check):
    check(_oracle_f64)


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_long_double_pins(check):
    check(_oracle_ld)


def test_long_double_closer_to_exact():
    """On an ill-conditioned system (near-singular Neumann-like operator) the
    extended-precision variant must sit closer to the exact rational answer."""
    n = 24
    a = np.full(n, 1.0); a[0] = 0.0
    c = np.full(n, 1.0); c[-1] = 0.0
    b = -(a + c) - 1e-6
    b[0] = -1.0 - 1e-6
    rs = np.random.default_rng(11)
    d = rs.uniform(-1, 1, n)
    ref = np.array([float(v) for v in pins.exact_solve(a, b, c, d)])
    e64 = pins.relerr(_oracle_f64(a, b, c, d), ref)
    eld = pins.relerr(_oracle_ld(a, b, c, d), ref)
    # kappa ~ 4e6: FP64 loses ~1e-11, the 64-bit-mantissa variant ~1e-15
    assert eld < e64 / 100
    assert eld <= 1e-13


def test_singular_pivot_reported():
    with pytest.raises(oracle.OracleError):
        oracle.thomas([0.0, 1.0], [0.0, 1.0], [1.0, 0.0], [1.0, 1.0])
    lay = configs.Layout(n=2, nsys0=2, nsys1=1, row_stride=1, sys_stride0=2)
    a = np.array([0.0, 1.0, 0.0, 1.0]); b = np.array([1.0, 1.0, 1.0, 1.0])
    c = np.array([1.0, 0.0, 1.0, 0.0]); d = np.ones(4)
    x, st = oracle.solve_batch(lay, 0, a, b, c, d, status=True)
    assert list(st) == [oracle.ESINGULAR, oracle.ESINGULAR]


# ---------------------------------------------------------------------------
# batch/layout wrapper: gather/scatter and coefficient modes vs numpy indexing

def test_batch_zsystems_match_column_solves():
    p = configs.partitioned(6, 5, 33)
    a, b, c, d = configs.full_arrays(p)
    x = oracle.solve_batch(p.layout, 0, a, b, c, d)
    A3 = a.reshape(33, 5, 6); B3 = b.reshape(33, 5, 6); C3 = c.reshape(33, 5, 6)
    D3 = d.reshape(33, 5, 6); X3 = x.reshape(33, 5, 6)
    for j in range(5):
        for i in range(6):
            ref = np.linalg.solve(pins.dense(A3[:, j, i], B3[:, j, i], C3[:, j, i]), D3[:, j, i])
            assert pins.relerr(X3[:, j, i], ref) <= 1e-13


def test_batch_contiguous_and_ragged():
    p = configs.plain(nsys=5, n=40)
    a, b, c, d = configs.full_arrays(p)
    x = oracle.solve_batch(p.layout, 0, a, b, c, d)
    for s in range(5):
        sl = slice(40 * s, 40 * (s + 1))
        ref = np.linalg.solve(pins.dense(a[sl], b[sl], c[sl]), d[sl])
        assert pins.relerr(x[sl], ref) <= 1e-13
    r = configs.ragged(nsys=7, nmin=2, nmax=50)
    a, b, c, d = configs.full_arrays(r)
    x = oracle.solve_batch(r.layout, 0, a, b, c, d)
    off = r.layout.offsets
    for s in range(7):
        sl = slice(off[s], off[s + 1])
        ref = np.linalg.solve(pins.dense(a[sl], b[sl], c[sl]), d[sl])
        assert pins.relerr(x[sl], ref) <= 1e-13


def test_batch_shared_shift_equals_expanded():
    p = configs.poisson(8, 4, 20)
    _, _, _, d = configs.full_arrays(p)
    x = oracle.solve_batch(p.layout, 1, p.a, p.b, p.c, d, shift=p.shift)
    X = x.reshape(20, 4, 8)
    D = d.reshape(20, 4, 8)
    for s in range(32):
        i, j = s % 8, s // 8
        bb = p.b + p.shift[s]
        ref = np.linalg.solve(pins.dense(p.a, bb, p.c), D[:, j, i])
        assert pins.relerr(X[:, j, i], ref) <= 1e-12


def test_batch_system_range_and_aliasing():
    p = configs.plain(nsys=6, n=9)
    a, b, c, d = configs.full_arrays(p)
    full = oracle.solve_batch(p.layout, 0, a, b, c, d)
    part = oracle.solve_batch(p.layout, 0, a, b, c, d, systems=(2, 4))
    assert np.array_equal(part[18:36], full[18:36])
    assert not part[:18].any() and not part[36:].any()


# ---------------------------------------------------------------------------
# mutation test: the pins must reject a plausibly broken oracle

MUTANTS = {
    "dropped_term": ("m = b[i] - a[i] * cp[i - 1];", "m = b[i];"),
    "wrong_sign": ("dp[i] = (d[i] - a[i] * dp[i - 1]) / m;", "dp[i] = (d[i] + a[i] * dp[i - 1]) / m;"),
    "shifted_index": ("x[i] = dp[i] - cp[i] * x[i + 1];", "x[i] = dp[i] - cp[i + 1] * x[i + 1];"),
    "transposed": ("dp[i] = (d[i] - a[i] * dp[i - 1]) / m;", "dp[i] = (d[i] - c[i - 1] * dp[i - 1]) / m;"),
    "swapped_diagonals": ("m = b[i] - a[i] * cp[i - 1];", "m = b[i] - c[i] * cp[i - 1];"),
    "stale_super": ("cp[i] = (i < n - 1) ? c[i] / m : 0.0;", "cp[i] = (i < n - 1) ? c[i - 1] / m : 0.0;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    old, new = MUTANTS[name]
    # mutate only the FP64 routine (the first occurrence)
    assert old in src
    mutated = src.replace(old, new, 1)
    cfile = tmp_path / "m.c"
    cfile.write_text(mutated)
    so = tmp_path / "libm_.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so),
                    str(cfile), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_thomas.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_int]

    def solve(a, b, c, d):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d)]
        x = np.empty(arrs[3].size)
        rc = lib.oracle_thomas(x.size, *[v.ctypes.data_as(dp) for v in arrs],
                               x.ctypes.data_as(dp), 0)
        if rc != 0:
            raise AssertionError("mutant reported failure")
        return x

    caught = []
    for check in pins.ALL_CHECKS:
        try:
            check(solve)
        except (AssertionError, ZeroDivisionError, FloatingPointError, ValueError):
            caught.append(check.__name__)
    assert caught, f"no pin caught mutant {name}"
