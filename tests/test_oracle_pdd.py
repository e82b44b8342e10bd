"""Pins of the oracle's PDD approximation (CPU only).

PDD (Sun 1989, the method the paper uses for its momentum solves, Sec. 5.1)
is an approximation, so its pins are: exactness where the dropped couplings
vanish (one partition; partitions that do not couple), an independent dense
re-computation of the same steps (LAPACK block solves, explicit 2 x 2
solves), the truncation bound (the error against the exact solution is of
the order of the dropped spike tips, which are computed independently by
dense solves) and a mutation test.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from tests import oracle_pins as pins


def _dense_pdd(a, b, c, d, m):
    """The PDD steps with dense LAPACK block solves (numpy), as a second,
    independent computation."""
    n = len(d)
    np_ = (n + m - 1) // m
    xt, v, w = np.zeros(n), np.zeros(n), np.zeros(n)
    for k in range(np_):
        r0, r1 = k * m, min((k + 1) * m, n)
        A = pins.dense(np.r_[0.0, a[r0 + 1:r1]], b[r0:r1], np.r_[c[r0:r1 - 1], 0.0])
        xt[r0:r1] = np.linalg.solve(A, d[r0:r1])
        e = np.zeros(r1 - r0)
        if k > 0:
            e[0] = a[r0]
            v[r0:r1] = np.linalg.solve(A, e)
        if k < np_ - 1:
            e = np.zeros(r1 - r0)
            e[-1] = c[r1 - 1]
            w[r0:r1] = np.linalg.solve(A, e)
    last_x, first_x = {}, {}
    for k in range(np_ - 1):
        l, f = (k + 1) * m - 1, (k + 1) * m
        y = np.linalg.solve(np.array([[1.0, w[l]], [v[f], 1.0]]), np.array([xt[l], xt[f]]))
        last_x[k], first_x[k + 1] = y
    x = np.empty(n)
    for k in range(np_):
        r0, r1 = k * m, min((k + 1) * m, n)
        x[r0:r1] = xt[r0:r1] - v[r0:r1] * last_x.get(k - 1, 0.0) - w[r0:r1] * first_x.get(k + 1, 0.0)
    return x, v, w


def _system(seed, n, margin=(1.0, 2.0)):
    rs = np.random.default_rng(seed)
    return pins.random_dominant(rs, n, margin)


def test_one_partition_is_thomas():
    for seed in range(10):
        a, b, c, d = _system(100 + seed, 50 + seed)
        n = d.size
        for m in (n, n + 5, 4 * n):
            assert np.array_equal(oracle.pdd(a, b, c, d, m), oracle.thomas(a, b, c, d))


def test_decoupled_partitions_are_exact():
    for seed in range(10):
        a, b, c, d = _system(200 + seed, 97)
        m = 8 + seed
        a = a.copy(); c = c.copy()
        a[::m] = 0.0                       # no partition couples to its left
        c[m - 1::m] = 0.0                  # nor to its right
        ref = np.linalg.solve(pins.dense(a, b, c), d)
        assert pins.relerr(oracle.pdd(a, b, c, d, m), ref) <= 1e-14


@pytest.mark.parametrize("m", [2, 3, 5, 8, 16, 33])
def test_matches_dense_steps(m):
    for seed in range(12):
        a, b, c, d = _system(300 + seed, 40 + 7 * seed, margin=(0.2, 1.0))
        ref, _, _ = _dense_pdd(a, b, c, d, m)
        assert pins.relerr(oracle.pdd(a, b, c, d, m), ref) <= 1e-13, (m, seed)


def test_truncation_bound_and_decay():
    """|x_pdd - x| <= 4 * max(dropped tip) * max|x| (tips from dense solves),
    and on a Toeplitz operator the error falls with m."""
    for seed in range(10):
        a, b, c, d = _system(400 + seed, 120, margin=(0.1, 0.5))
        x = np.linalg.solve(pins.dense(a, b, c), d)
        for m in (4, 6, 10, 15):
            _, v, w = _dense_pdd(a, b, c, d, m)
            n, np_ = d.size, (d.size + m - 1) // m
            tips = [abs(v[min((k + 1) * m, n) - 1]) for k in range(1, np_)] + \
                   [abs(w[k * m]) for k in range(1, np_ - 1)]
            tip = max(tips) if tips else 0.0
            err = np.max(np.abs(oracle.pdd(a, b, c, d, m) - x))
            assert err <= 4 * tip * np.max(np.abs(x)) + 1e-14, (seed, m, err, tip)
    n = 240
    a = np.full(n, -1.0); a[0] = 0.0
    c = np.full(n, -1.0); c[-1] = 0.0
    b = np.full(n, 3.0)
    d = np.random.default_rng(5).uniform(-1, 1, n)
    x = oracle.thomas(a, b, c, d)
    errs = [np.max(np.abs(oracle.pdd(a, b, c, d, m) - x)) for m in (4, 8, 12, 24)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    # decay factor of tridiag(-1, 3, -1): ((3 - sqrt 5) / 2)^m per spike tip
    q = (3 - np.sqrt(5)) / 2
    assert errs[1] <= 10 * q ** 8 * np.max(np.abs(x))


MUTANTS = {
    "no_left_correction": ("x[r0 + i] = xt[r0 + i] - v[r0 + i] * left - w[r0 + i] * right;",
                           "x[r0 + i] = xt[r0 + i] - w[r0 + i] * right;"),
    "wrong_sign": ("x[r0 + i] = xt[r0 + i] - v[r0 + i] * left - w[r0 + i] * right;",
                   "x[r0 + i] = xt[r0 + i] + v[r0 + i] * left - w[r0 + i] * right;"),
    "swapped_tips": ("const double det = 1.0 - w[last] * v[first];",
                     "const double det = 1.0 - v[last] * w[first];"),
    "stale_interface": ("yl[2 * k] = (xt[last] - w[last] * xt[first]) / det;",
                        "yl[2 * k] = xt[last];"),
    "shifted_spike": ("if (k > 0) e[0] = a[r0];", "if (k > 0) e[0] = a[r0 + 1];"),
}

CHECKS = [test_one_partition_is_thomas, test_decoupled_partitions_are_exact,
          test_truncation_bound_and_decay]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pdd_pins_reject_mutant(name, tmp_path, monkeypatch):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    old, new = MUTANTS[name]
    start = src.index("int oracle_pdd(")
    end = src.index("void oracle_matvec(")
    body = src[start:end]
    assert old in body
    mutated = src[:start] + body.replace(old, new, 1) + src[end:]
    cfile = tmp_path / "m.c"
    cfile.write_text(mutated)
    so = tmp_path / "libmp.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(so), str(cfile), "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_pdd.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_int64]

    def pdd(a, b, c, d, m):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d)]
        x = np.empty(arrs[3].size)
        if lib.oracle_pdd(x.size, *[v.ctypes.data_as(dp) for v in arrs], x.ctypes.data_as(dp), int(m)):
            raise AssertionError("mutant reported failure")
        return x

    monkeypatch.setattr(oracle, "pdd", pdd)
    caught = []
    for check in CHECKS + [lambda: test_matches_dense_steps(5)]:
        try:
            check()
        except (AssertionError, ZeroDivisionError, FloatingPointError, ValueError, np.linalg.LinAlgError):
            caught.append(getattr(check, "__name__", "dense"))
    assert caught, f"no pin caught mutant {name}"
