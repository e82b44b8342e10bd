"""The lowest FFT-Poisson modes (|kx|, |ky| <= 3, the pinned mode (0, 0)
included) on lines of n = 1024, through every path that solves them: each
mode's error against the FP64 oracle and against the long-double oracle, the
FP64 oracle's own distance from the long-double one, and their ratio, printed
as a table (run with -s to see it) and checked under the conditioned rule of
tests/parity.py.  The ratios printed here are the ones its factor is derived
from."""
import numpy as np
import pytest

from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRID = (32, 16, 1024)


def _dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


def _shared(p):
    co = dict(mode=1, a=_dev(p.a), b=_dev(p.b), c=_dev(p.c))
    if p.shift is not None:
        co["shift"] = _dev(p.shift)
    return co


@pytest.fixture(scope="module")
def real_problem():
    p = configs.poisson(*GRID)
    pin = configs.poisson_pinned(p)
    _, _, _, d = configs.full_arrays(p)
    return p, pin, d


def _table(label, p, pin, x):
    def get(q, s):
        return x[q.layout.sys_rows(int(s))]
    return parity.mode_table(label, parity.poisson_mode_rows(p, get, pin), parity.TOL_F64)


def _solve_real(problem, solve):
    p, pin, d = problem
    td = _dev(d)
    tx = torch.full_like(td, float("nan"))
    solve(p, td, tx)
    solve(pin, td, tx)
    import paper_2509_03933_amd as tdma
    tdma.check()
    return tx.cpu().numpy()


@pytest.mark.parametrize("path", ["default", "shift_k4", "generic_k0", "staged"])
def test_fp64_paths(real_problem, path):
    import paper_2509_03933_amd as tdma

    def solve(q, td, tx):
        co = _shared(q)
        if path == "default":
            tdma.solve_batched(q.layout, co, td, tx)
        elif path == "shift_k4":
            if q.shift is None:   # the pinned mode has no shift: the default kernel
                tdma.solve_batched(q.layout, co, td, tx)
            else:
                tdma.solve_batched_tiled(q.layout, co, td, tx, M=16, S=16, P=64, kernel=4)
        elif path == "generic_k0":
            tdma.solve_batched_tiled(q.layout, co, td, tx, M=8, S=8, P=128, kernel=0)
        else:
            tdma.solve_partitioned(q.layout, co, td, tx)
    x = _solve_real(real_problem, solve)
    p, pin, _ = real_problem
    _table(f"FP64 {path}", p, pin, x)


@pytest.mark.parametrize("opts", [dict(max_iters=2, tol=1e-13, criterion=1),
                                  dict(max_iters=3, tol=1e-15, criterion=0)],
                         ids=["two_steps_criterion1", "three_steps_criterion0"])
def test_refined(real_problem, opts):
    import paper_2509_03933_amd as tdma
    reps = []

    def solve(q, td, tx):
        reps.append(tdma.solve_refined(q.layout, _shared(q), td, tx, **opts))
    x = _solve_real(real_problem, solve)
    p, pin, _ = real_problem
    print("reports", reps)
    _table(f"FP32 + refinement {opts}", p, pin, x)


def test_complex_two_rhs():
    import paper_2509_03933_amd as tdma
    p = configs.poisson_complex(*GRID)
    pin = configs.poisson_complex_pinned(p)
    _, _, _, d = configs.full_arrays(p)
    td = _dev(d)
    tx = torch.full_like(td, float("nan"))
    tdma.solve_multi(p.layout, _shared(p), td, tx, 2, 1)
    tdma.solve_multi(pin.layout, _shared(pin), td, tx, 2, 1)
    tdma.check()
    x = tx.cpu().numpy()

    def get(q, s):
        rows = q.layout.sys_rows(int(s))
        return x[rows] + 1j * x[rows + 1]
    parity.mode_table("FP64 complex (two right-hand sides)",
                      parity.poisson_mode_rows(p, get, pin), parity.TOL_F64)
