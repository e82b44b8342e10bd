"""GPU parity of the per-row streaming kernel (kernel 5: a, b, c laid out
like d on strided layouts, the per-row z-lines) against the oracle, through
tdma_solve_batched and tdma_solve_batched_tiled.

Workgroups walk tiles of S systems x P partitions x M rows; each lane
consumes its rows through a window of loads in flight and keeps three
values per interior row.  Shapes cover P*M == n (no padding) and padded
lengths down to partitions wholly past the end, tile widths from one to 16
systems, last tiles only partly filled, walks of several tiles per
workgroup, M = 16 and 32, FP32, and in-place solves."""
import dataclasses

import numpy as np
import pytest

from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve(p, shape=None, dtype=np.float64, inplace=False):
    import paper_2509_03933_amd as tdma
    tt = torch.float64 if dtype == np.float64 else torch.float32
    a, b, c, d = parity.host_problem(p)
    if dtype == np.float32:
        a, b, c, d = [v.astype(np.float32).astype(np.float64) for v in (a, b, c, d)]
    ref = parity.oracle_solution(p, a, b, c, d)
    coeffs = parity.device_coeffs(p, a, b, c, tt)
    (td,) = parity.to_device([d], tt)
    tx = td if inplace else torch.full_like(td, float("nan"))
    if shape is None:
        tdma.solve_batched(p.layout, coeffs, td, tx)
    else:
        tdma.solve_batched_tiled(p.layout, coeffs, td, tx, **shape)
    tdma.check()
    x = tx.double().cpu().numpy()
    return parity.per_system_error(p.layout, x, ref), x


_ids = lambda s: "M%d_S%d_P%d" % (s["M"], s["S"], s["P"])
SHAPES_1024 = [dict(M=16, S=16, P=64), dict(M=32, S=16, P=32), dict(M=16, S=8, P=64),
               dict(M=16, S=1, P=64), dict(M=32, S=4, P=32), dict(M=32, S=2, P=64)]


@pytest.mark.parametrize("shape", SHAPES_1024, ids=_ids)
def test_shapes_fp64_n1024(shape):
    """n = 1024 (padded when P*M > n); 20 x 11 systems leave the last tile
    partly filled for every tile width above 4."""
    err, _ = _solve(configs.partitioned(20, 11, 1024), dict(shape, kernel=5))
    assert err.max() <= parity.TOL_F64, err.max()


@pytest.mark.parametrize("nz", [1000, 700, 250, 100, 33, 17])
@pytest.mark.parametrize("M", [16, 32])
def test_padded_lengths_fp64(nz, M):
    """Lengths that leave identity padding rows, including partitions that lie
    wholly past the end of the system (n = 17 with P = 2 x 16 rows: the
    second partition has one row; n = 700 with P = 64 x 16: the last 20
    partitions have none)."""
    P = 2
    while P * M < nz:
        P *= 2
    maxt = 512 if M == 32 else 1024
    S = min(16, maxt // P)
    err, _ = _solve(configs.partitioned(12, 7, nz), dict(M=M, S=S, P=P, kernel=5))
    assert err.max() <= parity.TOL_F64, (nz, err.max())


def test_default_plan_perrow_lines():
    """The built-in plan takes kernel 5 for per-row strided layouts; many
    tiles per workgroup (40 x 26 systems of n = 1024)."""
    err, _ = _solve(configs.partitioned(40, 26, 1024))
    assert err.max() <= parity.TOL_F64, err.max()


@pytest.mark.parametrize("shape", [None, dict(M=16, S=16, P=64, kernel=5), dict(M=32, S=16, P=32, kernel=5)],
                         ids=["default", "M16", "M32"])
def test_fp32(shape):
    err, _ = _solve(configs.partitioned(18, 10, 1024), shape, np.float32)
    assert err.max() <= parity.TOL_F32, err.max()


@pytest.mark.parametrize("shape", [dict(M=16, S=16, P=64, kernel=5), dict(M=16, S=16, P=32, kernel=5)],
                         ids=["full", "padded"])
def test_in_place(shape):
    """x aliases d: a tile reads all its rows (and the next tile's first rows)
    before it writes any of its own."""
    err, _ = _solve(configs.partitioned(16, 16, 1000 if shape["P"] == 64 else 500), shape,
                    inplace=True)
    assert err.max() <= parity.TOL_F64, err.max()


def test_needs_perrow_coefficients():
    import paper_2509_03933_amd as tdma
    p = configs.adi(8, 8, 64)
    a, b, c, d = parity.host_problem(p)
    coeffs = parity.device_coeffs(p, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    with pytest.raises(tdma.TdmaError):
        tdma.solve_batched_tiled(p.layout, coeffs, td, torch.empty_like(td), M=16, S=16, P=4,
                                 kernel=5)


def test_singular_pivot_flagged():
    """A zero pivot in one system sets the flag (and only the solve reports it)."""
    import paper_2509_03933_amd as tdma
    p = configs.partitioned(16, 4, 256)
    a, b, c, d = parity.host_problem(p)
    rows = p.layout.sys_rows(5)
    a, b, c = a.copy(), b.copy(), c.copy()
    b[rows[0]] = 0.0
    coeffs = parity.device_coeffs(p, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    tdma.solve_batched_tiled(p.layout, coeffs, td, torch.empty_like(td), M=16, S=16, P=16, kernel=5)
    with pytest.raises(tdma.TdmaError):
        tdma.check()
