"""GPU parity of the rolling shared-operator kernel (kernel 6: one register
set of right-hand sides, refilled with the next tile's rows as Stage C
stores, the row order alternating between tiles) against the oracle and
against the two-set streaming kernel (kernel 2), which runs the same
arithmetic per row.  Shapes cover 8 to 24 rows per lane, tiles of 4 to 64
systems, many tiles per workgroup (both register orders), a last tile only
partly filled, FP32, in-place solves, and the line lengths of the
768 x 512 x 1536 sweeps."""
import numpy as np
import pytest

from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solve(p, shape, dtype=np.float64, inplace=False):
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
SHAPES_256 = [dict(M=16, S=16, P=16), dict(M=16, S=64, P=16), dict(M=8, S=16, P=32),
              dict(M=8, S=4, P=32), dict(M=16, S=32, P=16)]


@pytest.mark.parametrize("shape", SHAPES_256, ids=_ids)
@pytest.mark.parametrize("dtype,tol", [(np.float64, parity.TOL_F64), (np.float32, parity.TOL_F32)],
                         ids=["f64", "f32"])
def test_shapes_n256(shape, dtype, tol):
    """ADI z-lines of n = 256 (P*M = n); 257 x 255 systems: many tiles per
    workgroup and a partly filled last tile."""
    p = configs.adi(257, 255, 256)
    err, x6 = _solve(p, dict(shape, kernel=6), dtype)
    assert err.max() <= tol, err.max()
    if shape["S"] * shape["P"] <= 512:
        _, x2 = _solve(p, dict(shape, kernel=2), dtype)
        assert np.array_equal(x6, x2)


@pytest.mark.parametrize("grid,shape", [((10, 12, 1536), dict(M=24, S=16, P=64)),
                                        ((10, 512, 12), dict(M=16, S=32, P=32)),
                                        ((10, 512, 12), dict(M=16, S=16, P=32)),
                                        ((40, 24, 768), dict(M=12, S=16, P=64))],
                         ids=["z1536_M24", "y512_M16_S32", "y512_M16_S16", "z768_M12"])
def test_sweep_lengths(grid, shape):
    """The line lengths of the 768 x 512 x 1536 sweeps (z-lines of 1536 rows
    with 16 systems of 64 partitions: the shape two register sets cannot
    hold)."""
    px, py, pz = configs.sweeps(*grid)
    p = pz if grid[2] >= 768 else py
    err, _ = _solve(p, dict(shape, kernel=6))
    assert err.max() <= parity.TOL_F64, err.max()


def test_in_place():
    """x aliases d: a tile's next-tile loads are of other systems."""
    err, _ = _solve(configs.adi(64, 32, 256), dict(M=16, S=16, P=16, kernel=6), inplace=True)
    assert err.max() <= parity.TOL_F64, err.max()


def test_needs_exact_cover():
    """Kernel 6 refuses partitions that do not cover n exactly."""
    import paper_2509_03933_amd as tdma
    p = configs.adi(16, 8, 250)
    a, b, c, d = parity.host_problem(p)
    coeffs = parity.device_coeffs(p, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    with pytest.raises(tdma.TdmaError):
        tdma.solve_batched_tiled(p.layout, coeffs, td, torch.empty_like(td), M=16, S=16, P=16,
                                 kernel=6)


def test_refuses_contiguous_rows():
    """Kernel 6 walks strided rows only; contiguous rows are refused."""
    import paper_2509_03933_amd as tdma
    px, _, _ = configs.sweeps(64, 4, 4)
    a, b, c, d = parity.host_problem(px)
    coeffs = parity.device_coeffs(px, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    with pytest.raises(tdma.TdmaError):
        tdma.solve_batched_tiled(px.layout, coeffs, td, torch.empty_like(td), M=16, S=16, P=4, kernel=6)
