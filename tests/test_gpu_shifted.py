"""GPU parity of the shifted-operator streaming kernel (shared a, b, c tables
plus a per-system diagonal shift on strided layouts: the FFT-Poisson lines)
against the oracle, through tdma_solve_batched and tdma_solve_batched_tiled.

kernel 3 walks the tiles loading the next tile's rows as the current one is
stored, kernel 4 loads each tile at its start; both keep d and the pivot
reciprocals per row and re-solve the partition interior from d in Stage C.
Kernel 7 (FP64, partitions covering n) keeps d alone and recomputes the
pivots in Stage C, in workgroups of up to 1024 lanes.  Shapes cover P*M == n (no padding) and padded lengths,
tile widths from one to 32 systems, a last tile that is only partly filled,
M = 8, 16 (and 32 in FP32), FP32, and in-place solves."""
import dataclasses

import numpy as np
import pytest

from tests import parity
from workloads import configs, rng

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _shifted(nx, ny, nz, lo=0.0, hi=0.5):
    """The ADI operator plus a seeded per-system diagonal shift in [lo, hi)."""
    p = configs.adi(nx, ny, nz)
    u = rng.uniform01(p.seed, rng.STREAM_NOISE, np.arange(p.layout.nsys))
    return dataclasses.replace(p, shift=lo + (hi - lo) * u)


def _solve(p, shape=None, dtype=np.float64, inplace=False):
    import paper_2509_03933_amd as tdma
    tt = torch.float64 if dtype == np.float64 else torch.float32
    a, b, c, d = parity.host_problem(p)
    if dtype == np.float32:
        a, b, c, d = [v.astype(np.float32).astype(np.float64) for v in (a, b, c, d)]
        p = dataclasses.replace(p, shift=p.shift.astype(np.float32).astype(np.float64))
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


SHAPES_1024 = [dict(M=16, S=16, P=64, kernel=3), dict(M=16, S=16, P=64, kernel=4),
               dict(M=16, S=8, P=64, kernel=3), dict(M=16, S=1, P=64, kernel=4),
               dict(M=16, S=4, P=64, kernel=3), dict(M=32, S=16, P=32, kernel=3),
               dict(M=32, S=16, P=32, kernel=4), dict(M=32, S=8, P=32, kernel=3),
               dict(M=32, S=2, P=64, kernel=3), dict(M=32, S=32, P=32, kernel=7),
               dict(M=32, S=16, P=32, kernel=7), dict(M=16, S=16, P=64, kernel=7),
               dict(M=32, S=4, P=32, kernel=7), dict(M=16, S=1, P=64, kernel=7)]
SHAPES_512 = [dict(M=8, S=16, P=64, kernel=3), dict(M=16, S=32, P=32, kernel=3),
              dict(M=16, S=16, P=32, kernel=4), dict(M=8, S=2, P=64, kernel=4),
              dict(M=16, S=32, P=32, kernel=7), dict(M=32, S=32, P=16, kernel=7),
              dict(M=32, S=16, P=16, kernel=3), dict(M=32, S=4, P=16, kernel=4)]
_ids = lambda s: "k%d_M%d_S%d_P%d" % (s["kernel"], s["M"], s["S"], s["P"])


@pytest.mark.parametrize("shape", SHAPES_1024, ids=_ids)
def test_shapes_fp64_n1024(shape):
    """n = 1024 = P*M (no padding); 20 x 11 systems leave the last tile
    partly filled for every tile width above 4."""
    err, _ = _solve(_shifted(20, 11, 1024), shape)
    assert err.max() <= parity.TOL_F64, err.max()


@pytest.mark.parametrize("shape", SHAPES_512, ids=_ids)
def test_shapes_fp64_n512(shape):
    err, _ = _solve(_shifted(24, 9, 512), shape)
    assert err.max() <= parity.TOL_F64, err.max()


@pytest.mark.parametrize("nz", [1000, 250, 100, 48, 16, 5])
@pytest.mark.parametrize("kernel,M", [(3, 16), (4, 16), (3, 32), (4, 32)])
def test_padded_lengths_fp64(nz, kernel, M):
    """Lengths that leave identity padding rows in the last partition(s)."""
    p = _shifted(12, 7, nz)
    P = 1
    while P * M < nz:
        P *= 2
    err, _ = _solve(p, dict(M=M, S=16, P=P, kernel=kernel))
    assert err.max() <= parity.TOL_F64, (nz, err.max())


def test_default_plan_n512_lines():
    """Lines of 512 rows: the built-in plan takes 32 rows per lane, 16
    partitions and 32-system tiles (the interface solve in its DPP form)."""
    p = configs.poisson(40, 30, 512)
    err, x = _solve(p)
    for s in np.nonzero(err > parity.TOL_F64)[0]:
        if s == 0:
            continue   # mode (0, 0) carries a placeholder shift in the bulk call
        sa, sb, sc, sd = configs.system_inputs(p, int(s))
        ok, e64, eld, eorc = parity.conditioned_error(x[p.layout.sys_rows(int(s))], sa, sb, sc, sd,
                                                      parity.TOL_F64)
        assert ok, (int(s), e64, eld, eorc)


def test_default_plan_poisson_lines():
    """The built-in plan for the FFT-Poisson lines takes the shifted kernel;
    every mode is checked (the ill-conditioned low modes against the
    long-double oracle)."""
    p = configs.poisson(32, 16, 1024)
    err, x = _solve(p)
    for s in np.nonzero(err > parity.TOL_F64)[0]:
        if s == 0:
            continue   # mode (0, 0) carries a placeholder shift in the bulk call
        sa, sb, sc, sd = configs.system_inputs(p, int(s))
        ok, e64, eld, eorc = parity.conditioned_error(x[p.layout.sys_rows(int(s))], sa, sb, sc, sd,
                                                      parity.TOL_F64)
        assert ok, (int(s), e64, eld, eorc)


def test_same_results_both_register_forms():
    """Kernels 3 and 4 run the same arithmetic per tile: identical results."""
    p = _shifted(33, 9, 512)
    _, x3 = _solve(p, dict(M=16, S=16, P=32, kernel=3))
    _, x4 = _solve(p, dict(M=16, S=16, P=32, kernel=4))
    assert np.array_equal(x3, x4)


@pytest.mark.parametrize("shape", [None, dict(M=32, S=32, P=32, kernel=3),
                                   dict(M=16, S=16, P=64, kernel=4), dict(M=8, S=16, P=64, kernel=3)],
                         ids=["default", "k3_M32_S32_P32", "k4_M16_S16_P64", "k3_M8_S16_P64"])
def test_fp32(shape):
    p = _shifted(18, 10, 512)
    if shape is not None and shape["M"] * shape["P"] < 512:
        pytest.skip("shape does not cover n")
    err, _ = _solve(p, shape, np.float32)
    assert err.max() <= parity.TOL_F32, err.max()


def test_same_results_recomputed_pivots():
    """Kernel 7 recomputes the pivots of kernel 3 with the same operations
    (and walks 32-system tiles): identical results, many tiles per
    workgroup, a partly filled last tile."""
    p = _shifted(61, 37, 1024)
    _, x3 = _solve(p, dict(M=32, S=16, P=32, kernel=3))
    _, x7 = _solve(p, dict(M=32, S=32, P=32, kernel=7))
    assert np.array_equal(x3, x7)


def test_recomputed_pivots_rules():
    """Kernel 7 takes FP64 with partitions covering n, at most 1024 lanes."""
    import paper_2509_03933_amd as tdma
    for p, shape, tt in [(_shifted(8, 8, 1000), dict(M=32, S=16, P=32), torch.float64),
                         (_shifted(8, 8, 1024), dict(M=32, S=32, P=32), torch.float32),
                         (_shifted(8, 8, 1024), dict(M=16, S=32, P=64), torch.float64)]:
        a, b, c, d = parity.host_problem(p)
        coeffs = parity.device_coeffs(p, a, b, c, tt)
        (td,) = parity.to_device([d], tt)
        with pytest.raises(tdma.TdmaError) as ei:
            tdma.solve_batched_tiled(p.layout, coeffs, td, torch.empty_like(td), kernel=7, **shape)
        assert ei.value.status == tdma.EINVAL


@pytest.mark.parametrize("kernel", [3, 4, 7])
def test_in_place(kernel):
    """x aliases d: a tile reads all its rows before it writes any."""
    p = _shifted(16, 16, 256)
    err, _ = _solve(p, dict(M=16, S=16, P=16, kernel=kernel), inplace=True)
    assert err.max() <= parity.TOL_F64, err.max()


def test_weakly_dominant_shift():
    """Shifts near zero on the Poisson operator (the lowest modes' regime):
    every system checked, the ill-conditioned ones under the conditioned rule."""
    p = configs.poisson(16, 8, 512)
    err, x = _solve(p, dict(M=16, S=16, P=32, kernel=4))
    for s in np.nonzero(err > parity.TOL_F64)[0]:
        if s == 0:
            continue
        sa, sb, sc, sd = configs.system_inputs(p, int(s))
        ok, e64, eld, eorc = parity.conditioned_error(x[p.layout.sys_rows(int(s))], sa, sb, sc, sd,
                                                      parity.TOL_F64)
        assert ok, (int(s), e64, eld, eorc)


def test_shifted_kernel_needs_a_shift():
    import paper_2509_03933_amd as tdma
    p = configs.adi(8, 8, 64)
    a, b, c, d = parity.host_problem(p)
    coeffs = parity.device_coeffs(p, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    with pytest.raises(tdma.TdmaError) as ei:
        tdma.solve_batched_tiled(p.layout, coeffs, td, torch.empty_like(td), M=16, S=16, P=4, kernel=3)
    assert ei.value.status == tdma.EINVAL


# --- the precision form on the shifted operator (tdma_solve_refined takes the
# shifted-operator refinement kernel for these layouts)

def _refined(p, **opts):
    import paper_2509_03933_amd as tdma
    a, b, c, d = parity.host_problem(p)
    coeffs = parity.device_coeffs(p, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    tx = torch.full_like(td, float("nan"))
    rep = tdma.solve_refined(p.layout, coeffs, td, tx, **opts)
    tdma.check()
    ref = parity.oracle_solution(p, a, b, c, d)
    return parity.per_system_error(p.layout, tx.cpu().numpy(), ref), rep, tx.cpu().numpy()


@pytest.mark.parametrize("grid", [(20, 11, 1024), (24, 9, 1000), (40, 13, 512), (7, 3, 100)],
                         ids=["n1024", "n1000_padded", "n512", "n100_padded"])
def test_refined_well_conditioned(grid):
    """Two steps at tol 1e-12 (the benchmark's setting) on the ADI operator
    with per-system shifts: the 1e-12 bar without fallback, for lengths that
    fill the partitions and lengths that leave padding rows, and tile counts
    that leave the last tile partly filled."""
    err, rep, _ = _refined(_shifted(*grid), max_iters=2, tol=1e-12, criterion=1)
    assert err.max() <= parity.TOL_REFINED, err.max()
    assert rep["fallback_systems"] == 0, rep


def test_refined_three_steps_tight_tol():
    err, rep, _ = _refined(_shifted(16, 16, 1024), max_iters=3, tol=1e-15)
    assert err.max() <= parity.TOL_REFINED, err.max()
    assert rep["not_converged"] == 0, rep


def test_refined_poisson_lines():
    """The FFT-Poisson lines (n = 1024) in the benchmark's setting (two
    steps, tol 1e-13, criterion 1; the predicted error is an estimate, so the
    tolerance sits a decade under the bar): every mode within the bar against
    the FP64 oracle, or, for the ill-conditioned low modes, within the
    conditioned rule against the long-double oracle."""
    p = configs.poisson(32, 16, 1024)
    err, rep, x = _refined(p, max_iters=2, tol=1e-13, criterion=1)
    for s in np.nonzero(err > parity.TOL_F64)[0]:
        if s == 0:
            continue   # mode (0, 0) carries a placeholder shift in the bulk call
        sa, sb, sc, sd = configs.system_inputs(p, int(s))
        ok, e64, eld, eorc = parity.conditioned_error(x[p.layout.sys_rows(int(s))], sa, sb, sc, sd,
                                                      parity.TOL_F64)
        assert ok, (int(s), e64, eld, eorc, rep)


def test_refined_no_steps_is_plain_fp32():
    """max_iters 0 without fallback: one FP32 solve, within the plain FP32
    bar against the oracle on the FP64 inputs."""
    import paper_2509_03933_amd as tdma
    p = _shifted(16, 8, 1024)
    a, b, c, d = parity.host_problem(p)
    coeffs = parity.device_coeffs(p, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    tx = torch.empty_like(td)
    tdma.solve_refined(p.layout, coeffs, td, tx, max_iters=0, fallback=0, report=False)
    torch.cuda.synchronize()
    ref = parity.oracle_solution(p, a, b, c, d)
    assert parity.per_system_error(p.layout, tx.cpu().numpy(), ref).max() <= parity.TOL_F32
