"""GPU parity of the staged, stream-pipelined solve (tdma_solve_partitioned).

Besides oracle parity, every system's arithmetic must not depend on how the
systems are batched or scheduled: results are compared bit for bit across
batch sizes (1, 2, 3 and many batches: pipeline start and end), stream
counts and both schedules -- the race detector for the triple-buffered
workspaces."""
import numpy as np
import pytest

from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _inputs(p, dtype=np.float64):
    tt = torch.float64 if dtype == np.float64 else torch.float32
    a, b, c, d = parity.host_problem(p)
    if dtype == np.float32:
        a, b, c, d = [None if v is None else v.astype(np.float32).astype(np.float64)
                      for v in (a, b, c, d)]
    ref = parity.oracle_solution(p, a, b, c, d)
    coeffs = parity.device_coeffs(p, a, b, c, tt)
    (td,) = parity.to_device([d], tt)
    return ref, coeffs, td


def _solve(p, coeffs, td, **opts):
    import paper_2509_03933_amd as tdma
    tx = torch.full_like(td, float("nan"))
    tdma.solve_partitioned(p.layout, coeffs, td, tx, **opts)
    tdma.check()
    return tx.double().cpu().numpy()


def test_partitioned_perrow_paper_shape():
    """n = 1024 z-systems split into P = 8 partitions of 128 rows (16-row reduced systems)."""
    p = configs.partitioned(24, 20, 1024)
    ref, coeffs, td = _inputs(p)
    x = _solve(p, coeffs, td, partitions=8, batch=128)
    err = parity.per_system_error(p.layout, x, ref)
    assert err.max() <= parity.TOL_F64, err.max()


def test_bit_identical_across_batching_and_streams():
    p = configs.partitioned(30, 17, 300)      # 510 systems
    ref, coeffs, td = _inputs(p)
    base = _solve(p, coeffs, td, partitions=8, batch=510)
    assert parity.per_system_error(p.layout, base, ref).max() <= parity.TOL_F64
    for batch in (1, 7, 255, 256, 170, 509, 4096):
        for nstreams in (1, 2, 4, 8):
            for schedule in (0, 1, 2):
                x = _solve(p, coeffs, td, partitions=8, batch=batch, nstreams=nstreams,
                           schedule=schedule)
                assert np.array_equal(x, base), (batch, nstreams, schedule)


@pytest.mark.parametrize("P", [1, 2, 3, 7, 16, 64, 100, 128])
def test_partition_counts(P):
    """Powers of two up to 64 use the shuffle PCR, others the sequential reduced
    solve; n = 1000 is not a multiple of most P (uneven partitions)."""
    p = configs.partitioned(20, 6, 1000)
    ref, coeffs, td = _inputs(p)
    x = _solve(p, coeffs, td, partitions=P, batch=50)
    err = parity.per_system_error(p.layout, x, ref)
    assert err.max() <= parity.TOL_F64, (P, err.max())


def test_minimum_partition_size():
    p = configs.partitioned(8, 4, 16)       # P = 8 -> every partition has m = 2 rows
    ref, coeffs, td = _inputs(p)
    x = _solve(p, coeffs, td, partitions=8, batch=5)
    assert parity.per_system_error(p.layout, x, ref).max() <= parity.TOL_F64


@pytest.mark.parametrize("make", [lambda: configs.adi(40, 12, 256),
                                  lambda: configs.poisson(32, 16, 512),
                                  lambda: configs.plain(nsys=50, n=300)],
                         ids=["shared", "shared_shift", "contiguous"])
def test_partitioned_coefficient_modes(make):
    p = make()
    ref, coeffs, td = _inputs(p)
    x = _solve(p, coeffs, td, partitions=8, batch=100)
    err = parity.per_system_error(p.layout, x, ref)
    assert err.max() <= parity.TOL_F64, err.max()


def test_partitioned_fp32():
    p = configs.partitioned(24, 10, 512)
    ref, coeffs, td = _inputs(p, np.float32)
    x = _solve(p, coeffs, td, partitions=8, batch=64)
    assert parity.per_system_error(p.layout, x, ref).max() <= parity.TOL_F32


def test_partitioned_in_place():
    import paper_2509_03933_amd as tdma
    p = configs.partitioned(16, 8, 256)
    ref, coeffs, td = _inputs(p)
    tdma.solve_partitioned(p.layout, coeffs, td, td, partitions=4, batch=40)
    tdma.check()
    assert parity.per_system_error(p.layout, td.cpu().numpy(), ref).max() <= parity.TOL_F64


def test_partitioned_rejects_bad_options():
    import paper_2509_03933_amd as tdma
    p = configs.partitioned(4, 4, 10)
    ref, coeffs, td = _inputs(p)
    tx = torch.empty_like(td)
    for kw in (dict(partitions=6), dict(partitions=-1), dict(nstreams=9), dict(schedule=3),
               dict(batch=-5)):
        with pytest.raises(tdma.TdmaError) as ei:
            tdma.solve_partitioned(p.layout, coeffs, td, tx, **kw)
        assert ei.value.status == tdma.EINVAL
