"""Parity of tdma_solve_pdd (the PDD approximation in the fused kernel)
against the oracle's PDD on the same partitions, per system; and the
expected relation to the exact solution (one partition: exact; otherwise the
truncation error the oracle's PDD also shows)."""
import numpy as np
import pytest

import oracle
from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lib():
    import paper_2509_03933_amd as tdma
    return tdma


def _dev(v, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(v)).to("cuda", dtype)


def _check(p, m, x, tol, f32=False):
    """Every system against oracle.pdd on the same inputs (FP32-rounded for
    the FP32 path); returns the worst error and the worst distance of the
    oracle's PDD from the exact solution."""
    worst = trunc = 0.0
    for s in range(p.layout.nsys):
        a, b, c, d = configs.system_inputs(p, s)
        if f32:
            a, b, c, d = (v.astype(np.float32).astype(np.float64) for v in (a, b, c, d))
        ref = oracle.pdd(a, b, c, d, m)
        got = x[p.layout.sys_rows(s)]
        e = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        worst = max(worst, e)
        ex = oracle.thomas(a, b, c, d)
        trunc = max(trunc, np.max(np.abs(ref - ex)) / np.max(np.abs(ex)))
    assert worst <= tol, (worst, m)
    return worst, trunc


def _solve(p, m, dtype=torch.float64, inplace=False):
    tdma = _lib()
    a, b, c, d = configs.full_arrays(p)
    td = _dev(d, dtype)
    co = dict(mode=p.mode, a=_dev(a, dtype), b=_dev(b, dtype), c=_dev(c, dtype),
              shift=_dev(p.shift, dtype) if p.shift is not None else None)
    tx = td if inplace else torch.full_like(td, float("nan"))
    tdma.solve_pdd(p.layout, co, td, tx, m)
    tdma.check()
    return tx.double().cpu().numpy()


@pytest.mark.parametrize("m", [4, 8, 16])
def test_perrow_contiguous_and_strided(m):
    # contiguous rows (LDS-staged path), n not a multiple of m, ragged tile tail
    p = configs.plain(nsys=37, n=203)
    w, t = _check(p, m, _solve(p, m), parity.TOL_F64)
    print(f"plain m={m}: vs oracle PDD {w:.2e}, oracle PDD vs exact {t:.2e}")
    # strided z-lines, per-row coefficients
    q = configs.partitioned(12, 5, 150)
    w, t = _check(q, m, _solve(q, m), parity.TOL_F64)
    print(f"z-lines m={m}: vs oracle PDD {w:.2e}, oracle PDD vs exact {t:.2e}")


@pytest.mark.parametrize("m", [8, 16])
def test_shared_operators(m):
    # the ADI operator (shared tables, operator rows in LDS) and the Poisson
    # lines (shared + per-mode shift)
    p = configs.adi(16, 8, 256)
    w, t = _check(p, m, _solve(p, m), parity.TOL_F64)
    print(f"adi m={m}: vs oracle PDD {w:.2e}, oracle PDD vs exact {t:.2e}")
    q = configs.poisson(8, 8, 200)
    q.shift[0] = q.shift[1]
    w, t = _check(q, m, _solve(q, m), parity.TOL_F64)
    print(f"poisson m={m}: vs oracle PDD {w:.2e}, oracle PDD vs exact {t:.2e}")


def test_one_partition_is_exact():
    p = configs.plain(nsys=20, n=16)
    x = _solve(p, 16)
    a, b, c, d = configs.full_arrays(p)
    ref = oracle.solve_batch(p.layout, 0, a, b, c, d)
    assert parity.per_system_error(p.layout, x, ref).max() <= parity.TOL_F64


def test_fp32_and_in_place():
    p = configs.plain(nsys=33, n=500)
    _check(p, 32, _solve(p, 32, torch.float32), parity.TOL_F32, f32=True)
    x = _solve(p, 8, inplace=True)
    _check(p, 8, x, parity.TOL_F64)


def test_errors():
    tdma = _lib()
    p = configs.plain(nsys=4, n=64)
    a, b, c, d = configs.full_arrays(p)
    co = dict(mode=0, a=_dev(a), b=_dev(b), c=_dev(c))
    td = _dev(d)
    tx = torch.empty_like(td)
    for m, status in ((12, tdma.EINVAL), (32, tdma.EINVAL), (0, tdma.EINVAL)):
        with pytest.raises(tdma.TdmaError) as e:
            tdma.solve_pdd(p.layout, co, td, tx, m)
        assert e.value.status == status
    long = configs.Layout(n=8193, nsys0=1, nsys1=1, row_stride=1, sys_stride0=0, sys_stride1=0)
    tl = torch.ones(8193, dtype=torch.float64, device="cuda")
    with pytest.raises(tdma.TdmaError) as e:
        tdma.solve_pdd(long, dict(mode=1, a=tl, b=tl * 3, c=tl), tl, tl.clone(), 4)
    assert e.value.status == tdma.EUNSUPPORTED
