"""The no-allocation refined entry point (tdma_solve_refined_noalloc),
called through the C ABI, against tdma_solve_refined on the same inputs: two
calls in a row, the second on a smaller problem, each equal to the
allocating entry point's result and report (same kernels, so bit for bit),
and within the refined bar of the oracle."""
import dataclasses

import numpy as np
import pytest

from tests import parity
from workloads import configs, rng

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _shifted(nx, ny, nz):
    p = configs.adi(nx, ny, nz)
    u = rng.uniform01(p.seed, rng.STREAM_NOISE, np.arange(p.layout.nsys))
    return dataclasses.replace(p, shift=0.5 * u)


def _both(p, **opts):
    import paper_2509_03933_amd as tdma
    a, b, c, d = parity.host_problem(p)
    coeffs = parity.device_coeffs(p, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    x_ref = torch.full_like(td, float("nan"))
    x_na = torch.full_like(td, float("nan"))
    rep_ref = tdma.solve_refined(p.layout, coeffs, td, x_ref, **opts)
    rep_na = tdma.solve_refined(p.layout, coeffs, td, x_na, noalloc=True, **opts)
    tdma.check()
    return x_ref.cpu().numpy(), x_na.cpu().numpy(), rep_ref, rep_na, (a, b, c, d)


def test_noalloc_matches_allocating_entry_point_twice():
    # first call: FFT-Poisson lines with many systems sent to the FP64
    # fallback (the list in the static array is used); second call: a
    # smaller, well-conditioned problem (the array keeps the first call's
    # contents, which the second must not see)
    big = configs.poisson(32, 16, 1024)
    x_ref, x_na, rep_ref, rep_na, _ = _both(big, max_iters=2, tol=1e-13, criterion=1)
    print("poisson lines:", rep_ref, rep_na)
    assert rep_na == rep_ref and rep_ref["fallback_systems"] > 0, (rep_ref, rep_na)
    assert np.array_equal(x_na, x_ref)
    small = _shifted(12, 7, 250)
    x_ref, x_na, rep_ref, rep_na, (a, b, c, d) = _both(small, max_iters=2, tol=1e-13, criterion=1)
    print("shifted ADI:", rep_ref, rep_na)
    assert rep_na == rep_ref and rep_na["fallback_systems"] == 0, (rep_ref, rep_na)
    assert np.array_equal(x_na, x_ref)
    ref = parity.oracle_solution(small, a, b, c, d)
    assert parity.per_system_error(small.layout, x_na, ref).max() <= parity.TOL_REFINED


def test_noalloc_other_operators():
    """The per-row and shared-operator refinement kernels through the same
    entry point (their fallback lists in the static array too)."""
    for p in (configs.partitioned(20, 12, 300), configs.adi(48, 20, 256)):
        x_ref, x_na, rep_ref, rep_na, (a, b, c, d) = _both(p, max_iters=1, tol=1e-15)
        assert rep_na == rep_ref and rep_na["fallback_systems"] == p.layout.nsys, (rep_ref, rep_na)
        assert np.array_equal(x_na, x_ref)
        ref = parity.oracle_solution(p, a, b, c, d)
        assert parity.per_system_error(p.layout, x_na, ref).max() <= parity.TOL_REFINED


def test_noalloc_refuses_aliasing_with_fallback():
    import paper_2509_03933_amd as tdma
    p = configs.adi(16, 8, 64)
    a, b, c, d = parity.host_problem(p)
    coeffs = parity.device_coeffs(p, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    with pytest.raises(tdma.TdmaError) as ei:
        tdma.solve_refined(p.layout, coeffs, td, td, noalloc=True)
    assert ei.value.status == tdma.EINVAL
