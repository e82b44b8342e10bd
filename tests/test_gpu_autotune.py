"""Autotuner on the GPU: cached shapes keep parity, and the pipeline model's
choice of partition count and batch size is within 5% of the measured best
(the paper reports <= 1.6% for its estimator at full size; this problem is a
quarter of that and its timings are noisier)."""
import numpy as np
import pytest

from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_fused_autotune_then_solve():
    import paper_2509_03933_amd as tdma
    p = configs.adi(64, 32, 256)
    a, b, c, d = parity.host_problem(p)
    coeffs = parity.device_coeffs(p, a, b, c, torch.float64)
    (td,) = parity.to_device([d], torch.float64)
    tx = torch.empty_like(td)
    rec = tdma.autotune(p.layout, coeffs, td, tx, what=0)
    assert rec["path"] == "fused" and len(rec["candidates"]) >= 4
    best = rec["best"]
    assert best["ms"] == min(cand["ms"] for cand in rec["candidates"])
    tx.fill_(float("nan"))
    tdma.solve_batched(p.layout, coeffs, td, tx)      # now uses the cached shape
    tdma.check()
    ref = parity.oracle_solution(p, a, b, c, d)
    assert parity.per_system_error(p.layout, tx.cpu().numpy(), ref).max() <= parity.TOL_F64


def test_partitioned_autotune_model_vs_brute():
    import paper_2509_03933_amd as tdma
    from workloads import device
    # 262,144 systems of n = 512 (~0.13 G unknowns): large enough that stage
    # times, not per-launch overheads, decide the batch size
    p = configs.partitioned(512, 512, 512)
    td, coeffs = device.device_inputs(p)
    tx = torch.empty_like(td)
    rec = tdma.autotune(p.layout, coeffs, td, tx, what=2)
    cands = rec["candidates"]
    assert rec["path"] == "partitioned" and len(cands) >= 2
    assert sorted({c["P"] for c in cands}) == [2, 4, 8, 16, 32]
    by_choice = {(c["P"], c["batch"]): c for c in cands}
    chosen = by_choice[(rec["P"], rec["model_choice"])]["measured_ms"]
    print("autotune", rec)
    assert chosen <= 1.05 * rec["brute_ms"], (chosen, rec["brute_ms"])
    # the cached batch is used and keeps parity on sampled systems
    tx.fill_(float("nan"))
    tdma.solve_partitioned(p.layout, coeffs, td, tx)
    tdma.check()
    import oracle
    x = tx.cpu().numpy()
    for s in (0, 77, p.layout.nsys - 1):
        sa, sb, sc, sd = configs.system_inputs(p, s)
        ref = oracle.thomas(sa, sb, sc, sd)
        got = x[p.layout.sys_rows(s)]
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= parity.TOL_F64
