"""The staged path's pipeline model (host logic, CPU only).

Pinned to (1) a literal step-by-step simulation of Algorithm 2's schedule
(oracle/pipeline.py), (2) closed forms, and (3) the paper's Table 2, whose
pipelined-v2 weak-scaling rows show the per-batch time settling at A + C
with Stage B hidden (the steady state of the concurrent model)."""
import os

import numpy as np
import pytest

from oracle import pipeline as sim

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_table2_weak_pipelined_v2.txt")


@pytest.fixture(scope="module")
def tdma():
    import paper_2509_03933_amd as t
    if not os.path.exists(t.LIB_PATH):
        from paper_2509_03933_amd import build
        build.build()
    return t


def test_model_matches_schedule_simulation(tdma):
    rs = np.random.default_rng(5)
    for _ in range(300):
        nsys = int(rs.integers(1, 5000))
        batch = int(rs.integers(1, 800))
        ta, tb, tc = rs.uniform(0.01, 3.0, 3)
        for conc in (0, 1):
            got = tdma.pipeline_model_ms(nsys, batch, ta, tb, tc, conc)
            ref = sim.simulate(nsys, batch, ta, tb, tc, concurrent=bool(conc))
            assert abs(got - ref) <= 1e-9 * max(1.0, ref), (nsys, batch, conc, got, ref)


def test_model_closed_forms(tdma):
    # one batch: the three stages in sequence, whatever the overlap
    for conc in (0, 1):
        assert tdma.pipeline_model_ms(100, 100, 1.0, 2.0, 3.0, conc) == pytest.approx(6.0)
    # sequential reading: every stage runs once per batch
    assert tdma.pipeline_model_ms(1000, 10, 1.0, 0.5, 0.25, 0) == pytest.approx(100 * 1.75)
    # concurrent with B shorter than A and C: steps cost A, A, (A+C) x (N_b-2), C, C,
    # i.e. B is hidden completely and the total is N_b (A + C)
    nb = 50
    got = tdma.pipeline_model_ms(nb * 7, 7, 4.0, 1.0, 2.0, 1)
    assert got == pytest.approx(nb * (4.0 + 2.0))
    # concurrent with B longer than A + C: B dominates every middle step
    got = tdma.pipeline_model_ms(nb, 1, 1.0, 5.0, 1.0, 1)
    assert got == pytest.approx(1.0 + nb * 5.0 + 1.0)


def test_steady_state_matches_paper_table2(tdma):
    """Per-batch time of the concurrent model for many batches -> max(A + C, B);
    the paper's measured totals sit within 1.5% of A + C on these rows."""
    rows = [list(map(float, l.split())) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    nb = 10000
    for gpus, total, a, c, b, comm in rows:
        per_batch = tdma.pipeline_model_ms(nb, 1, a, b, c, 1) / nb
        assert per_batch == pytest.approx(max(a + c, b), rel=1e-3)
        assert abs(per_batch - total) / total <= 0.015, (gpus, per_batch, total)
        # the sequential reading would not hide B
        seq = tdma.pipeline_model_ms(nb, 1, a, b, c, 0) / nb
        assert seq > total
