"""Batching form: a list of solves recorded into one hipGraph.

The three ADI sweeps of one grid are chained (y reads x's output, z reads
y's) beside an independent ragged batch that runs on a parallel branch of
the graph.  Each output is compared with the oracle applied in the same
chain; every item's output must also equal, bit for bit, what
solve_batched gives for the same input (the graph records the same
launches); and the graph is replayed several times with eager work in
between, every replay reproducing the first bit for bit."""
import numpy as np
import pytest

import oracle
from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


def _chain_reference(px, py, pz, R):
    u1 = oracle.solve_batch(px.layout, 1, px.a, px.b, px.c, R)
    u2 = oracle.solve_batch(py.layout, 1, py.a, py.b, py.c, u1)
    u3 = oracle.solve_batch(pz.layout, 1, pz.a, pz.b, pz.c, u2)
    return u1, u2, u3


@pytest.mark.parametrize("grid", [(96, 40, 72), (64, 16, 200)])
def test_graph_adi_sweeps_and_ragged(grid):
    import paper_2509_03933_amd as tdma
    px, py, pz = configs.sweeps(*grid)
    _, _, _, R = configs.full_arrays(px)
    u1r, u2r, u3r = _chain_reference(px, py, pz, R)
    rg = configs.ragged(nsys=257, nmin=2, nmax=3000)
    ra, rb, rc, rd = configs.full_arrays(rg)
    rref = oracle.solve_batch(rg.layout, 0, ra, rb, rc, rd)

    tR = _dev(R)
    u1, u2, u3 = (torch.full_like(tR, float("nan")) for _ in range(3))
    shared = lambda p: dict(mode=1, a=_dev(p.a), b=_dev(p.b), c=_dev(p.c))
    td, tx = _dev(rd), torch.full_like(_dev(rd), float("nan"))
    items = [dict(layout=px.layout, coeffs=shared(px), d=tR, x=u1),
             dict(layout=py.layout, coeffs=shared(py), d=u1, x=u2, after=0),
             dict(layout=pz.layout, coeffs=shared(pz), d=u2, x=u3, after=1),
             dict(layout=rg.layout, coeffs=dict(mode=0, a=_dev(ra), b=_dev(rb), c=_dev(rc)),
                  d=td, x=tx)]
    g = tdma.graph_create(items)
    outs = []
    for rep in range(3):
        for t in (u1, u2, u3, tx):
            t.fill_(float("nan"))              # eager work between replays
        g.launch()
        tdma.check()
        outs.append([t.cpu().numpy() for t in (u1, u2, u3, tx)])
    g.destroy()
    for got, ref, p in zip(outs[0][:3], (u1r, u2r, u3r), (px, py, pz)):
        err = parity.per_system_error(p.layout, got, ref)
        assert err.max() <= parity.TOL_F64, (p.name, err.max())
    err = parity.per_system_error(rg.layout, outs[0][3], rref)
    assert err.max() <= parity.TOL_F64, err.max()
    for rep in (1, 2):
        for a, b in zip(outs[0], outs[rep]):
            assert np.array_equal(a, b)
    # the same launches as solve_batched, item by item, on the same inputs
    # (u1 and u2 still hold the last replay's outputs, equal to the first's)
    chk = torch.empty_like(tR)
    for it, got in zip(items[:3], outs[0][:3]):
        tdma.solve_batched(it["layout"], it["coeffs"], it["d"], chk)
        tdma.check()
        assert np.array_equal(chk.cpu().numpy(), got)
    chk_r = torch.empty_like(td)
    tdma.solve_batched(items[3]["layout"], items[3]["coeffs"], td, chk_r)
    tdma.check()
    assert np.array_equal(chk_r.cpu().numpy(), outs[0][3])


def test_graph_single_item_fp32():
    import paper_2509_03933_amd as tdma
    p = configs.adi(40, 24, 128)
    a, b, c, d = configs.full_arrays(p)
    d32 = d.astype(np.float32)
    ref = oracle.solve_batch(p.layout, 1, p.a.astype(np.float32).astype(np.float64),
                             p.b.astype(np.float32).astype(np.float64),
                             p.c.astype(np.float32).astype(np.float64), d32.astype(np.float64))
    t32 = lambda v: torch.from_numpy(np.ascontiguousarray(v.astype(np.float32))).cuda()
    td = t32(d)
    tx = torch.empty_like(td)
    g = tdma.graph_create([dict(layout=p.layout, coeffs=dict(mode=1, a=t32(p.a), b=t32(p.b),
                                                              c=t32(p.c)), d=td, x=tx)])
    g.launch()
    tdma.check()
    err = parity.per_system_error(p.layout, tx.double().cpu().numpy(), ref)
    assert err.max() <= parity.TOL_F32


def test_graph_keeps_its_tensors_alive():
    """A graph built from temporary coefficient tensors keeps them alive:
    zero-filled tensors of the same sizes allocated after graph_create cannot
    take their memory, so a replay still solves the recorded systems."""
    import gc
    import paper_2509_03933_amd as tdma
    p = configs.adi(40, 24, 128)
    _, _, _, d = configs.full_arrays(p)
    rg = configs.ragged(nsys=64, nmin=2, nmax=500)
    ra, rb, rc, rd = configs.full_arrays(rg)
    td, trd = _dev(d), _dev(rd)
    tx, trx = torch.full_like(td, float("nan")), torch.full_like(trd, float("nan"))
    g = tdma.graph_create([dict(layout=p.layout, coeffs=dict(mode=1, a=_dev(p.a), b=_dev(p.b),
                                                              c=_dev(p.c)), d=td, x=tx),
                           dict(layout=rg.layout, coeffs=dict(mode=0, a=_dev(ra), b=_dev(rb),
                                                               c=_dev(rc)), d=trd, x=trx)])
    gc.collect()
    junk = [torch.zeros(v.size, dtype=torch.float64, device="cuda")
            for v in (p.a, p.b, p.c, ra, rb, rc) for _ in range(2)]
    g.launch()
    tdma.check()
    g.destroy()
    del junk
    ref = oracle.solve_batch(p.layout, 1, p.a, p.b, p.c, d)
    assert parity.per_system_error(p.layout, tx.cpu().numpy(), ref).max() <= parity.TOL_F64
    rref = oracle.solve_batch(rg.layout, 0, ra, rb, rc, rd)
    assert parity.per_system_error(rg.layout, trx.cpu().numpy(), rref).max() <= parity.TOL_F64


def test_graph_rejects_bad_dependencies():
    import paper_2509_03933_amd as tdma
    p = configs.adi(8, 4, 16)
    _, _, _, d = configs.full_arrays(p)
    td = _dev(d)
    tx = torch.empty_like(td)
    co = dict(mode=1, a=_dev(p.a), b=_dev(p.b), c=_dev(p.c))
    with pytest.raises(tdma.TdmaError):
        tdma.graph_create([dict(layout=p.layout, coeffs=co, d=td, x=tx, after=0)])
    with pytest.raises(tdma.TdmaError):
        tdma.graph_create([dict(layout=p.layout, coeffs=co, d=td, x=tx),
                           dict(layout=p.layout, coeffs=co, d=tx, x=td, after=5)])


def test_ragged_solve_refused_under_caller_capture():
    """A ragged solve on a stream the caller is capturing is refused (its plan
    tables are allocated and cached by the library; tdma_graph_create records
    ragged solves), and nothing is left half-recorded."""
    import numpy as np
    import paper_2509_03933_amd as tdma
    from workloads import configs
    r = configs.ragged(nsys=50, nmin=2, nmax=300)
    a, b, c, d = configs.full_arrays(r)
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v)).cuda()
    co = dict(mode=0, a=dev(a), b=dev(b), c=dev(c))
    td = dev(d)
    tx = torch.empty_like(td)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.stream(s):
        try:
            with torch.cuda.graph(g, stream=s):
                tx.fill_(0.0)   # a fill kernel, so the captured graph is not empty
                tdma.solve_batched(r.layout, co, td, tx, stream=s)
        except tdma.TdmaError as e:
            err = e
    torch.cuda.synchronize()
    assert err is not None and err.status == tdma.EUNSUPPORTED, err
    # the same solve outside capture works
    tdma.solve_batched(r.layout, co, td, tx)
    tdma.check()
