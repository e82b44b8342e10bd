"""Parity of tdma_solve_multi (several right-hand sides over one shared
operator) against the oracle.

The complex Poisson lines (real operator, complex right-hand side stored as
interleaved (re, im) pairs) are checked against the oracle's complex Thomas
solve; general right-hand-side counts and strides against the oracle's real
solve of each right-hand side.  Sizes span several tiles and a ragged tail;
edge cases cover n = 2, one system, no systems, the longest supported n, odd
right-hand-side counts, in-place solves and the argument errors."""
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


def _coeffs(p, dtype=torch.float64, shift=True):
    return dict(mode=1, a=_dev(p.a, dtype), b=_dev(p.b, dtype), c=_dev(p.c, dtype),
                shift=_dev(p.shift, dtype) if (shift and p.shift is not None) else None)


def _complex_ref(p, d):
    lay = configs.complex_layout(p)
    dz = d[0::2] + 1j * d[1::2]
    return oracle.solve_batch_complex(lay, p.a, p.b, p.c, dz, shift=p.shift), lay


def _per_system_complex(lay, xz, refz):
    X = parity.gather_rows(lay, xz)
    R = parity.gather_rows(lay, refz)
    return np.max(np.abs(X - R), axis=1) / np.maximum(np.max(np.abs(R), axis=1), 1e-300)


@pytest.mark.parametrize("grid", [(16, 8, 1024), (12, 7, 1000), (9, 5, 77), (33, 3, 16),
                                  (5, 4, 2), (40, 40, 256)])
def test_complex_poisson_lines(grid):
    """Interleaved complex right-hand sides (vector path) against the complex
    oracle; mode (0, 0) carries a placeholder shift and is compared too."""
    tdma = _lib()
    p = configs.poisson_complex(*grid)
    _, _, _, d = configs.full_arrays(p)
    ref, clay = _complex_ref(p, d)
    td = _dev(d)
    tx = torch.full_like(td, float("nan"))
    tdma.solve_multi(p.layout, _coeffs(p), td, tx, 2, 1)
    tdma.check()
    x = tx.cpu().numpy()
    err = _per_system_complex(clay, x[0::2] + 1j * x[1::2], ref)
    print(f"{grid}: {clay.nsys} complex systems, max rel err {err.max():.3e}", flush=True)
    # well-conditioned bulk to the FP64 bar; the lowest modes via the
    # long-double oracle (their kappa grows like n^2 / |k|^2)
    nx, ny, n = grid
    bad = np.nonzero(err > parity.TOL_F64)[0]
    for s in bad:
        rows = clay.sys_rows(int(s))
        ok, e64, eld, eorc = parity.conditioned_error_complex(
            x[2 * rows] + 1j * x[2 * rows + 1], p.a, p.b + p.shift[s], p.c,
            d[2 * rows] + 1j * d[2 * rows + 1], parity.TOL_F64)
        print(f"mode {int(s)}: {e64:.2e} vs FP64 oracle, {eld} vs long double ({eorc})")
        assert ok, (int(s), e64, eld, eorc)


def test_complex_entry_point_with_complex_tensors():
    tdma = _lib()
    p = configs.poisson_complex(24, 10, 300)
    _, _, _, d = configs.full_arrays(p)
    ref, clay = _complex_ref(p, d)
    dz = torch.from_numpy(d[0::2] + 1j * d[1::2]).cuda()
    xz = torch.empty_like(dz)
    tdma.solve_complex(clay, _coeffs(p), dz, xz)
    tdma.check()
    err = _per_system_complex(clay, xz.cpu().numpy(), ref)
    assert err[1:].max() <= parity.TOL_F64, err.max()


def _planes_problem(nx, ny, n, nrhs, seed):
    """nrhs right-hand-side planes (rhs_stride = one plane) of z-lines over
    the Poisson operator with a per-mode shift."""
    base = configs.poisson(nx, ny, n)
    rs = np.random.default_rng(seed)
    lay = configs.zsys_layout(nx, ny, n)
    plane = lay.extent()
    d = rs.uniform(-1, 1, plane * nrhs)
    return base, lay, plane, d


def _oracle_planes(base, lay, plane, d, nrhs, shift=True):
    out = np.zeros_like(d)
    for r in range(nrhs):
        out[r * plane:(r + 1) * plane] = oracle.solve_batch(
            lay, 1, base.a, base.b, base.c, d[r * plane:(r + 1) * plane],
            shift=base.shift if shift else None)
    return out


@pytest.mark.parametrize("nrhs", [1, 2, 3, 5])
def test_rhs_planes_fp64(nrhs):
    """Right-hand sides one plane apart (scalar path, odd counts run a single
    right-hand side last) against the oracle's solve of each plane."""
    tdma = _lib()
    base, lay, plane, d = _planes_problem(20, 9, 200, nrhs, 40 + nrhs)
    ref = _oracle_planes(base, lay, plane, d, nrhs)
    td = _dev(d)
    tx = torch.full_like(td, float("nan"))
    tdma.solve_multi(lay, _coeffs(base), td, tx, nrhs, plane)
    tdma.check()
    x = tx.cpu().numpy()
    for r in range(nrhs):
        sl = slice(r * plane, (r + 1) * plane)
        err = parity.per_system_error(lay, x[sl], ref[sl])
        assert err[1:].max() <= parity.TOL_F64, (r, err.max())


def test_rhs_planes_fp32_no_shift():
    """FP32 storage and sweeps (FP64 interface solve) without a shift: the
    FP32-rounded problem against the oracle to the FP32 bar."""
    tdma = _lib()
    nrhs = 3
    base, lay, plane, d = _planes_problem(17, 6, 700, nrhs, 7)
    d32 = d.astype(np.float32).astype(np.float64)
    a, b, c = (v.astype(np.float32).astype(np.float64) for v in (base.a, base.b, base.c))
    # without the per-mode shift the Neumann operator is singular: make it
    # strictly dominant (its diagonal is negative, its off-diagonals positive)
    b = b - 0.5 * np.abs(b)
    b32 = b.astype(np.float32).astype(np.float64)
    ref = np.zeros_like(d32)
    for r in range(nrhs):
        sl = slice(r * plane, (r + 1) * plane)
        ref[sl] = oracle.solve_batch(lay, 1, a, b32, c, d32[sl])
    co = dict(mode=1, a=_dev(a, torch.float32), b=_dev(b32, torch.float32),
              c=_dev(c, torch.float32))
    td = _dev(d32, torch.float32)
    tx = torch.full_like(td, float("nan"))
    tdma.solve_multi(lay, co, td, tx, nrhs, plane)
    tdma.check()
    x = tx.double().cpu().numpy()
    for r in range(nrhs):
        sl = slice(r * plane, (r + 1) * plane)
        err = parity.per_system_error(lay, x[sl], ref[sl])
        assert err.max() <= parity.TOL_F32, (r, err.max())


def test_complex_fp32_interleaved():
    """FP32 interleaved complex right-hand sides (vector path, M = 32, P = 64
    at n = 2048) over a well-conditioned operator: the ADI viscous tables of
    the same n with a positive per-mode shift (the Poisson lines' condition
    numbers, ~1e5 at this n, are beyond plain FP32; the precision form covers
    them).  The FP32-rounded problem against the complex oracle."""
    from workloads import grids
    tdma = _lib()
    p = configs.poisson_complex(16, 16, 2048)
    _, _, _, d = configs.full_arrays(p)
    rs = np.random.default_rng(17)
    f32 = lambda v: np.asarray(v).astype(np.float32).astype(np.float64)
    a, b, c = (f32(v) for v in grids.adi_viscous_coeffs(2048, 2.0, 0.5))
    sh = f32(rs.uniform(0.0, 1.0, p.layout.nsys))
    d32 = f32(d)
    clay = configs.complex_layout(p)
    ref = oracle.solve_batch_complex(clay, a, b, c, d32[0::2] + 1j * d32[1::2], shift=sh)
    co = dict(mode=1, a=_dev(a, torch.float32), b=_dev(b, torch.float32),
              c=_dev(c, torch.float32), shift=_dev(sh, torch.float32))
    td = _dev(d32, torch.float32)
    tx = torch.full_like(td, float("nan"))
    tdma.solve_multi(p.layout, co, td, tx, 2, 1)
    tdma.check()
    x = tx.double().cpu().numpy()
    err = _per_system_complex(clay, x[0::2] + 1j * x[1::2], ref)
    print(f"FP32 complex n = 2048: max rel err {err.max():.3e}", flush=True)
    assert err.max() <= parity.TOL_F32, err.max()


def test_vector_and_scalar_paths_bit_identical():
    """The pair-vector access changes only the loads and stores: a d and x
    one element off a pair boundary (scalar path) give identical bits."""
    tdma = _lib()
    p = configs.poisson_complex(10, 6, 130)
    _, _, _, d = configs.full_arrays(p)
    co = _coeffs(p)
    td = _dev(d)
    tx = torch.empty_like(td)
    tdma.solve_multi(p.layout, co, td, tx, 2, 1)
    big = torch.zeros(d.size + 1, dtype=torch.float64, device="cuda")
    big[1:] = td
    bx = torch.zeros_like(big)
    tdma.solve_multi(p.layout, co, big[1:], bx[1:], 2, 1)
    tdma.check()
    assert torch.equal(tx, bx[1:])


def test_matches_single_rhs_solver():
    """Two right-hand sides against tdma_solve_batched on each one (the real
    and imaginary systems as their own layouts): same problem, another kernel."""
    tdma = _lib()
    p = configs.poisson_complex(32, 16, 512)
    _, _, _, d = configs.full_arrays(p)
    co = _coeffs(p)
    td = _dev(d)
    tx = torch.empty_like(td)
    tdma.solve_multi(p.layout, co, td, tx, 2, 1)
    ty = torch.empty_like(td)
    tdma.solve_batched(p.layout, co, td, ty)
    tdma.solve_batched(p.layout, co, td[1:], ty[1:])
    tdma.check()
    x, y = tx.cpu().numpy(), ty.cpu().numpy()
    # the two kernels round in different orders; the lowest modes amplify
    # that by their condition number (measured up to 5.2e-13 here)
    err = parity.per_system_error(p.layout, x, y)
    assert err[1:].max() <= parity.TOL_F64, err.max()


def test_in_place_and_edges():
    tdma = _lib()
    # in place: x aliases d
    p = configs.poisson_complex(8, 8, 96)
    _, _, _, d = configs.full_arrays(p)
    ref, clay = _complex_ref(p, d)
    td = _dev(d)
    tdma.solve_multi(p.layout, _coeffs(p), td, td, 2, 1)
    tdma.check()
    x = td.cpu().numpy()
    err = _per_system_complex(clay, x[0::2] + 1j * x[1::2], ref)
    assert err[1:].max() <= parity.TOL_F64
    # one system, and no systems
    one = configs.Layout(n=50, nsys0=1, nsys1=1, row_stride=2, sys_stride0=0, sys_stride1=0)
    rs = np.random.default_rng(3)
    a = np.r_[0.0, rs.uniform(-1, 0, 49)]
    c = np.r_[rs.uniform(-1, 0, 49), 0.0]
    b = 2.5 + np.abs(a) + np.abs(c)
    dd = rs.uniform(-1, 1, 100)
    co = dict(mode=1, a=_dev(a), b=_dev(b), c=_dev(c))
    td = _dev(dd)
    tx = torch.empty_like(td)
    tdma.solve_multi(one, co, td, tx, 2, 1)
    tdma.check()
    got = tx.cpu().numpy()
    refz = oracle.thomas_complex(a, b, c, dd[0::2] + 1j * dd[1::2])
    assert np.max(np.abs(got[0::2] + 1j * got[1::2] - refz)) / np.max(np.abs(refz)) <= parity.TOL_F64
    empty = configs.Layout(n=50, nsys0=0, nsys1=1, row_stride=2, sys_stride0=0, sys_stride1=0)
    tdma.solve_multi(empty, co, td, tx, 2, 1)
    tdma.check()


def test_argument_errors():
    tdma = _lib()
    p = configs.poisson_complex(4, 4, 64)
    _, _, _, d = configs.full_arrays(p)
    co = _coeffs(p)
    td = _dev(d)
    tx = torch.empty_like(td)
    for nrhs, stride, status in ((0, 1, tdma.EINVAL), (2, 0, tdma.EINVAL), (2, -1, tdma.EINVAL)):
        with pytest.raises(tdma.TdmaError) as e:
            tdma.lib()  # loaded
            L = tdma._make_layout(p.layout, [])
            C = tdma._make_coeffs(p.layout, co, td, 1)
            import ctypes
            tdma._raise(tdma.lib().tdma_solve_multi(ctypes.byref(L), ctypes.byref(C), tdma.F64,
                                                    nrhs, stride, ctypes.c_void_p(td.data_ptr()),
                                                    ctypes.c_void_p(tx.data_ptr()), None))
        assert e.value.status == status
    # per-row coefficients are not shared by the right-hand sides
    with pytest.raises(tdma.TdmaError) as e:
        rowco = dict(mode=0, a=td, b=td, c=td)
        tdma.solve_multi(p.layout, rowco, td, tx, 2, 1)
    assert e.value.status == tdma.EUNSUPPORTED
    # longer than 1024 rows in FP64
    long = configs.Layout(n=1025, nsys0=2, nsys1=1, row_stride=4, sys_stride0=2, sys_stride1=0)
    tl = torch.zeros(4 * 1025 + 8, dtype=torch.float64, device="cuda")
    lco = dict(mode=1, a=tl[:1025], b=tl[:1025] + 1, c=tl[:1025])
    with pytest.raises(tdma.TdmaError) as e:
        tdma.solve_multi(long, lco, tl, tl.clone(), 2, 1)
    assert e.value.status == tdma.EUNSUPPORTED
