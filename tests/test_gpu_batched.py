"""GPU parity of the fused on-chip solve (tdma_solve_batched) against the oracle."""
import numpy as np
import pytest

from tests import parity
from workloads import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(p, dtype=np.float64, inplace=False, shape=None):
    import paper_2509_03933_amd as tdma
    tt = torch.float64 if dtype == np.float64 else torch.float32
    a, b, c, d = parity.host_problem(p)
    if dtype == np.float32:
        # the FP32 path solves the FP32-rounded problem; the oracle sees the same values
        import dataclasses
        a, b, c, d = [None if v is None else v.astype(np.float32).astype(np.float64)
                      for v in (a, b, c, d)]
        if p.shift is not None:
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
    return parity.per_system_error(p.layout, x, ref), x, d


def test_plain_contiguous_fp64():
    """64 contiguous systems of n = 256, random dominant rows, FP64."""
    err, _, _ = _run(configs.plain())
    assert err.max() <= parity.TOL_F64, err.max()


def test_plain_contiguous_fp32():
    err, _, _ = _run(configs.plain(), np.float32)
    assert err.max() <= parity.TOL_F32, err.max()


@pytest.mark.parametrize("grid", [(64, 32, 256), (48, 20, 256)])
def test_adi_zsweep_fp64(grid):
    """Strided z-lines, shared tanh-grid operator; 48*20 systems leave a ragged last tile."""
    err, _, _ = _run(configs.adi(*grid))
    assert err.max() <= parity.TOL_F64, err.max()


def test_adi_zsweep_full_size_fp64():
    """The full 256^3 ADI z-sweep, every system compared."""
    err, _, _ = _run(configs.adi(256, 256, 256))
    assert err.max() <= parity.TOL_F64, err.max()


def test_adi_zsweep_fp32():
    err, _, _ = _run(configs.adi(64, 32, 256), np.float32)
    assert err.max() <= parity.TOL_F32, err.max()


@pytest.mark.parametrize("nz", [1024, 1000, 333])
def test_perrow_zsystems_fp64(nz):
    """Per-row random law along z (n = 1024 and lengths not divisible by the tile)."""
    err, _, _ = _run(configs.partitioned(20, 16, nz))
    assert err.max() <= parity.TOL_F64, err.max()


def test_poisson_shift_fp64():
    """Shared Poisson operator plus per-mode shift (bulk modes except the pinned one)."""
    p = configs.poisson(32, 16, 512)
    err, x, _ = _run(p)
    # mode (0, 0) carries a placeholder shift in the bulk call; every mode is checked,
    # ill-conditioned low modes against the long-double oracle
    for s in np.nonzero(err > parity.TOL_F64)[0]:
        sa, sb, sc, sd = configs.system_inputs(p, int(s))
        ok, e64, eld, eorc = parity.conditioned_error(x[p.layout.sys_rows(int(s))], sa, sb, sc, sd,
                                                      parity.TOL_F64)
        assert ok, (int(s), e64, eld, eorc)


def _contiguous(p):
    """The same systems stored with contiguous rows (system s at s*n)."""
    import dataclasses
    nsys = p.layout.nsys
    lay = configs.Layout(n=p.layout.n, nsys0=nsys, nsys1=1, row_stride=1, sys_stride0=p.layout.n,
                         sys_stride1=0)
    return dataclasses.replace(p, layout=lay)


def _adi_with_shift(nx, ny, nz):
    """The ADI operator plus a seeded per-system diagonal shift in [0, 0.5):
    a shared operator with a shift, as diagonally dominant as the ADI one."""
    import dataclasses
    from workloads import rng
    p = configs.adi(nx, ny, nz)
    shift = 0.5 * rng.uniform01(p.seed, rng.STREAM_NOISE, np.arange(p.layout.nsys))
    return dataclasses.replace(p, shift=shift)


@pytest.mark.parametrize("dtype,tol", [(np.float64, parity.TOL_F64), (np.float32, parity.TOL_F32)])
@pytest.mark.parametrize("shape", [None, dict(M=8, S=4, P=32, kernel=0), dict(M=16, S=2, P=16, kernel=0)],
                         ids=["default", "M8_S4_P32", "M16_S2_P16"])
def test_shared_shift_contiguous_rows(shape, dtype, tol):
    """Shared operator plus per-system shift with contiguous rows (LDS-staged
    right-hand sides beside the LDS-held operator rows); n = 250 leaves
    padding rows."""
    err, _, _ = _run(_contiguous(_adi_with_shift(16, 12, 250)), dtype, shape=shape)
    assert err.max() <= tol, err.max()


@pytest.mark.parametrize("dtype,tol", [(np.float64, parity.TOL_F64), (np.float32, parity.TOL_F32)])
def test_shared_shift_strided(dtype, tol):
    """The same with strided z-lines (the FFT-Poisson layout)."""
    err, _, _ = _run(_adi_with_shift(24, 12, 250), dtype)
    assert err.max() <= tol, err.max()


def test_in_place():
    err, _, _ = _run(configs.adi(32, 16, 128), inplace=True)
    assert err.max() <= parity.TOL_F64


@pytest.mark.parametrize("n", [2, 3, 4, 5, 17, 63, 64, 65, 255])
def test_short_systems(n):
    err, _, _ = _run(configs.plain(nsys=37, n=n))
    assert err.max() <= parity.TOL_F64, (n, err.max())
    err, _, _ = _run(configs.partitioned(17, 3, n))
    assert err.max() <= parity.TOL_F64, (n, err.max())


def test_single_system():
    err, _, _ = _run(configs.partitioned(1, 1, 700))
    assert err.max() <= parity.TOL_F64


def test_ragged_fp64():
    r = configs.ragged(nsys=300, nmin=2, nmax=5000)
    err, _, _ = _run(r)
    assert err.max() <= parity.TOL_F64, err.max()


def _ragged_with_lengths(lens, seed=31):
    """A ragged per-row problem with the given system lengths (the ragged
    law of configs.ragged)."""
    import dataclasses
    lens = np.asarray(lens, dtype=np.int64)
    base = configs.ragged(nsys=len(lens), seed=seed)
    offsets = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    lay = configs.Layout(n=int(lens.max()), nsys0=len(lens), nsys1=1, offsets=offsets)
    return dataclasses.replace(base, layout=lay)


@pytest.mark.parametrize("case", ["one_longest", "many_shortest", "bucket_edges", "one_per_bucket"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_ragged_tile_list_edges(case, dtype):
    """The single-launch tile list at the edges of its bucketing: one system
    of the longest length; 5,000 systems of 2 rows (512 systems per tile);
    lengths at every power-of-two bucket edge and one row past it (tiles of
    one bucket cut short, last tiles partly filled); one system per bucket."""
    top = 8192 if dtype == np.float64 else 16384
    edges = [2 ** k for k in range(1, 14) if 2 ** k <= top]
    lens = {"one_longest": [top],
            "many_shortest": [2] * 5000,
            "bucket_edges": [e + o for e in edges for o in (0, 1) if e + o <= top] * 3,
            "one_per_bucket": [e - 1 for e in edges if e - 1 >= 2] + [top]}[case]
    p = _ragged_with_lengths(lens)
    err, _, _ = _run(p, dtype)
    assert err.max() <= (parity.TOL_F64 if dtype == np.float64 else parity.TOL_F32), err.max()


def test_ragged_fp32():
    r = configs.ragged(nsys=200, nmin=2, nmax=3000)
    err, _, _ = _run(r, np.float32)
    assert err.max() <= parity.TOL_F32, err.max()


SHAPES_F64 = [dict(M=4, S=16, P=16), dict(M=8, S=16, P=8), dict(M=16, S=16, P=4),
              dict(M=8, S=8, P=32), dict(M=4, S=64, P=16), dict(M=16, S=1, P=16)]


@pytest.mark.parametrize("shape", SHAPES_F64, ids=lambda s: "M%d_S%d_P%d" % (s["M"], s["S"], s["P"]))
def test_tile_shapes_fp64(shape):
    """Every register-tile size gives the oracle's answer (n = 64 fits all shapes)."""
    err, _, _ = _run(configs.partitioned(40, 2, 64), shape=shape)
    assert err.max() <= parity.TOL_F64, err.max()
    err, _, _ = _run(configs.plain(nsys=9, n=64), shape=shape)
    assert err.max() <= parity.TOL_F64, err.max()


def test_singular_flagged():
    import paper_2509_03933_amd as tdma
    n, nsys = 8, 16
    a = torch.zeros(n * nsys, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)        # zero diagonal: first pivot is 0
    c = torch.zeros_like(a)
    d = torch.ones_like(a)
    x = torch.empty_like(a)
    lay = configs.Layout(n=n, nsys0=nsys, row_stride=1, sys_stride0=n)
    tdma.solve_batched(lay, dict(mode=0, a=a, b=b, c=c), d, x)
    with pytest.raises(tdma.TdmaError) as ei:
        tdma.check()
    assert ei.value.status == tdma.ESINGULAR
    tdma.check()   # flag was cleared


SHAPES_SHARED = [dict(M=16, S=16, P=16, kernel=1), dict(M=8, S=16, P=32, kernel=1),
                 dict(M=32, S=16, P=8, kernel=1), dict(M=8, S=8, P=64, kernel=1),
                 dict(M=16, S=1, P=16, kernel=1), dict(M=16, S=16, P=16, kernel=0),
                 dict(M=16, S=16, P=16, kernel=2), dict(M=32, S=32, P=8, kernel=2),
                 dict(M=12, S=16, P=32, kernel=1), dict(M=24, S=16, P=16, kernel=1)]


@pytest.mark.parametrize("shape", SHAPES_SHARED,
                         ids=lambda s: "k%d_M%d_S%d_P%d" % (s["kernel"], s["M"], s["S"], s["P"]))
def test_shared_operator_shapes(shape):
    """Shared-operator kernel (tables in LDS) and the generic kernel on the same
    ADI problem; n = 200 leaves identity padding rows in the last partition."""
    err, _, _ = _run(configs.adi(40, 12, 200), shape=shape)
    assert err.max() <= parity.TOL_F64, err.max()


STREAM_SHAPES = [dict(M=16, S=1, P=16, kernel=2), dict(M=16, S=4, P=16, kernel=2),
                 dict(M=8, S=2, P=32, kernel=2), dict(M=32, S=8, P=8, kernel=2),
                 dict(M=12, S=16, P=32, kernel=2), dict(M=24, S=8, P=16, kernel=2)]


@pytest.mark.parametrize("dtype,tol", [(np.float64, parity.TOL_F64), (np.float32, parity.TOL_F32)])
@pytest.mark.parametrize("shape", STREAM_SHAPES,
                         ids=lambda s: "M%d_S%d_P%d" % (s["M"], s["S"], s["P"]))
def test_shared_streaming_walks_many_tiles(shape, dtype, tol):
    """Streaming form: far more tiles than resident workgroups, so each
    workgroup walks several tiles through both register sets; 65,535
    systems leave a partial last tile and n = 200 padding rows."""
    err, _, _ = _run(configs.adi(257, 255, 200), dtype, shape=shape)
    assert err.max() <= tol, err.max()


@pytest.mark.parametrize("dtype,tol", [(np.float64, parity.TOL_F64), (np.float32, parity.TOL_F32)])
def test_adi_sweeps_all_directions(dtype, tol):
    """x (contiguous rows, LDS-staged), y and z sweeps of one grid, shared operators."""
    px, py, pz = configs.sweeps(96, 40, 72)
    for p in (px, py, pz):
        err, _, _ = _run(p, dtype)
        assert err.max() <= tol, (p.name, err.max())


def test_shared_fp32_padding():
    err, _, _ = _run(configs.adi(33, 7, 100), np.float32)
    assert err.max() <= parity.TOL_F32, err.max()


CSTREAM_SHAPES = [dict(M=16, S=16, P=16, kernel=2), dict(M=8, S=8, P=32, kernel=2),
                  dict(M=32, S=16, P=8, kernel=2), dict(M=16, S=1, P=16, kernel=2),
                  dict(M=8, S=4, P=64, kernel=2), dict(M=12, S=8, P=32, kernel=2),
                  dict(M=24, S=8, P=16, kernel=2)]


@pytest.mark.parametrize("dtype,tol", [(np.float64, parity.TOL_F64), (np.float32, parity.TOL_F32)])
@pytest.mark.parametrize("shape", CSTREAM_SHAPES,
                         ids=lambda s: "M%d_S%d_P%d" % (s["M"], s["S"], s["P"]))
def test_shared_streaming_contiguous_rows(shape, dtype, tol):
    """Streaming form with contiguous rows of consecutive systems (x-lines):
    8,000 systems of n = 250 walk several tiles per workgroup through the LDS
    transpose; n = 250 leaves identity padding rows, and 8,000 systems a
    partial last tile for S = 16."""
    px, _, _ = configs.sweeps(250, 80, 100)
    err, _, _ = _run(px, dtype, shape=shape)
    assert err.max() <= tol, err.max()


@pytest.mark.parametrize("grid", [(256, 40, 50), (1000, 3, 7), (17, 5, 3)])
def test_shared_streaming_contiguous_sizes(grid):
    """The default contiguous-row shape at n = 256 (no padding rows), at
    n = 1000 (P = 64 partitions of 16 rows) with 21 systems (one partial
    tile), and at n = 17 (mostly padding)."""
    px, _, _ = configs.sweeps(*grid)
    err, _, _ = _run(px)
    assert err.max() <= parity.TOL_F64, err.max()


def test_shared_streaming_contiguous_gapped_layout():
    """Contiguous rows whose systems are not consecutive (6 unused elements
    after each system): the streaming shape runs the one-tile-per-block form
    and gives the oracle's answer."""
    import dataclasses
    p = configs.adi(20, 30, 256)            # right-hand sides defined on 256 x 600 elements
    a, b, c = p.a[:250].copy(), p.b[:250].copy(), p.c[:250].copy()
    c[-1] = 0.0
    lay = configs.Layout(n=250, nsys0=p.layout.nsys, nsys1=1, row_stride=1, sys_stride0=256,
                         sys_stride1=0)
    q = dataclasses.replace(p, layout=lay, a=a, b=b, c=c)
    err, _, _ = _run(q, shape=dict(M=16, S=16, P=16, kernel=2))
    assert err.max() <= parity.TOL_F64, err.max()


@pytest.mark.parametrize("tt", ["float64", "float32"])
def test_streamed_copy_is_exact(tt):
    """The measurement copy moves every system row bit for bit and leaves the
    elements outside the systems alone: z-lines of the first 18 of 20
    x-columns (n = 200, 540 systems; a partial last tile)."""
    import paper_2509_03933_amd as tdma
    dt = getattr(torch, tt)
    nx, ny, nz = 20, 30, 200
    lay = configs.Layout(n=nz, nsys0=18, nsys1=ny, row_stride=nx * ny, sys_stride0=1,
                         sys_stride1=nx)
    src = torch.randn(nx * ny * nz, dtype=torch.float64, device="cuda").to(dt)
    dst = torch.full_like(src, float("nan"))
    tdma.copy_streamed(lay, src, dst)
    torch.cuda.synchronize()
    s, g = src.view(nz, ny, nx), dst.view(nz, ny, nx)
    assert torch.equal(g[:, :, :18], s[:, :, :18])
    assert torch.isnan(g[:, :, 18:]).all()


@pytest.mark.parametrize("n", [2, 3, 5, 16, 17, 33])
def test_shared_streaming_short_systems(n):
    """Shared operator with very short systems (one or two partitions, most
    rows identity padding) in both streaming forms: contiguous x-lines of n
    rows and strided z-lines of n rows."""
    px, _, _ = configs.sweeps(n, 6, 7)
    _, _, pz = configs.sweeps(5, 6, n)
    for p in (px, pz):
        err, _, _ = _run(p)
        assert err.max() <= parity.TOL_F64, (p.name, n, err.max())
        err, _, _ = _run(p, np.float32)
        assert err.max() <= parity.TOL_F32, (p.name, n, err.max())


@pytest.mark.parametrize("dtype,tol", [(np.float64, parity.TOL_F64), (np.float32, parity.TOL_F32)])
def test_sweep_lengths_of_the_large_grid(dtype, tol):
    """The line lengths of the 768 x 512 x 1536 sweeps with few systems, in
    the default shapes: x-lines of 768 contiguous rows (contiguous streaming
    form), y-lines of 512 rows, z-lines of 1536 rows (32 rows x 64
    partitions per system); every system against the oracle."""
    px, _, _ = configs.sweeps(768, 12, 10)
    _, py, _ = configs.sweeps(10, 512, 12)
    _, _, pz = configs.sweeps(10, 12, 1536)
    for p in (px, py, pz):
        err, _, _ = _run(p, dtype)
        assert err.max() <= tol, (p.name, err.max())


def test_ragged_long_systems_fp32():
    """FP32 ragged systems of 4,000 to 16,384 rows (16 rows per lane beyond
    6,144 rows, up to 1,024 partitions)."""
    r = configs.ragged(nsys=60, nmin=4000, nmax=16384)
    err, _, _ = _run(r, np.float32)
    assert err.max() <= parity.TOL_F32, err.max()


def test_ragged_too_long_for_fp64():
    """An FP64 ragged system beyond 8,192 rows (more than 512 partitions of
    16 rows) is refused with EUNSUPPORTED before any launch."""
    import paper_2509_03933_amd as tdma
    offsets = np.array([0, 100, 100 + 9000], dtype=np.int64)
    lay = configs.Layout(n=9000, nsys0=2, nsys1=1, offsets=offsets)
    t = torch.zeros(9100, dtype=torch.float64, device="cuda")
    with pytest.raises(tdma.TdmaError) as ei:
        tdma.solve_batched(lay, dict(mode=0, a=t, b=t + 1, c=t), t, torch.empty_like(t))
    assert ei.value.status == tdma.EUNSUPPORTED


def test_concurrent_host_threads():
    """Four host threads, each on its own stream, solving a ragged batch and
    a shared-operator sweep at the same time (the per-device host state is
    locked per call; each thread has its own outputs): every result matches
    the oracle."""
    import threading
    import paper_2509_03933_amd as tdma
    r = configs.ragged(nsys=120, nmin=2, nmax=3000)
    ra, rb, rc, rd = parity.host_problem(r)
    rref = parity.oracle_solution(r, ra, rb, rc, rd)
    rco = parity.device_coeffs(r, ra, rb, rc, torch.float64)
    (trd,) = parity.to_device([rd], torch.float64)
    z = configs.adi(40, 12, 200)
    za, zb, zc, zd = parity.host_problem(z)
    zref = parity.oracle_solution(z, za, zb, zc, zd)
    zco = parity.device_coeffs(z, za, zb, zc, torch.float64)
    (tzd,) = parity.to_device([zd], torch.float64)
    outs = [(torch.full_like(trd, float("nan")), torch.full_like(tzd, float("nan"))) for _ in range(4)]
    errors = []

    def work(k):
        try:
            st = torch.cuda.Stream()
            for _ in range(5):
                tdma.solve_batched(r.layout, rco, trd, outs[k][0], stream=st)
                tdma.solve_batched(z.layout, zco, tzd, outs[k][1], stream=st)
            st.synchronize()
        except Exception as e:       # reported below, in the main thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    tdma.check()
    for xr, xz in outs:
        assert parity.per_system_error(r.layout, xr.cpu().numpy(), rref).max() <= parity.TOL_F64
        assert parity.per_system_error(z.layout, xz.cpu().numpy(), zref).max() <= parity.TOL_F64
