"""Host-side checks of the seeded workload generators (CPU only)."""
import numpy as np

from workloads import configs, grids, rng


def test_splitmix64_published_sequence():
    """seed 0, stream k, index 0 hashes the state (k+1)*golden, i.e. the first
    three outputs of SplitMix64 started from state 0 (Steele, Lea, Flood 2014)."""
    assert int(rng.raw64(0, 0, 0)) == 0xE220A8397B1DCDAF
    assert int(rng.raw64(0, 1, 0)) == 0x6E789E6AA1B965F4
    assert int(rng.raw64(0, 2, 0)) == 0x06C45D188009454F


def test_uniform_range_and_moments():
    u = rng.uniform(1234, rng.STREAM_D, np.arange(200000), -1.0, 1.0)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.01 and abs(u.var() - 1.0 / 3.0) < 0.01
    # counter-based: any subset regenerates identically
    idx = np.array([5, 77, 199999])
    assert np.array_equal(rng.uniform(1234, rng.STREAM_D, idx, -1.0, 1.0), u[idx])


def test_perrow_law_dominant_and_corners():
    p = configs.partitioned(8, 4, 50)
    a, b, c, d = configs.full_arrays(p)
    assert np.all(b >= np.abs(a) + np.abs(c) + 1.0)
    A = a.reshape(50, 32); C = c.reshape(50, 32)
    assert not A[0].any() and not C[-1].any()
    assert A[1:].all() and C[:-1].all()


def test_adi_operator_rows():
    a, b, c = grids.adi_viscous_coeffs(256)
    # flux form: interior rows sum to one; r values positive; mean r = 0.5
    assert np.allclose(b[1:-1] + a[1:-1] + c[1:-1], 1.0, atol=1e-12)
    r_lo = -a[1:]
    r_hi = -c[:-1]
    assert (r_lo > 0).all() and (r_hi > 0).all()
    assert np.all(b > np.abs(a) + np.abs(c))
    ua, ub, uc = grids.adi_viscous_coeffs(16, uniform=True)
    assert np.all(ub == 2.0) and np.all(ua[1:] == -0.5) and ua[0] == 0.0 and uc[-1] == 0.0


def test_tanh_grid_geometry():
    dz, zc, hlo, hhi = grids.tanh_grid(256, 2.0)
    assert abs(dz.sum() - 1.0) < 1e-14
    assert np.all(np.diff(zc) > 0)
    mean = 1.0 / 256
    assert 0.1 < dz.min() / mean < 0.2 and 2.0 < dz.max() / mean < 2.2
    assert np.allclose(dz, dz[::-1], rtol=1e-12)             # symmetric stretching


def test_poisson_operator_and_pinned_mode():
    p = configs.poisson(16, 8, 64)
    assert np.allclose(p.b, -(p.a + p.c))
    lam = -p.shift
    assert lam[1] > 0 and np.isclose(lam[1], (2 - 2 * np.cos(2 * np.pi / 16)) * 256)
    pin = configs.poisson_pinned(p)
    a, b, c, d = configs.system_inputs(pin, 0)
    assert b[0] == 1.0 and a[0] == 0.0 and c[0] == 0.0 and d[0] == 0.0


def test_ragged_lengths():
    r = configs.ragged()
    lens = np.diff(r.layout.offsets)
    assert lens.size == 10000 and lens.min() >= 32 and lens.max() <= 8192
    # log-uniform: median near sqrt(32*8192) = 512
    assert 400 < np.median(lens) < 650
    assert 0.01 <= r.margin.min() and r.margin.max() < 1.0


def test_system_inputs_match_full_arrays():
    for p in (configs.plain(nsys=4, n=30), configs.adi(8, 4, 24), configs.partitioned(4, 3, 10)):
        a, b, c, d = configs.full_arrays(p)
        for s in (0, p.layout.nsys - 1):
            sa, sb, sc, sd = configs.system_inputs(p, s)
            rows = p.layout.sys_rows(s)
            assert np.array_equal(sd, d[rows])
            if p.mode == configs.MODE_LIKE_D:
                assert np.array_equal(sa, a[rows]) and np.array_equal(sb, b[rows])
