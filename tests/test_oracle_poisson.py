"""Pins of the oracle's FFT-Poisson step (CPU only): a manufactured field is
differentiated by the discrete operator in physical space (periodic second
differences in x and y, the z tables in z, no transform involved) and the
step must return it up to a constant (the Neumann null space, fixed by the
pinned mode); plus the mode structure (a single Fourier mode in, the same
mode out, scaled by its 1-D solve)."""
import numpy as np
import pytest

import oracle
from oracle import poisson as op
from workloads import grids


def _apply(phi, nx, ny, nz, dx, dy, a, b, c):
    """The discrete operator L phi in physical space."""
    f = phi.reshape(nz, ny, nx)
    lx = (np.roll(f, -1, 2) - 2 * f + np.roll(f, 1, 2)) / (dx * dx)
    ly = (np.roll(f, -1, 1) - 2 * f + np.roll(f, 1, 1)) / (dy * dy)
    lz = b[:, None, None] * f
    lz[1:] += a[1:, None, None] * f[:-1]
    lz[:-1] += c[:-1, None, None] * f[1:]
    return (lx + ly + lz).reshape(-1)


@pytest.mark.parametrize("grid", [(8, 6, 20), (16, 16, 64), (12, 10, 33)])
def test_manufactured_field_recovered(grid):
    nx, ny, nz = grid
    dx, dy = 1.0 / nx, 1.0 / ny
    a, b, c = grids.poisson_line_coeffs(nz, 2.0)
    shift = grids.fft_half_shift(nx, ny, dx, dy)
    rs = np.random.default_rng(nx * 100 + nz)
    phi = rs.uniform(-1, 1, nx * ny * nz)
    q = _apply(phi, nx, ny, nz, dx, dy, a, b, c)
    got = op.poisson_fft(q, nx, ny, nz, a, b, c, shift)
    diff = got - phi
    # equal up to one constant; the operator's scale (~n^2 / dz_min^2) sets
    # the rounding of q, so the bar is relative to max|phi| times kappa-ish
    assert np.max(np.abs(diff - diff.mean())) <= 1e-8 * np.max(np.abs(phi)), \
        np.max(np.abs(diff - diff.mean()))


def test_single_mode_in_single_mode_out():
    nx, ny, nz = 16, 8, 24
    dx, dy = 1.0 / nx, 1.0 / ny
    a, b, c = grids.poisson_line_coeffs(nz, 2.0)
    full = grids.fft_mode_shift(nx, ny, dx, dy)
    shift = grids.fft_half_shift(nx, ny, dx, dy)
    kx, ky = 3, 2
    i = np.arange(nx); j = np.arange(ny)
    g = np.random.default_rng(4).uniform(-1, 1, nz)
    wave = np.cos(2 * np.pi * (kx * i[None, :] / nx + ky * j[:, None] / ny))
    q = (g[:, None, None] * wave[None]).reshape(-1)
    got = op.poisson_fft(q, nx, ny, nz, a, b, c, shift).reshape(nz, ny, nx)
    # the z profile is the 1-D solve with the mode's shift (lambda of (3, 2))
    prof = oracle.thomas(a, b + full[ky * nx + kx], c, g)
    ref = prof[:, None, None] * wave[None]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
