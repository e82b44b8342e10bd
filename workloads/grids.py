"""Grid and coefficient laws of the synthetic workloads (host, FP64, numpy).

These build the 1-D coefficient tables that stand in for the paper's ADI
viscous operators and FFT-Poisson line operators (paper Sec. 5.1 and 5.2).
The tables are computed once on the host and handed, bit-identical, to both
the oracle and the device solver.  Nothing here solves a system.
"""
import numpy as np


def tanh_faces(n, stretch=2.0):
    """Faces z_f[k], k = 0..n, of a tanh-stretched grid on [0, 1] (clustered at both walls)."""
    k = np.arange(n + 1, dtype=np.float64)
    return 0.5 * (1.0 + np.tanh(stretch * (2.0 * k / n - 1.0)) / np.tanh(stretch))


def tanh_grid(n, stretch=2.0):
    """Return (dz, zc, h_lo, h_hi): cell widths, centres, and centre-to-centre
    distances across the lower and upper face of every cell.  At the walls the
    distance is from the wall to the first centre (dz/2)."""
    zf = tanh_faces(n, stretch)
    dz = np.diff(zf)
    zc = 0.5 * (zf[:-1] + zf[1:])
    h = np.diff(zc)                      # h[k] = distance across face k+1/2, k = 0..n-2
    h_lo = np.empty(n)
    h_hi = np.empty(n)
    h_lo[0] = 0.5 * dz[0]
    h_lo[1:] = h
    h_hi[:-1] = h
    h_hi[-1] = 0.5 * dz[-1]
    return dz, zc, h_lo, h_hi


def uniform_grid(n):
    dz = np.full(n, 1.0 / n)
    zc = (np.arange(n) + 0.5) / n
    h = np.full(n, 1.0 / n)
    h_lo = h.copy(); h_lo[0] = 0.5 / n
    h_hi = h.copy(); h_hi[-1] = 0.5 / n
    return dz, zc, h_lo, h_hi


def adi_viscous_coeffs(n, stretch=2.0, r_mean=0.5, uniform=False):
    """(1 - A_z) operator of a Crank-Nicolson viscous sweep, flux form with
    Dirichlet walls: row k has a_k = -r_{k-1/2}, c_k = -r_{k+1/2},
    b_k = 1 + r_{k-1/2} + r_{k+1/2} (wall faces included), a_0 = c_{n-1} = 0.
    r_{k+-1/2} = S / (dz_k h_{k+-1/2}), S scaled so the mean of all 2n face
    values equals r_mean.  With ``uniform`` every r equals r_mean exactly."""
    if uniform:
        r_lo = np.full(n, float(r_mean))
        r_hi = np.full(n, float(r_mean))
    else:
        dz, _, h_lo, h_hi = tanh_grid(n, stretch)
        g_lo = 1.0 / (dz * h_lo)
        g_hi = 1.0 / (dz * h_hi)
        scale = r_mean / (0.5 * (g_lo.mean() + g_hi.mean()))
        r_lo = scale * g_lo
        r_hi = scale * g_hi
    a = -r_lo.copy()
    c = -r_hi.copy()
    b = 1.0 + r_lo + r_hi
    a[0] = 0.0
    c[-1] = 0.0
    return a, b, c


def poisson_line_coeffs(n, stretch=2.0):
    """Second-difference operator d^2/dz^2 on the stretched grid with Neumann
    walls: a_k = 1/(dz_k h_{k-1/2}) (k >= 1), c_k = 1/(dz_k h_{k+1/2}) (k <= n-2),
    a_0 = c_{n-1} = 0, b_k = -(a_k + c_k).  A mode's wavenumber enters as a
    diagonal shift -lambda (see ``fft_mode_shift``)."""
    dz, _, h_lo, h_hi = tanh_grid(n, stretch)
    a = 1.0 / (dz * h_lo)
    c = 1.0 / (dz * h_hi)
    a[0] = 0.0
    c[-1] = 0.0
    b = -(a + c)
    return a, b, c


def fft_mode_shift(nx, ny, dx, dy):
    """Per-mode diagonal shift -lambda(kx, ky) with the modified wavenumbers of
    the second-order difference: lambda = (2 - 2cos(2 pi kx/nx))/dx^2 +
    (2 - 2cos(2 pi ky/ny))/dy^2.  Returned flat, kx fastest."""
    kx = np.arange(nx, dtype=np.float64)
    ky = np.arange(ny, dtype=np.float64)
    lx = (2.0 - 2.0 * np.cos(2.0 * np.pi * kx / nx)) / (dx * dx)
    ly = (2.0 - 2.0 * np.cos(2.0 * np.pi * ky / ny)) / (dy * dy)
    lam = ly[:, None] + lx[None, :]
    return -(lam.reshape(-1))


def fft_half_shift(nx, ny, dx, dy):
    """``fft_mode_shift`` on the half spectrum of a real-to-complex transform
    in x: kx = 0..nx/2, mode (kx, ky) at ky * (nx//2 + 1) + kx."""
    full = fft_mode_shift(nx, ny, dx, dy).reshape(ny, nx)
    return np.ascontiguousarray(full[:, :nx // 2 + 1]).reshape(-1)
