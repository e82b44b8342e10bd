"""Oracle of the FFT-Poisson step -- TEST INFRASTRUCTURE ONLY (same rules as
the rest of ``oracle/``).

The paper's Poisson solve (Sec. 5.2): Fourier transforms in the two
periodic directions turn the 3-D Poisson equation into one tridiagonal
system per wavenumber pair along the remaining direction,
(d2/dz2 - lambda(kx, ky)) Phi = Q, solved by the TDMA; an inverse transform
returns the field.  Here, in the order the paper states it:
  1. Q = the forward real-to-complex 2-D DFT of q over (y, x) for every z
     (numpy.fft.rfft2, no scaling);
  2. every mode's z-line solved in complex arithmetic by the oracle's Thomas
     solve (``oracle.solve_batch_complex``) with the operator tables a, b, c
     plus the mode's diagonal shift; mode (0, 0), singular with Neumann walls,
     is pinned by replacing its row 0 with Phi_0 = Q_0 (a0 = c0 = 0, b0 = 1);
  3. phi = the inverse 2-D DFT (numpy.fft.irfft2, scaled by 1/(nx ny)).
The shift of mode (kx, ky) is shift_half[ky * (nx // 2 + 1) + kx] (only
kx <= nx/2 exist in the half spectrum; the table is an input, from
``workloads.grids.fft_half_shift``).
"""
import numpy as np

import oracle
from workloads import configs


def poisson_fft(q, nx, ny, nz, a, b, c, shift_half, precision=oracle.F64):
    """phi for the real field q laid out (nz, ny, nx), x fastest."""
    Q = np.fft.rfft2(np.asarray(q, dtype=np.float64).reshape(nz, ny, nx), axes=(1, 2))
    h = nx // 2 + 1
    lay = configs.Layout(n=nz, nsys0=h, nsys1=ny, row_stride=ny * h, sys_stride0=1, sys_stride1=h)
    flat = np.ascontiguousarray(Q).reshape(-1)
    sh = np.array(shift_half, dtype=np.float64).copy()
    X = oracle.solve_batch_complex(lay, a, b, c, flat, shift=sh, precision=precision)
    # mode (0, 0): row 0 replaced by Phi_0 = Q_0
    ap, bp, cp = np.array(a, dtype=np.float64), np.array(b, dtype=np.float64), np.array(c, dtype=np.float64)
    ap[0] = 0.0; bp[0] = 1.0; cp[0] = 0.0
    rows = lay.sys_rows(0)
    X[rows] = oracle.thomas_complex(ap, bp, cp, flat[rows], precision)
    return np.fft.irfft2(X.reshape(nz, ny, h), s=(ny, nx), axes=(1, 2)).reshape(-1)
