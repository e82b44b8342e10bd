"""Seeded synthetic workloads shaped like the paper's TDM systems.

Five workload families (seed 1000 + k for family k):

1. ``plain``        64 contiguous systems of n = 256, random diagonally dominant rows.
2. ``adi``          ADI viscous z-sweep on an nx*ny*nz grid (x fastest), one
                    tanh-grid operator shared by every z-line; smooth RHS + noise.
3. ``partitioned``  z-systems of an nx*ny*nz grid with the random per-row law of (1).
4. ``poisson``      FFT-Poisson line solves: one z-system per (kx, ky) mode, shared
                    second-difference operator plus a per-mode shift -lambda; mode
                    (0, 0) is pinned (row 0 replaced by x_0 = 0) and solved as a
                    separate one-system problem.
5. ``sweeps``       x, y and z ADI sweeps of one grid plus a ragged batch of
                    independent systems with log-uniform lengths.
6. ``poisson_complex`` the lines of (4) with complex right-hand sides stored as
                    interleaved (re, im) pairs: two right-hand sides per system.

Every random value is ``workloads.rng.uniform(seed, stream, index, lo, hi)`` of
the element's linear array index (or system index), so the oracle can rebuild
any single system on the host (``system_inputs``) while the device fills whole
arrays with the identical generator.  No solver arithmetic lives here.
"""
from dataclasses import dataclass, field
from typing import Optional
import numpy as np

from . import rng, grids

MODE_LIKE_D = 0      # coefficient arrays laid out exactly like d
MODE_SHARED = 1      # one length-n table for every system (+ optional per-system shift)

SEED_BASE = 1000


@dataclass
class Layout:
    """System k = s0 + nsys0*s1 has row i at  s0*sys_stride0 + s1*sys_stride1 + i*row_stride.
    Ragged layouts (offsets is not None): system s occupies offsets[s]..offsets[s+1]-1."""
    n: int
    nsys0: int
    nsys1: int = 1
    row_stride: int = 1
    sys_stride0: int = 0
    sys_stride1: int = 0
    offsets: Optional[np.ndarray] = None

    @property
    def nsys(self):
        return self.nsys0 * self.nsys1

    @property
    def ragged(self):
        return self.offsets is not None

    def sys_n(self, s):
        if self.ragged:
            return int(self.offsets[s + 1] - self.offsets[s])
        return self.n

    def sys_rows(self, s):
        """Linear element indices of the rows of system s (int64 ndarray)."""
        if self.ragged:
            return np.arange(self.offsets[s], self.offsets[s + 1], dtype=np.int64)
        s0, s1 = s % self.nsys0, s // self.nsys0
        base = s0 * self.sys_stride0 + s1 * self.sys_stride1
        return base + np.arange(self.n, dtype=np.int64) * self.row_stride

    def extent(self):
        """Number of elements an array in this layout spans."""
        if self.ragged:
            return int(self.offsets[-1])
        return 1 + (self.n - 1) * self.row_stride + (self.nsys0 - 1) * self.sys_stride0 \
            + (self.nsys1 - 1) * self.sys_stride1

    def unknowns(self):
        if self.ragged:
            return int(self.offsets[-1] - self.offsets[0])
        return self.n * self.nsys


@dataclass
class Problem:
    """One batched solve: layout, coefficient mode and the generator recipe.

    For MODE_SHARED, a/b/c are the length-n host tables and ``shift`` (if any)
    the per-system diagonal shift.  For MODE_LIKE_D the arrays are generated
    per element (``full_arrays`` / ``system_inputs``)."""
    name: str
    layout: Layout
    mode: int
    seed: int
    law: str                         # 'perrow' | 'smooth' | 'uniform_d' | 'ragged'
    a: Optional[np.ndarray] = None
    b: Optional[np.ndarray] = None
    c: Optional[np.ndarray] = None
    shift: Optional[np.ndarray] = None
    grid: tuple = ()                 # (nx, ny, nz) of the underlying 3-D array, if any
    smooth: dict = field(default_factory=dict)   # 1-D factor tables of the smooth RHS
    margin: Optional[np.ndarray] = None          # ragged: per-system dominance margin
    pin_row0: Optional[int] = None   # poisson: first element of d forced to 0
    pin_count: int = 1               # elements pin_row0 .. pin_row0+pin_count-1 are zero
    nrhs: int = 1                    # right-hand sides per system (shared operator)
    rhs_stride: int = 0              # elements between a system's right-hand sides

    def extent(self):
        """Elements an array of d spans, all right-hand sides included."""
        return self.layout.extent() + (self.nrhs - 1) * self.rhs_stride


# ----------------------------------------------------------------------------
# element laws (vectorised over linear indices)

def perrow_law(seed, idx, row, nrow, margin=None):
    """a, c ~ U(-1,1) (a_0 = c_{n-1} = 0), b = |a| + |c| + U(1,2) (or + margin),
    d ~ U(-1,1).  Evaluated at linear element indices ``idx`` whose in-system
    row numbers are ``row`` and system lengths ``nrow``."""
    a = rng.uniform(seed, rng.STREAM_A, idx, -1.0, 1.0)
    c = rng.uniform(seed, rng.STREAM_C, idx, -1.0, 1.0)
    a = np.where(row == 0, 0.0, a)
    c = np.where(row == nrow - 1, 0.0, c)
    if margin is None:
        extra = rng.uniform(seed, rng.STREAM_B, idx, 1.0, 2.0)
    else:
        extra = margin
    b = (np.abs(a) + np.abs(c)) + extra
    d = rng.uniform(seed, rng.STREAM_D, idx, -1.0, 1.0)
    return a, b, c, d


def smooth_rhs(seed, idx, sx, sy, cz, nx, ny, amp):
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    noise = rng.uniform(seed, rng.STREAM_NOISE, idx, -amp, amp)
    return (sx[i] * sy[j]) * cz[k] + noise


# ----------------------------------------------------------------------------
# workload builders

def zsys_layout(nx, ny, nz):
    return Layout(n=nz, nsys0=nx, nsys1=ny, row_stride=nx * ny, sys_stride0=1, sys_stride1=nx)


def plain(nsys=64, n=256):
    lay = Layout(n=n, nsys0=nsys, nsys1=1, row_stride=1, sys_stride0=n, sys_stride1=0)
    return Problem("plain", lay, MODE_LIKE_D, SEED_BASE + 1, "perrow")


def _smooth_tables(nx, ny, zc):
    sx = np.sin(2.0 * np.pi * (np.arange(nx) + 0.5) / nx)
    sy = np.sin(2.0 * np.pi * (np.arange(ny) + 0.5) / ny)
    cz = np.cos(np.pi * zc)
    return dict(sx=sx, sy=sy, cz=cz, amp=1e-3)


def adi(nx=256, ny=256, nz=256, stretch=2.0, r_mean=0.5):
    a, b, c = grids.adi_viscous_coeffs(nz, stretch, r_mean)
    _, zc, _, _ = grids.tanh_grid(nz, stretch)
    return Problem("adi", zsys_layout(nx, ny, nz), MODE_SHARED, SEED_BASE + 2, "smooth",
                   a=a, b=b, c=c, grid=(nx, ny, nz), smooth=_smooth_tables(nx, ny, zc))


def partitioned(nx=1024, ny=1024, nz=1024):
    return Problem("partitioned", zsys_layout(nx, ny, nz), MODE_LIKE_D, SEED_BASE + 3, "perrow",
                   grid=(nx, ny, nz))


def poisson(nx=1024, ny=1024, nz=1024, stretch=2.0):
    """Bulk problem over every mode.  Mode (0, 0) is singular with Neumann walls;
    in the bulk call it carries the shift of mode (1, 0) (a placeholder whose
    result is discarded) and its real, pinned system is ``poisson_pinned``."""
    a, b, c = grids.poisson_line_coeffs(nz, stretch)
    shift = grids.fft_mode_shift(nx, ny, 1.0 / nx, 1.0 / ny)
    shift[0] = shift[1] if nx > 1 else shift[nx]
    return Problem("poisson", zsys_layout(nx, ny, nz), MODE_SHARED, SEED_BASE + 4, "uniform_d",
                   a=a, b=b, c=c, shift=shift, grid=(nx, ny, nz), pin_row0=0)


def poisson_pinned(bulk):
    """The (0, 0) mode: lambda = 0 and row 0 replaced by x_0 = 0 (a_0 = c_0 = 0,
    b_0 = 1, d_0 = 0).  One system, shared-table mode, d/x strided like the bulk."""
    nx, ny, nz = bulk.grid
    a = bulk.a.copy(); b = bulk.b.copy(); c = bulk.c.copy()
    a[0] = 0.0; c[0] = 0.0; b[0] = 1.0
    lay = Layout(n=nz, nsys0=1, nsys1=1, row_stride=nx * ny, sys_stride0=1, sys_stride1=nx)
    return Problem("poisson_pinned", lay, MODE_SHARED, bulk.seed, "uniform_d",
                   a=a, b=b, c=c, grid=bulk.grid, pin_row0=0)


def poisson_complex(nx=1024, ny=1024, nz=1024, stretch=2.0):
    """The Poisson line solves with complex right-hand sides (the Fourier
    coefficients of a real field are complex, Sec. 8.1): the operator and the
    per-mode shift of ``poisson`` over a complex nx*ny*nz array stored as
    interleaved (re, im) FP64 pairs.  Counted in real elements, the real parts
    of mode (i, j) form a z-system with row stride 2*nx*ny and its imaginary
    parts the same system one element on: two right-hand sides per system,
    rhs_stride 1.  Both parts of d are U(-1, 1) of the real element index;
    mode (0, 0) is pinned as in ``poisson`` (both parts of its d_0 zero) and
    solved separately (``poisson_complex_pinned``)."""
    base = poisson(nx, ny, nz, stretch)
    lay = Layout(n=nz, nsys0=nx, nsys1=ny, row_stride=2 * nx * ny, sys_stride0=2,
                 sys_stride1=2 * nx)
    return Problem("poisson_complex", lay, MODE_SHARED, SEED_BASE + 6, "uniform_d",
                   a=base.a, b=base.b, c=base.c, shift=base.shift, grid=(nx, ny, nz),
                   pin_row0=0, pin_count=2, nrhs=2, rhs_stride=1)


def poisson_complex_pinned(bulk):
    """Mode (0, 0) of ``poisson_complex``: lambda = 0 and row 0 replaced by
    x_0 = 0, both right-hand sides (the real and imaginary parts)."""
    nx, ny, nz = bulk.grid
    a = bulk.a.copy(); b = bulk.b.copy(); c = bulk.c.copy()
    a[0] = 0.0; c[0] = 0.0; b[0] = 1.0
    lay = Layout(n=nz, nsys0=1, nsys1=1, row_stride=2 * nx * ny, sys_stride0=2,
                 sys_stride1=2 * nx)
    return Problem("poisson_complex_pinned", lay, MODE_SHARED, bulk.seed, "uniform_d",
                   a=a, b=b, c=c, grid=bulk.grid, pin_row0=0, pin_count=2, nrhs=2,
                   rhs_stride=1)


def complex_layout(p):
    """The layout of a two-right-hand-side interleaved problem counted in
    complex elements (the oracle's complex view of the same array)."""
    lay = p.layout
    assert p.nrhs == 2 and p.rhs_stride == 1
    assert lay.row_stride % 2 == 0 and lay.sys_stride0 % 2 == 0 and lay.sys_stride1 % 2 == 0
    return Layout(n=lay.n, nsys0=lay.nsys0, nsys1=lay.nsys1, row_stride=lay.row_stride // 2,
                  sys_stride0=lay.sys_stride0 // 2, sys_stride1=lay.sys_stride1 // 2)


def sweeps(nx=768, ny=512, nz=1536, stretch=2.0, r_mean=0.5):
    """The three ADI sweeps (x, y uniform r = r_mean; z on the tanh grid), applied
    in sequence to one field: (1-A_x) u1 = R, (1-A_y) u2 = u1, (1-A_z) u3 = u2."""
    seed = SEED_BASE + 5
    ax, bx, cx = grids.adi_viscous_coeffs(nx, uniform=True, r_mean=r_mean)
    ay, by, cy = grids.adi_viscous_coeffs(ny, uniform=True, r_mean=r_mean)
    az, bz, cz_ = grids.adi_viscous_coeffs(nz, stretch, r_mean)
    _, zc, _, _ = grids.tanh_grid(nz, stretch)
    sm = _smooth_tables(nx, ny, zc)
    px = Problem("sweep_x", Layout(n=nx, nsys0=ny, nsys1=nz, row_stride=1, sys_stride0=nx,
                                   sys_stride1=nx * ny), MODE_SHARED, seed, "smooth",
                 a=ax, b=bx, c=cx, grid=(nx, ny, nz), smooth=sm)
    py = Problem("sweep_y", Layout(n=ny, nsys0=nx, nsys1=nz, row_stride=nx, sys_stride0=1,
                                   sys_stride1=nx * ny), MODE_SHARED, seed, "smooth",
                 a=ay, b=by, c=cy, grid=(nx, ny, nz), smooth=sm)
    pz = Problem("sweep_z", zsys_layout(nx, ny, nz), MODE_SHARED, seed, "smooth",
                 a=az, b=bz, c=cz_, grid=(nx, ny, nz), smooth=sm)
    return px, py, pz


def ragged_lengths(seed, nsys, nmin=32, nmax=8192):
    u = rng.uniform01(seed, rng.STREAM_RAGGED_N, np.arange(nsys))
    lo, hi = np.log(nmin), np.log(nmax)
    return np.rint(np.exp(lo + (hi - lo) * u)).astype(np.int64)


def ragged(nsys=10000, nmin=32, nmax=8192, seed=None):
    seed = SEED_BASE + 5 if seed is None else seed
    lens = ragged_lengths(seed, nsys, nmin, nmax)
    offsets = np.zeros(nsys + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    margin = rng.uniform(seed, rng.STREAM_MARGIN, np.arange(nsys), 0.01, 1.0)
    lay = Layout(n=int(lens.max()), nsys0=nsys, nsys1=1, offsets=offsets)
    return Problem("ragged", lay, MODE_LIKE_D, seed, "ragged", margin=margin)


# ----------------------------------------------------------------------------
# host materialisation

def row_numbers(lay):
    """In-system row number of every element of a uniform layout (-1 where no
    system has a row).  O(extent) host memory: small problems only."""
    row = np.full(lay.extent(), -1, dtype=np.int64)
    s = np.arange(lay.nsys, dtype=np.int64)
    base = (s % lay.nsys0) * lay.sys_stride0 + (s // lay.nsys0) * lay.sys_stride1
    i = np.arange(lay.n, dtype=np.int64)
    row[base[:, None] + i[None, :] * lay.row_stride] = i[None, :]
    return row


def element_values(p, idx, row, nrow, sys_index=None):
    """Generate (a, b, c, d) at linear indices idx for MODE_LIKE_D problems, or d
    only (a/b/c None) for shared problems."""
    if p.law == "perrow":
        return perrow_law(p.seed, idx, row, nrow)
    if p.law == "ragged":
        return perrow_law(p.seed, idx, row, nrow, margin=p.margin[sys_index])
    if p.law == "smooth":
        nx, ny, _ = p.grid
        sm = p.smooth
        return None, None, None, smooth_rhs(p.seed, idx, sm["sx"], sm["sy"], sm["cz"], nx, ny, sm["amp"])
    if p.law == "uniform_d":
        d = rng.uniform(p.seed, rng.STREAM_D, idx, -1.0, 1.0)
        if p.pin_row0 is not None:
            d = np.where((idx >= p.pin_row0) & (idx < p.pin_row0 + p.pin_count), 0.0, d)
        return None, None, None, d
    raise ValueError(f"law {p.law!r} has no closed-form element values")


def system_inputs(p, s):
    """(a, b, c, d) of system s as contiguous FP64 arrays (host), including the
    per-system shift of MODE_SHARED problems folded into b."""
    lay = p.layout
    rows = lay.sys_rows(s)
    n = rows.size
    i = np.arange(n, dtype=np.int64)
    if p.mode == MODE_LIKE_D:
        a, b, c, d = element_values(p, rows, i, n, sys_index=s)
        return a, b, c, d
    _, _, _, d = element_values(p, rows, i, n)
    b = p.b.copy()
    if p.shift is not None:
        b = b + p.shift[s]
    return p.a.copy(), b, p.c.copy(), d


def system_rhs(p, s):
    """The p.nrhs right-hand sides of system s (list of contiguous FP64 arrays)."""
    rows = p.layout.sys_rows(s)
    out = []
    for r in range(p.nrhs):
        _, _, _, d = element_values(p, rows + r * p.rhs_stride, None, rows.size)
        out.append(d)
    return out


def full_arrays(p):
    """Whole host arrays (a, b, c, d) in the problem's layout.  For MODE_SHARED
    a/b/c are the tables.  Only for sizes that fit comfortably in host memory."""
    lay = p.layout
    size = p.extent()
    idx = np.arange(size, dtype=np.int64)
    if lay.ragged:
        lens = np.diff(lay.offsets)
        sys_of = np.repeat(np.arange(lay.nsys, dtype=np.int64), lens)
        row = idx - lay.offsets[sys_of]
        nrow = lens[sys_of]
        a, b, c, d = perrow_law(p.seed, idx, row, nrow, margin=p.margin[sys_of])
        return a, b, c, d
    if p.law == "perrow":
        a, b, c, d = perrow_law(p.seed, idx, row_numbers(lay), lay.n)
        return a, b, c, d
    _, _, _, d = element_values(p, idx, None, lay.n)
    return p.a, p.b, p.c, d
