"""Fill workload inputs directly in device memory (bit-identical to the host
generator), for problems too large to build on the host and copy.

``build()`` compiles devgen.hip into libwlgen.so (hipcc, gfx950,
-ffp-contract=off).  ``device_inputs(problem)`` returns torch tensors
(d and a coefficient dict) on cuda.  No solver arithmetic lives here.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

from . import configs

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "devgen.hip")
_LIB_PATH = os.path.join(_HERE, "libwlgen.so")
_lock = threading.Lock()
_lib = None


def build(force=True):
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["/opt/rocm/bin/hipcc", "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-o", tmp, _SRC]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build()
            L = ctypes.CDLL(_LIB_PATH)
            i64, u64, vp, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double
            L.wl_perrow_grid.argtypes = [u64, i64, i64, i64, vp, vp, vp, vp, vp]
            L.wl_smooth.argtypes = [u64, i64, i64, i64, vp, vp, vp, dbl, vp, vp]
            L.wl_uniform_d.argtypes = [u64, i64, i64, vp, vp]
            for f in (L.wl_perrow_grid, L.wl_smooth, L.wl_uniform_d):
                f.restype = ctypes.c_int
            _lib = L
    return _lib


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def device_inputs(p, dtype=None):
    """(d, coeffs) for problem p on cuda, float64 unless dtype says otherwise.
    Grid z-systems with the per-row law, smooth and uniform RHS are filled by
    the device generator; other problems are built on the host and copied."""
    import torch
    lay = p.layout
    total = p.extent()
    L = _load()
    st = _stream()
    dev = "cuda"
    f64 = torch.float64
    if p.law == "perrow" and p.grid and not lay.ragged and lay.row_stride == p.grid[0] * p.grid[1]:
        a = torch.empty(total, dtype=f64, device=dev)
        b = torch.empty_like(a); c = torch.empty_like(a); d = torch.empty_like(a)
        rc = L.wl_perrow_grid(p.seed, lay.row_stride, lay.n, total, _ptr(a), _ptr(b), _ptr(c),
                              _ptr(d), st)
        if rc:
            raise RuntimeError(f"wl_perrow_grid failed: {rc}")
        coeffs = dict(mode=configs.MODE_LIKE_D, a=a, b=b, c=c)
    elif p.law in ("smooth", "uniform_d") and p.grid:
        d = torch.empty(total, dtype=f64, device=dev)
        if p.law == "smooth":
            nx, ny, _ = p.grid
            sm = p.smooth
            tabs = [torch.from_numpy(np.ascontiguousarray(sm[k])).to(dev) for k in ("sx", "sy", "cz")]
            rc = L.wl_smooth(p.seed, nx, ny, total, _ptr(tabs[0]), _ptr(tabs[1]), _ptr(tabs[2]),
                             sm["amp"], _ptr(d), st)
            torch.cuda.current_stream().synchronize()
        else:
            pin = -1 if p.pin_row0 is None else int(p.pin_row0)
            rc = L.wl_uniform_d(p.seed, total, pin, _ptr(d), st)
            if pin >= 0 and p.pin_count > 1:
                d[pin + 1:pin + p.pin_count] = 0.0
        if rc:
            raise RuntimeError(f"device generator failed: {rc}")
        coeffs = dict(mode=p.mode, a=torch.from_numpy(p.a).to(dev), b=torch.from_numpy(p.b).to(dev),
                      c=torch.from_numpy(p.c).to(dev),
                      shift=None if p.shift is None else torch.from_numpy(p.shift).to(dev))
    else:
        a, b, c, d_h = configs.full_arrays(p)
        d = torch.from_numpy(np.ascontiguousarray(d_h)).to(dev)
        if p.mode == configs.MODE_LIKE_D:
            coeffs = dict(mode=p.mode, a=torch.from_numpy(a).to(dev), b=torch.from_numpy(b).to(dev),
                          c=torch.from_numpy(c).to(dev))
        else:
            coeffs = dict(mode=p.mode, a=torch.from_numpy(p.a).to(dev), b=torch.from_numpy(p.b).to(dev),
                          c=torch.from_numpy(p.c).to(dev),
                          shift=None if p.shift is None else torch.from_numpy(p.shift).to(dev))
    if dtype is not None and dtype != f64:
        d = d.to(dtype)
        coeffs = {k: (v.to(dtype) if hasattr(v, "to") else v) for k, v in coeffs.items()}
    return d, coeffs
