"""MI355X (gfx950) batched divide-and-conquer tridiagonal solver.

Thin ctypes binding of ``libtdma.so`` (C ABI in ``include/tdma.h``).  Every
step of the solve runs in the library's HIP kernels; this module only
marshals arguments: torch tensors supply device pointers and the current
HIP stream.  Before a call reaches the device it checks that every tensor is
a GPU tensor and that the layout stays inside each tensor's storage, so a
wrong layout is a Python exception, not an out-of-bounds access.

The library must be built (``python -m paper_2509_03933_amd.build``); there is
no fallback path.
"""
import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdma.so")

OK, EINVAL, ENOMEM, EHIP, ESINGULAR, ENOCONV, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
COEF_LIKE_D, COEF_SHARED = 0, 1
SCHED_ROLES, SCHED_ROUND_ROBIN = 0, 1

_c_i64p = ctypes.POINTER(ctypes.c_int64)


class _Layout(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nsys0", ctypes.c_int64), ("nsys1", ctypes.c_int64),
                ("row_stride", ctypes.c_int64), ("sys_stride0", ctypes.c_int64),
                ("sys_stride1", ctypes.c_int64), ("offsets", _c_i64p)]


class _Coeffs(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("b_shift", ctypes.c_void_p)]


class _Tile(ctypes.Structure):
    _fields_ = [("rows_per_lane", ctypes.c_int), ("systems_per_tile", ctypes.c_int),
                ("partitions", ctypes.c_int), ("kernel", ctypes.c_int)]


class _PartOpts(ctypes.Structure):
    _fields_ = [("partitions", ctypes.c_int), ("batch", ctypes.c_int64),
                ("nstreams", ctypes.c_int), ("schedule", ctypes.c_int)]


class _RefineOpts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int), ("tol", ctypes.c_double), ("fallback", ctypes.c_int),
                ("criterion", ctypes.c_int)]


class RefineReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("not_converged", ctypes.c_int64),
                ("fallback_systems", ctypes.c_int64), ("max_rel_correction", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _WorkItem(ctypes.Structure):
    _fields_ = [("layout", _Layout), ("coeffs", _Coeffs), ("d", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("after", ctypes.c_int)]


class TdmaError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(message)
        self.status = status


_lib = None
_lib_lock = threading.Lock()


def lib():
    """The loaded libtdma.so; raises if it has not been built."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run "
                                   "`python -m paper_2509_03933_amd.build` (no fallback exists)")
            L = ctypes.CDLL(LIB_PATH)
            vp, i = ctypes.c_void_p, ctypes.c_int
            L.tdma_solve_batched.argtypes = [ctypes.POINTER(_Layout), ctypes.POINTER(_Coeffs), i, vp, vp, vp]
            L.tdma_solve_batched_tiled.argtypes = [ctypes.POINTER(_Layout), ctypes.POINTER(_Coeffs), i, vp,
                                                   vp, ctypes.POINTER(_Tile), vp]
            L.tdma_solve_partitioned.argtypes = [ctypes.POINTER(_Layout), ctypes.POINTER(_Coeffs), i, vp,
                                                 vp, ctypes.POINTER(_PartOpts), vp]
            L.tdma_solve_refined.argtypes = [ctypes.POINTER(_Layout), ctypes.POINTER(_Coeffs), vp, vp,
                                             ctypes.POINTER(_RefineOpts), ctypes.POINTER(RefineReport), vp]
            L.tdma_solve_refined_noalloc.argtypes = L.tdma_solve_refined.argtypes
            L.tdma_graph_create.argtypes = [ctypes.POINTER(_WorkItem), i, i, ctypes.POINTER(vp)]
            L.tdma_graph_launch.argtypes = [vp, vp]
            L.tdma_graph_destroy.argtypes = [vp]
            L.tdma_graph_destroy.restype = None
            L.tdma_autotune.argtypes = [ctypes.POINTER(_Layout), ctypes.POINTER(_Coeffs), i, vp, vp, i, vp]
            L.tdma_copy_streamed.argtypes = [ctypes.POINTER(_Layout), i, vp, vp, vp]
            L.tdma_poisson_create.argtypes = [i, i, i, vp, vp, vp, vp, ctypes.POINTER(vp)]
            L.tdma_poisson_solve.argtypes = [vp, vp, vp, vp]
            L.tdma_poisson_destroy.argtypes = [vp]
            L.tdma_poisson_destroy.restype = None
            L.tdma_solve_pdd.argtypes = [ctypes.POINTER(_Layout), ctypes.POINTER(_Coeffs), i, i, vp, vp, vp]
            L.tdma_solve_multi.argtypes = [ctypes.POINTER(_Layout), ctypes.POINTER(_Coeffs), i, i,
                                           ctypes.c_int64, vp, vp, vp]
            L.tdma_check.argtypes = [vp]
            L.tdma_autotune_last_json.restype = ctypes.c_char_p
            L.tdma_pipeline_model_ms.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_double, ctypes.c_int]
            L.tdma_pipeline_model_ms.restype = ctypes.c_double
            L.tdma_status_string.argtypes = [i]
            L.tdma_status_string.restype = ctypes.c_char_p
            L.tdma_last_error.restype = ctypes.c_char_p
            L.tdma_shutdown.restype = None
            for f in ("tdma_solve_batched", "tdma_solve_batched_tiled", "tdma_solve_partitioned", "tdma_solve_refined",
                      "tdma_solve_refined_noalloc", "tdma_solve_multi", "tdma_solve_pdd", "tdma_copy_streamed",
                      "tdma_poisson_create", "tdma_poisson_solve",
                      "tdma_graph_create", "tdma_graph_launch", "tdma_autotune", "tdma_check"):
                getattr(L, f).restype = ctypes.c_int
            _lib = L
    return _lib


EXPORTED_SYMBOLS = ("tdma_solve_batched", "tdma_solve_batched_tiled", "tdma_solve_partitioned", "tdma_solve_refined",
                    "tdma_solve_refined_noalloc",
                    "tdma_copy_streamed", "tdma_solve_multi", "tdma_solve_pdd",
                    "tdma_poisson_create", "tdma_poisson_solve", "tdma_poisson_destroy",
                    "tdma_graph_create", "tdma_graph_launch", "tdma_graph_destroy",
                    "tdma_autotune", "tdma_autotune_last_json", "tdma_pipeline_model_ms",
                    "tdma_check", "tdma_status_string", "tdma_last_error", "tdma_shutdown")


def _raise(status):
    if status != OK:
        msg = lib().tdma_last_error().decode() or lib().tdma_status_string(status).decode()
        raise TdmaError(status, msg)


def status_string(status):
    return lib().tdma_status_string(status).decode()


# ---------------------------------------------------------------------------
# argument marshalling and bounds checks

def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _extent(layout):
    """Elements spanned by an array in this layout (max index + 1)."""
    if getattr(layout, "offsets", None) is not None:
        off = np.asarray(layout.offsets)
        return int(off.max()) if off.size else 0
    nsys = layout.nsys0 * layout.nsys1
    if nsys == 0:
        return 0
    return 1 + (layout.n - 1) * layout.row_stride + (layout.nsys0 - 1) * layout.sys_stride0 \
        + (layout.nsys1 - 1) * layout.sys_stride1


def _room(t):
    """Elements addressable from t.data_ptr() inside t's storage."""
    st = t.untyped_storage()
    return (st.nbytes() - t.storage_offset() * t.element_size()) // t.element_size()


def _check_tensor(name, t, need, dtype=None):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if need > _room(t):
        raise ValueError(f"{name}: layout reaches element {need - 1} but the tensor holds {_room(t)}")


def _make_layout(layout, keep):
    L = _Layout()
    offs = getattr(layout, "offsets", None)
    L.n = int(layout.n)
    L.nsys0 = int(layout.nsys0)
    L.nsys1 = int(getattr(layout, "nsys1", 1))
    L.row_stride = int(getattr(layout, "row_stride", 1))
    L.sys_stride0 = int(getattr(layout, "sys_stride0", 0))
    L.sys_stride1 = int(getattr(layout, "sys_stride1", 0))
    if offs is not None:
        arr = np.ascontiguousarray(offs, dtype=np.int64)
        if arr.size != L.nsys0 + 1:
            raise ValueError("offsets must have nsys0 + 1 entries")
        keep.append(arr)
        L.offsets = arr.ctypes.data_as(_c_i64p)
    else:
        L.offsets = None
    return L


def _make_coeffs(layout, coeffs, d, need):
    """coeffs: dict(mode=, a=, b=, c=, shift=) of torch tensors."""
    mode = int(coeffs.get("mode", COEF_LIKE_D))
    a, b, c = coeffs.get("a"), coeffs.get("b"), coeffs.get("c")
    shift = coeffs.get("shift")
    if mode == COEF_LIKE_D:
        for nm, t in (("a", a), ("b", b), ("c", c)):
            _check_tensor(nm, t, need, d.dtype)
    elif mode == COEF_SHARED:
        for nm, t in (("a", a), ("b", b), ("c", c)):
            _check_tensor(nm, t, int(layout.n), d.dtype)
    else:
        raise ValueError(f"unknown coefficient mode {mode}")
    nsys = int(layout.nsys0) * int(getattr(layout, "nsys1", 1))
    if shift is not None:
        _check_tensor("shift", shift, nsys, d.dtype)
    C = _Coeffs()
    C.mode = mode
    C.a, C.b, C.c = a.data_ptr(), b.data_ptr(), c.data_ptr()
    C.b_shift = shift.data_ptr() if shift is not None else None
    return C


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _prepare(layout, coeffs, d, x):
    """Marshalled layout and coefficients, and the Python objects their
    pointers refer to (offsets array, coefficient tensors): whoever keeps the
    pointers past the call (a recorded graph) must keep these alive."""
    keep = []
    need = _extent(layout)
    _check_tensor("d", d, need)
    _check_tensor("x", x, need, d.dtype)
    L = _make_layout(layout, keep)
    C = _make_coeffs(layout, coeffs, d, need)
    keep.extend(t for t in (coeffs.get(k) for k in ("a", "b", "c", "shift")) if t is not None)
    return L, C, keep


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI, without the tdma_ prefix)

def solve_batched(layout, coeffs, d, x, stream=None):
    """Fused on-chip solve of every system (tdma_solve_batched)."""
    L, C, keep = _prepare(layout, coeffs, d, x)
    _raise(lib().tdma_solve_batched(ctypes.byref(L), ctypes.byref(C), _dtype_code(d),
                                    ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                    _stream_handle(stream)))


def solve_batched_tiled(layout, coeffs, d, x, M, S, P, kernel=0, stream=None):
    """Fused solve with an explicit tile shape (tdma_solve_batched_tiled);
    kernel 0 = generic, 1 = shared-operator, 2 = its streaming form, 3 = shared
    operator + per-system shift, streaming (the next tile's rows loaded as the
    current one is stored), 4 = the same loading each tile at its start,
    5 = per-row coefficients on strided rows, streaming, 6 = kernel 2 with one
    register set refilled from the next tile as rows are stored (strided rows,
    M*P = n), which fits wider tiles, 7 = kernel 3 recomputing its pivots
    instead of keeping them (FP64, M*P = n), which fits 32-system tiles."""
    L, C, keep = _prepare(layout, coeffs, d, x)
    t = _Tile(int(M), int(S), int(P), int(kernel))
    _raise(lib().tdma_solve_batched_tiled(ctypes.byref(L), ctypes.byref(C), _dtype_code(d),
                                          ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                          ctypes.byref(t), _stream_handle(stream)))


class PoissonPlan:
    """The FFT-Poisson step (tdma_poisson_create / _solve / _destroy).  a, b, c:
    the z operator (nz values), shift: ny * (nx//2 + 1) values, mode (kx, ky)
    at ky * (nx//2 + 1) + kx; host arrays (numpy)."""

    def __init__(self, nx, ny, nz, a, b, c, shift):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, shift)]
        if any(v.size != nz for v in arrs[:3]) or arrs[3].size != ny * (nx // 2 + 1):
            raise ValueError("a, b, c need nz values and shift ny * (nx // 2 + 1)")
        self.shape = (int(nx), int(ny), int(nz))
        h = ctypes.c_void_p()
        _raise(lib().tdma_poisson_create(int(nx), int(ny), int(nz),
                                         *[ctypes.c_void_p(v.ctypes.data) for v in arrs],
                                         ctypes.byref(h)))
        self._h = h

    def solve(self, q, phi, stream=None):
        import torch
        nx, ny, nz = self.shape
        for nm, t in (("q", q), ("phi", phi)):
            _check_tensor(nm, t, nx * ny * nz, torch.float64)
        _raise(lib().tdma_poisson_solve(self._h, ctypes.c_void_p(q.data_ptr()),
                                        ctypes.c_void_p(phi.data_ptr()), _stream_handle(stream)))

    def destroy(self):
        if self._h is not None and self._h.value:
            lib().tdma_poisson_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def solve_pdd(layout, coeffs, d, x, rows_per_partition, stream=None):
    """PDD approximation with partitions of rows_per_partition rows
    (tdma_solve_pdd)."""
    L, C, keep = _prepare(layout, coeffs, d, x)
    _raise(lib().tdma_solve_pdd(ctypes.byref(L), ctypes.byref(C), _dtype_code(d),
                                int(rows_per_partition), ctypes.c_void_p(d.data_ptr()),
                                ctypes.c_void_p(x.data_ptr()), _stream_handle(stream)))


def solve_multi(layout, coeffs, d, x, nrhs, rhs_stride, stream=None):
    """nrhs right-hand sides per system, rhs_stride elements apart, over one
    shared operator per system (tdma_solve_multi)."""
    keep = []
    nrhs, rhs_stride = int(nrhs), int(rhs_stride)
    need = _extent(layout)
    if need and nrhs > 1:
        need += (nrhs - 1) * rhs_stride
    _check_tensor("d", d, need)
    _check_tensor("x", x, need, d.dtype)
    L = _make_layout(layout, keep)
    C = _make_coeffs(layout, coeffs, d, need)
    _raise(lib().tdma_solve_multi(ctypes.byref(L), ctypes.byref(C), _dtype_code(d), nrhs,
                                  rhs_stride, ctypes.c_void_p(d.data_ptr()),
                                  ctypes.c_void_p(x.data_ptr()), _stream_handle(stream)))


def solve_complex(layout, coeffs, d, x, stream=None):
    """Complex right-hand sides over a real shared operator: d and x are
    complex128 (complex64) tensors and ``layout`` counts complex elements; the
    coefficients are float64 (float32) tables.  The interleaved real and
    imaginary parts are solved as two right-hand sides (tdma_solve_multi)."""
    import torch
    if not (d.is_complex() and x.is_complex() and d.dtype == x.dtype):
        raise TypeError("d and x must be complex tensors of one dtype")
    dr = torch.view_as_real(d.reshape(-1) if d.is_contiguous() else d).reshape(-1)
    xr = torch.view_as_real(x.reshape(-1) if x.is_contiguous() else x).reshape(-1)
    if dr.data_ptr() != d.data_ptr() or xr.data_ptr() != x.data_ptr():
        raise ValueError("d and x must be contiguous")

    class _Real:
        pass

    lr = _Real()
    lr.n = int(layout.n)
    lr.nsys0 = int(layout.nsys0)
    lr.nsys1 = int(getattr(layout, "nsys1", 1))
    lr.row_stride = 2 * int(getattr(layout, "row_stride", 1))
    lr.sys_stride0 = 2 * int(getattr(layout, "sys_stride0", 0))
    lr.sys_stride1 = 2 * int(getattr(layout, "sys_stride1", 0))
    lr.offsets = None
    if getattr(layout, "offsets", None) is not None:
        raise ValueError("complex right-hand sides need a uniform layout")
    solve_multi(lr, coeffs, dr, xr, 2, 1, stream)


def copy_streamed(layout, src, dst, stream=None):
    """dst = src on every system row with the streaming solve's access pattern
    and no arithmetic (tdma_copy_streamed): the memory ceiling of that pattern."""
    keep = []
    need = _extent(layout)
    _check_tensor("src", src, need)
    _check_tensor("dst", dst, need, src.dtype)
    L = _make_layout(layout, keep)
    _raise(lib().tdma_copy_streamed(ctypes.byref(L), _dtype_code(src), ctypes.c_void_p(src.data_ptr()),
                                    ctypes.c_void_p(dst.data_ptr()), _stream_handle(stream)))


def solve_partitioned(layout, coeffs, d, x, partitions=0, batch=0, nstreams=0, schedule=0,
                      stream=None):
    """Staged A/B/C solve pipelined over HIP streams (tdma_solve_partitioned)."""
    L, C, keep = _prepare(layout, coeffs, d, x)
    o = _PartOpts(int(partitions), int(batch), int(nstreams), int(schedule))
    _raise(lib().tdma_solve_partitioned(ctypes.byref(L), ctypes.byref(C), _dtype_code(d),
                                        ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                        ctypes.byref(o), _stream_handle(stream)))


def solve_refined(layout, coeffs, d, x, max_iters=3, tol=1e-15, fallback=1, report=True,
                  stream=None, criterion=0, noalloc=False):
    """FP32 sweeps with FP64 refinement (tdma_solve_refined, or with
    noalloc=True tdma_solve_refined_noalloc, which allocates no device
    memory).  Returns the report as a dict when report=True (the call then
    synchronises).  criterion 0 tests the last correction against tol, 1 the
    remaining error estimated from the observed contraction."""
    import torch
    if d.dtype != torch.float64:
        raise TypeError("tdma_solve_refined takes FP64 d and x")
    L, C, keep = _prepare(layout, coeffs, d, x)
    o = _RefineOpts(int(max_iters), float(tol), int(fallback), int(criterion))
    rep = RefineReport()
    fn = lib().tdma_solve_refined_noalloc if noalloc else lib().tdma_solve_refined
    _raise(fn(ctypes.byref(L), ctypes.byref(C), ctypes.c_void_p(d.data_ptr()),
              ctypes.c_void_p(x.data_ptr()), ctypes.byref(o),
              ctypes.byref(rep) if report else None, _stream_handle(stream)))
    return rep.as_dict() if report else None


class Graph:
    """A recorded batching-form launch (tdma_graph_*).  The graph's kernels
    hold raw pointers to every item's d, x and coefficient tensors, so the
    Graph keeps references to them for as long as it exists."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def launch(self, stream=None):
        _raise(lib().tdma_graph_launch(self._h, _stream_handle(stream)))

    def destroy(self):
        if self._h:
            lib().tdma_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def graph_create(items):
    """items: list of dict(layout=, coeffs=, d=, x=, after=-1)."""
    keep = []
    arr = (_WorkItem * len(items))()
    dtype = None
    for k, it in enumerate(items):
        d, x = it["d"], it["x"]
        L, C, kk = _prepare(it["layout"], it["coeffs"], d, x)
        keep.extend(kk)
        keep.extend([d, x])
        dc = _dtype_code(d)
        if dtype is not None and dc != dtype:
            raise TypeError("all graph items must share one dtype")
        dtype = dc
        arr[k].layout = L
        arr[k].coeffs = C
        arr[k].d = d.data_ptr()
        arr[k].x = x.data_ptr()
        arr[k].after = int(it.get("after", -1))
    h = ctypes.c_void_p()
    _raise(lib().tdma_graph_create(arr, len(items), dtype if dtype is not None else F64,
                                   ctypes.byref(h)))
    return Graph(h, keep)


def autotune(layout, coeffs, d, x, what=0, stream=None):
    """Tune and cache (tdma_autotune); returns the JSON record as a dict."""
    import json
    L, C, keep = _prepare(layout, coeffs, d, x)
    _raise(lib().tdma_autotune(ctypes.byref(L), ctypes.byref(C), _dtype_code(d),
                               ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(x.data_ptr()), int(what),
                               _stream_handle(stream)))
    return json.loads(lib().tdma_autotune_last_json().decode())


def pipeline_model_ms(nsys, batch, t_a, t_b, t_c, concurrent=1):
    """The staged path's pipeline model (tdma_pipeline_model_ms)."""
    return lib().tdma_pipeline_model_ms(int(nsys), int(batch), float(t_a), float(t_b), float(t_c),
                                        int(concurrent))


def check(stream=None):
    """Synchronise and raise TdmaError(ESINGULAR) if a kernel met a bad pivot."""
    _raise(lib().tdma_check(_stream_handle(stream)))


def shutdown():
    lib().tdma_shutdown()
