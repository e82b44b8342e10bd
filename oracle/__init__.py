"""Oracle for the batched tridiagonal solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2509_03933_amd``) and never imports it.

``oracle.c`` computes x = A^{-1} d per system with the textbook Thomas
algorithm in FP64 (or long double), real or complex, and the PDD
approximation per system; see its header for the definitions and the paper
passages they follow.  This module builds ``liboracle.so`` with gcc
(``-O2 -ffp-contract=off``, no fast-math) and wraps it with ctypes.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OK = 0
EINVAL = -1
ENOMEM = -2
ESINGULAR = -4

F64 = 0
LONG_DOUBLE = 1


def build(force=False):
    """Compile liboracle.so (plain C, gcc).  Returns the path."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            dp = ctypes.POINTER(ctypes.c_double)
            i64 = ctypes.c_int64
            lib.oracle_thomas.argtypes = [i64, dp, dp, dp, dp, dp, ctypes.c_int]
            lib.oracle_thomas.restype = ctypes.c_int
            lib.oracle_solve_batch.argtypes = [
                i64, i64, i64, i64, i64, i64, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                dp, dp, dp, dp, dp, dp, ctypes.c_int, i64, i64, ctypes.POINTER(ctypes.c_int32)]
            lib.oracle_solve_batch.restype = ctypes.c_int64
            lib.oracle_matvec.argtypes = [i64, dp, dp, dp, dp, dp]
            lib.oracle_matvec.restype = None
            lib.oracle_pdd.argtypes = [i64, dp, dp, dp, dp, dp, i64]
            lib.oracle_pdd.restype = ctypes.c_int
            lib.oracle_thomas_z.argtypes = [i64, dp, dp, dp, dp, dp, ctypes.c_int]
            lib.oracle_thomas_z.restype = ctypes.c_int
            lib.oracle_solve_batch_z.argtypes = [
                i64, i64, i64, i64, i64, i64, dp, dp, dp, dp, dp, dp, ctypes.c_int, i64, i64,
                ctypes.POINTER(ctypes.c_int32)]
            lib.oracle_solve_batch_z.restype = ctypes.c_int64
            _lib = lib
    return _lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(x):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if x is not None else None


class OracleError(RuntimeError):
    pass


def thomas(a, b, c, d, precision=F64):
    """Solve one system (1-D arrays of equal length n).  a[0], c[n-1] unused."""
    a, b, c, d = _f64(a), _f64(b), _f64(c), _f64(d)
    n = d.size
    if not (a.size == b.size == c.size == n):
        raise ValueError("a, b, c, d must have equal length")
    x = np.empty(n)
    rc = _load().oracle_thomas(n, _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(x), precision)
    if rc != OK:
        raise OracleError(f"oracle_thomas failed: {rc}")
    return x


def solve_batch(layout, mode, a, b, c, d, shift=None, precision=F64, systems=None,
                x=None, status=False):
    """Solve every system of ``layout`` (a ``workloads.configs.Layout``-like
    object: n, nsys0, nsys1, row_stride, sys_stride0, sys_stride1, offsets).

    mode 0: a/b/c laid out like d;  mode 1: shared length-n tables (+ shift).
    ``systems`` = (begin, end) restricts the range.  Returns x (same shape as d);
    with status=True also the per-system status array."""
    d = _f64(d)
    a, b, c = _f64(a), _f64(b), _f64(c)
    shift = None if shift is None else _f64(shift)
    if x is None:
        x = np.zeros_like(d)
    nsys = layout.nsys0 * layout.nsys1
    beg, end = (0, nsys) if systems is None else systems
    st = np.zeros(nsys, dtype=np.int32)
    offs = None
    if layout.offsets is not None:
        offs = np.ascontiguousarray(layout.offsets, dtype=np.int64)
    failed = _load().oracle_solve_batch(
        layout.n, layout.nsys0, layout.nsys1, layout.row_stride, layout.sys_stride0,
        layout.sys_stride1,
        offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if offs is not None else None,
        mode, _ptr(a), _ptr(b), _ptr(c), _ptr(shift), _ptr(d), _ptr(x), precision, beg, end,
        st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if failed < 0:
        raise OracleError(f"oracle_solve_batch failed: {failed}")
    if status:
        return x, st
    if failed:
        raise OracleError(f"{failed} systems hit a zero or non-finite pivot")
    return x


def pdd(a, b, c, d, m):
    """PDD approximation (partitions of m rows) of one system; see oracle_pdd."""
    a, b, c, d = _f64(a), _f64(b), _f64(c), _f64(d)
    n = d.size
    if not (a.size == b.size == c.size == n):
        raise ValueError("a, b, c, d must have equal length")
    x = np.empty(n)
    rc = _load().oracle_pdd(n, _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(x), int(m))
    if rc != OK:
        raise OracleError(f"oracle_pdd failed: {rc}")
    return x


def _c128(x):
    return np.ascontiguousarray(x, dtype=np.complex128)


def _zptr(x):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def thomas_complex(a, b, c, d, precision=F64):
    """Solve one complex system (1-D arrays of equal length n, any of them
    complex) by the Thomas recurrences in complex arithmetic."""
    a, b, c, d = _c128(a), _c128(b), _c128(c), _c128(d)
    n = d.size
    if not (a.size == b.size == c.size == n):
        raise ValueError("a, b, c, d must have equal length")
    x = np.empty(n, dtype=np.complex128)
    rc = _load().oracle_thomas_z(n, _zptr(a), _zptr(b), _zptr(c), _zptr(d), _zptr(x), precision)
    if rc != OK:
        raise OracleError(f"oracle_thomas_z failed: {rc}")
    return x


def solve_batch_complex(layout, a, b, c, d, shift=None, precision=F64, systems=None, x=None):
    """Complex right-hand sides over shared real tables a, b, c (+ a real
    per-system shift): every system of ``layout``, whose strides count complex
    elements of the complex128 array ``d``.  Returns x (complex128, d's shape)."""
    d = _c128(d)
    a, b, c = _f64(a), _f64(b), _f64(c)
    shift = None if shift is None else _f64(shift)
    if x is None:
        x = np.zeros_like(d)
    nsys = layout.nsys0 * layout.nsys1
    beg, end = (0, nsys) if systems is None else systems
    st = np.zeros(nsys, dtype=np.int32)
    failed = _load().oracle_solve_batch_z(
        layout.n, layout.nsys0, layout.nsys1, layout.row_stride, layout.sys_stride0,
        layout.sys_stride1, _ptr(a), _ptr(b), _ptr(c), _ptr(shift), _zptr(d), _zptr(x), precision,
        beg, end, st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if failed < 0:
        raise OracleError(f"oracle_solve_batch_z failed: {failed}")
    if failed:
        raise OracleError(f"{failed} systems hit a zero or non-finite pivot")
    return x


def matvec(a, b, c, x):
    """y = A x for one system (FP64, no FMA)."""
    a, b, c, x = _f64(a), _f64(b), _f64(c), _f64(x)
    y = np.empty_like(x)
    _load().oracle_matvec(x.size, _ptr(a), _ptr(b), _ptr(c), _ptr(x), _ptr(y))
    return y


def solve_problem_systems(problem, sys_indices, precision=F64):
    """Oracle solution of selected systems of a ``workloads.configs.Problem``,
    rebuilt on the host from the seeded generator.  Returns a list of x arrays."""
    from workloads import configs
    out = []
    for s in sys_indices:
        a, b, c, d = configs.system_inputs(problem, int(s))
        out.append(thomas(a, b, c, d, precision))
    return out
