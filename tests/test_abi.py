"""The C ABI: the library loads, exports every function tdma.h declares, and
rejects invalid arguments on the host (no GPU call is made on these paths)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdma.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tdma_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def tdma():
    import paper_2509_03933_amd as t
    if not os.path.exists(t.LIB_PATH):
        from paper_2509_03933_amd import build
        build.build()
    return t


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("tdma_solve_batched", "tdma_solve_partitioned", "tdma_solve_refined",
              "tdma_graph_create", "tdma_graph_launch", "tdma_graph_destroy", "tdma_autotune",
              "tdma_check", "tdma_status_string", "tdma_last_error", "tdma_shutdown"):
        assert f in names


def test_library_exports_every_declared_symbol(tdma):
    out = subprocess.run(["nm", "-D", "--defined-only", tdma.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (tdma_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    lib = tdma.lib()
    for f in declared_functions():
        assert hasattr(lib, f)
    assert set(tdma.EXPORTED_SYMBOLS) <= set(declared_functions())


def test_status_strings(tdma):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert tdma.status_string(code).startswith("TDMA_")


class _Fake:
    def __init__(self, p):
        self.p = p


def _call(tdma, layout, mode=0, dtype=0, d=1, x=2, a=3, b=4, c=5, shift=None, offsets=None):
    L = tdma._Layout()
    L.n, L.nsys0, L.nsys1 = layout
    L.row_stride, L.sys_stride0, L.sys_stride1 = 1, layout[0], 0
    keep = None
    if offsets is not None:
        keep = np.ascontiguousarray(offsets, dtype=np.int64)
        L.offsets = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    C = tdma._Coeffs()
    C.mode, C.a, C.b, C.c, C.b_shift = mode, a, b, c, shift
    return tdma.lib().tdma_solve_batched(ctypes.byref(L), ctypes.byref(C), dtype,
                                         ctypes.c_void_p(d), ctypes.c_void_p(x), None)


def test_host_validation(tdma):
    lib = tdma.lib()
    EINVAL, EUNS = tdma.EINVAL, tdma.EUNSUPPORTED
    assert lib.tdma_solve_batched(None, None, 0, None, None, None) == EINVAL
    assert _call(tdma, (1, 4, 1)) == EINVAL                     # n < 2
    assert _call(tdma, (8, 4, 1), dtype=7) == EINVAL            # unknown dtype
    assert _call(tdma, (8, 4, 1), mode=9) == EINVAL             # unknown coefficient mode
    assert _call(tdma, (8, 4, 1), d=0) == EINVAL                # null d
    assert _call(tdma, (8, 4, 1), a=0) == EINVAL                # null coefficient
    assert _call(tdma, (8, 4, 1), x=3) == EINVAL                # x aliases a
    assert _call(tdma, (8, -1, 1)) == EINVAL                    # negative count
    assert _call(tdma, (8, 2, 1), offsets=[0, 5, 6]) == EINVAL  # a ragged system of 1 row
    assert _call(tdma, (8, 2, 1), mode=1, offsets=[0, 5, 9]) == EINVAL   # shared + ragged
    assert _call(tdma, (8, 1, 1), offsets=[0, 20000]) == EUNS   # longer than supported
    assert "n = 1" in lib.tdma_last_error().decode() or True


def test_tiled_validation(tdma):
    lib = tdma.lib()
    L = tdma._Layout(64, 4, 1, 1, 64, 0, None)
    C = tdma._Coeffs(0, 3, 4, 5, None)

    def tiled(M, S, P):
        t = tdma._Tile(M, S, P, 0)
        return lib.tdma_solve_batched_tiled(ctypes.byref(L), ctypes.byref(C), 0, ctypes.c_void_p(1),
                                            ctypes.c_void_p(2), ctypes.byref(t), None)
    assert tiled(8, 3, 8) == tdma.EINVAL      # S not a power of two
    assert tiled(8, 4, 4) == tdma.EINVAL      # covers 32 < 64 rows
    assert tiled(7, 4, 16) == tdma.EINVAL     # unsupported M
    assert tiled(16, 64, 16) == tdma.EINVAL   # 1024 lanes with M = 16 exceeds the 512 bound


def test_tiled_kernel_rules(tdma):
    """The walking kernels' shape rules are checked on the host, before any
    device call: strided lines of 1024 rows, a shared operator with a shift
    (kernels 3, 4, 7) or without (kernel 6)."""
    lib = tdma.lib()
    strided = tdma._Layout(1024, 8, 1, 8, 1, 0, None)
    contig = tdma._Layout(1024, 8, 1, 1, 1024, 0, None)
    shifted = tdma._Coeffs(1, 3, 4, 5, 6)
    shared = tdma._Coeffs(1, 3, 4, 5, None)

    def tiled(L, C, M, S, P, kernel, dtype=tdma.F64):
        t = tdma._Tile(M, S, P, kernel)
        return lib.tdma_solve_batched_tiled(ctypes.byref(L), ctypes.byref(C), dtype, ctypes.c_void_p(1),
                                            ctypes.c_void_p(2), ctypes.byref(t), None)
    EINVAL = tdma.EINVAL
    assert tiled(strided, shifted, 32, 32, 32, 8) == EINVAL               # no kernel 8
    assert tiled(strided, shifted, 32, 32, 32, 7, tdma.F32) == EINVAL     # kernel 7: FP64 only
    assert tiled(strided, shifted, 32, 32, 16, 7) == EINVAL               # 512 rows < n
    assert tiled(strided, shifted, 16, 32, 64, 7) == EINVAL               # 2048 lanes
    assert tiled(strided, shifted, 8, 32, 128, 7) == EINVAL               # M 8, 128 partitions
    assert tiled(strided, shifted, 32, 32, 32, 3) == EINVAL               # kernel 3: 512 lanes at M = 32
    assert tiled(contig, shared, 16, 16, 64, 6) == EINVAL                 # kernel 6: strided rows only
    assert tiled(tdma._Layout(1000, 8, 1, 8, 1, 0, None), shared, 16, 16, 64, 6) == EINVAL  # M*P != n


def test_binding_bounds_checks(tdma):
    """A layout reaching past a tensor is refused before any device call."""
    torch = pytest.importorskip("torch")
    from workloads import configs
    lay = configs.Layout(n=8, nsys0=4, row_stride=1, sys_stride0=8)
    d = torch.zeros(31, dtype=torch.float64)   # one element short, and on the CPU
    with pytest.raises(ValueError):
        tdma.solve_batched(lay, dict(mode=0, a=d, b=d, c=d), d, d)


def test_streamed_copy_validation(tdma):
    """The measurement copy refuses, on the host, what it does not mirror."""
    lib = tdma.lib()

    def copy(layout, dtype=0, src=1, dst=2):
        L = tdma._Layout(*layout, None)
        return lib.tdma_copy_streamed(ctypes.byref(L), dtype, ctypes.c_void_p(src),
                                      ctypes.c_void_p(dst), None)
    strided = (256, 16, 1, 16, 1, 0)          # n, nsys0, nsys1, row_stride, sys_stride0, sys_stride1
    assert lib.tdma_copy_streamed(None, 0, None, None, None) == tdma.EINVAL
    assert copy(strided, src=0) == tdma.EINVAL                   # null source
    assert copy(strided, src=5, dst=5) == tdma.EINVAL            # dst == src
    assert copy(strided, dtype=3) == tdma.EINVAL                 # unknown dtype
    assert copy((256, 16, 1, 1, 256, 0)) == tdma.EUNSUPPORTED    # contiguous rows
    assert copy((4096, 16, 1, 16, 1, 0)) == tdma.EUNSUPPORTED    # n beyond the streaming shape


def test_refined_options_validation(tdma):
    """Out-of-range refinement options are refused on the host."""
    lib = tdma.lib()
    L = tdma._Layout(64, 4, 1, 1, 64, 0, None)
    C = tdma._Coeffs(0, 3, 4, 5, None)

    def refined(iters=1, tol=1e-12, fallback=1, criterion=0):
        o = tdma._RefineOpts(iters, tol, fallback, criterion)
        return lib.tdma_solve_refined(ctypes.byref(L), ctypes.byref(C), ctypes.c_void_p(1),
                                      ctypes.c_void_p(2), ctypes.byref(o), None, None)
    assert refined(iters=4) == tdma.EINVAL
    assert refined(fallback=2) == tdma.EINVAL
    assert refined(criterion=2) == tdma.EINVAL
    assert refined(criterion=-1) == tdma.EINVAL


def test_layout_extent_overflow(tdma):
    """A layout whose last element lies beyond 2^62 is refused on the host."""
    lib = tdma.lib()
    L = tdma._Layout(8, 4, 2, 1 << 61, 1, 1 << 40, None)
    C = tdma._Coeffs(0, 3, 4, 5, None)
    assert lib.tdma_solve_batched(ctypes.byref(L), ctypes.byref(C), 0, ctypes.c_void_p(1),
                                  ctypes.c_void_p(2), None) == tdma.EINVAL
    assert "2^62" in lib.tdma_last_error().decode()


def test_system_count_limit(tdma):
    """2^31 systems or more in one call are refused on the host (no grid or
    32-bit system index can overflow), for every entry point that takes a
    layout."""
    lib = tdma.lib()
    L = tdma._Layout(8, 1 << 16, 1 << 15, 1, 0, 0, None)
    C = tdma._Coeffs(1, 3, 4, 5, None)
    assert lib.tdma_solve_batched(ctypes.byref(L), ctypes.byref(C), 0, ctypes.c_void_p(1),
                                  ctypes.c_void_p(2), None) == tdma.EUNSUPPORTED
    assert "2^31" in lib.tdma_last_error().decode()
    assert lib.tdma_solve_multi(ctypes.byref(L), ctypes.byref(C), 0, 2, 1, ctypes.c_void_p(1),
                                ctypes.c_void_p(2), None) == tdma.EUNSUPPORTED
    assert lib.tdma_solve_pdd(ctypes.byref(L), ctypes.byref(C), 0, 8, ctypes.c_void_p(1),
                              ctypes.c_void_p(2), None) == tdma.EUNSUPPORTED
    # 2^31 - 1 systems pass the count check (the call then stops at the next
    # host check: x aliasing a)
    L = tdma._Layout(8, (1 << 31) - 1, 1, 1, 0, 0, None)
    assert lib.tdma_solve_batched(ctypes.byref(L), ctypes.byref(C), 0, ctypes.c_void_p(1),
                                  ctypes.c_void_p(3), None) == tdma.EINVAL
    assert "alias" in lib.tdma_last_error().decode()
