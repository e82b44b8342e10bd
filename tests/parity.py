"""Helpers for GPU-vs-oracle parity tests.

Inputs come from ``workloads`` (seeded, host), the expected values from
``oracle`` (plain C FP64 Thomas), the candidate from the HIP library through
its C ABI.  Errors are per system: max_i |x_i - x^_i| / max_i |x^_i|.
"""
import numpy as np

import oracle
from workloads import configs

TOL_F64 = 1e-12      # FP64 bar (relative, per system, infinity norm)
TOL_F32 = 1e-5       # plain FP32 bar
TOL_REFINED = 1e-12  # FP32 sweeps + FP64 refinement
# Ill-conditioned systems (the pinned FFT-Poisson mode (0, 0), kappa ~1e10 at
# n = 1024): the forward error of any FP64 solve grows like kappa * eps, and
# the FP64 oracle's own distance from the long-double oracle measures it.  A
# system that misses the bar against the FP64 oracle passes if its error
# against the long-double oracle is within max(bar, ILL_FACTOR * that
# distance).  Well-conditioned systems keep the bar.  The factor is the
# largest ratio (error vs long double) / (FP64 oracle vs long double)
# measured where the rule decides, over every path that solves the Poisson
# lines (tests/test_gpu_modes.py prints the per-mode tables): 3.86, the
# generic fused kernel on the pinned mode; the shifted-operator kernels,
# the staged path and the complex solve give 2.4-2.5 there, FP32 +
# refinement 0.3-3.1.  With a margin of 1.5: 6 (it was 10).
ILL_FACTOR = 6.0


def conditioned_error(x, a, b, c, d, tol):
    """(passes, err_vs_fp64, err_vs_long_double, fp64_oracle_err) for one
    system; the last two are None when the FP64 oracle alone decides."""
    ref = oracle.thomas(a, b, c, d)
    err64 = float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    if err64 <= tol:
        return True, err64, None, None
    ref_ld = oracle.thomas(a, b, c, d, oracle.LONG_DOUBLE)
    return _ill_conditioned(x, ref, ref_ld, tol, err64)


def _ill_conditioned(x, ref, ref_ld, tol, err64):
    scale = np.max(np.abs(ref_ld))
    err_ld = float(np.max(np.abs(x - ref_ld)) / scale)
    e_orc = float(np.max(np.abs(ref - ref_ld)) / scale)
    return err_ld <= max(tol, ILL_FACTOR * e_orc), err64, err_ld, e_orc


def conditioned_error_complex(x, a, b, c, d, tol):
    """conditioned_error for a complex right-hand side (complex oracle)."""
    ref = oracle.thomas_complex(a, b, c, d)
    err64 = float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    if err64 <= tol:
        return True, err64, None, None
    ref_ld = oracle.thomas_complex(a, b, c, d, oracle.LONG_DOUBLE)
    return _ill_conditioned(x, ref, ref_ld, tol, err64)


def low_modes(nx, ny, reach=3):
    """[((kx, ky), system)] for every mode with |kx|, |ky| <= reach, (0, 0)
    first, then by |kx| + |ky|."""
    modes = [(kx, ky) for ky in range(-reach, reach + 1) for kx in range(-reach, reach + 1)]
    modes.sort(key=lambda m: (m != (0, 0), abs(m[0]) + abs(m[1]), m))
    return [(m, (m[0] % nx) + nx * (m[1] % ny)) for m in modes]


def mode_table(label, rows, tol):
    """Check and print one path's low modes.  rows: [((kx, ky), x, (a, b, c,
    d), is_complex)].  Every mode gets its error against the FP64 oracle and
    against the long-double oracle, the FP64 oracle's own distance from the
    long-double one, and their ratio; a mode passes within the bar against
    the FP64 oracle or under the conditioned rule.  Returns the table."""
    table = []
    print(f"{label}: mode, err vs FP64 oracle, err vs long double, FP64 oracle vs long double, "
          f"ratio, rule", flush=True)
    for m, x, (a, b, c, d), cplx in rows:
        th = oracle.thomas_complex if cplx else oracle.thomas
        ref = th(a, b, c, d)
        ref_ld = th(a, b, c, d, oracle.LONG_DOUBLE)
        e64 = float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
        ok, _, eld, eorc = _ill_conditioned(x, ref, ref_ld, tol, e64)
        ok = e64 <= tol or ok
        rule = "bar" if e64 <= tol else "conditioned"
        ratio = eld / eorc if eorc > 0 else float("inf")
        print(f"  {m}: {e64:.3g} {eld:.3g} {eorc:.3g} {ratio:.3g} {rule}{'' if ok else ' FAIL'}")
        table.append(dict(mode=m, vs_oracle=e64, vs_long_double=eld, oracle_vs_long_double=eorc,
                          ratio=ratio, rule=rule, ok=ok))
    bad = [r for r in table if not r["ok"]]
    assert not bad, (label, bad)
    return table


def poisson_mode_rows(p, get, pin=None, reach=3):
    """mode_table rows for the low modes of an FFT-Poisson problem (real or
    two interleaved right-hand sides): get(problem, system) returns that
    system's solution on the host (complex for the complex problems).  Mode
    (0, 0) is taken from the pinned problem, or left out without one."""
    nx, ny, _ = p.grid
    cplx = p.nrhs == 2
    rows = []
    for m, s in low_modes(nx, ny, reach):
        q, sys = (pin, 0) if s == 0 else (p, s)
        if q is None:
            continue
        if cplx:
            re, im = configs.system_rhs(q, sys)
            b = q.b + (q.shift[sys] if q.shift is not None else 0.0)
            inputs = (q.a, b, q.c, re + 1j * im)
        else:
            inputs = configs.system_inputs(q, sys)
        rows.append((m, get(q, sys), inputs, cplx))
    return rows


def gather_rows(layout, arr):
    """(nsys, n) view of a uniform layout (copy), or list of arrays (ragged)."""
    if layout.ragged:
        off = layout.offsets
        return [arr[off[s]:off[s + 1]] for s in range(layout.nsys)]
    s = np.arange(layout.nsys, dtype=np.int64)
    base = (s % layout.nsys0) * layout.sys_stride0 + (s // layout.nsys0) * layout.sys_stride1
    idx = base[:, None] + np.arange(layout.n, dtype=np.int64)[None, :] * layout.row_stride
    return arr[idx]


def per_system_error(layout, x, ref):
    if layout.ragged:
        xs, rs = gather_rows(layout, x), gather_rows(layout, ref)
        return np.array([np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)
                         for a, b in zip(xs, rs)])
    X = gather_rows(layout, x)
    R = gather_rows(layout, ref)
    return np.max(np.abs(X - R), axis=1) / np.maximum(np.max(np.abs(R), axis=1), 1e-300)


def host_problem(p, dtype=np.float64):
    """Full host arrays of a problem and the coefficient dict for the oracle."""
    a, b, c, d = configs.full_arrays(p)
    return a, b, c, d


def oracle_solution(p, a, b, c, d, precision=oracle.F64):
    return oracle.solve_batch(p.layout, p.mode, a, b, c, d, shift=p.shift, precision=precision)


def to_device(arrs, dtype):
    import torch
    return [None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to("cuda", dtype)
            for v in arrs]


def device_coeffs(p, a, b, c, dtype):
    import torch
    ta, tb, tc = to_device([a, b, c], dtype)
    shift = None
    if p.shift is not None:
        shift = torch.from_numpy(p.shift).to("cuda", dtype)
    return dict(mode=p.mode, a=ta, b=tb, c=tc, shift=shift)
