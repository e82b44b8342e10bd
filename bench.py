"""Benchmark: G unknowns/s and % of HBM roofline of the batched tridiagonal solve
on one MI355X, beside the CPU oracle.

Default workload: the ADI viscous z-sweep of a 256^3 grid (65,536 strided
z-lines of n = 256, one shared tanh-grid operator, smooth RHS + noise), FP64,
through tdma_solve_batched (fused on-chip Stage A/B/C).  One step = one full
solve of the workload.  Inputs are resident in HBM before timing; the step
cycles over several input/output buffer sets (>= 1 GiB in total) so the
256 MB Infinity Cache cannot serve a step from the previous one.

Prints ONE JSON line.  ``--gpus`` above 1 is refused: this build runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "G unknowns/s & % HBM peak: FP32+refine vs FP64 at ≤1e-12 rel err, 1 GPU"
HBM_PEAK_GBS = 8000.0


KERNEL_SOURCES = ["paper_2509_03933_amd/csrc/fused.hip", "paper_2509_03933_amd/csrc/tile.hip.h"]


def profiled_traffic(profile_name, sources):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile_name + ".md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "|", "#", "-")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if fields.get("kernel_source_sha256_16") != h.hexdigest()[:16]:
        return None
    try:
        return int(float(fields["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="adi", choices=["adi"])
    ap.add_argument("--grid", default="256,256,256")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "launches": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the systems shard across GPUs with no communication; see DESIGN.md).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        copy_calibration()
        return

    import paper_2509_03933_amd as tdma
    from workloads import configs, device

    nx, ny, nz = (int(v) for v in args.grid.split(","))
    p = configs.adi(nx, ny, nz)
    tt = torch.float64 if args.dtype == "f64" else torch.float32
    esz = 8 if args.dtype == "f64" else 4
    d0, coeffs = device.device_inputs(p, dtype=tt)
    lay = p.layout
    unknowns = lay.unknowns()
    bytes_per_step = 2 * esz * unknowns + 3 * esz * lay.n     # read d, write x, shared tables
    nsets = max(2, math.ceil((1 << 30) / (2 * esz * unknowns)))
    ds = [d0] + [d0.clone() for _ in range(nsets - 1)]
    xs = [torch.empty_like(d0) for _ in range(nsets)]
    stream = torch.cuda.current_stream()

    def step(i):
        tdma.solve_batched(lay, coeffs, ds[i % nsets], xs[i % nsets], stream=stream)

    for i in range(args.warmup):
        step(i)
    tdma.check(stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        step(i)
    e1.record(stream)
    torch.cuda.synchronize()
    tdma.check(stream)
    total_ms = e0.elapsed_time(e1)
    ms_step = total_ms / args.steps
    value = unknowns / (ms_step * 1e-3) / 1e9
    achieved = bytes_per_step / (ms_step * 1e-3) / 1e9

    # parity spot check of the timed output against the oracle (sampled systems)
    import oracle
    rs = np.random.default_rng(7)
    sample = np.unique(np.concatenate([[0, lay.nsys - 1], rs.integers(0, lay.nsys, 254)]))
    x_last = xs[(args.steps - 1) % nsets].double().cpu().numpy()
    worst = 0.0
    for s in sample:
        a, b, c, d = configs.system_inputs(p, int(s))
        if args.dtype == "f32":
            a, b, c, d = [v.astype(np.float32).astype(np.float64) for v in (a, b, c, d)]
        ref = oracle.thomas(a, b, c, d)
        got = x_last[lay.sys_rows(int(s))]
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded counter-based generator, generated in HBM)",
        "config": {"workload": f"adi_viscous_zsweep_{nx}x{ny}x{nz}", "systems": lay.nsys,
                   "n": lay.n, "coefficients": "shared tanh-grid operator",
                   "entry_point": "tdma_solve_batched", "buffer_sets": nsets},
        "max_rel_err_vs_oracle": worst,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(f"k_fused_adi{nx}x{ny}x{nz}_{args.dtype}", KERNEL_SOURCES),
                     "kernel": "k_fused", "algorithmic_bytes_per_launch": bytes_per_step},
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out))


def cpu_baseline(p, target_s):
    """The oracle (plain C FP64 Thomas, one thread) on the same workload's host
    inputs, repeated over whole passes until about target_s of CPU time."""
    import oracle
    from workloads import configs
    a, b, c, d = configs.full_arrays(p)
    x = None
    t0 = time.perf_counter()
    passes = 0
    while True:
        x = oracle.solve_batch(p.layout, p.mode, a, b, c, d, x=x)
        passes += 1
        el = time.perf_counter() - t0
        if el >= target_s or passes >= 1000:
            break
    unknowns = p.layout.unknowns() * passes
    return {"value": round(unknowns / el / 1e9, 4), "unit": "G unknowns/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{passes} full pass(es) of the same workload ({p.layout.unknowns()} unknowns "
                      f"each), {el:.1f} s wall, single-threaded C Thomas (FP64)"}


if __name__ == "__main__":
    main()
