"""Benchmark: momentum point-steps/s of one full solve on one MI355X.

A step is one whole solve of the precision-form workload: the 2048 x 2048
momentum grid on [-2,2]^2 under the sin^2 pulse (E0 = 0.1, omega = 0.5, 30
cycles), 80000 Strang steps (state init, propagation, projection on u_out,
density reduction and the copy of rho to the host).  The field table is
resident in HBM before the timed region (pd_set_field once, pd_rewind per
step).  The FP64 form of the same workload is timed beside it, and both are
checked against the FP64 CPU oracle on the 64 x 64 subsample (stride 32),
whose run is also the CPU baseline.

    python bench.py [--steps K] [--warmup W] [--precision fp32|fp64]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "momentum point-steps/s (FP32 vs FP64 form) at stated n(p) error; p50/p99 solve ms"

# Algorithmic work per point-step of the propagation kernel: three plane
# rotations of the Bloch vector per Strang step.
#   shear form (every rotation angle <= pi/2): 3 FMA per rotation -> 9 FMA = 18 flop, 9 VALU instructions
#   versine form, FP64: 2 FMA per rotated component -> 12 FMA = 24 flop, 12 instructions
#   versine form, FP32: mul + fma + add per rotated component -> 24 flop, 18 instructions
ALGO = {(0, "fp64"): (18, 9), (0, "fp32"): (18, 9), (1, "fp64"): (24, 12), (1, "fp32"): (24, 18)}
# MI355X vector peaks from its unit counts and clock (256 CU, 2.4 GHz): FP64
# issues 64 lanes per clock per CU (78.6 TFLOP/s with FMA); unpacked FP32 with
# VGPR operands issues 128 lanes per clock per CU (157.3 TFLOP/s with FMA).
CU_CLOCKS_PER_S = 256 * 2.4e9
LANES_PER_CLK = {"fp64": 64, "fp32": 128}
PEAK_TFLOPS = {p: CU_CLOCKS_PER_S * l * 2 / 1e12 for p, l in LANES_PER_CLK.items()}
KERNEL_SRC = os.path.join(ROOT, "paper_1607_03062_amd", "csrc", "kernels.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_from_profile(precision: str):
    """HBM bytes per launch of the propagation kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "strang_kernel_cfg3_%s_pmc.txt" % precision)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def time_form(pd, torch, c, precision, steps, warmup, ppl, block, stage=0, chunk=0):
    s = pd.Solver.for_grid(c["grid"], precision, "strang")
    if ppl or block or stage or chunk:
        s.set_launch(ppl, block, stage, chunk)
    s.set_field(c["field"], c["n_steps"])
    st = torch.cuda.Stream()
    for _ in range(warmup):
        s.rewind()
        s.propagate(-1, stream=st)
        s.density(stream=st)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    wall = []
    rho = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        w0 = time.perf_counter()
        s.rewind()
        starts[i].record(st)
        s.propagate(-1, stream=st)
        ends[i].record(st)
        rho = s.density(stream=st)  # copies rho to the host: waits for the stream
        wall.append(time.perf_counter() - w0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    import numpy as np

    n = np.empty(c["grid"]["nx"] * c["grid"]["ny"])
    s.density(n_out=n, stream=st)
    info = s.info()
    s.close()
    return {"t_total": t1 - t0, "wall": wall, "kernel_ms": kern_ms, "rho": rho, "n": n, "info": info}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--ppl", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=256,
                    help="oracle subsample edge (timed as the CPU baseline, and the n(p) error sample)")
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the solve shards over momentum points; "
              "multi-GPU runs are not part of it). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1607_03062_amd as pd
    from paper_1607_03062_amd import workloads as wl

    pd.require_native()
    torch.cuda.set_device(0)
    c = wl.config3(n=args.grid, precision=args.precision)
    npts = c["grid"]["nx"] * c["grid"]["ny"]
    ps_per_solve = npts * c["n_steps"]

    if args.calibrate_copy:
        nb = args.calibrate_copy * (1 << 20)
        a = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("copy calibration: %d bytes read, %d bytes written" % (nb, nb), file=sys.stderr)

    main_form = time_form(pd, torch, c, args.precision, args.steps, args.warmup, args.ppl, args.block)
    other = None
    if not args.no_fp64_form and args.precision != "fp64":
        other = time_form(pd, torch, wl.config3(n=args.grid, precision="fp64"), "fp64", args.steps, args.warmup,
                          args.ppl, args.block)

    # oracle on the 64 x 64 subsample: n(p) error of each form and the CPU baseline
    n_err = {}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        sub = min(args.cpu_sample, args.grid)
        idx = wl.subsample_indices(args.grid, sub)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        n_o = oracle.solve_grid(c["field"], c["grid"], c["n_steps"], "strang", idx=idx, threads=threads)[0]
        t_cpu = time.perf_counter() - t0
        cpu = {"value": idx.shape[0] * c["n_steps"] / t_cpu, "unit": "point-steps/s", "cores": threads,
               "kind": "oracle",
               "sample": "%dx%d subsample (stride %d) of the %d^2 grid, %d FP64 Strang steps, %.1f s" % (
                   sub, sub, args.grid // sub, args.grid, c["n_steps"], t_cpu)}
        # the 64 x 64 subsample (stride grid/64) is contained in the larger one
        in64 = np.isin(idx, wl.subsample_indices(args.grid, 64))
        n_err[args.precision] = float(np.max(np.abs(main_form["n"][idx] - n_o)))
        n_err[args.precision + "_64"] = float(np.max(np.abs(main_form["n"][idx[in64]] - n_o[in64])))
        if other is not None:
            n_err["fp64"] = float(np.max(np.abs(other["n"][idx] - n_o)))

    K = args.steps
    t = main_form["t_total"]
    value = ps_per_solve * K / t
    kern_ms = float(np.mean(main_form["kernel_ms"]))
    flops, instr = ALGO[(main_form["info"]["rotation_form"], args.precision)]
    achieved = flops * ps_per_solve / (kern_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    wall_ms = np.array(main_form["wall"]) * 1e3
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "point-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": t / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "%dx%d momentum grid on [-2,2]^2, sin^2 pulse E0=0.1 omega=0.5 30 cycles, "
                               "%d Strang steps, %s form" % (args.grid, args.grid, c["n_steps"],
                                                              args.precision.upper()),
                   "n_points": npts, "n_steps": c["n_steps"], "precision": args.precision, "scheme": "strang",
                   "points_per_lane": main_form["info"]["points_per_lane"],
                   "block_threads": main_form["info"]["block_threads"]},
        "n_error_max_abs": n_err.get(args.precision),
        "n_error_max_abs_64x64": n_err.get(args.precision + "_64"),
        "rho": main_form["rho"],
        "p50_ms": float(np.percentile(wall_ms, 50)),
        "p99_ms": float(np.percentile(wall_ms, 99)),
        "kernel_ms": kern_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic_from_profile(args.precision),
                     "valu_issue_frac": instr * ps_per_solve / (kern_ms * 1e-3) / (
                         CU_CLOCKS_PER_S * LANES_PER_CLK[args.precision])},
        "cpu_baseline": cpu,
    }
    if other is not None:
        okm = float(np.mean(other["kernel_ms"]))
        f64, i64 = ALGO[(other["info"]["rotation_form"], "fp64")]
        line["fp64_form"] = {
            "value": ps_per_solve * K / other["t_total"], "ms_per_step": other["t_total"] / K * 1e3,
            "kernel_ms": okm, "n_error_max_abs": n_err.get("fp64"), "rho": other["rho"],
            "rho_rel_diff_fp32_vs_fp64": main_form["rho"] / other["rho"] - 1,
            "roofline_frac": f64 * ps_per_solve / (okm * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"],
            "valu_issue_frac": i64 * ps_per_solve / (okm * 1e-3) / (CU_CLOCKS_PER_S * LANES_PER_CLK["fp64"])}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
