"""Benchmark: momentum point-steps/s on one MI355X, FP32 and FP64 forms, with the
n(p) error against the FP64 CPU oracle, batch throughput, and serving latency.

A step is one whole solve of the precision-form workload: the 2048 x 2048
momentum grid on [-2,2]^2 under the sin^2 pulse (E0 = 0.1, omega = 0.5, 30
cycles), 80000 Strang steps (state init, propagation, projection on u_out,
density reduction and the copy of rho to the host).  The field table is
resident in HBM before the timed region (pd_set_field once, pd_rewind per
step).  The main line is the fast FP32 form (PD_FP32_FAST: shears of alternating
orientation, the two rotations of a stage in one plane merged into five shears),
which on this workload is within 1e-5 of FP64 at every point; the once-rounded FP32
form (PD_FP32) and the FP64 form of the same workload are timed beside it.  All are
checked against the FP64 CPU oracle on the 64 x 64 subsample (stride 32) and on the
larger sample whose oracle run is also the CPU baseline; the two FP32 forms also
against the FP64 form at every point of the grid.

The same JSON line carries two more objects (skip them with --no-batch / --no-serve):
  batch  the 64 seeded solves of the batch workload (grids 256^2..2048^2 on [-4,4]^2,
         5k-80k steps, the once-rounded FP32 form, whose worst subsample error there is
         the smaller; --batch-precision fp32fast for the fast one) in one graph-captured
         launch sequence per pass,
         autotuned, with its own roofline, the oracle on every member's 64 x 64
         subsample (error and CPU baseline) and every point against its FP64 solve;
  serve  a Poisson stream of solve requests (batch-workload distributions, half FP32
         and half FP64) served by continuous batching at 0.7 of the capacity measured
         in the same run: p50 / p99 / mean latency and sustained point-steps/s.

    python bench.py [--steps K] [--warmup W] [--precision fp32fast|fp32|fp64] [--no-batch] [--no-serve]
    python bench.py --workload batch|serve ...       (one of the two objects as its own line)
    python bench.py --summarize-profile DIR [...]    (text summary of rocprofv3 output)
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "momentum point-steps/s (FP32 vs FP64 form) at stated n(p) error; p50/p99 solve ms"

# Work per point-step of the Strang propagation kernel: three plane rotations of the
# Bloch vector per step.  The method's own (algorithmic) work is what a rotation
# needs; the FP32 form executes more for accuracy: each component is rounded once per
# rotation, which costs one add per rotation beyond the three shears.
#   shear form (every rotation angle <= pi/2): 3 FMA per rotation -> 9 FMA = 18 flop
#     executed: FP64 and fp32fast 18 flop / 9 VALU instructions; FP32 21 flop / 12
#   versine form: 2 FMA per rotated component -> 12 FMA = 24 flop
#     executed: FP64 24 flop / 12 instructions; FP32 (mul + fma + add per component) 24 / 18
# (rotation form, precision) -> (algorithmic flop, executed flop, executed VALU instructions)
FORM_NAMES = {"fp32": "FP32", "fp32fast": "fast FP32", "fp64": "FP64"}
ALGO = {(0, "fp64"): (18, 18, 9), (0, "fp32"): (18, 21, 12), (0, "fp32fast"): (18, 17, 9),
        (1, "fp64"): (24, 24, 12), (1, "fp32"): (24, 24, 18), (1, "fp32fast"): (24, 24, 18)}


def host_cpu_model() -> str:
    """The host CPU's model name and logical CPU count (from /proc/cpuinfo)."""
    try:
        names = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")]
    except OSError:
        return "unknown"
    return "%s (%d logical CPUs)" % (names[0], len(names)) if names else "unknown"


def algo(info: dict, precision: str):
    """(algorithmic flop, executed flop, VALU instructions) per point-step of the solve
    described by pd_info; a fourth-order step is `stages` = 5 second-order stages.
    Strang stage: three rotations (ALGO), a fourth one (the field part of the y
    rotation) when the field has a y component.  The fast FP32 form applies each pair of
    rotations in one plane as five shears (8 FMA + 1 add for two rotations where the
    triples take 9 FMA): it executes 17 flop where the method's step counts 18.  The
    roofline counts the smaller of the two.
    Midpoint stage, phase X = c dt(px + A) (1 add, FP64) and x = X^2 + Y^2 (1 fma):
      tangent form (rotation_form 0), J series terms: tan(x)/x - 1 (J - 2 fma + 1 mul),
      alpha, beta (2 fma), the update: FP32 mul + fma + add per component (16 flop, 12
      instr), FP64 2 fma per component (16 flop, 8 instr); in FP32 plus the conversion of
      X (x is formed in FP32);
      cosine form (rotation_form 1), order J: cos - 1 (J - 1 fma + 1 mul) and sin(x)/x
      (J fma), alpha, beta (2 mul), the update: FP64 3 fma per component (24 flop, 12
      instr), FP32 mul + 2 fma + add per component (24 flop, 16 instr) plus 3 conversions.
    A y component adds Y = Y0 + dy and Y^2 (2 flop; 2 instr, 3 in FP32 tangent form).
    Every midpoint operation is part of the method's step: algorithmic = executed.  The
    points of a lane share their column, so the phase add (and its FP32 conversion) is one
    instruction per lane: the instruction count divides it by points_per_lane."""
    stages = info.get("stages", 1) or 1
    ell = info.get("elliptic", 0)
    if info["scheme"] in (0, 2):
        fa, fe, i = ALGO[(info["rotation_form"], precision)]
        r = 4 if ell else 3
        return stages * fa * r // 3, stages * fe * r // 3, stages * i * r // 3
    J = info["taylor_order"]
    f32 = precision != "fp64"  # fp32fast runs as fp32
    ppl = info.get("points_per_lane", 1) or 1
    if info["rotation_form"] == 0:
        flops = 3 + (2 * (J - 2) + 1) + 4 + 16 + (2 if ell else 0)
        shared = 2 if f32 else 1  # phase add (+ FP32 conversion), once per lane
        instr = shared / ppl + 1 + (J - 1) + 2 + (12 if f32 else 8) + ((3 if f32 else 2) if ell else 0)
    else:
        flops = 3 + (2 * (J - 1) + 1) + 2 * J + 2 + 24 + (2 if ell else 0)
        instr = 1.0 / ppl + 1 + 2 * J + 2 + (16 + 3 if f32 else 12) + (2 if ell else 0)
    return stages * flops, stages * flops, stages * instr


# MI355X vector peaks from its unit counts and clock (256 CU, 2.4 GHz): FP64
# issues 64 lanes per clock per CU (78.6 TFLOP/s with FMA); unpacked FP32 with
# VGPR operands issues 128 lanes per clock per CU (157.3 TFLOP/s with FMA).
CU_CLOCKS_PER_S = 256 * 2.4e9
LANES_PER_CLK = {"fp64": 64, "fp32": 128, "fp32fast": 128}
PEAK_TFLOPS = {p: CU_CLOCKS_PER_S * l * 2 / 1e12 for p, l in LANES_PER_CLK.items()}
KERNEL_SRC = os.path.join(ROOT, "paper_1607_03062_amd", "csrc", "kernels.hip")


def kernel_hash(path: str = KERNEL_SRC) -> str:
    """Hash of the kernel source's code: comments and whitespace removed, so that a
    profile stays valid across edits that do not change the code."""
    import re

    with open(path) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    code = "".join(text.split())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def environment(torch, pd) -> dict:
    """Where a line was measured: the device, its peak clock, the software versions, the
    kernel source hash and the host CPUs the process may use."""
    props = torch.cuda.get_device_properties(0)
    env = {"gpu": props.name, "arch": props.gcnArchName, "compute_units": props.multi_processor_count,
           "hbm_gib": round(props.total_memory / 2 ** 30, 1), "peak_clock_ghz": None, "hip": torch.version.hip,
           "rocm": None, "torch": torch.__version__, "libpd": pd.version(), "kernel_code_sha256_16": kernel_hash(),
           "host_cpus": len(os.sched_getaffinity(0))}
    try:
        with open(os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), ".info", "version")) as fh:
            env["rocm"] = fh.read().strip()
    except OSError:
        pass
    # the HIP runtime torch already loaded (the same handle, not a second copy)
    try:
        with open("/proc/self/maps") as fh:
            hip_path = next((ln.split()[-1] for ln in fh if ln.rstrip().endswith("libamdhip64.so")
                             or "libamdhip64.so." in ln.split()[-1]), None)
        if hip_path:
            khz = ctypes.c_int()
            attr_clock_rate = 5  # hipDeviceAttributeClockRate: peak clock in kHz
            if ctypes.CDLL(hip_path).hipDeviceGetAttribute(ctypes.byref(khz), attr_clock_rate,
                                                           torch.cuda.current_device()) == 0:
                env["peak_clock_ghz"] = khz.value / 1e6
    except (OSError, StopIteration, AttributeError):
        pass
    return env


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
    if vals.get("kernel_code_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def time_form(pd, torch, c, precision, steps, warmup, ppl, block, stage=0, chunk=0, scheme="strang"):
    s = pd.Solver.for_grid(c["grid"], precision, scheme)
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

    # n(p) into pinned host memory (a new page-locked buffer), as a caller that moves
    # results off the device would allocate it
    n = torch.empty(c["grid"]["nx"] * c["grid"]["ny"], dtype=torch.float64, pin_memory=True).numpy()
    copy_s = []
    for _ in range(2):  # reduction + copy of n(p) to the host; the second pass is reported
        w0 = time.perf_counter()
        s.density(n_out=n, stream=st)
        copy_s.append(time.perf_counter() - w0)
    info = s.info()
    s.close()
    return {"t_total": t1 - t0, "wall": wall, "kernel_ms": kern_ms, "rho": rho, "n": n, "info": info,
            "n_to_host_ms": copy_s[-1] * 1e3}


def log(msg: str):
    """Progress line on stderr (the JSON line alone goes to stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def batch_object(args, pd, torch, np):
    """The 64 seeded batch-workload solves, FP32 form, one persistent graph-captured launch
    per pass (a pass = every member's whole solve), autotuned; device time from HIP events
    on the launch stream; every member checked against the oracle on its own 64 x 64
    subsample, which is also the CPU baseline."""
    from paper_1607_03062_amd import workloads as wl

    cfgs = wl.config4(count=args.batch_count)
    prec = args.batch_precision
    solvers = []
    for c in cfgs:
        s = pd.Solver.for_grid(c["grid"], prec)
        s.set_field(c["field"], c["n_steps"])
        solvers.append(s)
    total = float(sum(c["grid"]["nx"] * c["grid"]["ny"] * c["n_steps"] for c in cfgs))
    forms = {s.info()["rotation_form"] for s in solvers}
    st = torch.cuda.Stream()
    b = pd.Batch(solvers)
    t_tune = time.perf_counter()
    if not args.no_autotune:
        b.autotune(512, stream=st)
    t_tune = time.perf_counter() - t_tune
    for _ in range(args.batch_warmup):
        b.run(stream=st)
    torch.cuda.synchronize()
    passes = args.batch_passes
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(passes)]
    wall = []
    t0 = time.perf_counter()
    for i in range(passes):
        w0 = time.perf_counter()
        ev[i][0].record(st)
        rho = b.run(stream=st)
        ev[i][1].record(st)
        wall.append(time.perf_counter() - w0)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    dev_ms = float(np.mean([a.elapsed_time(c) for a, c in ev]))
    info = b.info()
    log("batch: %d passes, %.1f ms device time per pass" % (passes, dev_ms))
    # the same solves one after another, each alone with its default launch
    t1 = time.perf_counter()
    rho_alone = []
    n_gpu = []
    for s, c in zip(solvers, cfgs):
        s.rewind()
        s.propagate(-1, stream=st)
        n = np.empty(c["grid"]["nx"] * c["grid"]["ny"])
        rho_alone.append(s.density(n_out=n, stream=st))
        n_gpu.append(n[wl.subsample_indices(c["grid"]["nx"], 64)])
    t_seq = time.perf_counter() - t1
    same = bool(np.array_equal(np.array(rho_alone), rho))
    # every point of every member against its FP64 solve (the FP64 path is within 1e-12 of
    # the oracle); untimed
    full = None
    if not args.no_fp64_form:
        full = {"max_abs": 0.0, "worst_member": None, "members_over_1e-5": 0, "points_over_1e-5": 0}
        for s, c in zip(solvers, cfgs):
            npts = c["grid"]["nx"] * c["grid"]["ny"]
            n32, n64 = np.empty(npts), np.empty(npts)
            s.density(n_out=n32, stream=st)
            s64 = pd.Solver.for_grid(c["grid"], "fp64")
            s64.set_field(c["field"], c["n_steps"])
            s64.propagate(-1, stream=st)
            s64.density(n_out=n64, stream=st)
            s64.close()
            d = np.abs(n32 - n64)
            over = int(np.count_nonzero(d > 1e-5))
            full["points_over_1e-5"] += over
            full["members_over_1e-5"] += int(over > 0)
            if float(d.max()) > full["max_abs"]:
                full["max_abs"], full["worst_member"] = float(d.max()), c["name"]
        log("batch: full grids against FP64, worst %.2e (%s), %d members with points over 1e-5" % (
            full["max_abs"], full["worst_member"], full["members_over_1e-5"]))
    b.close()
    for s in solvers:
        s.close()
    algo_flop, exec_flop, instr = ALGO[(0, prec)]
    algo_flop = min(algo_flop, exec_flop)
    achieved = algo_flop * total / (dev_ms * 1e-3) / 1e12
    out = {
        "workload": "%d seeded solves (grids 256^2..2048^2 on [-4,4]^2, 5k-80k steps, sin^2 pulses E0 in "
                    "[0.05,0.5], omega in [0.1,1], 4-40 cycles), %s form, one persistent graph-captured "
                    "launch per pass" % (len(cfgs), FORM_NAMES[prec]),
        "solves": len(cfgs), "passes": passes, "warmup": args.batch_warmup, "point_steps_per_pass": total,
        "ms_per_pass": t / passes * 1e3, "device_ms_per_pass": dev_ms, "value": total * passes / t,
        "unit": "point-steps/s", "graph_captured": info["graph_captured"],
        "points_per_lane": info["points_per_lane"], "block_threads": info["block_threads"],
        "work_items": info["work_items"], "autotune_s": t_tune,
        "p50_ms": float(np.percentile(np.array(wall) * 1e3, 50)),
        "p99_ms": float(np.percentile(np.array(wall) * 1e3, 99)),
        "sequential_alone": {"value": total / t_seq, "ms": t_seq * 1e3, "rho_bitwise_equal_to_batch": same},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["fp32"], "traffic": None,
                     "flop_per_point_step": algo_flop, "executed_flop_per_point_step": exec_flop,
                     "valu_issue_frac": instr * total / (dev_ms * 1e-3) / (CU_CLOCKS_PER_S * LANES_PER_CLK["fp32"]),
                     "rotation_forms": sorted(forms)},
        "cpu_baseline": None,
        "n_error_full_grid_vs_fp64": full,
    }
    if not args.no_cpu_baseline:
        import oracle

        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        worst, worst_name, pts = 0.0, None, 0.0
        t0 = time.perf_counter()
        for q, c in enumerate(cfgs):
            idx = wl.subsample_indices(c["grid"]["nx"], 64)
            n_o = oracle.solve_grid(c["field"], c["grid"], c["n_steps"], idx=idx, threads=threads)[0]
            pts += idx.shape[0] * c["n_steps"]
            err = float(np.max(np.abs(n_gpu[q] - n_o)))
            if err > worst:
                worst, worst_name = err, c["name"]
            if q % 16 == 15:
                log("batch oracle: %d of %d members, worst %.2e" % (q + 1, len(cfgs), worst))
        t_cpu = time.perf_counter() - t0
        out["n_error_max_abs"] = worst
        out["n_error_worst_member"] = worst_name
        out["n_error_sample"] = "each member's 64x64 subsample vs the FP64 oracle"
        out["cpu_baseline"] = {"value": pts / t_cpu, "unit": "point-steps/s", "cores": threads, "kind": "oracle",
                               "cpu_model": host_cpu_model(),
                               "sample": "64x64 subsample of each of the %d members, %.3g FP64 Strang point-steps, "
                                         "%.1f s" % (len(cfgs), pts, t_cpu)}
    return out


def serve_object(args, pd, torch, np):
    """The serving workload: a Poisson stream of solve requests (batch-workload distributions,
    50/50 FP32/FP64) served by continuous batching; arrival rate 0.7 x the capacity measured
    in the same run on a closed set of requests present at t = 0."""
    from paper_1607_03062_amd import serve
    from paper_1607_03062_amd import workloads as wl

    st = torch.cuda.Stream()

    def make_ex():
        return serve.GpuExecutor(pd, stream=st, background_setup=not args.no_background_setup)
    budget = int(args.budget_gb * (1 << 30))
    epoch_ms = args.epoch_ms if (args.epoch_ms > 0 or args.policy != "srpt") else 3.0
    # untimed warm-up passes (another draw of 16 requests): the first launches load the
    # code object and instantiate the batch graph, the first allocations map memory
    for i in range(args.serve_warmup):
        warm = [serve.Request.from_workload(w) for w in wl.config5(count=16, seed=54 + 100 * i, rate_per_s=1e9)]
        ex = make_ex()
        serve.Server(ex, budget, epoch_steps=args.epoch_steps, policy=args.policy, epoch_ms=epoch_ms).run(warm)
        ex.close()
    # capacity: a closed set of requests, all present at t = 0; with --epoch-ms 0 (srpt) the
    # epoch length is tuned on it first, and the chosen length's passes give the capacity
    def capacity_set():
        return [serve.Request.from_workload(w) for w in wl.config5(count=args.capacity_requests, seed=55,
                                                                     rate_per_s=1e9)]
    cap_reqs = capacity_set()
    if args.serve_warmup:
        # one untimed pass over the same set: the first pass of that size still ran 35-45 ms
        # longer than the next ones, which would bias the first timed candidate
        ex = make_ex()
        serve.Server(ex, budget, epoch_steps=args.epoch_steps, policy=args.policy, epoch_ms=epoch_ms).run(capacity_set())
        ex.close()
    total_ps = float(sum(r.point_steps for r in cap_reqs))
    tuning = None
    if args.epoch_ms <= 0 and args.policy == "srpt":
        cands = [float(c) for c in args.epoch_candidates.split(",")]
        epoch_ms, spans = serve.tune_epoch_ms(make_ex, budget, cap_reqs,
                                              candidates=cands, repeats=2, epoch_steps=args.epoch_steps,
                                              policy=args.policy, defer_admissions=not args.no_defer_admissions)
        tuning = {"candidates_ms": cands, "makespans_s": {"%g" % c: v for c, v in spans.items()},
                  "chosen_ms": epoch_ms}
        cap_makespan = float(np.median(spans[epoch_ms]))
        log("serve: epoch length %g ms chosen (median capacity-pass makespans %s)" % (
            epoch_ms, {c: "%.3f s" % float(np.median(v)) for c, v in spans.items()}))
    else:
        ex = make_ex()
        cap = serve.Server(ex, budget, epoch_steps=args.epoch_steps, policy=args.policy, epoch_ms=epoch_ms,
                           defer_admissions=not args.no_defer_admissions).run(cap_reqs)
        ex.close()
        cap_makespan = cap.makespan_s
    kw = dict(epoch_steps=args.epoch_steps, policy=args.policy, epoch_ms=epoch_ms,
              defer_admissions=not args.no_defer_admissions)
    cap_ps = total_ps / cap_makespan
    mean_ps = total_ps / len(cap_reqs)
    capacity_rps = cap_ps / mean_ps
    rate = args.rate_per_s if args.rate_per_s else args.load * capacity_rps
    log("serve: capacity %.1f requests/s (%.3g point-steps/s); stream of %d requests at %.1f/s" % (
        capacity_rps, cap_ps, args.requests, rate))
    reqs = [serve.Request.from_workload(w) for w in wl.config5(count=args.requests, seed=5, rate_per_s=rate)]
    ex = make_ex()
    res = serve.Server(ex, budget, **kw).run(
        reqs, progress=lambda done, n, now: log("serve: %d of %d requests done at %.0f s" % (done, n, now)))
    reused = ex.reused
    ex.close()
    return {
        "workload": "Poisson stream of %d solve requests (batch-workload grid, field and step distributions, "
                    "50/50 FP32/FP64), rate %.1f req/s = %.2f x capacity, HBM budget %.0f GiB, %s epochs "
                    "(%d steps / %g ms)" % (args.requests, rate, rate / capacity_rps, args.budget_gb, args.policy,
                                            args.epoch_steps, epoch_ms),
        "requests": args.requests, "rate_per_s": rate, "load": rate / capacity_rps, "value": res.point_steps_per_s,
        "unit": "point-steps/s", "p50_ms": res.p50_ms, "p99_ms": res.p99_ms, "mean_ms": res.mean_ms,
        "completed": res.completed, "rejected": res.rejected, "cancelled": res.cancelled, "expired": res.expired,
        "failed": res.failed, "retried": res.retried, "makespan_s": res.makespan_s, "epochs": res.epochs,
        "mean_active": res.mean_active, "peak_bytes": res.peak_bytes, "budget_bytes": res.budget_bytes,
        "handles_reused": reused, "policy": args.policy, "epoch_ms": epoch_ms, "epoch_steps": args.epoch_steps,
        "background_setup": not args.no_background_setup, "defer_admissions": not args.no_defer_admissions,
        "epoch_tuning": tuning,
        "capacity": {"requests_per_s": capacity_rps, "point_steps_per_s": cap_ps,
                     "requests": args.capacity_requests, "makespan_s": cap_makespan},
    }


def summarize_profile(args):
    """Text summary of rocprofv3 CSV output: per-kernel calls and durations from a
    --kernel-trace --stats run, and FETCH_SIZE / WRITE_SIZE per dispatch of the
    propagation kernel from two --pmc runs, scaled by what the counters read for a
    plain device copy of known size (--calibrate-copy) in the same runs."""
    import csv
    import glob

    import numpy as np

    def rows(d, name):
        out = []
        for f in sorted(glob.glob(os.path.join(d, "**", "*" + name), recursive=True)):
            with open(f) as fh:
                out.extend(csv.DictReader(fh))
        return out

    lines = ["kernel_code_sha256_16: %s" % kernel_hash()]
    stats = rows(args.summarize_profile, "kernel_stats.csv")
    if stats:
        lines.append("%-100s %6s %14s %14s %14s %14s" % ("kernel", "calls", "total_ns", "average_ns", "min_ns",
                                                         "max_ns"))
        for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
            lines.append("%-100s %6s %14s %14.0f %14s %14s" % (r["Name"][:100], r["Calls"], r["TotalDurationNs"],
                                                               float(r["AverageNs"]), r["MinNs"], r["MaxNs"]))
    trace = rows(args.summarize_profile, "kernel_trace.csv")
    if trace and args.pass_gap_ms > 0:
        # passes: runs of kernels separated by device idle gaps longer than pass_gap_ms
        ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in trace)
        passes, cur = [], [ev[0]]
        for e in ev[1:]:
            if e[0] - max(x[1] for x in cur) > args.pass_gap_ms * 1e6:
                passes.append(cur)
                cur = []
            cur.append(e)
        passes.append(cur)
        lines.append("passes (separated by device idle gaps above %g ms):" % args.pass_gap_ms)
        for q, ps in enumerate(passes):
            span = max(x[1] for x in ps) - ps[0][0]
            busy, end = 0, ps[0][0]
            gaps = []
            for a, b, _ in ps:  # union of the kernels' intervals
                if a > end:
                    gaps.append(a - end)
                busy += max(0, b - max(a, end))
                end = max(end, b)
            names = {}
            for a, b, n in ps:
                names[n] = names.get(n, 0) + 1
            top = max(names, key=names.get)
            lines.append("  pass %d: %d kernels, span %.1f ms, device busy %.1f ms (%.3f), idle gaps: %d under 100 us "
                         "(%.1f ms), %d of 100 us - 1 ms (%.1f ms), %d above 1 ms (%.1f ms); most launched: %s (%d)" % (
                             q, len(ps), span / 1e6, busy / 1e6, busy / max(span, 1),
                             sum(g < 1e5 for g in gaps), sum(g for g in gaps if g < 1e5) / 1e6,
                             sum(1e5 <= g < 1e6 for g in gaps), sum(g for g in gaps if 1e5 <= g < 1e6) / 1e6,
                             sum(g >= 1e6 for g in gaps), sum(g for g in gaps if g >= 1e6) / 1e6, top[:60],
                             names[top]))
    for d in args.counter_dir:
        # every counter of a --pmc run, per kernel: mean per dispatch and number of dispatches
        per = {}
        for r in rows(d, "counter_collection.csv"):
            key = (r["Kernel_Name"], r["Counter_Name"])
            per.setdefault(key, {}).setdefault(r.get("Dispatch_Id", len(per)), 0.0)
            per[key][r.get("Dispatch_Id", len(per))] += float(r["Counter_Value"])
        lines.append("counters of %s (per dispatch, summed over the dimensions):" % d)
        for (k, c), v in sorted(per.items()):
            lines.append("  %s %s: %.6e (mean of %d dispatches)" % (k[:100], c, float(np.mean(list(v.values()))),
                                                                   len(v)))
    for counter, d in (("FETCH_SIZE", args.fetch_dir), ("WRITE_SIZE", args.write_dir)):
        if not d:
            continue
        per_kernel = {}
        for r in rows(d, "counter_collection.csv"):
            if r.get("Counter_Name") != counter:
                continue
            per_kernel.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        for k, v in sorted(per_kernel.items()):
            lines.append("%s %s KiB per dispatch (mean of %d): %.3f" % (k[:100], counter, len(v), float(np.mean(v))))
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["cfg3", "batch", "serve"], default="cfg3",
                    help="cfg3 (default): the 2048^2 line with the batch and serve objects; batch / serve: one "
                         "of the objects alone")
    ap.add_argument("--no-batch", action="store_true", help="leave the batch object out of the cfg3 line")
    ap.add_argument("--no-serve", action="store_true", help="leave the serve object out of the cfg3 line")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-precision", choices=["fp32", "fp32fast"], default="fp32",
                    help="FP32 form of the batch's solves")
    ap.add_argument("--batch-passes", type=int, default=3)
    ap.add_argument("--batch-warmup", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--capacity-requests", type=int, default=48)
    ap.add_argument("--serve-warmup", type=int, default=2)
    ap.add_argument("--load", type=float, default=0.7)
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--epoch-steps", type=int, default=2048)
    ap.add_argument("--policy", choices=["lockstep", "srpt"], default="srpt",
                    help="serving: how an epoch shares the device (paper_1607_03062_amd/serve.py)")
    ap.add_argument("--epoch-ms", type=float, default=0.0,
                    help="serving (srpt): time budget of an epoch (0: tuned on the capacity requests)")
    ap.add_argument("--epoch-candidates", default="1.5,3,6", help="serving: epoch lengths (ms) the tuner times")
    ap.add_argument("--rate-per-s", type=float, default=0.0,
                    help="serving: arrival rate (default: --load x the capacity measured in the same run)")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp32", "fp64", "fp32fast"], default=None,
                    help="form of the main line (default: fp32fast for the Strang schemes, fp32 for the "
                         "midpoint schemes, whose FP32 forms are one)")
    ap.add_argument("--no-fast-form", action="store_true",
                    help="skip timing the other FP32 form (fp32 beside fp32fast, or fp32fast beside fp32)")
    ap.add_argument("--scheme", choices=["strang", "midpoint", "strang4", "midpoint4"], default="strang")
    ap.add_argument("--ellipticity", type=float, default=0.0,
                    help="give the workload pulse a y component E_y = e E0 sin^2(pi t/T) cos(omega t)")
    ap.add_argument("--n-steps", type=int, default=0, help="override the workload's 80000 steps")
    ap.add_argument("--ppl", type=int, default=0)
    ap.add_argument("--table-stage", type=int, default=0, help="1: LDS field rows, 2: scalar-unit rows (0: default)")
    ap.add_argument("--chunk-steps", type=int, default=0, help="LDS chunk length (0: default)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=256,
                    help="oracle subsample edge (timed as the CPU baseline, and the n(p) error sample)")
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (for counter calibration)")
    ap.add_argument("--summarize-profile", default="",
                    help="print a summary of the rocprofv3 --kernel-trace --stats output under this directory "
                         "and exit (no GPU work)")
    ap.add_argument("--fetch-dir", default="", help="with --summarize-profile: output of a --pmc FETCH_SIZE run")
    ap.add_argument("--write-dir", default="", help="with --summarize-profile: output of a --pmc WRITE_SIZE run")
    ap.add_argument("--counter-dir", action="append", default=[],
                    help="with --summarize-profile: output of a --pmc run; every counter per kernel (repeatable)")
    ap.add_argument("--pass-gap-ms", type=float, default=0.0,
                    help="with --summarize-profile: split the kernel trace into passes at device idle gaps longer "
                         "than this and report each pass's span and busy time")
    ap.add_argument("--no-background-setup", action="store_true",
                    help="serving: set up admitted requests on the scheduling thread (between epochs)")
    ap.add_argument("--no-defer-admissions", action="store_true",
                    help="serving: set up admissions right after a finishing epoch (before the next epoch)")
    args = ap.parse_args()
    if args.precision is None:
        args.precision = "fp32fast" if args.scheme.startswith("strang") else "fp32"
    if args.summarize_profile:
        return summarize_profile(args)
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (a solve would shard over bands of momentum "
              "rows, one reduction of rho; not implemented here). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1607_03062_amd as pd
    from paper_1607_03062_amd import workloads as wl

    pd.require_native()
    torch.cuda.set_device(0)
    if args.workload == "batch":
        print(json.dumps(dict(batch_object(args, pd, torch, np), metric=METRIC, n_gpus=1)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(dict(serve_object(args, pd, torch, np), metric=METRIC, n_gpus=1)), flush=True)
        return
    c = wl.config3(n=args.grid, precision=args.precision)
    if args.ellipticity:
        c["field"]["ellipticity"] = args.ellipticity
    if args.n_steps:
        c["n_steps"] = args.n_steps
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
        log("copy calibration: %d bytes read, %d bytes written" % (nb, nb))

    sch = args.scheme
    main_form = time_form(pd, torch, c, args.precision, args.steps, args.warmup, args.ppl, args.block,
                          args.table_stage, args.chunk_steps, scheme=sch)
    log("%s form: %.2f ms per solve" % (args.precision, main_form["t_total"] / args.steps * 1e3))
    other = None
    if not args.no_fp64_form and args.precision != "fp64":
        c64 = dict(c, field=dict(c["field"]), precision="fp64")
        other = time_form(pd, torch, c64, "fp64", args.steps, args.warmup, args.ppl, args.block, args.table_stage,
                          args.chunk_steps, scheme=sch)
        log("fp64 form: %.2f ms per solve" % (other["t_total"] / args.steps * 1e3))
    # the other FP32 form of the Strang schemes, timed and checked beside the main one
    alt_prec = {"fp32": "fp32fast", "fp32fast": "fp32"}.get(args.precision)
    fast = None
    if not args.no_fast_form and alt_prec and sch.startswith("strang"):
        fast = time_form(pd, torch, dict(c, field=dict(c["field"])), alt_prec, args.steps, args.warmup, args.ppl,
                         args.block, args.table_stage, args.chunk_steps, scheme=sch)
        log("%s form: %.2f ms per solve" % (alt_prec, fast["t_total"] / args.steps * 1e3))

    # oracle on the 64 x 64 subsample: n(p) error of each form and the CPU baseline
    n_err = {}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        sub = min(args.cpu_sample, args.grid)
        idx = wl.subsample_indices(args.grid, sub)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        n_o = oracle.solve_grid(c["field"], c["grid"], c["n_steps"], sch, idx=idx, threads=threads)[0]
        t_cpu = time.perf_counter() - t0
        log("oracle: %dx%d subsample in %.1f s" % (sub, sub, t_cpu))
        cpu = {"value": idx.shape[0] * c["n_steps"] / t_cpu, "unit": "point-steps/s", "cores": threads,
               "kind": "oracle", "cpu_model": host_cpu_model(),
               "sample": "%dx%d subsample (stride %d) of the %d^2 grid, %d FP64 %s steps, %.1f s" % (
                   sub, sub, args.grid // sub, args.grid, c["n_steps"], sch, t_cpu)}
        # the 64 x 64 subsample (stride grid/64) is contained in the larger one
        in64 = np.isin(idx, wl.subsample_indices(args.grid, 64))
        n_err[args.precision] = float(np.max(np.abs(main_form["n"][idx] - n_o)))
        n_err[args.precision + "_64"] = float(np.max(np.abs(main_form["n"][idx[in64]] - n_o[in64])))
        if other is not None:
            n_err["fp64"] = float(np.max(np.abs(other["n"][idx] - n_o)))
        if fast is not None:
            n_err["fast"] = float(np.max(np.abs(fast["n"][idx] - n_o)))
            n_err["fast_64"] = float(np.max(np.abs(fast["n"][idx[in64]] - n_o[in64])))

    # every point of the grid against the FP64 form, which is itself within 1e-12 of the oracle
    if other is not None:
        for key, form in (("", main_form), ("fast_", fast)):
            if form is not None:
                d = np.abs(form["n"] - other["n"])
                n_err[key + "full"] = float(d.max())
                n_err[key + "full_over"] = int(np.count_nonzero(d > 1e-5))

    K = args.steps
    t = main_form["t_total"]
    value = ps_per_solve * K / t
    kern_ms = float(np.mean(main_form["kernel_ms"]))
    flop_a, flop_e, instr = algo(main_form["info"], args.precision)
    flop_a = min(flop_a, flop_e)  # never more than the kernel executes
    achieved = flop_a * ps_per_solve / (kern_ms * 1e-3) / 1e12
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
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "%dx%d momentum grid on [-2,2]^2, sin^2 pulse E0=0.1 omega=0.5 30 cycles%s, "
                               "%d %s steps, %s form" % (args.grid, args.grid,
                                                         (" ellipticity %g" % args.ellipticity) if args.ellipticity
                                                         else "", c["n_steps"],
                                                         {"strang": "Strang", "midpoint": "midpoint",
                                                          "strang4": "fourth-order Strang",
                                                          "midpoint4": "fourth-order midpoint"}[sch],
                                                         FORM_NAMES[args.precision]),
                   "n_points": npts, "n_steps": c["n_steps"], "precision": args.precision, "scheme": sch,
                   "points_per_lane": main_form["info"]["points_per_lane"],
                   "block_threads": main_form["info"]["block_threads"]},
        # the workload's error is defined on the 64 x 64 subsample; the larger sample the CPU
        # baseline runs on is reported beside it
        "n_error_max_abs": n_err.get(args.precision + "_64"),
        "n_error_sample": "64x64 subsample (stride %d) vs the FP64 oracle" % (args.grid // 64),
        "n_error_max_abs_cpu_sample": n_err.get(args.precision),
        "cpu_sample_points": (min(args.cpu_sample, args.grid) ** 2) if not args.no_cpu_baseline else None,
        "n_error_max_abs_full_grid_vs_fp64": n_err.get("full"),
        "n_points_over_1e-5_full_grid_vs_fp64": n_err.get("full_over"),
        "rho": main_form["rho"],
        "p50_ms": float(np.percentile(wall_ms, 50)),
        "p99_ms": float(np.percentile(wall_ms, 99)),
        "kernel_ms": kern_ms,
        "n_to_host_ms": main_form["n_to_host_ms"],
        "value_with_n_to_host": ps_per_solve / (t / K + main_form["n_to_host_ms"] * 1e-3),
        # achieved and frac count the method's own work per point-step (flop_per_point_step);
        # the FP32 form's accuracy adds are reported as executed work beside it
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": traffic_from_profile(args.precision) if (sch == "strang" and not args.ellipticity)
                     else None,
                     "flop_per_point_step": flop_a, "executed_flop_per_point_step": flop_e,
                     "executed_tflops": flop_e * ps_per_solve / (kern_ms * 1e-3) / 1e12,
                     "valu_issue_frac": instr * ps_per_solve / (kern_ms * 1e-3) / (
                         CU_CLOCKS_PER_S * LANES_PER_CLK[args.precision])},
        "cpu_baseline": cpu,
    }
    if other is not None:
        okm = float(np.mean(other["kernel_ms"]))
        fa64, fe64, i64 = algo(other["info"], "fp64")
        fa64 = min(fa64, fe64)
        line["fp64_form"] = {
            "value": ps_per_solve * K / other["t_total"], "ms_per_step": other["t_total"] / K * 1e3,
            "kernel_ms": okm, "n_error_max_abs": n_err.get("fp64"), "rho": other["rho"],
            "rho_rel_diff_fp32_vs_fp64": main_form["rho"] / other["rho"] - 1,
            "roofline_frac": fa64 * ps_per_solve / (okm * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"],
            "valu_issue_frac": i64 * ps_per_solve / (okm * 1e-3) / (CU_CLOCKS_PER_S * LANES_PER_CLK["fp64"])}
    if fast is not None:
        fkm = float(np.mean(fast["kernel_ms"]))
        faf, fef, fi = algo(fast["info"], alt_prec)
        faf = min(faf, fef)
        line["fp32_fast_form" if alt_prec == "fp32fast" else "fp32_once_form"] = {
            "value": ps_per_solve * K / fast["t_total"], "ms_per_step": fast["t_total"] / K * 1e3,
            "kernel_ms": fkm, "n_error_max_abs": n_err.get("fast_64"),
            "n_error_max_abs_cpu_sample": n_err.get("fast"), "rho": fast["rho"],
            "n_error_max_abs_full_grid_vs_fp64": n_err.get("fast_full"),
            "n_points_over_1e-5_full_grid_vs_fp64": n_err.get("fast_full_over"),
            "roofline_frac": faf * ps_per_solve / (fkm * 1e-3) / 1e12 / PEAK_TFLOPS["fp32"],
            "valu_issue_frac": fi * ps_per_solve / (fkm * 1e-3) / (CU_CLOCKS_PER_S * LANES_PER_CLK["fp32"])}
    if not args.no_batch:
        line["batch"] = batch_object(args, pd, torch, np)
    if not args.no_serve:
        line["serve"] = serve_object(args, pd, torch, np)
    line["env"] = environment(torch, pd)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
