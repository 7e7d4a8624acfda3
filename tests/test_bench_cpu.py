"""The benchmark's bookkeeping on the CPU: the per-point-step work that `roofline`
divides by the kernel time (bench.ALGO, bench.algo) against the hardware counters the
committed rocprofv3 summaries recorded for the same kernels on the 2048^2 x 80000-step
workload, and the HBM traffic lookup against its summary."""
import os
import re

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
POINT_STEPS = 2048 * 2048 * 80000
KERNELS = {  # template arguments in the summaries -> (precision, executed flop, VALU instructions)
    "strang_kernel<double, 4, 0, 0, 1, 0, 0>": ("fp64", 18, 9),
    "strang_kernel<float, 1, 0, 0, 1, 0, 1>": ("fp32", 21, 12),
    "strang_kernel<float, 1, 0, 0, 1, 0, 2>": ("fp32fast", 17, 9),
}


def _blocks(path):
    """{kernel text: {key: first number}} of a VALU-issue summary."""
    out, cur = {}, None
    for line in open(path):
        if line.startswith("## "):
            cur = line[3:].strip()
            out[cur] = {}
        elif cur and ":" in line and not line.startswith("#"):
            key, rest = line.split(":", 1)
            m = re.search(r"[-+0-9.eE]+", rest)
            if m:
                out[cur][key.strip()] = float(m.group(0))
    return out


def test_strang_work_per_point_step():
    info = {"scheme": 0, "rotation_form": 0, "stages": 1, "elliptic": 0}
    assert bench.algo(info, "fp64") == (18, 18, 9)
    assert bench.algo(info, "fp32") == (18, 21, 12)
    assert bench.algo(info, "fp32fast") == (18, 17, 9)
    # a y component adds a fourth rotation per stage (the fast form merges it like the
    # x pair: two pairs of five shears); fourth order is five stages
    assert bench.algo(dict(info, elliptic=1), "fp32fast") == (24, 22, 12)
    assert bench.algo(dict(info, stages=5), "fp32") == (90, 105, 60)


def test_midpoint_work_per_point_step():
    """Tangent form of Eq. (13), J series terms, four points per lane sharing the phase."""
    info = {"scheme": 1, "rotation_form": 0, "taylor_order": 2, "points_per_lane": 4}
    flop_a, flop_e, instr = bench.algo(info, "fp32")
    assert flop_a == flop_e == 24 and instr == pytest.approx(16.5)
    flop_a, flop_e, instr = bench.algo(dict(info, taylor_order=5), "fp64")
    assert flop_a == flop_e == 30 and instr == pytest.approx(15.25)


def test_counts_match_the_recorded_hardware_counters():
    """FLOP counters equal the executed count exactly; VALU instructions are within 1.1% of
    the count (renormalisation and range ends are the rest)."""
    path = os.path.join(PROFILES, "strang_kernel_cfg3_valu_issue.txt")
    blocks = _blocks(path)
    seen = 0
    for name, vals in blocks.items():
        for key, (prec, flop, instr) in KERNELS.items():
            if key not in name:
                continue
            seen += 1
            a, e, i = bench.ALGO[(0, prec)]
            assert (e, i) == (flop, instr)
            assert vals["counted_flop"] == pytest.approx(e * POINT_STEPS, rel=2e-3), name
            assert vals["SQ_INSTS_VALU"] == pytest.approx(i * POINT_STEPS / 64, rel=1.1e-2), name
    assert seen == len(KERNELS)


def test_traffic_lookup_follows_the_kernel_source():
    """roofline.traffic is the summary's HBM bytes while the summary was taken on the
    current kernel source, else None."""
    for prec in ("fp32fast", "fp32", "fp64"):
        path = os.path.join(PROFILES, "strang_kernel_cfg3_%s_pmc.txt" % prec)
        vals = dict(ln.split(":", 1) for ln in open(path) if ":" in ln and not ln.startswith("#"))
        vals = {k.strip(): v.strip() for k, v in vals.items()}
        got = bench.traffic_from_profile(prec)
        if vals["kernel_code_sha256_16"] == bench.kernel_hash():
            assert got == float(vals["hbm_bytes_per_dispatch"])
            # at least the algorithmic bytes: n(p) written once, 8 bytes per point
            assert got >= 2048 * 2048 * 8
        else:
            assert got is None


def test_more_than_one_gpu_is_refused_with_a_message():
    """The benchmark runs on one GPU; --gpus 2 exits with status 2 and says why, before
    touching a device."""
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env=dict(os.environ, HIP_VISIBLE_DEVICES=""))
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr[-500:])
