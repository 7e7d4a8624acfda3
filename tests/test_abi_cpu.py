"""Host-side logic of libpd and its C ABI, without a GPU: the library loads and
exports every entry point declared in include/pd.h, validates its arguments,
samples the field like the oracle does, and reports device failures as
status codes."""
import ctypes
import json
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_1607_03062_amd as pd
from paper_1607_03062_amd import _lib
from paper_1607_03062_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(pd_\w+)\s*\(", text, flags=re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib = pd.require_native()
    names = declared_symbols()
    assert {"pd_create_grid", "pd_set_field", "pd_propagate", "pd_density"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), "libpd.so does not export %s" % n
    # the Python binding covers every declared entry point
    bound = {s[0] for s in _lib.SIGNATURES}
    assert names <= bound, names - bound


def test_version():
    assert "gfx950" in pd.version()


@pytest.mark.parametrize("args", [
    (0, 4, -1, 1, -1, 1, 0, 0),
    (4, 70000, -1, 1, -1, 1, 0, 0),
    (4, 4, 1, 1, -1, 1, 0, 0),
    (4, 4, -1, 1, 2, -2, 0, 0),
    (4, 4, -1, float("nan"), -1, 1, 0, 0),
    (4, 4, -1, float("inf"), -1, 1, 0, 0),
    (4, 4, -1, 1, -1, 1, 7, 0),
    (4, 4, -1, 1, -1, 1, 0, 9),
])
def test_create_grid_rejects_bad_arguments(args):
    lib = pd.require_native()
    h = ctypes.c_void_p(1)
    st = lib.pd_create_grid(*args, ctypes.byref(h))
    assert st == _lib.PD_ERR_INVALID
    assert h.value is None
    assert lib.pd_last_error().decode()


def test_last_error_is_per_thread():
    """Two threads fail different calls at the same time; after both have failed, each
    reads its own message (ctypes releases the GIL around the calls)."""
    import threading

    lib = pd.require_native()
    cases = [(0, 4, -1, 1, -1, 1, 0, 0), (4, 4, 2, 1, -1, 1, 0, 0)]
    msgs = [None, None]
    both_failed = threading.Barrier(2)

    def work(i):
        for _ in range(200):
            h = ctypes.c_void_p()
            assert lib.pd_create_grid(*cases[i], ctypes.byref(h)) == _lib.PD_ERR_INVALID
            both_failed.wait()
            m = lib.pd_last_error().decode()
            assert msgs[i] is None or m == msgs[i]
            msgs[i] = m
            both_failed.wait()

    ts = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert msgs[0] and msgs[1] and msgs[0] != msgs[1]
    ref = []
    for c in cases:  # the same messages as on a single thread
        assert lib.pd_create_grid(*c, ctypes.byref(ctypes.c_void_p())) == _lib.PD_ERR_INVALID
        ref.append(lib.pd_last_error().decode())
    assert msgs == ref


def test_null_handles():
    lib = pd.require_native()
    assert lib.pd_propagate(None, -1, None) == _lib.PD_ERR_INVALID
    assert lib.pd_density(None, None, 0, None, None) == _lib.PD_ERR_INVALID
    assert lib.pd_density_static(None, None, 0, None, None) == _lib.PD_ERR_INVALID
    assert lib.pd_state_bytes(None) == 0
    buf = np.zeros(64, dtype=np.uint8)
    assert lib.pd_save_state(None, buf.ctypes.data, 64, None, None) == _lib.PD_ERR_INVALID
    assert lib.pd_load_state(None, buf.ctypes.data, 64, 1, None) == _lib.PD_ERR_INVALID
    lib.pd_destroy_grid(None)


def test_static_density_rejects_grids_above_its_scratch():
    """pd_density_static serves grids of at most 2^28 points; a larger one is refused before
    any device work (the handle has no field and no device)."""
    big = pd.Solver(32768, 16384, (-1.0, 1.0), (-1.0, 1.0), "fp32")  # 2^29 points
    with pytest.raises(pd.PDError) as e:
        big.density_static()
    assert e.value.status == _lib.PD_ERR_INVALID and "static scratch" in e.value.message
    big.close()
    ok = pd.Solver(16384, 16384, (-1.0, 1.0), (-1.0, 1.0), "fp32")  # 2^28 points: size accepted, no field yet
    with pytest.raises(pd.PDError) as e:
        ok.density_static()
    assert e.value.status == _lib.PD_ERR_STATE
    ok.close()


@pytest.mark.parametrize("kind", ["sin2", "constant", "pulse"])
def test_field_sampling_matches_oracle(kind):
    """The library's host-side A(t) at the step midpoints equals the oracle's (independent code)."""
    if kind == "sin2":
        f, N = wl.sin2(0.16772546041219238, 0.25, 20), 40000
    elif kind == "constant":
        f, N = wl.constant(0.2, 200.0), 40000
    else:
        f = {"kind": "pulse", "E0": 1.0, "omega": 0.4876, "phi": 0.7, "omega_rise": 0.0609,
             "omega_fall": 0.0609, "duration": 70.9}
        N = 7000
    A, t_i, t_f, a_in, a_out = _lib.sample_field(f, N)
    Ao, a_in_o, a_out_o, dt_o = oracle.field_table(f, N)
    scale = max(1.0, np.abs(Ao).max())
    assert np.max(np.abs(A - Ao)) <= 4e-16 * scale * 8
    assert abs(a_in - a_in_o) <= 1e-16 and abs(a_out - a_out_o) <= 1e-15 * scale
    assert abs((t_f - t_i) / N - dt_o) <= 1e-18


def test_check_field_reports_step_bound_and_masking():
    s = pd.Solver.for_grid(wl.config1()["grid"])
    info = s.check_field(wl.config1()["field"], 4000)
    assert info["n_masked"] == 1
    assert abs(info["dt"] - 100.53096491487338 / 4000) < 1e-15
    # E_max: corner of the grid box (-2, 2 - 1/16) x A range
    A = oracle.field_table(wl.config1()["field"], 4000)[0]
    X = max(abs(-2 + A.min()), abs(-2 + A.max()), abs(1.9375 + A.min()), abs(1.9375 + A.max()))
    assert abs(info["E_max"] - math.hypot(X, 2.0)) < 1e-14
    # Sec. III step condition dt * E_max <= pi
    with pytest.raises(pd.PDError) as e:
        s.check_field(wl.config1()["field"], 90)
    assert e.value.status == _lib.PD_ERR_INVALID and "pi" in e.value.message
    s.close()


def test_rotation_form_choice():
    """Shears while every Bloch rotation angle (2 dt A_k, 2 dt px, 2 dt py) is <= pi/2."""
    s = pd.Solver(48, 40, (-4.0, 4.0), (-3.0, 3.0))
    assert s.check_field(wl.constant(0.2, 200.0), 4000)["rotation_form"] == 1  # 2 * 0.05 * 40 = 4
    assert s.check_field(wl.constant(0.2, 200.0), 40000)["rotation_form"] == 0  # 0.4
    s.close()
    s = pd.Solver.for_grid(wl.config3()["grid"], "fp32")
    assert s.check_field(wl.config3()["field"], 80000)["rotation_form"] == 0
    s.close()


def _tan_over_x_coefficients(n_max):
    """a_n of tan(z)/z = sum_{n>=1} a_n z^(2n-2), exactly, from the Bernoulli numbers:
    a_n = (-1)^(n-1) 2^(2n) (2^(2n) - 1) B_(2n) / (2n)!."""
    from fractions import Fraction

    B = [Fraction(1)]
    for m in range(1, 2 * n_max + 1):
        B.append(-sum(math.comb(m + 1, k) * B[k] for k in range(m)) / (m + 1))
    return [None] + [(-1) ** (n - 1) * 2 ** (2 * n) * (2 ** (2 * n) - 1) * B[2 * n] / math.factorial(2 * n)
                     for n in range(1, n_max + 1)]


def test_midpoint_form_and_series_order():
    """The midpoint step takes the tangent form while the state's growth over the
    1024-step renormalisation period, (1 / cos theta)^(1024 stages), stays below 2^32
    (theta = c_max dt E_max), else the cosine form.  The tangent series' order J keeps
    the omitted terms below the precision's rounding (2^-27 FP32, 2^-56 FP64) at the
    solve's largest x = theta^2, and the next smaller compiled order would not."""
    from fractions import Fraction

    a = _tan_over_x_coefficients(30)
    assert a[1:5] == [1, Fraction(1, 3), Fraction(2, 15), Fraction(17, 315)]
    compiled = {"fp32": [2, 3, 5], "fp64": [5, 7, 10]}
    g = {"nx": 37, "ny": 29, "px": (-3.0, 2.5), "py": (-2.0, 2.2)}
    seen = set()
    for scheme, stages, cmax in (("midpoint", 1, 1.0), ("midpoint4", 5, abs(1 - 4 / (4 - 4 ** (1 / 3))))):
        for prec in ("fp32", "fp64"):
            tol = 2.0 ** -27 if prec == "fp32" else 2.0 ** -56
            s = pd.Solver.for_grid(g, prec, scheme)
            for N in (60, 120, 200, 300, 450, 700, 1000, 2600, 9000, 40000):
                try:
                    info = s.check_field(wl.sin2(0.4, 0.7, 4), N)
                except pd.PDError:
                    continue
                theta = cmax * info["dt"] * info["E_max"]
                growth = 1024 * stages * -math.log2(math.cos(theta)) if theta < math.pi / 2 else math.inf
                x = theta * theta
                tail = lambda J: float(sum(a[n] * Fraction(x) ** (n - 1) for n in range(J + 1, 31)))
                fits = [J for J in compiled[prec] if tail(J) <= tol]
                want = 0 if growth <= 32 and fits else 1
                assert info["rotation_form"] == want, (scheme, prec, N, theta)
                if want == 0:
                    J = info["taylor_order"]
                    assert J == fits[0], (scheme, prec, N, J, fits)
                seen.add((scheme, prec, want))
            s.close()
    assert len(seen) == 8  # both forms in every scheme and precision


def test_masked_count_with_final_momentum_zero():
    """Constant field E0 = 0.2 on [0, 200]: A_out = -40, so p = (40, 0) has E_out = 0."""
    s = pd.Solver(81, 3, (0.0, 81.0), (-1.0, 2.0))  # p_x = 0, 1, ..., 80; p_y = -1, 0, 1
    info = s.check_field(wl.constant(0.2, 200.0), 40000)
    assert info["n_masked"] == 2  # p = (0, 0) and p = (40, 0)
    s.close()


@pytest.mark.parametrize("field,msg", [
    ({"kind": "sin2", "E0": 0.1, "omega": 0.5, "cycles": 1}, "cycles"),
    ({"kind": "sin2", "E0": float("nan"), "omega": 0.5, "cycles": 8}, "finite"),
    ({"kind": "constant", "E0": 0.1, "t_end": -1.0}, "t_end"),
    ({"kind": "pulse", "E0": 1.0, "omega": 0.5, "phi": 0, "omega_rise": 0.06, "omega_fall": 0.06,
      "duration": 10.0}, "shorter"),
    ({"kind": "sin2", "E0": 0.1, "omega": 0.0, "cycles": 8}, "omega > 0"),
    ({"kind": "sin2", "E0": 0.1, "omega": 0.5, "cycles": 8, "ellipticity": float("nan")}, "ellipticity"),
])
def test_bad_fields(field, msg):
    s = pd.Solver(8, 8, (-1, 1), (-1, 1))
    with pytest.raises(pd.PDError) as e:
        s.check_field(field, 1000)
    assert e.value.status == _lib.PD_ERR_INVALID and msg in e.value.message
    s.close()


@pytest.mark.parametrize("n_steps,msg", [(0, ">= 1"), (-5, ">= 1"), ((1 << 31) + 1, "2^31")])
def test_step_count_bounds(n_steps, msg):
    """N is at least 1 and at most 2^31 (checked before any table is allocated)."""
    s = pd.Solver(8, 8, (-1, 1), (-1, 1))
    with pytest.raises(pd.PDError) as e:
        s.check_field(wl.config1()["field"], n_steps)
    assert e.value.status == _lib.PD_ERR_INVALID and msg in e.value.message
    s.close()


def test_table_field_length_checked():
    s = pd.Solver(8, 8, (-1, 1), (-1, 1))
    f = {"kind": "table", "A_mid": np.zeros(10), "t_i": 0.0, "t_f": 1.0, "A_in": 0.0, "A_out": 0.0}
    with pytest.raises(pd.PDError):
        s.check_field(f, 11)
    assert s.check_field(f, 10)["n_steps"] == 10
    s.close()


def test_state_errors_without_device():
    s = pd.Solver(8, 8, (-1, 1), (-1, 1))
    with pytest.raises(pd.PDError) as e:
        s.propagate()
    assert e.value.status == _lib.PD_ERR_STATE
    with pytest.raises(pd.PDError) as e:
        s.density()
    assert e.value.status == _lib.PD_ERR_STATE
    with pytest.raises(pd.PDError):
        s.set_launch(3, 0)
    with pytest.raises(pd.PDError):
        s.set_launch(0, 512)
    with pytest.raises(pd.PDError):
        s.set_launch(0, 0, 3, 0)
    with pytest.raises(pd.PDError):
        s.set_launch(0, 0, 0, 100)
    with pytest.raises(pd.PDError):
        s.set_launch(0, 0, 0, 8192)
    with pytest.raises(pd.PDError) as e:
        s.resume(10)  # before pd_set_field
    assert e.value.status == _lib.PD_ERR_STATE and "pd_set_field" in e.value.message
    with pytest.raises(pd.PDError) as e:
        s.save_state()  # no solve in progress
    assert e.value.status == _lib.PD_ERR_STATE
    with pytest.raises(pd.PDError) as e:
        s.load_state(np.zeros(s.state_bytes(), dtype=np.uint8), 10)  # before pd_set_field
    assert e.value.status == _lib.PD_ERR_STATE
    s.set_launch(4, 64, 1, 256)
    info = s.info()
    assert (info["points_per_lane"], info["block_threads"], info["table_stage"], info["chunk_steps"]) == (4, 64, 1, 256)
    s.close()
    s = pd.Solver(8, 8, (-1, 1), (-1, 1), "fp32")
    assert s.info()["table_stage"] == 2 and s.info()["points_per_lane"] == 1
    with pytest.raises(pd.PDError):
        s.set_launch(0, 0, 0, 2048)  # FP32 chunks must divide the renormalisation period
    s.close()


def test_device_failure_is_a_status_not_a_crash():
    """Without a GPU the first device call fails with PD_ERR_DEVICE and a message."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    s = pd.Solver(8, 8, (-1, 1), (-1, 1))
    with pytest.raises(pd.PDError) as e:
        s.set_field(wl.sin2(0.1, 0.5, 8), 4000)
    assert e.value.status == _lib.PD_ERR_DEVICE
    s.close()


def test_state_bytes():
    s = pd.Solver(10, 7, (-1, 1), (-1, 1), "fp64", "strang")
    assert s.state_bytes() == 70 * 3 * 8
    s.close()
    s = pd.Solver(10, 7, (-1, 1), (-1, 1), "fp32", "midpoint")
    assert s.state_bytes() == 70 * 4 * 4
    s.close()


# ---------------------------------------------------------------------------
# Fourth-order composition, y component of the field, valley (host side)

ELLIPTIC_FIELDS = {
    "sin2": (wl.sin2(0.16772546041219238, 0.25, 20, 0.7), 4000),
    "constant": (wl.constant(0.2, 200.0, -0.5), 4000),
    "pulse": ({"kind": "pulse", "E0": 1.0, "omega": 0.4876, "phi": 0.7, "omega_rise": 0.0609,
               "omega_fall": 0.0609, "duration": 70.9, "ellipticity": 0.8}, 3000),
}


@pytest.mark.parametrize("scheme", ["strang", "strang4", "midpoint4"])
@pytest.mark.parametrize("kind", sorted(ELLIPTIC_FIELDS))
def test_field_sampling_xy_matches_oracle(kind, scheme):
    """Both components at every stage sample time equal the oracle's (independent code)."""
    f, N = ELLIPTIC_FIELDS[kind]
    Ax, Ay, ends = _lib.sample_field_xy(f, N, scheme)
    Ao, ax_in, ax_out, dt_o = oracle.field_table(f, N, scheme)
    Ayo, ay_in, ay_out = oracle.field_table_y(f, N, scheme)
    assert Ax.shape == Ao.shape == Ay.shape == Ayo.shape == (N * _lib.STAGES[scheme],)
    scale = max(1.0, np.abs(Ao).max(), np.abs(Ayo).max())
    assert np.max(np.abs(Ax - Ao)) <= 4e-15 * scale
    assert np.max(np.abs(Ay - Ayo)) <= 4e-15 * scale
    assert np.max(np.abs(Ay)) > 0.01  # the y component is there
    t_i, t_f, a_in, a_out, b_in, b_out = ends
    assert abs(a_in - ax_in) <= 1e-16 and abs(a_out - ax_out) <= 1e-14 * scale
    assert abs(b_in - ay_in) <= 1e-16 and abs(b_out - ay_out) <= 1e-14 * scale


def test_check_field_fourth_order_and_elliptic():
    """info reports the stages and the y component; E_max includes A_y; the step bound and
    masking use both components."""
    g = wl.grid(32, 2.0)
    f = wl.sin2(0.1, 0.5, 8, 0.6)
    s = pd.Solver.for_grid(g, "fp64", "strang4")
    info = s.check_field(f, 1000)
    assert info["stages"] == 5 and info["elliptic"] == 1 and info["valley"] == _lib.PD_VALLEYS_BOTH
    Ax, Ay, _ = _lib.sample_field_xy(f, 1000, "strang4")
    X = max(abs(-2 + Ax.min()), abs(-2 + Ax.max()), abs(1.875 + Ax.min()), abs(1.875 + Ax.max()))
    Y = max(abs(-2 + Ay.min()), abs(-2 + Ay.max()), abs(1.875 + Ay.min()), abs(1.875 + Ay.max()))
    assert abs(info["E_max"] - math.hypot(X, Y)) <= 1e-14
    s.close()
    s = pd.Solver.for_grid(g, "fp64", "midpoint")
    assert s.check_field(wl.sin2(0.1, 0.5, 8), 1000)["elliptic"] == 0
    s.close()


def test_fourth_order_table_needs_stage_samples():
    s = pd.Solver(8, 8, (-1, 1), (-1, 1), "fp64", "midpoint4")
    f = {"kind": "table", "A_mid": np.zeros(10), "t_i": 0.0, "t_f": 1.0, "A_in": 0.0, "A_out": 0.0}
    with pytest.raises(pd.PDError) as e:
        s.check_field(f, 10)
    assert "5 * n_steps" in e.value.message
    f["A_mid"] = np.zeros(50)
    assert s.check_field(f, 10)["stages"] == 5
    f["Ay_mid"], f["Ay_in"], f["Ay_out"] = np.zeros(49), 0.0, 0.0
    with pytest.raises(ValueError):
        s.check_field(f, 10)
    s.close()


def test_masked_count_with_Ay():
    """A table field with A_y(t_i) = 0.25 masks the point p = (-A_x(t_i), -0.25)."""
    s = pd.Solver(8, 8, (-1.0, 1.0), (-1.0, 1.0))  # nodes -1, -0.75, ..., 0.75
    f = {"kind": "table", "A_mid": np.full(10, 0.5), "t_i": 0.0, "t_f": 1.0, "A_in": 0.5, "A_out": 0.3,
         "Ay_mid": np.full(10, 0.25), "Ay_in": 0.25, "Ay_out": 0.0}
    info = s.check_field(f, 10)
    # E_in = 0 at (-0.5, -0.25); E_out = 0 at (-0.3, 0) is not a node (-0.25 and -0.5 are)
    assert info["n_masked"] == 1 and info["Ay_in"] == 0.25
    f["A_out"] = 0.25
    assert s.check_field(f, 10)["n_masked"] == 2  # and (-0.25, 0)
    s.close()


def test_valley_selection():
    s = pd.Solver(8, 8, (-1, 1), (-1, 1))
    with pytest.raises(pd.PDError) as e:
        load_status = _lib.load().pd_set_valley(s.handle, 7)
        _lib.check(load_status, "pd_set_valley")
    assert e.value.status == _lib.PD_ERR_INVALID
    s.set_valley("K-")
    assert s.info()["valley"] == _lib.PD_VALLEY_KMINUS
    s.set_valley("both")
    s.close()
    h = _lib._vp()
    assert _lib.load().pd_create_grid(8, 8, -1.0, 1.0, -1.0, 1.0, 0, 4, ctypes.byref(h)) == _lib.PD_ERR_INVALID
    for scheme in ("strang4", "midpoint4"):
        pd.Solver(8, 8, (-1, 1), (-1, 1), "fp32", scheme).close()


def test_snapshot_and_valley_state_errors_without_device():
    s = pd.Solver(8, 8, (-1, 1), (-1, 1))
    with pytest.raises(pd.PDError) as e:
        s.snapshot()
    assert e.value.status == _lib.PD_ERR_STATE
    s.close()


def test_precision_values():
    """PD_FP32_FAST is an FP32 form (4-byte state); anything past it is rejected."""
    for prec, size in (("fp64", 8), ("fp32", 4), ("fp32fast", 4)):
        s = pd.Solver(10, 7, (-1, 1), (-1, 1), prec)
        assert s.state_bytes() == 10 * 7 * 3 * size
        assert s.info()["precision"] == _lib.PRECISIONS[prec] and s.info()["points_per_lane"] == (4 if size == 8 else 1)
        s.close()
    h = _lib._vp()
    assert _lib.load().pd_create_grid(8, 8, -1.0, 1.0, -1.0, 1.0, 3, 0, ctypes.byref(h)) == _lib.PD_ERR_INVALID


@pytest.mark.parametrize("spec,ok", [("alloc@1", True), ("launch@3", True), ("alloc@1000000", True), ("", True),
                                     (None, True), ("alloc", False), ("alloc@0", False), ("launch@-2", False),
                                     ("launch@", False), ("launch@2x", False), ("free@1", False), ("@1", False)])
def test_fault_spec(spec, ok):
    """pd_set_fault arms "alloc@K" / "launch@K" (K >= 1) and disarms on NULL or ""; any other
    text is PD_ERR_INVALID with a message naming the accepted forms (host-side only)."""
    lib = pd.require_native()
    st = lib.pd_set_fault(spec.encode() if spec is not None else None)
    if ok:
        assert st == _lib.PD_OK
    else:
        assert st == _lib.PD_ERR_INVALID and "alloc@K" in lib.pd_last_error().decode()
    assert lib.pd_set_fault(None) == _lib.PD_OK  # disarm for the other tests


def test_trace_lines_on_request():
    """PD_TRACE=1 makes traced entry points write "pd_trace <name> <ms> ms" to stderr as
    they return (here pd_set_field, which fails without a device); without it they write
    nothing."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1607_03062_amd as pd\n"
            "from paper_1607_03062_amd import workloads as wl\n"
            "s = pd.Solver.for_grid(wl.grid(8, 1.0), 'fp32')\n"
            "try:\n    s.set_field(wl.sin2(0.1, 0.5, 2), 100)\nexcept Exception:\n    pass\n") % ROOT
    env = dict(os.environ, HIP_VISIBLE_DEVICES="", PD_TRACE="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert re.search(r"^pd_trace pd_set_field [0-9.]+ ms$", out.stderr, flags=re.M), out.stderr
    env["PD_TRACE"] = "0"
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert "pd_trace" not in out.stderr


def test_checkpoint_file_is_checked_before_any_device_work(tmp_path):
    """A checkpoint file is plain .npz (no pickled objects); load_checkpoint refuses one
    written for another grid, precision, scheme or valley before it touches the device."""
    meta = {"grid": {"nx": 8, "ny": 8, "px": [-1.0, 1.0], "py": [-1.0, 1.0]}, "precision": "fp32",
            "scheme": "strang", "valley": "both", "field": wl.sin2(0.1, 0.5, 8), "n_steps": 4000,
            "steps_done": 100}
    path = tmp_path / "ck.npz"
    with open(path, "wb") as fh:
        np.savez(fh, state=np.zeros(8 * 8 * 3 * 4, dtype=np.uint8), meta=np.array(json.dumps(meta)))
    with np.load(path, allow_pickle=False) as z:
        assert json.loads(str(z["meta"]))["steps_done"] == 100
    for kwargs in ({"precision": "fp64"}, {"scheme": "midpoint"}, {"valley": "K-"}):
        args = dict({"precision": "fp32", "scheme": "strang", "valley": "both"}, **kwargs)
        s = pd.Solver(8, 8, (-1, 1), (-1, 1), **args)
        with pytest.raises(pd.PDError) as e:
            s.load_checkpoint(path)
        assert e.value.status == _lib.PD_ERR_INVALID and "does not match" in e.value.message
        s.close()
    s = pd.Solver(8, 9, (-1, 1), (-1, 1), "fp32")
    with pytest.raises(pd.PDError) as e:
        s.load_checkpoint(path)
    assert "grid" in e.value.message
    s.close()
