"""GPU path (HIP kernels behind the C ABI) against the FP64 CPU oracle.

Tolerances:
  FP64 forms: |n_gpu - n_oracle| <= 1e-12 per point and |rho_gpu / rho_oracle - 1| <= 1e-12.
    Both sides are FP64 with rounding ~1e-16 per operation; the difference grows
    with the number of unitary steps N (7e-14 at N = 80000 on the 2048^2 benchmark
    solve), and the GPU's factorised rotations add no truncation, so 1e-12 leaves
    more than a decade.
  FP32 precision form: |n_gpu - n_oracle| <= 1e-5 per point (the bar set for
    the FP32 form; FP32 rounding of the state grows to a few 1e-6 after 80000 steps,
    as tests/fp32_model.py predicts;
    the once-rounded form rounds each component once per rotation; the fast form's
    shears, of alternating orientation with same-plane rotations merged, reach up to
    about 1.8x its worst-point error on long solves over wide grids).
  p_y = 0 lines: exactly 0.0 on both sides (the sigma_x eigenstate is kept).
  Launch shape, chunking and repeats: bit-identical n and rho.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1607_03062_amd import workloads as wl

pytestmark = pytest.mark.gpu

FP64_N_ABS = 1e-12
FP64_RHO_REL = 1e-12
FP32_N_ABS = 1e-5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def run(pd, grid, field, N, precision="fp64", scheme="strang", ppl=0, block=0, chunks=None, bind=None, stage=0,
        chunk_steps=0):
    print("gpu solve: grid %dx%d N=%d %s %s ppl=%s block=%s stage=%s chunk=%s chunks=%s" % (
        grid["nx"], grid["ny"], N, precision, scheme, ppl, block, stage, chunk_steps, chunks), flush=True)
    s = pd.Solver.for_grid(grid, precision, scheme)
    s.set_launch(ppl, block, stage, chunk_steps)
    s.set_field(field, N)
    if bind is not None:
        s.bind_state(bind)
    if chunks:
        for c in chunks:
            s.propagate(c)
    else:
        s.propagate(-1)
    n = np.empty(grid["nx"] * grid["ny"])
    rho = s.density(n_out=n)
    info = s.info()
    s.close()
    return n, rho, info


RAGGED = {"nx": 37, "ny": 53, "px": (-1.3, 2.1), "py": (-0.9, 1.7)}
RAGGED_FIELD = wl.sin2(0.3, 0.6, 3)


@pytest.fixture(scope="module")
def cfg1_oracle():
    c = wl.config1()
    return {s: oracle.solve_grid(c["field"], c["grid"], c["n_steps"], s) for s in ("strang", "midpoint")}


@pytest.mark.parametrize("scheme", ["strang", "midpoint"])
def test_config1_fp64_full_grid(gpu, cfg1_oracle, scheme):
    c = wl.config1()
    n, rho, info = run(gpu, c["grid"], c["field"], c["n_steps"], "fp64", scheme)
    n_o, nd, masked = cfg1_oracle[scheme]
    rho_o = oracle.density(c["grid"], n_o)
    assert np.max(np.abs(n - n_o)) <= FP64_N_ABS
    assert abs(rho / rho_o - 1) <= FP64_RHO_REL
    assert info["n_masked"] == masked == 1
    row = n.reshape(64, 64)[32]  # p_y = 0
    assert np.all(row == 0.0)


@pytest.mark.parametrize("scheme", ["strang", "midpoint"])
def test_config1_fp32_form(gpu, cfg1_oracle, scheme):
    c = wl.config1()
    n, rho, info = run(gpu, c["grid"], c["field"], c["n_steps"], "fp32", scheme)
    n_o = cfg1_oracle[scheme][0]
    assert np.max(np.abs(n - n_o)) <= FP32_N_ABS
    assert np.all(n.reshape(64, 64)[32] == 0.0)
    assert abs(rho / oracle.density(c["grid"], n_o) - 1) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32fast"])
@pytest.mark.parametrize("scheme", ["strang", "midpoint"])
def test_ragged_grid_every_launch_shape(gpu, precision, scheme):
    """37 x 53 points (not a multiple of any tile), 777 steps: every launch shape gives the
    same bits, and the oracle's values."""
    N = 2777  # crosses the FP32 renormalisation steps 1024 and 2048
    n_o = oracle.solve_grid(RAGGED_FIELD, RAGGED, N, scheme)[0]
    ref = None
    shapes = [(ppl, block, 0, 0) for ppl in (1, 2, 4) for block in (64, 256)]
    if scheme == "strang":
        shapes += [(2, 128, 1, 64), (4, 256, 1, 1024), (1, 64, 2, 0), (2, 256, 1, 256)]
    for ppl, block, stage, chunk in shapes:
        n, rho, _ = run(gpu, RAGGED, RAGGED_FIELD, N, precision, scheme, ppl, block, stage=stage, chunk_steps=chunk)
        if ref is None:
            ref = (n, rho)
            tol = FP64_N_ABS if precision == "fp64" else FP32_N_ABS
            assert np.max(np.abs(n - n_o)) <= tol
        else:
            assert np.array_equal(n, ref[0]) and rho == ref[1], (ppl, block, stage, chunk)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32fast"])
@pytest.mark.parametrize("scheme", ["strang", "midpoint"])
def test_chunked_equals_single_launch(gpu, precision, scheme):
    """Propagation split into chunks that cross the FP32 renormalisation boundaries
    (every 1024 steps) reproduces the single launch bit for bit, with the handle's
    own state buffer and with a caller-owned torch buffer."""
    import torch

    N = 5000
    chunks = [1, 1023, 1, 2047, 1, 900, 1027]
    single = run(gpu, RAGGED, RAGGED_FIELD, N, precision, scheme)
    chunked = run(gpu, RAGGED, RAGGED_FIELD, N, precision, scheme, chunks=chunks)
    assert np.array_equal(single[0], chunked[0]) and single[1] == chunked[1]
    nbytes = RAGGED["nx"] * RAGGED["ny"] * (3 if scheme == "strang" else 4) * (8 if precision == "fp64" else 4)
    buf = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device="cuda")
    bound = run(gpu, RAGGED, RAGGED_FIELD, N, precision, scheme, chunks=[2500, 2500], bind=buf)
    assert np.array_equal(single[0], bound[0])


def test_every_point_of_a_long_solve_against_the_oracle(gpu):
    """256^2 on [-4,4]^2 under a 12-cycle sin^2 pulse (E0 = 0.25, omega = 0.4), 30000 Strang
    steps: every one of the 65536 points against the FP64 oracle (Sec. II Eq. (1), Sec. III
    Eqs. (9)-(12)), within 1e-12 in FP64 and 1e-5 in the FP32 form, and rho within 1e-12
    relative in FP64."""
    grid, field, N = wl.grid(256, 4.0), wl.sin2(0.25, 0.4, 12), 30000
    n_o = oracle.solve_grid(field, grid, N)[0]
    n64, rho64, _ = run(gpu, grid, field, N, "fp64")
    assert np.max(np.abs(n64 - n_o)) <= FP64_N_ABS
    assert abs(rho64 / oracle.density(grid, n_o) - 1) <= 1e-12
    n32, _, _ = run(gpu, grid, field, N, "fp32")
    err32 = np.max(np.abs(n32 - n_o))
    print("every point, 256^2 x 30000: fp32 max |dn| = %.3e, fp64 %.3e" % (err32, np.max(np.abs(n64 - n_o))))
    assert err32 <= FP32_N_ABS


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32fast"])
@pytest.mark.parametrize("scheme,ellipticity", [("strang", 0.0), ("midpoint", 0.0), ("strang4", 0.0),
                                                ("strang4", 0.5), ("strang", 0.5)])
def test_short_chunks_cover_every_group_count(gpu, precision, scheme, ellipticity):
    """The step loops run whole groups of steps (8 or 16 Strang steps, 4 midpoint steps) from
    two row sets in turn, or, for the long rows of the fourth-order and y-component FP32
    solves, groups of 4 steps each loading its next row one step ahead; then single steps.
    Chunks of 1-40 steps starting at every phase give ranges with no whole group, one, an
    odd and an even number of them, each with and without single steps around them; the
    result is the single launch bit for bit."""
    chunks = [5, 8, 16, 24, 17, 15, 9, 33, 64, 7, 40, 3, 32, 1, 31, 48, 4, 12, 20, 2]
    N = sum(chunks)
    field = dict(RAGGED_FIELD, ellipticity=ellipticity) if ellipticity else RAGGED_FIELD
    single = run(gpu, RAGGED, field, N, precision, scheme)
    chunked = run(gpu, RAGGED, field, N, precision, scheme, chunks=chunks)
    assert np.array_equal(single[0], chunked[0]) and single[1] == chunked[1]
    if scheme == "strang4" or ellipticity:
        n_o = oracle.solve_grid(field, RAGGED, N, scheme)[0]
        assert np.max(np.abs(single[0] - n_o)) <= (FP64_N_ABS if precision == "fp64" else FP32_N_ABS)


@pytest.mark.parametrize("precision,scheme,N,k", [("fp32", "strang", 3000, 1500), ("fp64", "strang", 2777, 1024),
                                                  ("fp64", "midpoint", 3000, 2047), ("fp32", "midpoint", 2600, 700),
                                                  ("fp32", "strang4", 600, 333), ("fp32fast", "strang", 3000, 701)])
def test_checkpoint_and_resume(gpu, precision, scheme, N, k):
    """A chunked solve stops after k steps and its bound state is saved to host memory; a new
    handle for the same solve gets the saved state in its own bound buffer, resumes at k and
    finishes: n(p) and rho bit-identical to the uninterrupted solve.  (The elliptic field puts
    the fourth-order case on the y-component path.)"""
    import torch

    field = dict(RAGGED_FIELD, ellipticity=0.5) if scheme == "strang4" else RAGGED_FIELD
    single = run(gpu, RAGGED, field, N, precision, scheme)
    s = gpu.Solver.for_grid(RAGGED, precision, scheme)
    s.set_field(field, N)
    nb = s.state_bytes()
    buf = torch.zeros(nb // 4 + 64, dtype=torch.float32, device="cuda")
    s.bind_state(buf)
    s.propagate(k)
    torch.cuda.synchronize()
    saved = buf.cpu().clone()
    s.close()
    del buf
    s2 = gpu.Solver.for_grid(RAGGED, precision, scheme)
    s2.set_field(field, N)
    with pytest.raises(gpu.PDError):
        s2.resume(k)  # no buffer bound yet
    buf2 = saved.to("cuda")
    s2.bind_state(buf2)
    for bad in (0, N):
        with pytest.raises(gpu.PDError):
            s2.resume(bad)
    s2.resume(k)
    assert s2.info()["steps_done"] == k
    s2.propagate(-1)
    n = np.empty(RAGGED["nx"] * RAGGED["ny"])
    rho = s2.density(n_out=n)
    s2.close()
    assert np.array_equal(n, single[0]) and rho == single[1]


@pytest.mark.parametrize("precision,scheme,field_kind,valley,N,k", [
    ("fp64", "strang", "sin2", "both", 2777, 1500), ("fp32", "midpoint", "sin2", "K-", 2600, 1031),
    ("fp32", "strang4", "elliptic", "both", 600, 333), ("fp32fast", "strang", "table", "K+", 3000, 2049)])
def test_checkpoint_file_restart(gpu, tmp_path, precision, scheme, field_kind, valley, N, k):
    """save_checkpoint after k steps writes the state (pd_save_state) with the solve's grid,
    precision, scheme, valley and field to an .npz file; the handle is closed; a new handle
    from the file (pd_load_state) finishes the solve: n(p) and rho bit-identical to the
    uninterrupted solve, which matches the oracle.  A second restart loads the same file
    into an existing handle with a caller-bound state buffer.  A handle of another precision
    refuses the file; a state of the wrong size and a step count outside 1 .. N - 1 are
    refused by the library."""
    import torch

    if field_kind == "table":
        t_f = 3 * 2 * math.pi / 0.6
        tt = (np.arange(N) + 0.5) * t_f / N
        field = {"kind": "table", "A_mid": 0.2 * np.sin(0.5 * tt) * np.sin(math.pi * tt / t_f) ** 2,
                 "t_i": 0.0, "t_f": t_f, "A_in": 0.0, "A_out": 0.0}
    else:
        field = dict(RAGGED_FIELD, ellipticity=0.5) if field_kind == "elliptic" else RAGGED_FIELD
    print("checkpoint file: %s %s %s %s N=%d k=%d" % (precision, scheme, field_kind, valley, N, k), flush=True)
    s0 = gpu.Solver.for_grid(RAGGED, precision, scheme, valley).set_field(field, N)
    s0.propagate(-1)
    n_single = np.empty(RAGGED["nx"] * RAGGED["ny"])
    rho_single = s0.density(n_out=n_single)
    s0.close()
    vsign = -1 if valley == "K-" else 1
    if scheme != "strang4":
        n_o = oracle.solve_grid(field, RAGGED, N, scheme, valley=vsign)[0]
        assert np.max(np.abs(n_single - n_o)) <= (FP64_N_ABS if precision == "fp64" else FP32_N_ABS)

    s = gpu.Solver.for_grid(RAGGED, precision, scheme, valley).set_field(field, N)
    with pytest.raises(gpu.PDError):
        s.save_checkpoint(tmp_path / "early.npz")  # nothing to save before the first step
    s.propagate(k)
    s.snapshot()  # reads the state, leaves it as it was
    path = tmp_path / "ck.npz"
    assert s.save_checkpoint(path) == k
    state, done = s.save_state()
    s.close()
    assert done == k and state.nbytes == RAGGED["nx"] * RAGGED["ny"] * (3 if "strang" in scheme else 4) * (
        8 if precision == "fp64" else 4)

    r = gpu.Solver.from_checkpoint(path)
    assert r.info()["steps_done"] == k and r.valley == valley and r.precision == precision
    r.propagate(-1)
    n = np.empty_like(n_single)
    rho = r.density(n_out=n)
    r.close()
    assert np.array_equal(n, n_single) and rho == rho_single

    q = gpu.Solver.for_grid(RAGGED, precision, scheme, valley)
    buf = torch.zeros(state.nbytes // 4 + 64, dtype=torch.float32, device="cuda")
    q.bind_state(buf)
    q.load_checkpoint(path)
    for bad_k in (0, N):
        with pytest.raises(gpu.PDError):
            q.load_state(state, bad_k)
    with pytest.raises(gpu.PDError):
        q.load_state(state[:-4], k)
    q.propagate((N - k) // 2)
    q.propagate(-1)
    n2 = np.empty_like(n_single)
    rho2 = q.density(n_out=n2)
    q.close()
    assert np.array_equal(n2, n_single) and rho2 == rho_single

    other = gpu.Solver.for_grid(RAGGED, "fp64" if precision != "fp64" else "fp32", scheme, valley)
    with pytest.raises(gpu.PDError):
        other.load_checkpoint(path)
    other.close()


@pytest.mark.parametrize("precision,arrangement", [("fp32", "once"), ("fp32fast", "fast")])
def test_fp32_error_matches_the_rounding_model(gpu, precision, arrangement):
    """Each FP32 form's error against the oracle is the one the CPU model of its arithmetic
    (tests/fp32_model.py: FP32 state and coefficients, the form's arrangement of the
    roundings) predicts: on a 48^2 grid under the 8-cycle sin^2 pulse, at 4000 and 16000
    Strang steps, the GPU's rms error within 0.6-1.6 times the model's and its largest
    error within 0.4-2.5 times (both sides' roundings differ in detail, not in kind)."""
    from tests import fp32_model

    field, grid = wl.config1()["field"], {"nx": 48, "ny": 48, "px": (-2.0, 2.0), "py": (-2.0, 2.0)}
    for N in (4000, 16000):
        n_o = oracle.solve_grid(field, grid, N)[0]
        gpu_mx, gpu_rms = fp32_model.error_stats(run(gpu, grid, field, N, precision)[0], n_o)
        mod_mx, mod_rms = fp32_model.error_stats(fp32_model.solve_grid(field, grid, N, arrangement=arrangement), n_o)
        print("N=%d: GPU %s max %.3e rms %.3e; model max %.3e rms %.3e" % (
            N, precision, gpu_mx, gpu_rms, mod_mx, mod_rms))
        assert 0.6 <= gpu_rms / mod_rms <= 1.6 and 0.4 <= gpu_mx / mod_mx <= 2.5, (N, gpu_rms, mod_rms, gpu_mx, mod_mx)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_midpoint_step_forms(gpu, precision):
    """Both forms of the midpoint step match the oracle: the tangent form (step angles
    small enough; the state grows by 1 / cos(dt E) per step and is renormalised every
    1024 steps, in FP64 too) and the cosine form (larger angles).  A chunked
    tangent-form solve, cut next to the renormalisation steps, reproduces the single
    launch, and so does a snapshot taken between the chunks."""
    g = {"nx": 37, "ny": 29, "px": (-3.0, 2.5), "py": (-2.0, 2.2)}
    f = wl.sin2(0.4, 0.7, 4)
    tol = FP64_N_ABS if precision == "fp64" else FP32_N_ABS
    for N, form in ((2600, 0), (300, 1)):
        n, rho, info = run(gpu, g, f, N, precision, "midpoint")
        assert info["rotation_form"] == form, (N, info["rotation_form"])
        n_o = oracle.solve_grid(f, g, N, "midpoint")[0]
        assert np.max(np.abs(n - n_o)) <= tol, N
        if precision == "fp64":
            assert abs(rho / oracle.density(g, n_o) - 1) <= FP64_RHO_REL
    chunked = run(gpu, g, f, 2600, precision, "midpoint", chunks=[1023, 2, 1023, 552])
    single = run(gpu, g, f, 2600, precision, "midpoint")
    assert np.array_equal(chunked[0], single[0]) and chunked[1] == single[1]
    s = gpu.Solver.for_grid(g, precision, "midpoint")
    s.set_field(f, 2600)
    s.propagate(1500)
    n_mid = np.empty(g["nx"] * g["ny"])
    s.snapshot(n_out=n_mid)
    s.close()
    n_o = oracle.snapshot_grid(f, g, 2600, 1500, "midpoint")[0]
    assert np.max(np.abs(n_mid - n_o)) <= (5e-12 if precision == "fp64" else tol)


def test_degenerate_inputs(gpu):
    # one point, one step
    g1 = {"nx": 1, "ny": 1, "px": (0.3, 0.4), "py": (0.2, 0.3)}
    f = wl.sin2(0.1, 0.5, 8)
    n, rho, info = run(gpu, g1, f, 400)
    n_o = oracle.solve_grid(f, g1, 400)[0]
    assert abs(n[0] - n_o[0]) <= FP64_N_ABS
    # a grid made of the masked point only
    g0 = {"nx": 1, "ny": 1, "px": (0.0, 1.0), "py": (0.0, 1.0)}
    n, rho, info = run(gpu, g0, f, 400)
    assert n[0] == 0.0 and rho == 0.0 and info["n_masked"] == 1
    # a single step on config 1's grid (constant field over a short time)
    c = wl.config1()
    short = wl.constant(0.2, 0.5)
    for scheme in ("strang", "midpoint"):
        n, rho, info = run(gpu, c["grid"], short, 1, "fp64", scheme)
        n_o = oracle.solve_grid(short, c["grid"], 1, scheme)[0]
        assert np.max(np.abs(n - n_o)) <= FP64_N_ABS
    # E_out = 0 inside the grid (constant field, A_out = -40): masked, n = 0
    gm = {"nx": 81, "ny": 3, "px": (0.0, 81.0), "py": (-1.0, 2.0)}
    for scheme in ("strang", "midpoint"):
        n, rho, info = run(gpu, gm, wl.constant(0.2, 200.0), 40000, "fp64", scheme)
        assert info["n_masked"] == 2
        assert n[81 + 0] == 0.0 and n[81 + 40] == 0.0
        idx = np.array([81 * 2 + 3, 81 * 0 + 30])
        n_o = oracle.solve_grid(wl.constant(0.2, 200.0), gm, 40000, scheme, idx=idx)[0]
        assert np.max(np.abs(n[idx] - n_o)) <= FP64_N_ABS


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_large_step_angles_use_versine_form(gpu, precision):
    """dt = 0.05 under the constant field (A reaches -40): the rotation by 2 dt A_k exceeds pi/2,
    so the solve takes the versine rotation form; still the oracle's values."""
    g = {"nx": 48, "ny": 40, "px": (-4.0, 4.0), "py": (-3.0, 3.0)}
    f = wl.constant(0.2, 200.0)
    N = 4000
    n, rho, info = run(gpu, g, f, N, precision)
    assert info["rotation_form"] == 1
    n_o = oracle.solve_grid(f, g, N)[0]
    assert np.max(np.abs(n - n_o)) <= (FP64_N_ABS if precision == "fp64" else FP32_N_ABS)
    chunked = run(gpu, g, f, N, precision, chunks=[1500, 2500])
    assert np.array_equal(n, chunked[0])


PAPER_PULSE = {"kind": "pulse", "E0": 1.0, "omega": 0.4876, "phi": 0.3, "omega_rise": 0.0609,
               "omega_fall": 0.0609, "duration": 70.9}


@pytest.mark.parametrize("scheme", ["strang", "midpoint"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paper_laser_pulse(gpu, scheme, precision):
    """The rise / flat / fall pulse of Sec. IV, Eq. (14) in reduced units (10 THz, 1e7 V/m,
    5.5 periods): A_out != 0, so the final spinor uses p + A(t_f)."""
    g = {"nx": 48, "ny": 40, "px": (-3.0, 3.0), "py": (-2.5, 2.5)}
    N = 4000
    n, rho, info = run(gpu, g, PAPER_PULSE, N, precision, scheme)
    assert abs(info["A_out"]) > 1e-3
    n_o = oracle.solve_grid(PAPER_PULSE, g, N, scheme)[0]
    tol = FP64_N_ABS if precision == "fp64" else FP32_N_ABS
    assert np.max(np.abs(n - n_o)) <= tol
    if precision == "fp64":
        assert abs(rho / oracle.density(g, n_o) - 1) <= FP64_RHO_REL


@pytest.mark.parametrize("scheme", ["strang", "midpoint"])
def test_caller_field_table(gpu, scheme):
    """A field given as its own midpoint table (any time dependence): a sum of sinusoids."""
    N = 3000
    t_i, t_f = 0.0, 60.0
    dt = (t_f - t_i) / N
    tm = t_i + (np.arange(N) + 0.5) * dt
    def A(t):
        return 0.3 * np.sin(0.7 * t) * np.exp(-((t - 30.0) / 15.0) ** 2) + 0.05 * np.sin(1.9 * t + 0.4)
    f = {"kind": "table", "A_mid": A(tm), "t_i": t_i, "t_f": t_f, "A_in": float(A(t_i)), "A_out": float(A(t_f))}
    n, rho, info = run(gpu, RAGGED, f, N, "fp64", scheme)
    n_o = oracle.solve_grid(f, RAGGED, N, scheme)[0]
    assert np.max(np.abs(n - n_o)) <= FP64_N_ABS
    assert n.max() > 1e-6


def test_repeat_is_bitwise(gpu):
    c = wl.config1()
    a = run(gpu, c["grid"], c["field"], c["n_steps"])
    b = run(gpu, c["grid"], c["field"], c["n_steps"])
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


def test_density_reduction(gpu):
    c = wl.config1()
    n, rho, info = run(gpu, RAGGED, RAGGED_FIELD, 777)
    dx = (RAGGED["px"][1] - RAGGED["px"][0]) / RAGGED["nx"]
    dy = (RAGGED["py"][1] - RAGGED["py"][0]) / RAGGED["ny"]
    exact = 4 * dx * dy / (4 * math.pi ** 2) * math.fsum(n)
    assert abs(rho / exact - 1) <= 1e-14


def test_torch_stream_and_device_output(gpu):
    import torch

    c = wl.config1()
    ref = run(gpu, c["grid"], c["field"], c["n_steps"])
    s = gpu.Solver.for_grid(c["grid"])
    s.set_field(c["field"], c["n_steps"])
    st = torch.cuda.Stream()
    out = torch.empty(64 * 64, dtype=torch.float64, device="cuda")
    s.propagate(-1, stream=st)
    rho = s.density(n_out=out, stream=st)
    st.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref[0]) and rho == ref[1]
    s.close()


def test_error_paths_on_device(gpu):
    c = wl.config1()
    s = gpu.Solver.for_grid(c["grid"])
    s.set_field(c["field"], 100)
    with pytest.raises(gpu.PDError) as e:
        s.density()
    assert e.value.status == 2
    s.propagate(50)
    with pytest.raises(gpu.PDError):
        s.density()
    s.propagate(-1)
    with pytest.raises(gpu.PDError) as e:
        s.propagate(-1)
    assert e.value.status == 2
    s.density()
    import torch

    small = torch.empty(16, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu.PDError) as e:
        s.bind_state(small)
    assert e.value.status == 1
    s.close()


# ---------------------------------------------------------------------------
# Full-size workloads, in the launch configuration the benchmark uses


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def test_config2a_full_size(gpu):
    """1024^2 on [-4,4]^2, seeded E0, omega = 0.25, 20 cycles, 40000 steps, FP64: sampled points
    against the oracle, exact p_y = 0 row, mirror symmetry, and rho against the oracle's full grid."""
    c = wl.config2a()
    n, rho, info = run(gpu, c["grid"], c["field"], c["n_steps"])
    N = c["grid"]["nx"]
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(N * N, size=200, replace=False))
    n_o = oracle.solve_grid(c["field"], c["grid"], c["n_steps"], idx=idx)[0]
    assert np.max(np.abs(n[idx] - n_o)) <= FP64_N_ABS
    m = n.reshape(N, N)
    assert np.all(m[N // 2] == 0.0)
    assert np.max(np.abs(m[1:] - m[1:][::-1])) <= 1e-13
    gold = _golden("oracle_config2a.json")
    if gold is not None:
        assert abs(rho / gold["rho"] - 1) <= FP64_RHO_REL
        ks = np.array([int(k) for k in gold["samples"]])
        vs = np.array(list(gold["samples"].values()))
        assert np.max(np.abs(n[ks] - vs)) <= FP64_N_ABS


def test_config2b_constant_field_landau_zener(gpu):
    """Constant field E0 = 0.2 on [0, 200], 1024^2, 40000 steps: for 2 <= p_x < 4 the density
    is the Landau-Zener value exp(-pi p_y^2 / E0) within 2e-3; sampled points match the oracle."""
    c = wl.config2b()
    n, rho, info = run(gpu, c["grid"], c["field"], c["n_steps"])
    N = c["grid"]["nx"]
    m = n.reshape(N, N)
    p = -4.0 + np.arange(N) * (8.0 / N)
    cols = (p >= 2.0) & (p < 4.0)
    lz = np.exp(-math.pi * p ** 2 / 0.2)
    dev = np.abs(m[:, cols] - lz[:, None]).max()
    assert dev <= 2e-3
    rng = np.random.default_rng(12)
    idx = np.sort(rng.choice(N * N, size=120, replace=False))
    n_o = oracle.solve_grid(c["field"], c["grid"], c["n_steps"], idx=idx)[0]
    assert np.max(np.abs(n[idx] - n_o)) <= FP64_N_ABS
    gold = _golden("oracle_config2b.json")
    if gold is not None:
        assert abs(rho / gold["rho"] - 1) <= FP64_RHO_REL


@pytest.fixture(scope="module")
def cfg3_subsample_oracle():
    c = wl.config3()
    idx = wl.subsample_indices(2048, 64)
    n_o = oracle.solve_grid(c["field"], c["grid"], c["n_steps"], idx=idx)[0]
    return idx, n_o


def test_config3_precision_form(gpu, cfg3_subsample_oracle):
    """2048^2 on [-2,2]^2, 80000 steps, FP32 form: the 64 x 64 subsample (stride 32) within
    1e-5 of the FP64 oracle per point; the FP64 form within 1e-12; total densities agree."""
    idx, n_o = cfg3_subsample_oracle
    c = wl.config3()
    n32, rho32, _ = run(gpu, c["grid"], c["field"], c["n_steps"], "fp32")
    err32 = np.max(np.abs(n32[idx] - n_o))
    print("config3 fp32 max |dn| on subsample = %.3e" % err32)
    assert err32 <= FP32_N_ABS
    n64, rho64, _ = run(gpu, c["grid"], c["field"], c["n_steps"], "fp64")
    assert np.max(np.abs(n64[idx] - n_o)) <= FP64_N_ABS
    print("config3 rho fp32 %.15e fp64 %.15e rel %.3e" % (rho32, rho64, rho32 / rho64 - 1))
    assert abs(rho32 / rho64 - 1) <= 1e-5
    m = n32.reshape(2048, 2048)
    assert np.all(m[1024] == 0.0)
    # every point of the grid: the FP64 form stands in for the oracle there (it is within
    # 1e-12 of it on the subsample above); the FP32 form is within 1e-5 everywhere
    full32 = np.max(np.abs(n32 - n64))
    print("config3 fp32 max |dn| over the full grid (against fp64) = %.3e" % full32)
    assert full32 <= FP32_N_ABS
    # the fast FP32 form (alternating shears, same-plane rotations merged), the benchmark's
    # main line: within 1e-5 on the subsample and at every point of the grid
    nf, rhof, _ = run(gpu, c["grid"], c["field"], c["n_steps"], "fp32fast")
    errf, fullf = np.max(np.abs(nf[idx] - n_o)), np.max(np.abs(nf - n64))
    print("config3 fp32fast max |dn| on subsample = %.3e, over the full grid (against fp64) = %.3e" % (errf, fullf))
    assert errf <= FP32_N_ABS and fullf <= FP32_N_ABS
