"""Property tests of the library's host-side logic against the oracle (independent
code) over random inputs: the field samples of every kind, scheme and polarisation,
the end values, dt, E_max, and the count of masked points."""
import math

import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
import paper_1607_03062_amd as pd
from paper_1607_03062_amd import _lib

SCHEMES = st.sampled_from(["strang", "midpoint", "strang4", "midpoint4"])
ELL = st.one_of(st.just(0.0), st.floats(-1.0, 1.0))


def sin2_fields():
    return st.builds(lambda E0, w, c, e: {"kind": "sin2", "E0": E0, "omega": w, "cycles": c, "ellipticity": e},
                     st.floats(0.01, 1.0), st.floats(0.1, 2.0), st.integers(2, 40), ELL)


def pulse_fields():
    def make(E0, w, phi, wr, wf, extra, e):
        d = math.pi / (2 * wr) + math.pi / (2 * wf) + extra
        return {"kind": "pulse", "E0": E0, "omega": w, "phi": phi, "omega_rise": wr, "omega_fall": wf,
                "duration": d, "ellipticity": e}
    return st.builds(make, st.floats(0.1, 2.0), st.floats(0.2, 2.0), st.floats(-3.2, 3.2), st.floats(0.02, 0.5),
                     st.floats(0.02, 0.5), st.floats(0.0, 50.0), ELL)


def constant_fields():
    return st.builds(lambda E0, t, e: {"kind": "constant", "E0": E0, "t_end": t, "ellipticity": e},
                     st.floats(-1.0, 1.0), st.floats(0.5, 300.0), ELL)


@settings(max_examples=60, deadline=None)
@given(field=st.one_of(sin2_fields(), pulse_fields(), constant_fields()), n=st.integers(1, 600), scheme=SCHEMES)
def test_field_samples_match_oracle(field, n, scheme):
    Ax, Ay, ends = _lib.sample_field_xy(field, n, scheme)
    Ao, ax_in, ax_out, dt = oracle.field_table(field, n, scheme)
    Ayo, ay_in, ay_out = oracle.field_table_y(field, n, scheme)
    scale = max(1.0, float(np.abs(Ao).max()), float(np.abs(Ayo).max()))
    tol = 1e-13 * scale
    assert np.max(np.abs(Ax - Ao)) <= tol
    assert np.max(np.abs(Ay - Ayo)) <= tol
    t_i, t_f, a_in, a_out, b_in, b_out = ends
    assert abs(a_in - ax_in) <= tol and abs(a_out - ax_out) <= tol
    assert abs(b_in - ay_in) <= tol and abs(b_out - ay_out) <= tol
    assert abs((t_f - t_i) / n - dt) <= 1e-15 * max(1.0, dt)
    if not field.get("ellipticity"):
        assert np.all(Ay == 0.0)


@settings(max_examples=40, deadline=None)
@given(field=sin2_fields(), nx=st.integers(1, 40), ny=st.integers(1, 40), w=st.floats(0.5, 5.0),
       scheme=SCHEMES, n=st.integers(100, 2000))
def test_check_field_extent_matches_definition(field, nx, ny, w, scheme, n):
    """E_max is the largest |p + A| over the grid nodes and every sample (and the end values)."""
    s = pd.Solver(nx, ny, (-w, w), (-0.7 * w, 1.3 * w), "fp64", scheme)
    try:
        info = s.check_field(field, n)
    except pd.PDError as e:
        assert e.status == _lib.PD_ERR_INVALID and "pi" in e.message  # only the step condition may refuse
        return
    finally:
        s.close()
    Ax, Ay, ends = _lib.sample_field_xy(field, n, scheme)
    Ax = np.concatenate([Ax, ends[2:4]])
    Ay = np.concatenate([Ay, ends[4:6]])
    px = -w + np.arange(nx) * (2 * w / nx)
    py = -0.7 * w + np.arange(ny) * (2 * w / ny)
    X = max(abs(px[0] + Ax.min()), abs(px[0] + Ax.max()), abs(px[-1] + Ax.min()), abs(px[-1] + Ax.max()))
    Y = max(abs(py[0] + Ay.min()), abs(py[0] + Ay.max()), abs(py[-1] + Ay.min()), abs(py[-1] + Ay.max()))
    assert abs(info["E_max"] - math.hypot(X, Y)) <= 1e-12 * max(1.0, info["E_max"])
    assert info["dt"] * info["E_max"] <= math.pi


@settings(max_examples=40, deadline=None)
@given(nx=st.integers(1, 24), ny=st.integers(1, 24), k_in=st.integers(0, 23), k_out=st.integers(0, 23),
       j_in=st.integers(0, 23), j_out=st.integers(0, 23), ell=st.booleans())
def test_masked_count_matches_oracle(nx, ny, k_in, k_out, j_in, j_out, ell):
    """Put p + A(t_i) or p + A(t_f) exactly on a node (or not): the library's count of masked points
    equals the oracle's (which masks where |P_in| or |P_out| vanishes)."""
    g = {"nx": nx, "ny": ny, "px": (-1.0, 1.0), "py": (-1.0, 1.0)}
    node = lambda lo, n, j: oracle.grid_p(lo, 1.0, n, j % n)
    a_in, a_out = -node(-1.0, nx, k_in), -node(-1.0, nx, k_out)
    f = {"kind": "table", "A_mid": np.zeros(1), "t_i": 0.0, "t_f": 1.0, "A_in": a_in, "A_out": a_out}
    if ell:
        f.update({"Ay_mid": np.zeros(1), "Ay_in": -node(-1.0, ny, j_in), "Ay_out": -node(-1.0, ny, j_out)})
    s = pd.Solver.for_grid(g)
    m_lib = s.check_field(f, 1)["n_masked"]
    s.close()
    m_or = oracle.solve_grid(f, g, 1, "strang")[2]
    assert m_lib == m_or


def test_pulse_without_flat_part_is_accepted():
    """duration = pi/(2 W_r) + pi/(2 W_f) exactly (no flat part) is a valid pulse even when the
    rounding of duration - pi/(2 W_f) lands below pi/(2 W_r); the samples still match the oracle."""
    wr, wf = 0.2, 0.0609  # D - pi/(2 wf) rounds 1.8e-15 below pi/(2 wr)
    f = {"kind": "pulse", "E0": 1.0, "omega": 0.7, "phi": 0.1, "omega_rise": wr, "omega_fall": wf,
         "duration": math.pi / (2 * wr) + math.pi / (2 * wf)}
    Ax, Ay, ends = _lib.sample_field_xy(f, 200, "strang")
    Ao = oracle.field_table(f, 200)[0]
    assert np.max(np.abs(Ax - Ao)) <= 1e-13


def test_long_field_sampling_matches_oracle():
    """Long solves sample A on several host threads (contiguous ranges of steps): every sample,
    end value and dt still equals the oracle's, for each analytic kind, both polarisations and
    both stage counts."""
    fields = [{"kind": "sin2", "E0": 0.3, "omega": 0.5, "cycles": 30, "ellipticity": 0.6},
              {"kind": "pulse", "E0": 1.0, "omega": 0.4876, "phi": 0.3, "omega_rise": 0.0609, "omega_fall": 0.0609,
               "duration": 70.9},
              {"kind": "constant", "E0": 0.2, "t_end": 200.0, "ellipticity": -0.4}]
    for field in fields:
        for n, scheme in ((50000, "strang"), (20000, "strang4")):
            Ax, Ay, ends = _lib.sample_field_xy(field, n, scheme)
            Ao, ax_in, ax_out, dt = oracle.field_table(field, n, scheme)
            Ayo, ay_in, ay_out = oracle.field_table_y(field, n, scheme)
            scale = max(1.0, float(np.abs(Ao).max()), float(np.abs(Ayo).max()))
            assert Ax.shape == Ao.shape and Ay.shape == Ayo.shape
            assert np.max(np.abs(Ax - Ao)) <= 1e-13 * scale, (field["kind"], scheme)
            assert np.max(np.abs(Ay - Ayo)) <= 1e-13 * scale, (field["kind"], scheme)
            assert abs(ends[2] - ax_in) <= 1e-13 * scale and abs(ends[3] - ax_out) <= 1e-13 * scale
            assert abs((ends[1] - ends[0]) / n - dt) <= 1e-15 * max(1.0, dt)
