"""The pins are sensitive: a plausible mistake planted in a copy of the oracle
source (a flipped sign, a dropped or swapped term, an off-by-one, a wrong
factor) makes at least one pin fail.  The copy is built and run on the CPU
only; the oracle itself is untouched."""
import numpy as np
import pytest

import oracle
from paper_1607_03062_amd import workloads as wl

from . import test_oracle_pins as pins
from . import test_oracle_pins_ext as ext

MUTANTS = {
    "apply_x_sign": ("psi[0] = a1 + (h * a1 + s * b2);", "psi[0] = a1 + (h * a1 - s * b2);"),
    "apply_y_sign": ("psi[2] = a2 + (h * a2 + s * a1);", "psi[2] = a2 + (h * a2 - s * a1);"),
    "midpoint_axis_swap": ("double al = g * sig * Px, be = g * sig * Py;",
                           "double al = g * sig * Py, be = g * sig * Px;"),
    "midpoint_term_sign": ("psi[1] = b1 + ((h * b1 - be * b2) - al * a2);",
                           "psi[1] = b1 + ((h * b1 - be * b2) + al * a2);"),
    "strang_full_first_half": ("apply_y(psi, g * 0.5 * dt * Py);\n    apply_x",
                               "apply_y(psi, g * dt * Py);\n    apply_x"),
    "step_time_not_midpoint": ("double t = t_i + ((double)k + sg[j]) * dt;", "double t = t_i + ((double)k) * dt;"),
    "sin2_A_sign": ("return -E0 * I;", "return E0 * I;"),
    "sin2_A_term_sign": ("- one_minus_cos((w + W) * t) / (4.0 * (w + W))",
                         "+ one_minus_cos((w + W) * t) / (4.0 * (w + W))"),
    "constant_A_sign": ("return -f->E0 * t;", "return f->E0 * t;"),
    "projection_conj": ("(u[2] * psi[3] - u[3] * psi[2]);", "(u[2] * psi[3] + u[3] * psi[2]);"),
    "v_spinor_sign": ("v[0] = -Px / d; v[1] = Py / d;", "v[0] = -Px / d; v[1] = -Py / d;"),
    "u_spinor_sign": ("u[0] = E / d; u[1] = 0.0; u[2] = Px / d; u[3] = Py / d;",
                      "u[0] = E / d; u[1] = 0.0; u[2] = Px / d; u[3] = -Py / d;"),
    "kahan_compensation_sign": ("c = (t - s) - y;", "c = (t - s) + y;"),
    "kahan_drops_compensation": ("double y = n[k] - c;", "double y = n[k];"),
    "density_factor": ("return 4.0 * dx * dy / (4.0 * M_PI * M_PI) * s;",
                       "return 2.0 * dx * dy / (4.0 * M_PI * M_PI) * s;"),
    "grid_spacing": ("double d = (p_max - p_min) / (double)n;", "double d = (p_max - p_min) / (double)(n - 1);"),
    "final_momentum_uses_A_in": ("double Px_out = px + ax, Py_out = py + ay;",
                                 "double Px_out = px + t->e.Ax_in, Py_out = py + ay;"),
    "one_step_short": ("for (long long k = 0; k < k_stop; ++k) full_step(",
                       "for (long long k = 0; k < k_stop - 1; ++k) full_step("),
    # fourth-order composition
    "suzuki_middle_coefficient": ("c[2] = 1.0 - 4.0 * p;", "c[2] = 1.0 - 3.0 * p;"),
    "suzuki_p_value": ("double p = 1.0 / (4.0 - cbrt(4.0));", "double p = 1.0 / (4.0 - cbrt(2.0));"),
    "stage_time_at_start": ("sigma[j] = start + 0.5 * c[j];", "sigma[j] = start;"),
    "stage_coefficient_not_applied": ("step(f->scheme, g, psi, c[j] * dt,", "step(f->scheme, g, psi, dt / S,"),
    # elliptic polarisation
    "Ay_sign_in_step": ("double Px = px + Ax, Py = py + Ay;", "double Px = px + Ax, Py = py - Ay;"),
    "projection_drops_Ay": ("double Px_out = px + ax, Py_out = py + ay;", "double Px_out = px + ax, Py_out = py;"),
    "initial_state_drops_Ay": ("Py_in = py + t->e.Ay_in;", "Py_in = py;"),
    "sin2_Ay_term_sign": ("- sin((w + W) * t) / (4.0 * (w + W))", "+ sin((w + W) * t) / (4.0 * (w + W))"),
    "pulse_Ay_quarter_period": ("return f->ellipticity * pulse_A_phase(f, f->phi - 0.5 * M_PI, t);",
                                "return f->ellipticity * pulse_A_phase(f, f->phi + 0.5 * M_PI, t);"),
    "constant_Ay_sign": ("return -f->ellipticity * f->E0 * t;", "return f->ellipticity * f->E0 * t;"),
    # snapshots
    "snapshot_time_half_step_late": ("double t = t_i + (double)k * e->dt;",
                                     "double t = t_i + ((double)k + 0.5) * e->dt;"),
    "snapshot_projects_on_final_state": ("boundary_A(f, k_stop, t->Ax, t->Ay, &t->e, &ax, &ay);",
                                         "boundary_A(f, f->n_steps, t->Ax, t->Ay, &t->e, &ax, &ay);"),
}


def _py_zero_row():
    g, f = wl.config1()["grid"], wl.config1()["field"]
    idx = 32 * 64 + np.arange(64)
    for s in ("strang", "midpoint"):
        n = oracle.solve_grid(f, g, 400, s, idx=idx)[0]
        assert np.all(n == 0.0)


QUICK_PINS = [
    lambda: pins.test_spinors_orthonormal_eigenvectors(1),
    lambda: pins.test_spinors_orthonormal_eigenvectors(-1),
    lambda: pins.test_step_equals_matrix_exponential("strang", 1),
    lambda: pins.test_step_equals_matrix_exponential("midpoint", 1),
    pins.test_sin2_vector_potential_is_minus_integral_of_E,
    pins.test_constant_and_pulse_vector_potentials,
    pins.test_density_scale,
    pins.test_density_compensated_sum,
    lambda: pins.test_brute_force_tiny_grid("strang"),
    lambda: pins.test_brute_force_tiny_grid("midpoint"),
    pins.test_masked_point_at_zero_momentum,
    _py_zero_row,
    pins.test_landau_zener_constant_field,
    ext.test_composition_order_conditions,
    lambda: ext.test_fourth_order_convergence("midpoint4"),
    lambda: ext.test_step_with_Ay_equals_matrix_exponential("strang"),
    lambda: ext.test_step_with_Ay_equals_matrix_exponential("midpoint"),
    lambda: ext.test_sin2_Ay_is_minus_integral_of_Ey(1.0),
    ext.test_pulse_and_constant_Ay,
    lambda: ext.test_rotation_covariance("midpoint"),
    lambda: ext.test_y_reflection_symmetry("strang"),
    ext.test_snapshot_at_start_is_zero,
    lambda: ext.test_snapshot_adiabatic_perturbation(1.0),
    lambda: ext.test_snapshot_continuum_dop853(((0.25, 0.125),)),
]


def _failures():
    bad = 0
    for pin in QUICK_PINS:
        try:
            pin()
        except Exception:
            bad += 1
    return bad


def test_unmodified_source_passes_quick_pins(tmp_path):
    lib = oracle.compile_source(oracle.source_text(), str(tmp_path / "liboracle_copy.so"))
    with oracle.use_library(lib):
        assert _failures() == 0


@pytest.mark.filterwarnings("ignore")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, "mutation site not unique: %s" % name
    lib = oracle.compile_source(src.replace(old, new), str(tmp_path / ("liboracle_%s.so" % name)))
    with oracle.use_library(lib):
        assert _failures() > 0, "no pin caught the planted mistake %s" % name
