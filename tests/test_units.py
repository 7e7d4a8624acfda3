"""SI <-> reduced units for the paper's run (Sec. IV: 1e7 V/m, 10 THz, envelope
frequencies 7.85e12 1/s, 5.5 periods; v_F = 1.093e6 m/s from Sec. I).

Pins: the scales are checked against each other by independent routes
(dimensional identities), against a dimensionless quantity computed once in
SI and once in reduced units (the Keldysh parameter), and the reduced pulse is
the one the GPU tests run."""
import math

import pytest

from paper_1607_03062_amd import units

E = 1.602176634e-19
HBAR = 1.054571817e-34  # CODATA rounded value, independent of the module's h / 2 pi


def test_scales_are_consistent():
    u = units.ReducedUnits(1.0e7)
    # tau from the length scale sqrt(hbar v_F / (e E)) divided by v_F
    ell = math.sqrt(HBAR * 1.093e6 / (E * 1.0e7))
    assert abs(u.length_m / ell - 1) <= 1e-9
    assert abs(u.time_s / (ell / 1.093e6) - 1) <= 1e-9
    # e E_ref tau = p_u (a unit field changes the momentum by one unit per unit time)
    assert abs(E * 1.0e7 * u.time_s / u.momentum_kg_m_per_s - 1) <= 1e-12
    # energy unit = v_F p_u = hbar / tau
    assert abs(u.energy_J / (1.093e6 * u.momentum_kg_m_per_s) - 1) <= 1e-12
    assert abs(u.energy_J / (HBAR / u.time_s) - 1) <= 1e-9
    # magnitudes: tau ~ 7.76 fs, energy ~ 0.0848 eV, length ~ 8.48 nm, density ~ 1.39e12 / cm^2
    assert abs(u.time_s - 7.760e-15) <= 0.001e-15
    assert abs(u.energy_eV - 0.0848) <= 0.0001
    assert abs(u.length_m - 8.48e-9) <= 0.01e-9
    assert abs(u.density_per_cm2 / 1.39e12 - 1) <= 0.005


def test_paper_pulse_in_reduced_units():
    u = units.ReducedUnits(1.0e7)
    f = u.paper_pulse(1.0e7, 10.0e12, 7.85e12, 7.85e12, 5.5, phi=0.3)
    assert f["E0"] == 1.0
    assert abs(f["omega"] - 0.4876) <= 0.0001
    assert abs(f["omega_rise"] - 0.0609) <= 0.0001 and f["omega_fall"] == f["omega_rise"]
    assert abs(f["duration"] - 70.9) <= 0.05
    # rise window pi / (2 Omega) = 200 fs, well inside the 550 fs pulse
    assert abs(math.pi / (2 * f["omega_rise"]) * u.time_s - math.pi / (2 * 7.85e12)) <= 1e-18
    # the pulse the GPU tests run (test_gpu_parity.PAPER_PULSE) is this one to its quoted digits
    from .test_gpu_parity import PAPER_PULSE

    for k in ("E0", "omega", "omega_rise", "duration"):
        assert abs(PAPER_PULSE[k] - f[k]) <= 0.0005 * max(1.0, abs(f[k])), k


def test_keldysh_parameter_is_unit_free():
    """gamma = |p_y| omega / (e E0) in SI equals the reduced-unit value."""
    u = units.ReducedUnits(1.0e7)
    p_y = 0.8  # reduced
    p_si = p_y * u.momentum_kg_m_per_s
    w_si = 2 * math.pi * 10.0e12
    g_si = p_si * w_si / (E * 1.0e7)
    g_red = units.keldysh(p_y, u.rate(w_si), u.field(1.0e7))
    assert abs(g_si / g_red - 1) <= 1e-12
    assert g_red < 1  # the paper's regime (Sec. IV) at this p_y


def test_dirac_cone_validity_momentum():
    """The paper's Dirac-cone regime, |p| up to ~100 eV, is ~1179 momentum units at 1e7 V/m."""
    u = units.ReducedUnits(1.0e7)
    assert abs(u.momentum_from_energy_eV(100.0) - 1179) <= 2
    assert abs(u.momentum_to_energy_eV(u.momentum_from_energy_eV(3.0)) - 3.0) <= 1e-12


def test_bad_reference():
    with pytest.raises(ValueError):
        units.ReducedUnits(0.0)
