"""SI quantities <-> the solver's reduced units.

The solver works in units where hbar = v_F = e = 1 (the Dirac equation of
Sec. II with H = sigma.(p + A)).  Fixing a reference field strength E_ref sets
every other scale:

    time      tau = sqrt(hbar / (e v_F E_ref))
    momentum  p_u = hbar / (v_F tau)            (so that e E_ref tau = p_u)
    energy    hbar / tau = v_F p_u
    length    v_F tau
    density   1 / (v_F tau)^2                   (per unit area)

A field of E_ref is then E0 = 1, an angular frequency w becomes w tau, and the
pair density rho the solver returns is a number per (v_F tau)^2.  The Fermi
velocity defaults to the value the paper quotes for graphene in its
introduction, 1.093e6 m/s; e and hbar are the exact SI values.
"""
from __future__ import annotations

import math

E_CHARGE = 1.602176634e-19  # C (exact)
HBAR = 6.62607015e-34 / (2.0 * math.pi)  # J s (h exact)
V_F_GRAPHENE = 1.093e6  # m/s


class ReducedUnits:
    """Scales of the reduced units for a reference field E_ref (V/m) and Fermi velocity v_F (m/s)."""

    def __init__(self, field_V_per_m: float, v_F: float = V_F_GRAPHENE):
        if not (field_V_per_m > 0.0 and v_F > 0.0):
            raise ValueError("the reference field and the Fermi velocity must be positive")
        self.field_V_per_m = float(field_V_per_m)
        self.v_F = float(v_F)
        self.time_s = math.sqrt(HBAR / (E_CHARGE * self.v_F * self.field_V_per_m))
        self.momentum_kg_m_per_s = HBAR / (self.v_F * self.time_s)
        self.energy_J = HBAR / self.time_s
        self.energy_eV = self.energy_J / E_CHARGE
        self.length_m = self.v_F * self.time_s
        self.density_per_cm2 = 1.0 / (self.length_m * 100.0) ** 2

    # SI -> reduced
    def field(self, E_V_per_m: float) -> float:
        return E_V_per_m / self.field_V_per_m

    def time(self, t_s: float) -> float:
        return t_s / self.time_s

    def rate(self, per_s: float) -> float:
        """An angular frequency (rad/s) or an envelope frequency (1/s)."""
        return per_s * self.time_s

    def momentum_from_energy_eV(self, energy_eV: float) -> float:
        """The momentum whose Dirac-cone energy v_F |p| is energy_eV."""
        return energy_eV / self.energy_eV

    # reduced -> SI
    def density_to_per_cm2(self, rho: float) -> float:
        return rho * self.density_per_cm2

    def momentum_to_energy_eV(self, p: float) -> float:
        return p * self.energy_eV

    def paper_pulse(self, E0_V_per_m: float, frequency_Hz: float, omega_rise_per_s: float,
                    omega_fall_per_s: float, periods: float, phi: float = 0.0, ellipticity: float = 0.0) -> dict:
        """The rise / flat / fall laser pulse of Sec. IV, Eq. (14), from SI parameters, as a field
        description in reduced units (t_i = 0, duration = periods carrier periods)."""
        w = self.rate(2.0 * math.pi * frequency_Hz)
        f = {"kind": "pulse", "E0": self.field(E0_V_per_m), "omega": w, "phi": float(phi),
             "omega_rise": self.rate(omega_rise_per_s), "omega_fall": self.rate(omega_fall_per_s),
             "duration": periods * 2.0 * math.pi / w}
        if ellipticity:
            f["ellipticity"] = float(ellipticity)
        return f


def keldysh(p_y: float, omega: float, E0: float) -> float:
    """Keldysh parameter |p_y| omega / (e E0) in reduced units (the paper's tunnelling regime has
    gamma << 1, Sec. IV)."""
    return abs(p_y) * omega / E0
