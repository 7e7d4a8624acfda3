"""Seeded synthetic workloads: grids, field parameters and step counts.

This module holds only input descriptions and the seeded draws that make
them; it computes nothing of the method itself (no vector potential, no
spinor, no density).  Both the GPU path and the CPU oracle take their inputs
from here.

Units are hbar = v_F = e = 1.  A field is a plain dict:

  {"kind": "sin2", "E0", "omega", "cycles"}   E(t) = E0 sin^2(pi t/T) sin(omega t),
                                              T = cycles * 2 pi / omega, t in [0, T]
  {"kind": "constant", "E0", "t_end"}         E(t) = E0 on [0, t_end]
  {"kind": "pulse", "E0", "omega", "phi", "omega_rise", "omega_fall", "duration"}
                                              the rise / flat / fall laser pulse of
                                              Sec. IV, Eq. (14), t in [0, duration]
  {"kind": "table", "A_mid", "t_i", "t_f", "A_in", "A_out"}

Elliptic polarisation adds a y component: "ellipticity" e (sin2: E_y =
e E0 sin^2(pi t/T) cos(omega t); pulse: E_y = e E0 env(t) sin(omega t + phi);
constant: E_y = e E0), or for a table "Ay_mid", "Ay_in", "Ay_out".

A grid is {"nx", "ny", "px": (min, max), "py": (min, max)} on the node
convention p_j = p_min + j (p_max - p_min) / n, j < n.
"""
from __future__ import annotations

import math

import numpy as np


def grid(n: int, half_width: float) -> dict:
    return {"nx": int(n), "ny": int(n), "px": (-float(half_width), float(half_width)),
            "py": (-float(half_width), float(half_width))}


def sin2(E0: float, omega: float, cycles: int, ellipticity: float = 0.0) -> dict:
    f = {"kind": "sin2", "E0": float(E0), "omega": float(omega), "cycles": int(cycles)}
    if ellipticity:
        f["ellipticity"] = float(ellipticity)
    return f


def constant(E0: float, t_end: float, ellipticity: float = 0.0) -> dict:
    f = {"kind": "constant", "E0": float(E0), "t_end": float(t_end)}
    if ellipticity:
        f["ellipticity"] = float(ellipticity)
    return f


def sin2_duration(field: dict) -> float:
    return field["cycles"] * 2.0 * math.pi / field["omega"]


# Config 1: plain FP64, 64x64 on [-2,2]^2, E0 = 0.1, omega = 0.5, 8 cycles, 4000 Strang steps.
def config1() -> dict:
    return {"name": "cfg1_64sq_n4000_fp64", "grid": grid(64, 2.0), "field": sin2(0.1, 0.5, 8),
            "n_steps": 4000, "precision": "fp64", "scheme": "strang"}


# Config 2a: FP64 on 1024x1024, [-4,4]^2, E0 ~ U[0.05, 0.5] seeded, omega = 0.25, 20 cycles, 40000 steps.
def config2a_E0() -> float:
    return float(np.random.default_rng(2).uniform(0.05, 0.5))


def config2a(n: int = 1024) -> dict:
    return {"name": "cfg2a_%dsq_n40000_fp64" % n, "grid": grid(n, 4.0), "field": sin2(config2a_E0(), 0.25, 20),
            "n_steps": 40000, "precision": "fp64", "scheme": "strang"}


# Config 2b: constant field E0 = 0.2 on [0, 200], 40000 steps (dt = 0.005), 1024x1024 on [-4,4]^2.
def config2b(n: int = 1024) -> dict:
    return {"name": "cfg2b_%dsq_n40000_const" % n, "grid": grid(n, 4.0), "field": constant(0.2, 200.0),
            "n_steps": 40000, "precision": "fp64", "scheme": "strang"}


# Config 3: precision form, 2048x2048 on [-2,2]^2, E0 = 0.1, omega = 0.5, 30 cycles, 80000 steps.
def config3(n: int = 2048, precision: str = "fp32") -> dict:
    return {"name": "cfg3_%dsq_n80000_%s" % (n, precision), "grid": grid(n, 2.0), "field": sin2(0.1, 0.5, 30),
            "n_steps": 80000, "precision": precision, "scheme": "strang"}


def subsample_indices(n_full: int, n_sub: int) -> np.ndarray:
    """Linear indices j*n_full + i of the n_sub x n_sub subsample with stride n_full // n_sub."""
    stride = n_full // n_sub
    ii = np.arange(n_sub, dtype=np.int64) * stride
    return (ii[:, None] * n_full + ii[None, :]).ravel()


def steps_for(field: dict, half_width: float, n_requested: int, max_phase: float = 0.5) -> int:
    """Raise a requested step count so that dt * E_bound <= max_phase, where
    E_bound = sqrt(2) L + 3 E0 / omega bounds |p + A(t)| on [-L, L]^2 for a
    sin^2-envelope pulse with at least two cycles (|A| <= E0 (1/w + 1/(2(w+W))
    + 1/(2|w-W|)) <= 7/3 E0/w when W <= w/2).  A loose sizing rule for the
    synthetic draws; the library itself checks the exact bound."""
    T = sin2_duration(field)
    e_bound = math.sqrt(2.0) * half_width + 3.0 * field["E0"] / field["omega"]
    return max(int(n_requested), int(math.ceil(T * e_bound / max_phase)))


# Config 4: 64 solves, E0 ~ U[0.05,0.5], omega ~ U[0.1,1.0], cycles ~ U{4..40}, steps ~ U{5000..80000}
# (raised per steps_for), square grids from {256,512,1024,2048} on [-4,4]^2.
def _draw_solve(rng, sizes, step_range, max_steps):
    E0 = float(rng.uniform(0.05, 0.5))
    omega = float(rng.uniform(0.1, 1.0))
    cycles = int(rng.integers(4, 41))
    n_req = int(rng.integers(step_range[0], step_range[1] + 1))
    n = int(rng.choice(np.asarray(sizes)))
    f = sin2(E0, omega, cycles)
    # raised to keep dt * E_bound <= 0.5, capped at max_steps (dt * E_bound stays below pi:
    # T <= 2513 and E_bound <= 21 give dt * E_bound <= 0.66 at 80000 steps)
    steps = max(n_req, min(steps_for(f, 4.0, n_req), max_steps))
    return n, f, steps


# Config 4: 64 solves, E0 ~ U[0.05,0.5], omega ~ U[0.1,1.0], cycles ~ U{4..40}, steps ~ U{5000..80000}
# (raised per steps_for, at most 80000), square grids from {256,512,1024,2048} on [-4,4]^2.
# step_range and sizes shrink the same recipe for tests.
def config4(count: int = 64, seed: int = 4, sizes=(256, 512, 1024, 2048), precision: str = "fp32",
            step_range=(5000, 80000), max_steps: int = 80000) -> list:
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        n, f, steps = _draw_solve(rng, sizes, step_range, max_steps)
        out.append({"name": "cfg4_%02d" % q, "grid": grid(n, 4.0), "field": f, "n_steps": steps,
                    "precision": precision, "scheme": "strang"})
    return out


# Config 5: a Poisson stream of solve requests with config-4 parameter and size distributions,
# accuracy class 50/50 FP32 / FP64.
def config5(count: int = 10000, seed: int = 5, rate_per_s: float = 1.0, sizes=(256, 512, 1024, 2048),
            step_range=(5000, 80000), max_steps: int = 80000) -> list:
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for q in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        n, f, steps = _draw_solve(rng, sizes, step_range, max_steps)
        prec = "fp32" if rng.random() < 0.5 else "fp64"
        out.append({"name": "req_%05d" % q, "arrival_s": t, "grid": grid(n, 4.0), "field": f, "n_steps": steps,
                    "precision": prec, "scheme": "strang"})
    return out
