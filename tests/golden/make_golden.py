"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

These are regression values of the oracle's conventions (grid, midpoints,
masking, density factor); they are not an independent check of the physics,
which the pins in tests/test_oracle_pins.py provide.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1607_03062_amd import workloads as wl  # noqa: E402


def config1_values():
    c = wl.config1()
    out = {"config": c["name"], "n_steps": c["n_steps"]}
    for s in ("strang", "midpoint"):
        n, nd, masked = oracle.solve_grid(c["field"], c["grid"], c["n_steps"], s)
        k = int(np.argmax(n))
        out[s] = {"rho": oracle.density(c["grid"], n), "n_max": float(n[k]), "argmax": k, "n_masked": masked,
                  "max_norm_dev": float(np.abs(nd).max()),
                  "n_at": {str(i): float(n[i]) for i in (0, 100, 1000, 2047, 2080, 3000, 4095)}}
    return out


def full_grid_values(c, n_samples=512, seed=7):
    """rho over the full grid and n at seeded sample points (FP64 Strang oracle)."""
    n, nd, masked = oracle.solve_grid(c["field"], c["grid"], c["n_steps"], "strang")
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n.shape[0], size=n_samples, replace=False))
    return {"config": c["name"], "n_steps": c["n_steps"], "rho": oracle.density(c["grid"], n),
            "rho_kahan": oracle.density(c["grid"], n, kahan=True), "n_masked": masked,
            "n_max": float(n.max()), "max_norm_dev": float(np.abs(nd).max()),
            "samples": {str(int(i)): float(n[i]) for i in idx}}


if __name__ == "__main__":
    which = sys.argv[1:] or ["config1"]
    for w in which:
        if w == "config1":
            vals, name = config1_values(), "oracle_config1.json"
        elif w == "config2a":
            vals, name = full_grid_values(wl.config2a()), "oracle_config2a.json"
        elif w == "config2b":
            vals, name = full_grid_values(wl.config2b()), "oracle_config2b.json"
        else:
            raise SystemExit("unknown golden set %s" % w)
        path = os.path.join(HERE, name)
        with open(path, "w") as fh:
            json.dump(vals, fh, indent=1, sort_keys=True)
        print("wrote", path, flush=True)
