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


if __name__ == "__main__":
    path = os.path.join(HERE, "oracle_config1.json")
    with open(path, "w") as fh:
        json.dump(config1_values(), fh, indent=1, sort_keys=True)
    print("wrote", path)
