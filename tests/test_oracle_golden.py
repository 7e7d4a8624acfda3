"""Regression of the oracle's conventions on config 1 (values written by
tests/golden/make_golden.py, which calls only the oracle).  Not an independent
check: the pins in test_oracle_pins.py are."""
import json
import os

import numpy as np

import oracle
from paper_1607_03062_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_config1.json")


def test_config1_regression():
    with open(GOLDEN) as fh:
        ref = json.load(fh)
    c = wl.config1()
    for s in ("strang", "midpoint"):
        n, nd, masked = oracle.solve_grid(c["field"], c["grid"], c["n_steps"], s)
        assert masked == ref[s]["n_masked"] == 1
        assert abs(oracle.density(c["grid"], n) - ref[s]["rho"]) <= 1e-15 * ref[s]["rho"]
        for k, v in ref[s]["n_at"].items():
            assert abs(n[int(k)] - v) <= 1e-15
        assert int(np.argmax(n)) == ref[s]["argmax"]
