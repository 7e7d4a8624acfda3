"""The FP32 precision-budget model (tests/fp32_model.py) on the CPU: in FP64 arithmetic
its steps reproduce the oracle (so the model computes the method's step, Sec. III
Eqs. (11)-(12)); in FP32 it predicts an error well inside the FP32 bar of 1e-5 per point
for a 4000-step solve, growing about linearly with the step count (the roundings of a
slowly varying state are correlated).  The GPU test in test_gpu_parity.py holds the FP32
kernels to the same prediction."""
import numpy as np
import pytest

import oracle
from paper_1607_03062_amd import workloads as wl
from tests import fp32_model

FIELD = wl.config1()["field"]  # sin^2 pulse, E0 = 0.1, omega = 0.5, 8 cycles
GRID = {"nx": 48, "ny": 48, "px": (-2.0, 2.0), "py": (-2.0, 2.0)}


@pytest.mark.parametrize("arrangement", ["once", "fast"])
def test_model_in_fp64_is_the_oracle(arrangement):
    """Both arrangements, the fast one with its merged shears, are the method's step."""
    n_o = oracle.solve_grid(FIELD, GRID, 1500)[0]
    n = fp32_model.solve_grid(FIELD, GRID, 1500, arithmetic=np.float64, arrangement=arrangement)
    assert fp32_model.error_stats(n, n_o)[0] <= 1e-12


def test_model_fp32_error_and_its_growth():
    stats = {}
    for N in (4000, 16000):
        n_o = oracle.solve_grid(FIELD, GRID, N)[0]
        stats[N] = fp32_model.error_stats(fp32_model.solve_grid(FIELD, GRID, N), n_o)
    print("FP32 model vs oracle, 48^2: %s" % stats)
    mx, rms = stats[4000]
    assert 1e-7 <= mx <= 1e-5 and 1e-8 <= rms <= 1e-6  # an FP32 effect, inside the bar
    growth = stats[16000][1] / rms
    assert 1.5 <= growth <= 4.0, growth  # between sqrt(4) and 4 for four times the steps


def test_coefficient_phases_average_to_the_fp64_value():
    c = np.random.default_rng(3).uniform(-0.05, 0.05, 10000)
    ph = fp32_model._phases(c)
    ulp = np.spacing(np.abs(c.astype(np.float32))).astype(np.float64)
    assert ph.dtype == np.float32 and ph.shape == (4, c.size)
    assert np.all(np.abs(ph.astype(np.float64).mean(axis=0) - c) <= ulp / 8 + 1e-300)
    assert np.all(np.abs(ph.astype(np.float64) - c) <= ulp)
