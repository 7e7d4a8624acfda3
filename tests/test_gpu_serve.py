"""Serving on the GPU: requests arriving while others run are admitted at epoch
boundaries as memory frees up, share persistent launches, and each result equals
the same request solved alone (bit for bit: n(p) and rho)."""
import numpy as np
import pytest

from paper_1607_03062_amd import serve
from paper_1607_03062_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("policy", ["lockstep", "srpt"])
def test_results_in_the_mix_equal_alone(gpu, policy):
    ws = wl.config5(count=14, seed=5, rate_per_s=400.0, sizes=(64, 96, 128, 192), step_range=(800, 5000))
    # a few requests of the other schemes, precisions, polarisations and valleys in the stream
    extras = [("strang4", "fp32", "both", 0.0), ("midpoint", "fp64", "K-", 0.6), ("strang", "fp32fast", "K+", 0.8),
              ("midpoint4", "fp32", "both", 0.0)]
    for q, (scheme, prec, valley, e) in enumerate(extras):
        w = ws[3 * q + 1]
        w.update(scheme=scheme, precision=prec, valley=valley, field=dict(w["field"], ellipticity=e))
        if scheme.endswith("4"):
            w["n_steps"] = max(200, w["n_steps"] // 5)
    reqs = [serve.Request.from_workload(w) for w in ws]
    ex = serve.GpuExecutor(gpu, keep_n=True)
    fp = [ex.footprint(r) for r in reqs]
    budget = int(2.5 * max(fp))  # a few at a time: arrivals queue behind running solves
    # srpt: a small time budget so that epochs give the solves unequal step counts
    st = serve.Server(ex, budget, epoch_steps=700, policy=policy, epoch_ms=0.2).run(reqs)
    print("serve:", st.as_dict(), flush=True)
    assert st.completed == len(reqs) and st.peak_bytes <= budget
    assert any(r.admitted_s > r.arrival_s + 1e-4 for r in reqs)
    for r in reqs:
        s = gpu.Solver.for_grid(r.grid, r.precision, r.scheme, r.valley)
        s.set_field(r.field, r.n_steps)
        s.propagate(-1)
        n = np.empty(s.nx * s.ny)
        rho = s.density(n_out=n)
        s.close()
        assert r.rho == rho, r.name
        assert np.array_equal(ex.n_results[r.name], n), r.name
    ex.close()


def test_footprint_matches_allocation(gpu):
    """solve_bytes (used for admission) covers what a chunked solve allocates."""
    c = wl.config1()
    for prec in ("fp32", "fp64"):
        s = gpu.Solver.for_grid(c["grid"], prec)
        need = s.check_field(c["field"], c["n_steps"])["solve_bytes"]
        s.set_field(c["field"], c["n_steps"])
        s.propagate(100)  # chunked: allocates the state buffer
        have = s.info()["device_bytes"]
        assert have <= need <= have + 4096, (prec, have, need)
        s.close()
