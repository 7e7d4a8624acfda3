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
    for r in reqs[:5]:
        r.arrival_s = 0.0  # a burst larger than the budget: some of it must wait for a finish
    ex = serve.GpuExecutor(gpu, keep_n=True)
    fp = [ex.footprint(r) for r in reqs]
    budget = int(2.5 * max(fp))  # a few at a time: arrivals queue behind running solves
    assert sum(fp[:5]) > budget
    # srpt: a small time budget so that epochs give the solves unequal step counts
    st = serve.Server(ex, budget, epoch_steps=700, policy=policy, epoch_ms=0.2).run(reqs)
    print("serve:", st.as_dict(), "handles reused:", ex.reused, flush=True)
    assert st.completed == len(reqs) and st.peak_bytes <= budget
    first_done = min(r.done_s for r in reqs)
    assert any(r.admitted_s >= first_done for r in reqs)  # admitted only once memory was freed
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


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_reused_handles_equal_fresh_ones(gpu, precision):
    """Requests of one shape, one at a time: each after the first reuses the finished one's
    handle (its table shrinking and growing with the step count) and gives the n(p) and rho
    of a fresh handle, bit for bit."""
    g = wl.grid(64, 2.0)
    steps = [3000, 800, 5000, 1200, 4000]
    reqs = [serve.Request("r%d" % i, 0.001 * i, g, wl.sin2(0.1 + 0.02 * i, 0.5, 8), n, precision)
            for i, n in enumerate(steps)]
    ex = serve.GpuExecutor(gpu, keep_n=True)
    fp = sorted(ex.footprint(r) for r in reqs)
    assert fp[0] + fp[1] > fp[-1]  # a budget of the largest footprint admits one request at a time
    budget = fp[-1]
    st = serve.Server(ex, budget, epoch_steps=700, policy="lockstep").run(reqs)
    assert st.completed == len(reqs) and st.peak_bytes <= budget
    assert ex.reused == len(reqs) - 1
    for r in reqs:
        s = gpu.Solver.for_grid(r.grid, r.precision)
        s.set_field(r.field, r.n_steps)
        s.propagate(-1)
        n = np.empty(s.nx * s.ny)
        rho = s.density(n_out=n)
        s.close()
        assert r.rho == rho and np.array_equal(ex.n_results[r.name], n), r.name
    ex.close()


def test_set_field_waits_for_its_own_work_only(gpu):
    """A new field on a handle waits for that handle's earlier work, not for the device: a
    long solve on another stream is still running when the call returns (the new field is
    shorter, so its table fits the allocation and nothing is freed).  The reused handle's
    chunked solve then matches a fresh handle bit for bit."""
    import torch

    c3 = wl.config3()
    long_solve = gpu.Solver.for_grid(c3["grid"], "fp64")
    long_solve.set_field(c3["field"], c3["n_steps"])
    small = gpu.Solver.for_grid(wl.config1()["grid"], "fp32")
    f1 = wl.config1()["field"]
    small.set_field(f1, 3000)
    st_small = torch.cuda.Stream()
    small.propagate(700, stream=st_small)  # chunked: the state buffer is in use
    small.propagate(-1, stream=st_small)
    small.density(stream=st_small)  # waits for the small solve
    st_long = torch.cuda.Stream()
    long_solve.propagate(-1, stream=st_long)  # about 0.1 s of device time
    small.set_field(wl.sin2(0.15, 0.5, 8), 2000)
    still_running = not st_long.query()
    small.propagate(1000, stream=st_small)
    small.propagate(-1, stream=st_small)
    n = np.empty(64 * 64)
    rho = small.density(n_out=n, stream=st_small)
    st_long.synchronize()
    long_solve.close()
    small.close()
    assert still_running
    fresh = gpu.Solver.for_grid(wl.config1()["grid"], "fp32")
    fresh.set_field(wl.sin2(0.15, 0.5, 8), 2000)
    fresh.propagate(1000)
    fresh.propagate(-1)
    n_f = np.empty(64 * 64)
    rho_f = fresh.density(n_out=n_f)
    fresh.close()
    assert rho == rho_f and np.array_equal(n, n_f)
