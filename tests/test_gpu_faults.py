"""Injected faults (pd_set_fault) on the GPU: a failed device allocation or launch
sequence is reported as a status, leaves every grid where it stood, and the work around
it still ends bit for bit as without the fault; the serving loop retires what the fault
touched, or retries it from its last checkpoint, and serves the rest."""
import numpy as np
import pytest

from paper_1607_03062_amd import _lib
from paper_1607_03062_amd import serve
from paper_1607_03062_amd import workloads as wl

pytestmark = pytest.mark.gpu

FIELD = wl.sin2(0.2, 0.6, 3)


@pytest.fixture
def faults(gpu):
    yield gpu.set_fault
    gpu.set_fault(None)


def clean(gpu, grid, prec, N, scheme="strang"):
    s = gpu.Solver.for_grid(grid, prec, scheme)
    s.set_field(FIELD, N)
    s.propagate(-1)
    n = np.empty(s.nx * s.ny)
    rho = s.density(n_out=n)
    s.close()
    return n, rho


@pytest.mark.parametrize("prec,scheme", [("fp32", "strang"), ("fp64", "midpoint")])
def test_allocation_and_launch_faults_of_a_solve(gpu, faults, prec, scheme):
    grid, N = wl.grid(96, 2.0), 1500
    ref = clean(gpu, grid, prec, N, scheme)
    s = gpu.Solver.for_grid(grid, prec, scheme)
    faults("alloc@1")
    with pytest.raises(gpu.PDError) as e:
        s.set_field(FIELD, N)
    assert e.value.status == _lib.PD_ERR_NOMEM
    s.set_field(FIELD, N)  # the fault fired once
    s.propagate(400)
    faults("launch@1")
    with pytest.raises(gpu.PDError) as e:
        s.propagate(300)
    assert e.value.status == _lib.PD_ERR_DEVICE and s.info()["steps_done"] == 400
    s.propagate(-1)
    n = np.empty(s.nx * s.ny)
    rho = s.density(n_out=n)
    s.close()
    assert np.array_equal(n, ref[0]) and rho == ref[1]


def test_launch_faults_of_batch_epochs_and_runs(gpu, faults):
    specs = [(wl.grid(64, 2.0), "fp32", 900), (wl.grid(96, 2.0), "fp64", 1300), (wl.grid(1024, 3.0), "fp32", 700),
             (wl.grid(80, 2.0), "fp32", 1100)]
    refs = [clean(gpu, g, p, N) for g, p, N in specs]
    ms = []
    for g, p, N in specs:
        s = gpu.Solver.for_grid(g, p)
        s.set_field(FIELD, N)
        ms.append(s)
    b = gpu.Batch(ms)
    faults("launch@2")
    b.step(300)
    before = [s.info()["steps_done"] for s in ms]
    with pytest.raises(gpu.PDError) as e:
        b.step(300)
    assert e.value.status == _lib.PD_ERR_DEVICE and [s.info()["steps_done"] for s in ms] == before
    done = {}
    for _ in range(20):
        rho, fin = b.step(300)
        for i in range(len(ms)):
            if not np.isnan(rho[i]):
                done[i] = rho[i]
        if fin.all():
            break
    for i, s in enumerate(ms):
        n = np.empty(s.nx * s.ny)
        s.density(n_out=n)
        assert done[i] == refs[i][1] and np.array_equal(n, refs[i][0]), i
    # a whole-solve run: the failed call captures nothing; the next one captures and runs
    for s in ms:
        s.rewind()
    faults("launch@1")
    with pytest.raises(gpu.PDError):
        b.run()
    for s in ms:
        s.rewind()
    rho = b.run()
    assert [float(r) for r in rho] == [r[1] for r in refs]
    b.close()
    for s in ms:
        s.close()


def test_serving_retires_what_a_fault_touched(gpu, faults):
    """A failed epoch retires the solves planned in it ("failed", handles closed); a failed
    set-up allocation rejects that request; the rest complete equal to their solves alone,
    and all memory returns to the budget."""
    ws = wl.config5(count=10, seed=11, rate_per_s=1e9, sizes=(64, 96, 128), step_range=(1000, 4000))
    reqs = [serve.Request.from_workload(w) for w in ws]
    for r in reqs[5:]:
        r.arrival_s = 0.2  # after the failed epoch: served normally
    ex = serve.GpuExecutor(gpu, keep_n=True, background_setup=False)
    srv = serve.Server(ex, 10 ** 10, epoch_steps=512, policy="lockstep")
    faults("launch@3")
    st = srv.run(reqs)
    print("serve with a launch fault:", st.as_dict(), [(r.name, r.n_steps, r.status) for r in reqs], flush=True)
    failed = [r for r in reqs if r.status == "failed"]
    # the first five (3000 steps or more, all admitted by the second epoch) are all in the
    # third epoch and fail there; the later arrivals never see the fault
    assert all(r.n_steps > 3 * 512 for r in reqs[:5])
    assert {r.name for r in failed} == {r.name for r in reqs[:5]}
    assert st.failed == 5 and st.completed == 5
    assert srv.in_use == 0 and not srv.active
    for r in reqs:
        if r.status != "done":
            continue
        n, rho = clean_like(gpu, r)
        assert r.rho == rho and np.array_equal(ex.n_results[r.name], n), r.name
    ex.close()
    # an allocation fault at admission: that request is rejected, the others are served
    reqs = [serve.Request.from_workload(w) for w in ws[:4]]
    ex = serve.GpuExecutor(gpu, keep_n=True, background_setup=False, idle_per_shape=0)
    faults("alloc@2")
    st = serve.Server(ex, 10 ** 10, epoch_steps=512, policy="srpt").run(reqs)
    rejected = [r for r in reqs if r.status == "rejected"]
    assert len(rejected) == 1 and "hipMalloc" in rejected[0].reason and st.completed == 3
    ex.close()


@pytest.mark.parametrize("checkpoints", [True, False])
def test_serving_retries_a_failed_epoch(gpu, faults, checkpoints):
    """With max_retries the five solves of the failed third epoch are queued again on new
    handles: from the state the server copied to host memory after the second epoch
    (pd_save_state, then pd_load_state into the new handle), or from step 0 without
    checkpoints.  Every request completes, each equal to its solve alone bit for bit and
    to the FP64 oracle on its full grid (FP64 1e-12 per point and relative on rho; FP32
    1e-5 per point), and all memory returns to the budget."""
    import oracle

    ws = wl.config5(count=10, seed=11, rate_per_s=1e9, sizes=(64, 96, 128), step_range=(1000, 4000))
    reqs = [serve.Request.from_workload(w) for w in ws]
    for r in reqs[5:]:
        r.arrival_s = 0.2
    ex = serve.GpuExecutor(gpu, keep_n=True, background_setup=False)
    srv = serve.Server(ex, 10 ** 10, epoch_steps=512, policy="lockstep", max_retries=1,
                       checkpoint_every_s=0.0 if checkpoints else None)
    faults("launch@3")
    st = srv.run(reqs)
    print("serve with a launch fault and retries:", st.as_dict(),
          [(r.name, r.n_steps, r.status, r.retries, r.resumed_from) for r in reqs], flush=True)
    assert st.completed == 10 and st.failed == 0 and st.retried == 5
    assert [r.retries for r in reqs] == [1] * 5 + [0] * 5
    # admitted four in the first epoch and one in the second: 1024 or 512 steps done before
    # the failed epoch, where a checkpoint resumes them
    if checkpoints:
        assert sorted(r.resumed_from for r in reqs[:5]) == [512] + [1024] * 4
    else:
        assert all(r.resumed_from == 0 for r in reqs)
    assert srv.in_use == 0 and not srv.active
    for r in reqs:
        n, rho = clean_like(gpu, r)
        assert r.rho == rho and np.array_equal(ex.n_results[r.name], n), r.name
        n_o = oracle.solve_grid(r.field, r.grid, r.n_steps, r.scheme)[0]
        err = float(np.max(np.abs(n - n_o)))
        if r.precision == "fp64":
            assert err <= 1e-12 and abs(rho / oracle.density(r.grid, n_o) - 1) <= 1e-12, (r.name, err)
        else:
            assert err <= 1e-5, (r.name, err)
    ex.close()


def clean_like(gpu, r):
    s = gpu.Solver.for_grid(r.grid, r.precision, r.scheme, r.valley)
    s.set_field(r.field, r.n_steps)
    s.propagate(-1)
    n = np.empty(s.nx * s.ny)
    rho = s.density(n_out=n)
    s.close()
    return n, rho
