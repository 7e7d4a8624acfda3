"""The continuous-batching scheduler with the CPU fake executor (simulated device time):
admission by footprint, queueing, rejection, completion and latency accounting."""
import numpy as np
import pytest

from paper_1607_03062_amd import serve
from paper_1607_03062_amd import workloads as wl


def stream(count=40, rate=200.0, seed=5):
    ws = wl.config5(count=count, seed=seed, rate_per_s=rate, sizes=(64, 128, 256), step_range=(500, 4000))
    return [serve.Request.from_workload(w) for w in ws]


def test_every_request_completes_within_budget():
    ex = serve.FakeExecutor(rate_point_steps_per_s=2e10)
    reqs = stream()
    budget = 4 * max(ex.footprint(r) for r in reqs)
    st = serve.Server(ex, budget, epoch_steps=512, policy="lockstep").run(reqs, simulated=True)
    assert st.completed == len(reqs) and st.rejected == 0
    assert st.peak_bytes <= budget
    for r in reqs:
        assert r.status == "done"
        assert r.admitted_s >= r.arrival_s - 1e-12 and r.done_s >= r.admitted_s
        # at least its own work at the full device rate
        assert r.done_s - r.admitted_s >= r.point_steps / 2e10 * (1 - 1e-9)


def test_fifo_admission_and_queueing():
    ex = serve.FakeExecutor(rate_point_steps_per_s=1e10)
    reqs = stream(count=30, rate=1000.0)
    budget = max(ex.footprint(r) for r in reqs) + 1  # forces queueing
    st = serve.Server(ex, budget, epoch_steps=1024, policy="lockstep").run(reqs, simulated=True)
    assert st.completed == len(reqs)
    adm = [r.admitted_s for r in sorted(reqs, key=lambda r: r.arrival_s)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))  # in arrival order
    assert any(r.admitted_s > r.arrival_s for r in reqs)  # someone waited
    assert st.peak_bytes <= budget


def test_oversized_request_is_rejected():
    ex = serve.FakeExecutor()
    reqs = stream(count=10)
    big = serve.Request("huge", 0.0, wl.grid(4096, 4.0), wl.sin2(0.1, 0.5, 8), 1000)
    budget = max(ex.footprint(r) for r in reqs) * 2
    st = serve.Server(ex, budget, policy="lockstep").run(reqs + [big], simulated=True)
    assert big.status == "rejected" and "budget" in big.reason
    assert st.rejected == 1 and st.completed == len(reqs)


def test_percentiles_and_throughput():
    ex = serve.FakeExecutor(rate_point_steps_per_s=5e10)
    reqs = stream(count=25)
    st = serve.Server(ex, 10 ** 12, epoch_steps=256, policy="lockstep").run(reqs, simulated=True)
    lat = np.array([r.latency_s for r in reqs]) * 1e3
    assert st.p50_ms == pytest.approx(np.percentile(lat, 50))
    assert st.p99_ms == pytest.approx(np.percentile(lat, 99))
    total = sum(r.point_steps for r in reqs)
    assert st.point_steps_per_s == pytest.approx(total / st.makespan_s)
    assert st.point_steps_per_s <= 5e10 * (1 + 1e-9)


def test_epoch_count_of_a_lone_request():
    ex = serve.FakeExecutor()
    r = serve.Request("one", 0.0, wl.grid(64, 2.0), wl.sin2(0.1, 0.5, 8), 5000)
    st = serve.Server(ex, 10 ** 12, epoch_steps=2048, policy="lockstep").run([r], simulated=True)
    assert st.epochs == 3 and r.status == "done"


def test_backfill_admits_smaller_requests_past_a_blocked_head():
    ex = serve.FakeExecutor(rate_point_steps_per_s=1e10)
    small = [serve.Request("s%d" % i, 0.001 * (i + 1), wl.grid(64, 2.0), wl.sin2(0.1, 0.5, 8), 2000)
             for i in range(4)]
    first = serve.Request("first", 0.0, wl.grid(256, 2.0), wl.sin2(0.1, 0.5, 8), 20000)
    head = serve.Request("head", 0.0005, wl.grid(256, 2.0), wl.sin2(0.1, 0.5, 8), 2000)
    budget = ex.footprint(first) + ex.footprint(small[0]) * 4 + 1
    serve.Server(ex, budget, epoch_steps=512, backfill=True, policy="lockstep").run([first, head] + small, simulated=True)
    assert all(s.admitted_s < head.admitted_s for s in small)


def test_request_refused_at_admission_is_rejected_and_frees_nothing():
    class Picky(serve.FakeExecutor):
        def admit(self, req, background=True):
            if req.name == "bad":
                raise RuntimeError("dt * E_max exceeds pi")
            super().admit(req, background)

    ex = Picky()
    reqs = stream(count=6)
    bad = serve.Request("bad", 0.0, wl.grid(64, 2.0), wl.sin2(0.1, 0.5, 8), 10)
    srv = serve.Server(ex, 10 ** 12, policy="lockstep")
    st = srv.run(reqs + [bad], simulated=True)
    assert bad.status == "rejected" and "pi" in bad.reason
    assert st.completed == len(reqs) and srv.in_use == 0


def test_solve_bytes_closed_form_matches_check_field():
    import paper_1607_03062_amd as pd

    for prec in ("fp32", "fp64"):
        for scheme in ("strang", "midpoint"):
            s = pd.Solver(100, 60, (-4, 4), (-4, 4), prec, scheme)
            info = s.check_field(wl.sin2(0.2, 0.5, 8), 5000)
            assert s.solve_bytes(5000) == info["solve_bytes"] > 6000 * 8
            s.close()


def mixed_stream(count=120, seed=7, rate=None):
    """Poisson arrivals of grids 32^2..256^2 with 500..6000 steps (both precisions)."""
    ws = wl.config5(count=count, seed=seed, rate_per_s=rate or 1.0, sizes=(32, 64, 128, 256),
                    step_range=(500, 6000))
    return [serve.Request.from_workload(w) for w in ws]


def test_srpt_serves_everything_and_cuts_latency():
    """At 0.7 load, shortest-remaining-work-first epochs complete every request and lower the
    mean and median latency against lockstep epochs, at the same device throughput."""
    rate_dev, tile = 2e10, 2e-6
    probe = mixed_stream()
    mean_work = np.mean([r.point_steps for r in probe]) / rate_dev
    stats = {}
    for policy in ("lockstep", "srpt"):
        reqs = mixed_stream(rate=0.7 / mean_work)
        ex = serve.FakeExecutor(rate_point_steps_per_s=rate_dev, tile_step_s=tile, epoch_overhead_s=1e-5)
        srv = serve.Server(ex, 10 ** 12, epoch_steps=256, policy=policy, epoch_ms=1.0,
                           rates={"fp32": rate_dev, "fp64": rate_dev}, tile_step_s=tile)
        st = srv.run(reqs, simulated=True)
        assert st.completed == len(reqs) and st.rejected == 0
        assert all(r.status == "done" for r in reqs) and not srv.left
        stats[policy] = st
    assert stats["srpt"].mean_ms < 0.9 * stats["lockstep"].mean_ms
    assert stats["srpt"].p50_ms < stats["lockstep"].p50_ms
    assert stats["srpt"].makespan_s <= 1.05 * stats["lockstep"].makespan_s


def test_srpt_epoch_plan():
    """The plan fills the epoch's time budget with the least remaining work first, each solve
    up to one tile's share of steps and never past its last step; a solve larger than the whole
    budget still advances when it is alone."""
    ex = serve.FakeExecutor()
    srv = serve.Server(ex, 10 ** 12, epoch_steps=100, policy="srpt", epoch_ms=1.0,
                       rates={"fp32": 1e9, "fp64": 1e9}, tile_step_s=1e-6)  # share = 1000 steps
    sizes = {"a": (16, 5000), "b": (32, 300), "c": (64, 4000), "d": (256, 9000)}
    for name, (n, steps) in sizes.items():
        r = serve.Request(name, 0.0, wl.grid(n, 2.0), wl.sin2(0.1, 0.5, 8), steps)
        srv.active[name] = r
        srv.left[name] = steps
        srv.ready.add(name)
    plan = srv.plan_epoch()
    # remaining work: b 3.1e5 < a 1.3e6 < c 1.6e7 < d 5.9e8 point-steps; budget 1e6 point-steps
    assert plan["b"] == 300 and plan["a"] == 1000
    assert "d" not in plan
    used = sum(srv.active[k].points * m for k, m in plan.items())
    assert used <= 1e6 + 1e-6
    assert all(m <= srv.left[k] for k, m in plan.items())
    for k in ("a", "b", "c"):
        del srv.active[k], srv.left[k]
    assert srv.plan_epoch() == {"d": 15}  # 1e6 / 65536 points
    srv.rates = {"fp32": 1e6, "fp64": 1e6}  # now larger than the whole budget
    assert srv.plan_epoch() == {"d": 100}


def test_policy_arguments_are_checked():
    ex = serve.FakeExecutor()
    with pytest.raises(ValueError):
        serve.Server(ex, 10 ** 9, policy="fifo")
    with pytest.raises(ValueError):
        serve.Server(ex, 10 ** 9, policy="srpt", epoch_ms=0)


def test_srpt_does_not_starve_a_large_request():
    """Overload: small requests (1 ms of device time each) arrive every 0.8 ms after a large
    one, so that on their own they would take every epoch.  Without aging the large request
    gets no steps until the stream ends; with aging (max_wait_epochs = 8) the solves that
    waited long are served in turn, the longest waiting first, and the large one keeps
    advancing while the stream lasts."""
    def progress_by_last_arrival(max_wait):
        rate_dev, tile = 1e9, 1e-6
        big = serve.Request("big", 0.0, wl.grid(256, 2.0), wl.sin2(0.1, 0.5, 8), 3000)
        smalls = [serve.Request("s%d" % i, 8e-4 * i, wl.grid(32, 2.0), wl.sin2(0.1, 0.5, 8), 1000)
                  for i in range(1, 800)]
        ex = serve.FakeExecutor(rate_point_steps_per_s=rate_dev, tile_step_s=tile)
        # admissions right after finishing epochs (defer_admissions off), so that the small
        # requests alone could take every epoch and only the aging rule serves the large one
        srv = serve.Server(ex, 10 ** 12, epoch_steps=100, policy="srpt", epoch_ms=1.0,
                           rates={"fp32": rate_dev, "fp64": rate_dev}, tile_step_s=tile, max_wait_epochs=max_wait,
                           defer_admissions=False)
        seen = []
        epoch_each = ex.epoch_each

        def record(steps):
            out = epoch_each(steps)
            seen.append((ex.clock, ex.active["big"][1] if "big" in ex.active else big.n_steps))
            return out
        ex.epoch_each = record
        st = srv.run([big] + smalls, simulated=True)
        assert big.status == "done" and st.completed == len(smalls) + 1
        return max(k for clock, k in seen if clock <= smalls[-1].arrival_s)

    starved = progress_by_last_arrival(10 ** 9)
    aged = progress_by_last_arrival(8)
    assert starved <= 100  # only the epochs before the small requests arrived
    assert aged >= 150 and aged >= 5 * starved


def test_admissions_per_epoch_are_capped():
    """A burst of 10 requests at t = 0 with admit_per_epoch = 3: the first epochs run with 3, 6
    and 9 admitted solves, in arrival order; all complete."""
    ex = serve.FakeExecutor(rate_point_steps_per_s=1e10)
    reqs = [serve.Request("r%d" % i, 0.0, wl.grid(64, 2.0), wl.sin2(0.1, 0.5, 8), 20000) for i in range(10)]
    srv = serve.Server(ex, 10 ** 12, epoch_steps=512, admit_per_epoch=3, policy="lockstep")
    sizes = []
    epoch_each = ex.epoch_each

    def record(steps):
        sizes.append(len(ex.active))
        return epoch_each(steps)
    ex.epoch_each = record
    st = srv.run(reqs, simulated=True)
    assert sizes[:4] == [3, 6, 9, 10]
    assert st.completed == 10
    adm = [r.admitted_s for r in reqs]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    with pytest.raises(ValueError):
        serve.Server(ex, 10 ** 9, admit_per_epoch=0, policy="lockstep")


def test_admissions_wait_for_the_epoch_after_a_finish():
    """After an epoch in which a request finished (the host waited for the device, now idle),
    the next epoch of the remaining solves is enqueued before new arrivals are set up: the
    epoch that follows a finish never contains a request admitted after that finish."""
    ex = serve.FakeExecutor(rate_point_steps_per_s=1e10)
    reqs = [serve.Request("r%d" % i, 0.0, wl.grid(64, 2.0), wl.sin2(0.1, 0.5, 8), 600 + 500 * i)
            for i in range(6)]
    srv = serve.Server(ex, 10 ** 12, epoch_steps=500, admit_per_epoch=2, policy="lockstep")
    members = []
    epoch_each = ex.epoch_each

    def record(steps):
        members.append(set(ex.active))
        return epoch_each(steps)
    ex.epoch_each = record
    finished_after = []
    release = ex.release

    def on_release(name):
        finished_after.append((len(members), name))
        release(name)
    ex.release = on_release
    st = srv.run(reqs, simulated=True)
    assert st.completed == 6
    for epoch, name in finished_after:
        if epoch < len(members):
            # the epoch right after a finish runs the solves that were there before it
            assert members[epoch] <= members[epoch - 1], (epoch, name)
    off = serve.Server(serve.FakeExecutor(rate_point_steps_per_s=1e10), 10 ** 12, epoch_steps=500,
                       admit_per_epoch=2, policy="lockstep", defer_admissions=False)
    assert off.run([serve.Request(r.name, 0.0, r.grid, r.field, r.n_steps) for r in reqs],
                   simulated=True).completed == 6


def test_requests_join_when_their_set_up_finishes():
    """Background set-up: an admitted request joins the epochs only once its set-up has
    finished (here two epochs later), never before; a set-up the library refuses rejects
    the request and frees its memory; everything else completes."""
    reqs = [serve.Request("r%d" % i, 0.0, wl.grid(64, 2.0), wl.sin2(0.1, 0.5, 8), 900 + 300 * i)
            for i in range(8)]
    ex = serve.FakeExecutor(rate_point_steps_per_s=1e10, setup_epochs=2, refuse=lambda r: r.name == "r5")
    srv = serve.Server(ex, 10 ** 12, epoch_steps=300, admit_per_epoch=3, policy="lockstep")
    planned = []
    epoch_each = ex.epoch_each

    def record(steps):
        planned.append((set(k for k, m in steps.items() if m > 0), set(ex.active), set(ex.setting_up)))
        return epoch_each(steps)
    ex.epoch_each = record
    st = srv.run(reqs, simulated=True)
    assert st.completed == 7 and st.rejected == 1
    assert reqs[5].status == "rejected" and "refused" in reqs[5].reason
    for stepped, joined, setting_up in planned:
        assert stepped <= joined and not (stepped & setting_up)
    assert srv.in_use == 0 and not srv.active and not srv.ready


def test_epoch_tuner_keeps_the_shortest_candidate_near_the_fastest_and_caches(tmp_path):
    """tune_epoch_ms serves the same closed set once per candidate and repetition and keeps
    the shortest candidate within the tolerance of the shortest median makespan; a cached
    value for the key is returned without timing."""
    reqs = [serve.Request("r%d" % i, 0.5 * i, wl.grid(64 * (1 + i % 4), 2.0), wl.sin2(0.1, 0.5, 8), 2000 + 700 * i)
            for i in range(12)]
    made = []

    def make():
        made.append(1)  # a per-epoch overhead makes the shortest epochs slow
        return serve.FakeExecutor(rate_point_steps_per_s=2e10, tile_step_s=2e-7, epoch_overhead_s=2e-4)
    kw = dict(epoch_steps=64, rates={"fp32": 2e10, "fp64": 2e10}, tile_step_s=2e-7)
    cache = str(tmp_path / "epochs.txt")
    best, spans = serve.tune_epoch_ms(make, 10 ** 12, reqs, candidates=(0.1, 0.5, 2.0), repeats=2, simulated=True,
                                      cache_path=cache, cache_key="gfx950 srpt", **kw)
    assert len(made) == 6 and all(len(v) == 2 for v in spans.values())
    med = {c: float(np.median(v)) for c, v in spans.items()}
    assert best == min(c for c in med if med[c] <= 1.02 * min(med.values())) and best != 0.1
    # with no tolerance the fastest candidate wins; with a wide one the shortest
    mk = dict(kw, simulated=True, candidates=(0.1, 0.5, 2.0), repeats=1)
    assert serve.tune_epoch_ms(make, 10 ** 12, reqs, tolerance=0.0, **mk)[0] == min(med, key=med.get)
    assert serve.tune_epoch_ms(make, 10 ** 12, reqs, tolerance=10.0, **mk)[0] == 0.1
    assert all(r.status == "pending" for r in reqs)  # the caller's requests are not served
    again, spans2 = serve.tune_epoch_ms(lambda: pytest.fail("timed despite the cache"), 10 ** 12, reqs,
                                        cache_path=cache, cache_key="gfx950 srpt")
    assert again == best and spans2 == {}
    with pytest.raises(ValueError):
        serve.tune_epoch_ms(make, 10 ** 12, reqs, candidates=(0.0, 1.0), simulated=True)


def test_idle_pool_keeps_reuses_and_evicts():
    """Kept handles: at most per_shape per shape; reserve() evicts other shapes oldest first,
    then the requested shape's newer handles, and keeps the oldest one, which take() returns."""
    closed = []
    pool = serve.IdlePool(2, closed.append)
    assert pool.put("A", "a1", 10) and pool.put("A", "a2", 20)
    assert not pool.put("A", "a3", 5)  # a third of shape A is not kept
    assert pool.put("B", "b1", 100)
    assert pool.bytes == 130
    pool.reserve("A", 15)  # room for 15 bytes beyond a1, which the request will reuse
    assert closed == ["b1", "a2"] and pool.bytes == 10
    assert pool.take("A") == "a1" and pool.bytes == 0
    assert pool.take("A") is None
    pool.reserve("C", 0)  # nothing kept: nothing to do
    assert pool.put("C", "c1", 7)
    pool.reserve("D", 100)  # enough room: c1 stays
    assert pool.bytes == 7
    pool.clear()
    assert closed == ["b1", "a2", "c1"] and pool.bytes == 0


@pytest.mark.parametrize("slack", [4.0, 1.0])
def test_kept_handles_are_reused_within_the_budget(slack):
    """With handles kept for reuse, requests of a shape seen before reuse one, and the
    admitted footprints plus the kept handles never exceed the budget, also when the budget
    holds one request only (every admission then evicts what is kept)."""
    ex = serve.FakeExecutor(rate_point_steps_per_s=2e10, idle_per_shape=2)
    reqs = stream(count=60)
    budget = int(slack * max(ex.footprint(r) for r in reqs)) + 1
    srv = serve.Server(ex, budget, epoch_steps=512, policy="lockstep")
    over = []
    admit = ex.admit

    def checked(r, background=True):
        admit(r, background)  # the server adds r.bytes to in_use after this returns
        over.append(srv.in_use + r.bytes + ex.idle_bytes - budget)
    ex.admit = checked
    st = srv.run(reqs, simulated=True)
    assert st.completed == len(reqs) and st.rejected == 0
    assert ex.reused > 0
    assert max(over) <= 0 and st.peak_bytes <= budget
    shapes = {serve.shape_key(r) for r in reqs}
    assert len(ex.idle.entries) <= 2 * len(shapes)


def _req(name, arrival, n, steps, **kw):
    return serve.Request(name, arrival, wl.grid(n, 2.0), wl.sin2(0.1, 0.5, 4), steps, **kw)


@pytest.mark.parametrize("policy", ["srpt", "lockstep"])
def test_cancelled_and_expired_requests_leave_and_free_their_memory(policy):
    """A request cancelled part-way through (cancel_s), one cancelled before it arrives
    (Server.cancel), one that expires in the queue and one that expires part-way through
    all leave with their status; the others complete as usual, the memory returns to the
    budget (in_use 0 at the end), and a later request of the cancelled one's shape reuses
    its kept handle."""
    ex = serve.FakeExecutor(rate_point_steps_per_s=1e9, idle_per_shape=2)
    reqs = [_req("long_cancelled", 0.0, 256, 40000, cancel_s=0.5),
            _req("blocker", 0.001, 256, 20000),
            _req("running_expires", 0.002, 128, 200000, deadline_s=1.0),
            _req("queued_expires", 0.003, 512, 1000, deadline_s=0.05),
            _req("withdrawn", 0.004, 64, 1000),
            _req("after", 5.0, 256, 2000)]
    first3 = sum(ex.footprint(r) for r in reqs[:3])
    assert first3 + ex.footprint(reqs[3]) > first3 + first3 // 10  # the 512^2 one has to wait
    srv = serve.Server(ex, first3 + first3 // 10, epoch_steps=256, policy=policy, epoch_ms=3.0,
                       rates={"fp32": 1e9})
    srv.cancel("withdrawn")
    st = srv.run(reqs, simulated=True)
    by = {r.name: r for r in reqs}
    assert by["long_cancelled"].status == "cancelled" and not np.isfinite(by["long_cancelled"].rho)
    assert abs(by["long_cancelled"].done_s - 0.5) < 0.05  # at the first epoch boundary past 0.5 s
    assert by["withdrawn"].status == "cancelled" and by["withdrawn"].admitted_s != by["withdrawn"].admitted_s
    assert by["queued_expires"].status == "expired" and by["queued_expires"].admitted_s != by["queued_expires"].admitted_s
    assert by["running_expires"].status == "expired" and by["running_expires"].admitted_s >= 0
    assert 1.0 < by["running_expires"].done_s < 1.1
    assert by["blocker"].status == "done" and by["after"].status == "done"
    assert st.completed == 2 and st.cancelled == 2 and st.expired == 2 and st.rejected == 0
    assert srv.in_use == 0 and not srv.active and not srv.left and not srv.ready
    assert ex.reused >= 1  # "after" took a kept 256^2 handle
    assert st.peak_bytes <= srv.budget


def test_cancel_during_background_set_up():
    """A request withdrawn while its set-up is still in flight is abandoned from there."""
    ex = serve.FakeExecutor(rate_point_steps_per_s=1e10, setup_epochs=3)
    reqs = [_req("a", 0.0, 128, 30000), _req("b", 0.0, 128, 30000, cancel_s=0.002), _req("c", 0.0, 64, 500)]
    srv = serve.Server(ex, 10 ** 12, epoch_steps=512, policy="srpt", epoch_ms=1.0)
    st = srv.run(reqs, simulated=True)
    assert [r.status for r in reqs] == ["done", "cancelled", "done"]
    assert st.cancelled == 1 and srv.in_use == 0 and not ex.setting_up and not ex.active


@pytest.mark.parametrize("policy", ["srpt", "lockstep"])
def test_failed_epochs_retire_their_members_only(policy):
    """Epochs whose launch fails (they advance nothing) retire the solves planned in them
    with status "failed" and close their handles; every other request completes with its
    full work, and the memory returns to the budget."""
    reqs = stream(count=24, rate=500.0)
    ex = serve.FakeExecutor(rate_point_steps_per_s=2e10, idle_per_shape=2, fail_epochs={3, 10})
    planned = []
    orig = ex.epoch_each

    def spy(steps):
        planned.append(sorted(n for n, m in steps.items() if m > 0))
        return orig(steps)
    ex.epoch_each = spy
    budget = 4 * max(ex.footprint(r) for r in reqs)
    srv = serve.Server(ex, budget, epoch_steps=512, policy=policy, epoch_ms=0.5, rates={"fp32": 2e10, "fp64": 2e10})
    st = srv.run(reqs, simulated=True)
    failed = {r.name for r in reqs if r.status == "failed"}
    assert failed == set(planned[2]) | set(planned[9]) and failed
    assert st.failed == len(failed) and st.completed == len(reqs) - len(failed)
    assert all(r.status == "done" for r in reqs if r.name not in failed)
    assert all("injected epoch failure" in r.reason for r in reqs if r.name in failed)
    assert srv.in_use == 0 and not srv.active and not ex.active


@pytest.mark.parametrize("checkpoints", [True, False])
@pytest.mark.parametrize("policy", ["srpt", "lockstep"])
def test_failed_epochs_are_retried(policy, checkpoints):
    """With max_retries the solves of a failed epoch are queued again and complete.  With a
    checkpoint after every epoch each resumes where the failed epoch would have started
    it, so its successful epochs add up to exactly its step count; without checkpoints it
    restarts from step 0 and its successful epochs add up to its step count plus the
    steps it had done before the failure."""
    reqs = stream(count=24, rate=500.0)
    ex = serve.FakeExecutor(rate_point_steps_per_s=2e10, idle_per_shape=2, fail_epochs={3, 10})
    log = []  # (planned steps, failed)
    orig = ex.epoch_each

    def spy(steps):
        planned = {n: m for n, m in steps.items() if m > 0}
        try:
            out = orig(steps)
        except RuntimeError:
            log.append((planned, True))
            raise
        log.append((planned, False))
        return out
    ex.epoch_each = spy
    budget = 4 * max(ex.footprint(r) for r in reqs)
    srv = serve.Server(ex, budget, epoch_steps=512, policy=policy, epoch_ms=0.5, rates={"fp32": 2e10, "fp64": 2e10},
                       max_retries=2, checkpoint_every_s=0.0 if checkpoints else None)
    st = srv.run(reqs, simulated=True)
    hit = set(log[2][0]) | set(log[9][0])
    assert hit and log[2][1] and log[9][1]
    assert st.completed == len(reqs) and st.failed == 0 and st.retried == len(log[2][0]) + len(log[9][0])
    assert {r.name for r in reqs if r.retries} == hit
    for r in reqs:
        ran = sum(p.get(r.name, 0) for p, failed in log if not failed)
        # successful steps before the last failed epoch that planned it
        last = max((i for i, (p, failed) in enumerate(log) if failed and r.name in p), default=-1)
        before = sum(p.get(r.name, 0) for p, failed in log[:max(last, 0)] if not failed)
        assert r.retries == sum(1 for p, failed in log if failed and r.name in p)
        if r.name not in hit:
            assert ran == r.n_steps
        elif checkpoints:
            assert ran == r.n_steps and r.resumed_from == before, r.name
        else:
            assert ran == r.n_steps + before and r.resumed_from == 0, r.name
        assert r.checkpoint is None  # host copies released when the request left
    assert (st.checkpoints > 0) == checkpoints
    assert srv.in_use == 0 and not srv.active and not ex.active


def test_retries_are_bounded():
    """A solve whose every epoch fails is retried max_retries times, then fails."""
    reqs = stream(count=1, rate=500.0)
    ex = serve.FakeExecutor(rate_point_steps_per_s=2e10, fail_epochs=set(range(1, 100)))
    srv = serve.Server(ex, 4 * ex.footprint(reqs[0]), epoch_steps=512, max_retries=3, checkpoint_every_s=0.0)
    st = srv.run(reqs, simulated=True)
    assert st.failed == 1 and st.retried == 3 and reqs[0].retries == 3 and ex.epoch_calls == 4
    assert reqs[0].status == "failed" and reqs[0].checkpoint is None
