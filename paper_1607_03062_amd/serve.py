"""Continuous-batching solve server.

Requests (a grid, a field, a step count, a precision, a scheme and a valley)
arrive over time.  The server keeps a set of active solves on the device and runs
them in epochs: each epoch advances active solves in one batched launch sequence
(pd_batch_step_each: one persistent kernel for the second-order Strang solves of
fields along x, the others' own launches beside it), with every solve's state
resident in device memory between epochs.  Solves that reach their last step are
projected and reduced in the same epoch and leave the set (their handles are kept
for later requests of the same shape, within the memory budget); arrivals are admitted
between epochs, in arrival order, while their device footprint (tables, state,
n(p), partials; pd_info.solve_bytes) fits in the memory budget, at most
`admit_per_epoch` at a time so that a burst of arrivals is set up on the host while
the device runs the epochs of those already admitted.  A request larger
than the whole budget is rejected.  Latency is the time from a request's arrival
to its density being on the host.  A request withdrawn by the client (Server.cancel,
or its cancel_s) or past its deadline_s leaves at the next epoch boundary, queued or
part-way through, with status "cancelled" or "expired"; its memory goes back to the
budget and its handle is kept like a finished one.  If an epoch's launch fails (the
library reports it; nothing was advanced), the solves planned in it lose their handles
(after a real device fault their device state cannot be trusted); each is queued again,
ahead of later arrivals, while it has retries left (`max_retries`), else it leaves with
status "failed"; the others go on.  A retried solve restarts from its last checkpoint
(with `checkpoint_every_s`, the server copies each active solve's state to host memory,
pd_save_state, at most that often), else from step 0; either way its result is the
uninterrupted solve's, bit for bit.

How an epoch shares the device is the policy:
  lockstep  every active solve advances `epoch_steps` steps;
  srpt      (the default) shortest remaining work first: the solves with the least remaining
            work (points x steps left / the device rate of their precision)
            take an epoch's time budget (`epoch_ms`) in that order, each up to
            the steps one tile of it runs in that time; the largest may get
            none in an epoch.  This cuts the waiting of small solves behind
            large ones at the same device throughput.  Solves that got no steps
            for `max_wait_epochs` epochs in a row go first (the longest waiting
            first, each with at least a minimal share), so a large request keeps
            advancing even when a flow of small ones could fill every epoch.

The device work is in libpd; this module is the host-side scheduler.  The
executor interface (footprint / reserve / admit / collect / epoch_each / release /
abandon / checkpoint, and
idle_bytes: the memory of kept handles) has a GPU implementation over the C ABI
and a CPU fake with a cost model, used to test the scheduling without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np


@dataclasses.dataclass
class Request:
    name: str
    arrival_s: float
    grid: dict
    field: dict
    n_steps: int
    precision: str = "fp32"
    scheme: str = "strang"
    valley: str = "both"
    # seconds after arrival: the result is wanted by deadline_s (past it the request
    # expires, unserved or part-way through); the client withdraws it at cancel_s
    deadline_s: float = float("inf")
    cancel_s: float = float("inf")
    # filled by the server
    admitted_s: float = float("nan")
    done_s: float = float("nan")
    rho: float = float("nan")
    bytes: int = 0
    status: str = "pending"
    reason: str = ""
    retries: int = 0  # failed epochs survived
    # the last checkpoint: (state bytes on the host, steps done), or None; a retry resumes
    # from it; resumed_from is the step the last admission started at
    checkpoint: tuple = None
    checkpoint_s: float = float("-inf")
    resumed_from: int = 0

    @property
    def points(self) -> int:
        return int(self.grid["nx"]) * int(self.grid["ny"])

    @property
    def point_steps(self) -> float:
        return float(self.points) * float(self.n_steps)

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s

    @classmethod
    def from_workload(cls, w: dict) -> "Request":
        return cls(name=w["name"], arrival_s=float(w.get("arrival_s", 0.0)), grid=w["grid"], field=w["field"],
                   n_steps=int(w["n_steps"]), precision=w.get("precision", "fp32"), scheme=w.get("scheme", "strang"),
                   valley=w.get("valley", "both"))


class IdlePool:
    """Finished solves' handles kept for reuse by shape, oldest first, with their device
    bytes.  `close` is called on a handle that is evicted."""

    def __init__(self, per_shape: int, close):
        self.per_shape = int(per_shape)
        self.close = close
        self.entries = collections.OrderedDict()  # serial -> (shape key, handle, bytes)
        self.bytes = 0
        self._serial = 0

    def take(self, key):
        for i, (k, h, b) in self.entries.items():
            if k == key:
                del self.entries[i]
                self.bytes -= b
                return h
        return None

    def put(self, key, handle, nbytes: int) -> bool:
        """Keep the handle unless its shape already has per_shape kept; False: not kept."""
        if sum(k == key for k, _, _ in self.entries.values()) >= self.per_shape:
            return False
        self._serial += 1
        self.entries[self._serial] = (key, handle, int(nbytes))
        self.bytes += int(nbytes)
        return True

    def reserve(self, key, spare: int):
        """Evict until the kept handles hold at most `spare` bytes beyond the one a request
        of shape `key` will reuse (the oldest of that shape, which take() returns).  Other
        shapes go first, oldest first; then that shape's newer handles, newest first."""
        credit = next((b for k, _, b in self.entries.values() if k == key), 0)
        limit = spare + credit
        others = [i for i, (k, _, _) in self.entries.items() if k != key]
        same = [i for i, (k, _, _) in self.entries.items() if k == key][1:]
        for i in others + same[::-1]:
            if self.bytes <= limit:
                return
            _, h, b = self.entries.pop(i)
            self.bytes -= b
            self.close(h)

    def clear(self):
        for _, h, _ in self.entries.values():
            self.close(h)
        self.entries.clear()
        self.bytes = 0


def shape_key(req: "Request"):
    """Requests of one key can reuse each other's handles (grid, precision, scheme, valley)."""
    g = req.grid
    return (int(g["nx"]), int(g["ny"]), tuple(map(float, g["px"])), tuple(map(float, g["py"])), req.precision,
            req.scheme, req.valley)


class GpuExecutor:
    """Active solves as pd_grid handles in one pd_batch."""

    def __init__(self, pd, stream=None, points_per_lane: int = 0, block_threads: int = 0, keep_n: bool = False,
                 idle_per_shape: int = 8, background_setup: bool = True):
        """Every scheme, precision, field and valley is served; second-order Strang requests
        with fields along x share the batch's persistent kernel (see pd_batch).

        A finished solve's handle is kept (at most `idle_per_shape` per grid, precision,
        scheme and valley) and set up again for a later request of the same shape: that
        request then allocates nothing, and the finished one frees nothing (freeing device
        memory waits for the whole device).  Kept handles count against the server's
        memory budget and are closed when admitted work needs the room.

        With background_setup, an admitted request's set-up (pd_set_field: field sampling,
        tables, their upload) runs on a host thread of its own while the device runs
        epochs, and the request joins the batch at the first epoch boundary after it
        (collect); the handle is in no batch meanwhile."""
        import concurrent.futures

        self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=1) if background_setup else None
        self.setting_up = collections.OrderedDict()  # request name -> (Solver, shape key, n_steps, future)
        self.joined = []  # names joined to the batch since the last collect()
        self.pd = pd
        self.stream = stream
        self.batch = pd.Batch()
        if points_per_lane or block_threads:
            self.batch.set_launch(points_per_lane, block_threads)
        self.solvers = {}   # request name -> Solver
        self.order = []     # request names in batch member order
        self.left = {}      # request name -> steps still to run
        self.keys = {}      # request name -> shape key
        self.idle = IdlePool(idle_per_shape, lambda h: h.close())
        self.reused = 0
        self.keep_n = keep_n
        self.n_results = {}

    @property
    def idle_bytes(self) -> int:
        return self.idle.bytes

    def reserve(self, req: Request, spare: int):
        """Close kept handles so that, with req admitted, they hold at most `spare` bytes."""
        self.idle.reserve(shape_key(req), spare)

    def footprint(self, req: Request) -> int:
        s = self.pd.Solver.for_grid(req.grid, req.precision, req.scheme, req.valley)
        try:
            return s.solve_bytes(req.n_steps)
        finally:
            s.close()

    def admit(self, req: Request, background: bool = True):
        """Set the request up and join it to the batch; with background_setup and
        background, start the set-up in the background instead (the request is ready once
        collect() reports it).  A set-up on the calling thread raises PDError if the
        library refuses the request (e.g. the step-size condition)."""
        key = shape_key(req)
        s = self.idle.take(key)
        if s is None:
            s = self.pd.Solver.for_grid(req.grid, req.precision, req.scheme, req.valley)
        else:
            self.reused += 1
        left = req.n_steps - (req.checkpoint[1] if req.checkpoint else 0)
        if self._pool is not None and background:
            self.setting_up[req.name] = (s, key, left, self._pool.submit(self._set_up, s, req))
            return
        try:
            self._set_up(s, req)
        except Exception:
            s.close()
            raise
        self._join(req.name, s, key, left)

    def _set_up(self, s, req: Request):
        """The field; then, for a request that resumes, its checkpointed state (pd_load_state)."""
        s.set_field(req.field, req.n_steps)
        if req.checkpoint:
            s.load_state(req.checkpoint[0], req.checkpoint[1], self.stream)

    def _join(self, name, s, key, left):
        self.solvers[name] = s
        self.keys[name] = key
        self.order.append(name)
        self.left[name] = left
        self.batch.add(s)
        self.joined.append(name)

    def checkpoint(self, name: str):
        """(state bytes on the host, steps done) of an active solve part-way through, or None
        (pd_save_state: waits for the solve's enqueued epochs)."""
        s = self.solvers.get(name)
        if s is None or not 0 < s.n_steps - self.left[name] < s.n_steps:
            return None
        return s.save_state(self.stream)

    def collect(self, block: bool = False):
        """Requests whose set-up has finished since the last call, joined to the batch in
        admission order: (ready names, [(name, exception)] of set-ups the library refused,
        whose handles are closed).  block: wait for the oldest set-up in flight first."""
        failed = []
        if block and self.setting_up:
            next(iter(self.setting_up.values()))[3].exception()  # waits; errors are read below
        for name, (s, key, n_steps, fut) in list(self.setting_up.items()):
            if not fut.done():
                break  # later ones join after it, keeping admission order
            del self.setting_up[name]
            err = fut.exception()
            if err is not None:
                s.close()
                failed.append((name, err))
            else:
                self._join(name, s, key, n_steps)
        ready = list(self.joined)
        self.joined.clear()
        return ready, failed

    def epoch(self, steps: int):
        """Advance every active solve by up to `steps` steps (see epoch_each)."""
        return self.epoch_each({name: steps for name in self.order})

    def epoch_each(self, steps: dict):
        """Advance each active solve by up to steps[name] steps (absent: 0); returns
        [(name, rho)] of the solves that completed.  Which solves complete is known on
        the host, so the call only waits for the device in epochs where one does;
        otherwise the next epoch is enqueued behind this one."""
        lim = [min(self.left[name], max(0, int(steps.get(name, 0)))) for name in self.order]
        completing = any(m > 0 and m == self.left[name] for name, m in zip(self.order, lim))
        rho, fin = self.batch.step_each(lim, stream=self.stream, want_rho=completing)
        done = []
        for i, name in enumerate(self.order):
            self.left[name] -= lim[i]
            if completing and lim[i] > 0 and self.left[name] == 0:
                done.append((name, float(rho[i])))
        return done

    def abandon(self, name: str, keep: bool = True):
        """Drop an admitted request that will not complete (cancelled, expired, or failed): a
        set-up still in flight is waited for; the handle leaves the batch and, with keep, is
        kept for a later request of its shape (set up again from step 0), else closed."""
        if name in self.setting_up:
            s, key, n_steps, fut = self.setting_up.pop(name)
            if fut.exception() is not None:
                s.close()
                return
        else:
            s = self.solvers.pop(name)
            key = self.keys.pop(name)
            self.order.remove(name)
            del self.left[name]
            if name in self.joined:
                self.joined.remove(name)
            self.batch.remove(s)
        if not (keep and self.idle.put(key, s, int(s.info()["device_bytes"]))):
            s.close()

    def release(self, name: str):
        s = self.solvers.pop(name)
        if self.keep_n:
            n = np.empty(s.nx * s.ny)
            s.density(n_out=n, stream=self.stream)
            self.n_results[name] = n
        self.order.remove(name)
        del self.left[name]
        key = self.keys.pop(name)
        self.batch.remove(s)  # leave the batch before the grid is kept or destroyed
        if not self.idle.put(key, s, int(s.info()["device_bytes"])):
            s.close()

    def close(self):
        if self._pool is not None:
            self._pool.shutdown(wait=True)
        for s, _, _, _ in self.setting_up.values():
            s.close()
        self.setting_up.clear()
        self.batch.close()
        for s in self.solvers.values():
            s.close()
        self.idle.clear()
        self.solvers = {}
        self.order = []


class FakeExecutor:
    """CPU stand-in with the same interface: an epoch costs its point-steps / rate seconds
    of device time, or, if longer, the steps of its longest share times tile_step_s (the
    time one tile takes per step, which bounds how fast a small solve can go), plus
    epoch_overhead_s; rho is a fixed function of the request."""

    def __init__(self, rate_point_steps_per_s: float = 1e12, bytes_per_point: int = 40, tile_step_s: float = 0.0,
                 epoch_overhead_s: float = 0.0, idle_per_shape: int = 0, setup_epochs: int = 0, refuse=None,
                 fail_epochs=()):
        """setup_epochs > 0 models background set-up: an admitted request becomes ready
        (collect) only after that many epochs have run; refuse(request) -> True makes its
        set-up fail; the epoch_each calls numbered in fail_epochs (from 1) raise, as a
        failed launch would, advancing nothing."""
        self.rate = rate_point_steps_per_s
        self.bytes_per_point = bytes_per_point
        self.tile_step_s = tile_step_s
        self.epoch_overhead_s = epoch_overhead_s
        self.active = collections.OrderedDict()  # name -> [request, steps_done]
        self.clock = 0.0                          # simulated device time
        self.idle = IdlePool(idle_per_shape, lambda h: None)  # kept "handles": the finished requests
        self.reused = 0
        self.joined = []
        self.setup_epochs = int(setup_epochs)
        self.refuse = refuse
        self.setting_up = collections.OrderedDict()  # name -> (request, epochs left)
        self.epochs_run = 0
        self.fail_epochs = set(fail_epochs)
        self.epoch_calls = 0

    @property
    def idle_bytes(self) -> int:
        return self.idle.bytes

    def reserve(self, req: Request, spare: int):
        self.idle.reserve(shape_key(req), spare)

    def footprint(self, req: Request) -> int:
        return req.points * self.bytes_per_point + 16 * req.n_steps

    def admit(self, req: Request, background: bool = True):
        if self.idle.take(shape_key(req)) is not None:
            self.reused += 1
        if self.setup_epochs > 0 or self.refuse is not None:
            self.setting_up[req.name] = (req, self.setup_epochs)
            return
        self.active[req.name] = [req, req.checkpoint[1] if req.checkpoint else 0]
        self.joined.append(req.name)

    def checkpoint(self, name: str):
        entry = self.active.get(name)
        if entry is None or not 0 < entry[1] < entry[0].n_steps:
            return None
        return (None, entry[1])

    def collect(self, block: bool = False):
        """Requests whose (modelled) set-up has finished, in admission order; block: the
        oldest set-up in flight finishes now (the host waits for it)."""
        failed = []
        for name, (req, left) in list(self.setting_up.items()):
            if left > 0 and not (block and not self.joined and not failed):
                break
            block = False
            del self.setting_up[name]
            if self.refuse is not None and self.refuse(req):
                failed.append((name, RuntimeError("set-up refused")))
            else:
                self.active[name] = [req, req.checkpoint[1] if req.checkpoint else 0]
                self.joined.append(name)
        ready = list(self.joined)
        self.joined.clear()
        return ready, failed

    def epoch(self, steps: int):
        return self.epoch_each({name: steps for name in self.active})

    def epoch_each(self, steps: dict):
        self.epoch_calls += 1
        if self.epoch_calls in self.fail_epochs:
            raise RuntimeError("injected epoch failure")
        work = 0.0
        longest = 0
        done = []
        for name, entry in self.active.items():
            req, k = entry
            m = min(max(0, int(steps.get(name, 0))), req.n_steps - k)
            work += float(req.points) * m
            longest = max(longest, m)
            entry[1] = k + m
            if entry[1] == req.n_steps and m > 0:
                done.append((name, 1e-3 * req.points / (1.0 + req.n_steps)))
        self.clock += max(work / self.rate, longest * self.tile_step_s) + self.epoch_overhead_s
        self.epochs_run += 1
        for name, (req, left) in self.setting_up.items():
            self.setting_up[name] = (req, max(0, left - 1))
        return done

    def release(self, name: str):
        req = self.active.pop(name)[0]
        self.idle.put(shape_key(req), req, self.footprint(req))

    def abandon(self, name: str, keep: bool = True):
        if name in self.setting_up:
            req = self.setting_up.pop(name)[0]
        else:
            req = self.active.pop(name)[0]
            if name in self.joined:
                self.joined.remove(name)
        if keep:
            self.idle.put(shape_key(req), req, self.footprint(req))

    def close(self):
        self.idle.clear()


@dataclasses.dataclass
class ServeStats:
    completed: int
    rejected: int
    makespan_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    point_steps_per_s: float
    epochs: int
    mean_active: float
    peak_bytes: int
    budget_bytes: int
    cancelled: int = 0
    expired: int = 0
    failed: int = 0
    retried: int = 0      # solves queued again after a failed epoch
    checkpoints: int = 0  # states copied to host memory

    def as_dict(self) -> dict:
        return dataclasses.asdict(self)


# Device rates (point-steps/s) the srpt policy prices work with, and the time one
# 1024-point tile of a small member takes per step while the members that fill the
# device run their own launches beside it (MI355X measurements, Strang; 0.09-0.11 us
# with the device to itself).  It caps the steps a solve gets in one epoch.
DEFAULT_RATES = {"fp32": 5.0e12, "fp32fast": 6.5e12, "fp64": 3.4e12}
DEFAULT_TILE_STEP_S = 0.15e-6


class Server:
    def __init__(self, executor, budget_bytes: int, epoch_steps: int = 2048, max_active: int = 4096,
                 backfill: bool = False, policy: str = "srpt", epoch_ms: float = 3.0, rates: dict = None,
                 tile_step_s: float = DEFAULT_TILE_STEP_S, max_wait_epochs: int = 32, admit_per_epoch: int = 4,
                 defer_admissions: bool = True, max_retries: int = 0, checkpoint_every_s: float = None):
        if epoch_steps < 1:
            raise ValueError("epoch_steps must be >= 1")
        if policy not in ("lockstep", "srpt"):
            raise ValueError("policy must be 'lockstep' or 'srpt'")
        if not (epoch_ms > 0 and tile_step_s > 0):
            raise ValueError("epoch_ms and tile_step_s must be > 0")
        if max_wait_epochs < 1:
            raise ValueError("max_wait_epochs must be >= 1")
        if admit_per_epoch < 1:
            raise ValueError("admit_per_epoch must be >= 1")
        if max_retries < 0 or (checkpoint_every_s is not None and not checkpoint_every_s >= 0):
            raise ValueError("max_retries and checkpoint_every_s must be >= 0")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.epoch_steps = int(epoch_steps)
        self.max_active = int(max_active)
        self.backfill = backfill
        self.policy = policy
        self.epoch_s = epoch_ms * 1e-3
        self.rates = dict(DEFAULT_RATES, **(rates or {}))
        self.tile_step_s = tile_step_s
        self.max_wait = int(max_wait_epochs)
        self.admit_per_epoch = int(admit_per_epoch)
        # after an epoch in which requests finished the host has waited for the device, which
        # is then idle: enqueue the next epoch of the remaining solves before setting up new
        # admissions, so that their set-up (field sampling, table upload) overlaps it
        self.defer_admissions = bool(defer_admissions)
        # recovery: a solve in a failed epoch is queued again up to max_retries times, from
        # its last checkpoint (taken at most every checkpoint_every_s seconds; None: never)
        self.max_retries = int(max_retries)
        self.checkpoint_every_s = checkpoint_every_s
        self.retried = 0
        self.checkpoints = 0
        self.waited = {}  # request name -> epochs in a row without steps (srpt)
        self.in_use = 0
        self.peak = 0
        self.active = {}
        self.left = {}  # request name -> steps still to run
        self.ready = set()  # admitted requests whose set-up has finished (members of the batch)
        self._cancel = set()  # names withdrawn by cancel(), from any thread
        self._cancel_lock = threading.Lock()

    def cancel(self, name: str):
        """Withdraw a request (waiting or active) from another thread while run() serves;
        it leaves at the next epoch boundary with status "cancelled"."""
        with self._cancel_lock:
            self._cancel.add(name)

    def _withdrawn(self, r: "Request", now: float):
        with self._cancel_lock:
            if r.name in self._cancel:
                return "cancelled", "cancelled by the client"
        if now >= r.arrival_s + r.cancel_s:
            return "cancelled", "cancelled by the client at %.3f s" % (r.arrival_s + r.cancel_s)
        if now > r.arrival_s + r.deadline_s:
            return "expired", "deadline %.3f s after arrival passed" % r.deadline_s
        return None

    def _retire(self, r: "Request", status: str, reason: str, now: float, keep: bool = True):
        """An admitted request that will not complete leaves the batch; its memory goes back
        to the budget (keep: its handle is kept for reuse, else closed)."""
        name = r.name
        del self.left[name]
        self.ready.discard(name)
        self.waited.pop(name, None)
        self.active.pop(name)
        self.in_use -= r.bytes
        self.ex.abandon(name, keep=keep)
        r.status, r.reason, r.done_s = status, reason, now
        if status != "failed":  # a failed solve may still resume from its checkpoint
            r.checkpoint = None

    def plan_epoch(self) -> dict:
        """Steps each ready solve advances in the next epoch (absent: none)."""
        if self.policy == "lockstep":
            return {name: min(self.epoch_steps, left) for name, left in self.left.items() if name in self.ready}
        budget = self.epoch_s
        share = max(self.epoch_steps, int(self.epoch_s / self.tile_step_s))  # steps a tile runs in an epoch
        rate = {name: self.rates.get(r.precision, self.rates["fp32"]) for name, r in self.active.items()}
        # solves that waited max_wait epochs in a row first, the longest waiting first;
        # then the least remaining work first
        def key(n):
            w = self.waited.get(n, 0)
            return (0, -w, n) if w >= self.max_wait else (1, self.active[n].points * self.left[n] / rate[n], n)

        order = sorted((n for n in self.left if n in self.ready), key=key)
        if not order:
            return {}
        plan = {}
        for name in order:
            pts = self.active[name].points
            m = min(self.left[name], share)
            if pts * m / rate[name] > budget:
                m = int(budget * rate[name] / pts)
                floor = min(self.left[name], self.epoch_steps // 8 or 1)
                if m < floor:
                    if self.waited.get(name, 0) < self.max_wait:
                        continue  # too little of the budget left for a useful share of this solve
                    m = floor  # a solve that waited long advances, past the budget if need be
            plan[name] = m
            budget -= pts * m / rate[name]
            if budget <= 0:
                break
        if not plan:  # a single solve larger than the whole budget still advances
            name = order[0]
            plan[name] = min(self.left[name], self.epoch_steps)
        return plan

    def _now(self, t0, simulated):
        return self.ex.clock if simulated else time.perf_counter() - t0

    def run(self, requests, simulated: bool = False, progress=None, progress_every: int = 1000) -> ServeStats:
        """Serve the requests (arrival times in seconds from the start).  With
        simulated=True the clock is the executor's device-time model (FakeExecutor).
        progress(completed, total, now_s), if given, is called after every
        progress_every completions."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        finished = 0
        idle_after_finish = False  # the last epoch finished requests (the host waited for it)
        pending = collections.deque(reqs)
        waiting = collections.deque()  # arrived, not yet admitted
        t0 = time.perf_counter()
        epochs = 0
        active_sum = 0
        while pending or waiting or self.active:
            now = self._now(t0, simulated)
            while pending and pending[0].arrival_s <= now:
                r = pending.popleft()
                w = self._withdrawn(r, now)
                if w is not None:
                    r.status, r.reason = w
                    r.done_s = now
                    continue
                r.bytes = self.ex.footprint(r)
                if r.bytes > self.budget:
                    r.status, r.reason = "rejected", "footprint %d bytes exceeds the budget %d" % (r.bytes, self.budget)
                    r.done_s = now
                    continue
                waiting.append(r)
            # cancelled and expired requests leave the queue, or the batch at this epoch
            # boundary (their memory goes back to the budget, the handle is kept for reuse)
            for r in list(waiting):
                w = self._withdrawn(r, now)
                if w is not None:
                    waiting.remove(r)
                    r.status, r.reason = w
                    r.done_s = now
                    r.checkpoint = None  # a retried request's host copy goes with it
            for name in list(self.active):
                r = self.active[name]
                w = self._withdrawn(r, now)
                if w is not None:
                    self._retire(r, w[0], w[1], now)
            # admit in arrival order while memory and slots allow (optionally skipping a blocked
            # head), at most admit_per_epoch before the next epoch: the device then runs that
            # epoch (enqueued without waiting) while the host sets up the next arrivals.  Right
            # after a finishing epoch the device is idle: then the next epoch goes first.
            blocked = []
            admitted = 0
            hold = self.defer_admissions and idle_after_finish and self.active
            while (not hold and waiting and len(self.active) < self.max_active
                   and admitted < self.admit_per_epoch):
                r = waiting[0]
                if self.in_use + r.bytes <= self.budget:
                    waiting.popleft()
                    self.ex.reserve(r, self.budget - self.in_use - r.bytes)  # kept handles give way
                    try:
                        # a lone admission is set up at once (its latency counts); several, as in a
                        # burst, in the background while the device runs epochs (throughput counts)
                        self.ex.admit(r, background=admitted > 0 or len(waiting) > 0)
                    except Exception as e:  # refused by the solver: reported, not retried
                        r.status, r.reason, r.done_s = "rejected", str(e), now
                        continue
                    r.admitted_s, r.status = now, "active"
                    admitted += 1
                    self.active[r.name] = r
                    r.resumed_from = r.checkpoint[1] if r.checkpoint else 0
                    self.left[r.name] = r.n_steps - r.resumed_from
                    self.in_use += r.bytes
                    self.peak = max(self.peak, self.in_use + self.ex.idle_bytes)
                elif self.backfill:
                    blocked.append(waiting.popleft())
                else:
                    break
            for r in reversed(blocked):
                waiting.appendleft(r)
            # requests whose set-up finished join the next epoch; with none ready, wait for one
            ready, failed = self.ex.collect(block=bool(self.active) and not self.ready)
            self.ready.update(ready)
            for name, err in failed:  # refused by the solver during set-up: reported, not retried
                r = self.active.pop(name)
                del self.left[name]
                self.in_use -= r.bytes
                r.status, r.reason, r.done_s = "rejected", str(err), self._now(t0, simulated)
            if self.active and not self.ready:
                continue
            if not self.active:
                if pending:
                    if simulated:
                        self.ex.clock = max(self.ex.clock, pending[0].arrival_s)
                    else:
                        time.sleep(max(0.0, min(pending[0].arrival_s - (time.perf_counter() - t0), 0.05)))
                    continue
                if waiting:
                    raise RuntimeError("a waiting request can never be admitted")
                break
            plan = self.plan_epoch()
            try:
                done = self.ex.epoch_each(plan)
            except Exception as e:  # the epoch's launch failed and advanced nothing
                # its planned members lose their handles (after a real device fault their
                # state cannot be trusted); those with retries left are queued again ahead
                # of later arrivals, to resume from their last checkpoint; the others fail
                now = self._now(t0, simulated)
                again = []
                for name in plan:
                    r = self.active[name]
                    self._retire(r, "failed", "epoch failed: %s" % e, now, keep=False)
                    if r.retries < self.max_retries:
                        r.retries += 1
                        r.status, r.done_s = "waiting", float("nan")
                        again.append(r)
                        self.retried += 1
                    else:
                        r.checkpoint = None
                for r in reversed(again):
                    waiting.appendleft(r)
                epochs += 1
                continue
            for name in self.ready:
                self.waited[name] = 0 if plan.get(name, 0) > 0 else self.waited.get(name, 0) + 1
            for name, m in plan.items():
                self.left[name] -= m
            epochs += 1
            active_sum += len(self.active)
            now = self._now(t0, simulated)
            idle_after_finish = bool(done)
            if self.checkpoint_every_s is not None:
                finishing = {name for name, _ in done}
                for name, m in plan.items():
                    r = self.active[name]
                    if m > 0 and name not in finishing and now - r.checkpoint_s >= self.checkpoint_every_s:
                        ck = self.ex.checkpoint(name)
                        if ck is not None:
                            r.checkpoint, r.checkpoint_s = ck, now
                            self.checkpoints += 1
            for name, rho in done:
                del self.left[name]
                self.ready.discard(name)
                self.waited.pop(name, None)
                r = self.active.pop(name)
                r.rho, r.done_s, r.status = rho, now, "done"
                r.checkpoint = None
                self.in_use -= r.bytes
                self.ex.release(name)
                finished += 1
                if progress is not None and finished % progress_every == 0:
                    progress(finished, len(reqs), now)
        end = self._now(t0, simulated)
        done = [r for r in reqs if r.status == "done"]
        lat = np.array([r.latency_s for r in done]) * 1e3 if done else np.zeros(1)
        first = min((r.arrival_s for r in reqs), default=0.0)
        makespan = max(end - first, 1e-12)
        return ServeStats(completed=len(done), rejected=sum(r.status == "rejected" for r in reqs),
                          cancelled=sum(r.status == "cancelled" for r in reqs),
                          expired=sum(r.status == "expired" for r in reqs),
                          failed=sum(r.status == "failed" for r in reqs), retried=self.retried,
                          checkpoints=self.checkpoints,
                          makespan_s=makespan, p50_ms=float(np.percentile(lat, 50)),
                          p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                          point_steps_per_s=sum(r.point_steps for r in done) / makespan, epochs=epochs,
                          mean_active=active_sum / max(epochs, 1), peak_bytes=self.peak, budget_bytes=self.budget)


def tune_epoch_ms(make_executor, budget_bytes: int, requests, candidates=(1.5, 3.0, 6.0), repeats: int = 2,
                  simulated: bool = False, cache_path: str = None, cache_key: str = None, tolerance: float = 0.02,
                  **server_kw):
    """The srpt epoch length (epoch_ms) from timed candidates.  The same closed set of
    requests (arrival times ignored: all present at t = 0) is served once per candidate and
    repetition, the repetitions interleaved, each on a fresh executor from make_executor().
    The shortest candidate whose median makespan is within `tolerance` of the shortest
    median is kept: a longer epoch runs a small request's steps in fewer, later epochs, so
    it is taken only for capacity it really adds.  The epoch length changes no result bit
    (each solve's steps are the same arithmetic however they are grouped into epochs), only
    how the device is shared.

    With cache_path and cache_key, a value stored for the key is returned without timing,
    and a newly chosen one is appended (lines "key<TAB>epoch_ms").  Returns (epoch_ms,
    {candidate: [makespans]}) -- the dict is empty when the value came from the cache."""
    if cache_path and cache_key:
        try:
            with open(cache_path) as fh:
                hits = [ln.rstrip("\n").split("\t") for ln in fh if ln.startswith(cache_key + "\t")]
            if hits:
                return float(hits[-1][1]), {}
        except OSError:
            pass
    cands = [float(c) for c in candidates]
    if not cands or any(not c > 0 for c in cands) or repeats < 1 or not tolerance >= 0:
        raise ValueError("candidates must be positive epoch lengths, repeats >= 1 and tolerance >= 0")
    spans = {c: [] for c in cands}
    for _ in range(repeats):
        for c in cands:
            reqs = [Request(r.name, 0.0, r.grid, r.field, r.n_steps, r.precision, r.scheme, r.valley)
                    for r in requests]
            ex = make_executor()
            try:
                st = Server(ex, budget_bytes, epoch_ms=c, **server_kw).run(reqs, simulated=simulated)
            finally:
                ex.close()
            if st.completed != len(reqs):
                raise RuntimeError("epoch tuning: %d of %d requests completed" % (st.completed, len(reqs)))
            spans[c].append(st.makespan_s)
    fastest = min(float(np.median(spans[c])) for c in cands)
    best = min(c for c in cands if float(np.median(spans[c])) <= fastest * (1.0 + tolerance))
    if cache_path and cache_key:
        with open(cache_path, "a") as fh:
            fh.write("%s\t%r\n" % (cache_key, best))
    return best, spans

