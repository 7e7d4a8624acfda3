"""Host threads on one GPU: the library's entry points run from several threads at once,
each thread with its own handles and stream (the ctypes calls release the interpreter
lock, so the calls overlap in the library).  Every result is bit-identical to the same
solve run alone, and the FP64 ones match the oracle (Sec. II Eq. (1); Sec. III)."""
import threading

import numpy as np
import pytest

import oracle
from paper_1607_03062_amd import workloads as wl

pytestmark = pytest.mark.gpu

FIELD = wl.sin2(0.2, 0.6, 3)
JOBS = [  # (grid size, precision, scheme, steps, how)
    (96, "fp64", "strang", 2100, "whole"),
    (128, "fp32", "strang", 3000, "chunked"),
    (80, "fp64", "midpoint", 1700, "checkpoint"),
    (160, "fp32fast", "strang", 2500, "autotune"),
    (64, "fp32", "strang4", 900, "whole"),
    (112, "fp32", "midpoint4", 800, "chunked"),
    (144, "fp64", "strang", 1500, "autotune"),
]


def solve(gpu, size, precision, scheme, N, how, stream=None):
    grid = wl.grid(size, 2.0)
    s = gpu.Solver.for_grid(grid, precision, scheme)
    s.set_field(FIELD, N)
    if how == "autotune":
        s.autotune(trial_steps=256, use_cache=True, stream=stream)
        s.rewind()
    if how == "chunked":
        for c in (N // 3, 1, N // 3):
            s.propagate(c, stream=stream)
    elif how == "checkpoint":
        s.propagate(N // 2, stream=stream)
        state, done = s.save_state(stream)
        s.close()
        s = gpu.Solver.for_grid(grid, precision, scheme)
        s.set_field(FIELD, N)
        s.load_state(state, done, stream)
    s.propagate(-1, stream=stream)
    n = np.empty(size * size)
    rho = s.density(n_out=n, stream=stream)  # waits for the copy to the host
    s.close()
    return n, rho


def test_concurrent_solves_from_host_threads(gpu, tmp_path, monkeypatch):
    """Seven threads, seven streams: whole, chunked, checkpointed (save, new handle, load)
    and autotuned solves of every scheme and precision at once, and a batch of three more
    solves from an eighth thread; three rounds.  Each result equals its solve alone bit
    for bit (launch shapes do not change results, so the autotuned ones are compared with
    a solve at the default shape); the autotune cache, empty in the first round, gets its
    two entries from concurrent stores as whole lines."""
    import torch

    cache = tmp_path / "autotune.txt"
    monkeypatch.setenv("PD_AUTOTUNE_CACHE", str(cache))
    alone = [solve(gpu, *job[:4], "whole" if job[4] == "autotune" else job[4]) for job in JOBS]
    for (size, precision, scheme, N, how), (n, rho) in zip(JOBS, alone):
        if precision == "fp64":
            n_o = oracle.solve_grid(FIELD, wl.grid(size, 2.0), N, scheme)[0]
            assert np.max(np.abs(n - n_o)) <= 1e-12, (size, scheme)
    batch_specs = [(64, 1200), (96, 1500), (72, 900)]
    batch_alone = [solve(gpu, size, "fp32", "strang", N, "whole")[1] for size, N in batch_specs]

    def batch_job(out):
        st = torch.cuda.Stream()
        members = [gpu.Solver.for_grid(wl.grid(size, 2.0), "fp32").set_field(FIELD, N) for size, N in batch_specs]
        b = gpu.Batch(members)
        out["batch"] = [float(r) for r in b.run(stream=st)]
        st.synchronize()
        b.close()
        for m in members:
            m.close()

    for rnd in range(3):
        print("threads round %d" % rnd, flush=True)
        results, errors = {}, []

        def work(i):
            try:
                st = torch.cuda.Stream()
                results[i] = solve(gpu, *JOBS[i], stream=st)
                st.synchronize()
            except Exception as e:  # reported below with the job
                errors.append((i, repr(e)))

        def bwork():
            try:
                batch_job(results)
            except Exception as e:
                errors.append(("batch", repr(e)))

        threads = [threading.Thread(target=work, args=(i,)) for i in range(len(JOBS))]
        threads.append(threading.Thread(target=bwork))
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=120)
        assert not any(t.is_alive() for t in threads), "a thread did not finish"
        assert not errors, errors
        for i, job in enumerate(JOBS):
            n, rho = results[i]
            assert np.array_equal(n, alone[i][0]) and rho == alone[i][1], job
        assert results["batch"] == batch_alone
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and all(len(ln.split("\t")) == 2 and len(ln.split("\t")[1].split()) == 5 for ln in lines), lines
