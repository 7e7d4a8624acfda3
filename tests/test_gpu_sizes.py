"""GPU parity at the largest grids the library accepts (nx, ny up to 65536).

A dispatch packet holds a grid's size in work-items in 32 bits, so a full
65536 x 65536 grid (2^32 points) at one point per lane runs as two launches of
2^31 lanes each (the snapshot kernel's too).  The tests check the points on both
sides of that split, the first and the last point and whole rows against the
oracle, the masked point p = 0 and the p_y = 0 row (exactly 0 under a field along
x), and rho against its definition, 4 dx dy / (2 pi)^2 times the sum of n, with
the sum taken by torch over the device output.  A batch with such a member runs
it as 4M work items of the persistent kernel.  The thin grids at the maximum
extent (65536 x 1, 1 x 65536) are compared point by point.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1607_03062_amd import workloads as wl

from .test_gpu_parity import FP32_N_ABS, FP64_N_ABS, FP64_RHO_REL

pytestmark = pytest.mark.gpu

NMAX = 65536
FIELD = wl.sin2(0.1, 0.5, 8)
N_STEPS = 256
SPLIT = 1 << 31


def _sample():
    rng = np.random.default_rng(20260)
    fixed = [0, 1, NMAX - 1, NMAX, SPLIT - 257, SPLIT - 256, SPLIT - 1, SPLIT, SPLIT + 1, SPLIT + 255,
             SPLIT + 256, SPLIT + NMAX // 2, NMAX * NMAX - NMAX, NMAX * NMAX - 2, NMAX * NMAX - 1]
    return np.unique(np.concatenate([np.array(fixed, dtype=np.int64),
                                     rng.integers(0, NMAX * NMAX, 240, dtype=np.int64)]))


@pytest.mark.parametrize("scheme,precision,ppl", [
    ("strang", "fp32", 1), ("strang", "fp32fast", 1), ("strang", "fp64", 0), ("strang", "fp64", 1),
    ("midpoint", "fp32", 1),
])
def test_full_maximum_grid(gpu, scheme, precision, ppl):
    import torch

    g = {"nx": NMAX, "ny": NMAX, "px": (-2.0, 2.0), "py": (-2.0, 2.0)}
    print("gpu solve: grid 65536x65536 N=%d %s %s ppl=%d" % (N_STEPS, scheme, precision, ppl), flush=True)
    out = torch.empty(NMAX * NMAX, dtype=torch.float64, device="cuda")
    s = gpu.Solver.for_grid(g, precision, scheme)
    try:
        s.set_launch(ppl, 0, 0, 0)
        s.set_field(FIELD, N_STEPS)
        s.propagate(-1)
        rho = s.density(n_out=out)
        info = s.info()
    finally:
        s.close()
    torch.cuda.synchronize()
    assert info["n_masked"] == 1
    tol = FP64_N_ABS if precision == "fp64" else FP32_N_ABS
    # sampled points, the split between launches among them
    idx = _sample()
    n_o = oracle.solve_grid(FIELD, g, N_STEPS, scheme, idx=idx)[0]
    got = out[torch.from_numpy(idx).cuda()].cpu().numpy()
    err = np.max(np.abs(got - n_o))
    print("65536^2 %s %s max |dn| on %d samples = %.3e" % (scheme, precision, idx.size, err), flush=True)
    assert err <= tol
    # the last row before the split and the first row after it (p_y = 0: exactly 0 under a field along x)
    row = np.arange(SPLIT - NMAX, SPLIT, dtype=np.int64)
    n_row = oracle.solve_grid(FIELD, g, N_STEPS, scheme, idx=row)[0]
    assert np.max(np.abs(out[SPLIT - NMAX:SPLIT].cpu().numpy() - n_row)) <= tol
    assert torch.all(out[SPLIT:SPLIT + NMAX] == 0.0).item()
    # p = 0 is the grid node (32768, 32768): masked
    assert out[SPLIT + NMAX // 2].item() == 0.0
    # rho against its definition over the whole device output
    dx = dy = 4.0 / NMAX
    rho_def = 4.0 * dx * dy / (4.0 * math.pi ** 2) * float(out.sum().item())
    print("65536^2 rho = %.15e, definition %.15e" % (rho, rho_def), flush=True)
    assert abs(rho / rho_def - 1) <= FP64_RHO_REL
    del out
    torch.cuda.empty_cache()


def test_snapshot_on_maximum_grid(gpu):
    """A snapshot after 100 of 256 steps on the 65536^2 grid reads the stored state
    (48 GiB in FP32) in two launches; sampled points on both sides of the split."""
    import torch

    g = {"nx": NMAX, "ny": NMAX, "px": (-2.0, 2.0), "py": (-2.0, 2.0)}
    print("gpu snapshot: grid 65536x65536 N=%d k=100 strang fp32" % N_STEPS, flush=True)
    out = torch.empty(NMAX * NMAX, dtype=torch.float64, device="cuda")
    s = gpu.Solver.for_grid(g, "fp32", "strang")
    try:
        s.set_field(FIELD, N_STEPS)
        s.propagate(100)
        s.snapshot(n_out=out)
    finally:
        s.close()
    torch.cuda.synchronize()
    idx = _sample()
    n_o = oracle.snapshot_grid(FIELD, g, N_STEPS, 100, "strang", idx=idx)[0]
    got = out[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.max(np.abs(got - n_o)) <= FP32_N_ABS
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("shape", [(NMAX, 1), (1, NMAX), (NMAX, 3)])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32fast"])
def test_thin_grids_at_maximum_extent(gpu, shape, precision):
    nx, ny = shape
    g = {"nx": nx, "ny": ny, "px": (-3.0, 2.5), "py": (-1.5, 1.0)}
    print("gpu solve: grid %dx%d N=%d strang %s" % (nx, ny, N_STEPS, precision), flush=True)
    s = gpu.Solver.for_grid(g, precision, "strang")
    try:
        s.set_field(FIELD, N_STEPS)
        s.propagate(-1)
        n = np.empty(nx * ny)
        rho = s.density(n_out=n)
    finally:
        s.close()
    n_o = oracle.solve_grid(FIELD, g, N_STEPS)[0]
    if precision == "fp64":
        assert np.max(np.abs(n - n_o)) <= FP64_N_ABS
        assert abs(rho / oracle.density(g, n_o) - 1) <= FP64_RHO_REL
    else:
        assert np.max(np.abs(n - n_o)) <= FP32_N_ABS


def test_batch_with_a_maximum_grid_member(gpu):
    """A batch holding a 65536^2 member (2^32 points: 4M work items of the persistent
    kernel) beside a 64^2 one: sampled points, the split rows and rho of the large member
    against the oracle and the definition; the small member equals its solve alone."""
    import torch

    g = {"nx": NMAX, "ny": NMAX, "px": (-2.0, 2.0), "py": (-2.0, 2.0)}
    print("gpu batch: 65536x65536 N=%d + 64x64, fp32" % N_STEPS, flush=True)
    big = gpu.Solver.for_grid(g, "fp32")
    small = gpu.Solver.for_grid(wl.grid(64, 2.0), "fp32")
    b = gpu.Batch()
    out = torch.empty(NMAX * NMAX, dtype=torch.float64, device="cuda")
    try:
        big.set_field(FIELD, N_STEPS)
        small.set_field(wl.sin2(0.15, 0.5, 8), 700)
        b.add(big)
        b.add(small)
        rho = b.run()
        rho_big = big.density(n_out=out)
        n_small = np.empty(64 * 64)
        rho_small = small.density(n_out=n_small)
    finally:
        b.close()
        big.close()
        small.close()
    torch.cuda.synchronize()
    assert rho[0] == rho_big and rho[1] == rho_small
    idx = _sample()
    n_o = oracle.solve_grid(FIELD, g, N_STEPS, "strang", idx=idx)[0]
    assert np.max(np.abs(out[torch.from_numpy(idx).cuda()].cpu().numpy() - n_o)) <= FP32_N_ABS
    assert torch.all(out[SPLIT:SPLIT + NMAX] == 0.0).item()
    rho_def = 4.0 * (4.0 / NMAX) ** 2 / (4.0 * math.pi ** 2) * float(out.sum().item())
    assert abs(rho_big / rho_def - 1) <= FP64_RHO_REL
    alone = gpu.Solver.for_grid(wl.grid(64, 2.0), "fp32")
    alone.set_field(wl.sin2(0.15, 0.5, 8), 700)
    alone.propagate(-1)
    n_alone = np.empty(64 * 64)
    rho_alone = alone.density(n_out=n_alone)
    alone.close()
    assert rho_small == rho_alone and np.array_equal(n_small, n_alone)
    del out
    torch.cuda.empty_cache()
