"""pd_density_static, the density entry point that allocates nothing (its reduction
scratch is a static device array of the library), against pd_density: two calls in a
row on one device, the second on a smaller grid, each bit for bit equal to pd_density
(same kernels, same fixed summation order), with n(p) to host and to device memory; and
inside a HIP graph the caller captures, with the solve before it."""
import numpy as np
import pytest

from paper_1607_03062_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_static_density_equals_density(gpu):
    import torch

    st = torch.cuda.Stream()
    grids = [wl.grid(1100, 2.0), wl.grid(37, 1.5)]  # 1.21M points (591 tiles), then 1369 (one ragged tile)
    for q, g in enumerate(grids):
        for prec in ("fp64", "fp32"):
            s = gpu.Solver.for_grid(g, prec)
            s.set_field(wl.sin2(0.1 + 0.05 * q, 0.5, 4), 600)
            s.propagate(-1, stream=st)
            n_ref = np.empty(g["nx"] * g["ny"])
            rho_ref = s.density(n_out=n_ref, stream=st)
            n_host = np.empty_like(n_ref)
            rho = s.density_static(n_out=n_host, stream=st)
            n_dev = torch.empty(n_ref.shape[0], dtype=torch.float64, device="cuda")
            rho_dev = s.density_static(n_out=n_dev, stream=st)
            st.synchronize()
            s.close()
            print("grid %d^2 %s: rho %.15e static %.15e" % (g["nx"], prec, rho_ref, rho), flush=True)
            assert rho == rho_ref and rho_dev == rho_ref, (q, prec)
            assert np.array_equal(n_host, n_ref) and np.array_equal(n_dev.cpu().numpy(), n_ref), (q, prec)


def test_static_density_errors(gpu):
    s = gpu.Solver.for_grid(wl.grid(64, 2.0), "fp32")
    with pytest.raises(gpu.PDError) as e:
        s.density_static()  # no field yet
    assert e.value.status == 2
    s.set_field(wl.sin2(0.1, 0.5, 4), 300)
    s.propagate(100)
    with pytest.raises(gpu.PDError) as e:
        s.density_static()  # before the last step
    assert e.value.status == 2
    s.propagate(-1)
    assert s.density_static() == s.density()
    s.close()


def test_solve_and_static_density_in_a_captured_graph(gpu):
    """A whole solve (pd_propagate) and pd_density_static with n(p) to device memory,
    captured by the caller into a HIP graph (torch.cuda.graph): the static density can be
    captured because it allocates nothing and clears nothing.  Five replays, each after
    eager solves of other grids on the device, each bit for bit equal to the eager
    pd_density result."""
    import torch

    g, field, N = wl.grid(96, 2.0), wl.sin2(0.15, 0.5, 4), 1500
    for prec in ("fp32fast", "fp64"):
        print("captured solve %s" % prec, flush=True)
        ref = gpu.Solver.for_grid(g, prec).set_field(field, N)
        ref.propagate(-1)
        n_ref = np.empty(g["nx"] * g["ny"])
        ref.density(n_out=n_ref)
        ref.close()
        # an eager call first: it looks up the static array's device address, which a
        # capture could not
        warm = gpu.Solver.for_grid(wl.grid(16, 1.0), prec).set_field(field, 200)
        warm.propagate(-1)
        warm.density_static()
        warm.close()
        s = gpu.Solver.for_grid(g, prec).set_field(field, N)
        n_dev = torch.zeros(g["nx"] * g["ny"], dtype=torch.float64, device="cuda")
        graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(graph, stream=cap, capture_error_mode="thread_local"):
            s.propagate(-1, stream=cap)
            s.density_static(n_out=n_dev, want_rho=False, stream=cap)
        torch.cuda.synchronize()
        for r in range(5):
            n_dev.zero_()
            graph.replay()
            torch.cuda.synchronize()
            assert np.array_equal(n_dev.cpu().numpy(), n_ref), (prec, r)
            other = gpu.Solver.for_grid(wl.grid(40, 1.5), prec).set_field(field, 300)
            other.propagate(-1)
            other.density()
            other.close()
        del graph
        s.close()

