"""pd_density_static, the density entry point that allocates nothing (its reduction
scratch is a static device array of the library), against pd_density: two calls in a
row on one device, the second on a smaller grid, each bit for bit equal to pd_density
(same kernels, same fixed summation order), with n(p) to host and to device memory."""
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
