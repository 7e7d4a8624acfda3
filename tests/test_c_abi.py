"""include/pd.h is plain C: it compiles as strict C99 (no C++ in the header), a C
program linked against libpd.so drives the host-side entry points without a device,
and (GPU) another runs whole solves on the device through the ABI alone, checked
against the oracle (Sec. II Eq. (1); Sec. III Eqs. (11)-(13))."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_1607_03062_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_header_is_strict_c99(tmp_path):
    src = tmp_path / "h.c"
    src.write_text('#include "pd.h"\nint main(void) { return (int)sizeof(pd_field) > 0 ? 0 : 1; }\n')
    subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-c", str(src), "-o", str(tmp_path / "h.o")], check=True)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_c_program_uses_the_abi(tmp_path):
    if not os.path.exists(os.path.join(LIB_DIR, "libpd.so")):
        pytest.skip("libpd.so not built")
    exe = tmp_path / "abi_host"
    subprocess.run(["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_host.c"), "-L", LIB_DIR, "-lpd", "-lm",
                    "-Wl,-rpath," + LIB_DIR, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout and r.stdout.count("ok  ") == 17


@pytest.mark.gpu
@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("precision,scheme", [(0, 0), (0, 1), (1, 0)])
def test_c_program_solves_on_the_device(gpu, tmp_path, precision, scheme):
    """tests/c/abi_device.c: a ragged 37 x 29 grid, 1500 steps in two pd_propagate calls on
    the default stream (and a second handle restarted from the state saved between them,
    pd_save_state / pd_load_state, bit for bit), pd_density and pd_density_static, from a
    plain C99 process with no torch; its n(p) and rho against the FP64 oracle (FP64 1e-12
    per point and relative on rho, FP32 1e-5 per point)."""
    import oracle
    from paper_1607_03062_amd import workloads as wl

    exe = tmp_path / "abi_device"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_device.c"), "-L", LIB_DIR, "-lpd",
                    "-Wl,-rpath," + LIB_DIR, "-o", str(exe)], check=True)
    print("abi_device precision %d scheme %d" % (precision, scheme), flush=True)
    r = subprocess.run([str(exe), str(precision), str(scheme)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    vals = {}
    n = np.full(37 * 29, np.nan)
    for line in r.stdout.splitlines():
        parts = line.split()
        if parts[0] == "n":
            n[int(parts[1])] = float(parts[2])
        elif parts[0] in ("rho", "rho_static"):
            vals[parts[0]] = float(parts[1])
    grid = {"nx": 37, "ny": 29, "px": (-2.0, 2.0), "py": (-1.5, 1.5)}
    n_o = oracle.solve_grid(wl.sin2(0.1, 0.5, 4), grid, 1500, ("strang", "midpoint")[scheme])[0]
    err = float(np.max(np.abs(n - n_o)))
    if precision == 0:
        rho_o = oracle.density(grid, n_o)
        assert err <= 1e-12 and abs(vals["rho"] / rho_o - 1) <= 1e-12, (err, vals, rho_o)
    else:
        assert err <= 1e-5, err
    assert vals["rho"] == vals["rho_static"]


@pytest.mark.gpu
@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_c_program_runs_a_batch_on_the_device(gpu, tmp_path):
    """tests/c/abi_batch.c: four members (FP32, FP64 and fast FP32 Strang in the persistent
    kernel, an FP64 midpoint member in its own launch) run by pd_batch_run twice (capture,
    replay) and by pd_batch_step_each epochs of uneven limits, from a plain C99 process;
    every rho and n(p) equals the member's solve alone bit for bit."""
    exe = tmp_path / "abi_batch"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_batch.c"), "-L", LIB_DIR, "-lpd",
                    "-Wl,-rpath," + LIB_DIR, "-o", str(exe)], check=True)
    print("abi_batch", flush=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "batch ok" in r.stdout, r.stdout[-3000:] + r.stderr[-2000:]
