"""The C oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: no sanitizer reaches the kernels).

tests/c/oracle_sanitize.c drives every entry point of oracle/oracle.c over both schemes,
second and fourth order, both valleys and every field kind on small grids; any
out-of-bounds access, use of uninitialised stack memory caught by ASan, signed overflow,
misaligned load or similar undefined behaviour aborts the run.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sanitizers_available(tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", str(probe), "-o", str(tmp_path / "probe")],
                       capture_output=True, text=True)
    return r.returncode == 0


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if not _sanitizers_available(tmp_path):
        pytest.skip("gcc has no libasan/libubsan here")
    exe = tmp_path / "oracle_sanitize"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-Wall", "-Wno-unknown-pragmas",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-ffp-contract=off", os.path.join(ROOT, "tests", "c", "oracle_sanitize.c"), "-o", str(exe), "-lm"],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle paths ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


HOST_SOURCES = ["pd_api.cpp", "field.cpp", "batch.cpp", "autotune.cpp"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="gcc not available")
def test_library_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The library's host sources built with g++ and both sanitizers, linked with the
    kernel object of the normal build into a shared library, and driven without a
    device by tests/c/host_sanitize.c (field sampling of every kind and scheme,
    pd_check_field, argument checks, batch membership, fault specifications, error
    messages from eight threads); LeakSanitizer runs at exit."""
    if not _sanitizers_available(tmp_path):
        pytest.skip("gcc has no libasan/libubsan here")
    pkg = os.path.join(ROOT, "paper_1607_03062_amd")
    kernels_obj = os.path.join(pkg, "_build", "kernels.hip.o")
    if not os.path.exists(kernels_obj):
        pytest.skip("kernel object not built (python -m paper_1607_03062_amd.build)")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", *san,
                        "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(rocm, "include"),
                        "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(pkg, "csrc"),
                        "-c", os.path.join(pkg, "csrc", src), "-o", obj], check=True, capture_output=True, text=True)
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, HOST_SOURCES))
    lib_dir = tmp_path / "lib"
    lib_dir.mkdir()
    subprocess.run(["g++", "-shared", *san, "-o", str(lib_dir / "libpd.so"), *objs, kernels_obj,
                    "-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")],
                   check=True, capture_output=True, text=True)
    exe = tmp_path / "host_sanitize"
    subprocess.run(["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-g", "-Wall", "-Werror", *san,
                    "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "host_sanitize.c"),
                    "-L" + str(lib_dir), "-lpd", "-lm", "-lpthread", "-Wl,-rpath," + str(lib_dir), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, HIP_VISIBLE_DEVICES="", ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("PD_FAULT", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "host paths ok" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
