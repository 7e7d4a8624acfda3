"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code only).

tests/c/oracle_sanitize.c drives every entry point of oracle/oracle.c over both schemes,
second and fourth order, both valleys and every field kind on small grids; any
out-of-bounds access, use of uninitialised stack memory caught by ASan, signed overflow,
misaligned load or similar undefined behaviour aborts the run.
"""
import os
import shutil
import subprocess

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
