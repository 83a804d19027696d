"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code, gcc) and driven through every entry point on small 2-D and 3-D
grids with periodic and wall axes and both collisions
(tests/sanitize/oracle_driver.c): no invalid access, leak or undefined
operation, mass conserved, selected-cell update equal to the full step."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    build = subprocess.run(
        ["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-o", exe, os.path.join(HERE, "sanitize", "oracle_driver.c"),
         os.path.join(ROOT, "oracle", "elmrt_oracle.c"), "-lm"],
        capture_output=True, text=True)
    if build.returncode != 0 and "asan" in (build.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stderr[-2000:]
