"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: its
C source is built with a small driver (tests/oracle_sanitizer_driver.c)
into one executable with both sanitizers (no recovery, leak checking on)
and run on small 2D and 3D problems that reach every code path the tests
use; it must report no error and its results must match the direct sum."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
SRC = os.path.join(REPO, "oracle", "bfsft_oracle.c")
DRIVER = os.path.join(HERE, "oracle_sanitizer_driver.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", str(exe), DRIVER, SRC, "-lm"])
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert "all checks passed" in r.stdout
