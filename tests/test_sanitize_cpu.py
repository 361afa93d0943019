"""Host sanitizers on the C code the tests stand on: the CPU oracle and the
input generators, built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host only) and driven by tests/c/sanitize_driver.c over graphs of every
family.  Any sanitizer report or failed cross-check fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "graphgen", "graphgen.c"),
           os.path.join(ROOT, "tests", "c", "sanitize_driver.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all checks passed" in r.stdout
