"""The serving loop's admission rule on the CPU (no GPU): fixed cases and a simulated scheduler,
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer (tests/serve_policy_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_14775_amd", "csrc")
GXX = shutil.which("g++")


@pytest.mark.skipif(GXX is None, reason="g++ not available")
def test_admission_rule(tmp_path):
    exe = str(tmp_path / "serve_policy_check")
    cmd = [GXX, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", CSRC, os.path.join(ROOT, "tests", "serve_policy_check.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert run.returncode == 0 and "ALL OK" in run.stdout, run.stdout[-3000:] + run.stderr[-3000:]
