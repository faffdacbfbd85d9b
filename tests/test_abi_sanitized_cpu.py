"""The host side of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds librfi's sources with the sanitizers on the host pass only (device code is compiled
as usual) together with tests/abi_check.cpp, and runs it without a GPU: every argument
check and the host helpers must behave and be free of memory errors and undefined behaviour.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_14775_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")


@pytest.mark.skipif(HIPCC is None, reason="hipcc not available")
def test_host_abi_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "abi_check")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "screen.hip"), os.path.join(CSRC, "api.hip"), os.path.join(CSRC, "serve.hip"),
           os.path.join(CSRC, "calibrate.cpp"), os.path.join(ROOT, "tests", "abi_check.cpp"),
           "-lrocprofiler-sdk-roctx", "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0 and "ALL OK" in run.stdout, run.stdout[-3000:] + run.stderr[-3000:]
