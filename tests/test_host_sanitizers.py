"""The library's host logic (argument checks, workspace sizing, overlap
checks, plan building, offset and size arithmetic) built for the CPU under
AddressSanitizer and UndefinedBehaviorSanitizer, with the GPU code compiled
but never launched: tests/host/check_host_logic.cpp drives it on random and
boundary inputs.  CPU only (no GPU call is made)."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1802_00036_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
DRIVER = os.path.join(ROOT, "tests", "host", "check_host_logic.cpp")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is needed to build the library's sources")
def test_host_logic_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "check_host_logic")
        # sanitizers on the host side only (the device code is not instrumented)
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
               f"-I{CSRC}", f"-I{INCLUDE}",
               os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "stream.hip"), os.path.join(CSRC, "api.hip"),
               DRIVER, "-o", exe]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-6000:]
        assert "host logic ok" in run.stdout
