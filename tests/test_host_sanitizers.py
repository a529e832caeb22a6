"""The host planning code (plan.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer by g++ and run over cubic, orthorhombic and
triclinic requests of both methods (tests/host_plan_checks.cpp). No GPU."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_plan_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2505_09727_amd", "csrc")
    exe = str(tmp_path / "host_plan_checks")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(ROOT, "tests", "host_plan_checks.cpp"), os.path.join(csrc, "plan.cpp"), "-o", exe,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ok (0 failures)" in r.stdout
