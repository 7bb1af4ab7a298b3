"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/native/host_checks.cpp links host.cpp
(instance generator, schedules, tables) and tn_plan.cpp (tensor-network
planner) and drives the anneal server's admission policy (admission.hpp)
with a scripted clock; g++ builds it with both sanitizers, and any report
or failed check ends the program with a nonzero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_17267_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_checks")
    # the sanitizer runtimes linked statically, so the program does not
    # depend on the order of the process's preloaded libraries
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-static-libasan", "-static-libubsan",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(NATIVE, "host_checks.cpp"), os.path.join(CSRC, "host.cpp"), os.path.join(CSRC, "tn_plan.cpp"),
           "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks passed" in r.stdout
