"""Host-only planning logic of the runtime (range arithmetic of the
multi-rate resampling, interpolation hops, trigger windows, device-memory
admission of serving banks, window readiness of a stream, the BF16 hi/lo
split of the interpolation filters of the BF16 path), compiled for the
CPU with the address and undefined-behaviour sanitizers and checked against
brute force, a queue model and the invariants the runtime relies on
(tests/host/test_plan.cpp).  The admission check is the host-side contract
of lloid_stream_admit / _remove (EAGAIN queueing under a small budget,
arrival order, ENOMEM above the budget) without a device."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_16416_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_planning_logic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "test_plan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", CSRC, os.path.join(ROOT, "tests", "host", "test_plan.cpp"),
           os.path.join(CSRC, "lloid_plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host planning checks passed" in r.stdout
