"""The host planner (trajectory tables, boundary taps, angle pairs, the
App. D eigen-decomposition) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and run on several grains (CPU only)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_planner_under_address_and_ub_sanitizers():
    src = os.path.join(ROOT, "tests", "asan", "plan_harness.cpp")
    plan = os.path.join(ROOT, "paper_2205_15000_amd", "csrc", "plan.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "plan_harness")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "paper_2205_15000_amd", "csrc"),
               src, plan, "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "OK" in r.stdout and "runtime error" not in r.stderr
