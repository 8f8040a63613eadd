"""The library's host planning (csrc/sht_plan.cpp: level layout, tile lists,
blocked table copies and seed rows) and host numerics (csrc/sht_host.cpp)
built with AddressSanitizer, UndefinedBehaviorSanitizer and the planner's
bounds assertions (SHT_CHECK), and driven over many plan shapes by
tests/native/plan_check.cpp (no GPU)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1711_11296_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_planning_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-DSHT_CHECK", "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
           os.path.join(CSRC, "sht_plan.cpp"), os.path.join(CSRC, "sht_host.cpp"),
           os.path.join(ROOT, "tests", "native", "plan_check.cpp"), "-pthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
