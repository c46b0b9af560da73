"""The host planner (topology, CSR pattern, scatter slots, tables) built with
AddressSanitizer and UndefinedBehaviorSanitizer (g++, no GPU code) and run
over seeded meshes of every order, with natural-face masks and every error
path of the planner (tests/sanitize/plan_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_planner_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = tmp_path / "plan_check"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", "/opt/rocm/include",
           os.path.join(ROOT, "tests", "sanitize", "plan_check.cpp"),
           os.path.join(ROOT, "paper_1801_08914_amd", "csrc", "plan.cpp"), "-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert run.stdout.strip().endswith("ok")
