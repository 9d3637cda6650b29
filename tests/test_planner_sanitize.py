"""The host planner built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host sources only: planner.cpp, gates.cpp, density.cpp) plans valid,
invalid and adversarial circuits over the whole option space; any sanitizer
report or crash fails the test, and invalid inputs must come back as error
statuses (tests/planner_sanitize.cpp)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_02957_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "planner_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "planner_sanitize.cpp")]
    cmd += [os.path.join(CSRC, f) for f in ("planner.cpp", "gates.cpp", "density.cpp")]
    subprocess.run(cmd + ["-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.startswith("ok "), r.stdout
    assert int(r.stdout.split()[1]) > 500
