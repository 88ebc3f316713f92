"""CPU tests of the serving scheduler (admission by memory, FIFO fairness,
in-flight limits, cancellation, timeouts, executor failure, shutdown, a
threaded stress run) with a mock executor, under ThreadSanitizer and under
AddressSanitizer + UndefinedBehaviorSanitizer.  Host code only (g++)."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "test_sched.cpp")
INC = os.path.join(ROOT, "paper_2008_08483_amd", "csrc")


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_scheduler_under_sanitizer(tmp_path, san):
    exe = tmp_path / "test_sched"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", f"-fsanitize={san}",
           "-fno-omit-frame-pointer", "-I", INC, SRC, "-o", str(exe)]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240, env=env)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "OK" in res.stdout
