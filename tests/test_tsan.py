"""ThreadSanitizer run of the library's threaded host code on the CPU: the
host TM's worker threads, the merge worker and its scatter pool, and the
serving path's helper pool, driven by tests/tsan/tsan_driver.cpp in a g++
build with -fsanitize=thread (host code only; no GPU, no HIP runtime)."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_00661_amd", "csrc")


def _build(tmp_path) -> str:
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "tsan_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread", "-D__HIP_PLATFORM_AMD__",
           "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "tsan", "tsan_driver.cpp"), os.path.join(CSRC, "host_tm.cpp"),
           os.path.join(CSRC, "merge_host.cpp"), "-o", exe]
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stderr[-4000:]
    return exe


def test_threaded_host_code_has_no_data_race(tmp_path):
    exe = _build(tmp_path)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66 second_deadlock_stack=1")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert "ThreadSanitizer" not in p.stderr, p.stderr[-6000:]
    assert p.returncode == 0, (p.returncode, p.stdout[-2000:], p.stderr[-4000:])
    assert "all checks passed" in p.stdout
