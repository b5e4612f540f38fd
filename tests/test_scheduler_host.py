"""The render server's request bookkeeping (csrc/scheduler.h) on the CPU:
a C++ unit test built with g++ (with the address and undefined-behaviour
sanitisers) drives it with fake ticks, including the GPU-error path with
ticks in flight, memory admission and the release of finished tickets."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_unit(tmp_path):
    exe = str(tmp_path / "scheduler_test")
    src = os.path.join(ROOT, "tests", "cpp", "scheduler_test.cpp")
    inc = os.path.join(ROOT, "paper_2306_16541_amd", "csrc")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", inc, src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
