"""Host logic of the render server: the scheduling core (memory arena, idle
slot cache, admission order, retry/resume/cancel rules) is plain C++; this
builds tests/cpp/test_sched.cpp with g++ and runs it (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduling_core(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "test_sched")
    src = os.path.join(ROOT, "tests", "cpp", "test_sched.cpp")
    inc = os.path.join(ROOT, "paper_2405_05446_amd", "csrc")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-Wall", "-I", inc, src, "-o", exe],
                   check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(res.stdout)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ALL OK" in res.stdout
