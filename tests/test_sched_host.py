"""Host logic of the render server: the scheduling core (memory arena, idle
slot cache, admission order, retry/resume/cancel rules) is plain C++; this
builds tests/cpp/test_sched.cpp with g++ and runs it (no GPU), once as an
ordinary build and once under AddressSanitizer + UndefinedBehaviorSanitizer
(host code only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "test_sched.cpp")
INC = os.path.join(ROOT, "paper_2405_05446_amd", "csrc")


def _build_and_run(tmp_path, name, extra):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / name)
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-Wall", *extra, "-I", INC, SRC, "-o", exe],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(res.stdout[-2000:])
    assert res.returncode == 0, res.stdout[-4000:] + res.stderr[-4000:]
    assert "ALL OK" in res.stdout


def test_scheduling_core(tmp_path):
    _build_and_run(tmp_path, "test_sched", [])


def test_scheduling_core_under_address_and_ub_sanitizers(tmp_path):
    _build_and_run(tmp_path, "test_sched_san",
                   ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=undefined"])
