"""The host log level read from GDGS_LOG (host-only calls: runs without a
GPU).  Each case runs in a fresh process, since the level is read once."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2405_05446_amd", "libgdgs.so")
CODE = r"""
import ctypes, sys
lib = ctypes.CDLL(sys.argv[1])
n = ctypes.c_size_t(0)
f = lib.gdgs_raster_workspace_size
f.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
assert f(-1, ctypes.byref(n)) == 1      # out of range: an error is recorded
assert f(10, ctypes.byref(n)) == 0
"""


def _stderr(level):
    env = dict(os.environ)
    env.pop("GDGS_LOG", None)
    if level is not None:
        env["GDGS_LOG"] = str(level)
    r = subprocess.run([sys.executable, "-c", CODE, LIB], env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return [ln for ln in r.stderr.splitlines() if ln.startswith("gdgs[")]


def test_silent_by_default_and_at_level_0():
    assert _stderr(None) == []
    assert _stderr(0) == []


def test_level_1_reports_the_recorded_errors():
    lines = _stderr(1)
    assert len(lines) == 1 and lines[0].startswith("gdgs[error] ") and "out of range" in lines[0]


def test_level_3_reports_every_entry_point_call():
    lines = _stderr(3)
    calls = [ln for ln in lines if ln == "gdgs[debug] call gdgs_raster_workspace_size"]
    assert len(calls) == 2
    assert any(ln.startswith("gdgs[error] ") for ln in lines)
