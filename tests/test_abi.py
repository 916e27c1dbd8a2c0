"""The C-ABI library loads and exports every entry point include/gdgs.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2405_05446_amd", "libgdgs.so")
HEADER = os.path.join(ROOT, "include", "gdgs.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gdgs_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libgdgs.so is not built; run python -m paper_2405_05446_amd.build")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    import paper_2405_05446_amd._lib as L
    assert sorted(L.declared_symbols()) == declared()


def test_host_only_calls_validate_arguments(lib):
    # status strings and size queries run on the host only
    lib.gdgs_status_string.restype = ctypes.c_char_p
    assert lib.gdgs_status_string(0) == b"ok"
    lib.gdgs_last_error.restype = ctypes.c_char_p
    n = ctypes.c_size_t(0)
    f = lib.gdgs_raster_workspace_size
    f.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
    assert f(1000, ctypes.byref(n)) == 0 and n.value >= 1000 * 64
    assert f(-1, ctypes.byref(n)) == 1
    assert b"out of range" in lib.gdgs_last_error()
    g = lib.gdgs_bin_sort_workspace_size
    g.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                  ctypes.POINTER(ctypes.c_size_t)]
    assert g(10, 2, 64, 100, ctypes.byref(n)) == 1     # W < 3
    assert g(10, 64, 64, 0, ctypes.byref(n)) == 1      # zero capacity
    assert g(10, 64, 64, 100, ctypes.byref(n)) == 0


def test_image_size_limits(lib):
    # tile rectangles pack 16-bit tile coordinates: at most 65535 tiles a side
    n = ctypes.c_size_t(0)
    g = lib.gdgs_bin_sort_workspace_size
    g.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                  ctypes.POINTER(ctypes.c_size_t)]
    assert g(10, 16 * 65535 + 1, 64, 100, ctypes.byref(n)) == 1
    assert g(10, 64, 16 * 65535 + 1, 100, ctypes.byref(n)) == 1
    assert g(10, 16 * 65535, 64, 100, ctypes.byref(n)) == 0
    assert g(10, 3, 3, 100, ctypes.byref(n)) == 0


def test_timer_repeats_validate_on_the_host(lib):
    # repeats apply to an armed multigrid post pass only; nothing here touches
    # the GPU (no timer is armed)
    f = lib.gdgs_set_kernel_timer_repeats
    f.argtypes = [ctypes.c_char_p, ctypes.c_int]
    lib.gdgs_last_error.restype = ctypes.c_char_p
    assert f(b"raster", 4) == 1
    assert b"post passes only" in lib.gdgs_last_error()
    assert f(b"mg_post_fine", 0) == 1 and f(b"mg_post_fine", 65) == 1
    assert f(b"mg_post_fine", 4) == 1
    assert b"not armed" in lib.gdgs_last_error()
    assert f(None, 4) == 1


def test_smoothing_weight_validates_on_the_host(lib):
    # the multigrid parameters are checked before any device call
    import paper_2405_05446_amd._lib as L
    f = lib.gdgs_poisson_workspace_size
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(L.MgParams),
                  ctypes.POINTER(ctypes.c_size_t)]
    lib.gdgs_last_error.restype = ctypes.c_char_p
    n = ctypes.c_size_t(0)
    for w in (2.0, 1.6, 0.4, -1.0, float("nan")):
        mg = L.MgParams(0, 2, 2, 20, 0, 0, 1e-6, w)
        assert f(64, 64, ctypes.byref(mg), ctypes.byref(n)) == 1, w
        assert b"smoothing weight" in lib.gdgs_last_error(), w
