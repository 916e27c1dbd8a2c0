"""ctypes binding of libgdgs (include/gdgs.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.

torch is imported before the library is loaded so that both share torch's HIP
runtime; device buffers are torch tensors, streams are torch streams.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgdgs.so")

OK = 0
STATUS = {0: "GDGS_OK", 1: "GDGS_ERR_INVALID_ARGUMENT", 2: "GDGS_ERR_CAPACITY",
          3: "GDGS_ERR_WORKSPACE", 4: "GDGS_ERR_BUDGET", 5: "GDGS_ERR_HIP",
          6: "GDGS_ERR_UNSUPPORTED", 7: "GDGS_ERR_NOT_READY", 8: "GDGS_ERR_CANCELLED"}
ERR_BUDGET, ERR_CANCELLED = 4, 8


class GdgsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


c_float_p = ctypes.c_void_p   # device pointers travel as plain addresses


class Scene(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("log_scale", ctypes.c_void_p),
                ("quat", ctypes.c_void_p), ("opacity", ctypes.c_void_p),
                ("value", ctypes.c_void_p), ("K", ctypes.c_int64)]


class Camera(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3)]


class Proj(ctypes.Structure):
    _fields_ = [("mean2d", ctypes.c_void_p), ("conic", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("rect", ctypes.c_void_p),
                ("count", ctypes.c_void_p)]


class Bins(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("tile_of_pair", ctypes.c_void_p),
                ("splat_of_pair", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("ranges", ctypes.c_void_p), ("num_pairs", ctypes.c_void_p),
                ("tile_order", ctypes.c_void_p)]


class MgParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("pre_sweeps", ctypes.c_int32),
                ("post_sweeps", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
                ("coarse_sweeps", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("tol", ctypes.c_double), ("smooth_weight", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32 * 3), ("converged", ctypes.c_int32),
                ("eta", ctypes.c_double * 3), ("rel_res", ctypes.c_double * 3),
                ("b_norm", ctypes.c_double * 3), ("delta", ctypes.c_double * 3),
                ("num_pairs", ctypes.c_int64),
                ("overflow", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServerParams(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("mg", MgParams)]


class Request(ctypes.Structure):
    _fields_ = [("cam", Camera), ("boundary", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("tag", ctypes.c_uint64), ("arrival_ns", ctypes.c_int64),
                ("u_init", ctypes.c_void_p)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("attempts", ctypes.c_int32), ("num_pairs", ctypes.c_int64),
                ("arrival_ns", ctypes.c_int64), ("admit_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64)]


class ServerState(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("used_bytes", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("submitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("waiting", ctypes.c_int32),
                ("running", ctypes.c_int32), ("idle_slots", ctypes.c_int32),
                ("streams", ctypes.c_int32)]


P = ctypes.POINTER
_SIGS = {
    "gdgs_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gdgs_last_error": (ctypes.c_char_p, []),
    "gdgs_version": (ctypes.c_char_p, []),
    "gdgs_set_graphs": (None, [ctypes.c_int]),
    "gdgs_clear_graphs": (None, []),
    "gdgs_set_channel_streams": (None, [ctypes.c_int]),
    "gdgs_set_kernel_timer": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int]),
    "gdgs_set_kernel_timer_repeats": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int]),
    "gdgs_rewind_kernel_timers": (None, []),
    "gdgs_kernel_timer_count": (ctypes.c_int, [ctypes.c_char_p]),
    "gdgs_bin_sort_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.c_int64, P(ctypes.c_size_t)]),
    "gdgs_raster_workspace_size": (ctypes.c_int, [ctypes.c_int64, P(ctypes.c_size_t)]),
    "gdgs_poisson_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, P(MgParams),
                                                   P(ctypes.c_size_t)]),
    "gdgs_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int64, P(MgParams), P(ctypes.c_size_t)]),
    "gdgs_raster_backward_workspace_size": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64,
                                                           P(ctypes.c_size_t)]),
    "gdgs_project": (ctypes.c_int, [P(Scene), P(Camera), P(Proj), ctypes.c_void_p]),
    "gdgs_project_2d": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P(Proj),
                                       ctypes.c_void_p]),
    "gdgs_bin_sort": (ctypes.c_int, [P(Proj), ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     P(Bins), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gdgs_raster_grad": (ctypes.c_int, [P(Proj), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        P(Bins), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gdgs_raster_laplacian": (ctypes.c_int, [P(Proj), ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64, P(Bins), ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p]),
    "gdgs_raster_count": (ctypes.c_int, [P(Proj), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                         P(Bins), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gdgs_poisson_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_int32, P(MgParams), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p]),
    "gdgs_poisson_solve_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                              ctypes.c_int32, P(MgParams), ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                              ctypes.c_void_p]),
    "gdgs_raster_laplacian_threshold": (ctypes.c_int, [P(Proj), ctypes.c_void_p, ctypes.c_void_p,
                                                       ctypes.c_int64, P(Bins), ctypes.c_int32,
                                                       ctypes.c_int32, ctypes.c_float,
                                                       ctypes.c_void_p, ctypes.c_void_p,
                                                       ctypes.c_void_p, ctypes.c_size_t,
                                                       ctypes.c_void_p]),
    "gdgs_render_laplacian_sparse": (ctypes.c_int, [P(Scene), P(Camera), ctypes.c_void_p,
                                                    P(MgParams), ctypes.c_int64, ctypes.c_float,
                                                    ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_int,
                                                    ctypes.c_void_p, ctypes.c_size_t,
                                                    ctypes.c_void_p]),
    "gdgs_poisson_solve_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_int32, ctypes.c_int32, P(MgParams),
                                                 ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p]),
    "gdgs_render": (ctypes.c_int, [P(Scene), P(Camera), ctypes.c_void_p, P(MgParams),
                                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "gdgs_render_laplacian": (ctypes.c_int, [P(Scene), P(Camera), ctypes.c_void_p, P(MgParams),
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                             ctypes.c_void_p]),
    "gdgs_project_backward": (ctypes.c_int, [P(Scene), P(Camera), ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "gdgs_image_loss_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32,
                                                      ctypes.POINTER(ctypes.c_size_t)]),
    "gdgs_image_loss": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p]),
    "gdgs_threshold": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_float,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "gdgs_adam_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_void_p]),
    "gdgs_div_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "gdgs_div_adjoint_neumann": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_void_p, ctypes.c_void_p]),
    "gdgs_raster_grad_backward": (ctypes.c_int, [P(Proj), ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_int64, P(Bins), ctypes.c_int32,
                                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_size_t, ctypes.c_void_p]),
    "gdgs_now_ns": (ctypes.c_int64, []),
    "gdgs_server_create": (ctypes.c_int, [P(Scene), P(ServerParams), P(ctypes.c_void_p)]),
    "gdgs_server_submit": (ctypes.c_int, [ctypes.c_void_p, P(Request), P(ctypes.c_int64)]),
    "gdgs_server_poll": (ctypes.c_int, [ctypes.c_void_p, P(Completion), ctypes.c_int32,
                                        ctypes.c_int32, P(ctypes.c_int32)]),
    "gdgs_server_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "gdgs_server_query": (ctypes.c_int, [ctypes.c_void_p, P(ServerState)]),
    "gdgs_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
}

_lib = None


def load(path: str | None = None):
    """Load libgdgs.so (once).  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing; build it with "
                           "`python -m paper_2405_05446_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols() -> list[str]:
    return list(_SIGS)


def check(status: int):
    if status != OK:
        msg = load().gdgs_last_error().decode()
        raise GdgsError(status, msg)


def ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def stream_handle(stream: torch.cuda.Stream | None = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream
