"""Serving binding: many views of one resident scene through the library's
native render server (gdgs_server_* in include/gdgs.h).

The scheduler, the memory arena and every launch live in libgdgs; this
module only marshals requests and completions and keeps the caller's
tensors alive until their request has completed.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .api import DeviceScene, camera_struct, mg_params

F32 = torch.float32
BATCHED = 1   # GDGS_SERVER_BATCHED


def now_ns() -> int:
    """The library's steady clock (time base of arrivals and completions)."""
    return int(L.load().gdgs_now_ns())


class Server:
    """Continuous-batching render server on the current device.

    budget: bytes of device memory for in-flight requests (allocated once);
    streams: requests whose front half runs at once (1 without batching = the
    plain one-at-a-time path);
    batched: the solves of all in-flight requests advance together in
    persistent-kernel rounds on one solver stream (GDGS_SERVER_BATCHED;
    Dirichlet problem only), with streams + 1 HIP streams in all.
    """

    def __init__(self, scene: DeviceScene, budget: int = 4 << 30, streams: int = 4, mg=None,
                 batched: bool = False):
        self.lib = L.load()
        self.scene = scene
        self.mg = mg if mg is not None else mg_params()
        self.batched = bool(batched)
        p = L.ServerParams(int(budget), int(streams), BATCHED if batched else 0, self.mg)
        h = ctypes.c_void_p()
        L.check(self.lib.gdgs_server_create(ctypes.byref(scene.struct(6)), ctypes.byref(p),
                                            ctypes.byref(h)))
        self.h = h
        self.live: dict[int, tuple] = {}    # id -> (u, boundary, u_init) kept alive until completed

    def submit(self, cam, boundary: torch.Tensor | None = None, u: torch.Tensor | None = None,
               tag: int = 0, arrival_ns: int = 0,
               u_init: torch.Tensor | None = None) -> tuple[int, torch.Tensor]:
        """Queue one view; returns (request id, the tensor u that will hold it).
        u_init: starting image of the solve (warm start), e.g. the previous view
        of a moving camera.  The caller must not touch u, boundary or u_init
        until the completion arrives."""
        W, H = int(cam.W), int(cam.H)
        dev = self.scene.opacity.device
        if u is None:
            u = torch.empty((3, H, W), dtype=F32, device=dev)
        if tuple(u.shape) != (3, H, W) or u.dtype != F32 or not u.is_contiguous():
            raise ValueError("u must be a contiguous float32 [3][H][W] tensor")
        if boundary is not None and (tuple(boundary.shape) != (3, H, W) or boundary.dtype != F32
                                     or not boundary.is_contiguous()):
            raise ValueError("boundary must be a contiguous float32 [3][H][W] tensor")
        if u_init is not None and (tuple(u_init.shape) != (3, H, W) or u_init.dtype != F32
                                   or not u_init.is_contiguous()):
            raise ValueError("u_init must be a contiguous float32 [3][H][W] tensor")
        # work queued on torch's stream (e.g. filling the boundary) must be
        # done before the server's streams read it
        torch.cuda.current_stream(dev).synchronize()
        req = L.Request(camera_struct(cam), L.ptr(boundary), L.ptr(u), int(tag), int(arrival_ns),
                        L.ptr(u_init))
        rid = ctypes.c_int64()
        L.check(self.lib.gdgs_server_submit(self.h, ctypes.byref(req), ctypes.byref(rid)))
        self.live[rid.value] = (u, boundary, u_init)
        return rid.value, u

    def poll(self, max_n: int = 64, wait_us: int = 0) -> list[dict]:
        """Completions (oldest first) as dicts; waits up to wait_us for the first."""
        buf = (L.Completion * max_n)()
        n = ctypes.c_int32()
        L.check(self.lib.gdgs_server_poll(self.h, buf, max_n, int(wait_us), ctypes.byref(n)))
        out = []
        for c in buf[:n.value]:
            d = {f: getattr(c, f) for f, _ in L.Completion._fields_}
            u = self.live.pop(c.id, (None,))[0]
            d["u"] = u
            out.append(d)
        return out

    def cancel(self, rid: int):
        L.check(self.lib.gdgs_server_cancel(self.h, int(rid)))

    def state(self) -> dict:
        s = L.ServerState()
        L.check(self.lib.gdgs_server_query(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in L.ServerState._fields_}

    def drain(self, n: int, timeout_s: float = 120.0) -> list[dict]:
        """Wait for n completions."""
        import time
        out, t0 = [], time.perf_counter()
        while len(out) < n:
            out += self.poll(max(1, min(256, n - len(out))), wait_us=20_000)
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"{len(out)} of {n} requests completed in {timeout_s} s")
        return out

    def close(self):
        if self.h:
            L.check(self.lib.gdgs_server_destroy(self.h))
            self.h = None
            self.live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
