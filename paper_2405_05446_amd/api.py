"""Python entry points with the C ABI's names (include/gdgs.h), taking torch
device tensors.  Each function validates shapes, allocates outputs and
workspaces with torch, and calls the library; no arithmetic of the method
happens here.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

F32 = torch.float32
U32 = torch.int32          # u32 arrays are held in int32 tensors (same bytes)
STATS_BYTES = ctypes.sizeof(L.Stats)


def _dev(device=None) -> torch.device:
    return torch.device(device if device is not None else "cuda")


def _need(t: torch.Tensor, shape, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)}")


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """A 256-byte aligned uint8 device buffer of at least nbytes."""
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=_dev(device))
    off = (-buf.data_ptr()) % 256
    return buf[off:off + int(nbytes)]


def camera_struct(cam) -> L.Camera:
    c = L.Camera()
    c.W, c.H = int(cam.W), int(cam.H)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, dtype=np.float64).reshape(9)
    t = np.asarray(cam.t, dtype=np.float64).reshape(3)
    c.R = (ctypes.c_double * 9)(*R.tolist())
    c.t = (ctypes.c_double * 3)(*t.tolist())
    return c


WARM_START = 1
RESUME = 2
NEUMANN = 4  # no flux across the image border, zero-mean image (boundary must be None)
FMG = 8      # full-multigrid start of a fresh solve
STOP_ETA = 16  # stop on the normwise backward error eta instead of the relative correction


def mg_params(levels: int = 0, pre: int = 2, post: int = 2, max_cycles: int = 20,
              tol: float = 1e-6, coarse_sweeps: int = 0, flags: int = 0,
              smooth_weight: float = 0.0) -> L.MgParams:
    """smooth_weight: over-relaxation of the red-black sweeps (0 = the library's
    default, 1 = plain Gauss-Seidel)."""
    return L.MgParams(levels, pre, post, max_cycles, coarse_sweeps, flags, float(tol),
                      float(smooth_weight))


@dataclass
class DeviceScene:
    mean: torch.Tensor       # [3][K]
    log_scale: torch.Tensor  # [3][K]
    quat: torch.Tensor       # [4][K]
    opacity: torch.Tensor    # [K]
    value: torch.Tensor      # [6][K] image gradients, or [3][K] Laplacians (Laplacian form)

    @property
    def K(self) -> int:
        return int(self.opacity.shape[0])

    @staticmethod
    def from_host(scene, device=None) -> "DeviceScene":
        d = _dev(device)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(d)
        return DeviceScene(t(scene.mean), t(scene.log_scale), t(scene.quat), t(scene.opacity),
                           t(scene.value))

    @property
    def nch(self) -> int:
        return int(self.value.shape[0])

    def struct(self, nch: int | None = None) -> L.Scene:
        K = self.K
        nch = self.nch if nch is None else nch
        if nch not in (3, 6):
            raise ValueError("value must have 6 (gradient) or 3 (Laplacian) rows")
        _need(self.mean, (3, K), F32, "mean")
        _need(self.log_scale, (3, K), F32, "log_scale")
        _need(self.quat, (4, K), F32, "quat")
        _need(self.opacity, (K,), F32, "opacity")
        _need(self.value, (nch, K), F32, "value")
        return L.Scene(L.ptr(self.mean), L.ptr(self.log_scale), L.ptr(self.quat),
                       L.ptr(self.opacity), L.ptr(self.value), K)


def alloc_proj(K: int, device=None) -> dict:
    d = _dev(device)
    k = max(K, 1)
    return dict(mean2d=torch.empty((2, k), dtype=F32, device=d)[:, :K],
                conic=torch.empty((3, k), dtype=F32, device=d)[:, :K],
                depth=torch.empty(k, dtype=F32, device=d)[:K],
                rect=torch.empty((2, k), dtype=U32, device=d)[:, :K],
                count=torch.empty(k, dtype=U32, device=d)[:K])


def _proj_struct(p: dict) -> L.Proj:
    return L.Proj(L.ptr(p["mean2d"]), L.ptr(p["conic"]), L.ptr(p["depth"]), L.ptr(p["rect"]),
                  L.ptr(p["count"]))


def alloc_bins(K: int, W: int, H: int, capacity: int, device=None,
               tile_order: bool = True) -> dict:
    """Device arrays of gdgs_bins; tile_order=False leaves the heaviest-first
    tile schedule out (the compositing kernels then take tiles by id)."""
    d = _dev(device)
    T = ((W + 15) // 16) * ((H + 15) // 16)
    return dict(capacity=int(capacity),
                tile_of_pair=torch.empty(capacity, dtype=U32, device=d),
                splat_of_pair=torch.empty(capacity, dtype=U32, device=d),
                order=torch.empty(max(K, 1), dtype=U32, device=d),
                ranges=torch.empty((2, T), dtype=U32, device=d),
                num_pairs=torch.zeros(1, dtype=torch.int64, device=d),
                tile_order=torch.empty(T, dtype=U32, device=d) if tile_order else None)


def _bins_struct(b: dict) -> L.Bins:
    return L.Bins(b["capacity"], L.ptr(b["tile_of_pair"]), L.ptr(b["splat_of_pair"]),
                  L.ptr(b["order"]), L.ptr(b["ranges"]), L.ptr(b["num_pairs"]),
                  L.ptr(b.get("tile_order")))


def read_stats(stats: torch.Tensor) -> dict:
    raw = bytes(stats.cpu().numpy().tobytes())
    s = L.Stats.from_buffer_copy(raw)
    return dict(cycles=list(s.cycles), converged=bool(s.converged), eta=list(s.eta),
                rel_res=list(s.rel_res), b_norm=list(s.b_norm), delta=list(s.delta),
                num_pairs=int(s.num_pairs),
                overflow=bool(s.overflow))


def new_stats(device=None) -> torch.Tensor:
    return torch.zeros(STATS_BYTES, dtype=torch.uint8, device=_dev(device))


def _size(fn, *args) -> int:
    n = ctypes.c_size_t(0)
    L.check(fn(*args, ctypes.byref(n)))
    return int(n.value)


# ---------------------------------------------------------------- steps
def gdgs_project(scene: DeviceScene, cam, proj: dict | None = None, stream=None) -> dict:
    lib = L.load()
    proj = proj if proj is not None else alloc_proj(scene.K, scene.opacity.device)
    c = camera_struct(cam)
    L.check(lib.gdgs_project(ctypes.byref(scene.struct()), ctypes.byref(c),
                             ctypes.byref(_proj_struct(proj)), L.stream_handle(stream)))
    return proj


def gdgs_project_2d(mean2d: torch.Tensor, conic: torch.Tensor, depth: torch.Tensor, W: int, H: int,
                    proj: dict | None = None, stream=None) -> dict:
    lib = L.load()
    K = int(depth.shape[0])
    _need(mean2d, (2, K), F32, "mean2d")
    _need(conic, (3, K), F32, "conic")
    _need(depth, (K,), F32, "depth")
    proj = proj if proj is not None else alloc_proj(K, depth.device)
    L.check(lib.gdgs_project_2d(L.ptr(mean2d), L.ptr(conic), L.ptr(depth), K, W, H,
                                ctypes.byref(_proj_struct(proj)), L.stream_handle(stream)))
    return proj


def gdgs_bin_sort(proj: dict, K: int, W: int, H: int, capacity: int, bins: dict | None = None,
                  ws: torch.Tensor | None = None, stream=None) -> dict:
    lib = L.load()
    dev = proj["depth"].device
    bins = bins if bins is not None else alloc_bins(K, W, H, capacity, dev)
    need = _size(lib.gdgs_bin_sort_workspace_size, K, W, H, bins["capacity"])
    ws = ws if ws is not None else workspace(need, dev)
    L.check(lib.gdgs_bin_sort(ctypes.byref(_proj_struct(proj)), K, W, H,
                              ctypes.byref(_bins_struct(bins)), L.ptr(ws), ws.numel(),
                              L.stream_handle(stream)))
    return bins


def gdgs_raster_grad(proj: dict, opacity: torch.Tensor, value: torch.Tensor, K: int, bins: dict,
                     W: int, H: int, grad: torch.Tensor | None = None,
                     ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    lib = L.load()
    dev = bins["ranges"].device
    _need(opacity, (K,), F32, "opacity")
    _need(value, (6, K), F32, "value")
    grad = grad if grad is not None else torch.empty((6, H, W), dtype=F32, device=dev)
    _need(grad, (6, H, W), F32, "grad")
    need = _size(lib.gdgs_raster_workspace_size, K)
    ws = ws if ws is not None else workspace(need, dev)
    L.check(lib.gdgs_raster_grad(ctypes.byref(_proj_struct(proj)), L.ptr(opacity), L.ptr(value),
                                 K, ctypes.byref(_bins_struct(bins)), W, H, L.ptr(grad),
                                 L.ptr(ws), ws.numel(), L.stream_handle(stream)))
    return grad


def _poisson(fn_name: str, src: torch.Tensor, src_ch: int, boundary, W, H, mg, u, stats, ws,
             stream):
    lib = L.load()
    dev = src.device
    _need(src, (src_ch, H, W), F32, "grad" if src_ch == 6 else "rho")
    if boundary is not None:
        _need(boundary, (3, H, W), F32, "boundary")
    mg = mg if mg is not None else mg_params()
    u = u if u is not None else torch.empty((3, H, W), dtype=F32, device=dev)
    _need(u, (3, H, W), F32, "u")
    stats = stats if stats is not None else new_stats(dev)
    need = _size(lib.gdgs_poisson_workspace_size, W, H, ctypes.byref(mg))
    ws = ws if ws is not None else workspace(need, dev)
    fn = getattr(lib, fn_name)
    L.check(fn(L.ptr(src), L.ptr(boundary), W, H, ctypes.byref(mg), L.ptr(u), L.ptr(stats),
               L.ptr(ws), ws.numel(), L.stream_handle(stream)))
    return u, stats


def gdgs_poisson_solve(grad: torch.Tensor, boundary: torch.Tensor | None, W: int, H: int,
                       mg: L.MgParams | None = None, u=None, stats=None, ws=None, stream=None):
    return _poisson("gdgs_poisson_solve", grad, 6, boundary, W, H, mg, u, stats, ws, stream)


def gdgs_poisson_solve_rhs(rho: torch.Tensor, boundary: torch.Tensor | None, W: int, H: int,
                           mg: L.MgParams | None = None, u=None, stats=None, ws=None,
                           stream=None):
    return _poisson("gdgs_poisson_solve_rhs", rho, 3, boundary, W, H, mg, u, stats, ws, stream)


def gdgs_poisson_solve_static(grad: torch.Tensor, boundary: torch.Tensor | None, W: int, H: int,
                              mg: L.MgParams | None = None, u=None, stats=None, stream=None):
    """gdgs_poisson_solve with the library's fixed scratch array instead of a
    workspace (the library allocates nothing for it; u and stats are
    allocated here unless given)."""
    lib = L.load()
    dev = grad.device
    _need(grad, (6, H, W), F32, "grad")
    if boundary is not None:
        _need(boundary, (3, H, W), F32, "boundary")
    mg = mg if mg is not None else mg_params()
    u = u if u is not None else torch.empty((3, H, W), dtype=F32, device=dev)
    _need(u, (3, H, W), F32, "u")
    L.check(lib.gdgs_poisson_solve_static(L.ptr(grad), L.ptr(boundary), W, H, ctypes.byref(mg),
                                          L.ptr(u), L.ptr(stats), L.stream_handle(stream)))
    return u, stats


def poisson_workspace_size(W: int, H: int, mg=None) -> int:
    lib = L.load()
    mg = mg if mg is not None else mg_params()
    return _size(lib.gdgs_poisson_workspace_size, W, H, ctypes.byref(mg))


def render_workspace_size(K: int, W: int, H: int, capacity: int, mg=None) -> int:
    lib = L.load()
    mg = mg if mg is not None else mg_params()
    return _size(lib.gdgs_workspace_size, K, W, H, capacity, ctypes.byref(mg))


def gdgs_render(scene: DeviceScene, cam, boundary: torch.Tensor | None, mg=None,
                capacity: int | None = None, u=None, stats=None, ws=None, sync_stats=False,
                stream=None):
    lib = L.load()
    dev = scene.opacity.device
    W, H = int(cam.W), int(cam.H)
    mg = mg if mg is not None else mg_params()
    capacity = int(capacity if capacity is not None else max(1 << 16, 16 * scene.K))
    if boundary is not None:
        _need(boundary, (3, H, W), F32, "boundary")
    u = u if u is not None else torch.empty((3, H, W), dtype=F32, device=dev)
    _need(u, (3, H, W), F32, "u")
    stats = stats if stats is not None else new_stats(dev)
    if ws is None:
        ws = workspace(render_workspace_size(scene.K, W, H, capacity, mg), dev)
    c = camera_struct(cam)
    L.check(lib.gdgs_render(ctypes.byref(scene.struct(6)), ctypes.byref(c), L.ptr(boundary),
                            ctypes.byref(mg), capacity, L.ptr(u), L.ptr(stats),
                            1 if sync_stats else 0, L.ptr(ws), ws.numel(),
                            L.stream_handle(stream)))
    return u, stats


def gdgs_project_backward(scene: DeviceScene, cam, dmean2d: torch.Tensor, dconic: torch.Tensor,
                          stream=None) -> dict:
    """dL/d(mean2d [2][K], conic [3][K]) -> dL/d(mean [3][K], log_scale [3][K],
    quat [4][K]) through the projection."""
    lib = L.load()
    K = scene.K
    dev = scene.opacity.device
    _need(dmean2d, (2, K), F32, "dmean2d")
    _need(dconic, (3, K), F32, "dconic")
    out = dict(mean=torch.empty((3, K), dtype=F32, device=dev),
               log_scale=torch.empty((3, K), dtype=F32, device=dev),
               quat=torch.empty((4, K), dtype=F32, device=dev))
    c = camera_struct(cam)
    L.check(lib.gdgs_project_backward(ctypes.byref(scene.struct()), ctypes.byref(c),
                                      L.ptr(dmean2d), L.ptr(dconic), L.ptr(out["mean"]),
                                      L.ptr(out["log_scale"]), L.ptr(out["quat"]),
                                      L.stream_handle(stream)))
    return out


def gdgs_image_loss(c: torch.Tensor, im: torch.Tensor, lam: float = 0.2, beta: float = 0.1,
                    want_grad: bool = True, ws=None, stream=None):
    """Eq. 22 between images c, im [3][H][W]: (loss [4] float64 device tensor
    (L, L1 term, gradient term, D_SSIM), dL/dc or None)."""
    lib = L.load()
    H, W = int(c.shape[1]), int(c.shape[2])
    _need(c, (3, H, W), F32, "c")
    _need(im, (3, H, W), F32, "im")
    out = torch.zeros(4, dtype=torch.float64, device=c.device)
    dc = torch.empty_like(c) if want_grad else None
    need = _size(lib.gdgs_image_loss_workspace_size, W, H)
    ws = ws if ws is not None else workspace(need, c.device)
    L.check(lib.gdgs_image_loss(L.ptr(c), L.ptr(im), W, H, float(lam), float(beta), L.ptr(out),
                                L.ptr(dc), L.ptr(ws), ws.numel(), L.stream_handle(stream)))
    return out, dc


def gdgs_threshold(x: torch.Tensor, t: float, count: bool = True, stream=None):
    """In-place hard threshold (Eq. 24) of a float32 device tensor; returns a
    device int64 tensor with the non-zero count (or None)."""
    lib = L.load()
    if x.dtype != F32 or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("x must be a contiguous float32 device tensor")
    nz = torch.zeros(1, dtype=torch.int64, device=x.device) if count else None
    L.check(lib.gdgs_threshold(L.ptr(x), x.numel(), float(t), L.ptr(nz),
                               L.stream_handle(stream)))
    return nz


def gdgs_adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                   t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                   eps: float = 1e-15, lo: float = 0.0, hi: float = 0.0, stream=None):
    """In-place Adam update of param (and its moments m, v) at step t >= 1;
    clamped to [lo, hi] when lo < hi."""
    lib = L.load()
    for name, x in (("grad", grad), ("m", m), ("v", v)):
        _need(x, tuple(param.shape), F32, name)
    L.check(lib.gdgs_adam_step(L.ptr(param), L.ptr(grad), L.ptr(m), L.ptr(v), param.numel(),
                               int(t), float(lr), float(beta1), float(beta2), float(eps),
                               float(lo), float(hi), L.stream_handle(stream)))


def gdgs_raster_laplacian(proj: dict, opacity: torch.Tensor, lap: torch.Tensor, K: int,
                          bins: dict, W: int, H: int, rho: torch.Tensor | None = None,
                          ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Three-channel composite of Laplacian splats (lap [3][K]) -> rho [3][H][W]."""
    lib = L.load()
    dev = bins["ranges"].device
    _need(opacity, (K,), F32, "opacity")
    _need(lap, (3, K), F32, "lap")
    rho = rho if rho is not None else torch.empty((3, H, W), dtype=F32, device=dev)
    if rho.dtype != F32 or not rho.is_contiguous() or rho.numel() < 3 * H * W:
        raise ValueError("rho must be a contiguous float32 buffer of at least 3*H*W values")
    need = _size(lib.gdgs_raster_workspace_size, K)
    ws = ws if ws is not None else workspace(need, dev)
    L.check(lib.gdgs_raster_laplacian(ctypes.byref(_proj_struct(proj)), L.ptr(opacity),
                                      L.ptr(lap), K, ctypes.byref(_bins_struct(bins)), W, H,
                                      L.ptr(rho), L.ptr(ws), ws.numel(), L.stream_handle(stream)))
    return rho


def gdgs_raster_laplacian_threshold(proj: dict, opacity: torch.Tensor, lap: torch.Tensor, K: int,
                                    bins: dict, W: int, H: int, t: float,
                                    rho: torch.Tensor | None = None, count: bool = True,
                                    ws: torch.Tensor | None = None, stream=None):
    """Three-channel composite with the hard threshold of Eq. 24 fused in:
    (rho [3][H][W], device int64 count of the kept non-zero values or None)."""
    lib = L.load()
    dev = bins["ranges"].device
    _need(opacity, (K,), F32, "opacity")
    _need(lap, (3, K), F32, "lap")
    rho = rho if rho is not None else torch.empty((3, H, W), dtype=F32, device=dev)
    if rho.dtype != F32 or not rho.is_contiguous() or rho.numel() < 3 * H * W:
        raise ValueError("rho must be a contiguous float32 buffer of at least 3*H*W values")
    nz = torch.zeros(1, dtype=torch.int64, device=dev) if count else None
    need = _size(lib.gdgs_raster_workspace_size, K)
    ws = ws if ws is not None else workspace(need, dev)
    L.check(lib.gdgs_raster_laplacian_threshold(
        ctypes.byref(_proj_struct(proj)), L.ptr(opacity), L.ptr(lap), K,
        ctypes.byref(_bins_struct(bins)), W, H, float(t), L.ptr(rho), L.ptr(nz), L.ptr(ws),
        ws.numel(), L.stream_handle(stream)))
    return rho, nz


def gdgs_render_laplacian_sparse(scene: DeviceScene, cam, boundary: torch.Tensor | None,
                                 t: float = 0.0, mg=None, capacity: int | None = None, u=None,
                                 stats=None, ws=None, sync_stats=False, count: bool = True,
                                 stream=None):
    """gdgs_render_laplacian with the threshold of Eq. 24 fused into the
    compositing and a set-up that skips tiles without splats: (u, stats,
    device int64 non-zero count or None)."""
    lib = L.load()
    dev = scene.opacity.device
    W, H = int(cam.W), int(cam.H)
    mg = mg if mg is not None else mg_params()
    capacity = int(capacity if capacity is not None else max(1 << 16, 16 * scene.K))
    if boundary is not None:
        _need(boundary, (3, H, W), F32, "boundary")
    u = u if u is not None else torch.empty((3, H, W), dtype=F32, device=dev)
    _need(u, (3, H, W), F32, "u")
    stats = stats if stats is not None else new_stats(dev)
    nz = torch.zeros(1, dtype=torch.int64, device=dev) if count else None
    if ws is None:
        ws = workspace(render_workspace_size(scene.K, W, H, capacity, mg), dev)
    c = camera_struct(cam)
    L.check(lib.gdgs_render_laplacian_sparse(ctypes.byref(scene.struct(3)), ctypes.byref(c),
                                             L.ptr(boundary), ctypes.byref(mg), capacity,
                                             float(t), L.ptr(u), L.ptr(stats), L.ptr(nz),
                                             1 if sync_stats else 0, L.ptr(ws), ws.numel(),
                                             L.stream_handle(stream)))
    return u, stats, nz


def gdgs_render_laplacian(scene: DeviceScene, cam, boundary: torch.Tensor | None, mg=None,
                          capacity: int | None = None, u=None, stats=None, ws=None,
                          sync_stats=False, stream=None):
    """gdgs_render for a scene of Laplacian splats (scene.value is [3][K])."""
    lib = L.load()
    dev = scene.opacity.device
    W, H = int(cam.W), int(cam.H)
    mg = mg if mg is not None else mg_params()
    capacity = int(capacity if capacity is not None else max(1 << 16, 16 * scene.K))
    if boundary is not None:
        _need(boundary, (3, H, W), F32, "boundary")
    u = u if u is not None else torch.empty((3, H, W), dtype=F32, device=dev)
    _need(u, (3, H, W), F32, "u")
    stats = stats if stats is not None else new_stats(dev)
    if ws is None:
        ws = workspace(render_workspace_size(scene.K, W, H, capacity, mg), dev)
    c = camera_struct(cam)
    L.check(lib.gdgs_render_laplacian(ctypes.byref(scene.struct(3)), ctypes.byref(c),
                                      L.ptr(boundary), ctypes.byref(mg), capacity, L.ptr(u),
                                      L.ptr(stats), 1 if sync_stats else 0, L.ptr(ws),
                                      ws.numel(), L.stream_handle(stream)))
    return u, stats


def set_kernel_timer(name: str | None, starts=None, stops=None):
    """Bracket launches of a named library kernel with torch CUDA events
    (see gdgs_set_kernel_timer).  starts/stops: equal-length lists of
    torch.cuda.Event(enable_timing=True); name None clears every timer."""
    lib = L.load()
    if name is None:
        L.check(lib.gdgs_set_kernel_timer(None, None, None, 0))
        return
    n = len(starts)
    for e in list(starts) + list(stops):
        if e.cuda_event == 0:
            e.record()          # create the underlying event
    torch.cuda.synchronize()
    A = (ctypes.c_void_p * n)(*[e.cuda_event for e in starts])
    B = (ctypes.c_void_p * n)(*[e.cuda_event for e in stops])
    set_kernel_timer._keep = getattr(set_kernel_timer, "_keep", {})
    set_kernel_timer._keep[name] = (A, B)   # the library keeps the pointers
    L.check(lib.gdgs_set_kernel_timer(name.encode(), A, B, n))


def set_channel_streams(enable: bool):
    """Run each colour channel's V-cycles on a helper stream of its own (the
    default) or every multigrid launch over all three channels on the
    caller's stream (see gdgs_set_channel_streams); results are the same."""
    L.load().gdgs_set_channel_streams(1 if enable else 0)


def set_kernel_timer_repeats(name: str, repeats: int):
    """Issue each timed launch of an armed multigrid post pass ("mg_post_fine",
    "mg_post_coarse") `repeats` times between its events (see
    gdgs_set_kernel_timer_repeats); results are unchanged."""
    L.check(L.load().gdgs_set_kernel_timer_repeats(name.encode(), int(repeats)))


def rewind_kernel_timers():
    """Start every armed kernel timer at its first event pair again."""
    L.load().gdgs_rewind_kernel_timers()


def kernel_timer_count(name: str) -> int:
    """Launches of `name` bracketed since arming or the last rewind."""
    return int(L.load().gdgs_kernel_timer_count(name.encode()))


def gdgs_raster_count(proj: dict, opacity: torch.Tensor, value: torch.Tensor, K: int, bins: dict,
                      W: int, H: int, ws: torch.Tensor | None = None, stream=None) -> int:
    """Number of (pixel, splat) contributions of the composite (profiling)."""
    lib = L.load()
    dev = bins["ranges"].device
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    need = _size(lib.gdgs_raster_workspace_size, K)
    ws = ws if ws is not None else workspace(need, dev)
    L.check(lib.gdgs_raster_count(ctypes.byref(_proj_struct(proj)), L.ptr(opacity), L.ptr(value),
                                  K, ctypes.byref(_bins_struct(bins)), W, H, L.ptr(counts),
                                  L.ptr(ws), ws.numel(), L.stream_handle(stream)))
    return int(counts[0].item())


def gdgs_div_adjoint(lam: torch.Tensor, W: int, H: int, dgrad=None, stream=None,
                     neumann: bool = False) -> torch.Tensor:
    lib = L.load()
    _need(lam, (3, H, W), F32, "lam")
    dgrad = dgrad if dgrad is not None else torch.empty((6, H, W), dtype=F32, device=lam.device)
    _need(dgrad, (6, H, W), F32, "dgrad")
    fn = lib.gdgs_div_adjoint_neumann if neumann else lib.gdgs_div_adjoint
    L.check(fn(L.ptr(lam), W, H, L.ptr(dgrad), L.stream_handle(stream)))
    return dgrad


def gdgs_raster_grad_backward(proj: dict, opacity: torch.Tensor, value: torch.Tensor, K: int,
                              bins: dict, W: int, H: int, grad: torch.Tensor,
                              dgrad: torch.Tensor, ws=None, stream=None) -> dict:
    lib = L.load()
    dev = grad.device
    _need(grad, (6, H, W), F32, "grad")
    _need(dgrad, (6, H, W), F32, "dgrad")
    out = dict(mean2d=torch.empty((2, K), dtype=F32, device=dev),
               conic=torch.empty((3, K), dtype=F32, device=dev),
               opacity=torch.empty(K, dtype=F32, device=dev),
               value=torch.empty((6, K), dtype=F32, device=dev))
    need = _size(lib.gdgs_raster_backward_workspace_size, K, bins["capacity"])
    ws = ws if ws is not None else workspace(need, dev)
    L.check(lib.gdgs_raster_grad_backward(
        ctypes.byref(_proj_struct(proj)), L.ptr(opacity), L.ptr(value), K,
        ctypes.byref(_bins_struct(bins)), W, H, L.ptr(grad), L.ptr(dgrad), L.ptr(out["mean2d"]),
        L.ptr(out["conic"]), L.ptr(out["opacity"]), L.ptr(out["value"]), L.ptr(ws), ws.numel(),
        L.stream_handle(stream)))
    return out


class Renderer:
    """Plain per-request render path for one scene and image size.

    Owns every buffer and workspace, so a frame allocates nothing.  A frame
    runs the four library steps (project, bin_sort, raster_grad,
    poisson_solve) on the current stream, then reads the device statistics:
      * on a pair-capacity overflow the buffers grow to the reported count and
        the frame is redone;
      * the V-cycle budget of a frame is the cycle count the previous frame
        needed (consecutive views need about the same), so converged channels
        do not leave idle cycles behind; if a frame has not met the tolerance
        within its budget the solve continues from its current iterate
        (GDGS_MG_RESUME) until it does or the limit max_cycles is reached; the
        result is therefore the same whatever the budget was.
    """

    def __init__(self, scene: DeviceScene, W: int, H: int, mg=None, capacity: int | None = None,
                 adaptive: bool = True, warm_start: bool = False, threshold: float = 0.0,
                 neumann: bool = False):
        self.scene, self.W, self.H = scene, int(W), int(H)
        # threshold (Laplacian form only): the hard threshold of Eq. 24 applied
        # to the composited Laplacian before the solve; the non-zero count of
        # each frame is kept in self.nonzero (device)
        self.threshold = float(threshold)
        self.nonzero = None
        # warm_start: each frame's solve starts from the previous frame's image
        # (GDGS_MG_WARM_START) instead of zero; for consecutive views of a
        # moving camera it needs fewer V-cycles to the same tolerance
        self.warm_start = warm_start
        self._prev_u = None
        # six values per splat: gradient splats; three: Laplacian splats
        # (Sec. 2.2), whose composite is the right-hand side itself
        if scene.nch not in (3, 6):
            raise ValueError("scene.value must have 6 (gradient) or 3 (Laplacian) rows")
        self.laplacian = scene.nch == 3
        if self.threshold > 0.0 and not self.laplacian:
            raise ValueError("the threshold applies to the Laplacian form")
        self.mg = mg if mg is not None else mg_params()
        # neumann: the paper's boundary condition (GDGS_MG_NEUMANN) instead of
        # Dirichlet data on the image ring; boundary must then be None
        self.neumann = bool(neumann) or bool(self.mg.flags & NEUMANN)
        self.max_cycles = int(self.mg.max_cycles)
        self.budget = self.max_cycles
        self.adaptive = adaptive
        self.dev = scene.opacity.device
        K = scene.K
        self.stats = new_stats(self.dev)
        self.u = torch.empty((3, self.H, self.W), dtype=F32, device=self.dev)
        self.grad = torch.empty((6, self.H, self.W), dtype=F32, device=self.dev)
        self.proj = alloc_proj(K, self.dev)
        lib = L.load()
        self.ws_ras = workspace(_size(lib.gdgs_raster_workspace_size, K), self.dev)
        self.ws_poi = workspace(_size(lib.gdgs_poisson_workspace_size, self.W, self.H,
                                      ctypes.byref(self._mg(self.max_cycles))), self.dev)
        self._set_capacity(capacity if capacity is not None else max(1 << 16, 16 * K))
        self.last = None

    def _set_capacity(self, cap: int):
        lib = L.load()
        self.capacity = int(cap)
        self.bins = alloc_bins(self.scene.K, self.W, self.H, self.capacity, self.dev)
        self.ws_bin = workspace(_size(lib.gdgs_bin_sort_workspace_size, self.scene.K, self.W,
                                      self.H, self.capacity), self.dev)

    def _mg(self, cycles: int, flags: int = 0) -> L.MgParams:
        m = self.mg
        keep = (m.flags & (FMG | STOP_ETA)) | (NEUMANN if self.neumann else 0)
        return mg_params(m.levels, m.pre_sweeps, m.post_sweeps, cycles, m.tol, m.coarse_sweeps,
                         flags | keep, m.smooth_weight)

    def _enqueue(self, cam, boundary, events, stream):
        """Enqueue one frame (no waiting): the four steps, then an asynchronous
        copy of its statistics and pair count to pinned host memory."""
        s = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self._enqueue_front(cam, events, s)
        self._enqueue_solve(boundary, events, s)

    def _host_buffers(self):
        if not hasattr(self, "_h_stats"):
            self._h_stats = torch.empty(STATS_BYTES, dtype=torch.uint8, pin_memory=True)
            self._h_pairs = torch.empty(1, dtype=torch.int64, pin_memory=True)
            self._done = torch.cuda.Event()

    def _enqueue_front(self, cam, events, s):
        """Projection, binning and compositing of one frame on stream s."""
        K, W, H = self.scene.K, self.W, self.H
        self._host_buffers()
        rec = (lambda i: events[i].record(s)) if events else (lambda i: None)
        rec(0)
        gdgs_project(self.scene, cam, self.proj, s)
        rec(1)
        gdgs_bin_sort(self.proj, K, W, H, self.capacity, self.bins, self.ws_bin, s)
        rec(2)
        if self.laplacian and self.threshold > 0.0:
            # Eq. 24 fused into the compositing kernel
            _, self.nonzero = gdgs_raster_laplacian_threshold(
                self.proj, self.scene.opacity, self.scene.value, K, self.bins, W, H,
                self.threshold, self.grad, ws=self.ws_ras, stream=s)
        elif self.laplacian:
            gdgs_raster_laplacian(self.proj, self.scene.opacity, self.scene.value, K, self.bins,
                                  W, H, self.grad, self.ws_ras, s)
        else:
            gdgs_raster_grad(self.proj, self.scene.opacity, self.scene.value, K, self.bins, W, H,
                             self.grad, self.ws_ras, s)
        rec(3)

    def _enqueue_solve(self, boundary, events, s):
        """The Poisson solve of the composited frame on stream s, then the
        copies of its statistics and pair count to pinned host memory."""
        self._host_buffers()
        rec = (lambda i: events[i].record(s)) if events else (lambda i: None)
        flags = 0
        if self.warm_start and self._prev_u is not None:
            if self._prev_u is not self.u:
                with torch.cuda.stream(s):
                    self.u.copy_(self._prev_u, non_blocking=True)
            flags = WARM_START
        self._solve(boundary, self._mg(self.budget, flags), s)
        rec(4)
        with torch.cuda.stream(s):
            self._h_stats.copy_(self.stats, non_blocking=True)
            self._h_pairs.copy_(self.bins["num_pairs"], non_blocking=True)
        self._done.record(s)

    def _finish(self, cam, boundary, events, stream) -> torch.Tensor:
        """Wait for the enqueued frame (only it) and settle it: a pair overflow
        grows the buffers and renders the frame again; an unconverged solve
        is resumed."""
        self._done.synchronize()
        raw = bytes(self._h_stats.numpy().tobytes())
        sr = L.Stats.from_buffer_copy(raw)
        st = dict(cycles=list(sr.cycles), converged=bool(sr.converged), eta=list(sr.eta),
                  rel_res=list(sr.rel_res), b_norm=list(sr.b_norm), delta=list(sr.delta))
        pairs = int(self._h_pairs[0])
        if pairs > self.capacity:
            self._extra = True   # the frame is rendered again after its first solve
            self._set_capacity(int(pairs * 1.25) + 1024)
            self.budget = self.max_cycles
            return self.render(cam, boundary, events, stream)
        total = max(st["cycles"])
        s = stream if stream is not None else torch.cuda.current_stream(self.dev)
        while not st["converged"] and total < self.max_cycles:
            self._extra = True   # resumed cycles follow the frame's first solve
            step = min(2, self.max_cycles - total)
            self._solve(boundary, self._mg(step, RESUME), s)
            # the resumed cycles run on s, which the current stream need not
            # follow: wait for s itself before reading the statistics
            s.synchronize()
            st = read_stats(self.stats)
            total = max(st["cycles"])     # cycle counts accumulate over resumed calls
        st["total_cycles"] = total
        st["num_pairs"] = pairs
        self._prev_u = self.u
        if self.adaptive:
            self.budget = max(1, min(self.max_cycles, total))
        self.last = st
        return self.u

    def _solve(self, boundary, mg, stream):
        if self.laplacian:  # the first three planes hold rho
            gdgs_poisson_solve_rhs(self.grad[:3], boundary, self.W, self.H, mg, self.u,
                                   self.stats, self.ws_poi, stream)
        else:
            gdgs_poisson_solve(self.grad, boundary, self.W, self.H, mg, self.u, self.stats,
                               self.ws_poi, stream)

    def render(self, cam, boundary=None, events=None, stream=None) -> torch.Tensor:
        self._enqueue(cam, boundary, events, stream)
        return self._finish(cam, boundary, events, stream)

    def render_sequence(self, cams, boundary=None, events=None, on_frame=None, stream=None,
                        overlap=False):
        """Render views one after another without the host waiting in between:
        frame i + 1 is enqueued before frame i is settled.  Two buffer sets
        alternate (this renderer and a twin), so frame i's result stays intact
        until on_frame(i, u, stats) has seen it; results equal render()'s.
        With warm_start, frame i starts from frame i - 1's image as it stands
        when frame i is enqueued (before any resumed cycles of frame i - 1),
        so results meet the same tolerance but may differ from render()'s in
        the last bits.

        overlap (without warm_start): two frames in flight.  Each frame's
        projection, binning and compositing run on the caller's stream and
        its solve on one solve stream of this renderer (plus the two channel
        streams the library binds to it: four streams in all, the hardware
        queues a process gets), so one frame's front half runs beside the
        previous frame's solve; results are unchanged.  A buffer set's next
        front half waits for its previous solve (resumed cycles included),
        and work that on_frame(i) enqueues on the caller's stream follows
        frame i's solve."""
        if not hasattr(self, "_twin"):
            self._twin = Renderer(self.scene, self.W, self.H, self.mg, self.capacity,
                                  self.adaptive, self.warm_start, self.threshold, self.neumann)
        rs = [self, self._twin]
        caller = stream if stream is not None else torch.cuda.current_stream(self.dev)
        if overlap and not self.warm_start:
            self._sequence_overlap(rs, cams, boundary, events, on_frame, caller)
            return
        prev = None
        for i, cam in enumerate(cams):
            r = rs[i % 2]
            if prev is not None:
                r.budget = prev[0].budget
                if self.warm_start:
                    r._prev_u = prev[0].u
            r._enqueue(cam, boundary, events[i] if events else None, stream)
            if prev is not None:
                pr, pcam, pi = prev
                u = pr._finish(pcam, boundary, events[pi] if events else None, stream)
                r.budget = max(r.budget, pr.budget)
                if on_frame is not None:
                    on_frame(pi, u, pr.last)
            prev = (r, cam, i)
        if prev is not None:
            pr, pcam, pi = prev
            u = pr._finish(pcam, boundary, events[pi] if events else None, stream)
            self.budget = self._twin.budget = pr.budget
            if on_frame is not None:
                on_frame(pi, u, pr.last)

    def _sequence_overlap(self, rs, cams, boundary, events, on_frame, C):
        if not hasattr(self, "_solve_stream"):
            self._solve_stream = torch.cuda.Stream(device=self.dev)
        P = self._solve_stream
        for r in rs:
            r._host_buffers()
            if not hasattr(r, "_fronted"):
                r._fronted = torch.cuda.Event()
                r._solved = torch.cuda.Event()
            r._in_flight = False
            r._settled = None
        P.wait_stream(C)   # the solves follow the caller's earlier work

        def settle(pr, pcam, pi):
            # The frame's own done event marks the end of its solve; when the
            # settling adds work (resumed cycles or a re-render, queued on P
            # behind the next frame's solve), a new event after that work.
            pr._extra = False
            u = pr._finish(pcam, boundary, events[pi] if events else None, P)
            if pr._extra:
                pr._solved.record(P)
                pr._settled = pr._solved
            else:
                pr._settled = pr._done
            C.wait_event(pr._settled)   # on_frame's work follows the frame
            if on_frame is not None:
                on_frame(pi, u, pr.last)

        prev = None
        for i, cam in enumerate(cams):
            r = rs[i % 2]
            ev = events[i] if events else None
            if prev is not None:
                r.budget = prev[0].budget
            if r._in_flight:
                C.wait_event(r._settled)  # the set's previous frame is done with its buffers
            r._enqueue_front(cam, ev, C)
            r._fronted.record(C)
            P.wait_event(r._fronted)
            r._enqueue_solve(boundary, ev, P)
            r._in_flight = True
            if prev is not None:
                pr, pcam, pi = prev
                settle(pr, pcam, pi)
                r.budget = max(r.budget, pr.budget)
            prev = (r, cam, i)
        if prev is not None:
            pr, pcam, pi = prev
            settle(pr, pcam, pi)
            self.budget = self._twin.budget = pr.budget
        C.wait_stream(P)
