"""Helpers for the GPU parity tests: run the library's steps on seeded
workloads and bring results back as numpy arrays."""
from __future__ import annotations

import sys

import numpy as np
import torch

import paper_2405_05446_amd as G
import workloads as wl


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def np_(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def u32(t: torch.Tensor) -> np.ndarray:
    return np_(t).view(np.uint32)


def gpu_stages(scene: wl.Scene, cam: wl.Camera, capacity: int | None = None):
    """project -> bin_sort -> raster_grad on the GPU; numpy results."""
    K, W, H = scene.K, cam.W, cam.H
    ds = G.DeviceScene.from_host(scene)
    proj = G.gdgs_project(ds, cam)
    cap = capacity if capacity is not None else max(4096, 16 * K)
    bins = G.gdgs_bin_sort(proj, K, W, H, cap)
    grad = G.gdgs_raster_grad(proj, ds.opacity, ds.value, K, bins, W, H)
    torch.cuda.synchronize()
    P = int(np_(bins["num_pairs"])[0])
    n = min(P, cap)
    rect = u32(proj["rect"])
    out = dict(
        mean2d_rel=np_(proj["mean2d"]).astype(np.float64), conic=np_(proj["conic"]),
        depth=np_(proj["depth"]), rect=rect, count=u32(proj["count"]),
        tx0=(rect[0] & 0xFFFF).astype(np.int64), tx1=(rect[0] >> 16).astype(np.int64),
        ty0=(rect[1] & 0xFFFF).astype(np.int64), ty1=(rect[1] >> 16).astype(np.int64),
        num_pairs=P, tiles=u32(bins["tile_of_pair"])[:n].astype(np.int64),
        splats=u32(bins["splat_of_pair"])[:n].astype(np.int64),
        order=u32(bins["order"])[:K].astype(np.int64), ranges=u32(bins["ranges"]),
        tile_order=u32(bins["tile_order"]).astype(np.int64),
        grad=np_(grad).astype(np.float64))
    out["mean2d"] = np.stack([out["mean2d_rel"][0] + 16 * out["tx0"],
                              out["mean2d_rel"][1] + 16 * out["ty0"]])
    return out


def fp32_ulp_diff(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    ia = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(ia - ib)
