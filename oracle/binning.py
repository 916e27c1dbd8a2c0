"""Tile binning and the compositing order, as plain definitions (test oracle).

The paper only requires that splats be composited in order along the view
direction (Sec. 1.2, the sentence after Eq. 11).  The rasteriser orders work
by 16x16 screen tiles; its expected output is defined here directly:

* a splat produces one (tile, splat) pair for every tile that intersects its
  pixel support box (see ``project.pixel_box``);
* the pairs are ordered lexicographically by (tile id, FP32 depth, splat
  index), tile id = ty * ceil(W / 16) + tx;
* tile t's pairs occupy the half-open range [start_t, end_t).
"""
from __future__ import annotations

import numpy as np

from .constants import TILE


def tiles_x(W: int) -> int:
    return (W + TILE - 1) // TILE


def emit_pairs(proj: dict, W: int):
    """All (tile id, splat index) pairs, in splat-index order."""
    tx0, tx1, ty0, ty1 = proj["tile_rect"]
    nx = tiles_x(W)
    tiles, splats = [], []
    for k in np.nonzero(proj["count"] > 0)[0]:
        ty, tx = np.meshgrid(np.arange(ty0[k], ty1[k]), np.arange(tx0[k], tx1[k]), indexing="ij")
        t = (ty * nx + tx).ravel()
        tiles.append(t)
        splats.append(np.full(t.size, k))
    if not tiles:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(tiles).astype(np.int64), np.concatenate(splats).astype(np.int64)


def depth_bits(depth) -> np.ndarray:
    """IEEE-754 bit pattern of the FP32-rounded depth, as unsigned integers
    (for positive depths their integer order is the numeric order)."""
    return np.asarray(depth, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.int64)


def sorted_pairs(proj: dict, W: int):
    """Pairs sorted by (tile, FP32 depth, splat index): (tiles, splats)."""
    tiles, splats = emit_pairs(proj, W)
    order = np.lexsort((splats, depth_bits(proj["depth"])[splats], tiles))
    return tiles[order], splats[order]


def tile_ranges(sorted_tiles: np.ndarray, num_tiles: int):
    """[start, end) of every tile in a sorted tile-id array."""
    t = np.arange(num_tiles)
    start = np.searchsorted(sorted_tiles, t, side="left")
    end = np.searchsorted(sorted_tiles, t, side="right")
    return start, end
