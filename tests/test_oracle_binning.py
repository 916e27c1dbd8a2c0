"""Pins of the oracle's tile binning and ordering definition."""
import numpy as np

import workloads as wl
from oracle import binning as ob
from oracle.constants import E_CUT, TILE
from oracle.project import project


def test_sorted_pairs_match_bruteforce_tuple_sort():
    sc = wl.make_scene(300, seed=6, ls=(-2.5, 0.6))
    cam = wl.make_camera(100, 72)
    p = project(sc, cam)
    tiles, splats = ob.emit_pairs(p, 100)
    d32 = p["depth"].astype(np.float32)
    ref = sorted(zip(tiles.tolist(), [float(d32[k]) for k in splats], splats.tolist()))
    st, ss = ob.sorted_pairs(p, 100)
    assert [(t, k) for t, _, k in ref] == list(zip(st.tolist(), ss.tolist()))
    assert tiles.size == p["count"].sum()


def test_every_supported_tile_is_emitted():
    sc = wl.make_scene(250, seed=8, ls=(-2.2, 0.5))
    W, H = 90, 50
    cam = wl.make_camera(W, H)
    p = project(sc, cam)
    tiles, splats = ob.emit_pairs(p, W)
    have = set(zip(tiles.tolist(), splats.tolist()))
    nx = ob.tiles_x(W)
    py, px = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    needed = 0
    for k in np.nonzero(p["valid"])[0]:
        a, b, c = p["conic"][:, k]
        dx = px - p["mean2d"][0, k]
        dy = py - p["mean2d"][1, k]
        ii, jj = np.nonzero(a * dx * dx + 2 * b * dx * dy + c * dy * dy <= E_CUT)
        for t in set(((ii // TILE) * nx + jj // TILE).tolist()):
            needed += 1
            assert (t, k) in have
    assert needed > 100


def test_tile_ranges_partition_the_sorted_pairs():
    sc = wl.make_scene(200, seed=9, ls=(-2.5, 0.6))
    W, H = 70, 40
    p = project(sc, wl.make_camera(W, H))
    st, _ = ob.sorted_pairs(p, W)
    T = ob.tiles_x(W) * ((H + TILE - 1) // TILE)
    start, end = ob.tile_ranges(st, T)
    assert (end - start).sum() == st.size
    for t in range(T):
        assert (st[start[t]:end[t]] == t).all()


def test_depth_bits_order_is_numeric_order_for_positive_depths():
    rng = np.random.default_rng(1)
    d = rng.uniform(0.2, 50, 1000)
    bits = ob.depth_bits(d)
    assert (np.argsort(bits, kind="stable") == np.argsort(d.astype(np.float32), kind="stable")).all()
