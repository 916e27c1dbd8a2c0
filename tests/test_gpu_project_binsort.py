"""GPU parity of projection and tile binning/sorting against the oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import binning as ob
from oracle.project import project as oproject
from oracle.constants import E_CUT
from tests.gpu_util import gpu_stages, say, fp32_ulp_diff

pytestmark = pytest.mark.gpu

CASES = [
    ("tiny", dict(K=2000, W=64, H=64, z=(2, 6), ls=(-4, 0.5), pose=None)),
    ("ragged", dict(K=3000, W=100, H=72, z=(2, 6), ls=(-3, 0.6), pose=3)),
    ("wide", dict(K=20000, W=333, H=190, z=(2, 20), ls=(-4, 0.7), pose=7)),
]
# the sort alone at the mid and full sizes: hundreds of 2048-key tiles in the
# depth sort and thousands in the pair sort, so every pass's look-back walks
# across many tiles
SORT_CASES = CASES + [
    ("mid", dict(K=200_000, W=800, H=800, z=(2, 6), ls=(-4, 0.5), pose=2)),
    ("full", dict(K=1_000_000, W=1920, H=1080, z=(2, 20), ls=(-5, 0.7), pose=5)),
]


def _boundary_fluke(o, k):
    """True if splat k's FP64 support-box edge lies within 1e-9 of an integer,
    where FP64 rounding order may move the edge by one pixel."""
    mx, my = o["mean2d"][:, k]
    sxx, _, syy = o["cov2d"][:, k]
    rx, ry = np.sqrt(E_CUT * sxx), np.sqrt(E_CUT * syy)
    edges = np.array([mx - rx - 0.5, mx + rx - 0.5, my - ry - 0.5, my + ry - 0.5])
    return bool(np.any(np.abs(edges - np.round(edges)) < 1e-9 * np.maximum(1, np.abs(edges))))


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
def test_project_matches_oracle(name, cfg):
    say(f"[project] {name} {cfg}")
    sc = wl.make_scene(cfg["K"], seed=0, z=cfg["z"], ls=cfg["ls"])
    cam = wl.make_camera(cfg["W"], cfg["H"], pose_index=cfg["pose"])
    g = gpu_stages(sc, cam)
    o = oproject(sc, cam)
    # integer outputs: bit-exact except FP64 rounding flukes at a pixel edge
    bad = np.nonzero(g["count"] != o["count"])[0]
    assert all(_boundary_fluke(o, k) for k in bad), bad[:10]
    live = np.nonzero((g["count"] > 0) & (o["count"] > 0))[0]
    assert live.size > 0.3 * cfg["K"]
    # tile rectangles of every live splat that is not an edge fluke
    sure = np.array([k for k in live if not (k in set(bad.tolist()) or _boundary_fluke(o, k))],
                    dtype=np.int64)
    assert sure.size > 0.9 * live.size
    for w, key in enumerate(("tx0", "tx1", "ty0", "ty1")):
        assert np.array_equal(g[key][sure], o["tile_rect"][w][sure]), key
    assert fp32_ulp_diff(g["depth"][live], o["depth"][live]).max() <= 1
    np.testing.assert_allclose(g["conic"][:, live], o["conic"][:, live], rtol=2e-6, atol=0)
    mrel_o = o["mean2d"][:, live] - 16 * np.stack([o["tile_rect"][0][live], o["tile_rect"][2][live]])
    np.testing.assert_allclose(g["mean2d_rel"][:, live], mrel_o, rtol=1e-6, atol=2e-6)


@pytest.mark.parametrize("name,cfg", SORT_CASES, ids=[c[0] for c in SORT_CASES])
def test_bin_sort_is_bit_exact(name, cfg):
    say(f"[bin_sort] {name} {cfg}")
    sc = wl.make_scene(cfg["K"], seed=1, z=cfg["z"], ls=cfg["ls"])
    cam = wl.make_camera(cfg["W"], cfg["H"], pose_index=cfg["pose"])
    g = gpu_stages(sc, cam)
    W, H, K = cfg["W"], cfg["H"], cfg["K"]
    nx = (W + 15) // 16
    T = nx * ((H + 15) // 16)
    # expected from the GPU's own rectangles and FP32 depths: every tile of
    # each live splat's rectangle, row by row
    live = np.nonzero(g["count"] > 0)[0]
    w = g["tx1"][live] - g["tx0"][live]
    h = g["ty1"][live] - g["ty0"][live]
    cnt = w * h
    splats = np.repeat(live, cnt)
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(splats.size) - first
    wr = np.repeat(w, cnt)
    tiles = ((np.repeat(g["ty0"][live], cnt) + local // wr) * nx
             + np.repeat(g["tx0"][live], cnt) + local % wr)
    say(f"[bin_sort] {name}: {K} splats, {splats.size} pairs, {T} tiles")
    assert g["num_pairs"] == tiles.size == int(g["count"].sum())
    dbits = g["depth"].view(np.uint32).astype(np.int64)
    o = np.lexsort((splats, dbits[splats], tiles))
    assert np.array_equal(g["tiles"], tiles[o])
    assert np.array_equal(g["splats"], splats[o])
    # depth order: permutation, sorted by (count>0 ? depth bits : max, index)
    key = np.where(g["count"] > 0, dbits, 0xFFFFFFFF)
    assert np.array_equal(g["order"], np.lexsort((np.arange(K), key)))
    start, end = ob.tile_ranges(g["tiles"], T)
    nonempty = end > start
    assert np.array_equal(g["ranges"][0][nonempty], start[nonempty])
    assert np.array_equal(g["ranges"][1][nonempty], end[nonempty])
    assert np.all(g["ranges"][1][~nonempty] == g["ranges"][0][~nonempty])
    # heaviest-first schedule: tile ids stably sorted by 32 - bitlen(pairs)
    n = (end - start).astype(np.int64)
    bitlen = np.where(n > 0, np.floor(np.log2(np.maximum(n, 1))).astype(np.int64) + 1, 0)
    assert np.array_equal(g["tile_order"], np.lexsort((np.arange(T), 32 - bitlen)))


@pytest.mark.parametrize("seed,pose", [(2, 1), (4, 6)])
def test_bin_sort_matches_oracle_pairs(seed, pose):
    """The GPU's sorted (tile, splat) pairs equal the oracle's, splat by
    splat: every splat whose support-box edge is not an FP64 rounding fluke
    has the same pairs in the same order on both sides."""
    say(f"[bin_sort vs oracle] seed {seed} pose {pose}")
    sc = wl.make_scene(3000, seed=seed, z=(2, 6), ls=(-3, 0.6))
    cam = wl.make_camera(100, 72, pose_index=pose)
    g = gpu_stages(sc, cam)
    o = oproject(sc, cam)
    ot, os_ = ob.sorted_pairs(o, 100)
    K = sc.K
    fluke = np.array([_boundary_fluke(o, k) for k in range(K)])
    diff = g["count"] != o["count"]
    assert np.all(fluke[diff]), np.nonzero(diff & ~fluke)[0][:10]
    keep = ~fluke
    gm, om = keep[g["splats"]], keep[os_]
    assert gm.sum() > 0.9 * g["splats"].size
    assert np.array_equal(g["tiles"][gm], ot[om])
    assert np.array_equal(g["splats"][gm], os_[om])
