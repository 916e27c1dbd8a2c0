"""Sparse compositing (Sec. 2.2 "Projection": the projected Laplacian field of
Eq. 20 is sparse; Sec. 3.1, Eq. 24: hard threshold) on the GPU through the C
ABI: the threshold fused into the compositing kernel against the separate
threshold pass and the oracle, the sparse render (fused threshold, set-up
that skips tiles without splats) against the dense render and the oracle,
and the paper-like sparse workload (1920x1080, 5,100 Laplacian splats)."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
import workloads as wl
from oracle import composite as oc, poisson as P
from oracle.project import project as oproject
from oracle.render import render_laplacian as orender_lap, threshold as othreshold
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _stages(sc, cam, cap=None):
    ds = G.DeviceScene.from_host(sc)
    K, W, H = sc.opacity.shape[0], cam.W, cam.H
    proj = G.gdgs_project(ds, cam)
    bins = G.gdgs_bin_sort(proj, K, W, H, cap or max(4096, 16 * K))
    return ds, proj, bins


@pytest.mark.parametrize("W,H,t", [(100, 72, 0.0), (100, 72, 0.004), (333, 190, 0.01)])
def test_fused_threshold_equals_separate_pass_and_oracle(W, H, t):
    say(f"[sparse] fused threshold {W}x{H} t={t}")
    sc = wl.laplacian_scene(wl.make_scene(4000, seed=2, ls=(-3, 0.6)), seed=0)
    cam = wl.make_camera(W, H, pose_index=4)
    ds, proj, bins = _stages(sc, cam)
    K = sc.opacity.shape[0]
    rho = G.api.gdgs_raster_laplacian(proj, ds.opacity, ds.value, K, bins, W, H)
    sep = rho.clone()
    nz_sep = G.api.gdgs_threshold(sep, t)
    fused, nz = G.api.gdgs_raster_laplacian_threshold(proj, ds.opacity, ds.value, K, bins, W, H, t)
    torch.cuda.synchronize()
    assert torch.equal(fused, sep) and int(nz.item()) == int(nz_sep.item())
    # the decision on the same FP32 values as the oracle's threshold of Eq. 24
    r32 = np_(rho)
    assert np.array_equal(np_(fused), othreshold(r32, np.float32(t)))
    # and the composite itself against brute force
    ref = oc.render_grad(oproject(sc, cam), sc.opacity, sc.value, H, W)
    assert np.abs(r32 - ref).max() <= TOL
    assert int(nz.item()) == int(np.count_nonzero(np_(fused)))


@pytest.mark.parametrize("t", [0.0, 0.004])
def test_sparse_render_matches_oracle(t):
    W, H = 64, 48
    say(f"[sparse] render vs oracle {W}x{H} t={t}")
    sc = wl.laplacian_scene(wl.make_scene(1500, seed=3, ls=(-3, 0.6)), seed=1)
    cam = wl.make_camera(W, H, pose_index=2)
    ring = wl.reference_image(H, W, seed=1).astype(np.float32)
    ds = G.DeviceScene.from_host(sc)
    u, st, nz = G.api.gdgs_render_laplacian_sparse(ds, cam, torch.from_numpy(ring).cuda(), t,
                                                   G.mg_params(tol=1e-6, max_cycles=40),
                                                   sync_stats=True)
    torch.cuda.synchronize()
    o = orender_lap(sc, cam, ring.astype(np.float64), t=t)
    err = np.abs(np_(u) - o["u"]).max()
    say(f"  max-abs {err:.3e}, non-zero {int(nz.item())} (oracle {np.count_nonzero(o['rho'])})")
    assert err <= TOL and G.read_stats(st)["converged"]


def test_sparse_workload_stagewise_and_equal_to_the_dense_path():
    """1920x1080, 5,100 Laplacian splats: the sparse render equals the dense
    render bit for bit without a threshold and the Renderer's thresholded path
    with one; composite on sampled pixels vs brute force; the solve of the
    thresholded field vs the exact DST-I solve; the threshold decided on the
    kernel's own FP32 values."""
    cfg = wl.CONFIGS["sparse"]
    W, H, K = cfg["W"], cfg["H"], cfg["K"]
    say(f"[sparse] workload {W}x{H}, {K} splats")
    sc = wl.laplacian_scene(wl.make_scene(K, seed=0, z=cfg["z"], ls=cfg["ls"]), seed=0)
    cam = wl.make_camera(W, H, pose_index=0)
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    ds = G.DeviceScene.from_host(sc)
    mg = G.mg_params(levels=cfg["levels"], tol=cfg["tol"])
    dense, _ = G.gdgs_render_laplacian(ds, cam, ring, mg, sync_stats=True)
    sparse0, _, _ = G.api.gdgs_render_laplacian_sparse(ds, cam, ring, 0.0, mg, sync_stats=True)
    torch.cuda.synchronize()
    assert torch.equal(dense, sparse0)
    t = 0.004
    r = G.Renderer(ds, W, H, mg, threshold=t)
    want = r.render(cam, ring).clone()
    u, st, nz = G.api.gdgs_render_laplacian_sparse(ds, cam, ring, t, mg, sync_stats=True)
    torch.cuda.synchronize()
    assert torch.equal(u, want) and int(nz.item()) == int(r.nonzero.item())
    # stage-wise against the oracle
    ds_, proj, bins = _stages(sc, cam)
    rho = G.api.gdgs_raster_laplacian(proj, ds_.opacity, ds_.value, K, bins, W, H)
    fused, nz2 = G.api.gdgs_raster_laplacian_threshold(proj, ds_.opacity, ds_.value, K, bins,
                                                      W, H, t)
    torch.cuda.synchronize()
    r32 = np_(rho)
    assert np.array_equal(np_(fused), othreshold(r32, np.float32(t)))
    o = oproject(sc, cam)
    rows, cols = wl.sample_pixels(H, W, 1500, seed=17)
    ref = oc.render_grad(o, sc.opacity, sc.value, H, W, rows, cols)
    e1 = np.abs(r32[:, rows, cols] - ref).max()
    exact = P.solve(np_(fused).astype(np.float64), np_(ring).astype(np.float64))
    e2 = np.abs(np_(u) - exact).max()
    ranges = np_(bins["ranges"]).view(np.uint32)
    live = float(np.mean(ranges[1] > ranges[0]))
    say(f"  composite max-abs {e1:.3e}, solve max-abs {e2:.3e}, non-zero "
        f"{int(nz.item()) / (3 * H * W):.4f} of rho, tiles with splats {live:.3f}")
    assert e1 <= TOL and e2 <= TOL and G.read_stats(st)["converged"]
    assert int(nz2.item()) == int(nz.item())
