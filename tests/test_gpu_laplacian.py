"""Laplacian-splat form (Sec. 2.2) on the GPU through the C ABI: the
three-channel composite against the oracle's brute force, its channels
against the six-value kernel, the whole render against the oracle, and the
Renderer's per-step path against gdgs_render_laplacian."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
import workloads as wl
from oracle import composite as oc
from oracle.project import project as oproject
from oracle.render import render_laplacian as orender_lap
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.mark.parametrize("K,W,H,pose", [(2000, 64, 64, None), (3000, 100, 72, 3),
                                        (1500, 37, 21, 5)])
def test_composite_matches_oracle_and_gradient_kernel(K, W, H, pose):
    say(f"[laplacian] composite K={K} {W}x{H}")
    sc = wl.laplacian_scene(wl.make_scene(K, seed=0, ls=(-3, 0.6)), seed=0)
    cam = wl.make_camera(W, H, pose_index=pose)
    ds = G.DeviceScene.from_host(sc)
    proj = G.gdgs_project(ds, cam)
    bins = G.gdgs_bin_sort(proj, K, W, H, max(4096, 16 * K))
    rho = G.api.gdgs_raster_laplacian(proj, ds.opacity, ds.value, K, bins, W, H)
    six = torch.zeros((6, K), dtype=torch.float32, device=ds.value.device)
    six[:3] = ds.value
    g6 = G.gdgs_raster_grad(proj, ds.opacity, six, K, bins, W, H)
    torch.cuda.synchronize()
    ref = oc.render_grad(oproject(sc, cam), sc.opacity, sc.value, H, W)
    err = np.abs(np_(rho) - ref).max()
    say(f"  max-abs {err:.3e}")
    assert err <= TOL
    # the three-channel kernel does the same arithmetic as the first three
    # channels of the six-channel one
    assert torch.equal(rho, g6[:3])


def test_render_matches_oracle():
    H, W, K = 45, 70, 800
    sc = wl.laplacian_scene(wl.make_scene(K, seed=3, ls=(-2.5, 0.5)), seed=3)
    cam = wl.make_camera(W, H, pose_index=2)
    ring = wl.reference_image(H, W, seed=1)
    ds = G.DeviceScene.from_host(sc)
    b = torch.from_numpy(ring.astype(np.float32)).cuda()
    u, st = G.api.gdgs_render_laplacian(ds, cam, b, G.mg_params(tol=1e-6, max_cycles=40),
                                        sync_stats=True)
    torch.cuda.synchronize()
    o = orender_lap(sc, cam, ring.astype(np.float32).astype(np.float64))
    s = G.read_stats(st)
    err = np.abs(np_(u) - o["u"]).max()
    say(f"[laplacian] render 70x45 max-abs {err:.3e}, cycles {s['cycles']}")
    assert err <= TOL and s["converged"]


def test_renderer_equals_render_entry_point():
    W, H, K = 320, 180, 20000
    sc = wl.laplacian_scene(wl.make_scene(K, seed=0, z=(2.0, 20.0), ls=(-5.0, 0.7)), seed=0)
    ds = G.DeviceScene.from_host(sc)
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    mg = G.mg_params(tol=1e-6, max_cycles=30)
    r = G.Renderer(ds, W, H, mg)
    assert r.laplacian
    for i in range(3):
        cam = wl.make_camera(W, H, pose_index=i)
        u = r.render(cam, ring).clone()
        u2, st = G.api.gdgs_render_laplacian(ds, cam, ring, mg, capacity=r.capacity,
                                             sync_stats=True)
        torch.cuda.synchronize()
        assert r.last["converged"]
        # same kernels; the resumed path of the Renderer continues bit for bit
        assert (u - u2).abs().max().item() <= 1e-6


def test_threshold_kernel_is_exact_and_counts():
    rng = np.random.default_rng(4)
    x = rng.laplace(0.0, 0.01, 100003).astype(np.float32)
    t = np.float32(0.007)
    g = torch.from_numpy(x).cuda()
    nz = G.api.gdgs_threshold(g, float(t))
    torch.cuda.synchronize()
    ref = np.where(np.abs(x) >= t, x, np.float32(0.0))
    assert np.array_equal(np_(g), ref)
    assert int(nz.item()) == int(np.count_nonzero(ref))


def test_thresholded_laplacian_render_solves_the_sparse_field():
    from oracle import poisson as P
    H, W, K = 60, 90, 3000
    sc = wl.laplacian_scene(wl.make_scene(K, seed=5, ls=(-3, 0.6)), seed=5)
    cam = wl.make_camera(W, H, pose_index=4)
    ds = G.DeviceScene.from_host(sc)
    proj = G.gdgs_project(ds, cam)
    bins = G.gdgs_bin_sort(proj, K, W, H, 16 * K)
    rho = np_(G.api.gdgs_raster_laplacian(proj, ds.opacity, ds.value, K, bins, W, H))
    t = float(np.float32(0.5 * np.abs(rho).mean()))
    r = G.Renderer(ds, W, H, G.mg_params(tol=1e-6, max_cycles=40), threshold=t)
    u = np_(r.render(cam))
    nz = int(r.nonzero.item())
    rho_t = np.where(np.abs(rho) >= np.float32(t), rho, np.float32(0.0))
    ref = P.solve(rho_t.astype(np.float64), None)
    err = np.abs(u - ref).max()
    say(f"[laplacian] threshold {t:.3g}: {nz / rho.size:.2%} non-zero, max-abs {err:.2e}")
    assert nz == int(np.count_nonzero(rho_t)) and err <= TOL
