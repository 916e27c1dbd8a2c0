"""Edge cases of the whole path against the oracle: the smallest images, an
empty scene, degenerate splats (zero quaternion, behind the near plane, one
splat covering the image), and image shapes that are one tile or one pixel
past a tile boundary."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
import workloads as wl
from oracle import poisson as P
from oracle.render import render as orender
from tests.gpu_util import say, np_, gpu_stages

pytestmark = pytest.mark.gpu
TOL = 1e-4


def render(sc, cam, ring=None, mg=None):
    ds = G.DeviceScene.from_host(sc)
    b = None if ring is None else torch.from_numpy(ring.astype(np.float32)).cuda()
    u, st = G.gdgs_render(ds, cam, b, mg or G.mg_params(tol=1e-6, max_cycles=40),
                          capacity=max(4096, 64 * max(sc.K, 1)), sync_stats=True)
    torch.cuda.synchronize()
    return np_(u), G.read_stats(st)


@pytest.mark.parametrize("W,H", [(3, 3), (3, 40), (40, 3), (17, 16), (16, 17), (33, 5)])
def test_smallest_and_off_by_one_images(W, H):
    sc = wl.make_scene(300, seed=11, ls=(-2.5, 0.5))
    cam = wl.make_camera(W, H, pose_index=3)
    ring = wl.reference_image(H, W, seed=1)
    u, s = render(sc, cam, ring)
    o = orender(sc, cam, ring.astype(np.float32).astype(np.float64))
    err = np.abs(u - o["u"]).max()
    say(f"[edges] {W}x{H}: max-abs {err:.3e}, cycles {s['cycles']}")
    assert err <= TOL and s["converged"]
    # the ring is the Dirichlet data, untouched
    assert np.array_equal(u[:, 0, :], ring.astype(np.float32)[:, 0, :])
    assert np.array_equal(u[:, :, -1], ring.astype(np.float32)[:, :, -1])


def test_empty_scene_renders_the_harmonic_extension_of_the_ring():
    H, W = 45, 70
    cam = wl.make_camera(W, H)
    ring = wl.reference_image(H, W, seed=1)
    u, s = render(wl.make_scene(0, seed=0), cam, ring)
    exact = P.solve(np.zeros((3, H, W)), ring.astype(np.float32).astype(np.float64))
    assert np.abs(u - exact).max() <= TOL and s["num_pairs"] == 0 and s["converged"]
    # and with a zero ring the image is exactly zero, after no cycle at all
    u0, s0 = render(wl.make_scene(0, seed=0), cam, None)
    assert np.all(u0 == 0) and s0["cycles"] == [0, 0, 0]


def test_degenerate_splats():
    H, W = 40, 56
    sc = wl.make_scene(400, seed=12, ls=(-2.5, 0.5))
    sc.quat[:, 0:10] = 0.0               # zero quaternions: culled
    sc.mean[2, 10:20] = 0.15             # in front of the near plane: culled
    sc.mean[2, 20:25] = -3.0             # behind the camera: culled
    sc.mean[:, 25] = [0.0, 0.0, 2.5]     # one splat covering the whole image
    sc.log_scale[:, 25] = 1.5
    cam = wl.make_camera(W, H, pose_index=6)
    g = gpu_stages(sc, cam)
    assert np.all(g["count"][:25] == 0)
    assert g["count"][25] == ((W + 15) // 16) * ((H + 15) // 16)
    o = orender(sc, cam, None)
    err_g = np.abs(g["grad"] - o["grad"]).max()
    u, s = render(sc, cam, None)
    err_u = np.abs(u - o["u"]).max()
    say(f"[edges] degenerate: grad {err_g:.3e}, u {err_u:.3e}")
    assert err_g <= TOL and err_u <= TOL


@pytest.mark.parametrize("W,H", [(3, 3), (3, 40), (40, 3), (17, 16), (33, 5)])
def test_neumann_smallest_and_off_by_one_images(W, H):
    sc = wl.make_scene(300, seed=11, ls=(-2.5, 0.5))
    cam = wl.make_camera(W, H, pose_index=3)
    u, s = render(sc, cam, None, G.mg_params(tol=1e-6, max_cycles=40, flags=G.NEUMANN))
    o = orender(sc, cam, neumann=True)
    err = np.abs(u - o["u"]).max()
    say(f"[edges] neumann {W}x{H}: max-abs {err:.3e}, cycles {s['cycles']}")
    assert err <= TOL and s["converged"]
    assert np.abs(u.astype(np.float64).mean(axis=(1, 2))).max() <= 1e-6


def test_neumann_laplacian_form_with_threshold():
    from oracle.render import render_laplacian as orender_lap
    H, W, K = 40, 56, 1500
    sc = wl.laplacian_scene(wl.make_scene(K, seed=4, ls=(-2.5, 0.5)), seed=4)
    cam = wl.make_camera(W, H, pose_index=2)
    ds = G.DeviceScene.from_host(sc)
    r = G.Renderer(ds, W, H, G.mg_params(tol=1e-6, max_cycles=40), neumann=True,
                   threshold=0.01)
    u = r.render(cam)
    torch.cuda.synchronize()
    # the oracle solves the GPU's thresholded composite (the threshold is an
    # exact FP32 comparison, checked elsewhere against the oracle's)
    rho = np_(r.grad[:3]).astype(np.float64)
    exact = P.solve_neumann(rho)
    err = np.abs(np_(u) - exact).max()
    o = orender_lap(sc, cam, t=0.01, neumann=True)
    say(f"[edges] neumann laplacian thresholded: max-abs {err:.3e}, "
        f"vs oracle render {np.abs(np_(u) - o['u']).max():.3e}")
    assert r.last["converged"] and err <= TOL
    assert np.abs(np_(u) - o["u"]).max() <= 10 * TOL
