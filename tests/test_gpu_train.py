"""Algorithm-1 iteration on the GPU through the C ABI: the loss of Eq. 22 and
its image gradient against the oracle, the Adam update against the oracle,
one whole step (render, loss, reverse chain to the 3D parameters) against
the oracle's composition, and the loss falling over a few steps toward a
synthetic target."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
from paper_2405_05446_amd import train as TR
import workloads as wl
from oracle import backward as obk, loss as OL
from oracle.project import project as oproject
from oracle.project_backward import project_backward as oproject_backward
from oracle.render import render as orender
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu


def _pair(H, W, seed=0):
    rng = np.random.default_rng(seed)
    im = wl.reference_image(H, W, seed=1)
    c = im + 0.05 * rng.normal(size=im.shape)
    return c.astype(np.float32), im.astype(np.float32)


@pytest.mark.parametrize("H,W", [(37, 53), (64, 96), (3, 5)])
def test_loss_and_image_gradient_match_oracle(H, W):
    c, im = _pair(H, W)
    out, dc = G.api.gdgs_image_loss(torch.from_numpy(c).cuda(), torch.from_numpy(im).cuda())
    torch.cuda.synchronize()
    o = OL.loss(c.astype(np.float64), im.astype(np.float64))
    got = out.cpu().numpy()
    ref = np.array([o["loss"], o["l1"], o["grad_l1"], o["dssim"]])
    say(f"[train] loss {H}x{W}: {got} vs {ref}")
    assert np.allclose(got, ref, rtol=2e-5, atol=1e-9)
    g = np_(dc).astype(np.float64)
    assert np.abs(g - o["dc"]).max() <= 1e-4 * np.abs(o["dc"]).max()


def test_adam_matches_oracle():
    rng = np.random.default_rng(2)
    n = 10000
    p, g = rng.normal(size=n), rng.normal(size=n)
    m, v = 0.1 * rng.normal(size=n), 0.01 * rng.random(n)
    t32 = lambda a: torch.from_numpy(a.astype(np.float32)).cuda()
    P, Gd, M, V = t32(p), t32(g), t32(m), t32(v)
    G.api.gdgs_adam_step(P, Gd, M, V, 3, 0.01, lo=-0.5, hi=0.5)
    torch.cuda.synchronize()
    f = lambda a: a.astype(np.float32).astype(np.float64)
    rp, rm, rv = OL.adam(f(p), f(g), f(m), f(v), 3, 0.01, lo=-0.5, hi=0.5)
    assert np.abs(np_(P) - rp).max() <= 1e-6
    assert np.abs(np_(M) - rm).max() <= 1e-6 and np.abs(np_(V) - rv).max() <= 1e-6


def test_one_step_matches_the_oracle_composition():
    H, W, K = 32, 40, 150
    sc = wl.make_scene(K, seed=2, z=(2.0, 4.0), ls=(-1.5, 0.3))
    cam = wl.make_camera(W, H, pose_index=1)
    target = wl.reference_image(H, W, seed=3).astype(np.float32)
    tr = TR.Trainer(G.DeviceScene.from_host(sc), mg=G.mg_params(tol=1e-9, max_cycles=60))
    res = tr.step(cam, torch.from_numpy(target).cuda())
    torch.cuda.synchronize()
    o = orender(sc, cam)
    lo = OL.loss(o["u"], target.astype(np.float64))
    assert abs(res["loss"] - lo["loss"]) <= 1e-4 * lo["loss"]
    p = oproject(sc, cam)
    p2 = dict(mean2d=p["mean2d"], conic=p["conic"], opacity=sc.opacity.astype(np.float64),
              value=sc.value.astype(np.float64), depth=p["depth"])
    g2 = obk.gradients_from_du(p2, H, W, lo["dc"])
    g3 = oproject_backward(sc, cam, g2["mean2d"], g2["conic"])
    ref = dict(mean=g3["mean"], log_scale=g3["log_scale"], quat=g3["quat"],
               opacity=g2["opacity"], value=g2["value"])
    for name in TR.GROUPS:
        a, b = np_(res["grads"][name]).astype(np.float64), ref[name]
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        say(f"[train] step gradient {name}: rel L2 {err:.2e}")
        assert err <= 2e-3, name


def test_loss_falls_toward_a_synthetic_target():
    H, W, K = 64, 64, 2000
    truth = wl.make_scene(K, seed=7, ls=(-3.0, 0.4))
    ds_true = G.DeviceScene.from_host(truth)
    cam = wl.make_camera(W, H, pose_index=0)
    target, _ = G.gdgs_render(ds_true, cam, None, sync_stats=True)
    start = wl.make_scene(K, seed=7, ls=(-3.0, 0.4))
    rng = np.random.default_rng(8)
    start.value = (start.value + 0.5 * np.abs(start.value).mean()
                   * rng.normal(size=start.value.shape)).astype(np.float32)
    tr = TR.Trainer(G.DeviceScene.from_host(start))
    losses = [tr.step(cam, target)["loss"] for _ in range(12)]
    say(f"[train] losses {['%.4g' % x for x in losses]}")
    assert losses[-1] < 0.8 * losses[0]


def test_loss_falls_under_the_neumann_condition():
    # Algorithm 1 with the paper's boundary condition: target and iterate are
    # both zero-mean Neumann reconstructions
    H, W, K = 64, 64, 2000
    mg = G.mg_params(tol=1e-6, max_cycles=40, flags=G.NEUMANN)
    truth = wl.make_scene(K, seed=7, ls=(-3.0, 0.4))
    cam = wl.make_camera(W, H, pose_index=0)
    target, st = G.gdgs_render(G.DeviceScene.from_host(truth), cam, None, mg, sync_stats=True)
    assert G.read_stats(st)["converged"]
    start = wl.make_scene(K, seed=7, ls=(-3.0, 0.4))
    rng = np.random.default_rng(8)
    start.value = (start.value + 0.5 * np.abs(start.value).mean()
                   * rng.normal(size=start.value.shape)).astype(np.float32)
    tr = TR.Trainer(G.DeviceScene.from_host(start), mg=mg)
    losses = [tr.step(cam, target)["loss"] for _ in range(12)]
    say(f"[train] neumann losses {['%.4g' % x for x in losses]}")
    assert losses[-1] < 0.8 * losses[0]
