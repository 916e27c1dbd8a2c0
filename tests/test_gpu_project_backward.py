"""Reverse mode of the projection on the GPU through the C ABI: against the
oracle's chain rule on random incoming gradients, and the whole 3D gradient
(adjoint solve, divergence adjoint, reverse compositing, reverse projection)
against the oracle's composition of the same steps."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
from paper_2405_05446_amd import autograd as AG
import workloads as wl
from oracle import backward as obk
from oracle.project import project as oproject
from oracle.project_backward import project_backward as oproject_backward
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_matches_oracle_on_random_incoming_gradients():
    sc = wl.make_scene(3000, seed=4, z=(0.1, 6.0), ls=(-3, 0.6))
    sc.quat[:, 0:5] = 0.0                      # culled: zero quaternion
    cam = wl.make_camera(200, 150, pose_index=2)
    K = sc.opacity.shape[0]
    rng = np.random.default_rng(1)
    gm = rng.normal(size=(2, K)).astype(np.float32)
    gc = (rng.normal(size=(3, K)) * 10).astype(np.float32)
    ds = G.DeviceScene.from_host(sc)
    g = G.gdgs_project_backward(ds, cam, torch.from_numpy(gm).cuda(), torch.from_numpy(gc).cuda())
    torch.cuda.synchronize()
    ref = oproject_backward(sc, cam, gm.astype(np.float64), gc.astype(np.float64))
    for name in ("mean", "log_scale", "quat"):
        a, b = np_(g[name]).astype(np.float64), ref[name]
        err = np.abs(a - b).max() / np.abs(b).max()
        say(f"[project_backward] {name}: max-abs / max {err:.2e}")
        assert err <= 1e-5, name
        assert np.all(a[:, :5] == 0)


def test_end_to_end_3d_gradients_match_oracle():
    H, W, K = 32, 40, 150
    sc = wl.make_scene(K, seed=2, z=(2.0, 4.0), ls=(-1.5, 0.3))
    cam = wl.make_camera(W, H, pose_index=1)
    target = (wl.reference_image(H, W, seed=1) - 0.5).astype(np.float64)
    ds = G.DeviceScene.from_host(sc)
    params = [t.clone().requires_grad_(True) for t in (ds.mean, ds.log_scale, ds.quat,
                                                        ds.opacity, ds.value)]
    mg = G.mg_params(tol=1e-9, max_cycles=60)
    u = AG.render3d(*params, cam, mg=mg)
    tgt = torch.from_numpy(target.astype(np.float32)).cuda()
    e = (u - tgt)[:, 1:-1, 1:-1]
    loss = 0.5 * (e * e).sum()
    loss.backward()
    torch.cuda.synchronize()
    # oracle: project, 2D gradients of the same loss, reverse projection
    o = oproject(sc, cam)
    p2 = dict(mean2d=o["mean2d"], conic=o["conic"], opacity=sc.opacity.astype(np.float64),
              value=sc.value.astype(np.float64), depth=o["depth"])
    g2 = obk.gradients(p2, H, W, target)
    g3 = oproject_backward(sc, cam, g2["mean2d"], g2["conic"])
    ref = dict(mean=g3["mean"], log_scale=g3["log_scale"], quat=g3["quat"],
               opacity=g2["opacity"], value=g2["value"])
    for name, t in zip(("mean", "log_scale", "quat", "opacity", "value"), params):
        err = rel_l2(np_(t.grad).astype(np.float64), ref[name])
        say(f"[project_backward] end to end {name}: rel L2 {err:.2e}")
        assert err <= 1e-3, name
