"""Neumann variant of the Poisson solve (the paper's boundary condition,
Sec. 2.1 and Sec. 2.2, Eq. 21) on the GPU through the C ABI: solves against
the oracle's exact zero-mean solution at ragged sizes and at 1080p, the
gradient form recovering an image up to its mean, both render forms against
the oracle, the Renderer against the entry point, a resumed solve against
one call, the argument checks, and the reverse chain against the oracle's
exact gradients."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
import workloads as wl
from oracle import poisson as op
from oracle.render import render as orender
from oracle.render import render_laplacian as orender_lap
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _mg(**kw):
    kw.setdefault("tol", 1e-6)
    kw.setdefault("max_cycles", 40)
    flags = kw.pop("flags", 0) | G.NEUMANN
    return G.mg_params(flags=flags, **kw)


def _smooth(H, W, seed):
    # a smooth test image: the seeded reference image (sums of sines)
    return wl.reference_image(H, W, seed=seed).astype(np.float64)


@pytest.mark.parametrize("H,W", [(21, 37), (64, 64), (45, 70), (131, 257), (800, 800),
                                 (1080, 1920)])
def test_solve_rhs_matches_oracle(H, W):
    say(f"[neumann] solve_rhs {W}x{H}")
    f = _smooth(H, W, seed=H + W)
    # rho = L f plus a constant per channel, which the solve must project out
    rho = (op.laplacian_neumann(f) + np.array([0.01, -0.02, 0.0])[:, None, None])
    rho32 = rho.astype(np.float32)
    ref = op.solve_neumann(rho32.astype(np.float64))
    u, st = G.gdgs_poisson_solve_rhs(torch.from_numpy(rho32).cuda(), None, W, H, _mg())
    torch.cuda.synchronize()
    s = G.read_stats(st)
    un = np_(u)
    err = np.abs(un - ref).max()
    say(f"  max-abs {err:.3e}, cycles {s['cycles']}, mean {np.abs(un.mean(axis=(1, 2))).max():.1e}")
    assert s["converged"]
    assert err <= TOL
    assert np.abs(un.astype(np.float64).mean(axis=(1, 2))).max() <= 1e-6
    # the exact solution is the image minus its mean
    assert np.abs(ref - (f - f.mean(axis=(1, 2), keepdims=True))).max() < 1e-4


@pytest.mark.parametrize("H,W", [(77, 129), (1080, 1920)])
def test_gradient_form_recovers_the_image_up_to_its_mean(H, W):
    say(f"[neumann] gradient form {W}x{H}")
    f = _smooth(H, W, seed=3)
    rng = np.random.default_rng(5)
    grad = rng.standard_normal((6, H, W))  # the border-crossing entries are dropped
    grad[0::2, :, :-1] = f[:, :, 1:] - f[:, :, :-1]
    grad[1::2, :-1, :] = f[:, 1:, :] - f[:, :-1, :]
    g32 = grad.astype(np.float32)
    u, st = G.gdgs_poisson_solve(torch.from_numpy(g32).cuda(), None, W, H, _mg())
    torch.cuda.synchronize()
    s = G.read_stats(st)
    ref = op.solve_neumann(op.divergence_neumann(g32.astype(np.float64)))
    un = np_(u)
    err = np.abs(un - ref).max()
    err_f = np.abs(un - (f - f.mean(axis=(1, 2), keepdims=True))).max()
    say(f"  vs oracle {err:.3e}, vs image {err_f:.3e}, cycles {s['cycles']}")
    assert s["converged"] and err <= TOL and err_f <= TOL


def test_render_matches_oracle():
    H, W, K = 45, 70, 800
    sc = wl.make_scene(K, seed=3, ls=(-2.5, 0.5))
    cam = wl.make_camera(W, H, pose_index=2)
    ds = G.DeviceScene.from_host(sc)
    u, st = G.gdgs_render(ds, cam, None, _mg(), sync_stats=True)
    torch.cuda.synchronize()
    o = orender(sc, cam, neumann=True)
    s = G.read_stats(st)
    err = np.abs(np_(u) - o["u"]).max()
    say(f"[neumann] render 70x45 max-abs {err:.3e}, cycles {s['cycles']}")
    assert s["converged"] and err <= TOL


def test_laplacian_render_matches_oracle():
    H, W, K = 72, 100, 3000
    sc = wl.laplacian_scene(wl.make_scene(K, seed=0, ls=(-3, 0.6)), seed=0)
    cam = wl.make_camera(W, H, pose_index=3)
    ds = G.DeviceScene.from_host(sc)
    u, st = G.api.gdgs_render_laplacian(ds, cam, None, _mg(), sync_stats=True)
    torch.cuda.synchronize()
    o = orender_lap(sc, cam, neumann=True)
    s = G.read_stats(st)
    err = np.abs(np_(u) - o["u"]).max()
    say(f"[neumann] laplacian render 100x72 max-abs {err:.3e}, cycles {s['cycles']}")
    assert s["converged"] and err <= TOL


def test_renderer_equals_render_entry_point_and_warm_start():
    W, H, K = 320, 180, 20000
    sc = wl.make_scene(K, seed=0, z=(2.0, 20.0), ls=(-5.0, 0.7))
    ds = G.DeviceScene.from_host(sc)
    mg = _mg(max_cycles=30)
    r = G.Renderer(ds, W, H, mg)
    assert r.neumann
    rw = G.Renderer(ds, W, H, G.mg_params(tol=1e-6, max_cycles=30), neumann=True,
                    warm_start=True)
    for i in range(3):
        cam = wl.trajectory_camera(W, H, i)
        u = r.render(cam).clone()
        uw = rw.render(cam).clone()
        u2, st = G.gdgs_render(ds, cam, None, mg, capacity=r.capacity, sync_stats=True)
        torch.cuda.synchronize()
        assert r.last["converged"] and rw.last["converged"]
        assert (u - u2).abs().max().item() <= 1e-6
        # warm-started solves meet the same tolerance from another start
        assert (uw - u).abs().max().item() <= TOL
        say(f"[neumann] renderer frame {i}: cycles cold {r.last['total_cycles']}, "
            f"warm {rw.last['total_cycles']}")


def test_resumed_solve_equals_one_call():
    H, W = 130, 250
    f = _smooth(H, W, seed=8)
    rho = torch.from_numpy(op.laplacian_neumann(f).astype(np.float32)).cuda()
    mg6 = _mg(max_cycles=6, tol=0.0)
    u1, _ = G.gdgs_poisson_solve_rhs(rho, None, W, H, mg6)
    ws = G.workspace(G.api.poisson_workspace_size(W, H, mg6))
    u2, st = G.gdgs_poisson_solve_rhs(rho, None, W, H, _mg(max_cycles=4, tol=0.0), ws=ws)
    u2, st = G.gdgs_poisson_solve_rhs(rho, None, W, H,
                                      _mg(max_cycles=2, tol=0.0, flags=G.RESUME), u=u2,
                                      stats=st, ws=ws)
    torch.cuda.synchronize()
    assert G.read_stats(st)["cycles"] == [6, 6, 6]
    assert torch.equal(u1, u2)


def test_zero_rhs_and_argument_checks():
    H, W = 40, 60
    u, st = G.gdgs_poisson_solve_rhs(torch.zeros((3, H, W), device="cuda"), None, W, H, _mg())
    torch.cuda.synchronize()
    assert torch.count_nonzero(u).item() == 0 and G.read_stats(st)["converged"]
    # a constant right-hand side is all incompatible part: the answer is zero
    u, st = G.gdgs_poisson_solve_rhs(torch.full((3, H, W), 0.25, device="cuda"), None, W, H,
                                     _mg())
    torch.cuda.synchronize()
    assert u.abs().max().item() == 0.0
    ring = torch.zeros((3, H, W), device="cuda")
    with pytest.raises(G.GdgsError):
        G.gdgs_poisson_solve_rhs(torch.zeros((3, H, W), device="cuda"), ring, W, H, _mg())
    with pytest.raises(ValueError):
        from paper_2405_05446_amd import autograd as AG
        AG.render(torch.zeros((1, 2), device="cuda"), torch.zeros((1, 3), device="cuda"),
                  torch.zeros(1, device="cuda"), torch.zeros((6, 1), device="cuda"),
                  torch.ones(1, device="cuda"), W, H, boundary=ring, mg=_mg())


def test_div_adjoint_matches_oracle_bit_exactly():
    H, W = 37, 53
    lam = np.random.default_rng(0).normal(size=(3, H, W)).astype(np.float32)
    got = np_(G.gdgs_div_adjoint(torch.from_numpy(lam).cuda(), W, H, neumann=True))
    ref = op.div_adjoint_neumann(lam.astype(np.float64)).astype(np.float32)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("H,W,K,seed", [(24, 24, 120, 3), (40, 56, 400, 4)])
def test_gradients_match_oracle(H, W, K, seed):
    from oracle import backward as obk
    from paper_2405_05446_amd.autograd import render as diff_render
    say(f"[neumann] backward {W}x{H} K={K}")
    params = wl.raster_scene(K, W, H, seed=seed, ls=(-1.5, 0.3), fx=W)
    target = (wl.reference_image(H, W, seed=2) - 0.5).astype(np.float32)
    p64 = {k: v.astype(np.float64) for k, v in params.items()}
    ref = obk.gradients(p64, H, W, target.astype(np.float64), neumann=True)
    t = {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).cuda().requires_grad_(
        k != "depth") for k, v in params.items()}
    u = diff_render(t["mean2d"], t["conic"], t["opacity"], t["value"], t["depth"], W, H, None,
                    _mg(tol=1e-7))
    loss = 0.5 * ((u - torch.from_numpy(target).cuda()) ** 2).sum()
    loss.backward()
    say(f"  loss gpu {loss.item():.6e} oracle {ref['loss']:.6e}")
    assert abs(loss.item() - ref["loss"]) <= 1e-4 * ref["loss"] + 1e-9
    for name in ["mean2d", "conic", "opacity", "value"]:
        g = np_(t[name].grad).astype(np.float64)
        err = float(np.linalg.norm(g - ref[name]) / max(np.linalg.norm(ref[name]), 1e-30))
        say(f"  {name}: rel L2 {err:.2e}")
        assert err <= 1e-3, name
