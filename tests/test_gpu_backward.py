"""GPU backward pass (adjoint Poisson solve, divergence adjoint, reverse
compositing) against the oracle's exact FP64 gradients and adjoint identities."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
from paper_2405_05446_amd.autograd import render as diff_render
import workloads as wl
from oracle import backward as obk
from oracle import poisson as P
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def test_div_adjoint_matches_oracle_bit_exactly():
    H, W = 37, 53
    lam = np.random.default_rng(0).normal(size=(3, H, W)).astype(np.float32)
    got = np_(G.gdgs_div_adjoint(dev(lam), W, H))
    ref = P.div_adjoint(lam.astype(np.float64)).astype(np.float32)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("H,W,K,seed", [(32, 32, 200, 2), (40, 56, 400, 4)])
def test_gradients_match_oracle(H, W, K, seed):
    say(f"[backward] {W}x{H} K={K}")
    params = wl.raster_scene(K, W, H, seed=seed, ls=(-1.5, 0.3), fx=W)
    target = (wl.reference_image(H, W, seed=1) - 0.5).astype(np.float32)
    p64 = {k: v.astype(np.float64) for k, v in params.items()}
    ref = obk.gradients(p64, H, W, target.astype(np.float64))
    t = {k: dev(v).requires_grad_(k != "depth") for k, v in params.items()}
    mg = G.mg_params(tol=1e-7, max_cycles=40)
    u = diff_render(t["mean2d"], t["conic"], t["opacity"], t["value"], t["depth"], W, H, None, mg)
    tgt = dev(target)
    e = torch.zeros_like(u)
    e[:, 1:-1, 1:-1] = (u - tgt)[:, 1:-1, 1:-1]
    loss = 0.5 * (e * e).sum()
    loss.backward()
    say(f"  loss gpu {loss.item():.6e} oracle {ref['loss']:.6e}")
    assert abs(loss.item() - ref["loss"]) <= 1e-4 * ref["loss"] + 1e-9
    for name in ["mean2d", "conic", "opacity", "value"]:
        err = rel_l2(np_(t[name].grad), ref[name])
        say(f"  {name}: rel L2 {err:.2e}")
        assert err <= 1e-3, name


def test_raster_backward_alone_matches_oracle():
    H, W, K = 32, 32, 200
    params = wl.raster_scene(K, W, H, seed=2, ls=(-1.5, 0.3), fx=W)
    p64 = {k: v.astype(np.float64) for k, v in params.items()}
    target = wl.reference_image(H, W, seed=1) - 0.5
    ref = obk.gradients(p64, H, W, target)
    t = {k: dev(v) for k, v in params.items()}
    proj = G.gdgs_project_2d(t["mean2d"], t["conic"], t["depth"], W, H)
    bins = G.gdgs_bin_sort(proj, K, W, H, 1 << 14)
    grad = G.gdgs_raster_grad(proj, t["opacity"], t["value"], K, bins, W, H)
    g = G.gdgs_raster_grad_backward(proj, t["opacity"], t["value"], K, bins, W, H, grad,
                                    dev(ref["dgrad"]))
    for name in ["mean2d", "conic", "opacity", "value"]:
        assert rel_l2(np_(g[name]), ref[name]) <= 1e-4, name
    # deterministic: a second run is bitwise identical
    g2 = G.gdgs_raster_grad_backward(proj, t["opacity"], t["value"], K, bins, W, H, grad,
                                     dev(ref["dgrad"]))
    for name in g:
        assert torch.equal(g[name], g2[name])
    # tiles taken by id instead of heaviest first: the same bits
    b_id = dict(bins, tile_order=None)
    g3 = G.gdgs_raster_grad_backward(proj, t["opacity"], t["value"], K, b_id, W, H, grad,
                                     dev(ref["dgrad"]))
    for name in g:
        assert torch.equal(g[name], g3[name])


def test_gradients_match_oracle_at_differentiation_workload_on_sampled_splats():
    """Differentiation workload (512x512, 100k splats): the GPU's gradients of
    a squared-error loss against the oracle's exact ones on 200 seeded
    splats.  The oracle takes the loss gradient e = u - target of the GPU's
    forward image, solves the adjoint Poisson problem exactly (DST-I, zero
    ring), applies the divergence adjoint and reverse-composites each sampled
    splat over the pixels of its support box (Sec. 1.1, Eq. 5-7 through
    Eq. 20/21)."""
    cfg = wl.CONFIGS["diff"]
    H, W, K = cfg["H"], cfg["W"], cfg["K"]
    say(f"[backward] sampled splats vs oracle {W}x{H} K={K}")
    params = wl.raster_scene(K, W, H, seed=0, ls=cfg["ls"], z=cfg["z"], fx=W)
    target = (wl.reference_image(H, W, seed=1) - 0.5).astype(np.float32)
    t = {k: dev(v).requires_grad_(k != "depth") for k, v in params.items()}
    mg = G.mg_params(tol=1e-7, max_cycles=40)
    u = diff_render(t["mean2d"], t["conic"], t["opacity"], t["value"], t["depth"], W, H, None, mg)
    e = torch.zeros_like(u)
    e[:, 1:-1, 1:-1] = (u - dev(target))[:, 1:-1, 1:-1]
    (0.5 * (e * e).sum()).backward()
    torch.cuda.synchronize()
    # the oracle's reverse chain from the same loss gradient
    lam = P.solve_dst(np_(e).astype(np.float64), None)
    dgrad = P.div_adjoint(lam)
    p64 = {k: v.astype(np.float64) for k, v in params.items()}
    rng = np.random.default_rng(21)
    cand = np.nonzero((params["mean2d"][0] > 8) & (params["mean2d"][0] < W - 8) &
                      (params["mean2d"][1] > 8) & (params["mean2d"][1] < H - 8))[0]
    splats = np.sort(rng.choice(cand, size=200, replace=False))
    ref = obk.splat_gradients(p64, H, W, dgrad, splats)
    for name in ["mean2d", "conic", "opacity", "value"]:
        got = np_(t[name].grad)[..., splats]
        err = rel_l2(got, ref[name])
        say(f"  {name}: rel L2 {err:.2e} over {splats.size} splats")
        assert err <= 1e-3, name


def test_adjoint_identity_at_differentiation_workload_size():
    """u is linear in the gradient values: for the differentiation workload
    (512x512, 100k splats) check <J dv, w> = <dv, J^T w> with J the map from
    values to the recovered image (forward with values dv) and J^T the
    backward pass seeded with dL/du = w."""
    cfg = wl.CONFIGS["diff"]
    H, W, K = cfg["H"], cfg["W"], cfg["K"]
    say(f"[backward] adjoint identity {W}x{H} K={K}")
    params = wl.raster_scene(K, W, H, seed=0, ls=cfg["ls"], z=cfg["z"], fx=W)
    t = {k: dev(v) for k, v in params.items()}
    rng = np.random.default_rng(5)
    dv = dev(rng.normal(size=(6, K)))
    w = torch.zeros((3, H, W), device="cuda")
    w[:, 1:-1, 1:-1] = dev(rng.normal(size=(3, H - 2, W - 2)))
    mg = G.mg_params(tol=1e-7, max_cycles=40)
    v = dv.clone().requires_grad_(True)
    u = diff_render(t["mean2d"], t["conic"], t["opacity"], v, t["depth"], W, H, None, mg)
    lhs = float((u.double() * w.double()).sum())
    (u * w).sum().backward()
    rhs = float((dv.double() * v.grad.double()).sum())
    say(f"  <J dv, w> = {lhs:.8e}, <dv, J^T w> = {rhs:.8e}")
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_adjoint_solve_is_self_adjoint():
    H, W = 200, 300
    rng = np.random.default_rng(6)
    x = np.zeros((3, H, W)); x[:, 1:-1, 1:-1] = rng.normal(size=(3, H - 2, W - 2))
    y = np.zeros((3, H, W)); y[:, 1:-1, 1:-1] = rng.normal(size=(3, H - 2, W - 2))
    mg = G.mg_params(tol=1e-7, max_cycles=40)
    ax, _ = G.gdgs_poisson_solve_rhs(dev(x), None, W, H, mg)
    ay, _ = G.gdgs_poisson_solve_rhs(dev(y), None, W, H, mg)
    a = float((ax.double().cpu().numpy() * y).sum())
    b = float((x * ay.double().cpu().numpy()).sum())
    assert abs(a - b) <= 1e-5 * abs(a)
