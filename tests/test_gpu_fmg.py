"""Full-multigrid start of the Poisson solve (GDGS_MG_FMG) on the GPU through
the C ABI: the same tolerance against the oracle's exact solves as the plain
V-cycles (Dirichlet data from the reference image, the Neumann condition, a
warm start), no more cycles than they need, and the render entry point."""
import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
import workloads as wl
from oracle import poisson as P
from oracle.render import render as orender
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _solve(rho, ring, flags, **kw):
    H, W = rho.shape[1:]
    r = torch.from_numpy(np.ascontiguousarray(rho, np.float32)).cuda()
    b = None if ring is None else torch.from_numpy(np.ascontiguousarray(ring, np.float32)).cuda()
    u, st = G.gdgs_poisson_solve_rhs(r, b, W, H, G.mg_params(tol=1e-6, max_cycles=40,
                                                            flags=flags, **kw))
    torch.cuda.synchronize()
    return np_(u).astype(np.float64), G.read_stats(st)


@pytest.mark.parametrize("H,W", [(64, 64), (97, 61), (131, 257), (800, 800), (1080, 1920)])
def test_dirichlet_matches_direct_solver(H, W):
    rng = np.random.default_rng(H + W)
    ring = wl.reference_image(H, W, seed=1).astype(np.float32).astype(np.float64)
    rho = np.zeros((3, H, W))
    rho[:, 1:-1, 1:-1] = rng.laplace(0, 0.02, (3, H - 2, W - 2))
    rho = rho.astype(np.float32).astype(np.float64)
    exact = P.solve(rho, ring)
    got_f, st_f = _solve(rho, ring, G.FMG)
    got_v, st_v = _solve(rho, ring, 0)
    err = np.abs(got_f - exact).max()
    say(f"[fmg] dirichlet {W}x{H}: max-abs {err:.3e}, cycles fmg {st_f['cycles']} "
        f"v {st_v['cycles']}")
    assert st_f["converged"] and err <= TOL
    assert max(st_f["cycles"]) <= max(st_v["cycles"])
    assert np.array_equal(got_f[:, 0, :], ring[:, 0, :])


@pytest.mark.parametrize("H,W", [(130, 250), (1080, 1920)])
def test_neumann_matches_oracle(H, W):
    f = wl.reference_image(H, W, seed=4)
    rho = P.laplacian_neumann(f).astype(np.float32).astype(np.float64)
    exact = P.solve_neumann(rho)
    got, st = _solve(rho, None, G.FMG | G.NEUMANN)
    err = np.abs(got - exact).max()
    say(f"[fmg] neumann {W}x{H}: max-abs {err:.3e}, cycles {st['cycles']}")
    assert st["converged"] and err <= TOL


def test_warm_start_and_render_entry_point():
    H, W, K = 180, 320, 20000
    sc = wl.make_scene(K, seed=0, z=(2.0, 20.0), ls=(-5.0, 0.7))
    ds = G.DeviceScene.from_host(sc)
    ring = torch.from_numpy(wl.reference_image(H, W, seed=1).astype(np.float32)).cuda()
    cam = wl.make_camera(W, H, pose_index=1)
    mg = G.mg_params(tol=1e-6, max_cycles=30, flags=G.FMG)
    u, st = G.gdgs_render(ds, cam, ring, mg, sync_stats=True)
    torch.cuda.synchronize()
    ref, _ = G.gdgs_render(ds, cam, ring, G.mg_params(tol=1e-6, max_cycles=30), sync_stats=True)
    torch.cuda.synchronize()
    assert G.read_stats(st)["converged"]
    assert (u - ref).abs().max().item() <= TOL
    # the Renderer keeps the flag; a resumed continuation ignores it
    r = G.Renderer(ds, W, H, mg)
    u2 = r.render(cam, ring)
    torch.cuda.synchronize()
    assert (u2 - u).abs().max().item() <= 1e-6
    # warm start from the converged image, with the full-multigrid start
    uw = u.clone()
    uw, stw = G.gdgs_render(ds, cam, ring, G.mg_params(tol=1e-6, max_cycles=30,
                                                         flags=G.FMG | G.WARM_START), u=uw,
                            sync_stats=True)
    torch.cuda.synchronize()
    assert G.read_stats(stw)["converged"] and (uw - ref).abs().max().item() <= TOL


def test_tiny_render_against_the_oracle():
    H, W, K = 48, 80, 1500
    sc = wl.make_scene(K, seed=2, ls=(-2.5, 0.5))
    cam = wl.make_camera(W, H, pose_index=3)
    ds = G.DeviceScene.from_host(sc)
    u, st = G.gdgs_render(ds, cam, None, G.mg_params(tol=1e-6, max_cycles=30, flags=G.FMG),
                          sync_stats=True)
    torch.cuda.synchronize()
    o = orender(sc, cam)
    err = np.abs(np_(u) - o["u"]).max()
    say(f"[fmg] tiny render max-abs {err:.3e}, cycles {G.read_stats(st)['cycles']}")
    assert err <= TOL
