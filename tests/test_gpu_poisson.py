"""GPU parity of the Poisson stage (divergence + multigrid) against closed
forms and the oracle's exact direct solvers."""
import math

import numpy as np
import pytest
import torch

import paper_2405_05446_amd as G
import workloads as wl
from oracle import poisson as P
from tests.gpu_util import say, np_

pytestmark = pytest.mark.gpu
TOL = 1e-4


def solve_rhs(rho, ring, mg=None):
    H, W = rho.shape[1:]
    r = torch.from_numpy(np.ascontiguousarray(rho, np.float32)).cuda()
    b = None if ring is None else torch.from_numpy(np.ascontiguousarray(ring, np.float32)).cuda()
    u, st = G.gdgs_poisson_solve_rhs(r, b, W, H, mg)
    torch.cuda.synchronize()
    return np_(u).astype(np.float64), G.read_stats(st)


@pytest.mark.parametrize("H,W,a,b", [(64, 64, 1, 1), (72, 100, 2, 3), (17, 33, 1, 2),
                                     (3, 3, 1, 1), (5, 130, 1, 4), (800, 800, 3, 2),
                                     (1080, 1920, 2, 5)])
def test_sin_product_closed_form(H, W, a, b):
    say(f"[poisson] sin-product {H}x{W} a={a} b={b}")
    i = np.arange(H)[:, None]
    j = np.arange(W)[None, :]
    u = np.sin(math.pi * a * i / (H - 1)) * np.sin(math.pi * b * j / (W - 1))
    lam = 2 * math.cos(math.pi * a / (H - 1)) + 2 * math.cos(math.pi * b / (W - 1)) - 4
    rho = np.zeros((3, H, W))
    for c in range(3):
        rho[c, 1:-1, 1:-1] = (c + 1) * lam * u[1:-1, 1:-1]
    got, st = solve_rhs(rho, None, G.mg_params(tol=1e-6, max_cycles=40))
    for c in range(3):
        err = np.abs(got[c] - (c + 1) * u).max()
        say(f"  channel {c}: max-abs {err:.3e}, cycles {st['cycles'][c]}, eta {st['eta'][c]:.2e}")
        assert err <= TOL
    assert st["converged"]


@pytest.mark.parametrize("H,W", [(64, 64), (72, 100), (97, 61), (800, 800), (1080, 1920)])
def test_matches_direct_solver_with_reference_ring(H, W):
    say(f"[poisson] vs direct {H}x{W}")
    rng = np.random.default_rng(H + W)
    ref = wl.reference_image(H, W, seed=1)
    rho = np.zeros((3, H, W))
    rho[:, 1:-1, 1:-1] = rng.laplace(0, 0.02, (3, H - 2, W - 2))
    rho32 = rho.astype(np.float32).astype(np.float64)
    ring32 = ref.astype(np.float32).astype(np.float64)
    got, st = solve_rhs(rho32, ring32, G.mg_params(tol=1e-6))
    exact = P.solve(rho32, ring32)
    err = np.abs(got - exact).max()
    say(f"  max-abs {err:.3e} cycles {st['cycles']} eta {st['eta']} rel_res {st['rel_res']}")
    assert err <= TOL
    assert st["converged"] and max(st["cycles"]) <= 20
    # ring is copied through
    assert np.array_equal(got[:, 0, :], ring32[:, 0, :])


def test_gradient_input_divergence_and_integrable_field():
    H, W = 90, 123
    f = wl.reference_image(H, W, seed=3)
    g = np.zeros((6, H, W))
    g[0::2, :, :-1] = f[:, :, 1:] - f[:, :, :-1]
    g[1::2, :-1, :] = f[:, 1:, :] - f[:, :-1, :]
    g32 = torch.from_numpy(g.astype(np.float32)).cuda()
    ring = torch.from_numpy(f.astype(np.float32)).cuda()
    u, st = G.gdgs_poisson_solve(g32, ring, W, H, G.mg_params(tol=1e-6, max_cycles=40))
    torch.cuda.synchronize()
    exact = P.solve(P.divergence(g.astype(np.float32)), f.astype(np.float32))
    assert np.abs(np_(u) - exact).max() <= TOL
    assert np.abs(np_(u) - f).max() <= TOL       # integrable field recovers the image


def test_convergence_factor_per_cycle():
    H, W = 1080, 1920
    rng = np.random.default_rng(1)
    rho = np.zeros((3, H, W))
    rho[:, 1:-1, 1:-1] = rng.normal(0, 0.05, (3, H - 2, W - 2))
    # Only the cycles before the relative residual of this white-noise
    # right-hand side reaches the FP32 rounding floor of the iterate (about
    # 4.5 x 2^-24 x rms(u) / rms(rho), ~3e-5 here), where the ratio means
    # nothing: cycles 1-3 with plain Gauss-Seidel sweeps (factor about 0.06),
    # cycles 1-2 with the default over-relaxed sweeps (about 0.02).
    for weight, cycles, bar in ((1.0, (1, 2, 3), 0.1), (0.0, (1, 2), 0.04)):
        etas = []
        for cyc in cycles:
            _, st = solve_rhs(rho, None, G.mg_params(tol=0.0, max_cycles=cyc,
                                                     smooth_weight=weight))
            etas.append(max(st["rel_res"]))
        factors = [etas[i + 1] / etas[i] for i in range(len(etas) - 1)]
        say(f"[poisson] weight {weight}: rel_res per cycle {etas}, factors {factors}")
        assert max(factors) <= bar


def test_over_relaxed_sweeps_stop_sooner_at_the_same_accuracy():
    # 1080p frame-like right-hand side (smooth ring, white-noise divergence):
    # the default weight meets the 1e-6 correction stop in fewer V-cycles over
    # the three channels than plain Gauss-Seidel, and both stay within the bar
    # of the exact solve
    H, W = 1080, 1920
    rng = np.random.default_rng(4)
    rho = np.zeros((3, H, W))
    rho[:, 1:-1, 1:-1] = rng.normal(0, 0.02, (3, H - 2, W - 2))
    ring = wl.reference_image(H, W, seed=1)
    exact = P.solve(rho, ring)
    cyc = {}
    for weight in (1.0, 0.0):
        u, st = solve_rhs(rho, ring, G.mg_params(tol=1e-6, max_cycles=20, smooth_weight=weight))
        assert st["converged"]
        cyc[weight] = st["cycles"]
        err = np.abs(u - exact).max()
        say(f"[poisson] weight {weight}: cycles {st['cycles']}, max-abs vs exact {err:.2e}")
        assert err <= TOL
    assert sum(cyc[0.0]) < sum(cyc[1.0])


def test_warm_start_continues_from_the_given_iterate():
    H, W = 300, 411
    rng = np.random.default_rng(3)
    rho = np.zeros((3, H, W))
    rho[:, 1:-1, 1:-1] = rng.normal(0, 0.05, (3, H - 2, W - 2))
    ring = wl.reference_image(H, W, seed=1)
    r = torch.from_numpy(rho.astype(np.float32)).cuda()
    b = torch.from_numpy(ring.astype(np.float32)).cuda()
    u, st = G.gdgs_poisson_solve_rhs(r, b, W, H, G.mg_params(tol=0.0, max_cycles=2))
    torch.cuda.synchronize()
    u2, st2 = G.gdgs_poisson_solve_rhs(r, b, W, H, G.mg_params(tol=1e-6, max_cycles=30,
                                                               flags=G.api.WARM_START), u=u)
    torch.cuda.synchronize()
    s2 = G.read_stats(st2)
    exact = P.solve(rho.astype(np.float32).astype(np.float64), ring.astype(np.float32))
    assert s2["converged"] and np.abs(np_(u2) - exact).max() <= TOL
    # a converged iterate needs a single further cycle
    u3, st3 = G.gdgs_poisson_solve_rhs(r, b, W, H, G.mg_params(tol=1e-6, max_cycles=30,
                                                               flags=G.api.WARM_START), u=u2)
    torch.cuda.synchronize()
    assert G.read_stats(st3)["cycles"] == [1, 1, 1]


def test_resumed_calls_equal_one_call_bit_for_bit():
    """GDGS_MG_RESUME: 1 + 2 + 3 cycles in three calls == 6 cycles in one call,
    also after a channel has converged (its flag and cycle count carry over)."""
    H, W = 257, 390
    rng = np.random.default_rng(4)
    rho = np.zeros((3, H, W))
    rho[:, 1:-1, 1:-1] = rng.normal(0, 0.05, (3, H - 2, W - 2))
    rho[2] = 0.0                      # channel 2 is exact from the start
    ring = wl.reference_image(H, W, seed=1)
    ring[2] = 0.0
    r = torch.from_numpy(rho.astype(np.float32)).cuda()
    b = torch.from_numpy(ring.astype(np.float32)).cuda()
    for tol in (0.0, 1e-5):
        one, st1 = G.gdgs_poisson_solve_rhs(r, b, W, H, G.mg_params(tol=tol, max_cycles=6))
        torch.cuda.synchronize()
        s1 = G.read_stats(st1)
        u = torch.empty_like(one)
        st = G.new_stats()
        ws = G.workspace(G.api.poisson_workspace_size(W, H))
        for k, cyc in enumerate((1, 2, 3)):
            G.gdgs_poisson_solve_rhs(r, b, W, H, G.mg_params(tol=tol, max_cycles=cyc,
                                                           flags=G.api.RESUME if k else 0),
                                     u=u, stats=st, ws=ws)
        torch.cuda.synchronize()
        s3 = G.read_stats(st)
        say(f"[poisson] tol {tol}: one call {s1['cycles']}, resumed {s3['cycles']}")
        assert s3["cycles"] == s1["cycles"] and s3["converged"] == s1["converged"]
        assert torch.equal(u, one)
    assert s1["cycles"][2] == 0


def test_zero_rhs_zero_ring_is_immediately_exact():
    u, st = solve_rhs(np.zeros((3, 40, 50)), None)
    assert np.all(u == 0) and st["converged"] and st["cycles"] == [0, 0, 0]


def test_deterministic():
    rng = np.random.default_rng(2)
    rho = rng.normal(0, 0.05, (3, 300, 411))
    a, _ = solve_rhs(rho, None)
    b, _ = solve_rhs(rho, None)
    assert np.array_equal(a, b)
