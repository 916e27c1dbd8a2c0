"""Pins of the oracle's analytic gradients by FP64 central finite differences."""
import numpy as np
import pytest

import workloads as wl
from oracle import backward as obk
from oracle import poisson as P


@pytest.fixture(scope="module")
def instance():
    H = W = 32
    params = wl.raster_scene(200, W, H, seed=2, ls=(-1.5, 0.3), fx=W)
    params = {k: v.astype(np.float64) for k, v in params.items()}
    target = wl.reference_image(H, W, seed=1) - 0.5
    g = obk.gradients(params, H, W, target)
    return H, W, params, target, g


def test_loss_gradient_matches_finite_differences(instance):
    H, W, params, target, g = instance
    rng = np.random.default_rng(0)
    checked = 0
    for name, rows in [("mean2d", 2), ("conic", 3), ("opacity", None), ("value", 6)]:
        for _ in range(8):
            k = int(rng.integers(0, 200))
            idx = (k,) if rows is None else (int(rng.integers(0, rows)), k)
            an = g[name][idx]
            fd, crossed = obk.finite_difference(params, H, W, target, name, idx)
            if crossed:
                continue
            scale = np.abs(g[name]).max()
            assert abs(fd - an) <= 1e-6 * scale + 1e-6 * abs(an), (name, idx, fd, an)
            checked += 1
    assert checked >= 28


def test_adjoint_solve_identity(instance):
    # lam solves L lam = e with a zero ring, i.e. lam = -A^{-1} e
    H, W, params, target, g = instance
    fw = obk.forward(params, H, W, target)
    assert np.abs(P.laplacian(g["lam"])[:, 1:-1, 1:-1] - fw["e"][:, 1:-1, 1:-1]).max() < 1e-12


def test_splat_subset_mode_equals_full_reverse_compositing(instance):
    """The per-splat mode (sums over each splat's support box, with the
    compositing list formed from the splats whose boxes meet it) gives the
    same gradients as the per-pixel accumulation over the whole image."""
    H, W, params, target, g = instance
    splats = np.arange(200)
    sub = obk.splat_gradients(params, H, W, g["dgrad"], splats)
    for name in ["mean2d", "conic", "opacity", "value"]:
        ref = g[name][..., splats]
        scale = np.abs(ref).max()
        assert np.abs(sub[name] - ref).max() <= 1e-12 * scale, name
    # a subset in any order picks the same entries
    pick = np.array([170, 3, 99, 41])
    sub2 = obk.splat_gradients(params, H, W, g["dgrad"], pick)
    for name in ["mean2d", "conic", "opacity", "value"]:
        assert np.array_equal(sub2[name], sub[name][..., pick]), name


@pytest.fixture(scope="module")
def instance_neumann():
    H = W = 24
    params = wl.raster_scene(120, W, H, seed=3, ls=(-1.5, 0.3), fx=W)
    params = {k: v.astype(np.float64) for k, v in params.items()}
    target = wl.reference_image(H, W, seed=2) - 0.5
    g = obk.gradients(params, H, W, target, neumann=True)
    return H, W, params, target, g


def test_neumann_loss_gradient_matches_finite_differences(instance_neumann):
    H, W, params, target, g = instance_neumann
    rng = np.random.default_rng(1)
    checked = 0
    for name, rows in [("mean2d", 2), ("conic", 3), ("opacity", None), ("value", 6)]:
        for _ in range(6):
            k = int(rng.integers(0, 120))
            idx = (k,) if rows is None else (int(rng.integers(0, rows)), k)
            an = g[name][idx]
            fd, crossed = obk.finite_difference(params, H, W, target, name, idx, neumann=True)
            if crossed:
                continue
            scale = np.abs(g[name]).max()
            assert abs(fd - an) <= 1e-6 * scale + 1e-6 * abs(an), (name, idx, fd, an)
            checked += 1
    assert checked >= 20


def test_neumann_divergence_adjoint_identity():
    # <div(g), lam> = <g, div^T lam> for the Neumann divergence
    rng = np.random.default_rng(5)
    g = rng.standard_normal((6, 9, 13))
    lam = rng.standard_normal((3, 9, 13))
    lhs = float((P.divergence_neumann(g) * lam).sum())
    rhs = float((g * P.div_adjoint_neumann(lam)).sum())
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)
