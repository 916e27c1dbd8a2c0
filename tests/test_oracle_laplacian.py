"""Pins of the oracle's Laplacian-splat form (Sec. 2.2): the composite of the
splats' Laplacian values is the right-hand side of the Poisson equation
(Eq. 21) itself.  Checked against the equation (5-point Laplacian of the
result equals the composite on the interior, ring equals the Dirichlet
data), linearity in the carried values, the harmonic extension for zero
values, and the gradient form's composite for the same values."""
import numpy as np

import workloads as wl
from oracle import composite, poisson
from oracle.project import project
from oracle.render import render_laplacian

H, W = 14, 19


def _scene(seed, K=60):
    sc = wl.make_scene(K, seed=seed, ls=(-2.5, 0.4))
    return wl.laplacian_scene(sc, seed=seed)


def test_result_satisfies_the_poisson_equation_with_the_composite_as_rhs():
    sc = _scene(1)
    cam = wl.make_camera(W, H, pose_index=2)
    ring = wl.reference_image(H, W, seed=1)
    o = render_laplacian(sc, cam, ring)
    assert o["rho"].shape == (3, H, W) and np.abs(o["rho"]).max() > 1e-3
    lap = poisson.laplacian(o["u"])
    assert np.abs(lap[:, 1:-1, 1:-1] - o["rho"][:, 1:-1, 1:-1]).max() < 1e-10
    for side in (o["u"][:, 0, :] - ring[:, 0, :], o["u"][:, -1, :] - ring[:, -1, :],
                 o["u"][:, :, 0] - ring[:, :, 0], o["u"][:, :, -1] - ring[:, :, -1]):
        assert np.abs(side).max() == 0.0


def test_linear_in_the_carried_values_and_harmonic_for_zero_values():
    a, b = _scene(2), _scene(3)
    b = wl.Scene(mean=a.mean, log_scale=a.log_scale, quat=a.quat, opacity=a.opacity,
                 value=b.value)
    s = wl.Scene(mean=a.mean, log_scale=a.log_scale, quat=a.quat, opacity=a.opacity,
                 value=(a.value.astype(np.float64) + b.value.astype(np.float64)))
    cam = wl.make_camera(W, H, pose_index=4)
    ua, ub, us = (render_laplacian(x, cam)["u"] for x in (a, b, s))
    assert np.abs(us - ua - ub).max() < 1e-12
    ring = wl.reference_image(H, W, seed=5)
    z = wl.Scene(mean=a.mean, log_scale=a.log_scale, quat=a.quat, opacity=a.opacity,
                 value=np.zeros_like(a.value))
    uz = render_laplacian(z, cam, ring)["u"]
    assert np.abs(poisson.laplacian(uz)[:, 1:-1, 1:-1]).max() < 1e-10


def test_composite_matches_the_gradient_forms_channels():
    # the same splats carrying (lap_r, lap_g, lap_b, 0, 0, 0) in the six-value
    # form composite to the same first three channels
    sc = _scene(6)
    cam = wl.make_camera(W, H, pose_index=1)
    six = np.zeros((6, sc.value.shape[1]))
    six[:3] = sc.value
    proj = project(sc, cam)
    g6 = composite.render_grad(proj, sc.opacity, six, H, W)
    o = render_laplacian(sc, cam)
    assert np.array_equal(g6[:3], o["rho"]) and np.abs(g6[3:]).max() == 0.0


def test_hard_threshold_of_eq_24():
    from oracle.render import threshold
    x = np.array([-0.5, 0.002, 0.003, -0.003, 0.0, 0.0031])
    assert np.array_equal(threshold(x, 0.003), np.array([-0.5, 0.0, 0.003, -0.003, 0.0, 0.0031]))
    assert np.array_equal(threshold(x, 0.0), x)
    # thresholding the composite before the solve: u solves L u = T(rho)
    sc = _scene(4)
    cam = wl.make_camera(W, H, pose_index=3)
    full = render_laplacian(sc, cam)
    t = 0.5 * np.abs(full["rho"]).mean()
    o = render_laplacian(sc, cam, t=t)
    assert 0 < np.count_nonzero(o["rho"]) < np.count_nonzero(full["rho"])
    lap = poisson.laplacian(o["u"])
    assert np.abs(lap[:, 1:-1, 1:-1] - threshold(full["rho"], t)[:, 1:-1, 1:-1]).max() < 1e-10
