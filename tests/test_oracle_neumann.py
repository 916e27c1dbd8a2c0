"""Pins of the oracle's Neumann solve (Sec. 2.1 and Sec. 2.2, Eq. 21: no flux
across the image border, image defined up to a constant, fixed here by a
zero mean).  Checked against two independent exact methods (bordered dense
LU and the cosine transform), against the least-squares gradient fit the
equation comes from (Eq. 13-14, solved from the difference matrix alone),
the cosine eigenfunctions in closed form, a hand-solved 1 x 2 case, the
telescoping sum of the divergence, and the invariance to a constant added to
rho."""
import numpy as np
import pytest

import workloads as wl
from oracle import composite, poisson
from oracle.project import project
from oracle.render import render, render_laplacian


def _diff_matrix(H, W):
    """Forward differences inside the image, one row per difference (x first,
    then y), written out entry by entry."""
    rows = []
    for i in range(H):
        for j in range(W - 1):
            r = np.zeros(H * W)
            r[i * W + j + 1], r[i * W + j] = 1.0, -1.0
            rows.append(r)
    for i in range(H - 1):
        for j in range(W):
            r = np.zeros(H * W)
            r[(i + 1) * W + j], r[i * W + j] = 1.0, -1.0
            rows.append(r)
    return np.array(rows).reshape(-1, H * W)


@pytest.mark.parametrize("H,W", [(7, 5), (16, 16), (9, 13), (1, 6), (2, 2)])
def test_dense_and_cosine_solves_agree(H, W):
    rho = np.random.default_rng(H * 31 + W).standard_normal((3, H, W))
    a = poisson.solve_neumann_dense(rho)
    b = poisson.solve_neumann_dct(rho)
    assert np.abs(a - b).max() < 1e-11
    assert np.abs(a.mean(axis=(1, 2))).max() < 1e-13
    centred = rho - rho.mean(axis=(1, 2), keepdims=True)
    assert np.abs(poisson.laplacian_neumann(a) - centred).max() < 1e-11


@pytest.mark.parametrize("H,W", [(6, 9), (11, 4)])
def test_least_squares_gradient_fit(H, W):
    # Eq. 13: the image whose forward differences best fit g; lstsq returns
    # the minimum-norm minimiser, which is the zero-mean one
    rng = np.random.default_rng(H + 7 * W)
    grad = rng.standard_normal((6, H, W))
    D = _diff_matrix(H, W)
    u = poisson.solve_neumann(poisson.divergence_neumann(grad))
    for c in range(3):
        g = np.concatenate([grad[2 * c][:, :-1].ravel(), grad[2 * c + 1][:-1, :].ravel()])
        ls = np.linalg.lstsq(D, g, rcond=None)[0].reshape(H, W)
        assert np.abs(u[c] - ls).max() < 1e-10


def test_exact_gradients_recover_the_image_up_to_its_mean():
    H, W = 12, 17
    rng = np.random.default_rng(4)
    f = rng.uniform(0.0, 1.0, (3, H, W))
    grad = rng.standard_normal((6, H, W))  # border-crossing entries are garbage
    grad[0::2, :, :-1] = f[:, :, 1:] - f[:, :, :-1]
    grad[1::2, :-1, :] = f[:, 1:, :] - f[:, :-1, :]
    rho = poisson.divergence_neumann(grad)
    assert np.abs(rho - poisson.laplacian_neumann(f)).max() < 1e-13
    u = poisson.solve_neumann(rho)
    assert np.abs(u - (f - f.mean(axis=(1, 2), keepdims=True))).max() < 1e-12


@pytest.mark.parametrize("p,q", [(1, 0), (0, 3), (2, 5), (4, 1)])
def test_cosine_eigenfunctions(p, q):
    H, W = 10, 14
    i = np.arange(H)[:, None] + 0.5
    j = np.arange(W)[None, :] + 0.5
    v = np.cos(np.pi * p * i / H) * np.cos(np.pi * q * j / W)
    lam = (2 - 2 * np.cos(np.pi * p / H)) + (2 - 2 * np.cos(np.pi * q / W))
    v3 = np.stack([v, 2 * v, -v])
    assert np.abs(poisson.laplacian_neumann(v3) + lam * v3).max() < 1e-12
    assert np.abs(poisson.solve_neumann_dense(-lam * v3) - v3).max() < 1e-11
    assert np.abs(poisson.solve_neumann_dct(-lam * v3) - v3).max() < 1e-11


def test_hand_solved_two_pixel_case():
    # pixels a, b: (b - a) = 1, (a - b) = -1, a + b = 0
    u = poisson.solve_neumann_dense(np.array([[[1.0, -1.0]]]))
    assert np.abs(u - np.array([[[-0.5, 0.5]]])).max() < 1e-15


def test_divergence_sums_to_zero_and_constants_are_projected_out():
    rng = np.random.default_rng(9)
    grad = rng.standard_normal((6, 13, 8))
    rho = poisson.divergence_neumann(grad)
    assert np.abs(rho.sum(axis=(1, 2))).max() < 1e-12
    rho = rng.standard_normal((3, 13, 8))
    a = poisson.solve_neumann(rho)
    b = poisson.solve_neumann(rho + np.array([3.0, -1.0, 0.25])[:, None, None])
    assert np.abs(a - b).max() < 1e-12


def test_render_forms_satisfy_the_neumann_equation():
    H, W = 14, 19
    sc = wl.make_scene(60, seed=3, ls=(-2.5, 0.4))
    cam = wl.make_camera(W, H, pose_index=2)
    o = render(sc, cam, neumann=True)
    proj = project(sc, cam)
    grad = composite.render_grad(proj, sc.opacity, sc.value, H, W)
    assert np.abs(o["grad"] - grad).max() == 0.0
    rho = poisson.divergence_neumann(grad)
    assert np.abs(o["rho"] - rho).max() == 0.0
    centred = rho - rho.mean(axis=(1, 2), keepdims=True)
    assert np.abs(poisson.laplacian_neumann(o["u"]) - centred).max() < 1e-10
    assert np.abs(o["u"].mean(axis=(1, 2))).max() < 1e-13
    lp = wl.laplacian_scene(sc, seed=3)
    ol = render_laplacian(lp, cam, neumann=True)
    centred = ol["rho"] - ol["rho"].mean(axis=(1, 2), keepdims=True)
    assert np.abs(poisson.laplacian_neumann(ol["u"]) - centred).max() < 1e-10
