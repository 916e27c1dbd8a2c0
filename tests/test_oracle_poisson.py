"""Pins of the oracle's divergence and Poisson solve (Eq. 13-16, Eq. 21) by
discrete closed forms, identities and two independent direct solvers."""
import math

import numpy as np
import pytest

from oracle import poisson as P


@pytest.mark.parametrize("H,W,a,b", [(13, 21, 2, 3), (64, 64, 1, 1), (9, 40, 5, 7), (30, 17, 3, 1)])
@pytest.mark.parametrize("solver", ["dense", "dst"])
def test_sin_product_is_a_discrete_eigenfunction(H, W, a, b, solver):
    # u_ij = sin(pi a i/(H-1)) sin(pi b j/(W-1)) vanishes on the ring and satisfies
    # L u = [2cos(pi a/(H-1)) + 2cos(pi b/(W-1)) - 4] u exactly on the 5-point stencil.
    i = np.arange(H)[:, None]
    j = np.arange(W)[None, :]
    u = np.sin(math.pi * a * i / (H - 1)) * np.sin(math.pi * b * j / (W - 1))
    lam = 2 * math.cos(math.pi * a / (H - 1)) + 2 * math.cos(math.pi * b / (W - 1)) - 4
    rho = np.zeros((1, H, W))
    rho[0, 1:-1, 1:-1] = lam * u[1:-1, 1:-1]
    got = (P.solve_dense if solver == "dense" else P.solve_dst)(rho, None)[0]
    assert np.abs(got - u).max() < 1e-12
    assert np.abs(P.laplacian(u[None])[0, 1:-1, 1:-1] - lam * u[1:-1, 1:-1]).max() < 1e-13


def forward_diff(f):
    g = np.zeros((2 * f.shape[0],) + f.shape[1:])
    g[0::2, :, :-1] = f[:, :, 1:] - f[:, :, :-1]
    g[1::2, :-1, :] = f[:, 1:, :] - f[:, :-1, :]
    return g


@pytest.mark.parametrize("H,W", [(20, 31), (64, 64), (5, 3), (3, 3)])
def test_integrable_field_recovers_image(H, W):
    rng = np.random.default_rng(H * 100 + W)
    f = rng.normal(size=(3, H, W))
    g = forward_diff(f)
    # the unused last column of gx / last row of gy may hold anything
    g[0::2, :, -1] = rng.normal(size=(3, H))
    g[1::2, -1, :] = rng.normal(size=(3, W))
    rho = P.divergence(g)
    assert np.abs(rho[:, 1:-1, 1:-1] - P.laplacian(f)[:, 1:-1, 1:-1]).max() < 1e-12
    u = P.solve(rho, f)
    assert np.abs(u - f).max() < 1e-10
    # zero ring: the result is f minus the harmonic extension of f's ring
    u0 = P.solve(rho, None)
    h = P.solve(np.zeros_like(rho), f)
    assert np.abs(u0 + h - f).max() < 1e-10


def test_dense_lu_equals_dst():
    rng = np.random.default_rng(7)
    rho = rng.normal(size=(3, 62, 47))
    ring = rng.normal(size=(3, 62, 47))
    a = P.solve_dense(rho, ring)
    b = P.solve_dst(rho, ring)
    assert np.abs(a - b).max() < 1e-11
    assert P.relative_residual(a, rho, ring).max() < 1e-13
    assert P.relative_residual(b, rho, ring).max() < 1e-13


def test_system_matrix_spectrum_is_the_sine_basis_one():
    n, m = 7, 5
    A = P.system_matrix(n, m)
    assert np.array_equal(A, A.T)
    ev = np.sort(np.linalg.eigvalsh(A))
    ref = np.sort(P.dst_eigenvalues(n, m).ravel())
    assert np.abs(ev - ref).max() < 1e-12
    assert ev[0] > 0


def test_green_function_symmetry_and_sign():
    H, W = 15, 19
    p, q = (4, 6), (9, 13)
    rp = np.zeros((1, H, W)); rp[0][p] = 1.0
    rq = np.zeros((1, H, W)); rq[0][q] = 1.0
    up = P.solve(rp, None)[0]
    uq = P.solve(rq, None)[0]
    assert abs(up[q] - uq[p]) < 1e-14
    # a positive source of the Laplacian gives a non-positive potential (max principle)
    assert up.max() <= 1e-15 and up[p] < 0


def test_divergence_adjoint_dot_product():
    rng = np.random.default_rng(11)
    g = rng.normal(size=(6, 17, 23))
    lam = np.zeros((3, 17, 23))
    lam[:, 1:-1, 1:-1] = rng.normal(size=(3, 15, 21))
    lhs = (P.divergence(g) * lam).sum()
    rhs = (g * P.div_adjoint(lam)).sum()
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_solve_is_self_adjoint_with_zero_ring():
    rng = np.random.default_rng(12)
    x = np.zeros((1, 25, 18)); x[0, 1:-1, 1:-1] = rng.normal(size=(23, 16))
    y = np.zeros((1, 25, 18)); y[0, 1:-1, 1:-1] = rng.normal(size=(23, 16))
    a = (P.solve(x, None) * y).sum()
    b = (x * P.solve(y, None)).sum()
    assert abs(a - b) < 1e-12 * abs(a)


def test_backward_error_and_residual_of_exact_solution_are_tiny():
    rng = np.random.default_rng(13)
    rho = rng.normal(size=(3, 40, 33)) * 0.05
    ring = 0.5 + 0.1 * rng.normal(size=(3, 40, 33))
    u = P.solve(rho, ring)
    assert P.backward_error(u, rho, ring).max() < 1e-15
    u32 = u.astype(np.float32).astype(np.float64)
    assert P.backward_error(u32, rho, ring).max() < 1e-7
