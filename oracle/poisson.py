"""Divergence and exact discrete Poisson solve, FP64 (test oracle).

Sec. 2 of GDGS links a gradient field to the image through the Poisson
equation: minimising (1/2)||grad f - g||^2 gives Laplacian(f) = div(g)
(Eq. 13-14); with rho = Laplacian(f) (Eq. 15) the image u solves
Laplacian(u) = rho (Eq. 16), and in image space Laplacian(c) = rho2D (Eq. 21).
The paper names direct (Gaussian elimination, LU) and iterative solvers; the
oracle uses exact direct solves of the discrete system.

Readings where the paper is silent (its boundary condition is Neumann; the
workloads here fix Dirichlet data instead):
* grid = the H x W pixel grid, spacing 1; unknowns are the (H-2) x (W-2)
  interior pixels, the one-pixel outer ring holds Dirichlet values g;
* gradients are forward differences, gx[i,j] ~ f[i,j+1] - f[i,j] (channel
  2c), gy[i,j] ~ f[i+1,j] - f[i,j] (channel 2c+1); the divergence is the
  backward difference rho[i,j] = gx[i,j] - gx[i,j-1] + gy[i,j] - gy[i-1,j]
  on interior pixels, so div(grad f) is exactly the 5-point Laplacian;
* Laplacian(u)[i,j] = u[i-1,j] + u[i+1,j] + u[i,j-1] + u[i,j+1] - 4 u[i,j].
  Written as A w = b on the interior: A = -L_int (symmetric positive
  definite), b = -rho_int + sum of ring neighbours' g.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg


def divergence(grad: np.ndarray) -> np.ndarray:
    """rho[3][H][W] from grad[6][H][W]; zero on the ring."""
    grad = np.asarray(grad, dtype=np.float64)
    gx, gy = grad[0::2], grad[1::2]
    rho = np.zeros(gx.shape)
    rho[:, 1:-1, 1:-1] = (gx[:, 1:-1, 1:-1] - gx[:, 1:-1, :-2]
                          + gy[:, 1:-1, 1:-1] - gy[:, :-2, 1:-1])
    return rho


def div_adjoint(lam: np.ndarray) -> np.ndarray:
    """Transpose of ``divergence`` (interior rows of lam are used): returns
    dgrad[6][H][W] with dgx[i,j] = lam[i,j] - lam[i,j+1] and dgy[i,j] =
    lam[i,j] - lam[i+1,j], lam taken as 0 outside the interior."""
    lam = np.asarray(lam, dtype=np.float64)
    C, H, W = lam.shape
    li = np.zeros((C, H + 1, W + 1))
    li[:, 1:H - 1, 1:W - 1] = lam[:, 1:-1, 1:-1]
    out = np.zeros((2 * C, H, W))
    out[0::2] = li[:, :H, :W] - li[:, :H, 1:W + 1]
    out[1::2] = li[:, :H, :W] - li[:, 1:H + 1, :W]
    return out


def laplacian(u: np.ndarray) -> np.ndarray:
    """5-point Laplacian on interior pixels of u[C][H][W]; zero on the ring."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros(u.shape)
    out[:, 1:-1, 1:-1] = (u[:, :-2, 1:-1] + u[:, 2:, 1:-1] + u[:, 1:-1, :-2]
                          + u[:, 1:-1, 2:] - 4.0 * u[:, 1:-1, 1:-1])
    return out


def ring_of(boundary, shape) -> np.ndarray:
    """Image whose ring holds the Dirichlet data and whose interior is zero."""
    g = np.zeros(shape)
    if boundary is not None:
        b = np.asarray(boundary, dtype=np.float64)
        g[:, 0, :], g[:, -1, :] = b[:, 0, :], b[:, -1, :]
        g[:, :, 0], g[:, :, -1] = b[:, :, 0], b[:, :, -1]
    return g


def rhs(rho: np.ndarray, boundary) -> np.ndarray:
    """b[C][H-2][W-2] = -rho_int + the ring neighbours' Dirichlet values."""
    g = ring_of(boundary, np.shape(rho))
    return -np.asarray(rho, dtype=np.float64)[:, 1:-1, 1:-1] + laplacian(g)[:, 1:-1, 1:-1]


def system_matrix(n: int, m: int) -> np.ndarray:
    """Dense A = -L_int for an n x m interior (row-major unknowns)."""
    T = lambda k: 2.0 * np.eye(k) - np.eye(k, k=1) - np.eye(k, k=-1)
    return np.kron(np.eye(n), T(m)) + np.kron(T(n), np.eye(m))


def solve_dense(rho: np.ndarray, boundary=None) -> np.ndarray:
    """u[C][H][W] by LU factorisation of the dense interior system."""
    C, H, W = np.shape(rho)
    n, m = H - 2, W - 2
    u = ring_of(boundary, (C, H, W))
    if n <= 0 or m <= 0:
        return u
    lu = scipy.linalg.lu_factor(system_matrix(n, m))
    b = rhs(rho, boundary)
    for c in range(C):
        u[c, 1:-1, 1:-1] = scipy.linalg.lu_solve(lu, b[c].ravel()).reshape(n, m)
    return u


def dst_eigenvalues(n: int, m: int) -> np.ndarray:
    """Eigenvalues of A = -L_int on the sine basis: mu_pq = (2 - 2cos(pi p/(n+1)))
    + (2 - 2cos(pi q/(m+1))), p = 1..n, q = 1..m."""
    p = np.arange(1, n + 1)[:, None]
    q = np.arange(1, m + 1)[None, :]
    return (2.0 - 2.0 * np.cos(np.pi * p / (n + 1))) + (2.0 - 2.0 * np.cos(np.pi * q / (m + 1)))


def solve_dst(rho: np.ndarray, boundary=None, workers: int = -1) -> np.ndarray:
    """u[C][H][W] by diagonalising A with the type-I discrete sine transform
    (the textbook fast direct Poisson solver on a rectangle)."""
    C, H, W = np.shape(rho)
    n, m = H - 2, W - 2
    u = ring_of(boundary, (C, H, W))
    if n <= 0 or m <= 0:
        return u
    b = rhs(rho, boundary)
    mu = dst_eigenvalues(n, m)
    for c in range(C):
        bh = scipy.fft.dstn(b[c], type=1, workers=workers)
        u[c, 1:-1, 1:-1] = scipy.fft.idstn(bh / mu, type=1, workers=workers)
    return u


def solve(rho: np.ndarray, boundary=None) -> np.ndarray:
    """Exact solve: dense LU up to 4096 unknowns, DST-I beyond."""
    C, H, W = np.shape(rho)
    if (H - 2) * (W - 2) <= 4096:
        return solve_dense(rho, boundary)
    return solve_dst(rho, boundary)


def residual(u: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """r = rho - L u on the interior ([C][H-2][W-2]); equals b - A w."""
    return (np.asarray(rho, dtype=np.float64) - laplacian(u))[:, 1:-1, 1:-1]


def relative_residual(u: np.ndarray, rho: np.ndarray, boundary=None) -> np.ndarray:
    """Per channel ||b - A w||_2 / ||b||_2."""
    r = residual(u, rho)
    b = rhs(rho, boundary)
    num = np.sqrt((r * r).sum(axis=(1, 2)))
    den = np.sqrt((b * b).sum(axis=(1, 2)))
    return num / np.where(den > 0, den, 1.0)


def backward_error(u: np.ndarray, rho: np.ndarray, boundary=None) -> np.ndarray:
    """Per channel normwise backward error in the infinity norm,
    ||b - A w|| / (||A|| ||w|| + ||b||) with ||A||_inf = 8."""
    r = residual(u, rho)
    b = rhs(rho, boundary)
    w = np.asarray(u, dtype=np.float64)[:, 1:-1, 1:-1]
    num = np.abs(r).max(axis=(1, 2))
    den = 8.0 * np.abs(w).max(axis=(1, 2)) + np.abs(b).max(axis=(1, 2))
    return num / np.where(den > 0, den, 1.0)
