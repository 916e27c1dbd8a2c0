"""Divergence and exact discrete Poisson solve, FP64 (test oracle).

Sec. 2 of GDGS links a gradient field to the image through the Poisson
equation: minimising (1/2)||grad f - g||^2 gives Laplacian(f) = div(g)
(Eq. 13-14); with rho = Laplacian(f) (Eq. 15) the image u solves
Laplacian(u) = rho (Eq. 16), and in image space Laplacian(c) = rho2D (Eq. 21).
The paper names direct (Gaussian elimination, LU) and iterative solvers; the
oracle uses exact direct solves of the discrete system.

Readings where the paper is silent (its boundary condition is Neumann, built
below; the main workloads fix Dirichlet data instead):
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


# ---------------------------------------------------------------- Neumann
# The paper's own boundary condition for the reconstruction is Neumann
# (Sec. 2.1 and Sec. 2.2, Eq. 21), with the image defined up to a constant.
# Reading used here: every one of the H x W pixels is an unknown and no flux
# crosses the image border, i.e. the discrete Laplacian at a pixel sums only
# its neighbours inside the image (these are the normal equations of the
# least-squares fit of forward-difference gradients, Eq. 13-14, over the
# differences that lie inside the image).  The system is singular with the
# constants as null space: rho is replaced by its compatible part (minus its
# mean) and the solution is fixed by a zero mean per channel.


def divergence_neumann(grad: np.ndarray) -> np.ndarray:
    """rho[3][H][W] on every pixel from grad[6][H][W]: the backward-difference
    divergence of the forward differences that lie inside the image (gx in
    the last column and gy in the last row would cross the border: dropped)."""
    grad = np.asarray(grad, dtype=np.float64)
    gx = grad[0::2].copy()
    gy = grad[1::2].copy()
    gx[:, :, -1] = 0.0
    gy[:, -1, :] = 0.0
    rho = gx + gy
    rho[:, :, 1:] -= gx[:, :, :-1]
    rho[:, 1:, :] -= gy[:, :-1, :]
    return rho


def div_adjoint_neumann(lam: np.ndarray) -> np.ndarray:
    """Transpose of ``divergence_neumann``: dgrad[6][H][W] with
    dgx[i,j] = lam[i,j] - lam[i,j+1] for j < W-1 and 0 in the last column,
    dgy[i,j] = lam[i,j] - lam[i+1,j] for i < H-1 and 0 in the last row."""
    lam = np.asarray(lam, dtype=np.float64)
    C, H, W = lam.shape
    out = np.zeros((2 * C, H, W))
    out[0::2, :, :-1] = lam[:, :, :-1] - lam[:, :, 1:]
    out[1::2, :-1, :] = lam[:, :-1, :] - lam[:, 1:, :]
    return out


def laplacian_neumann(u: np.ndarray) -> np.ndarray:
    """Graph Laplacian of the pixel grid: sum over the neighbours inside the
    image of (u_neighbour - u), on every pixel of u[C][H][W]."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros(u.shape)
    dy = u[:, 1:, :] - u[:, :-1, :]
    dx = u[:, :, 1:] - u[:, :, :-1]
    out[:, :-1, :] += dy
    out[:, 1:, :] -= dy
    out[:, :, :-1] += dx
    out[:, :, 1:] -= dx
    return out


def neumann_matrix(H: int, W: int) -> np.ndarray:
    """Dense -L for the H x W grid with no flux across the border (row-major
    unknowns): the degree of each pixel on the diagonal, -1 per neighbour."""
    def path(k):
        T = 2.0 * np.eye(k) - np.eye(k, k=1) - np.eye(k, k=-1)
        if k > 0:
            T[0, 0] -= 1.0
            T[-1, -1] -= 1.0
        return T
    return np.kron(np.eye(H), path(W)) + np.kron(path(H), np.eye(W))


def solve_neumann_dense(rho: np.ndarray) -> np.ndarray:
    """Zero-mean u with L u = rho - mean(rho), per channel, from the bordered
    system [A 1; 1^T 0] [u; s] = [mean(rho) - rho; 0] (A = -L), by LU."""
    rho = np.asarray(rho, dtype=np.float64)
    C, H, W = rho.shape
    N = H * W
    K = np.zeros((N + 1, N + 1))
    K[:N, :N] = neumann_matrix(H, W)
    K[:N, N] = 1.0
    K[N, :N] = 1.0
    lu = scipy.linalg.lu_factor(K)
    u = np.zeros(rho.shape)
    for c in range(C):
        b = np.zeros(N + 1)
        b[:N] = -(rho[c] - rho[c].mean()).ravel()
        u[c] = scipy.linalg.lu_solve(lu, b)[:N].reshape(H, W)
    return u


def neumann_eigenvalues(H: int, W: int) -> np.ndarray:
    """Eigenvalues of -L on the cosine basis cos(pi p (i + 1/2) / H) cos(pi q
    (j + 1/2) / W): (2 - 2cos(pi p / H)) + (2 - 2cos(pi q / W)), p < H, q < W."""
    p = np.arange(H)[:, None]
    q = np.arange(W)[None, :]
    return (2.0 - 2.0 * np.cos(np.pi * p / H)) + (2.0 - 2.0 * np.cos(np.pi * q / W))


def solve_neumann_dct(rho: np.ndarray, workers: int = -1) -> np.ndarray:
    """Zero-mean u with L u = rho - mean(rho), by diagonalising -L with the
    type-II discrete cosine transform; the constant mode is set to zero."""
    rho = np.asarray(rho, dtype=np.float64)
    C, H, W = rho.shape
    lam = neumann_eigenvalues(H, W)
    lam[0, 0] = 1.0
    u = np.zeros(rho.shape)
    for c in range(C):
        bh = scipy.fft.dctn(-rho[c], type=2, norm="ortho", workers=workers)
        bh /= lam
        bh[0, 0] = 0.0
        u[c] = scipy.fft.idctn(bh, type=2, norm="ortho", workers=workers)
    return u


def solve_neumann(rho: np.ndarray) -> np.ndarray:
    """Exact Neumann solve with zero-mean gauge: dense up to 2500 pixels, DCT
    beyond."""
    C, H, W = np.shape(rho)
    if H * W <= 2500:
        return solve_neumann_dense(rho)
    return solve_neumann_dct(rho)
