"""Reverse mode of the projection (test oracle, FP64): gradients of a loss
with respect to the 3D splat parameters (world mean, log-scales, quaternion)
from its gradients with respect to the projected mean and conic.

The forward map is Sec. 1.2 / Sec. 2.2 "Projection" (Eq. 10 and Eq. 19):
x_c = W x + t, mu = pinhole(x_c), Sigma = R(q/|q|) diag(exp(2 l)) R^T,
Sigma2D = T Sigma T^T with T = J W and J the pinhole Jacobian at x_c, and the
conic A = Sigma2D^{-1} stored as (a, b, c), E = a dx^2 + 2 b dx dy + c dy^2.
The chain rule is taken step by step in that order, backwards:

* conic -> Sigma2D: with G_A the gradient as a symmetric matrix
  ([[ga, gb/2], [gb/2, gc]], since b fills two entries),
  G_Sigma2D = -A G_A A;
* Sigma2D = T Sigma T^T: G_T = 2 G_Sigma2D T Sigma, G_Sigma = T^T G_Sigma2D T;
* T = J W: G_J = G_T W^T; J and mu depend on x_c; G_x = W^T G_xc;
* Sigma = M M^T, M = R S: G_M = 2 G_Sigma M, G_R = G_M S, G_s = diag(R^T G_M),
  G_l = G_s * s;
* R(q_hat): the derivative of each entry of the rotation matrix formula;
  q_hat = q / |q|: G_q = (G_qhat - q_hat (q_hat . G_qhat)) / |q|.

Culled splats (zero quaternion, z_c <= Z_NEAR, det <= 0) get zero gradients.
"""
from __future__ import annotations

import numpy as np

from .project import covariance3d, jacobian, quat_to_rotmat
from .constants import Z_NEAR


def rotmat_vjp(qh: np.ndarray, GR: np.ndarray) -> np.ndarray:
    """Gradient with respect to the unit quaternion (w, x, y, z)[4][K] of
    sum(GR * R(q)) for R the rotation-matrix formula of quat_to_rotmat."""
    w, x, y, z = qh
    g = GR
    gw = 2 * (-z * g[0, 1] + y * g[0, 2] + z * g[1, 0] - x * g[1, 2] - y * g[2, 0] + x * g[2, 1])
    gx = 2 * (y * g[0, 1] + z * g[0, 2] + y * g[1, 0] - 2 * x * g[1, 1] - w * g[1, 2]
              + z * g[2, 0] + w * g[2, 1] - 2 * x * g[2, 2])
    gy = 2 * (-2 * y * g[0, 0] + x * g[0, 1] + w * g[0, 2] + x * g[1, 0] + z * g[1, 2]
              - w * g[2, 0] + z * g[2, 1] - 2 * y * g[2, 2])
    gz = 2 * (-2 * z * g[0, 0] - w * g[0, 1] + x * g[0, 2] + w * g[1, 0] - 2 * z * g[1, 1]
              + y * g[1, 2] + x * g[2, 0] + y * g[2, 1])
    return np.stack([gw, gx, gy, gz])


def project_backward(scene, cam, dmean2d, dconic) -> dict:
    """dmean2d[2][K], dconic[3][K] -> gradients mean[3][K], log_scale[3][K],
    quat[4][K] (FP64)."""
    mean = np.asarray(scene.mean, dtype=np.float64)
    ls = np.asarray(scene.log_scale, dtype=np.float64)
    q = np.asarray(scene.quat, dtype=np.float64)
    gm = np.asarray(dmean2d, dtype=np.float64)
    gc = np.asarray(dconic, dtype=np.float64)
    K = mean.shape[1]
    Wc = np.asarray(cam.R, dtype=np.float64)
    t = np.asarray(cam.t, dtype=np.float64)
    R, qok = quat_to_rotmat(q)
    Sigma, _ = covariance3d(ls, q)
    xc = Wc @ mean + t[:, None]
    X, Y, Z = xc
    valid = qok & (Z > Z_NEAR)
    Zs = np.where(valid, Z, 1.0)
    J = jacobian(np.stack([X, Y, Zs]), cam.fx, cam.fy)
    T = np.einsum("ijk,jl->ilk", J, Wc)
    S2 = np.einsum("ijk,jlk,mlk->imk", T, Sigma, T)
    det = S2[0, 0] * S2[1, 1] - S2[0, 1] ** 2
    valid &= det > 0
    dets = np.where(valid, det, 1.0)
    A = np.stack([np.stack([S2[1, 1], -S2[0, 1]]), np.stack([-S2[1, 0], S2[0, 0]])]) / dets
    GA = np.stack([np.stack([gc[0], 0.5 * gc[1]]), np.stack([0.5 * gc[1], gc[2]])])
    GS2 = -np.einsum("ijk,jlk,lmk->imk", A, GA, A)
    GT = 2.0 * np.einsum("ijk,jlk,lmk->imk", GS2, T, Sigma)
    GSig = np.einsum("jik,jlk,lmk->imk", T, GS2, T)
    GJ = np.einsum("ijk,lj->ilk", GT, Wc)
    fx, fy = cam.fx, cam.fy
    gX = GJ[0, 2] * (-fx / Zs ** 2) + gm[0] * (fx / Zs)
    gY = GJ[1, 2] * (-fy / Zs ** 2) + gm[1] * (fy / Zs)
    gZ = (GJ[0, 0] * (-fx / Zs ** 2) + GJ[0, 2] * (2 * fx * X / Zs ** 3)
          + GJ[1, 1] * (-fy / Zs ** 2) + GJ[1, 2] * (2 * fy * Y / Zs ** 3)
          + gm[0] * (-fx * X / Zs ** 2) + gm[1] * (-fy * Y / Zs ** 2))
    gmean = Wc.T @ np.stack([gX, gY, gZ])
    s = np.exp(ls)
    M = R * s[None, :, :]
    GM = 2.0 * np.einsum("ijk,jlk->ilk", GSig, M)
    GR = GM * s[None, :, :]
    gs = (R * GM).sum(axis=0)
    gls = gs * s
    n = np.sqrt((q * q).sum(axis=0))
    qh = q / np.where(qok, n, 1.0)
    gqh = rotmat_vjp(qh, GR)
    gq = (gqh - qh * (qh * gqh).sum(axis=0)) / np.where(qok, n, 1.0)
    z = lambda a: np.where(valid, a, 0.0)
    return dict(mean=z(gmean), log_scale=z(gls), quat=z(gq))
