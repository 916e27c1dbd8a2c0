"""Projection of 3D Gaussians onto the image plane, FP64 (test oracle).

Follows Sec. 1.2 of GDGS: a splat's covariance is Sigma = R S S^T R^T with S
the diagonal scale matrix and R a rotation (here from a unit quaternion), and
its image-plane covariance is Sigma2D = J W Sigma W^T J^T (Eq. 10, repeated in
Sec. 2.2 "Projection", Eq. 19), where W is the world-to-camera rotation and J
the local affine (Jacobian) matrix of the projection at the splat mean.

Readings where the paper is silent:
* camera: OpenCV axes, x_c = R_cw x + t_cw, pinhole pi(x, y, z) =
  (fx x / z + cx, fy y / z + cy); J = d pi / d x_c at the mean;
* pixel (i, j) has centre (j + 1/2, i + 1/2);
* no low-pass dilation is added to Sigma2D;
* splats with z_c <= Z_NEAR, a zero quaternion or det(Sigma2D) <= 0 are culled;
* the support box of a splat: columns j with |j + 1/2 - mu_x| <=
  sqrt(E_CUT * Sigma2D_xx), rows likewise (the exact axis extent of the
  ellipse E <= E_CUT).
"""
from __future__ import annotations

import numpy as np

from .constants import E_CUT, Z_NEAR, TILE


def quat_to_rotmat(q: np.ndarray):
    """Rotation matrices R[3][3][K] of quaternions q[4][K] = (w, x, y, z),
    normalised first; also returns the mask of non-zero quaternions."""
    q = np.asarray(q, dtype=np.float64)
    n = np.sqrt((q * q).sum(axis=0))
    ok = n > 0
    w, x, y, z = q / np.where(ok, n, 1.0)
    R = np.empty((3, 3) + w.shape)
    R[0, 0] = 1 - 2 * (y * y + z * z)
    R[0, 1] = 2 * (x * y - w * z)
    R[0, 2] = 2 * (x * z + w * y)
    R[1, 0] = 2 * (x * y + w * z)
    R[1, 1] = 1 - 2 * (x * x + z * z)
    R[1, 2] = 2 * (y * z - w * x)
    R[2, 0] = 2 * (x * z - w * y)
    R[2, 1] = 2 * (y * z + w * x)
    R[2, 2] = 1 - 2 * (x * x + y * y)
    return R, ok


def covariance3d(log_scale: np.ndarray, quat: np.ndarray):
    """Sigma[3][3][K] = R diag(exp(2 l)) R^T, and the valid-quaternion mask."""
    R, ok = quat_to_rotmat(quat)
    s2 = np.exp(2.0 * np.asarray(log_scale, dtype=np.float64))
    Sigma = np.einsum("ijk,jk,ljk->ilk", R, s2, R)
    return Sigma, ok


def jacobian(xc: np.ndarray, fx: float, fy: float):
    """J[2][3][K], the derivative of the pinhole map at camera points xc[3][K]."""
    x, y, z = xc
    J = np.zeros((2, 3) + x.shape)
    J[0, 0] = fx / z
    J[0, 2] = -fx * x / (z * z)
    J[1, 1] = fy / z
    J[1, 2] = -fy * y / (z * z)
    return J


def pixel_box(mx, my, sxx, syy, W: int, H: int, valid):
    """Inclusive pixel index box (j0, j1, i0, i1) of each splat's support,
    clamped to the image; empty boxes have j0 > j1 or i0 > i1."""
    big = 4.0 * (W + H) + 64.0
    rx = np.sqrt(E_CUT * np.where(valid, sxx, 0.0))
    ry = np.sqrt(E_CUT * np.where(valid, syy, 0.0))
    clip = lambda v: np.clip(np.where(np.isfinite(v), v, -big), -big, big)
    j0 = np.ceil(clip(mx - rx - 0.5))
    j1 = np.floor(clip(mx + rx - 0.5))
    i0 = np.ceil(clip(my - ry - 0.5))
    i1 = np.floor(clip(my + ry - 0.5))
    j0 = np.maximum(j0, 0).astype(np.int64)
    i0 = np.maximum(i0, 0).astype(np.int64)
    j1 = np.minimum(j1, W - 1).astype(np.int64)
    i1 = np.minimum(i1, H - 1).astype(np.int64)
    empty = (~valid) | (j0 > j1) | (i0 > i1)
    return j0, j1, i0, i1, empty


def project(scene, cam) -> dict:
    """Project every splat of ``scene`` (FP32 arrays, upcast) with ``cam``.

    Returns FP64 arrays: mean2d[2][K], cov2d (sxx, sxy, syy), conic (a, b, c)
    with E = a dx^2 + 2 b dx dy + c dy^2, depth[K] (camera z), valid[K], the
    pixel box (j0, j1, i0, i1), the tile rectangle (tx0, tx1, ty0, ty1;
    half-open) and the tile count per splat.
    """
    mean = np.asarray(scene.mean, dtype=np.float64)
    Sigma, qok = covariance3d(scene.log_scale, scene.quat)
    Rcw = np.asarray(cam.R, dtype=np.float64)
    tcw = np.asarray(cam.t, dtype=np.float64)
    xc = Rcw @ mean + tcw[:, None]
    z = xc[2]
    valid = qok & (z > Z_NEAR)
    zs = np.where(valid, z, 1.0)
    xs = np.stack([xc[0], xc[1], zs])
    J = jacobian(xs, cam.fx, cam.fy)
    T = np.einsum("ijk,jl->ilk", J, Rcw)                  # J W
    cov = np.einsum("ijk,jlk,mlk->imk", T, Sigma, T)      # J W Sigma W^T J^T
    sxx, sxy, syy = cov[0, 0], cov[0, 1], cov[1, 1]
    det = sxx * syy - sxy * sxy
    valid &= det > 0
    dets = np.where(valid, det, 1.0)
    conic = np.stack([syy / dets, -sxy / dets, sxx / dets])
    mx = cam.fx * xs[0] / zs + cam.cx
    my = cam.fy * xs[1] / zs + cam.cy
    with np.errstate(invalid="ignore"):
        j0, j1, i0, i1, empty = pixel_box(mx, my, sxx, syy, cam.W, cam.H, valid)
    tx0, tx1 = j0 // TILE, j1 // TILE + 1
    ty0, ty1 = i0 // TILE, i1 // TILE + 1
    count = np.where(empty, 0, (tx1 - tx0) * (ty1 - ty0))
    return dict(mean2d=np.stack([mx, my]), cov2d=np.stack([sxx, sxy, syy]),
                conic=conic, depth=z, valid=valid, box=(j0, j1, i0, i1),
                empty=empty, tile_rect=(tx0, tx1, ty0, ty1), count=count)


def project_2d(mean2d, conic, depth, W: int, H: int) -> dict:
    """Rasteriser-level splats given directly in image space (mean2d[2][K],
    conic[3][K], depth[K]): returns the same dictionary as ``project``, with
    Sigma2D recovered as the inverse of the conic."""
    mean2d = np.asarray(mean2d, dtype=np.float64)
    a, b, c = np.asarray(conic, dtype=np.float64)
    det = a * c - b * b
    valid = det > 0
    dets = np.where(valid, det, 1.0)
    sxx, sxy, syy = c / dets, -b / dets, a / dets
    mx, my = mean2d
    with np.errstate(invalid="ignore"):
        j0, j1, i0, i1, empty = pixel_box(mx, my, sxx, syy, W, H, valid)
    tx0, tx1 = j0 // TILE, j1 // TILE + 1
    ty0, ty1 = i0 // TILE, i1 // TILE + 1
    count = np.where(empty, 0, (tx1 - tx0) * (ty1 - ty0))
    return dict(mean2d=mean2d, cov2d=np.stack([sxx, sxy, syy]),
                conic=np.stack([a, b, c]), depth=np.asarray(depth, dtype=np.float64),
                valid=valid, box=(j0, j1, i0, i1), empty=empty,
                tile_rect=(tx0, tx1, ty0, ty1), count=count)
