"""Pins of the oracle's projection (Sec. 1.2, Eq. 10; Sec. 2.2, Eq. 19) against
closed forms and independent computations."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import project as op
from oracle.constants import E_CUT


def one_splat(mean, log_scale, quat, opacity=0.5, value=None):
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1, 1))
    v = np.zeros(6) if value is None else value
    return wl.Scene(mean=f(mean), log_scale=f(log_scale), quat=f(quat),
                    opacity=np.array([opacity], np.float32), value=f(v))


def test_rotation_matrix_is_a_rotation_and_sign_invariant():
    rng = np.random.default_rng(3)
    q = rng.normal(size=(4, 500))
    R, ok = op.quat_to_rotmat(q)
    assert ok.all()
    RtR = np.einsum("jik,jlk->ilk", R, R)
    assert np.abs(RtR - np.eye(3)[:, :, None]).max() < 1e-14
    det = np.linalg.det(np.moveaxis(R, 2, 0))
    assert np.abs(det - 1).max() < 1e-14
    R2, _ = op.quat_to_rotmat(-q)
    assert np.abs(R - R2).max() < 1e-15
    Rs, _ = op.quat_to_rotmat(3.7 * q)           # normalised inside
    assert np.abs(R - Rs).max() < 1e-14


def test_rotation_matrix_textbook_cases():
    I, _ = op.quat_to_rotmat(np.array([[1.0], [0], [0], [0]]))
    assert np.abs(I[:, :, 0] - np.eye(3)).max() == 0
    # 90 degrees about +z: q = (cos 45, 0, 0, sin 45) maps e_x to e_y.
    h = math.sqrt(0.5)
    R, _ = op.quat_to_rotmat(np.array([[h], [0], [0], [h]]))
    assert np.allclose(R[:, :, 0] @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    assert np.allclose(R[:, :, 0] @ [0, 1, 0], [-1, 0, 0], atol=1e-15)
    # 90 degrees about +x maps e_y to e_z.
    R, _ = op.quat_to_rotmat(np.array([[h], [h], [0], [0]]))
    assert np.allclose(R[:, :, 0] @ [0, 1, 0], [0, 0, 1], atol=1e-15)


def test_isotropic_on_axis_closed_form():
    s, z, f = 0.05, 3.0, 64.0
    sc = one_splat([0, 0, z], [math.log(s)] * 3, [0.3, -0.2, 0.5, 0.7])
    cam = wl.make_camera(64, 48, fx=f)
    p = op.project(sc, cam)
    sig = f * math.exp(float(np.float32(math.log(s)))) / z
    assert np.allclose(p["cov2d"][:, 0], [sig ** 2, 0, sig ** 2], rtol=1e-12, atol=1e-15)
    assert np.allclose(p["conic"][:, 0], [1 / sig ** 2, 0, 1 / sig ** 2], rtol=1e-12)
    assert np.allclose(p["mean2d"][:, 0], [32.0, 24.0])
    assert p["depth"][0] == z


def test_anisotropic_axis_aligned_and_rotated_about_view_axis():
    f, z = 100.0, 4.0
    sx, sy, sz = 0.2, 0.05, 0.7
    ls = np.log(np.array([sx, sy, sz], np.float32).astype(np.float64))
    sx, sy = np.exp(np.float32(ls[0])), np.exp(np.float32(ls[1]))
    cam = wl.make_camera(200, 200, fx=f)
    p = op.project(one_splat([0, 0, z], ls, [1, 0, 0, 0]), cam)
    assert np.allclose(p["cov2d"][:, 0], [(f * sx / z) ** 2, 0, (f * sy / z) ** 2], rtol=1e-6)
    # rotate the splat by theta about +z: Sigma2D = R2 diag R2^T, positive xy term
    th = math.radians(30)
    q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
    p = op.project(one_splat([0, 0, z], ls, q), cam)
    c, s_ = math.cos(th), math.sin(th)
    R2 = np.array([[c, -s_], [s_, c]])
    ref = R2 @ np.diag([(f * sx / z) ** 2, (f * sy / z) ** 2]) @ R2.T
    sxx, sxy, syy = p["cov2d"][:, 0]
    assert np.allclose([sxx, sxy, syy], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-5)
    assert sxy > 0
    a, b, c_ = p["conic"][:, 0]
    assert np.allclose(np.array([[a, b], [b, c_]]) @ np.array([[sxx, sxy], [sxy, syy]]), np.eye(2),
                       atol=1e-12)


def test_off_axis_isotropic_equals_s2_J_JT_with_finite_difference_jacobian():
    s = 0.03
    x = np.array([0.4, -0.3, 2.5])
    cam = wl.make_camera(320, 240, fx=300.0)
    cam.fy = 280.0
    p = op.project(one_splat(x, [math.log(s)] * 3, [1, 0, 0, 0]), cam)
    s = math.exp(float(np.float32(math.log(s))))
    x = x.astype(np.float32).astype(np.float64)

    def pinhole(v):
        return np.array([cam.fx * v[0] / v[2] + cam.cx, cam.fy * v[1] / v[2] + cam.cy])

    h = 1e-6
    J = np.stack([(pinhole(x + h * e) - pinhole(x - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    ref = s * s * J @ J.T
    sxx, sxy, syy = p["cov2d"][:, 0]
    assert np.allclose([sxx, sxy, syy], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-7)
    assert np.allclose(p["mean2d"][:, 0], pinhole(x), rtol=1e-14)


def test_camera_pose_acts_on_mean_and_covariance():
    """A splat seen by a posed camera equals the splat moved by (R, t) and
    rotated by R, seen by the identity camera."""
    rng = np.random.default_rng(9)
    for idx in range(5):
        cam = wl.make_camera(400, 300, pose_index=idx)
        mean = np.array([0.3, -0.2, 3.0])
        ls = np.log(np.array([0.1, 0.02, 0.05]))
        q = rng.normal(size=4)
        sc = one_splat(mean, ls, q)
        p = op.project(sc, cam)
        # moved splat: rotate its frame by cam.R (compose quaternions via matrices)
        Rs, _ = op.quat_to_rotmat(sc.quat.astype(np.float64))
        Rnew = cam.R @ Rs[:, :, 0]
        Sig_new = Rnew @ np.diag(np.exp(2 * sc.log_scale[:, 0].astype(np.float64))) @ Rnew.T
        xc = cam.R @ sc.mean[:, 0].astype(np.float64) + cam.t
        J = op.jacobian(xc.reshape(3, 1), cam.fx, cam.fy)[:, :, 0]
        ref = J @ Sig_new @ J.T
        sxx, sxy, syy = p["cov2d"][:, 0]
        assert np.allclose([sxx, sxy, syy], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-10)


def test_culling():
    cam = wl.make_camera(64, 64)
    near = op.project(one_splat([0, 0, 0.19], [-3] * 3, [1, 0, 0, 0]), cam)
    assert not near["valid"][0] and near["count"][0] == 0
    zero_q = op.project(one_splat([0, 0, 3], [-3] * 3, [0, 0, 0, 0]), cam)
    assert not zero_q["valid"][0] and zero_q["count"][0] == 0
    behind = op.project(one_splat([0, 0, -3], [-3] * 3, [1, 0, 0, 0]), cam)
    assert behind["count"][0] == 0
    outside = op.project(one_splat([50, 0, 3], [-3] * 3, [1, 0, 0, 0]), cam)
    assert outside["valid"][0] and outside["count"][0] == 0


def test_pixel_box_contains_support_bruteforce():
    sc = wl.make_scene(300, seed=4, ls=(-2.5, 0.5))
    cam = wl.make_camera(70, 45)
    p = op.project(sc, cam)
    j0, j1, i0, i1 = p["box"]
    py, px = np.meshgrid(np.arange(45) + 0.5, np.arange(70) + 0.5, indexing="ij")
    hits = 0
    for k in np.nonzero(p["valid"])[0]:
        dx = px - p["mean2d"][0, k]
        dy = py - p["mean2d"][1, k]
        a, b, c = p["conic"][:, k]
        E = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        ii, jj = np.nonzero(E <= E_CUT)
        if ii.size:
            hits += 1
            assert not p["empty"][k]
            assert j0[k] <= jj.min() and jj.max() <= j1[k]
            assert i0[k] <= ii.min() and ii.max() <= i1[k]
    assert hits > 50


def test_pixel_box_is_tight_for_axis_aligned_splat_on_pixel_row():
    # centre on a pixel-centre row, axis aligned: the extreme columns are attained
    cam = wl.make_camera(64, 64, fx=64)
    sc = one_splat([0, 0, 4], [math.log(0.2), math.log(0.1), -3], [1, 0, 0, 0])
    p = op.project(sc, cam)
    sig = 64 * math.exp(float(np.float32(math.log(0.2)))) / 4
    r = math.sqrt(E_CUT) * sig
    j0, j1 = p["box"][0][0], p["box"][1][0]
    assert j0 == math.ceil(32 - r - 0.5) and j1 == math.floor(32 + r - 0.5)
