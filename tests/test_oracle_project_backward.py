"""Pins of the oracle's projection reverse mode: central finite differences
of a random linear functional of the projected mean and conic, taken through
the forward projection itself, for every 3D parameter."""
import numpy as np
import pytest

import workloads as wl
from oracle.project import project
from oracle.project_backward import project_backward


def _scene(K=6, seed=3):
    sc = wl.make_scene(K, seed=seed, z=(2.0, 4.0), ls=(-1.5, 0.3))
    f64 = lambda a: np.array(a, dtype=np.float64)
    return wl.Scene(mean=f64(sc.mean), log_scale=f64(sc.log_scale), quat=f64(sc.quat),
                    opacity=f64(sc.opacity), value=f64(sc.value))


def _functional(sc, cam, wm, wc):
    p = project(sc, cam)
    return float((wm * p["mean2d"]).sum() + (wc * p["conic"]).sum())


@pytest.mark.parametrize("name", ["mean", "log_scale", "quat"])
def test_matches_central_differences(name):
    sc = _scene()
    cam = wl.make_camera(64, 48, pose_index=4)
    rng = np.random.default_rng(9)
    K = sc.mean.shape[1]
    wm = rng.normal(size=(2, K))
    wc = rng.normal(size=(3, K)) * 1e2
    g = project_backward(sc, cam, wm, wc)[name]
    arr = getattr(sc, name)
    fd = np.zeros_like(arr)
    for i in range(arr.shape[0]):
        for k in range(K):
            h = 1e-6 * max(1.0, abs(arr[i, k]))
            old = arr[i, k]
            arr[i, k] = old + h
            fp = _functional(sc, cam, wm, wc)
            arr[i, k] = old - h
            fm = _functional(sc, cam, wm, wc)
            arr[i, k] = old
            fd[i, k] = (fp - fm) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 0
    assert np.abs(g - fd).max() <= 1e-5 * scale, (name, np.abs(g - fd).max(), scale)


def test_culled_splats_get_zero_gradients():
    sc = _scene(K=4)
    sc.quat[:, 0] = 0.0              # zero quaternion
    sc.mean[2, 1] = 0.1              # in front of the near plane
    cam = wl.make_camera(64, 48)
    g = project_backward(sc, cam, np.ones((2, 4)), np.ones((3, 4)))
    for v in g.values():
        assert np.all(v[:, :2] == 0) and np.all(np.isfinite(v))
