"""Pins of the oracle's image loss (Eq. 22) and Adam update: SSIM of an image
with itself, closed forms for a constant offset, the filter against a direct
2D sum, central differences of the loss, and Adam's first step."""
import numpy as np

import workloads as wl
from oracle import loss as OL


def _imgs(H=13, W=17, seed=0):
    rng = np.random.default_rng(seed)
    im = wl.reference_image(H, W, seed=1).astype(np.float64)
    c = im + 0.05 * rng.normal(size=im.shape)
    return c, im


def test_filter_is_the_normalised_2d_gaussian_with_zero_padding():
    rng = np.random.default_rng(3)
    a = rng.normal(size=(9, 12))
    g = OL.gaussian_window()
    assert abs(g.sum() - 1.0) < 1e-15
    r = OL.WIN // 2
    ref = np.zeros_like(a)
    for i in range(9):
        for j in range(12):
            for di in range(-r, r + 1):
                for dj in range(-r, r + 1):
                    if 0 <= i + di < 9 and 0 <= j + dj < 12:
                        ref[i, j] += g[di + r] * g[dj + r] * a[i + di, j + dj]
    assert np.abs(OL.blur(a) - ref).max() < 1e-14


def test_identical_images_and_constant_offset():
    c, im = _imgs()
    o = OL.loss(im, im)
    assert o["loss"] == 0.0 and abs(o["dssim"]) < 1e-15
    assert np.abs(OL.ssim_map(im, im) - 1.0).max() < 1e-12
    o = OL.loss(im + 0.03, im, lam=0.0, beta=0.5)
    assert abs(o["l1"] - 0.03) < 1e-15 and o["grad_l1"] < 1e-15
    assert abs(o["loss"] - 0.03) < 1e-15


def test_gradient_matches_central_differences():
    c, im = _imgs(H=9, W=11)
    lam, beta = 0.2, 0.1
    o = OL.loss(c, im, lam, beta)
    rng = np.random.default_rng(5)
    idx = [tuple(rng.integers(0, s) for s in c.shape) for _ in range(25)]
    for p in idx:
        h = 1e-7
        cp, cm = c.copy(), c.copy()
        cp[p] += h
        cm[p] -= h
        fd = (OL.loss(cp, im, lam, beta)["loss"] - OL.loss(cm, im, lam, beta)["loss"]) / (2 * h)
        assert abs(fd - o["dc"][p]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (p, fd, o["dc"][p])


def test_adam_first_step_moves_by_lr_against_the_gradient_sign():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = OL.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-9, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    p, _, _ = OL.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=10.0, lo=-1.0, hi=2.0)
    assert np.array_equal(p, np.array([-1.0, 2.0, -1.0]))
