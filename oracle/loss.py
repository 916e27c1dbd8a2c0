"""Image loss of the method's optimisation (test oracle, FP64), Sec. 2.3
"Loss Function" (Eq. 22) as evaluated in each iteration of Algorithm 1:

    L(c, im) = (1 - lam) |c - im|_1 + beta |grad c - grad im|_1 + lam D_SSIM(c, im),

and its gradient with respect to the rendered image c.

Readings where the paper is silent (the loss extends the one of 3D Gaussian
Splatting that the paper builds on):
* |.|_1 terms are means: over the 3 H W values for the first, over the
  3 (H (W-1) + (H-1) W) forward differences (along columns, then rows) for
  the second;
* D_SSIM = 1 - mean SSIM over the 3 H W values, SSIM per colour channel with
  an 11 x 11 Gaussian window (sigma 1.5, weights normalised to sum 1) applied
  with zero padding ("same" size), C1 = 0.01^2, C2 = 0.03^2:
  SSIM = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sx^2 + sy^2 + C2))
  with mx = G*x, sx^2 = G*(x^2) - mx^2, sxy = G*(x y) - mx my;
* lam = 0.2 and beta = 0.1 unless given;
* the sign of 0 is 0.
"""
from __future__ import annotations

import numpy as np

C1, C2 = 0.01 ** 2, 0.03 ** 2
WIN, SIGMA = 11, 1.5


def gaussian_window() -> np.ndarray:
    x = np.arange(WIN) - WIN // 2
    g = np.exp(-(x * x) / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def blur(img: np.ndarray) -> np.ndarray:
    """Separable Gaussian filter of each 2D plane of img[..., H, W], zero
    padding, output the same size."""
    g = gaussian_window()
    r = WIN // 2
    a = np.asarray(img, dtype=np.float64)
    same = lambda v: np.convolve(v, g, mode="full")[r:r + v.size]  # g is symmetric
    rows = np.apply_along_axis(same, -1, a)
    return np.apply_along_axis(same, -2, rows)


def _maps(c, im):
    x, y = np.asarray(c, np.float64), np.asarray(im, np.float64)
    m1, m2 = blur(x), blur(y)
    m11, m22, m12 = blur(x * x), blur(y * y), blur(x * y)
    A1 = 2 * m1 * m2 + C1
    A2 = 2 * (m12 - m1 * m2) + C2
    B1 = m1 * m1 + m2 * m2 + C1
    B2 = (m11 - m1 * m1) + (m22 - m2 * m2) + C2
    return x, y, m1, m2, A1, A2, B1, B2


def ssim_map(c, im) -> np.ndarray:
    _, _, _, _, A1, A2, B1, B2 = _maps(c, im)
    return (A1 * A2) / (B1 * B2)


def loss(c, im, lam: float = 0.2, beta: float = 0.1) -> dict:
    """Loss terms and dL/dc for images c, im [3][H][W]."""
    x, y, m1, m2, A1, A2, B1, B2 = _maps(c, im)
    n = x.size
    d = x - y
    l1 = np.abs(d).mean()
    dl1 = np.sign(d) / n
    gx = (x[:, :, 1:] - x[:, :, :-1]) - (y[:, :, 1:] - y[:, :, :-1])
    gy = (x[:, 1:, :] - x[:, :-1, :]) - (y[:, 1:, :] - y[:, :-1, :])
    ng = gx.size + gy.size
    lg = (np.abs(gx).sum() + np.abs(gy).sum()) / ng
    sx, sy = np.sign(gx) / ng, np.sign(gy) / ng
    dlg = np.zeros(x.shape)
    dlg[:, :, 1:] += sx
    dlg[:, :, :-1] -= sx
    dlg[:, 1:, :] += sy
    dlg[:, :-1, :] -= sy
    S = (A1 * A2) / (B1 * B2)
    dssim = 1.0 - S.mean()
    # partial derivatives of S with respect to m1, m11 and m12 (x = c)
    BB = B1 * B2
    dS_dm1 = (2 * m2 * A2 + A1 * (-2 * m2)) / BB - S * (2 * m1 / B1 + (-2 * m1) / B2)
    dS_dm11 = -S / B2
    dS_dm12 = 2 * A1 / BB
    # chain through the (self-adjoint) filter; D_SSIM = 1 - mean S
    ddssim = -(blur(dS_dm1) + 2 * x * blur(dS_dm11) + y * blur(dS_dm12)) / n
    total = (1 - lam) * l1 + beta * lg + lam * dssim
    dc = (1 - lam) * dl1 + beta * dlg + lam * ddssim
    return dict(loss=total, l1=l1, grad_l1=lg, dssim=dssim, dc=dc)


def adam(param, grad, m, v, t: int, lr, b1=0.9, b2=0.999, eps=1e-15, lo=None, hi=None):
    """One Adam update (Kingma and Ba, Alg. 1) at step t >= 1; returns the new
    (param, m, v).  lo/hi clamp the parameter after the update."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = param - lr * mh / (np.sqrt(vh) + eps)
    if lo is not None or hi is not None:
        p = np.clip(p, lo, hi)
    return p, m, v
