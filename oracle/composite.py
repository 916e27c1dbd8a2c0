"""Front-to-back alpha compositing of the projected gradient field (test oracle).

Follows the alpha blend of Sec. 1.2 (Eq. 11) as the method reuses it for the
projected field in Sec. 2.2 "Projection" (Eq. 20): at image point p,

    out_m(p) = sum_k v_{k,m} a_k(p) T_{k-1}(p),  a_k = alpha_k G_k(p),
    T_0 = 1,  T_k = T_{k-1} (1 - a_k),

with G_k(p) = exp(-(p - mu_k)^T conic_k (p - mu_k)) (no factor 1/2, as in
Eq. 9 and Eq. 18) and k ordered front to back along the view direction.

Here each splat carries the six image-gradient values v_{k, 2c+d} (colour c,
direction d), the gradient form of the method (Sec. 1.6 and the loss of
Eq. 13), so the composite is the six-channel gradient image.

Readings where the paper is silent:
* G_k = 0 where the exponent exceeds E_CUT (support cut-off);
* order key: the camera depth rounded to FP32 (the precision the rasteriser
  sorts in), ties broken by the lower splat index;
* no opacity clamp, no minimum-alpha skip, no early termination.

Every pixel is computed by brute force over all splats; the per-splat pixel
box is an exact prefilter (outside it E > E_CUT, so the term is zero).
"""
from __future__ import annotations

import numpy as np

from .constants import E_CUT


def pixel_terms(row: int, col: int, proj: dict, opacity, use_box: bool = True):
    """Splats contributing at pixel (row, col), in compositing order.

    Returns (idx, G, dx, dy): splat indices sorted front to back, their
    Gaussian values and the offsets d = p - mu of the pixel centre.
    """
    px, py = col + 0.5, row + 0.5
    cand = proj["valid"].copy()
    if use_box:
        j0, j1, i0, i1 = proj["box"]
        cand &= (j0 <= col) & (col <= j1) & (i0 <= row) & (row <= i1)
    idx = np.nonzero(cand)[0]
    mx, my = proj["mean2d"][0][idx], proj["mean2d"][1][idx]
    a, b, c = (proj["conic"][r][idx] for r in range(3))
    dx, dy = px - mx, py - my
    E = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
    keep = E <= E_CUT
    idx, E, dx, dy = idx[keep], E[keep], dx[keep], dy[keep]
    depth32 = proj["depth"][idx].astype(np.float32)
    order = np.lexsort((idx, depth32))
    return idx[order], np.exp(-E[order]), dx[order], dy[order]


def composite_pixel(row: int, col: int, proj: dict, opacity, value,
                    use_box: bool = True) -> np.ndarray:
    """The six composited channels at one pixel (FP64)."""
    idx, G, _, _ = pixel_terms(row, col, proj, opacity, use_box)
    if idx.size == 0:
        return np.zeros(np.asarray(value).shape[0])
    a = np.asarray(opacity, dtype=np.float64)[idx] * G
    T_prev = np.concatenate([[1.0], np.cumprod(1.0 - a)[:-1]])
    v = np.asarray(value, dtype=np.float64)[:, idx]
    return (v * (a * T_prev)[None, :]).sum(axis=1)


def transmittance(row: int, col: int, proj: dict, opacity, use_box: bool = True) -> float:
    """T after every contributing splat at the pixel: prod_k (1 - a_k)."""
    idx, G, _, _ = pixel_terms(row, col, proj, opacity, use_box)
    a = np.asarray(opacity, dtype=np.float64)[idx] * G
    return float(np.prod(1.0 - a))


def render_grad(proj: dict, opacity, value, H: int, W: int,
                rows=None, cols=None, use_box: bool = True) -> np.ndarray:
    """Six-channel gradient image.  With rows/cols given, only those pixels
    are computed and an array [6][n] is returned; otherwise [6][H][W]."""
    nch = np.asarray(value).shape[0]
    if rows is None:
        out = np.zeros((nch, H, W))
        for i in range(H):
            for j in range(W):
                out[:, i, j] = composite_pixel(i, j, proj, opacity, value, use_box)
        return out
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    out = np.zeros((nch, rows.size))
    for n, (i, j) in enumerate(zip(rows.tolist(), cols.tolist())):
        out[:, n] = composite_pixel(i, j, proj, opacity, value, use_box)
    return out
