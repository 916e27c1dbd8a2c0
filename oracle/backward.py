"""Exact gradients through composite -> divergence -> Poisson, FP64 (test oracle).

Sec. 1.1 of GDGS writes the particle-parameter gradients of a squared-error
loss as the loss residual times the derivative of the kernel sum (Eq. 5-7).
For this pipeline the loss is l = 1/2 sum_c sum_interior (u - u_target)^2 on
the recovered image u and the parameters are the rasteriser inputs: image
mean mu[2][K], conic (a, b, c)[3][K], opacity alpha[K] and gradient values
v[6][K].  The chain is:

* Poisson (Eq. 21) with a zero ring: u_int = -A^{-1} rho_int with
  A = -L_int symmetric, so dl/drho = lam where L_int lam = (u - u_target)
  (the same Poisson problem with a different right-hand side; A's symmetry
  is the variational form of Sec. 3.2.4, Eq. 26);
* divergence: dl/dgrad = D^T lam (``poisson.div_adjoint``);
* compositing (Eq. 11 / Eq. 20): with w_k = a_k T_{k-1} and
  S_k = sum_{j>k} v_j w_j,  d out / d v_k = w_k and
  d out / d a_k = v_k T_{k-1} - S_k / (1 - a_k);
  a_k = alpha_k G_k, G_k = exp(-E_k), E_k = a dx^2 + 2 b dx dy + c dy^2,
  d = p - mu.

``finite_difference`` gives central differences of the same loss for the
self-check of these formulas.

neumann=True takes the paper's Neumann condition instead (every pixel an
unknown, no flux across the border, zero-mean u): the loss is over every
pixel, u = L+ rho with L+ the pseudo-inverse of the singular, symmetric
Neumann Laplacian, so dl/drho = L+ (u - u_target) (the same Neumann solve),
and the divergence adjoint is that of ``poisson.divergence_neumann``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import composite, poisson
from .constants import E_CUT
from .project import project_2d


class _Solver:
    """Zero-ring Poisson solver with the LU factors kept (tiny grids) or the
    DST-I path (larger grids)."""

    def __init__(self, H: int, W: int):
        self.H, self.W = H, W
        n, m = H - 2, W - 2
        self.lu = scipy.linalg.lu_factor(poisson.system_matrix(n, m)) if n * m <= 4096 else None

    def __call__(self, rho: np.ndarray) -> np.ndarray:
        if self.lu is None:
            return poisson.solve_dst(rho, None)
        C = rho.shape[0]
        n, m = self.H - 2, self.W - 2
        u = np.zeros(rho.shape)
        b = poisson.rhs(rho, None)
        for c in range(C):
            u[c, 1:-1, 1:-1] = scipy.linalg.lu_solve(self.lu, b[c].ravel()).reshape(n, m)
        return u


def forward(params: dict, H: int, W: int, target: np.ndarray, solver=None,
            neumann: bool = False):
    """Loss and intermediates for rasteriser-level params (FP64 copies)."""
    proj = project_2d(params["mean2d"], params["conic"], params["depth"], W, H)
    grad = composite.render_grad(proj, params["opacity"], params["value"], H, W)
    if neumann:
        rho = poisson.divergence_neumann(grad)
        u = poisson.solve_neumann(rho)
        e = u - np.asarray(target, dtype=np.float64)
        loss = 0.5 * float((e * e).sum())
        return dict(loss=loss, grad=grad, rho=rho, u=u, e=e, proj=proj)
    rho = poisson.divergence(grad)
    solver = solver or _Solver(H, W)
    u = solver(rho)
    e = np.zeros(u.shape)
    e[:, 1:-1, 1:-1] = u[:, 1:-1, 1:-1] - np.asarray(target, dtype=np.float64)[:, 1:-1, 1:-1]
    loss = 0.5 * float((e * e).sum())
    return dict(loss=loss, grad=grad, rho=rho, u=u, e=e, proj=proj)


def gradients(params: dict, H: int, W: int, target: np.ndarray, neumann: bool = False):
    """Loss and exact dl/d(mean2d, conic, opacity, value) (FP64)."""
    solver = None if neumann else _Solver(H, W)
    fw = forward(params, H, W, target, solver, neumann)
    return gradients_from_du(params, H, W, fw["e"], fw, solver, neumann)


def gradients_from_du(params: dict, H: int, W: int, du: np.ndarray, fw=None, solver=None,
                      neumann: bool = False):
    """dl/d(mean2d, conic, opacity, value) for any loss whose gradient with
    respect to u is du[3][H][W] (Dirichlet: its ring is not used, u's ring is
    data; Neumann: every pixel is used)."""
    if fw is None:
        fw = forward(params, H, W, np.zeros((3, H, W)), solver, neumann)
    if neumann:
        lam = poisson.solve_neumann(np.asarray(du, dtype=np.float64))   # L+ du
        dgrad = poisson.div_adjoint_neumann(lam)
    else:
        solver = solver or _Solver(H, W)
        e = np.zeros((3, H, W))
        e[:, 1:-1, 1:-1] = np.asarray(du, dtype=np.float64)[:, 1:-1, 1:-1]
        lam = solver(e)                   # L_int lam = e, zero ring
        dgrad = poisson.div_adjoint(lam)
    proj = fw["proj"]
    K = np.asarray(params["opacity"]).shape[0]
    alpha = np.asarray(params["opacity"], dtype=np.float64)
    value = np.asarray(params["value"], dtype=np.float64)
    conic = proj["conic"]
    dmean = np.zeros((2, K))
    dconic = np.zeros((3, K))
    dalpha = np.zeros(K)
    dvalue = np.zeros((6, K))
    for i in range(H):
        for j in range(W):
            idx, G, dx, dy = composite.pixel_terms(i, j, proj, alpha, use_box=False)
            if idx.size == 0:
                continue
            delta = dgrad[:, i, j]
            a = alpha[idx] * G
            T_prev = np.concatenate([[1.0], np.cumprod(1.0 - a)[:-1]])
            w = a * T_prev
            v = value[:, idx]
            contrib = v * w[None, :]
            S = np.cumsum(contrib[:, ::-1], axis=1)[:, ::-1] - contrib   # sum over j > k
            dvalue[:, idx] += delta[:, None] * w[None, :]
            dl_da = (delta[:, None] * (v * T_prev[None, :] - S / (1.0 - a)[None, :])).sum(axis=0)
            dalpha[idx] += dl_da * G
            dl_dE = -dl_da * alpha[idx] * G
            ca, cb, cc = conic[0][idx], conic[1][idx], conic[2][idx]
            dmean[0, idx] += dl_dE * (-2.0 * (ca * dx + cb * dy))
            dmean[1, idx] += dl_dE * (-2.0 * (cb * dx + cc * dy))
            dconic[0, idx] += dl_dE * dx * dx
            dconic[1, idx] += dl_dE * 2.0 * dx * dy
            dconic[2, idx] += dl_dE * dy * dy
    return dict(loss=fw["loss"], mean2d=dmean, conic=dconic, opacity=dalpha, value=dvalue,
                lam=lam, dgrad=dgrad, u=fw["u"], grad=fw["grad"])


def splat_gradients(params: dict, H: int, W: int, dgrad: np.ndarray, splats) -> dict:
    """dl/d(mean2d, conic, opacity, value) of the listed splats only, for a
    given dl/dgrad[6][H][W] (the reverse compositing step of
    ``gradients_from_du`` restricted to a subset of splats).

    A splat contributes only at pixels of its support box, so its sums run
    over that box; at each such pixel the whole front-to-back list is formed
    from the splats whose boxes meet the box (every other splat is zero
    there), and the splat's own terms are taken from it.  Meant for images
    too large to composite every pixel.  Returns arrays [.., len(splats)]."""
    splats = np.asarray(splats, dtype=np.int64)
    proj = project_2d(params["mean2d"], params["conic"], params["depth"], W, H)
    alpha = np.asarray(params["opacity"], dtype=np.float64)
    value = np.asarray(params["value"], dtype=np.float64)
    dgrad = np.asarray(dgrad, dtype=np.float64)
    j0, j1, i0, i1 = proj["box"]
    valid = proj["valid"]
    n = splats.size
    out = dict(mean2d=np.zeros((2, n)), conic=np.zeros((3, n)), opacity=np.zeros(n),
               value=np.zeros((6, n)))
    for s_, k in enumerate(splats.tolist()):
        if not valid[k] or j0[k] > j1[k] or i0[k] > i1[k]:
            continue
        near = np.nonzero(valid & (j0 <= j1[k]) & (j1 >= j0[k]) & (i0 <= i1[k]) &
                          (i1 >= i0[k]))[0]            # ascending: index order kept
        sub = dict(valid=valid[near], box=tuple(b[near] for b in proj["box"]),
                   mean2d=proj["mean2d"][:, near], conic=proj["conic"][:, near],
                   depth=proj["depth"][near])
        me = int(np.searchsorted(near, k))
        al, va = alpha[near], value[:, near]
        ca, cb, cc = (proj["conic"][r][k] for r in range(3))
        for i in range(int(i0[k]), int(i1[k]) + 1):
            for j in range(int(j0[k]), int(j1[k]) + 1):
                idx, G, dx, dy = composite.pixel_terms(i, j, sub, al, use_box=True)
                pos = np.nonzero(idx == me)[0]
                if pos.size == 0:
                    continue
                q = int(pos[0])
                delta = dgrad[:, i, j]
                a = al[idx] * G
                T_prev = np.concatenate([[1.0], np.cumprod(1.0 - a)[:-1]])
                w = a * T_prev
                contrib = va[:, idx] * w[None, :]
                S_q = contrib[:, q + 1:].sum(axis=1)          # sum over the splats behind
                out["value"][:, s_] += delta * w[q]
                dl_da = float((delta * (value[:, k] * T_prev[q] - S_q / (1.0 - a[q]))).sum())
                out["opacity"][s_] += dl_da * G[q]
                dl_dE = -dl_da * alpha[k] * G[q]
                ex, ey = dx[q], dy[q]
                out["mean2d"][0, s_] += dl_dE * (-2.0 * (ca * ex + cb * ey))
                out["mean2d"][1, s_] += dl_dE * (-2.0 * (cb * ex + cc * ey))
                out["conic"][0, s_] += dl_dE * ex * ex
                out["conic"][1, s_] += dl_dE * 2.0 * ex * ey
                out["conic"][2, s_] += dl_dE * ey * ey
    return out


def support_signature(params: dict, H: int, W: int) -> int:
    """Number of (pixel, splat) pairs inside the support cut-off; a finite
    difference whose two sides differ in this count crossed the cut-off."""
    mx, my = (np.asarray(params["mean2d"], dtype=np.float64)[r][None, :] for r in range(2))
    a, b, c = (np.asarray(params["conic"], dtype=np.float64)[r][None, :] for r in range(3))
    py, px = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    dx = px.reshape(-1, 1) - mx
    dy = py.reshape(-1, 1) - my
    E = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
    return int(((E <= E_CUT) & (a * c - b * b > 0)).sum())


def finite_difference(params: dict, H: int, W: int, target: np.ndarray, name: str,
                      index: tuple, rel_step: float = 1e-6, neumann: bool = False):
    """Central difference of the loss in one parameter entry.  Returns
    (derivative, crossed) where crossed says the support set changed."""
    solver = None if neumann else _Solver(H, W)
    base = {k: np.array(v, dtype=np.float64) for k, v in params.items()}
    x0 = base[name][index]
    h = rel_step * max(1.0, abs(x0))
    plus = {k: v.copy() for k, v in base.items()}
    minus = {k: v.copy() for k, v in base.items()}
    plus[name][index] = x0 + h
    minus[name][index] = x0 - h
    lp = forward(plus, H, W, target, solver, neumann)["loss"]
    lm = forward(minus, H, W, target, solver, neumann)["loss"]
    crossed = support_signature(plus, H, W) != support_signature(minus, H, W)
    return (lp - lm) / (2.0 * h), crossed


__all__ = ["forward", "gradients", "gradients_from_du", "splat_gradients",
           "finite_difference", "support_signature", "E_CUT"]
