"""End-to-end oracle of the three steps of the method (Sec. 2.2 and Algorithm 1):
project the splats (Eq. 19), composite the projected gradient field front to
back (Eq. 20), and recover the image by solving the 2D Poisson equation
(Eq. 21) on the divergence of the composited gradients (Sec. 1.5 and Eq. 14),
with Dirichlet data on the image ring or with the paper's Neumann condition.

render_laplacian is the literal form of Sec. 2.2: the splats carry the
Laplacian of each colour channel, the composite of those three values is the
right-hand side of Eq. 21 itself (no divergence step).  Test oracle only."""
from __future__ import annotations

import numpy as np

from . import composite, poisson
from .project import project


def render(scene, cam, boundary=None, neumann: bool = False) -> dict:
    """Full-image FP64 render.  Returns proj, grad[6][H][W], rho[3][H][W] and
    u[3][H][W] (ring = boundary's ring, or zero).  neumann: no flux across the
    image border, every pixel unknown, zero-mean u (boundary must be None)."""
    proj = project(scene, cam)
    grad = composite.render_grad(proj, scene.opacity, scene.value, cam.H, cam.W)
    if neumann:
        assert boundary is None
        rho = poisson.divergence_neumann(grad)
        u = poisson.solve_neumann(rho)
    else:
        rho = poisson.divergence(grad)
        u = poisson.solve(rho, boundary)
    return dict(proj=proj, grad=grad, rho=rho, u=u)


def threshold(x: np.ndarray, t: float) -> np.ndarray:
    """Hard threshold of Sec. 3.1 (Eq. 24): x where |x| >= t, else 0."""
    x = np.asarray(x)
    return np.where(np.abs(x) >= t, x, np.zeros_like(x))


def render_laplacian(scene, cam, boundary=None, t: float = 0.0, neumann: bool = False) -> dict:
    """Laplacian splats (scene.value is [3][K]): proj, rho[3][H][W] (the
    composite, hard-thresholded at t when t > 0) and u[3][H][W] with
    L u = rho on the interior, u = boundary (or zero) on the ring; neumann:
    L u = rho - mean(rho) on every pixel with no flux across the border and
    zero-mean u (boundary must be None)."""
    proj = project(scene, cam)
    rho = composite.render_grad(proj, scene.opacity, scene.value, cam.H, cam.W)
    if t > 0.0:
        rho = threshold(rho, t)
    if neumann:
        assert boundary is None
        u = poisson.solve_neumann(rho)
    else:
        u = poisson.solve(rho, boundary)
    return dict(proj=proj, rho=rho, u=u)

