"""Differentiable render + Poisson reconstruction (torch.autograd.Function).

Inputs are rasteriser-level splats: image-plane means, conics (a, b, c) with
E = a dx^2 + 2 b dx dy + c dy^2, opacities, six gradient values, and depths
(which only fix the compositing order, so they get no gradient).

Backward, for an incoming dL/du (the particle-parameter gradients of GDGS
Sec. 1.1, Eq. 5-7, through the Poisson reconstruction of Eq. 21):
  1. adjoint solve: L lam = dL/du on the interior with a zero ring (the
     interior Laplacian is symmetric, so this is the same multigrid solve with
     another right-hand side) -- gdgs_poisson_solve_rhs;
  2. divergence adjoint: dL/dgrad = D^T lam -- gdgs_div_adjoint;
  3. reverse compositing with transmittance recomputed per pixel --
     gdgs_raster_grad_backward;
  4. (render3d only) reverse projection to the world means, log-scales and
     quaternions -- gdgs_project_backward.
Every step runs in libgdgs; this module only sequences the calls.
"""
from __future__ import annotations

import torch

from . import api as A


def _forward_mg(mg, boundary):
    mg = mg if mg is not None else A.mg_params()
    if (mg.flags & A.NEUMANN) and boundary is not None:
        raise ValueError("the Neumann problem takes no boundary data")
    return mg


def _adjoint(ctx, du, W, H):
    """dl/dgrad from dl/du.  Dirichlet: the same solve with a zero ring on the
    interior of du (u's ring is data), then the transpose of the interior
    divergence.  Neumann: u = L+ rho with L+ the symmetric pseudo-inverse, so
    dl/drho = L+ du, the same Neumann solve on every pixel of du, then the
    transpose of the Neumann divergence.  The adjoint solve starts from zero
    (warm-start and resume flags are not carried over)."""
    m = ctx.mg
    nm = bool(m.flags & A.NEUMANN)
    mg = A.mg_params(m.levels, m.pre_sweeps, m.post_sweeps, m.max_cycles, m.tol,
                     m.coarse_sweeps, m.flags & (A.NEUMANN | A.FMG), m.smooth_weight)
    lam, _ = A.gdgs_poisson_solve_rhs(du, None, W, H, mg)
    return A.gdgs_div_adjoint(lam, W, H, neumann=nm)


class GDGSRenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean2d, conic, opacity, value, depth, W: int, H: int, boundary=None,
                mg=None, capacity: int | None = None):
        K = int(depth.shape[0])
        mean2d = mean2d.detach().contiguous()
        conic = conic.detach().contiguous()
        opacity = opacity.detach().contiguous()
        value = value.detach().contiguous()
        depth = depth.detach().contiguous()
        mg = _forward_mg(mg, boundary)
        proj = A.gdgs_project_2d(mean2d, conic, depth, W, H)
        cap = int(capacity if capacity is not None else max(1 << 16, 16 * K))
        bins = A.gdgs_bin_sort(proj, K, W, H, cap)
        P = int(bins["num_pairs"].item())
        if P > cap:
            cap = int(P * 1.25) + 1024
            bins = A.gdgs_bin_sort(proj, K, W, H, cap)
        grad = A.gdgs_raster_grad(proj, opacity, value, K, bins, W, H)
        u, stats = A.gdgs_poisson_solve(grad, boundary, W, H, mg)
        ctx.save_for_backward(opacity, value, grad)
        ctx.proj, ctx.bins, ctx.W, ctx.H, ctx.K, ctx.mg = proj, bins, W, H, K, mg
        ctx.stats = stats
        return u

    @staticmethod
    def backward(ctx, du):
        opacity, value, grad = ctx.saved_tensors
        W, H, K = ctx.W, ctx.H, ctx.K
        du = du.contiguous().to(torch.float32)
        dgrad = _adjoint(ctx, du, W, H)
        g = A.gdgs_raster_grad_backward(ctx.proj, opacity, value, K, ctx.bins, W, H, grad, dgrad)
        return g["mean2d"], g["conic"], g["opacity"], g["value"], None, None, None, None, None, None


def render(mean2d, conic, opacity, value, depth, W: int, H: int, boundary=None, mg=None,
           capacity: int | None = None):
    """u[3][H][W] recovered from rasteriser-level gradient splats; differentiable
    in mean2d, conic, opacity and value."""
    return GDGSRenderFn.apply(mean2d, conic, opacity, value, depth, W, H, boundary, mg, capacity)


class GDGSRender3DFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity, value, cam, W: int, H: int, boundary=None,
                mg=None, capacity: int | None = None):
        ds = A.DeviceScene(mean.detach().contiguous(), log_scale.detach().contiguous(),
                           quat.detach().contiguous(), opacity.detach().contiguous(),
                           value.detach().contiguous())
        K = ds.K
        mg = _forward_mg(mg, boundary)
        proj = A.gdgs_project(ds, cam)
        cap = int(capacity if capacity is not None else max(1 << 16, 16 * K))
        bins = A.gdgs_bin_sort(proj, K, W, H, cap)
        P = int(bins["num_pairs"].item())
        if P > cap:
            cap = int(P * 1.25) + 1024
            bins = A.gdgs_bin_sort(proj, K, W, H, cap)
        grad = A.gdgs_raster_grad(proj, ds.opacity, ds.value, K, bins, W, H)
        u, stats = A.gdgs_poisson_solve(grad, boundary, W, H, mg)
        ctx.ds, ctx.cam, ctx.proj, ctx.bins, ctx.grad = ds, cam, proj, bins, grad
        ctx.W, ctx.H, ctx.K, ctx.mg, ctx.stats = W, H, K, mg, stats
        return u

    @staticmethod
    def backward(ctx, du):
        ds, W, H, K = ctx.ds, ctx.W, ctx.H, ctx.K
        du = du.contiguous().to(torch.float32)
        dgrad = _adjoint(ctx, du, W, H)
        g = A.gdgs_raster_grad_backward(ctx.proj, ds.opacity, ds.value, K, ctx.bins, W, H,
                                        ctx.grad, dgrad)
        g3 = A.gdgs_project_backward(ds, ctx.cam, g["mean2d"], g["conic"])
        return (g3["mean"], g3["log_scale"], g3["quat"], g["opacity"], g["value"], None, None,
                None, None, None, None)


def render3d(mean, log_scale, quat, opacity, value, cam, boundary=None, mg=None,
             capacity: int | None = None):
    """u[3][H][W] of a view of 3D gradient splats; differentiable in the world
    means, log-scales, quaternions, opacities and gradient values."""
    return GDGSRender3DFn.apply(mean, log_scale, quat, opacity, value, cam, int(cam.W),
                                int(cam.H), boundary, mg, capacity)

