"""One optimisation iteration of Algorithm 1 (GDGS Sec. 2.2-2.3) for a scene of
3D gradient splats against observed images: render the view (projection,
compositing, Poisson), evaluate the loss of Eq. 22, back-propagate to the
world means, log-scales, quaternions, opacities and gradient values, and
update them with Adam.  Every step runs in libgdgs (the loss and the update
included); this module sequences the calls.

Readings where the paper is silent: Adam (beta1 0.9, beta2 0.999, eps 1e-15)
with per-group learning rates after the 3D Gaussian Splatting defaults the
paper builds on (means 3e-4, log-scales 5e-3, quaternions 1e-3, opacities
1e-2 on the opacity itself, clamped to [1e-4, 1 - 1e-4], values 2.5e-3);
lam = 0.2, beta = 0.1 in the loss.
"""
from __future__ import annotations

import torch

from . import api as A
from .autograd import render3d

LRS = {"mean": 3e-4, "log_scale": 5e-3, "quat": 1e-3, "opacity": 1e-2, "value": 2.5e-3}
GROUPS = ("mean", "log_scale", "quat", "opacity", "value")


class ImageLossFn(torch.autograd.Function):
    """Eq. 22 as a differentiable scalar (value and dL/dc from one library call)."""

    @staticmethod
    def forward(ctx, c, im, lam: float, beta: float):
        out, dc = A.gdgs_image_loss(c.detach().contiguous(), im.contiguous(), lam, beta)
        ctx.save_for_backward(dc)
        ctx.terms = out
        return out[0].to(torch.float32)

    @staticmethod
    def backward(ctx, g):
        (dc,) = ctx.saved_tensors
        return dc * g, None, None, None


class Trainer:
    """Parameters (device tensors, updated in place) and Adam moments."""

    def __init__(self, scene: A.DeviceScene, mg=None, lam: float = 0.2, beta: float = 0.1,
                 lrs: dict | None = None):
        self.p = {g: getattr(scene, g).detach().clone().contiguous() for g in GROUPS}
        self.m = {g: torch.zeros_like(t) for g, t in self.p.items()}
        self.v = {g: torch.zeros_like(t) for g, t in self.p.items()}
        self.t = 0
        self.mg = mg if mg is not None else A.mg_params()
        self.lam, self.beta = lam, beta
        self.lrs = dict(LRS, **(lrs or {}))

    def scene(self) -> A.DeviceScene:
        return A.DeviceScene(*(self.p[g] for g in GROUPS))

    def step(self, cam, target: torch.Tensor, boundary=None) -> dict:
        """One iteration on one view; returns the loss terms before the update
        and the gradients used."""
        leaves = [self.p[g].clone().requires_grad_(True) for g in GROUPS]
        u = render3d(*leaves, cam, boundary=boundary, mg=self.mg)
        loss = ImageLossFn.apply(u, target, self.lam, self.beta)
        t = loss.grad_fn.terms.cpu().tolist()   # the loss node keeps the four terms
        terms = dict(loss=t[0], l1=t[1], grad_l1=t[2], dssim=t[3])
        loss.backward()
        self.t += 1
        grads = {}
        for g, leaf in zip(GROUPS, leaves):
            lo, hi = (1e-4, 1.0 - 1e-4) if g == "opacity" else (0.0, 0.0)
            grads[g] = leaf.grad.contiguous()
            A.gdgs_adam_step(self.p[g], grads[g], self.m[g], self.v[g], self.t, self.lrs[g],
                             lo=lo, hi=hi)
        return dict(terms, u=u.detach(), grads=grads)
