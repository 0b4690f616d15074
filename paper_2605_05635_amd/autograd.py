"""torch.autograd binding of the image and its gradient.

    I = traced_image(q, img)                # q: float64 tensor [4]
    loss = ((I - target) ** 2).sum()
    loss.backward()                         # q.grad = dL/dq via rt_image_vjp

q holds the four differentiable image parameters, in the basis "native"
(spin, incl, halo0, halo1) or, for the cored-NFW halo, "density"
(spin, incl, rho_s, r_s) with eta = 4 pi rho_s r_s^2 and lambda_c = r_s.
The forward pass is rt_trace_image, the backward pass rt_image_vjp: the
derivative of the traced discrete map with its step sizes and decisions held
fixed (both run in the gfx950 kernels; nothing here computes).
"""
from __future__ import annotations

import math

import torch

from . import rt


def image_params(q, img: dict, basis: str = "native") -> dict:
    """The workload dict `img` with its parameters replaced by q's values."""
    v = [float(x) for x in q.detach().cpu().tolist()]
    d = dict(img, spin=v[0], incl=v[1])
    if basis == "density":
        d["halo"] = (4.0 * math.pi * v[2] * v[3] ** 2, v[3])
    else:
        d["halo"] = (v[2], v[3])
    return d


class TraceImage(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, img, basis, device):
        d = image_params(q, img, basis)
        I = rt.trace(d, device=device)["intensity"]
        ctx.img, ctx.basis, ctx.q_device = d, basis, q.device
        return I

    @staticmethod
    def backward(ctx, gI):
        g = rt.image_vjp(ctx.img, gI.to(torch.float64).contiguous(), ctx.basis)
        return g.to(ctx.q_device), None, None, None


def traced_image(q, img: dict, basis: str = "native", device="cuda"):
    """Thin-disc image [ny][nx] of `img` at parameters q, differentiable in q."""
    if basis not in ("native", "density"):
        raise ValueError("basis must be 'native' or 'density'")
    return TraceImage.apply(q, img, basis, device)
