"""Differentiable rendering as a torch.autograd.Function.

render(params, cams, pose_xi, rasterizer) returns colour [V,3,H,W], depth
[V,H,W] (sum_j T_j alpha_j z_j, the appendix's depth volume rendering) and the
final transmittance T_final [V,H,W] (the opacity image is 1 - T_final); backward
gives gradients for the Gaussian
means, log-scales, quaternions, opacity logits, SH coefficients and the 6-DoF
pose tangent of every view.  Nothing per pixel is kept between the passes
but the final transmittance and the last blended position: the backward
recomputes every pixel's front-to-back sequence.  With recompute=True (the
default) the backward also re-runs projection and binning, so no (tile,
Gaussian) list survives the forward either; with recompute=False the lists
of the forward are reused when no other projection ran in between.
"""
from __future__ import annotations

from typing import Optional

import torch

from .rasterizer import GaussianParams, Image, Rasterizer
from .scenes import CAMERA_DTYPE


class KgsRasterFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, logits, sh, pose_xi, cams, rasterizer: Rasterizer, sh_degree: int,
                recompute: bool):
        R = rasterizer
        g = GaussianParams(means.detach().contiguous(), log_scales.detach().contiguous(),
                           quats.detach().contiguous(), logits.detach().contiguous(), sh.detach().contiguous(),
                           sh_degree)
        xi = pose_xi.detach().contiguous() if pose_xi is not None else None
        V = R.project(g, cams, xi)
        R.bin_sort()
        img = Image.empty(V, R.height, R.width, device=means.device)
        R.render_fwd(img)
        ctx.R = R
        ctx.g = g
        ctx.xi = xi
        ctx.cams = cams
        ctx.img = img
        ctx.generation = R.generation
        ctx.recompute = recompute
        ctx.has_pose = pose_xi is not None
        return img.color, img.depth, img.t_final

    @staticmethod
    def backward(ctx, g_color, g_depth, g_tfinal):
        R, g, xi, cams, img = ctx.R, ctx.g, ctx.xi, ctx.cams, ctx.img
        if ctx.recompute or R.generation != ctx.generation:
            R.project(g, cams, xi)
            R.bin_sort()
        V = cams.numel() // CAMERA_DTYPE.itemsize
        grads = g.zeros_like()
        pose_grad = torch.zeros(V, 6, device=g.means.device) if ctx.has_pose else None
        gc = g_color.contiguous() if g_color is not None else torch.zeros_like(img.color)
        gd = g_depth.contiguous() if g_depth is not None else None
        gt = g_tfinal.contiguous() if g_tfinal is not None else None
        R.render_bwd(g, cams, xi, img, gc, gd, grads=grads, pose_grad=pose_grad, dl_dtfinal=gt)
        return (grads.means, grads.log_scales, grads.quats, grads.logits, grads.sh, pose_grad, None, None, None, None)


def render(params: dict, cams: torch.Tensor, pose_xi: Optional[torch.Tensor], rasterizer: Rasterizer,
           sh_degree: int, recompute: bool = True):
    """params: means [3,N], log_scales [3,N], quats [4,N], logits [N], sh [K,3,N]
    (float32 CUDA tensors, may require grad); cams: device camera bytes;
    pose_xi: [V,6] tangent (may require grad) or None."""
    return KgsRasterFn.apply(params["means"], params["log_scales"], params["quats"], params["logits"],
                             params["sh"], pose_xi, cams, rasterizer, sh_degree, recompute)
