"""The mapping loss of the sliding-window optimisation in plain PyTorch FP64.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Sec. 3.2 (Eq. "mapping loss": L_total = L_photo + lambda_g L_geo +
lambda_iso L_iso) and the appendix section "Rendering Objectives":

    L_photo = 0.8 ||I - I^||_1 + 0.2 (1 - SSIM(I, I^))
    L_geo   = ||D - D^||_1
    L_iso   = sum_i ||s_i - s~_i 1||_1,   s~_i the mean of the scale vector s_i

with lambda_g = 0.01 and lambda_iso = 10 (hyper-parameter table).

Readings where the paper is silent:
  * ||.||_1 of an image is the mean absolute difference over its pixels (and its
    three channels), per view; so is L_geo.  The chunk's loss is the sum over
    its views, and L_photo of a view is the per-view loss the pruning score's
    gamma_v uses (appendix, "Pruning Score").
  * SSIM is the structural similarity of Wang et al. (2004) with an 11x11
    Gaussian window of standard deviation 1.5 (sampled, normalised to sum 1),
    C1 = (0.01)^2 and C2 = (0.03)^2 for images in [0, 1], each channel on its
    own, zero padding outside the image, averaged over pixels and channels.
  * s_i = exp(log-scales): the regulariser acts on the scales the rasterizer
    uses, and its gradient reaches the log-scales through s = exp(log s).
  * |x| has derivative sign(x), 0 at 0.
Gradients are those of these definitions, taken by autograd in FP64.
"""
from __future__ import annotations


import numpy as np
import torch

W_L1, W_SSIM = 0.8, 0.2
LAMBDA_G, LAMBDA_ISO = 0.01, 10.0
WINDOW, SIGMA = 11, 1.5
C1, C2 = 0.01 ** 2, 0.03 ** 2


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """The sampled, normalised 1D Gaussian; the 2D window is its outer product."""
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2
    w = np.exp(-x * x / (2 * sigma * sigma))
    return w / w.sum()


def _blur(x: torch.Tensor) -> torch.Tensor:
    """x [C, H, W] -> 2D Gaussian-window filter of each channel, zero padding."""
    w1 = torch.tensor(gaussian_window(), dtype=torch.float64)
    w2 = torch.outer(w1, w1)[None, None].expand(x.shape[0], 1, WINDOW, WINDOW)
    return torch.nn.functional.conv2d(x[None], w2, padding=WINDOW // 2, groups=x.shape[0])[0]


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Per-pixel, per-channel SSIM of x and y [C, H, W] (FP64)."""
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def photo_loss(rendered: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """L_photo of one view: 0.8 mean |I - I^| + 0.2 (1 - mean SSIM)."""
    return W_L1 * (rendered - target).abs().mean() + W_SSIM * (1.0 - ssim_map(rendered, target).mean())


def geo_loss(rendered_depth: torch.Tensor, depth: torch.Tensor) -> torch.Tensor:
    """L_geo of one view: mean |D - D^|."""
    return (rendered_depth - depth).abs().mean()


def iso_loss(log_scales: torch.Tensor) -> torch.Tensor:
    """L_iso = sum_i sum_k |s_ik - mean_k s_ik| over Gaussians i, s = exp(log s); log_scales [3, N]."""
    s = torch.exp(log_scales)
    return (s - s.mean(dim=0, keepdim=True)).abs().sum()


def ssim_gradient_term_scale(color, target) -> np.ndarray:
    """Diagnostic for comparisons in another arithmetic (not part of the loss):
    dL/dC of the D-SSIM term is the sum of three parts -- through the local
    mean, through the local second moment and through the local cross moment
    of C -- which cancel almost exactly where the image is flat.  Returns, per
    element of color [V, 3, H, W], w_ssim / (3 H W) times the sum of the three
    parts' magnitudes, each part taken by autograd through its own copy of C."""
    col = np.asarray(color, np.float64)
    tgt = np.asarray(target, np.float64)
    V, _, H, W = col.shape
    out = np.zeros_like(col)
    for v in range(V):
        xa, xb, xc = (torch.tensor(col[v], requires_grad=True) for _ in range(3))
        y = torch.tensor(tgt[v])
        mx, my = _blur(xa), _blur(y)
        sxx = _blur(xb * xb) - mx * mx
        syy = _blur(y * y) - my * my
        sxy = _blur(xc * y) - mx * my
        s = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
        s.sum().backward()
        out[v] = (xa.grad.abs() + xb.grad.abs() + xc.grad.abs()).numpy() * W_SSIM / (3 * H * W)
    return out


def mapping_loss(color, target, depth=None, target_depth=None, log_scales=None, lambda_g=LAMBDA_G,
                 lambda_iso=LAMBDA_ISO) -> dict:
    """color, target: [V, 3, H, W]; depth, target_depth: [V, H, W] or None; log_scales [3, N] or None
    (NumPy or torch, any float type; computed in FP64).  Returns the per-view photometric and geometric
    losses, the isotropy term, the total L = sum_v (L_photo,v + lambda_g L_geo,v) + lambda_iso L_iso, and
    dL/dcolor, dL/ddepth, dL/dlog_scales."""
    c = torch.tensor(np.asarray(color, np.float64), requires_grad=True)
    t = torch.tensor(np.asarray(target, np.float64))
    V = c.shape[0]
    photo = torch.stack([photo_loss(c[v], t[v]) for v in range(V)])
    total = photo.sum()
    d = geo = None
    if depth is not None:
        d = torch.tensor(np.asarray(depth, np.float64), requires_grad=True)
        td = torch.tensor(np.asarray(target_depth, np.float64))
        geo = torch.stack([geo_loss(d[v], td[v]) for v in range(V)])
        total = total + lambda_g * geo.sum()
    ls = iso = None
    if log_scales is not None:
        ls = torch.tensor(np.asarray(log_scales, np.float64), requires_grad=True)
        iso = iso_loss(ls)
        total = total + lambda_iso * iso
    total.backward()
    return dict(photo=photo.detach().numpy(), geo=None if geo is None else geo.detach().numpy(),
                iso=None if iso is None else float(iso.detach()), total=float(total.detach()),
                dl_dcolor=c.grad.numpy(), dl_ddepth=None if d is None else d.grad.numpy(),
                dl_dlog_scales=None if ls is None else ls.grad.numpy())
