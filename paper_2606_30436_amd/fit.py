"""Equal-PSNR check of the batched chunk against the plain per-view loop.

Both runs start from the same perturbed map (means moved by 5 cm, colours by
0.05) and take the same number of Adam steps on every Gaussian parameter, the
gradient of each step being the chunk's L1 loss over its keyframes: once from
the chunk captured as one HIP graph, once from the library called view by view
(the plain loop).  The two gradients agree to rounding (they sum the same terms
in another order), so the fits should end at the same PSNR against the
renders of the noise-free map.  Every step runs in the library: the chunk or
the per-view calls, then kgs_adam per parameter tensor."""
from __future__ import annotations

import math
import time

import torch

from . import _lib as L
from .rasterizer import GaussianParams, Image, Rasterizer, ViewStats, device_cameras

# learning rates per parameter tensor (the paper states none): position steps of ~1 mm, the 3DGS-style
# rates for colour, opacity, scale and rotation
LR = dict(means=1e-3, log_scales=5e-3, quats=1e-3, logits=5e-2, sh=2.5e-3)
PARAMS = ("means", "log_scales", "quats", "logits", "sh")


def psnr(color: torch.Tensor, target: torch.Tensor) -> float:
    mse = float(((color.clamp(0, 1) - target.clamp(0, 1)) ** 2).mean().item())
    return 10 * math.log10(1.0 / mse) if mse > 0 else float("inf")


def fit(sc, target: torch.Tensor, mode: str, iters: int = 200, tile=(32, 16), batch: int = 64, far_z: float = 80.0,
        slot_capacity: int = 0, pair_capacity: int = 0) -> dict:
    """mode 'batched' (one graph launch per step) or 'plain' (per-view calls).  Returns the final PSNR, the
    PSNR before the first step, the chunk's L1 loss at the last step (the objective, summed over the views)
    and the time per step (gradient plus Adam)."""
    V, H, W = sc.n_views, sc.height, sc.width
    dev = target.device
    g = GaussianParams.from_scene(sc)
    cams = device_cameras(sc.cams)
    grads = g.zeros_like()
    m = {k: torch.zeros_like(getattr(g, k)) for k in PARAMS}
    v2 = {k: torch.zeros_like(getattr(g, k)) for k in PARAMS}
    img = Image.empty(V, H, W)
    dl = torch.empty_like(img.color)
    loss = torch.empty(V, device=dev)
    pose = torch.zeros(V, 6, device=dev)
    stats = ViewStats.zeros(sc.n)
    if mode == "batched":
        R = Rasterizer(W, H, V, sc.n, slot_capacity=slot_capacity, pair_capacity=pair_capacity, tile=tile,
                       batch=batch, far_z=far_z)
        desc = R.chunk_desc(g, cams, None, target, img, dl, loss, grads, pose, stats, tau_err=0.1,
                            zero_accumulators=True)
        graph = R.chunk_capture(desc)
        step_fn = lambda: R.chunk_launch(graph)
    else:
        # the same tiling as the batched run, so that the two differ only in batching
        R = Rasterizer(W, H, 1, sc.n, slot_capacity=slot_capacity, pair_capacity=pair_capacity, tile=tile,
                       batch=batch, far_z=far_z)
        cam_rows = cams.view(V, -1)

        def step_fn():
            for t in (grads.means, grads.log_scales, grads.quats, grads.logits, grads.sh, stats.kappa_sum,
                      stats.omega_sum, stats.gamma_sum, stats.grad_norm_sum, stats.view_count, stats.max_radius):
                t.zero_()
            for v in range(V):
                vi = Image(img.color[v:v + 1], img.depth[v:v + 1], img.t_final[v:v + 1], img.last[v:v + 1])
                R.project(g, cam_rows[v])
                R.bin_sort()
                R.render_fwd(vi)
                R.loss_l1(target[v:v + 1], vi, dl[v:v + 1], loss[v:v + 1])
                R.render_bwd(g, cam_rows[v], None, vi, dl[v:v + 1], target=target[v:v + 1], tau_err=0.1,
                             view_loss=loss[v:v + 1], grads=grads, pose_grad=pose[v:v + 1], stats=stats)

    def render_all():
        out = Image.empty(V, H, W)
        Rr = Rasterizer(W, H, V, sc.n, slot_capacity=slot_capacity, pair_capacity=pair_capacity, tile=tile,
                        batch=batch, far_z=far_z)
        Rr.project(g, cams)
        Rr.bin_sort()
        Rr.render_fwd(out)
        torch.cuda.synchronize()
        assert Rr.status() == 0
        return out.color

    p0 = psnr(render_all(), target)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(1, iters + 1):
        step_fn()
        for k in PARAMS:
            p, gr = getattr(g, k), getattr(grads, k)
            L.kgs_adam(p, m[k], v2[k], gr, p.numel(), it, LR[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert R.status() == 0, f"capacity status {R.status()}"
    l1 = float(loss.double().sum().item())
    p1 = psnr(render_all(), target)
    return dict(psnr_db=p1, psnr_start_db=p0, l1_last_step=l1, ms_per_step=1e3 * dt / iters, iterations=iters)
