"""The autograd wrapper on the GPU: gradients for all Gaussian parameters and
the 6-DoF poses against PyTorch FP64 autograd through a tile-free reference,
recompute-in-backward against stored lists, and pose recovery by descent."""
import math

import numpy as np
import pytest
import torch

from oracle import OracleConfig, brute
from paper_2606_30436_amd import scenes
from paper_2606_30436_amd.raster import render
from paper_2606_30436_amd.rasterizer import GaussianParams, Rasterizer, device_cameras
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _params(sc, grad=True):
    g = GaussianParams.from_scene(sc)
    out = {"means": g.means, "log_scales": g.log_scales, "quats": g.quats, "logits": g.logits, "sh": g.sh}
    for t in out.values():
        t.requires_grad_(grad)
    return out


@pytest.mark.parametrize("seed,bg", [(5, (0.0, 0.0, 0.0)), (6, (0.3, 0.1, 0.7))])
def test_autograd_matches_fp64_tile_free_autograd(seed, bg):
    sc = scenes.tiny_scene(seed=seed, n=50, degree=3, W=48, H=40, n_views=2, pose_sigma=0.03)
    say(f"[gpu] autograd vs FP64 autograd seed={seed}")
    R = Rasterizer(sc.width, sc.height, max_views=2, max_gaussians=sc.n, bg=bg)
    P = _params(sc)
    xi = torch.from_numpy(sc.pose_xi).cuda().requires_grad_(True)
    cams = device_cameras(sc.cams)
    C, D, Tf = render(P, cams, xi, R, sc.sh_degree)
    rng = np.random.default_rng(seed)
    wC = rng.normal(size=C.shape)
    wD = rng.normal(size=D.shape) * 0.05
    wT = rng.normal(size=Tf.shape)
    L = (C * torch.from_numpy(wC).float().cuda()).sum() + (D * torch.from_numpy(wD).float().cuda()).sum() + \
        (Tf * torch.from_numpy(wT).float().cuda()).sum()
    L.backward()
    cfg = OracleConfig(bg=bg)
    ref = {k: torch.tensor(getattr(sc, k).astype(np.float64), requires_grad=True)
           for k in ("means", "log_scales", "quats", "logits", "sh")}
    xr = torch.tensor(sc.pose_xi.astype(np.float64), requires_grad=True)
    Lr = 0.0
    for v in range(2):
        Cr, Dr, Ar = brute.render(ref, sc.cams[v], sc.sh_degree, cfg, xr[v])
        assert np.abs(Cr.detach().numpy() - C[v].detach().cpu().numpy()).max() < 2e-3
        # the tile-free reference gives the opacity image A = 1 - T_final
        Lr = Lr + (Cr * torch.tensor(wC[v])).sum() + (Dr * torch.tensor(wD[v])).sum() + \
            ((1.0 - Ar) * torch.tensor(wT[v])).sum()
    Lr.backward()
    for k in ref:
        got = P[k].grad.detach().cpu().numpy().astype(np.float64)
        want = ref[k].grad.numpy()
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        say(f"  {k}: rel {rel:.2e}")
        assert rel < 1e-3, k
    gx = xi.grad.detach().cpu().numpy()
    rel = np.linalg.norm(gx - xr.grad.numpy()) / np.linalg.norm(xr.grad.numpy())
    say(f"  pose: rel {rel:.2e}")
    assert rel < 1e-3


def test_recompute_in_backward_equals_stored_lists():
    sc = scenes.tiny_scene(seed=8, n=120, degree=2, W=80, H=64, n_views=3, pose_sigma=0.02)
    R = Rasterizer(sc.width, sc.height, max_views=3, max_gaussians=sc.n)
    cams = device_cameras(sc.cams)
    grads = []
    for recompute in (True, False):
        P = _params(sc)
        xi = torch.from_numpy(sc.pose_xi).cuda().requires_grad_(True)
        C, D, Tf = render(P, cams, xi, R, sc.sh_degree, recompute=recompute)
        (C.square().sum() + 0.01 * D.sum() + Tf.sum()).backward()
        grads.append([P[k].grad.clone() for k in P] + [xi.grad.clone()])
    for a, b in zip(*grads):
        assert torch.equal(a, b)


def test_pose_descent_recovers_a_perturbed_camera():
    """Render targets at the true pose; start from a 0.5 degree / 0.2 m
    perturbation and descend on the pose alone."""
    sc = scenes.tiny_scene(seed=9, n=400, degree=1, W=96, H=72, n_views=1, depth=(2.0, 5.0), spread=0.9,
                           log_scale_mu=-2.3)
    R = Rasterizer(sc.width, sc.height, max_views=1, max_gaussians=sc.n)
    cams = device_cameras(sc.cams)
    P = _params(sc, grad=False)
    with torch.no_grad():
        target, _, _ = render(P, cams, None, R, sc.sh_degree)
    xi0 = scenes.random_pose_perturbation(np.random.default_rng(3), 1, angle_deg=0.5, trans=0.05)
    xi = torch.from_numpy(xi0).cuda().requires_grad_(True)
    opt = torch.optim.Adam([xi], lr=2e-3)
    losses = []
    for it in range(150):
        opt.zero_grad()
        C, _, _ = render(P, cams, xi, R, sc.sh_degree)
        loss = (C - target).abs().mean()
        loss.backward()
        opt.step()
        losses.append(float(loss))
    err0 = np.linalg.norm(xi0)
    err1 = float(xi.detach().norm())
    say(f"[gpu] pose descent: loss {losses[0]:.4f} -> {losses[-1]:.4f}, |xi| {err0:.4f} -> {err1:.4f}")
    assert losses[-1] < 0.5 * losses[0]
    assert err1 < 0.5 * err0
