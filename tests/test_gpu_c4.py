"""Differentiable pose + map workload (5M Gaussians, 16 keyframes, each pose
perturbed by 0.5 degrees / 0.2 m): finite-difference check of every gradient
on a 2k-Gaussian subset, and the full-size chunk against the oracle and the
translation identity."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import OracleConfig
from paper_2606_30436_amd import scenes
from paper_2606_30436_amd.raster import render
from paper_2606_30436_amd.rasterizer import GaussianParams, Image, Rasterizer, device_cameras
from tests.gpu_util import affected_gaussians, compare_image, grad_close, oracle_cfg, say

pytestmark = pytest.mark.gpu

FAR = 80.0


@pytest.fixture(scope="module")
def c4():
    return scenes.make_c4()


def _crop_subset(sc, v, W=112, H=84, n_keep=2000, seed=0):
    """A W x H window at the centre of view v and 2000 Gaussians that project
    into it (camera-frame geometry of the unperturbed pose)."""
    cam = sc.cams[v]
    R = cam["R"].reshape(3, 3).astype(np.float64)
    t = cam["t"].astype(np.float64)
    x = R @ sc.means.astype(np.float64) + t[:, None]
    ok = (x[2] > 2.0) & (x[2] < FAR)
    u = cam["fx"] * x[0] / np.where(ok, x[2], 1) + cam["cx"]
    w = cam["fy"] * x[1] / np.where(ok, x[2], 1) + cam["cy"]
    x0, y0 = float(cam["cx"]) - W / 2, float(cam["cy"]) - H / 2
    inside = ok & (u > x0 - 8) & (u < x0 + W + 8) & (w > y0 - 8) & (w < y0 + H + 8)
    idx = np.nonzero(inside)[0]
    idx = np.sort(np.random.default_rng(seed).choice(idx, size=min(n_keep, len(idx)), replace=False))
    sub = sc.subset(idx).views([v])
    crop = scenes.make_camera(R, t, cam["fx"], cam["fy"], cam["cx"] - x0, cam["cy"] - y0, W, H)
    sub.cams = scenes.stack_cameras([crop])
    return sub


def test_c4_subset_gradients_match_fp64_finite_differences(c4):
    sub = _crop_subset(c4, 0)
    say(f"[gpu] C4 FD subset n={sub.n} xi={sub.pose_xi[0]}")
    smooth = dict(alpha_min=1e-12, alpha_max=1.0, t_min=0.0, far_z=FAR)
    R = Rasterizer(sub.width, sub.height, max_views=1, max_gaussians=sub.n, **smooth)
    g = GaussianParams.from_scene(sub)
    cams = device_cameras(sub.cams)
    xi = torch.from_numpy(sub.pose_xi).cuda()
    R.project(g, cams, xi)
    R.bin_sort()
    img = Image.empty(1, sub.height, sub.width)
    R.render_fwd(img)
    rng = np.random.default_rng(1)
    wC = rng.normal(size=(1, 3, sub.height, sub.width))
    wD = rng.normal(size=(1, sub.height, sub.width)) * 0.02
    grads = g.zeros_like()
    pg = torch.zeros(1, 6, device="cuda")
    R.render_bwd(g, cams, xi, img, torch.from_numpy(wC.astype(np.float32)).cuda(),
                 torch.from_numpy(wD.astype(np.float32)).cuda(), grads=grads, pose_grad=pg)
    torch.cuda.synchronize()
    cfg = OracleConfig.smooth(far=FAR)
    ov = oracle.View(sub, 0, cfg)
    an = ov.backward(wC[0], wD[0])
    got = {k: getattr(grads, k).cpu().numpy().astype(np.float64) for k in ("means", "log_scales", "quats", "sh")}
    got["logits"] = grads.logits.cpu().numpy().astype(np.float64)
    for k in got:
        rel = np.linalg.norm(got[k] - an[k]) / np.linalg.norm(an[k])
        say(f"  {k}: GPU vs FP64 analytic rel {rel:.2e}")
        assert rel < 1e-3, k
    gx = pg.cpu().numpy()[0].astype(np.float64)
    assert np.linalg.norm(gx - an["pose_xi"]) / np.linalg.norm(an["pose_xi"]) < 1e-3

    base = {k: getattr(sub, k).astype(np.float64) for k in ("means", "log_scales", "quats", "logits", "sh")}
    base["pose_xi"] = sub.pose_xi.astype(np.float64)

    def loss(pp):
        im = oracle.View(sub, 0, cfg, pp).image()
        return float((im["color"] * wC[0]).sum() + (im["depth"] * wD[0]).sum())

    # 40 parameter entries of the Gaussians with the largest gradients, plus all 6 pose DOF
    order = np.argsort(-np.abs(an["means"]).sum(0))[:64]
    checks = []
    names = [("means", 3), ("log_scales", 3), ("quats", 4), ("logits", 0), ("sh", 0)]
    for j in range(40):
        gi = int(order[rng.integers(len(order))])
        name, dim = names[j % len(names)]
        if name == "logits":
            idx = (gi,)
        elif name == "sh":
            idx = (int(rng.integers(sub.sh.shape[0])), int(rng.integers(3)), gi)
        else:
            idx = (int(rng.integers(dim)), gi)
        checks.append((name, idx))
    checks += [("pose_xi", (0, k)) for k in range(6)]
    scale = {k: math.sqrt(np.mean(an[k] ** 2)) for k in ("means", "log_scales", "quats", "logits", "sh")}
    scale["pose_xi"] = float(np.abs(an["pose_xi"]).max())
    worst = 0.0
    for name, idx in checks:
        h = 1e-6 * max(1.0, abs(base[name][idx]))
        vals = []
        for sgn in (1, -1):
            pp = {k: v.copy() for k, v in base.items()}
            pp[name][idx] += sgn * h
            vals.append(loss(pp))
        fd = (vals[0] - vals[1]) / (2 * h)
        gpu = gx[idx[1]] if name == "pose_xi" else got[name][idx]
        err = abs(gpu - fd) / (abs(fd) + 0.01 * scale[name])
        worst = max(worst, err)
        assert err < 1e-3, (name, idx, gpu, fd)
    say(f"  {len(checks)} FD checks, worst relative error {worst:.2e}")


def test_c4_full_chunk(c4):
    """5M Gaussians, 16 keyframes each perturbed by 0.5 degrees / 0.2 m, at 1242x375: one batched call through
    the autograd path (recompute in backward) with random colour and depth weights.  All 16 images, all 16
    pose gradients at the perturbed poses and the parameter gradients summed over the 16 views against the
    oracle's 16 views; then the translation identity for two single-view calls at the unperturbed pose."""
    sc = c4
    V = sc.n_views
    say(f"[gpu] C4 full chunk n={sc.n} V={V}")
    R = Rasterizer(sc.width, sc.height, max_views=V, max_gaussians=sc.n, slot_capacity=24_000_000,
                   pair_capacity=200_000_000, far_z=FAR)
    g0 = GaussianParams.from_scene(sc)
    P = {k: getattr(g0, k).requires_grad_(True) for k in ("means", "log_scales", "quats", "logits", "sh")}
    cams = device_cameras(sc.cams)
    xi = torch.from_numpy(sc.pose_xi).cuda().requires_grad_(True)
    rng = np.random.default_rng(44)
    wC = rng.normal(size=(V, 3, sc.height, sc.width)).astype(np.float32) * np.float32(1e-3)
    wD = rng.normal(size=(V, sc.height, sc.width)).astype(np.float32) * np.float32(1e-5)
    C, D, _ = render(P, cams, xi, R, 3)
    ((C * torch.from_numpy(wC).cuda()).sum() + (D * torch.from_numpy(wD).cuda()).sum()).backward()
    torch.cuda.synchronize()
    assert R.status() == 0
    ns, npairs = R.counts()
    say(f"  slots {ns} pairs {npairs}")
    cfg = oracle_cfg(R)
    col = C.detach().cpu().numpy()
    pg = xi.grad.cpu().numpy().astype(np.float64)
    ref = {k: 0.0 for k in ("means", "log_scales", "quats", "logits", "sh")}
    flagged = np.zeros(sc.n, bool)
    for v in range(V):
        ov = oracle.View(sc, v, cfg)
        oi = ov.image()
        err, nbad, namb = compare_image(col[v], oi)
        an = ov.backward(wC[v].astype(np.float64), wD[v].astype(np.float64))
        flagged |= affected_gaussians(ov, oi)
        prel = np.linalg.norm(pg[v] - an["pose_xi"]) / np.linalg.norm(an["pose_xi"])
        say(f"  view {v}: image error {err:.2e} (outside tolerance {nbad}, at a margin {namb}), "
            f"pose rel {prel:.2e}")
        assert prel < 1e-3, v
        for k in ref:
            ref[k] = ref[k] + an[k]
        del ov
    for k in ref:
        rel, nb = grad_close(k, P[k].grad.cpu().numpy(), ref[k], flagged)
        say(f"  summed over 16 views: {k} rel {rel:.2e}, Gaussians outside tolerance {nb} "
            f"(all flagged; {int(flagged.sum())} flagged)")
    # one view at a time at xi = 0: sum_i dL/dmu_i = R^T dL/drho
    for v in (0, V - 1):
        one = sc.views([v])
        one.pose_xi = np.zeros((1, 6), np.float32)
        R1 = Rasterizer(sc.width, sc.height, max_views=1, max_gaussians=sc.n, slot_capacity=4_000_000,
                        pair_capacity=40_000_000, far_z=FAR)
        g = GaussianParams.from_scene(one)
        c1 = device_cameras(one.cams)
        z = torch.zeros(1, 6, device="cuda")
        R1.project(g, c1, z)
        R1.bin_sort()
        img = Image.empty(1, sc.height, sc.width)
        R1.render_fwd(img)
        w1 = np.random.default_rng(4 + v).normal(size=(1, 3, sc.height, sc.width)) * 1e-3
        grads = g.zeros_like()
        pg1 = torch.zeros(1, 6, device="cuda")
        R1.render_bwd(g, c1, z, img, torch.from_numpy(w1.astype(np.float32)).cuda(), grads=grads, pose_grad=pg1)
        torch.cuda.synchronize()
        assert R1.status() == 0
        gm = grads.means.double().sum(1).cpu().numpy()
        Rm = one.cams[0]["R"].reshape(3, 3).astype(np.float64)
        rho = pg1.cpu().numpy()[0, :3].astype(np.float64)
        rel = np.linalg.norm(gm - Rm.T @ rho) / np.linalg.norm(rho)
        say(f"  view {v}: translation identity rel {rel:.2e}")
        assert rel < 1e-3
        del R1


@pytest.mark.parametrize("v", range(16))
def test_c4_pose_gradient_fd_every_view(c4, v):
    """The 6 pose degrees of freedom of every keyframe at its perturbed pose, on a 112x84 window of that view
    with 2000 of the Gaussians that project into it: GPU gradient against FP64 central differences of the
    oracle with thresholds switched off."""
    sub = _crop_subset(c4, v, seed=v)
    say(f"[gpu] C4 pose FD view {v} n={sub.n}")
    smooth = dict(alpha_min=1e-12, alpha_max=1.0, t_min=0.0, far_z=FAR)
    R = Rasterizer(sub.width, sub.height, max_views=1, max_gaussians=sub.n, **smooth)
    g = GaussianParams.from_scene(sub)
    cams = device_cameras(sub.cams)
    xi = torch.from_numpy(sub.pose_xi).cuda()
    R.project(g, cams, xi)
    R.bin_sort()
    img = Image.empty(1, sub.height, sub.width)
    R.render_fwd(img)
    rng = np.random.default_rng(100 + v)
    wC = rng.normal(size=(1, 3, sub.height, sub.width))
    wD = rng.normal(size=(1, sub.height, sub.width)) * 0.02
    grads = g.zeros_like()
    pg = torch.zeros(1, 6, device="cuda")
    R.render_bwd(g, cams, xi, img, torch.from_numpy(wC.astype(np.float32)).cuda(),
                 torch.from_numpy(wD.astype(np.float32)).cuda(), grads=grads, pose_grad=pg)
    torch.cuda.synchronize()
    gx = pg.cpu().numpy()[0].astype(np.float64)
    cfg = OracleConfig.smooth(far=FAR)
    base = {k: getattr(sub, k).astype(np.float64) for k in ("means", "log_scales", "quats", "logits", "sh")}
    base["pose_xi"] = sub.pose_xi.astype(np.float64)
    scale = float(np.abs(gx).max())
    worst = 0.0
    for k in range(6):
        h = 1e-6
        vals = []
        for sgn in (1, -1):
            pp = {a: b.copy() for a, b in base.items()}
            pp["pose_xi"][0, k] += sgn * h
            im = oracle.View(sub, 0, cfg, pp).image()
            vals.append(float((im["color"] * wC[0]).sum() + (im["depth"] * wD[0]).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        err = abs(gx[k] - fd) / (abs(fd) + 0.01 * scale)
        worst = max(worst, err)
        assert err < 1e-3, (v, k, gx[k], fd)
    say(f"  view {v}: worst pose FD relative error {worst:.2e}")
