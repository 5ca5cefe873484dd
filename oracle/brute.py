"""Tile-free compositing in plain PyTorch FP64, differentiable by autograd.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  A second, independent
opinion on tiny scenes: it never bins into tiles (every visible Gaussian is a
candidate for every pixel), builds the pose with torch.linalg.matrix_exp,
evaluates spherical harmonics from their explicit Cartesian polynomials and
lets autograd produce every gradient, including the 6-DoF pose one.

Colour and depth follow depth volume rendering (appendix, "Depth Volume
Rendering"): D = sum_j T_j alpha_j z_j, T_j = prod_{m<j} (1 - alpha_m); colour
uses the same weights.
"""
from __future__ import annotations

import math

import torch

SQ = math.sqrt


def real_sh_polys(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Real spherical harmonics (Condon-Shortley phase, index l^2 + l + m) of unit
    vectors d [..., 3], from their Cartesian polynomial forms."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    pi = math.pi
    out = [torch.full_like(x, 0.5 / SQ(pi))]
    if degree >= 1:
        c = SQ(3.0 / (4 * pi))
        out += [-c * y, c * z, -c * x]
    if degree >= 2:
        out += [0.5 * SQ(15 / pi) * x * y, -0.5 * SQ(15 / pi) * y * z,
                0.25 * SQ(5 / pi) * (3 * z * z - 1.0), -0.5 * SQ(15 / pi) * x * z,
                0.25 * SQ(15 / pi) * (x * x - y * y)]
    if degree >= 3:
        out += [-0.25 * SQ(35 / (2 * pi)) * y * (3 * x * x - y * y), 0.5 * SQ(105 / pi) * x * y * z,
                -0.25 * SQ(21 / (2 * pi)) * y * (5 * z * z - 1.0), 0.25 * SQ(7 / pi) * z * (5 * z * z - 3.0),
                -0.25 * SQ(21 / (2 * pi)) * x * (5 * z * z - 1.0), 0.25 * SQ(105 / pi) * z * (x * x - y * y),
                -0.25 * SQ(35 / (2 * pi)) * x * (x * x - 3 * y * y)]
    return torch.stack(out, dim=-1)


def _hat(xi: torch.Tensor) -> torch.Tensor:
    z = torch.zeros((), dtype=xi.dtype)
    r0, r1, r2, p0, p1, p2 = xi.unbind()
    return torch.stack([
        torch.stack([z, -p2, p1, r0]), torch.stack([p2, z, -p0, r1]),
        torch.stack([-p1, p0, z, r2]), torch.stack([z, z, z, z])])


def quat_rot(q: torch.Tensor) -> torch.Tensor:
    q = q / q.norm(dim=0, keepdim=True)
    w, x, y, z = q
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)])])  # [3,3,N]


def render(params: dict, cam, degree: int, cfg, xi: torch.Tensor):
    """params: means [3,N], log_scales [3,N], quats [4,N], logits [N], sh [K,3,N]
    (FP64 tensors); cam: one CAMERA_DTYPE record; xi: [6] tangent.  Returns
    colour [3,H,W], depth [H,W] and the opacity image 1 - T_final [H,W]."""
    dt = torch.float64
    W, H = int(cam["width"]), int(cam["height"])
    fx, fy, cx, cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    T0 = torch.eye(4, dtype=dt)
    T0[:3, :3] = torch.tensor(cam["R"].reshape(3, 3).astype("float64"))
    T0[:3, 3] = torch.tensor(cam["t"].astype("float64"))
    T = torch.linalg.matrix_exp(_hat(xi)) @ T0
    Rp, tp = T[:3, :3], T[:3, 3]
    ctr = -Rp.T @ tp
    mu = params["means"]
    t = Rp @ mu + tp[:, None]
    tx, ty, tz = t
    o = torch.sigmoid(params["logits"])
    # near plane; the single-level distance mask keeps camera depths below far
    vis = (tz > cfg.near) & (tz < cfg.far) & (o >= cfg.alpha_min)
    Rq = quat_rot(params["quats"])
    s = torch.exp(params["log_scales"])
    M = Rq * s[None, :, :]
    covw = torch.einsum("ikn,jkn->ijn", M, M)
    covc = torch.einsum("ai,ijn,bj->abn", Rp, covw, Rp)
    hx, hy = 0.5 * W / fx, 0.5 * H / fy
    mx, my = (0.5 * W - cx) / fx, (0.5 * H - cy) / fy
    ux = torch.clamp(tx / tz, mx - cfg.guard * hx, mx + cfg.guard * hx)
    uy = torch.clamp(ty / tz, my - cfg.guard * hy, my + cfg.guard * hy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * ux / tz]),
                     torch.stack([zero, fy / tz, -fy * uy / tz])])  # [2,3,N]
    S2 = torch.einsum("akn,kln,bln->abn", J, covc, J)
    Sxx = S2[0, 0] + cfg.eps2d
    Sxy = S2[0, 1]
    Syy = S2[1, 1] + cfg.eps2d
    det = Sxx * Syy - Sxy * Sxy
    ca, cb, cc = Syy / det, -Sxy / det, Sxx / det
    mux = fx * tx / tz + cx
    muy = fy * ty / tz + cy
    dv = mu - ctr[:, None]
    dirs = (dv / dv.norm(dim=0, keepdim=True)).T
    Y = real_sh_polys(dirs, degree)  # [N,K]
    raw = torch.einsum("nk,kcn->cn", Y, params["sh"]) + 0.5
    col = torch.clamp(raw, min=0.0)
    idx = torch.nonzero(vis).flatten()
    # front-to-back order: fp32 depth, then index
    zf = tz.detach().to(torch.float32)[idx]
    order = sorted(range(len(idx)), key=lambda k: (float(zf[k]), int(idx[k])))
    idx = idx[order]
    py, px = torch.meshgrid(torch.arange(H, dtype=dt) + 0.5, torch.arange(W, dtype=dt) + 0.5, indexing="ij")
    px, py = px.reshape(-1), py.reshape(-1)
    Tr = torch.ones_like(px)
    C = torch.zeros(3, px.shape[0], dtype=dt)
    D = torch.zeros_like(px)
    done = torch.zeros_like(px, dtype=torch.bool)
    for g in idx.tolist():
        dx, dy = px - mux[g], py - muy[g]
        q = ca[g] * dx * dx + 2 * cb[g] * dx * dy + cc[g] * dy * dy
        a_raw = o[g] * torch.exp(-0.5 * q)
        a = torch.clamp(a_raw, max=cfg.alpha_max)
        use = (a_raw >= cfg.alpha_min) & ~done
        Tn = Tr * (1 - a)
        stop = use & (Tn < cfg.t_min)
        done = done | stop
        use = use & ~stop
        w = torch.where(use, Tr * a, torch.zeros_like(a))
        C = C + w[None, :] * col[:, g:g + 1]
        D = D + w * tz[g]
        Tr = torch.where(use, Tn, Tr)
    bg = torch.tensor(cfg.bg, dtype=dt)[:, None]
    C = C + Tr[None, :] * bg
    return C.reshape(3, H, W), D.reshape(H, W), (1.0 - Tr).reshape(H, W)
