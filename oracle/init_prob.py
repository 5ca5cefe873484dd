"""Probabilistic Gaussian initialisation and level-of-detail quantisation in
NumPy FP64.  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Sec. 3.3 "Probabilistic Gaussian Initialization" and the voxel rule of
Sec. 3.2 "Hierarchical Anchor Management":

    DoG(u, v)  = min(|(G_s1 - G_s2) * I|(u, v), 1)
    P(u, v)    = min(lambda DoG(u, v) + (1 - lambda) norm(||grad D||)(u, v), 1),  lambda = 0.9
    P_kf(u, v) = max(P(u, v) - P^(u, v), 0)     (P^ : the same map of the rendered I^, D^)
    3x3 non-maximum suppression over P_kf; the surviving pixels are unprojected
    and quantised:  p = floor(x / eps_l) eps_l  at the level l of their distance.

Readings where the paper is silent or garbled:
  * I is the mean of the three colour channels.  s1 = 1.0, s2 = 1.6 (the
    classic difference-of-Gaussians ratio).  A blur G_s is the sampled Gaussian
    of radius round(3 s), normalised, applied along rows then columns, with
    the border pixel repeated outside the image.
  * grad D by central differences inside the image and one-sided differences
    on its border; norm() is the min-max normalisation over the image (0 where
    max == min).
  * Non-maximum suppression keeps a pixel whose P_kf is positive and not below
    any of its (up to eight) neighbours inside the image.
  * "Spawning probability": a kept pixel spawns with probability P_kf, decided
    as u < P_kf by a uniform number u in [0, 1) per pixel passed in.
  * The unprojection uses the depth map D at the pixel centre (x + 0.5,
    y + 0.5) of a world->camera pinhole camera (R, t): x_cam = D K^-1 (u, v, 1),
    x = R^T (x_cam - t).  A pixel without a positive depth does not spawn.
  * Levels: voxel sizes eps = (0.1, 0.25, 1, 5, 25) -- the printed third size
    0.1 breaks the increasing sequence and is read as 1 -- and level l covers
    camera distances [D_max^(l-1), D_max^l) with D_max^l = 100 eps_l (the last
    level unbounded): a voxel then spans about the same number of pixels at the
    far end of every level.  The same bands are the level-of-detail mask.
Every decision (the suppression, u < P_kf, the level and the floor) is taken in
FP64.
"""
from __future__ import annotations

import numpy as np

LAMBDA = 0.9
SIGMA1, SIGMA2 = 1.0, 1.6
EPS = (0.1, 0.25, 1.0, 5.0, 25.0)
DMAX = tuple(100.0 * e for e in EPS[:-1]) + (np.inf,)


def kernel1d(sigma: float) -> np.ndarray:
    r = int(round(3.0 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-x * x / (2.0 * sigma * sigma))
    return w / w.sum()


def blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur of a 2D image, border pixel repeated."""
    k = kernel1d(sigma)
    r = len(k) // 2
    H, W = img.shape
    p = np.pad(img.astype(np.float64), ((0, 0), (r, r)), mode="edge")
    rows = sum(k[j] * p[:, j:j + W] for j in range(len(k)))
    p = np.pad(rows, ((r, r), (0, 0)), mode="edge")
    return sum(k[j] * p[j:j + H, :] for j in range(len(k)))


def dog(color: np.ndarray) -> np.ndarray:
    """DoG of the mean of the three channels of color [3, H, W], clipped at 1."""
    g = np.asarray(color, np.float64).mean(axis=0)
    return np.minimum(np.abs(blur(g, SIGMA1) - blur(g, SIGMA2)), 1.0)


def depth_gradient_norm(depth: np.ndarray) -> np.ndarray:
    """||grad D||: central differences inside, one-sided on the border."""
    d = np.asarray(depth, np.float64)
    H, W = d.shape
    gx = np.zeros_like(d)
    gy = np.zeros_like(d)
    if W > 1:
        gx[:, 1:-1] = (d[:, 2:] - d[:, :-2]) / 2.0
        gx[:, 0] = d[:, 1] - d[:, 0]
        gx[:, -1] = d[:, -1] - d[:, -2]
    if H > 1:
        gy[1:-1] = (d[2:] - d[:-2]) / 2.0
        gy[0] = d[1] - d[0]
        gy[-1] = d[-1] - d[-2]
    return np.sqrt(gx * gx + gy * gy)


def minmax_norm(a: np.ndarray) -> np.ndarray:
    lo, hi = a.min(), a.max()
    return (a - lo) / (hi - lo) if hi > lo else np.zeros_like(a)


def probability(color, depth) -> np.ndarray:
    """P = min(lambda DoG + (1 - lambda) norm(||grad D||), 1)."""
    return np.minimum(LAMBDA * dog(color) + (1.0 - LAMBDA) * minmax_norm(depth_gradient_norm(depth)), 1.0)


def nms3(p: np.ndarray) -> np.ndarray:
    """Pixels with p > 0 that are not below any 3x3 neighbour inside the image."""
    H, W = p.shape
    q = np.pad(p, 1, mode="constant", constant_values=-np.inf)
    keep = p > 0
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                keep &= p >= q[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
    return keep


def level_of(distance: float) -> int:
    """0-based level whose distance band [D_max^(l-1), D_max^l) holds distance."""
    for l, dm in enumerate(DMAX):
        if distance < dm:
            return l
    return len(DMAX) - 1


def spawn_candidates(color, depth, cam, u, rendered=None, rendered_depth=None) -> dict:
    """One keyframe: color [3, H, W], depth prior [H, W], one camera record
    (R, t, fx, fy, cx, cy), uniforms u [H, W]; optional render I^ [3, H, W] and
    D^ [H, W].  Returns P, P_kf, the kept mask, the spawning mask and, for the
    spawning pixels in raster order, their index, world point, level and voxel
    index (and the decision margins, for comparisons in another arithmetic)."""
    P = probability(color, depth)
    Pk = P if rendered is None else np.maximum(P - probability(rendered, rendered_depth), 0.0)
    keep = nms3(Pk)
    u = np.asarray(u, np.float64)
    d = np.asarray(depth, np.float64)
    spawn = keep & (u < Pk) & (d > 0)
    H, W = Pk.shape
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    fx, fy, cx, cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    centre = -R.T @ t
    pix = np.flatnonzero(spawn.reshape(-1))
    ys, xs = pix // W, pix % W
    z = d[ys, xs]
    xc = np.stack([z * (xs + 0.5 - cx) / fx, z * (ys + 0.5 - cy) / fy, z])
    X = R.T @ (xc - t[:, None])
    dist = np.linalg.norm(X - centre[:, None], axis=0)
    lev = np.array([level_of(v) for v in dist], np.int64)
    eps = np.array(EPS)[lev] if len(lev) else np.zeros(0)
    idx = np.floor(X / eps[None, :]).astype(np.int64) if len(lev) else np.zeros((3, 0), np.int64)
    # margins: how close each decision came to its threshold (relative where it has a scale)
    m_u = np.abs(u - Pk)
    q = np.pad(Pk, 1, mode="constant", constant_values=np.nan)
    m_nms = np.full(Pk.shape, np.inf)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                nb = q[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
                gap = np.abs(Pk - nb) / np.maximum(np.maximum(Pk, nb), 1e-300)
                both_clipped = (Pk == 1.0) & (nb == 1.0)   # exact on every side: min(., 1)
                gap = np.where(np.isnan(nb) | both_clipped, np.inf, gap)
                m_nms = np.minimum(m_nms, gap)
    with np.errstate(invalid="ignore"):
        frac = X / eps[None, :] - np.floor(X / eps[None, :]) if len(lev) else np.zeros((3, 0))
    m_floor = np.minimum(frac, 1.0 - frac).min(axis=0) if len(lev) else np.zeros(0)
    bands = np.array([dm for dm in DMAX if np.isfinite(dm)])
    m_level = (np.abs(dist[:, None] - bands[None, :]) / bands[None, :]).min(axis=1) if len(lev) else np.zeros(0)
    return dict(P=P, P_kf=Pk, keep=keep, spawn=spawn, pixel=pix, point=X.T, level=lev, voxel=idx.T,
                margin_u=m_u, margin_nms=m_nms, margin_floor=m_floor, margin_level=m_level)
