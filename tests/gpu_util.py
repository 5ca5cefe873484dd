"""Shared helpers of the GPU parity tests: run the HIP path on a scene, run the
oracle on the same scene, and the comparison rules (tolerances and the
near-threshold exclusions)."""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

import oracle
from oracle import OracleConfig
from paper_2606_30436_amd import rasterizer as rz
from paper_2606_30436_amd.rasterizer import GaussianParams, Image, Rasterizer, ViewStats, device_cameras

LOG2E = 1.4426950408889634

# Relative margins below which an FP32 decision may differ from the FP64 one.
# The FP32 error of log2(alpha) at the alpha_min boundary is about 2e-5
# (centre and conic rounding); transmittance accumulates about ten of those
# before it reaches T_min.  The margins keep a factor of ten on both.
MARGIN_ALPHA = 2e-4
MARGIN_T = 2e-3
# Both sides order a pixel's Gaussians by the FP32 rounding of an FP64 camera
# depth, ties by index.  The two FP64 depths differ by ~1e-14 relative at
# kilometre map coordinates, so an order can differ only where two contributing
# Gaussians' FP32 keys are equal or adjacent AND one FP64 depth lies that close
# to an FP32 rounding boundary (the oracle's fourth margin plane).  1e-9 keeps
# five orders of magnitude.
MARGIN_DEPTH = 1e-9
# Largest share of pixels (images) or Gaussians (gradients, counts) whose
# comparison may fail; every failure must in addition sit at a margin.
MAX_MISMATCH_SHARE = 1e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_cfg(R: Rasterizer) -> OracleConfig:
    c = R.cfg
    return OracleConfig(alpha_min=c.alpha_min, alpha_max=c.alpha_max, t_min=c.t_min, near=c.near_z, eps2d=c.eps2d,
                        guard=c.guard, rect_margin=c.rect_margin, far=c.far_z, bg=tuple(c.bg), tile_w=c.tile_w,
                        tile_h=c.tile_h)


def run_forward(R: Rasterizer, sc, pose=True):
    g = GaussianParams.from_scene(sc)
    cams = device_cameras(sc.cams)
    xi = torch.from_numpy(sc.pose_xi.astype(np.float32)).cuda() if pose else None
    V = R.project(g, cams, xi)
    R.bin_sort()
    img = Image.empty(V, sc.height, sc.width)
    R.render_fwd(img)
    torch.cuda.synchronize()
    return g, cams, xi, img


def rect_hits(mask: np.ndarray, fxi, fyi, rx, ry) -> np.ndarray:
    """For each Gaussian, does its pixel rectangle hold a True pixel of mask?"""
    H, W = mask.shape
    sat = np.zeros((H + 1, W + 1), np.int64)
    sat[1:, 1:] = np.cumsum(np.cumsum(mask.astype(np.int64), 0), 1)
    x0 = np.clip(fxi - rx, 0, W)
    x1 = np.clip(fxi + rx + 1, 0, W)
    y0 = np.clip(fyi - ry, 0, H)
    y1 = np.clip(fyi + ry + 1, 0, H)
    s = sat[y1, x1] - sat[y0, x1] - sat[y1, x0] + sat[y0, x0]
    return (s > 0) & (x1 > x0) & (y1 > y0)


def ambiguous_pixels(oi) -> np.ndarray:
    m = oi["margins"]
    return (m[0] <= MARGIN_ALPHA) | (m[1] <= MARGIN_T) | (m[3] <= MARGIN_DEPTH)


def involved_gaussians(ov) -> np.ndarray:
    """Gaussians that themselves sit at a threshold somewhere in this view: own
    alpha at alpha_min or at the alpha_max clamp, ending a pixel's sequence at
    T_min, at the colour clamp or at the guard band."""
    gm = ov.gauss_margins()
    pr = ov.proj()
    m = pr["margins"]
    own = (gm[:, 0] <= MARGIN_ALPHA) | (gm[:, 1] <= MARGIN_ALPHA) | (gm[:, 2] <= MARGIN_T)
    return pr["visible"] & (own | (m[:, 4] < 1e-4) | (m[:, 2] < 1e-5) | (m[:, 3] < 1e-5))


def affected_gaussians(ov, oi=None) -> np.ndarray:
    """Gaussians whose gradient may legitimately differ between FP32 and FP64:
    those at a threshold themselves (involved_gaussians) and those whose
    rectangle holds a pixel at a margin (a flip there changes every gradient
    blended at that pixel)."""
    oi = ov.image() if oi is None else oi
    pr = ov.proj()
    return involved_gaussians(ov) | (rect_hits(ambiguous_pixels(oi), pr["fxi"], pr["fyi"], pr["rx"], pr["ry"])
                                     & pr["visible"])


def grad_close(name, got, ref, flagged, rel_norm=1e-3, rel_elem=1e-3):
    """Norm-wise ||d|| <= rel_norm ||g|| over every Gaussian, and per Gaussian
    |d| <= rel_elem (||g_i|| + 0.01 rms(g)) for every component of its gradient
    in this tensor (||g_i|| the norm of that Gaussian's components: a quaternion
    gradient is projected orthogonal to q, so one component can be small next to
    the others).  A Gaussian that fails must be flagged (affected_gaussians), and
    at most MAX_MISMATCH_SHARE of the Gaussians may fail.  Returns the relative
    error and the number of Gaussians that failed."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    d = got - ref
    nr = np.linalg.norm(ref)
    if nr == 0:
        assert np.abs(got).max(initial=0) < 1e-12, name
        return 0.0, 0
    rel = np.linalg.norm(d) / nr
    assert rel <= rel_norm, (name, rel)
    rms = math.sqrt(np.mean(ref * ref))
    n = ref.shape[-1]
    gnorm = np.sqrt((ref.reshape(-1, n) ** 2).sum(0))
    bad_g = (np.abs(d.reshape(-1, n)) > rel_elem * (gnorm + 0.01 * rms)).any(0)
    unexplained = bad_g & ~np.asarray(flagged, bool)
    assert not unexplained.any(), (name, int(unexplained.sum()), np.flatnonzero(unexplained)[:8])
    assert bad_g.mean() <= MAX_MISMATCH_SHARE, (name, int(bad_g.sum()), bad_g.size)
    return rel, int(bad_g.sum())


def compare_image(got_color, oi, tol=1e-4, got_depth=None, got_tfinal=None) -> tuple:
    """Every pixel compared: colour (and depth relative to max(1, D), final
    transmittance) within tol of the oracle; a pixel outside it must be at a
    margin (ambiguous_pixels), and at most MAX_MISMATCH_SHARE of the pixels may
    be.  Returns (max error over the pixels within tolerance, failing pixels,
    pixels at a margin)."""
    amb = ambiguous_pixels(oi)
    dc = np.abs(np.asarray(got_color, np.float64) - oi["color"]).max(0)
    bad = dc > tol
    if got_depth is not None:
        bad |= np.abs(np.asarray(got_depth, np.float64) - oi["depth"]) > tol * np.maximum(1.0, oi["depth"])
    if got_tfinal is not None:
        bad |= np.abs(np.asarray(got_tfinal, np.float64) - oi["tfinal"]) > tol
    unexplained = bad & ~amb
    assert not unexplained.any(), (int(unexplained.sum()), float(dc[unexplained].max()),
                                   np.argwhere(unexplained)[:4].tolist())
    assert bad.mean() <= MAX_MISMATCH_SHARE, (int(bad.sum()), bad.size)
    return float(dc[~bad].max(initial=0.0)), int(bad.sum()), int(amb.sum())
