"""Pins of the mapping-loss oracle (Sec. 3.2 mapping loss; appendix "Rendering
Objectives") against a library filter, closed forms, brute-force window sums
and FP64 finite differences.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage
import torch

from oracle import mapping_loss as ml

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_weights_are_the_papers():
    hp = json.load(open(os.path.join(GOLD, "hyperparameters.json")))
    assert ml.LAMBDA_G == hp["lambda_g"] and ml.LAMBDA_ISO == hp["lambda_iso"]
    assert (ml.W_L1, ml.W_SSIM) == (0.8, 0.2)


def test_window_blur_is_scipys_gaussian_filter():
    """The 11x11 window filter with zero padding equals scipy's Gaussian filter
    (sigma 1.5, radius 5, constant 0 outside)."""
    x = np.random.default_rng(0).uniform(size=(3, 23, 31))
    got = ml._blur(torch.tensor(x)).numpy()
    for c in range(3):
        ref = scipy.ndimage.gaussian_filter(x[c], 1.5, mode="constant", cval=0.0, truncate=5 / 1.5)
        assert np.allclose(got[c], ref, rtol=0, atol=1e-14)


def test_ssim_of_an_image_with_itself_is_one():
    x = torch.tensor(np.random.default_rng(1).uniform(size=(3, 20, 17)))
    assert torch.allclose(ml.ssim_map(x, x), torch.ones_like(x), rtol=0, atol=1e-14)
    assert ml.photo_loss(x, x).item() == pytest.approx(0.0, abs=1e-15)


def test_ssim_of_constant_images_closed_form():
    """Away from the border (5 pixels) two constant images a, b have sigma = 0, so
    SSIM = (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.7, 0.25
    x = torch.full((3, 24, 24), a, dtype=torch.float64)
    y = torch.full((3, 24, 24), b, dtype=torch.float64)
    s = ml.ssim_map(x, y)[:, 5:-5, 5:-5]
    want = (2 * a * b + ml.C1) / (a * a + b * b + ml.C1)
    assert torch.allclose(s, torch.full_like(s, want), rtol=0, atol=1e-12)


def _ssim_brute(x, y, c, py, px):
    """SSIM at one pixel from explicit window sums (zero outside the image)."""
    g = ml.gaussian_window()
    H, W = x.shape[1:]
    sums = dict(mx=0.0, my=0.0, xx=0.0, yy=0.0, xy=0.0)
    for i in range(11):
        for j in range(11):
            qy, qx = py + i - 5, px + j - 5
            if 0 <= qy < H and 0 <= qx < W:
                w = g[i] * g[j]
                a, b = x[c, qy, qx], y[c, qy, qx]
                sums["mx"] += w * a
                sums["my"] += w * b
                sums["xx"] += w * a * a
                sums["yy"] += w * b * b
                sums["xy"] += w * a * b
    mx, my = sums["mx"], sums["my"]
    vx, vy, cxy = sums["xx"] - mx * mx, sums["yy"] - my * my, sums["xy"] - mx * my
    return ((2 * mx * my + ml.C1) * (2 * cxy + ml.C2)) / ((mx * mx + my * my + ml.C1) * (vx + vy + ml.C2))


def test_ssim_matches_brute_force_window_sums():
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(3, 19, 26))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    s = ml.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    for c, py, px in [(0, 0, 0), (1, 9, 13), (2, 18, 25), (0, 3, 24), (2, 10, 2), (1, 17, 7)]:
        assert s[c, py, px] == pytest.approx(_ssim_brute(x, y, c, py, px), rel=1e-12, abs=1e-14)


def test_iso_closed_form():
    """Isotropic scales cost nothing; s = (c, 2c, 3c) costs |c - 2c| + 0 + |3c - 2c| = 2c."""
    ls = torch.tensor(np.log([[0.3, 0.1], [0.3, 0.2], [0.3, 0.3]]))
    assert ml.iso_loss(ls).item() == pytest.approx(2 * 0.1, rel=1e-14)


def test_gradients_match_fp64_central_differences():
    rng = np.random.default_rng(3)
    V, H, W, N = 2, 14, 18, 5
    col = rng.uniform(0.05, 0.95, (V, 3, H, W))
    tgt = np.clip(col + rng.normal(0, 0.15, col.shape), 0, 1)
    dep = rng.uniform(2, 20, (V, H, W))
    tdep = dep + rng.normal(0, 0.5, dep.shape)
    ls = rng.normal(-3, 0.5, (3, N))
    out = ml.mapping_loss(col, tgt, dep, tdep, ls)

    def total(c, d, l):
        return ml.mapping_loss(c, tgt, d, tdep, l)["total"]

    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 7, 9), (0, 1, 13, 17), (1, 0, 5, 0)]:
        cp, cm = col.copy(), col.copy()
        cp[idx] += h
        cm[idx] -= h
        fd = (total(cp, dep, ls) - total(cm, dep, ls)) / (2 * h)
        assert out["dl_dcolor"][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    for idx in [(0, 3, 4), (1, 13, 17)]:
        dp, dm = dep.copy(), dep.copy()
        dp[idx] += h
        dm[idx] -= h
        fd = (total(col, dp, ls) - total(col, dm, ls)) / (2 * h)
        assert out["dl_ddepth"][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    for idx in [(0, 1), (2, 4), (1, 3)]:
        lp, lm = ls.copy(), ls.copy()
        lp[idx] += h
        lm[idx] -= h
        fd = (total(col, dep, lp) - total(col, dep, lm)) / (2 * h)
        assert out["dl_dlog_scales"][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    # the L1 and depth parts in closed form: 0.8 sign / (3HW) per view plus the SSIM part;
    # lambda_g sign / (HW) for depth
    assert np.allclose(out["dl_ddepth"], ml.LAMBDA_G * np.sign(dep - tdep) / (H * W), rtol=1e-14, atol=0)
