"""Pins of the probabilistic-initialisation oracle (Sec. 3.3 "Probabilistic
Gaussian Initialization"; Sec. 3.2 voxel quantisation) against library
routines, closed forms and hand-worked cases.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
import scipy.ndimage

from oracle import init_prob as ip
from paper_2606_30436_amd import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_constants_follow_the_paper_and_the_readings():
    hp = json.load(open(os.path.join(GOLD, "hyperparameters.json")))
    assert ip.LAMBDA == hp["dog_depth_lambda"]
    printed = hp["voxel_sizes_as_printed"]
    # every printed size kept but the out-of-sequence third one, read as 1
    assert len(ip.EPS) == hp["lod_levels_m"] and [ip.EPS[k] for k in (0, 1, 3, 4)] == [printed[k] for k in (0, 1, 3, 4)]
    assert ip.EPS[2] == 1.0 and all(a < b for a, b in zip(ip.EPS, ip.EPS[1:]))


@pytest.mark.parametrize("sigma", [ip.SIGMA1, ip.SIGMA2])
def test_blur_is_scipys_gaussian_filter_with_repeated_border(sigma):
    x = np.random.default_rng(0).uniform(size=(17, 29))
    ref = scipy.ndimage.gaussian_filter(x, sigma, mode="nearest", truncate=3.0)
    assert np.allclose(ip.blur(x, sigma), ref, rtol=0, atol=1e-14)


def test_depth_gradient_is_numpys_gradient():
    d = np.random.default_rng(1).uniform(2, 50, size=(13, 21))
    gy, gx = np.gradient(d)
    assert np.allclose(ip.depth_gradient_norm(d), np.hypot(gx, gy), rtol=1e-15, atol=0)


def test_flat_inputs_give_zero_probability():
    """A uniform image has no DoG response; a plane of constant slope has a constant
    gradient norm, which min-max normalises to 0."""
    col = np.full((3, 12, 15), 0.37)
    yy, xx = np.mgrid[0:12, 0:15]
    depth = 5.0 + 0.125 * xx + 0.25 * yy   # binary fractions: every difference is exact
    assert np.abs(ip.dog(col)).max() < 1e-15            # the two normalised blurs of a constant agree to rounding
    assert not ip.minmax_norm(ip.depth_gradient_norm(depth)).any()
    assert ip.probability(col, depth).max() < 1e-15


def test_dog_of_an_impulse_and_the_clip():
    """A single bright pixel far from the border: (G_s1 - G_s2) * delta at the pixel is the
    product of the centre taps, k1(0)^2 - k2(0)^2, scaled by its value over three channels;
    a large enough value clips at 1."""
    col = np.zeros((3, 21, 21))
    col[:, 10, 10] = 1.0
    k1, k2 = ip.kernel1d(ip.SIGMA1), ip.kernel1d(ip.SIGMA2)
    want = abs(k1[len(k1) // 2] ** 2 - k2[len(k2) // 2] ** 2)
    assert ip.dog(col)[10, 10] == pytest.approx(want, rel=1e-12)
    assert 1.0 / (2.0 * math.pi * ip.SIGMA1 ** 2) > want > 0.05   # near the continuous peak difference
    col[:, 10, 10] = 1e3
    assert ip.dog(col)[10, 10] == 1.0


def test_residual_against_the_render():
    """P_kf = max(P - P^, 0): a render equal to the input leaves nothing to spawn."""
    sc_rng = np.random.default_rng(2)
    col = sc_rng.uniform(size=(3, 16, 20))
    dep = sc_rng.uniform(2, 30, size=(16, 20))
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 20.0, 20.0, 10.0, 8.0, 20, 16)
    u = sc_rng.uniform(size=(16, 20))
    out = ip.spawn_candidates(col, dep, cam, u, rendered=col, rendered_depth=dep)
    assert not out["P_kf"].any() and not out["spawn"].any()
    out = ip.spawn_candidates(col, dep, cam, u)
    assert np.array_equal(out["P_kf"], ip.probability(col, dep)) and out["spawn"].any()


def test_nms_truth_table():
    p = np.array([[0.0, 0.2, 0.2, 0.1],
                  [0.3, 0.1, 0.2, 0.0],
                  [0.0, 0.0, 0.0, 0.5],
                  [0.4, 0.0, 0.0, 0.5]])
    # (0,1) lies below the 0.3 at (1,0); (0,2) ties with (0,1) and (1,2) and is below none: kept
    # (a plateau keeps every member not below a neighbour); (1,2) lies below the 0.5 at (2,3);
    # (2,3) and (3,3) tie at 0.5: both kept; zeros never spawn
    want = np.array([[0, 0, 1, 0],
                     [1, 0, 0, 0],
                     [0, 0, 0, 1],
                     [1, 0, 0, 1]], bool)
    assert np.array_equal(ip.nms3(p), want)


def test_unprojection_round_trip_and_quantisation():
    """Spawned points project back to their pixel centres at their depth; a hand-worked
    point lands in level 0 (distance below 10 m, voxel 0.1) at floor(x / 0.1)."""
    R = np.array([[0.0, 0.0, -1.0], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0]])   # camera looks along world -x
    t = np.array([1.0, -2.0, 0.5])
    cam = scenes.make_camera(R, t, 100.0, 110.0, 20.0, 15.0, 40, 30)
    rng = np.random.default_rng(3)
    col = rng.uniform(size=(3, 30, 40))
    dep = rng.uniform(3, 600, size=(30, 40))
    out = ip.spawn_candidates(col, dep, cam, np.zeros((30, 40)))
    assert len(out["pixel"]) > 5
    Rf, tf = cam["R"].reshape(3, 3).astype(np.float64), cam["t"].astype(np.float64)
    xc = out["point"] @ Rf.T + tf
    ys, xs = out["pixel"] // 40, out["pixel"] % 40
    assert np.allclose(xc[:, 2], dep[ys, xs], rtol=1e-12)
    assert np.allclose(100.0 * xc[:, 0] / xc[:, 2] + 20.0, xs + 0.5, atol=1e-9)
    assert np.allclose(110.0 * xc[:, 1] / xc[:, 2] + 15.0, ys + 0.5, atol=1e-9)
    centre = -Rf.T @ tf
    dist = np.linalg.norm(out["point"] - centre, axis=1)
    for d, l in zip(dist, out["level"]):
        lo = 0.0 if l == 0 else ip.DMAX[l - 1]
        assert lo <= d < ip.DMAX[l]
    eps = np.array(ip.EPS)[out["level"]]
    assert np.array_equal(out["voxel"], np.floor(out["point"] / eps[:, None]).astype(np.int64))
    # hand-worked: (0.37, -1.26, 8.05) at 8.2 m from the origin -> level 0, voxel (3, -13, 80)
    assert ip.level_of(8.2) == 0 and ip.level_of(10.0) == 1 and ip.level_of(99.9) == 2 and ip.level_of(1e4) == 4
    assert [math.floor(v / 0.1) for v in (0.37, -1.26, 8.05)] == [3, -13, 80]
