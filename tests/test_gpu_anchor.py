"""Anchors on the GPU (kgs_anchor_decode, kgs_anchor_stats, through the C ABI)
against the FP64 oracle of the appendix's anchor decoding with its
level-of-detail mask, and of the per-anchor footprint statistics (the union of
the pixels of an anchor's Gaussians).

Decoding runs on the matrix cores with FP32 accumulation; an anchor is flagged
when one of its hidden units lies, in the oracle, within the FP32 accumulation
bound (48 2^-24 times the sum of the magnitudes it adds) of the ReLU kink or of
a BF16 rounding boundary -- there the BF16 operand of the second product may
differ by one unit.  Every other anchor's children must match to 1e-4
(relative, 1e-6 of the map's coordinates for the means) plus the FP32
accumulation bound of the second product carried through each output, and the
level-of-detail mask exactly.  Footprint counts are exact except for anchors with a
Gaussian at a threshold (as for the per-Gaussian statistics)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import anchors as an
from paper_2606_30436_amd import scenes
from paper_2606_30436_amd.mapping import Anchors, anchor_stats, decode_anchors
from paper_2606_30436_amd.rasterizer import GaussianParams, Image, Rasterizer, ViewStats, device_cameras
from tests.gpu_util import MAX_MISMATCH_SHARE, affected_gaussians, oracle_cfg, rect_hits, say

pytestmark = pytest.mark.gpu

FP32_ACC = 48 * 2.0 ** -24


def _flag_hidden(o):
    """Anchors whose hidden units the FP32 accumulation may round to another BF16 value or ReLU side."""
    z1, bound = o["z1"], FP32_ACC * o["z1_abs"]
    kink = np.abs(z1) <= bound
    h = np.maximum(z1, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.floor(np.log2(np.where(h > 0, h, 1.0)))
        ulp = np.exp2(e - 7)
        r = h / ulp - np.floor(h / ulp)
        dist = np.abs(r - 0.5) * ulp
    tie = (h > 0) & (dist <= bound)
    return (kink | tie).any(axis=1)


def _outside_tolerance(got, o, log_l, A, K):
    """Children whose outputs differ from the oracle's by more than 1e-4 relative (1e-6 of the coordinates
    for the means) plus what the FP32 accumulation of the second product may move each raw output (FP32_ACC
    times the sum of the magnitudes it adds), carried through each output's function: slope at most 1 for
    the rotation, the SH coefficient (sigmoid' / Y_00 < 1) and the log-scale (1 - sigmoid), the local scale for
    the means, and 2 / (1 - e^{-2y}) for the opacity logit ln((e^{2y} - 1) / 2)."""
    n = A * K
    tol_y = (FP32_ACC * o["y_abs"]).reshape(n, 14).T                      # [14][AK]
    y = o["raw"].reshape(n, 14).T
    l = np.repeat(np.exp(log_l.astype(np.float64)), K, axis=1)           # [3][AK]
    bad = np.zeros(n, bool)
    bad |= (np.abs(got["means"] - o["means"]) >
            1e-6 * np.maximum(1, np.abs(o["means"])) + l * (1e-4 + tol_y[11:14])).any(0)
    bad |= (np.abs(got["log_scales"] - o["log_scales"]) > 1e-4 * (1 + np.abs(o["log_scales"])) + tol_y[8:11]).any(0)
    bad |= (np.abs(got["quats"] - o["quats"]) > 1e-4 * (1 + np.abs(o["quats"])) + tol_y[4:8]).any(0)
    bad |= (np.abs(got["sh"][0] - o["sh"][0]) > 1e-4 * (1 + np.abs(o["sh"][0])) + tol_y[1:4]).any(0)
    live = o["logits"] > -100.0
    with np.errstate(divide="ignore", over="ignore"):
        slope = np.where(live, 2.0 / -np.expm1(-2.0 * np.maximum(y[0], 1e-300)), 0.0)
    bad |= np.abs(got["logits"] - o["logits"]) > 1e-4 * (1 + np.abs(o["logits"])) + slope * tol_y[0]
    return bad


def _decoded(anc_dev, theta, cams_dev, v, n):
    out = GaussianParams(torch.full((3, n), np.nan, device="cuda"), torch.full((3, n), np.nan, device="cuda"),
                         torch.full((4, n), np.nan, device="cuda"), torch.full((n,), np.nan, device="cuda"),
                         torch.full((1, 3, n), np.nan, device="cuda"), 0)
    decode_anchors(anc_dev, theta, cams_dev[v], out)
    return out


def _centre(cam):
    R = cam["R"].reshape(3, 3).astype(np.float64)
    return -R.T @ cam["t"].astype(np.float64)


@pytest.mark.parametrize("A,K,alpha_bias", [(3001, 10, 0.0), (16, 3, 0.0), (1, 16, 0.0), (40_000, 10, 0.0),
                                             (2000, 4, 1.0)])
def test_anchor_decode_matches_oracle(A, K, alpha_bias):
    """alpha_bias: opacity output biases spread over [0, 40 alpha_bias) -- tanh saturates in FP32 from about 9 and
    in FP64 from about 19, where the logit must come from the raw output."""
    sc = scenes.make_anchor_scene(seed=A + K, n_anchors=A, k=K, n_views=2)
    if alpha_bias:
        n_w = 32 * 36 + 32 + 14 * K * 32
        sc["theta"][n_w::14] += np.linspace(0.0, 40.0 * alpha_bias, K, endpoint=False).astype(np.float32)
    say(f"[gpu] anchor decode A={A} K={K} alpha_bias={alpha_bias}")
    anc = dict(p=sc["p"], f=sc["feat"], log_l=sc["log_l"], O=sc["offsets"], level=sc["level"])
    dev = Anchors.from_arrays(sc["p"], sc["feat"], sc["log_l"], sc["offsets"], sc["level"])
    theta = torch.from_numpy(sc["theta"]).cuda()
    cams = device_cameras(sc["cams"]).view(len(sc["cams"]), -1)   # one 72-byte record per row
    for v in range(2):
        g = _decoded(dev, theta, cams, v, A * K)
        torch.cuda.synchronize()
        o = an.decode(anc, sc["theta"], K, _centre(sc["cams"][v]))
        flagged = np.repeat(_flag_hidden(o), K)
        got = dict(means=g.means.cpu().numpy(), log_scales=g.log_scales.cpu().numpy(), quats=g.quats.cpu().numpy(),
                   logits=g.logits.cpu().numpy(), sh=g.sh.cpu().numpy())
        for k in got:
            assert np.isfinite(got[k]).all(), k
        masked = o["alpha_masked"].reshape(-1) <= 0
        assert np.array_equal(got["logits"][masked], np.full(masked.sum(), -100.0, np.float32))
        bad = _outside_tolerance(got, o, sc["log_l"], A, K)
        say(f"  view {v}: children outside tolerance {int(bad.sum())} (flagged {int(flagged.sum())}), "
            f"masked by the level of detail {int(masked.sum())}")
        assert not (bad & ~flagged).any(), np.flatnonzero(bad & ~flagged)[:8]


def _grouped_scene(seed):
    """Explicit Gaussians in groups of three around common centres (an anchor's children overlap), shuffled so
    that an anchor's Gaussians are not consecutive; 2 views."""
    sc = scenes.tiny_scene(seed=seed, n=120, degree=1, W=70, H=45, n_views=2, pose_sigma=0.02, log_scale_mu=-1.7)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(sc.n)
    anchor_of = np.empty(sc.n, np.int64)
    anchor_of[perm] = np.arange(sc.n) // 3
    centres = sc.means[:, perm[::3]]
    sc.means = (centres[:, anchor_of] + rng.normal(0, 0.05, sc.means.shape)).astype(np.float32)
    return sc, anchor_of, sc.n // 3


@pytest.mark.parametrize("tile", [(16, 16), (32, 16)])
def test_anchor_footprints_match_oracle(tile):
    sc, anchor_of, A = _grouped_scene(7)
    V, H, W = sc.n_views, sc.height, sc.width
    say(f"[gpu] anchor footprints tile={tile} A={A}")
    R = Rasterizer(W, H, max_views=V, max_gaussians=sc.n, tile=tile)
    g = GaussianParams.from_scene(sc)
    cams = device_cameras(sc.cams)
    xi = torch.from_numpy(sc.pose_xi).cuda()
    R.project(g, cams, xi)
    R.bin_sort()
    img = Image.empty(V, H, W)
    R.render_fwd(img)
    target = torch.from_numpy(sc.target).cuda()
    loss = torch.tensor([0.25, 0.5], device="cuda")
    st = ViewStats.zeros(A)
    counts = torch.zeros(2 * V * A, dtype=torch.int32, device="cuda")
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    a_of = torch.from_numpy(anchor_of.astype(np.int32)).cuda()
    anchor_stats(R, img, a_of, A, target, loss, counts, st, status)
    torch.cuda.synchronize()
    assert int(status[0].item()) == 0
    cfg = oracle_cfg(R)
    om, ka = np.zeros(A, np.int64), np.zeros(A, np.int64)
    gam = np.zeros(A)
    flagged = np.zeros(A, bool)
    for v in range(V):
        ov = oracle.View(sc, v, cfg)
        s = ov.anchor_stats(anchor_of, A, sc.target[v], 0.1)
        om += s["omega"]
        ka += s["kappa"]
        gam += loss[v].item() * s["omega"]
        pr = ov.proj()
        bad_g = affected_gaussians(ov) | (rect_hits(ov.stats(sc.target[v], 0.1)["mask_margin"] < 1e-4, pr["fxi"],
                                                    pr["fyi"], pr["rx"], pr["ry"]) & pr["visible"])
        flagged[np.unique(anchor_of[bad_g])] = True
    gom, gka = st.omega_sum.cpu().numpy(), st.kappa_sum.cpu().numpy()
    mism = (gom != om) | (gka != ka)
    say(f"  anchors with a footprint {int((om > 0).sum())}/{A}; mismatches {int(mism.sum())} "
        f"(flagged {int(flagged.sum())})")
    assert not (mism & ~flagged).any(), np.flatnonzero(mism & ~flagged)[:8]
    ok = ~mism
    assert np.allclose(st.gamma_sum.cpu().numpy()[ok], gam[ok], rtol=1e-6, atol=0)


def test_anchor_footprints_with_table_overflow():
    """1500 faint Gaussians (opacity about 0.01) stacked over a 24x16 image, each its own anchor: every
    8x8 sub-block meets more distinct anchors than its table holds, so it is walked again for parts of the
    anchors (split by hash bits).  The counts must still equal the oracle's union statistics."""
    sc = scenes.tiny_scene(seed=19, n=1500, W=24, H=16, degree=0, depth=(3.0, 5.0), log_scale_mu=-0.5,
                           log_scale_sigma=0.1, spread=0.2)
    sc.logits = np.random.default_rng(20).normal(-4.6, 0.2, sc.n).astype(np.float32)
    A = sc.n
    anchor_of = np.arange(A)
    V, H, W = sc.n_views, sc.height, sc.width
    say(f"[gpu] anchor footprints with table overflow A={A} {W}x{H}")
    R = Rasterizer(W, H, max_views=V, max_gaussians=sc.n, tile=(16, 16))
    g = GaussianParams.from_scene(sc)
    cams = device_cameras(sc.cams)
    R.project(g, cams)
    R.bin_sort()
    img = Image.empty(V, H, W)
    R.render_fwd(img)
    target = torch.from_numpy(sc.target).cuda()
    st = ViewStats.zeros(A)
    counts = torch.zeros(2 * V * A, dtype=torch.int32, device="cuda")
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    anchor_stats(R, img, torch.from_numpy(anchor_of.astype(np.int32)).cuda(), A, target, None, counts, st, status)
    torch.cuda.synchronize()
    assert R.status() == 0 and int(status[0].item()) == 0
    assert int(status[1].item()) > 0, "no sub-block overflowed its table"
    ov = oracle.View(sc, 0, oracle_cfg(R))
    s = ov.anchor_stats(anchor_of, A, sc.target[0], 0.1)
    pr = ov.proj()
    bad_g = affected_gaussians(ov) | (rect_hits(ov.stats(sc.target[0], 0.1)["mask_margin"] < 1e-4, pr["fxi"],
                                                pr["fyi"], pr["rx"], pr["ry"]) & pr["visible"])
    gom, gka = st.omega_sum.cpu().numpy(), st.kappa_sum.cpu().numpy()
    mism = (gom != s["omega"]) | (gka != s["kappa"])
    say(f"  re-walks {int(status[1].item())}, anchors with a footprint {int((s['omega'] > 0).sum())}, "
        f"mismatches {int(mism.sum())} (flagged {int(bad_g.sum())})")
    assert (s["omega"] > 0).sum() > 400
    assert not (mism & ~bad_g).any(), np.flatnonzero(mism & ~bad_g)[:8]
    # every Gaussian here shares a pixel with one near a threshold, so the flags exclude nothing: the
    # counts must match outright, up to the flip share allowed elsewhere
    assert mism.mean() <= MAX_MISMATCH_SHARE


def test_anchor_chunk_full_size():
    """200k anchors with 10 children each (2M Gaussians per view) along the 1 km trajectory, the first chunk's
    8 keyframes: per view decode, project, bin + sort, composite, per-anchor footprints, against the oracle's
    decode, rendering and per-anchor footprints of the same view."""
    sc = scenes.make_anchor_scene()
    A, K = len(sc["level"]), sc["k"]
    V, H, W = len(sc["cams"]), sc["height"], sc["width"]
    say(f"[gpu] anchor chunk A={A} K={K} V={V}")
    dev = Anchors.from_arrays(sc["p"], sc["feat"], sc["log_l"], sc["offsets"], sc["level"])
    theta = torch.from_numpy(sc["theta"]).cuda()
    # the target: the same anchors under a slightly different decoder
    theta_t = torch.from_numpy((sc["theta"] * (1 + 0.02 * np.random.default_rng(1).normal(size=sc["theta"].shape)))
                               .astype(np.float32)).cuda()
    cams = device_cameras(sc["cams"]).view(V, -1)   # one 72-byte record per row
    R = Rasterizer(W, H, max_views=1, max_gaussians=A * K, slot_capacity=A * K, pair_capacity=40_000_000,
                   far_z=1e30)
    a_of = torch.arange(A * K, device="cuda", dtype=torch.int32) // K
    st = ViewStats.zeros(A)
    counts = torch.zeros(2 * A, dtype=torch.int32, device="cuda")
    status = torch.zeros(2, dtype=torch.int32, device="cuda")
    anc = dict(p=sc["p"], f=sc["feat"], log_l=sc["log_l"], O=sc["offsets"], level=sc["level"])
    anchor_of = np.arange(A * K) // K
    cfg = oracle_cfg(R)
    mism_total = flagged_total = 0
    for v in range(V):
        tgt_img = Image.empty(1, H, W)
        gt = _decoded(dev, theta_t, cams, v, A * K)
        R.project(gt, cams[v])
        R.bin_sort()
        R.render_fwd(tgt_img)
        g = _decoded(dev, theta, cams, v, A * K)
        R.project(g, cams[v])
        R.bin_sort()
        img = Image.empty(1, H, W)
        R.render_fwd(img)
        one = ViewStats.zeros(A)
        anchor_stats(R, img, a_of, A, tgt_img.color, None, counts, one, status)
        torch.cuda.synchronize()
        assert R.status() == 0 and int(status[0].item()) == 0
        # the oracle decodes and renders the view itself
        o = an.decode(anc, sc["theta"], K, _centre(sc["cams"][v]))
        osc = scenes.Scene(o["means"].astype(np.float32), o["log_scales"].astype(np.float32),
                           o["quats"].astype(np.float32), o["logits"].astype(np.float32),
                           o["sh"].astype(np.float32), 0, sc["cams"][v:v + 1], np.zeros((1, 6), np.float32))
        ov = oracle.View(osc, 0, cfg)
        tgt = tgt_img.color.cpu().numpy()[0]
        s = ov.anchor_stats(anchor_of, A, tgt, 0.1)
        pr = ov.proj()
        amb = np.repeat(_flag_hidden(o), K)
        # anchors near a threshold, anchors decoded ambiguously, and anchors sharing pixels with the latter
        bad_g = affected_gaussians(ov) | (rect_hits(ov.stats(tgt, 0.1)["mask_margin"] < 1e-4, pr["fxi"], pr["fyi"],
                                                    pr["rx"], pr["ry"]) & pr["visible"])
        paint = np.zeros((H, W), bool)
        for gi in np.flatnonzero(amb & pr["visible"]):
            x0, x1 = max(0, pr["fxi"][gi] - pr["rx"][gi]), min(W, pr["fxi"][gi] + pr["rx"][gi] + 1)
            y0, y1 = max(0, pr["fyi"][gi] - pr["ry"][gi]), min(H, pr["fyi"][gi] + pr["ry"][gi] + 1)
            paint[y0:y1, x0:x1] = True
        bad_g |= amb | (rect_hits(paint, pr["fxi"], pr["fyi"], pr["rx"], pr["ry"]) & pr["visible"])
        flagged = np.zeros(A, bool)
        flagged[np.unique(anchor_of[bad_g])] = True
        gom, gka = one.omega_sum.cpu().numpy(), one.kappa_sum.cpu().numpy()
        mism = (gom != s["omega"]) | (gka != s["kappa"])
        say(f"  view {v}: anchors with a footprint {int((s['omega'] > 0).sum())}, mismatches {int(mism.sum())} "
            f"(flagged {int(flagged.sum())}), re-walks {int(status[1].item())}")
        assert not (mism & ~flagged).any(), np.flatnonzero(mism & ~flagged)[:8]
        assert mism.mean() <= MAX_MISMATCH_SHARE
        mism_total += int(mism.sum())
        flagged_total += int(flagged.sum())
        del ov
    say(f"  mismatches over the chunk {mism_total} (all flagged)")
