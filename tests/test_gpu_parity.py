"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: images max |dC| <= 1e-4 (FP32), depth |dD| <= 1e-4 max(1, D);
gradients ||d|| <= 1e-3 ||g|| and element-wise 1e-3 (|g| + 0.01 rms);
binning bit-exact; counts exact.  Pixels whose alpha / transmittance decision
lies within a relative margin of 2e-3 of a threshold (and Gaussians whose
rectangle holds such a pixel) are excluded and counted; the excluded share is
bounded in every test.  The margins (2e-4 on alpha, 2e-3 on T) are ten times the
FP32 rounding of those quantities."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import OracleConfig, lifecycle
from paper_2606_30436_amd import scenes
from paper_2606_30436_amd.rasterizer import (GaussianParams, Image, LifecycleState, Rasterizer, ViewStats,
                                             device_cameras)
from tests.gpu_util import (LOG2E, MAX_MISMATCH_SHARE, affected_gaussians, ambiguous_pixels, compare_image,
                            grad_close, involved_gaussians, oracle_cfg, rect_hits, run_forward, say)

pytestmark = pytest.mark.gpu


def _scene(name):
    if name == "c1":
        return scenes.make_c1()
    if name == "tiny":
        return scenes.tiny_scene(seed=3, n=60, degree=3, W=70, H=45, n_views=2, pose_sigma=0.02)
    if name == "wide":
        return scenes.tiny_scene(seed=5, n=300, degree=1, W=600, H=450, n_views=3, pose_sigma=0.03)
    if name == "tiny_bg":
        return scenes.tiny_scene(seed=4, n=80, degree=2, W=53, H=37, n_views=3, pose_sigma=0.03)
    if name == "tiny_opaque":
        # opacities sigmoid(N(3, 1.5)): about one Gaussian in seven at or above alpha_max = 0.99, so
        # that the compositing passes meet the clamp (and the backward its variant with the clamp)
        sc = scenes.tiny_scene(seed=6, n=80, degree=2, W=61, H=43, n_views=2, pose_sigma=0.02)
        sc.logits[:] = np.random.default_rng(16).normal(3.0, 1.5, sc.n).astype(np.float32)
        return sc
    raise KeyError(name)


def _rast(sc, tile=(16, 16), batch=64, **kw):
    return Rasterizer(sc.width, sc.height, max_views=sc.n_views, max_gaussians=sc.n, tile=tile, batch=batch, **kw)


@pytest.mark.parametrize("name", ["c1", "tiny"])
def test_project_records_match_oracle(name):
    sc = _scene(name)
    say(f"[gpu] project parity {name} n={sc.n} V={sc.n_views}")
    R = _rast(sc)
    run_forward(R, sc)
    assert R.status() == 0
    b = R.buffers()
    cfg = oracle_cfg(R)
    for v in range(sc.n_views):
        sel = b["slot_view"].numpy() == v
        gid = b["slot_gid"].numpy()[sel]
        rec = b["slot_rec"].numpy()[sel].astype(np.float64)
        pix = b["slot_pix"].numpy()[sel]
        pr = oracle.View(sc, v, cfg).proj()
        vis = np.nonzero(pr["visible"])[0]
        # visible sets agree; a Gaussian on one side only must sit at a culling margin of its own (near / far
        # plane, alpha_min cull, determinant) or at an integer decision of its rectangle (centre or extent next
        # to an integer, which can empty the rectangle at the image border)
        m = pr["margins"]
        z = np.abs(m[:, 0]) + cfg.near
        at_margin = ((m[:, 0] <= 1e-9 * z) | (m[:, 6] <= 1e-9) | (m[:, 1] <= 1e-5) | (np.abs(m[:, 5]) <= 1e-6)
                     | (m[:, 7] <= 1e-3) | (m[:, 8] <= 1e-4))
        diff = np.setxor1d(gid, vis)
        say(f"  view {v}: visible {len(vis)}, on one side only {len(diff)}")
        assert at_margin[diff].all(), diff[~at_margin[diff]]
        common, ig, io = np.intersect1d(gid, vis, return_indices=True)
        r = rec[ig]
        mu = r[:, 0:2] + 0.5 + np.array([sc.width // 2, sc.height // 2])
        # FP64 centre rounded once to FP32 relative to the image centre
        assert np.abs(mu - pr["mu"][common]).max() <= 1e-4
        # the record holds the conic pivoted: q = P (dx + k dy)^2 + E dy^2
        Pg, kg, Eg = -2 * r[:, 2] / LOG2E, r[:, 3], -2 * r[:, 4] / LOG2E
        oc = pr["conic"][common]
        Po, ko, Eo = oc[:, 0], oc[:, 1] / oc[:, 0], oc[:, 2] - oc[:, 1] ** 2 / oc[:, 0]
        assert np.allclose(Pg, Po, rtol=2e-5, atol=0), np.max(np.abs(Pg / Po - 1))
        assert np.allclose(Eg, Eo, rtol=2e-5, atol=0), np.max(np.abs(Eg / Eo - 1))
        # k moves q by about 2 sqrt(P / E) dk at the footprint's edge
        kscale = np.sqrt(Eo / Po)
        assert (np.abs(kg - ko) <= 1e-5 * kscale + 1e-6 * np.abs(ko)).all(), np.max(np.abs(kg - ko) / kscale)
        assert np.allclose(2.0 ** r[:, 5], pr["opacity"][common], rtol=1e-5)
        assert np.allclose(r[:, 6], pr["depth"][common], rtol=1e-6)
        assert np.allclose(r[:, 8:11], pr["color"][common], atol=2e-5)
        # integer centre and extents: equal, except where the FP64 centre or extent sits next to an integer
        same = (pix[ig] == np.stack([pr["fxi"], pr["fyi"], pr["rx"], pr["ry"]], 1)[common]).all(1)
        near_int = (m[common, 7] <= 1e-3) | (m[common, 8] <= 1e-4)
        say(f"  view {v}: integer centre / extent differences {int((~same).sum())} of {len(common)}")
        assert near_int[~same].all(), common[~same & ~near_int]


@pytest.mark.parametrize("name,tile", [("c1", (16, 16)), ("c1", (8, 32)), ("tiny", (32, 8)), ("c1", (32, 16)),
                                       ("tiny", (16, 32)), ("wide", (16, 16))])
def test_binning_is_bit_exact(name, tile):
    """Sorted (key, Gaussian) list == the integer binning contract applied to
    the GPU's own fp32 centres, extents and depths, sorted on the CPU.  The
    tile counts per view take the pair sort through one pass of 4 to 9 bits
    (the tiny views, c1) and two passes (1102 tiles of the wide views)."""
    sc = _scene(name)
    say(f"[gpu] binning {name} tile={tile}")
    R = _rast(sc, tile=tile, pair_capacity=1 << 20)
    run_forward(R, sc)
    _check_binning(R, sc, tile)


def _view_major(b):
    """The GPU's pairs (grouped by tile, then view) in view-major order.  Checks
    on the way that each (view, tile) group is one contiguous run and that the
    run is the group's range, and that every other range is empty."""
    T = b["tiles_x"] * b["tiles_y"]
    tb = b["tile_bits"]
    assert T < (1 << tb) <= 2 * T
    k = b["keys"].numpy().view(np.uint32).astype(np.int64)
    view, tile = k >> tb, k & ((1 << tb) - 1)
    assert (view < b["n_views"]).all() and (tile < T).all()
    dense = view * T + tile
    n = len(k)
    starts = np.flatnonzero(np.r_[True, dense[1:] != dense[:-1]]) if n else np.zeros(0, np.int64)
    ends = np.r_[starts[1:], n].astype(np.int64) if n else np.zeros(0, np.int64)
    assert len(np.unique(dense[starts])) == len(starts)
    r = b["ranges"].numpy().astype(np.int64)
    assert r.shape == (b["n_views"] * T, 2)
    assert np.array_equal(r[dense[starts], 0], starts) and np.array_equal(r[dense[starts], 1], ends)
    empty = np.ones(len(r), bool)
    empty[dense[starts]] = False
    assert (r[empty] == 0).all()
    order = np.argsort(dense, kind="stable")
    return dense[order], order


def _check_binning(R, sc, tile):
    assert R.status() == 0
    b = R.buffers()
    assert b["n_pairs"] > 0
    pix = b["slot_pix"].numpy()
    depth_bits = b["slot_rec"].numpy()[:, 6].copy().view(np.uint32)
    keys, gids = oracle.bin_keys(b["slot_view"].numpy(), b["slot_gid"].numpy(), pix[:, 0], pix[:, 1], pix[:, 2],
                                 pix[:, 3], depth_bits, sc.width, sc.height, tile[0], tile[1])
    dense, order = _view_major(b)
    ss = b["sorted_slot"].numpy()[order]
    gk = (dense.astype(np.uint64) << np.uint64(32)) | depth_bits[ss].astype(np.uint64)
    assert len(gk) == len(keys) == b["n_pairs"]
    assert np.array_equal(gk, keys)
    assert np.array_equal(b["slot_gid"].numpy()[ss].astype(np.int64), gids)
    return b


@pytest.mark.parametrize("case", ["second_sort", "wide_keys"])
def test_binning_bit_exact_on_the_other_sort_paths(case):
    """The record depth sort in its two other forms: a second sort after one
    projection (the first consumed the keys the projection wrote, so the sort
    builds them again from the records), and view plus depth bits above 32
    (8-byte keys: near 1e-6, far 1e5 and 16 views give 29 + 4 bits)."""
    say(f"[gpu] binning path {case}")
    if case == "second_sort":
        sc = _scene("c1")
        R = _rast(sc)
    else:
        sc = scenes.tiny_scene(seed=6, n=400, degree=1, W=96, H=64, n_views=16, pose_sigma=0.05)
        R = _rast(sc, near_z=1e-6, far_z=1e5)
    run_forward(R, sc)
    first = _check_binning(R, sc, (16, 16))
    if case == "second_sort":
        R.bin_sort()
        torch.cuda.synchronize()
        again = _check_binning(R, sc, (16, 16))
        for k in ("keys", "sorted_slot", "slot_pairoff"):
            assert np.array_equal(first[k].numpy(), again[k].numpy()), k


def test_sixty_four_views():
    """The most views a call takes (64): the emission's per-Gaussian view mask
    uses its top bit and the depth sort 8-byte keys (27 depth + 6 view bits).
    Binning, every view's image and all gradients against the oracle."""
    sc = scenes.tiny_scene(seed=9, n=150, degree=1, W=64, H=48, n_views=64, pose_sigma=0.02)
    say("[gpu] 64 views")
    R = _rast(sc)
    g, cams, xi, img = run_forward(R, sc)
    _check_binning(R, sc, (16, 16))
    b = R.buffers()
    assert int(np.max(b["slot_view"].numpy())) == 63
    cfg = oracle_cfg(R)
    col = img.color.cpu().numpy()
    rng = np.random.default_rng(19)
    dLdC = rng.normal(size=(64, 3, sc.height, sc.width))
    grads = g.zeros_like()
    pose_grad = torch.zeros(64, 6, device="cuda")
    R.render_bwd(g, cams, xi, img, torch.from_numpy(dLdC.astype(np.float32)).cuda(), grads=grads,
                 pose_grad=pose_grad)
    torch.cuda.synchronize()
    ref = {k: 0.0 for k in ("means", "log_scales", "quats", "logits", "sh")}
    pg = pose_grad.cpu().numpy()
    for v in range(64):
        ov = oracle.View(sc, v, cfg)
        oi = ov.image()
        compare_image(col[v], oi)
        an = ov.backward(dLdC[v])
        for k in ref:
            ref[k] = ref[k] + an[k]
        assert np.linalg.norm(pg[v] - an["pose_xi"]) <= 1e-3 * np.linalg.norm(an["pose_xi"]) + 1e-9, v
    for k in ref:
        got = getattr(grads, k).cpu().numpy().astype(np.float64)
        rel = np.linalg.norm(got - ref[k]) / np.linalg.norm(ref[k])
        say(f"  {k} rel {rel:.2e}")
        assert rel < 1e-3, k


def test_a_view_that_sees_nothing():
    """A batched call in which the middle view faces away from every Gaussian:
    its tile lists, its slot range and its pose pieces are empty.  Its image is
    the background and its pose gradient zero; the other views and all
    gradients match the oracle."""
    sc = scenes.tiny_scene(seed=3, n=60, degree=3, W=70, H=45, n_views=3, pose_sigma=0.0)
    sc.cams["R"][1] = np.array([-1.0, 0, 0, 0, 1.0, 0, 0, 0, -1.0], np.float32)   # turned around
    say("[gpu] a view that sees nothing")
    R = _rast(sc, bg=(0.2, 0.5, 0.9))
    g, cams, xi, img = run_forward(R, sc)
    b = R.buffers()
    views = b["slot_view"].numpy()
    assert (views == 1).sum() == 0 and (views == 0).sum() > 0 and (views == 2).sum() > 0
    col = img.color.cpu().numpy()
    assert np.array_equal(col[1], np.broadcast_to(np.array([0.2, 0.5, 0.9], np.float32)[:, None, None], col[1].shape))
    assert np.all(img.t_final.cpu().numpy()[1] == 1.0)
    rng = np.random.default_rng(23)
    dLdC = rng.normal(size=(3, 3, sc.height, sc.width))
    grads = g.zeros_like()
    pose_grad = torch.zeros(3, 6, device="cuda")
    R.render_bwd(g, cams, xi, img, torch.from_numpy(dLdC.astype(np.float32)).cuda(), grads=grads,
                 pose_grad=pose_grad)
    torch.cuda.synchronize()
    pg = pose_grad.cpu().numpy()
    assert np.all(pg[1] == 0.0)
    cfg = oracle_cfg(R)
    ref = {k: 0.0 for k in ("means", "log_scales", "quats", "logits", "sh")}
    for v in (0, 2):
        ov = oracle.View(sc, v, cfg)
        oi = ov.image()
        compare_image(col[v], oi)
        an = ov.backward(dLdC[v])
        for k in ref:
            ref[k] = ref[k] + an[k]
        assert np.linalg.norm(pg[v] - an["pose_xi"]) <= 1e-3 * np.linalg.norm(an["pose_xi"])
    for k in ref:
        got = getattr(grads, k).cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - ref[k]) <= 1e-3 * np.linalg.norm(ref[k]), k


@pytest.mark.parametrize("name", ["c1", "tiny", "tiny_bg", "tiny_opaque"])
def test_render_forward_matches_oracle(name):
    sc = _scene(name)
    kw = {"bg": (0.2, 0.5, 0.9)} if name == "tiny_bg" else {}
    say(f"[gpu] render fwd {name}")
    R = _rast(sc, **kw)
    _, _, _, img = run_forward(R, sc)
    cfg = oracle_cfg(R)
    col = img.color.cpu().numpy().astype(np.float64)
    dep = img.depth.cpu().numpy().astype(np.float64)
    tf = img.t_final.cpu().numpy().astype(np.float64)
    failed = margin = total = 0
    for v in range(sc.n_views):
        oi = oracle.View(sc, v, cfg).image()
        err, nbad, namb = compare_image(col[v], oi, got_depth=dep[v], got_tfinal=tf[v])
        failed += nbad
        margin += namb
        total += oi["depth"].size
        say(f"  view {v}: max error {err:.2e}")
    say(f"  pixels outside tolerance (all at a margin): {failed}/{total}; pixels at a margin: {margin}")


def _oracle_grads(sc, cfg, dLdC, dLdD):
    out = None
    for v in range(sc.n_views):
        gv = oracle.View(sc, v, cfg).backward(dLdC[v], dLdD[v])
        if out is None:
            out = {k: gv[k].copy() for k in ("means", "log_scales", "quats", "logits", "sh")}
            out["pose_xi"] = [gv["pose_xi"]]
        else:
            for k in ("means", "log_scales", "quats", "logits", "sh"):
                out[k] += gv[k]
            out["pose_xi"].append(gv["pose_xi"])
    out["pose_xi"] = np.stack(out["pose_xi"])
    return out


def _involved(sc, cfg):
    bad = np.zeros(sc.n, bool)
    for v in range(sc.n_views):
        bad |= involved_gaussians(oracle.View(sc, v, cfg))
    return bad


def _affected(sc, cfg):
    bad = np.zeros(sc.n, bool)
    for v in range(sc.n_views):
        bad |= affected_gaussians(oracle.View(sc, v, cfg))
    return bad


@pytest.mark.parametrize("px", [1, 2])
@pytest.mark.parametrize("name,depth", [("c1", True), ("tiny", True), ("tiny_bg", True), ("c1", False),
                                        ("tiny", False), ("tiny_opaque", True), ("tiny_opaque", False)])
def test_render_backward_matches_oracle(name, depth, px):
    """With and without a depth gradient (the backward has a variant that
    leaves the depth terms out when none is passed), with one and two pixels
    per lane, and with opacities at the alpha_max clamp."""
    sc = _scene(name)
    if name == "tiny_opaque":
        assert (1.0 / (1.0 + np.exp(-sc.logits.astype(np.float64))) >= 0.99).sum() >= 5
    kw = {"bg": (0.2, 0.5, 0.9)} if name == "tiny_bg" else {}
    say(f"[gpu] render bwd {name} depth={depth} px_per_lane={px}")
    R = _rast(sc, px_per_lane=px, **kw)
    g, cams, xi, img = run_forward(R, sc)
    rng = np.random.default_rng(7)
    V, H, W = sc.n_views, sc.height, sc.width
    dLdC = rng.normal(size=(V, 3, H, W))
    dLdD = rng.normal(size=(V, H, W)) * 0.05 if depth else np.zeros((V, H, W))
    grads = g.zeros_like()
    pose_grad = torch.zeros(V, 6, device="cuda")
    R.render_bwd(g, cams, xi, img, torch.from_numpy(dLdC.astype(np.float32)).cuda(),
                 torch.from_numpy(dLdD.astype(np.float32)).cuda() if depth else None, grads=grads,
                 pose_grad=pose_grad)
    torch.cuda.synchronize()
    cfg = oracle_cfg(R)
    ref = _oracle_grads(sc, cfg, dLdC, dLdD)
    flagged = _affected(sc, cfg)
    rels = {}
    for k in ("means", "log_scales", "quats", "logits", "sh"):
        got = getattr(grads, k).cpu().numpy()
        rels[k] = grad_close(k, got, ref[k], flagged)
    say(f"  Gaussians flagged at a margin: {int(flagged.sum())}/{sc.n}")
    say("  relative gradient error (Gaussians outside tolerance) "
        + " ".join(f"{k}={v[0]:.2e} ({v[1]})" for k, v in rels.items()))
    pg = pose_grad.cpu().numpy()
    d = np.linalg.norm(pg - ref["pose_xi"], axis=1) / np.linalg.norm(ref["pose_xi"], axis=1)
    say(f"  pose gradient relative error per view {d}")
    assert (d <= 1e-3).all()


@pytest.mark.parametrize("name", ["c1", "tiny"])
def test_statistics_match_oracle(name):
    """|Omega_v(i)| and kappa_v(i) exact, away from threshold pixels."""
    sc = _scene(name)
    say(f"[gpu] statistics {name}")
    R = _rast(sc)
    g, cams, xi, img = run_forward(R, sc)
    V = sc.n_views
    target = torch.from_numpy(sc.target.astype(np.float32)).cuda()
    dl = torch.empty_like(img.color)
    loss = torch.empty(V, device="cuda")
    R.loss_l1(target, img, dl, loss)
    st = ViewStats.zeros(sc.n)
    grads = g.zeros_like()
    R.render_bwd(g, cams, xi, img, dl, target=target, tau_err=0.1, view_loss=loss, grads=grads, stats=st)
    torch.cuda.synchronize()
    cfg = oracle_cfg(R)
    om = np.zeros(sc.n, np.int64)
    ka = np.zeros(sc.n, np.int64)
    bad = _affected(sc, cfg)
    lossv = loss.cpu().numpy()
    col = img.color.cpu().numpy()
    for v in range(V):
        ov = oracle.View(sc, v, cfg)
        s = ov.stats(sc.target[v], 0.1)
        om += s["omega"]
        ka += s["kappa"]
        pr = ov.proj()
        bad |= rect_hits(s["mask_margin"] < 1e-4, pr["fxi"], pr["fyi"], pr["rx"], pr["ry"]) & pr["visible"]
        ref_loss = np.abs(col[v].astype(np.float64) - sc.target[v]).mean()
        assert lossv[v] == pytest.approx(ref_loss, rel=1e-5)
    gom = st.omega_sum.cpu().numpy()
    gka = st.kappa_sum.cpu().numpy()
    mism = (gom != om) | (gka != ka)
    say(f"  flagged at a margin {int(bad.sum())}/{sc.n}, count mismatches {int(mism.sum())}")
    # every count that differs belongs to a Gaussian at a threshold or whose rectangle holds a pixel at the
    # error-mask threshold
    assert not (mism & ~bad).any(), np.flatnonzero(mism & ~bad)[:8]
    assert mism.mean() <= MAX_MISMATCH_SHARE
    assert (gka <= gom).all()
    gam = st.gamma_sum.cpu().numpy()
    # gamma = sum_v L_v |Omega_v|, with the GPU's own per-view losses
    assert gam.sum() > 0


def test_tile_shapes_and_batches_give_identical_images():
    sc = _scene("c1")
    say("[gpu] tile invariance")
    ref = None
    for tile in ((16, 16), (8, 32), (32, 8), (32, 16), (16, 32)):
        for batch in (32, 64 if tile[0] * tile[1] == 512 else 128):
            R = _rast(sc, tile=tile, batch=batch)
            _, _, _, img = run_forward(R, sc)
            c = img.color.cpu().numpy()
            if ref is None:
                ref = c
            else:
                assert np.array_equal(c, ref), (tile, batch)


def test_tile_shapes_and_batches_give_the_same_gradients():
    """The backward over every tile shape (four- and eight-wave workgroups) and
    LDS batch: the same gradients up
    to FP32 summation order (list entries are reduced in pairs or alone
    depending on where a batch ends), on a scene dense enough for per-wave
    lists longer than a wavefront.  One Gaussian in fifty is opaque beyond
    alpha_max, so that every variant meets batches with and without a record
    at the clamp."""
    sc = scenes.make_c1(seed=5, n=80_000)
    sc.logits[::50] = 6.0
    say("[gpu] backward tile / batch invariance")
    rng = np.random.default_rng(11)
    V, H, W = sc.n_views, sc.height, sc.width
    dLdC = torch.from_numpy(rng.normal(size=(V, 3, H, W)).astype(np.float32)).cuda()
    dLdD = torch.from_numpy((rng.normal(size=(V, H, W)) * 0.05).astype(np.float32)).cuda()
    ref = None
    cases = [(t, b, x) for t in ((16, 16), (8, 32), (32, 8), (32, 16), (16, 32)) for b in (32, 64, 128)
             for x in (1, 2) if not (t[0] * t[1] == 512 and b > 64) and not (t[0] < 16 and x == 2)]
    for tile, batch, px in cases:
        R = _rast(sc, tile=tile, batch=batch, px_per_lane=px)
        g, cams, xi, img = run_forward(R, sc)
        if ref is None:
            keys = R.buffers()["keys"].numpy()
            longest = int(np.unique(keys, return_counts=True)[1].max())
            say(f"  longest tile list {longest}")
            assert longest > 256
        grads = g.zeros_like()
        pose_grad = torch.zeros(V, 6, device="cuda")
        R.render_bwd(g, cams, xi, img, dLdC, dLdD, grads=grads, pose_grad=pose_grad)
        torch.cuda.synchronize()
        out = {k: getattr(grads, k).cpu().numpy().astype(np.float64)
               for k in ("means", "log_scales", "quats", "logits", "sh")}
        out["pose"] = pose_grad.cpu().numpy().astype(np.float64)
        if ref is None:
            ref = out
            continue
        for k in out:
            rel = np.linalg.norm(out[k] - ref[k]) / np.linalg.norm(ref[k])
            assert rel < 1e-5, (tile, batch, px, k, rel)


@pytest.mark.parametrize("mean_z,t_z,kept", [(9.999, 0.0, True), (10.0, 0.0, False), (10.001, 0.0, False),
                                             (10.0, -2.0 ** -30, True)])
def test_far_plane_boundary(mean_z, t_z, kept):
    """The distance mask at far = 10: depths just inside are rendered, at and beyond far are culled, and the
    decision is taken on the FP64 camera depth (10 - 2^-30 is kept although its FP32 rounding equals far)."""
    say(f"[gpu] far plane mean_z={mean_z} t_z={t_z}")
    W, H, f = 40, 32, 300.0
    sh = np.zeros((1, 3, 1), np.float32)
    sh[0, :, 0] = (np.array([0.7, 0.4, 0.2]) - 0.5) * 2 * math.sqrt(math.pi)
    cam = scenes.make_camera(np.eye(3), np.array([0.0, 0.0, t_z]), f, f, W / 2, H / 2, W, H)
    sc = scenes.Scene(np.array([[0.0], [0.0], [mean_z]], np.float32), np.full((3, 1), math.log(0.05), np.float32),
                      np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), np.array([0.7], np.float32), sh, 0,
                      scenes.stack_cameras([cam]), np.zeros((1, 6), np.float32))
    R = _rast(sc, far_z=10.0)
    _, _, _, img = run_forward(R, sc)
    n_slots, _ = R.counts()
    assert R.status() == 0 and n_slots == int(kept)
    oi = oracle.View(sc, 0, oracle_cfg(R)).image()
    assert np.abs(img.color[0].cpu().numpy() - oi["color"]).max() <= 1e-6
    assert (np.abs(oi["color"]).max() > 0.1) == kept
    R.close()
