"""Pins of the anchor-decoding oracle (appendix "Voxelized Representation and
MLP Decoding", "Level-of-Detail (LoD) Mask Computation") and of the per-anchor
footprint statistics (appendix "Densification Score" / "Pruning Score": an
anchor's footprint is the union of its Gaussians' pixels), against closed
forms, explicit loops and brute force.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import OracleConfig
from oracle import anchors as an
from paper_2606_30436_amd import scenes


def _anchors(rng, A, K, spread=5.0):
    p = rng.normal(size=(3, A)) * spread + np.array([[0.0], [0.0], [12.0]])
    return dict(p=p, f=rng.normal(size=(A, 32)), log_l=rng.normal(-2.0, 0.3, (3, A)),
                O=rng.normal(size=(K, 3, A)), level=rng.integers(0, 3, A))


def test_composition_closed_form():
    """W2 = 0: every child's outputs are b2.  alpha = tanh(atanh(0.5)) = 0.5, colour sigmoid(0) = 0.5,
    ds = sigmoid(0) = 0.5 so s = l / 2, x = p + (O + dO) l, and inside its band alpha~ = alpha."""
    rng = np.random.default_rng(0)
    K, A = 3, 5
    anc = _anchors(rng, A, K)
    anc["level"] = np.full(A, 2)                       # band [25, 100): distances about 12 m are outside ...
    anc["p"][2] += 30.0                                # ... so move the anchors to ~42 m
    W1 = rng.normal(size=(32, 36))
    b1 = rng.normal(size=32)
    W2 = np.zeros((14 * K, 32))
    child = np.array([math.atanh(0.5), 0, 0, 0, 1, 0.5, 0, 0, 0, 0, 0, 0.25, -0.5, 1.0])
    b2 = np.tile(child, K)
    theta = np.concatenate([W1.ravel(), b1, W2.ravel(), b2])
    out = an.decode(anc, theta, K, centre=[0, 0, 0])
    l = np.exp(anc["log_l"])
    for a in range(A):
        for k in range(K):
            j = a * K + k
            assert np.allclose(out["means"][:, j], anc["p"][:, a] + (anc["O"][k, :, a] + [0.25, -0.5, 1.0]) * l[:, a])
            assert np.allclose(out["log_scales"][:, j], np.log(0.5 * l[:, a]))
            assert np.allclose(out["quats"][:, j], [1, 0.5, 0, 0]) and np.allclose(out["sh"][0, :, j], 0.0)
            assert out["logits"][j] == pytest.approx(0.0, abs=1e-12)        # alpha~ = 0.5
    far = dict(anc, level=np.zeros(A, np.int64))          # level 0 (below 10 m): masked at ~42 m
    assert (an.decode(far, theta, K, centre=[0, 0, 0])["logits"] == -100.0).all()


def test_network_layout_against_explicit_loops():
    """BF16-exact values (small dyadic numbers), so the rounding is the identity: the outputs equal explicit
    loops over W1 [32][36] (rows = hidden units) and W2 [14K][32]; a transposed operand would not."""
    rng = np.random.default_rng(1)
    K, A = 2, 3
    anc = _anchors(rng, A, K)
    anc["f"] = rng.integers(-4, 5, (A, 32)) / 8.0
    anc["p"] = np.array([[0.0, 0.0, -4.0], [0.0, 4.0, 0.0], [2.0, 0.0, 0.0]])   # axis directions, distances 2, 4, 4
    W1 = rng.integers(-3, 4, (32, 36)) / 16.0
    b1 = rng.integers(-2, 3, 32) / 4.0
    W2 = rng.integers(-3, 4, (14 * K, 32)) / 16.0
    b2 = rng.integers(-2, 3, 14 * K) / 4.0
    out = an.decode(anc, np.concatenate([W1.ravel(), b1, W2.ravel(), b2]), K, centre=[0, 0, 0])
    for a in range(A):
        x = list(anc["f"][a]) + list(anc["p"][:, a] / np.linalg.norm(anc["p"][:, a])) + [np.linalg.norm(anc["p"][:, a])]
        h = [max(0.0, sum(W1[u][i] * x[i] for i in range(36)) + b1[u]) for u in range(32)]
        hb = an.bf16(np.array(h))
        y = [sum(W2[o][u] * hb[u] for u in range(32)) + b2[o] for o in range(14 * K)]
        assert np.allclose(out["raw"][a], y, rtol=0, atol=1e-12)


def test_tanh_logit():
    """ln(tanh y / (1 - tanh y)) three ways: the plain quotient where tanh is far from 1, the asymptote 2y - ln 2
    where e^{-2y} vanishes in FP64, and 60-digit decimal arithmetic of ln((e^{2y} - 1) / 2) in between."""
    import decimal
    y = np.array([1e-3, 0.1, 0.49, 0.5, 0.51, 1.0, 2.5])
    t = np.tanh(y)
    assert np.allclose(an.tanh_logit(y), np.log(t / (1 - t)), rtol=1e-12, atol=0)
    for big in (30.0, 400.0, 1e4):
        assert an.tanh_logit(np.array([big]))[0] == pytest.approx(2 * big - math.log(2.0), rel=1e-15)
    ctx = decimal.Context(prec=60)
    for v in (0.3, 0.75, 3.0, 9.5, 17.0):
        e = ctx.exp(ctx.multiply(decimal.Decimal(2), decimal.Decimal(v)))
        ref = float(ctx.ln(ctx.divide(ctx.subtract(e, 1), 2)))
        assert an.tanh_logit(np.array([v]))[0] == pytest.approx(ref, rel=1e-14)


def test_lod_mask_bands():
    d = np.array([0.0, 9.999, 10.0, 24.9, 25.0, 99.0, 100.0, 499.0, 500.0, 1e5])
    for lev, inside in [(0, [1, 1, 0, 0, 0, 0, 0, 0, 0, 0]), (1, [0, 0, 1, 1, 0, 0, 0, 0, 0, 0]),
                        (2, [0, 0, 0, 0, 1, 1, 0, 0, 0, 0]), (4, [0, 0, 0, 0, 0, 0, 0, 0, 1, 1])]:
        assert list(an.lod_mask(d, np.full(len(d), lev))) == inside


def test_bf16_margin():
    # 1 + 2^-8 is a BF16 rounding boundary (halfway between 1 and 1 + 2^-7); 1 is representable
    assert an._bf16_margin(np.array([1.0 + 2.0 ** -8]))[0] == 0.0
    assert an._bf16_margin(np.array([1.0]))[0] == pytest.approx(2.0 ** -8)
    assert an._bf16_margin(np.array([0.0]))[0] == np.inf


def _brute_union(ov, anchor_of, n_anchor, target, tau):
    """Tile-free: every visible Gaussian, in (fp32 depth, index) order, at every pixel."""
    pr = ov.proj()
    vis = np.flatnonzero(pr["visible"])
    order = sorted(vis, key=lambda g: (float(np.float32(pr["depth"][g])), int(g)))
    img = ov.image()
    om = np.zeros(n_anchor, np.int64)
    ka = np.zeros(n_anchor, np.int64)
    cfg = ov.cfg
    for py in range(ov.H):
        for px in range(ov.W):
            err = np.abs(target[:, py, px].astype(np.float64) - img["color"][:, py, px]).sum()
            T, seen = 1.0, set()
            for g in order:
                dx, dy = px + 0.5 - pr["mu"][g, 0], py + 0.5 - pr["mu"][g, 1]
                a_, b_, c_ = pr["conic"][g]
                raw = pr["opacity"][g] * math.exp(-0.5 * (a_ * dx * dx + 2 * b_ * dx * dy + c_ * dy * dy))
                if raw < cfg.alpha_min:
                    continue
                al = min(raw, cfg.alpha_max)
                if T * (1 - al) < cfg.t_min:
                    break
                seen.add(int(anchor_of[g]))
                T *= 1 - al
            for a in seen:
                om[a] += 1
                ka[a] += err > tau
    return om, ka


def test_anchor_union_statistics():
    sc = scenes.tiny_scene(seed=41, n=36, degree=1, W=40, H=30)
    ov = oracle.View(sc, 0, OracleConfig())
    # each Gaussian its own anchor: the per-Gaussian statistics
    st = ov.stats(sc.target[0], 0.1)
    s1 = ov.anchor_stats(np.arange(sc.n), sc.n, sc.target[0], 0.1)
    assert np.array_equal(s1["omega"], st["omega"]) and np.array_equal(s1["kappa"], st["kappa"])
    # groups of three: the union, against brute force; bounded by the children's sum and maximum
    anchor_of = np.arange(sc.n) // 3
    s3 = ov.anchor_stats(anchor_of, 12, sc.target[0], 0.1)
    om, ka = _brute_union(ov, anchor_of, 12, sc.target[0], 0.1)
    assert np.array_equal(s3["omega"], om) and np.array_equal(s3["kappa"], ka)
    child = st["omega"].reshape(12, 3)
    assert (s3["omega"] <= child.sum(1)).all() and (s3["omega"] >= child.max(1)).all()
    assert (s3["omega"] < child.sum(1)).any()          # overlapping children are counted once
