"""The learned head's kernels through the C ABI against the network oracle:
forward logits and decisions, the weighted cross-entropy gradient, Adam, the
feature kernel, and training on the plain criterion's labels."""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2606_30436_amd import head as hd
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, 1.5, (n, 16)).astype(np.float32)
    x[:, 15] = (rng.uniform(size=n) < 0.7).astype(np.float32)
    xb = mlp.bf16(x).astype(np.float32)          # features as the kernels read them
    theta = mlp.init_params(seed).astype(np.float64)
    theta[1024:1088] = rng.normal(0, 0.1, 64)
    theta[5184:5248] = rng.normal(0, 0.1, 64)
    theta[5440:] = rng.normal(0, 0.1, 3)
    y = rng.integers(0, 3, n).astype(np.uint8)
    return xb, theta.astype(np.float32), y


ACC = 8 * 2.0 ** -24    # eight FP32 roundings of a sum, relative to the sum of the magnitudes it adds


def _logit_bound(x, theta):
    """Per Gaussian and logit, how far the GPU's logits may lie from the FP64 oracle's.  The products of BF16
    operands are exact in FP32 and each sum may be off by ACC times the sum of the magnitudes it adds; a hidden
    unit whose interval of possible sums holds a BF16 rounding boundary (or zero) may round to the neighbouring
    BF16 value, one BF16 unit away, and that difference is carried through the next layers' magnitudes.  Also
    returns which Gaussians have such a unit."""
    f = mlp.forward(x, theta.astype(np.float64), True)
    b = mlp.unpack(theta.astype(np.float64))
    d_in = np.zeros_like(f["x"])                 # the inputs are the kernels' BF16 features, exactly
    amb = np.zeros(x.shape[0], bool)
    for z, W, bias, h_in in ((f["z1"], f["W1"], b["b1"], f["x"]), (f["z2"], f["W2"], b["b2"], f["h1"])):
        dz = d_in @ np.abs(W).T + ACC * (np.abs(h_in) @ np.abs(W).T + np.abs(bias) + 1e-30)
        lo, hi = np.maximum(z - dz, 0.0), np.maximum(z + dz, 0.0)
        flips = mlp.bf16_bits(lo) != mlp.bf16_bits(hi)
        amb |= flips.any(axis=1)
        # a flip moves the BF16 value by at most the gap between the two roundings of the interval's ends
        d_in = np.abs(mlp.bf16(hi) - mlp.bf16(lo))
    bound = d_in @ np.abs(f["W3"]).T + ACC * (np.abs(f["h2"]) @ np.abs(f["W3"]).T + np.abs(b["b3"]) + 1e-30)
    return bound, amb, f


def test_head_forward_matches_oracle():
    n = 5000
    x, theta, _ = _data(n, 1)
    h = hd.PruneHead(theta)
    feats = torch.from_numpy(x).to(torch.bfloat16).cuda()
    lg, dec = h.forward(feats)
    torch.cuda.synchronize()
    lg = lg.cpu().numpy().astype(np.float64)
    bound, amb, f = _logit_bound(x, theta)
    ref = f["logits"]
    err = np.abs(lg - ref)
    say(f"[gpu] head forward: Gaussians with a unit at a BF16 boundary {amb.sum()}/{n}; "
        f"max err / bound {np.max(err / bound):.3f}; max err elsewhere {err[~amb].max():.2e}")
    # every Gaussian, every logit: within the propagated rounding bound
    assert (err <= bound).all(), np.flatnonzero((err > bound).any(axis=1))[:8]
    # decisions: the argmax of the GPU logits, and the oracle's wherever the top two are further apart than the
    # bounds of both
    d = dec.cpu().numpy()
    assert np.array_equal(d, np.argmax(lg, axis=1))
    top = np.argsort(ref, axis=1)
    r = np.arange(n)
    clear = ref[r, top[:, 2]] - ref[r, top[:, 1]] > bound[r, top[:, 2]] + bound[r, top[:, 1]]
    say(f"  decisions compared {int(clear.sum())}/{n}")
    assert clear.mean() > 0.99
    assert np.array_equal(d[clear], top[clear, 2])


def test_head_forward_ragged_and_empty():
    x, theta, _ = _data(37, 2)
    h = hd.PruneHead(theta)
    feats = torch.from_numpy(x).to(torch.bfloat16).cuda()
    for n in (0, 1, 15, 16, 17, 37):
        lg, dec = h.forward(feats[:n].contiguous()) if n else h.forward(feats[:0])
        torch.cuda.synchronize()
        if n:
            ref = mlp.forward(x[:n], theta.astype(np.float64), True)["logits"]
            assert np.abs(lg.cpu().numpy() - ref).max() < 1e-3 * (np.abs(ref).max() + 1)


def test_head_gradient_matches_oracle():
    n = 4096
    x, theta, y = _data(n, 3)
    cw = mlp.class_weights(y).astype(np.float32)
    h = hd.PruneHead(theta)
    feats = torch.from_numpy(x).to(torch.bfloat16).cuda()
    loss, grad = h.loss_grad(feats, torch.from_numpy(y).cuda(), torch.from_numpy(cw).cuda())
    torch.cuda.synchronize()
    ref_loss, ref_g = mlp.loss_and_grad(x, y, cw.astype(np.float64), theta.astype(np.float64), True)
    g = grad.cpu().numpy().astype(np.float64)
    say(f"[gpu] head loss {float(loss.item()):.6f} vs {ref_loss:.6f}")
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * abs(ref_loss)
    for name, lo, hi in (("W1", 0, 1024), ("b1", 1024, 1088), ("W2", 1088, 5184), ("b2", 5184, 5248),
                         ("W3", 5248, 5440), ("b3", 5440, 5443)):
        rel = np.linalg.norm(g[lo:hi] - ref_g[lo:hi]) / np.linalg.norm(ref_g[lo:hi])
        say(f"  {name}: rel {rel:.2e}")
        assert rel < 1e-3, name
    # deterministic: a second call gives the same bits
    g2 = h.loss_grad(feats, torch.from_numpy(y).cuda(), torch.from_numpy(cw).cuda())[1].clone()
    assert torch.equal(g2, grad)


def test_head_adam_matches_oracle():
    rng = np.random.default_rng(4)
    theta = rng.normal(0, 0.1, mlp.N_PARAMS).astype(np.float32)
    h = hd.PruneHead(theta)
    t64, m64, v64 = theta.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for step in range(1, 4):
        g = rng.normal(0, 1e-2, mlp.N_PARAMS).astype(np.float32)
        h.grad.copy_(torch.from_numpy(g))
        h.adam(1e-3)
        t64, m64, v64 = mlp.adam(t64, m64, v64, g.astype(np.float64), step, 1e-3)
    torch.cuda.synchronize()
    assert np.abs(h.theta.cpu().numpy() - t64).max() < 1e-6


def test_head_training_reduces_the_loss_and_learns_a_threshold_rule():
    """A rule of the criterion's kind (prune above a score, densify above a
    count) is learned by the GPU kernels alone."""
    n = 20000
    rng = np.random.default_rng(5)
    x = np.zeros((n, 16), np.float32)
    x[:, 0] = rng.uniform(0, 10, n)           # S_d-like
    x[:, 2] = rng.uniform(0, 1, n)            # S_p-like
    x[:, 3:15] = rng.normal(0, 1, (n, 12))
    y = np.where(x[:, 2] > 0.8, 2, np.where(x[:, 0] > 5, 1, 0)).astype(np.uint8)
    feats = torch.from_numpy(mlp.bf16(x).astype(np.float32)).to(torch.bfloat16).cuda()
    lab = torch.from_numpy(y).cuda()
    cw = torch.from_numpy(mlp.class_weights(y)).float().cuda()   # balanced weights, computed by the oracle
    h = hd.PruneHead(seed=7)
    first = None
    for it in range(400):
        loss = float(h.train_step(feats, lab, cw, 3e-3).item()) if it % 50 == 0 else h.train_step(feats, lab, cw, 3e-3)
        if it == 0:
            first = loss
    _, dec = h.forward(feats)
    torch.cuda.synchronize()
    acc = float((dec == lab).float().mean())
    last = float(h.loss.item())
    say(f"[gpu] head training: loss {first:.3f} -> {last:.3f}, accuracy {acc:.4f}")
    assert last < 0.25 * first and acc > 0.97


def test_feature_kernel_matches_host_formulas():
    """Features of a real chunk against the same formulas on the host from the
    GPU's statistics (the chunk min / max of L over the active set in FP64)."""
    from paper_2606_30436_amd import scenes
    from paper_2606_30436_amd.rasterizer import (GaussianParams, Image, LifecycleState, Rasterizer, ViewStats,
                                                 device_cameras)
    sc = scenes.make_c3(seed=21, n=100_000, n_views=3)
    sc.target = scenes.random_target(22, 3, sc.height, sc.width)
    R = Rasterizer(sc.width, sc.height, max_views=3, max_gaussians=sc.n, far_z=80.0)
    g = GaussianParams.from_scene(sc)
    cams = device_cameras(sc.cams)
    img = Image.empty(3, sc.height, sc.width)
    R.project(g, cams)
    R.bin_sort()
    R.render_fwd(img)
    tgt = torch.from_numpy(sc.target).cuda()
    dl = torch.empty_like(img.color)
    loss = torch.empty(3, device="cuda")
    R.loss_l1(tgt, img, dl, loss)
    st = ViewStats.zeros(sc.n)
    R.render_bwd(g, cams, None, img, dl, target=tgt, tau_err=0.1, view_loss=loss, grads=g.zeros_like(), stats=st)
    before = LifecycleState.zeros(sc.n)
    before.prune_score.uniform_(0, 1)
    before.densify.copy_((torch.rand(sc.n, device="cuda") > 0.5).to(torch.uint8))
    f = hd.features(R, g, st, 3, before).float().cpu().numpy()
    torch.cuda.synchronize()
    k, om = st.kappa_sum.cpu().numpy().astype(np.float64), st.omega_sum.cpu().numpy().astype(np.float64)
    gam, vc = st.gamma_sum.cpu().numpy(), st.view_count.cpu().numpy().astype(np.float64)
    L = np.log1p(gam)
    act = om > 0
    lo, hi = L[act].min(), L[act].max()
    ls = np.sort(sc.log_scales.astype(np.float64), axis=0)[::-1]
    ref = np.stack([k / 3, L, np.where(act, (L - lo) / (hi - lo), 0), np.log1p(om), np.where(act, k / np.maximum(om, 1), 0),
                    vc / 3, st.grad_norm_sum.cpu().numpy() / np.maximum(vc, 1), np.log1p(st.max_radius.cpu().numpy()),
                    1 / (1 + np.exp(-sc.logits.astype(np.float64))), ls[0], ls[1], ls[2],
                    before.prune_score.cpu().numpy(), before.densify.cpu().numpy(),
                    np.where(act, gam / np.maximum(om, 1), 0), act.astype(np.float64)], axis=1)
    say(f"[gpu] features: active {int(act.sum())}/{sc.n}")
    assert act.sum() > 1000
    # BF16 keeps 8 significant bits; the FP32 arithmetic of the kernel adds ~1e-6
    assert np.all(np.abs(f - ref) <= 2 ** -8 * np.abs(ref) + 1e-6)


def test_head_gain_over_the_plain_criterion():
    """Trained by the library's kernels on the criterion's decisions of the first chunks (all 16 views), the
    head decides the held-out chunks from a cheap pass over 4 of their views.  Judged per class against the
    full criterion, beside the two ways to decide without it: keep everything, or apply the plain criterion
    to the same cheap pass.  The bars sit below what this configuration measures (densify recall 0.63,
    precision 0.54, F1 0.58 against 0.45 for the criterion on the cheap views; agreement on the Gaussians
    either side changes 0.41 against 0.29)."""
    from paper_2606_30436_amd import head_experiment as hx
    r = hx.run(n=1_000_000, chunks=8, views=16, train_chunks=6, steps=800, w_densify=3.0)
    pc, cb, ka = r["per_class"], r["cheap_views_criterion_baseline"], r["all_keep_baseline"]
    say(f"[gpu] head gain: agreement {r['test_global_agreement']} (keep-all {ka['test_global_agreement']}, "
        f"cheap criterion {cb['test_global_agreement']}), on touched {r['test_global_agreement_on_touched']} "
        f"(cheap criterion {cb['test_global_agreement_on_touched']}); densify {pc['densify']} vs "
        f"{cb['per_class']['densify']}; prune {pc['prune']}; confusion {r['confusion_criterion_rows_head_cols']}; "
        f"psnr {r['psnr_db']}; speedup {r['decision_speedup']}")
    conf = np.array(r["confusion_criterion_rows_head_cols"])
    assert conf.sum() == r["map_gaussians"]
    assert conf[hd.DENSIFY].sum() == pc["densify"]["criterion"] and conf[:, hd.DENSIFY].sum() == pc["densify"]["head"]
    # densify: the head finds most of the criterion's densifications and most of its own are right
    assert pc["densify"]["recall"] > 0.5 and pc["densify"]["precision"] > 0.45
    # better than deciding from the same cheap pass without it, and than keeping everything
    assert pc["densify"]["f1"] > cb["per_class"]["densify"]["f1"] + 0.05
    assert r["test_global_agreement_on_touched"] > cb["test_global_agreement_on_touched"] + 0.05
    assert r["test_global_agreement_on_touched"] > ka["test_global_agreement_on_touched"] + 0.3
    assert r["test_global_agreement"] > ka["test_global_agreement"]
    # pruning with the head costs no image quality against the unpruned map
    assert r["psnr_db"]["head_pruned"] >= r["psnr_db"]["unpruned"] - 0.05
    assert r["train_accuracy"] > 0.85
    # the criterion's own pass (the compositing backward over every view) is what the head saves
    assert r["decision_speedup"] > 1.5
