"""What the learned head gains over the plain multi-view criterion.

Workload: a long trajectory map (injected floaters, facade holes), chunks of
keyframes.  Per chunk the plain criterion (Sec. 3.3, App. D) renders all of the
chunk's sampled views forward and backward against the targets, accumulates
|Omega|, kappa and gamma, and decides per Gaussian: PRUNE if S_p^(i,c) > tau_p,
DENSIFY if S_d^(i,c) > tau_d, else KEEP; the global decision is PRUNE if some
chunk prunes, else DENSIFY if some chunk densifies (the OR / max rules).  The
head sees only the statistics of a cheap pass over four of the chunk's views
(what ordinary mapping iterations already render) and predicts the chunk's
decision; its global decision is aggregated the same way.  It is trained on the
first chunks' criterion decisions with the library's own kernels and judged on
the remaining chunks: agreement, PSNR of the maps pruned either way against the
targets, time per chunk of either path, and statistic bytes per Gaussian.

Run: python -m paper_2606_30436_amd.head_experiment [--n N] [--chunks C] ...
Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import head as hd
from . import scenes
from .rasterizer import GaussianParams, Image, LifecycleState, Rasterizer, ViewStats, device_cameras

TAU_ERR, TAU_D, TAU_P = 0.1, 5.0, 0.99
FAR = 80.0


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _subset(g: GaussianParams, idx: torch.Tensor) -> GaussianParams:
    return GaussianParams(g.means[:, idx].contiguous(), g.log_scales[:, idx].contiguous(), g.quats[:, idx].contiguous(),
                          g.logits[idx].contiguous(), g.sh[:, :, idx].contiguous(), g.sh_degree)


class ChunkRunner:
    """Renders a set of views of a map forward and backward against targets and
    returns the per-Gaussian chunk statistics."""

    def __init__(self, R: Rasterizer, n: int, views: int, dev):
        self.R = R
        self.n = n
        self.dev = dev
        self.img = Image.empty(views, R.height, R.width)
        self.grads = None

    def stats(self, g: GaussianParams, cams: torch.Tensor, target: torch.Tensor) -> ViewStats:
        V = cams.numel() // 72
        R = self.R
        img = Image(self.img.color[:V], self.img.depth[:V], self.img.t_final[:V], self.img.last[:V])
        dl = torch.empty_like(img.color)
        loss = torch.empty(V, device=self.dev)
        st = ViewStats.zeros(g.n, self.dev)
        R.project(g, cams)
        R.bin_sort()
        R.render_fwd(img)
        R.loss_l1(target, img, dl, loss)
        if self.grads is None or self.grads.n != g.n:
            self.grads = g.zeros_like()
        R.render_bwd(g, cams, None, img, dl, target=target, tau_err=TAU_ERR, view_loss=loss, grads=self.grads,
                     stats=st)
        return st

    def render(self, g: GaussianParams, cams: torch.Tensor) -> torch.Tensor:
        V = cams.numel() // 72
        img = Image(self.img.color[:V], self.img.depth[:V], self.img.t_final[:V], self.img.last[:V])
        self.R.project(g, cams)
        self.R.bin_sort()
        self.R.render_fwd(img)
        return img.color.clone()


def chunk_decision(R: Rasterizer, st: ViewStats, views: int, n: int, dev) -> torch.Tensor:
    state = LifecycleState.zeros(n, dev)
    R.accumulate_stats(st, views, state, tau_d=TAU_D, reset=True)
    dec, _, _ = R.decide(state, tau_p=TAU_P, keep_map=False)
    return dec


def aggregate(decs) -> torch.Tensor:
    """Global rule over chunk decisions: PRUNE if any, else DENSIFY if any."""
    out = torch.zeros_like(decs[0])
    anyp = torch.zeros_like(decs[0], dtype=torch.bool)
    anyd = torch.zeros_like(anyp)
    for d in decs:
        anyp |= d == hd.PRUNE
        anyd |= d == hd.DENSIFY
    out[anyd] = hd.DENSIFY
    out[anyp] = hd.PRUNE
    return out


def class_metrics(conf: torch.Tensor) -> dict:
    """Recall, precision and F1 of DENSIFY and PRUNE from a confusion matrix (criterion rows, head columns)."""
    out = {}
    for name, k in (("densify", hd.DENSIFY), ("prune", hd.PRUNE)):
        tp = int(conf[k, k])
        fn = int(conf[k].sum()) - tp
        fp = int(conf[:, k].sum()) - tp
        rec = tp / (tp + fn) if tp + fn else 1.0
        prec = tp / (tp + fp) if tp + fp else 1.0
        f1 = 2 * rec * prec / (rec + prec) if rec + prec else 0.0
        out[name] = {"criterion": tp + fn, "head": tp + fp, "recall": round(rec, 4), "precision": round(prec, 4),
                     "f1": round(f1, 4)}
    return out


def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    mse = float(((a.clamp(0, 1) - b.clamp(0, 1)) ** 2).mean().item())
    return 10 * math.log10(1.0 / mse) if mse > 0 else float("inf")


def collect(n=5_000_000, chunks=32, views=16, cheap=(0, 4, 8, 12), seed=5) -> dict:
    """Every chunk's criterion decision (all views) and the cheap pass's features, with the time of each."""
    dev = torch.device("cuda")
    t0 = time.time()
    sc = scenes.make_c5(seed=seed, n=n, n_chunks=chunks, views_per_chunk=views)
    _log(f"[head] scene {time.time() - t0:.1f}s")
    full = GaussianParams.from_scene(sc)
    map_idx = torch.from_numpy(sc.meta["map_index"]).to(dev)
    struct_idx = torch.from_numpy(sc.meta["struct_index"]).to(dev)
    g = _subset(full, map_idx)
    gt = _subset(full, struct_idx)
    nmax = max(g.n, gt.n)
    R = Rasterizer(sc.width, sc.height, views, nmax, slot_capacity=views * 400_000, pair_capacity=80_000_000,
                   far_z=FAR)
    run_ = ChunkRunner(R, g.n, views, dev)
    cam_all = device_cameras(sc.cams).view(chunks * views, -1)
    cheap_idx = torch.tensor(cheap, device=dev)
    feats, labels, dec_crit, targets, dec_cheap = [], [], [], [], []
    t_crit = t_cheap = 0.0
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for c in range(chunks):
        cams = cam_all[c * views:(c + 1) * views].reshape(-1).contiguous()
        target = run_.render(gt, cams)
        ev[0].record()
        st = run_.stats(g, cams, target)
        dec = chunk_decision(R, st, views, g.n, dev)
        ev[1].record()
        cams2 = cam_all[c * views:(c + 1) * views][cheap_idx].reshape(-1).contiguous()
        st2 = run_.stats(g, cams2, target[cheap_idx].contiguous())
        f = hd.features(R, g, st2, len(cheap))
        # the plain criterion on the cheap pass's views alone: what the same pass decides without the head
        dec_cheap.append(chunk_decision(R, st2, len(cheap), g.n, dev))
        ev[2].record()
        torch.cuda.synchronize()
        assert R.status() == 0, f"capacity overflow in chunk {c}"
        t_crit += ev[0].elapsed_time(ev[1])
        t_cheap += ev[1].elapsed_time(ev[2])
        feats.append(f)
        labels.append(dec)
        dec_crit.append(dec)
        if c >= chunks // 2:
            targets.append(target)
    _log(f"[head] chunks done {time.time() - t0:.1f}s")
    return dict(n=n, chunks=chunks, views=views, cheap=cheap, seed=seed, dev=dev, sc=sc, g=g, run_=run_,
                cam_all=cam_all, feats=feats, labels=labels, dec_crit=dec_crit, targets=targets, t_crit=t_crit,
                t_cheap=t_cheap, dec_cheap=dec_cheap)


def run(n=5_000_000, chunks=32, views=16, cheap=(0, 4, 8, 12), train_chunks=24, steps=1500, batch=65536, lr=3e-3,
        seed=5, w_prune=1.0, w_densify=1.0) -> dict:
    return evaluate(collect(n, chunks, views, cheap, seed), train_chunks, steps, batch, lr, w_prune, w_densify)


def evaluate(d: dict, train_chunks=24, steps=1500, batch=65536, lr=3e-3, w_prune=1.0, w_densify=1.0) -> dict:
    """Trains a head on the first train_chunks chunks' decisions and judges it on the others
    (train_chunks >= half the chunks: the held-out chunks' targets are kept for the last half only)."""
    assert d["chunks"] // 2 <= train_chunks < d["chunks"]
    n, chunks, views, cheap, seed, dev = d["n"], d["chunks"], d["views"], d["cheap"], d["seed"], d["dev"]
    sc, g, run_, cam_all = d["sc"], d["g"], d["run_"], d["cam_all"]
    feats, labels, dec_crit, t_crit, t_cheap = d["feats"], d["labels"], d["dec_crit"], d["t_crit"], d["t_cheap"]
    dec_cheap = d["dec_cheap"]
    # the held-out chunks' targets (collected for every chunk from the first held-out one on)
    targets = d["targets"][train_chunks - chunks:]

    # the head decides the Gaussians the cheap pass saw; the others are kept.
    # training set: those Gaussians of the training chunks
    tr_f, tr_y = [], []
    for c in range(train_chunks):
        act = feats[c][:, 15].float() > 0
        tr_f.append(feats[c][act])
        tr_y.append(labels[c][act])
    tr_f = torch.cat(tr_f).contiguous()
    tr_y = torch.cat(tr_y).contiguous()
    # cross-entropy with extra weights on the rare classes (a fully class-balanced
    # loss trades many wrong prunes for them)
    cw = torch.tensor([1.0, w_densify, w_prune], device=dev)
    head = hd.PruneHead(seed=seed)
    gen = torch.Generator(device=dev).manual_seed(seed)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for s in range(steps):
        idx = torch.randint(0, tr_f.shape[0], (min(batch, tr_f.shape[0]),), device=dev, generator=gen)
        head.train_step(tr_f[idx].contiguous(), tr_y[idx].contiguous(), cw, lr * (0.5 * (1 + math.cos(math.pi * s / steps))))
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    _, tr_pred = head.forward(tr_f)
    train_acc = float((tr_pred == tr_y).float().mean())
    # what the cheap pass cannot see: criterion decisions outside its footprint
    unseen = float(torch.stack([((feats[c][:, 15].float() == 0) & (labels[c] != hd.KEEP)).float().sum()
                                for c in range(chunks)]).sum() / max(1, sum(int((l != hd.KEEP).sum()) for l in labels)))

    # held-out chunks: per-chunk predictions (Gaussians outside the cheap
    # pass's footprint are kept), global aggregation
    t_head = 0.0
    pred = []
    head.forward(feats[train_chunks])
    torch.cuda.synchronize()
    for c in range(train_chunks, chunks):
        e0.record()
        _, dc = head.forward(feats[c])
        e1.record()
        torch.cuda.synchronize()
        t_head += e0.elapsed_time(e1)
        pred.append(torch.where(feats[c][:, 15].float() > 0, dc, torch.zeros_like(dc)))
    test_chunks = chunks - train_chunks
    glob_head = aggregate(pred)
    glob_crit = aggregate(dec_crit[train_chunks:])
    conf = torch.zeros(3, 3, dtype=torch.int64)
    for i in range(3):
        for j in range(3):
            conf[i, j] = int(((glob_crit == i) & (glob_head == j)).sum().item())
    touched = (glob_crit != hd.KEEP) | (glob_head != hd.KEEP)
    agree_all = float((glob_head == glob_crit).float().mean())
    agree_touched = float((glob_head[touched] == glob_crit[touched]).float().mean()) if touched.any() else 1.0
    per_class = class_metrics(conf)

    def judge(glob):
        cf = torch.zeros(3, 3, dtype=torch.int64)
        for i in range(3):
            for j in range(3):
                cf[i, j] = int(((glob_crit == i) & (glob == j)).sum().item())
        tch = (glob_crit != hd.KEEP) | (glob != hd.KEEP)
        return {"test_global_agreement": round(float((glob == glob_crit).float().mean()), 5),
                "test_global_agreement_on_touched": round(float((glob[tch] == glob_crit[tch]).float().mean()), 4)
                if tch.any() else 1.0, "confusion_criterion_rows_cols": cf.tolist(), "per_class": class_metrics(cf)}
    cheap_crit = judge(aggregate(dec_cheap[train_chunks:]))
    # the method without the head keeps every Gaussian it has no statistics for; the trivial stand-in for a
    # head is to keep all of them
    keep_all = {"test_global_agreement": round(float((glob_crit == hd.KEEP).float().mean()), 5),
                "test_global_agreement_on_touched": 0.0, "recall": {"densify": 0.0, "prune": 0.0}}
    chunk_agree = float(torch.stack([(p == d).float().mean() for p, d in zip(pred, dec_crit[train_chunks:])]).mean())

    # PSNR of the held-out views with the map pruned by either decision
    def pruned_psnr(glob):
        keep = torch.nonzero(glob != hd.PRUNE).squeeze(1)
        gk = _subset(g, keep)
        vals = []
        for k, c in enumerate(range(train_chunks, chunks)):
            cams = cam_all[c * views:(c + 1) * views].reshape(-1).contiguous()
            vals.append(psnr(run_.render(gk, cams), targets[k]))
        return float(np.mean(vals))
    p_none = pruned_psnr(torch.zeros_like(glob_crit))
    p_crit = pruned_psnr(glob_crit)
    p_head = pruned_psnr(glob_head)
    out = {
        "workload": f"{n} Gaussians (5% floaters, facade holes), {chunks} chunks x {views} keyframes at "
                    f"{sc.width}x{sc.height}; head trained on chunks 0-{train_chunks - 1}, tested on "
                    f"{train_chunks}-{chunks - 1}",
        "map_gaussians": g.n,
        "class_weights": [1.0, w_densify, w_prune], "cheap_views": list(cheap),
        "train_samples": int(tr_f.shape[0]), "train_steps": steps, "train_ms": round(train_ms, 2),
        "train_accuracy": round(train_acc, 4),
        "criterion_changes_outside_cheap_footprint": round(unseen, 4),
        "test_chunk_agreement": round(chunk_agree, 5),
        "test_global_agreement": round(agree_all, 5),
        "test_global_agreement_on_touched": round(agree_touched, 4),
        "confusion_criterion_rows_head_cols": conf.tolist(),
        "per_class": per_class,
        "all_keep_baseline": keep_all,
        "cheap_views_criterion_baseline": cheap_crit,
        "psnr_db": {"unpruned": round(p_none, 3), "criterion_pruned": round(p_crit, 3),
                    "head_pruned": round(p_head, 3)},
        "psnr_delta_head_minus_criterion_db": round(p_head - p_crit, 3),
        "ms_per_chunk": {"criterion_all_views": round(t_crit / chunks, 3),
                         "head_cheap_pass_and_features": round(t_cheap / chunks, 3),
                         "head_forward": round(t_head / test_chunks, 3)},
        "decision_speedup": round((t_crit / chunks) / (t_cheap / chunks + t_head / test_chunks), 2),
        # criterion: per-chunk kappa, |Omega|, gamma sums, global S_d flag and S_p score;
        # head: the cheap pass's six accumulators, the BF16 features, the aggregated decision
        "state_bytes_per_gaussian": {"criterion": {"per_chunk": 16, "persistent": 9},
                                     "head": {"per_chunk": 28 + 2 * hd.N_FEATURES, "persistent": 1}},
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=5_000_000)
    ap.add_argument("--chunks", type=int, default=32)
    ap.add_argument("--views", type=int, default=16)
    ap.add_argument("--train-chunks", type=int, default=24)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--w-prune", type=float, default=1.0)
    ap.add_argument("--w-densify", type=float, default=1.0)
    args = ap.parse_args()
    out = run(n=args.n, chunks=args.chunks, views=args.views, train_chunks=args.train_chunks, steps=args.steps,
              w_prune=args.w_prune, w_densify=args.w_densify)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
