#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload: the batched keyframe chunk -- 2M Gaussians along a 1 km synthetic
driving trajectory, the 8 sampled keyframes of one chunk at 1242x375, SH
degree 3, FP32 with FP32 gradient accumulation.  One step = one chunk: zero
the accumulators, project, bin + sort, composite forward, L1 loss, composite
backward, projection backward with footprint statistics, chunk scores and the
densify / prune decision -- all captured in one HIP graph and launched once.
The plain baseline runs the same library one view at a time with a host read
of the pair count between projection and sort, as a naive loop would.

Prints one JSON line (see the repository's measurement notes for the fields).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "fwd+bwd Mpix/s and ms/keyframe-chunk at 2M Gaussians; batched vs plain"
W, H, V, N = 1242, 375, 8, 2_000_000
FAR = 80.0
# algorithmic FP32 operations of the compositing backward: every tile-list
# entry up to a pixel's last blended Gaussian is tested (10 flop), every
# blended one is differentiated (52 flop); FMA counts 2.
FLOP_TEST, FLOP_BLEND = 10, 52
# non-packed FP32 VALU peak: 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_ALU_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
HBM_BYTES_PER_S = 8e12
# the forward's blend of an entry (exp2, clamp, weight, three colour and one depth FMA, T update)
FLOP_FWD_BLEND = 20
SH_K = 16  # SH degree 3
# mapping loss per pixel and channel: the products x^2, y^2, xy (3), five maps filtered by the separable
# 11-tap window (2 x 11 FMA each: 220), SSIM and its three derivative maps (35), those three filtered
# (132), the gradient (8)
MAPLOSS_FLOP_PER_PX_CH = 3 + 220 + 35 + 132 + 8
FIT_NOISE = 0.02   # standard deviation of the pixel noise on the equal-PSNR fit's targets


def chunk_roofline(stage_ms: dict, ms: float, N: int, S: int, P: int, P_live: int, E: int, E_b: int,
                   npix: int) -> dict:
    """Per-stage roofline of the chunk: T_roof = sum over stages of max(algorithmic bytes / 8 TB/s,
    counted flop / ALU peak), against the chunk's measured time.  'survey' charges every stage the
    per-unit figures of the hot-path plan (every pair gathered and reduced, a 4-pass 24 B/pair sort
    of 46-bit keys); 'strict' charges only the pairs some pixel of their tile still needs (P_live)
    and one read and write of the sort's keys and values."""
    par = 44 + 12 * SH_K  # bytes of one Gaussian's parameters
    peak = PEAK_ALU_TFLOPS * 1e12

    def stage(nbytes, flop=0.0):
        t_b, t_f = nbytes / HBM_BYTES_PER_S, flop / peak
        return {"bound": "alu" if t_f > t_b else "hbm", "bytes": int(nbytes), "flop": int(flop),
                "t_roof_ms": round(1e3 * max(t_b, t_f), 5)}

    out = {}
    for mode, pp, sort_bytes in (("survey", P, 96 * P), ("strict", P_live, 16 * (S + P))):
        st = {
            "project": stage(N * par + 60 * S),
            "bin": stage(16 * S + 12 * P),
            "sort": stage(sort_bytes),
            "ranges": stage(8 * P),
            "render_fwd": stage(48 * pp + 24 * npix, FLOP_TEST * E + FLOP_FWD_BLEND * E_b),
            "loss": stage(36 * npix),
            "render_bwd_pixels": stage(48 * pp + 48 * npix, FLOP_TEST * E + FLOP_BLEND * E_b),
            "project_bwd": stage(48 * pp + 60 * S + 2 * N * par),
            "stats_decide": stage(30 * N),
        }
        t = sum(v["t_roof_ms"] for v in st.values())
        out[mode] = {"t_roof_ms": round(t, 4), "frac": round(t / ms, 4), "stages": st}
    measured = dict(stage_ms)
    out["stage_ms_measured"] = {k: round(v, 4) for k, v in measured.items()}
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2606_30436_amd", "csrc", "kgs_render.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(tile, batch):
    """Per-launch HBM bytes of the compositing backward from the committed
    rocprofv3 counter summary; None if absent, taken on other kernel source or
    on another tile shape / LDS batch than the one timed."""
    path = os.path.join(ROOT, "profiles", f"k_render_bwd_2M_8view_chunk_{tile[0]}x{tile[1]}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if vals.get("tile") != f"{tile[0]}x{tile[1]}" or vals.get("batch") != str(batch):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=str, default=None, help="e.g. 16x16 (skips the autotuner)")
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--px-per-lane", type=int, default=0,
                    help="compositing backward pixels per lane (0: the library's choice)")
    ap.add_argument("--stage-reps", type=int, default=5)
    ap.add_argument("--no-fit", action="store_true")
    ap.add_argument("--no-adjacent", action="store_true", help="skip the timed rows of the other mapping kernels")
    ap.add_argument("--fit-steps", type=int, default=200)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device-to-device three times (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one GPU only; --gpus {args.gpus} is not supported "
              "(sharding the views over GPUs is a design, not run)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_30436_amd import scenes
    from paper_2606_30436_amd.autotune import autotune
    from paper_2606_30436_amd.rasterizer import (GaussianParams, Image, LifecycleState, Rasterizer, ViewStats,
                                                 device_cameras, TILE_SHAPES, BATCHES)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        src = torch.ones(args.copy_probe, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 3}), flush=True)
        return
    t0 = time.time()
    sc = scenes.make_c3()
    true = scenes.Scene(sc.meta["true"]["means"], sc.log_scales, sc.quats, sc.logits, sc.meta["true"]["sh"], 3,
                        sc.cams, sc.pose_xi)
    log(f"[bench] scene ready {time.time() - t0:.1f}s")
    g = GaussianParams.from_scene(sc)
    gt = GaussianParams.from_scene(true)
    cams = device_cameras(sc.cams)

    # ---- capacities: probe every tiling once with generous capacities
    probe = Rasterizer(W, H, V, N, slot_capacity=V * N, pair_capacity=64_000_000, far_z=FAR)
    max_s = max_p = 0
    counts = {}
    for tile in TILE_SHAPES:
        probe.set_tiling(tile, 64)
        probe.project(g, cams)
        probe.bin_sort()
        torch.cuda.synchronize()
        assert probe.status() == 0, "probe overflow"
        s, p = probe.counts()
        counts[tile] = (s, p)
        max_s, max_p = max(max_s, s), max(max_p, p)
    # targets: renders of the unperturbed scene
    probe.set_tiling((16, 16), 64)
    target_img = Image.empty(V, H, W)
    probe.project(gt, cams)
    probe.bin_sort()
    probe.render_fwd(target_img)
    torch.cuda.synchronize()
    target = target_img.color.clone()
    probe.set_tiling((16, 16), 64)
    probe.project(g, cams)
    probe.bin_sort()
    torch.cuda.synchronize()
    bufs = probe.buffers()
    visible = np.bincount(bufs["slot_view"].numpy(), minlength=V).tolist()
    del bufs, probe, target_img
    torch.cuda.empty_cache()
    log(f"[bench] counts {counts} visible/view {visible}")

    R = Rasterizer(W, H, V, N, slot_capacity=int(max_s * 1.25) + 1024, pair_capacity=int(max_p * 1.25) + 4096,
                   px_per_lane=args.px_per_lane,
                   far_z=FAR)
    img = Image.empty(V, H, W)
    dl = torch.empty_like(img.color)
    loss = torch.empty(V, device=dev)
    grads = g.zeros_like()
    pose_grad = torch.zeros(V, 6, device=dev)
    stats = ViewStats.zeros(N)
    state = LifecycleState.zeros(N)
    decision = torch.empty(N, dtype=torch.uint8, device=dev)

    def desc(reset=True, with_state=True):
        return R.chunk_desc(g, cams, None, target, img, dl, loss, grads, pose_grad, stats, tau_err=0.1,
                            zero_accumulators=reset, state=state if with_state else None,
                            decision=decision if with_state else None)

    # ---- autotune tile shape x batch
    if args.tile:
        best = (tuple(int(x) for x in args.tile.split("x")), args.batch or 64)
        table = None
    elif args.no_autotune:
        best, table = ((16, 16), args.batch or 64), None
    else:
        # each candidate is timed as what is deployed: its chunk captured as a graph, then replayed
        cand = {"graph": None}

        def set_tiling(tile, batch):
            R.set_tiling(tile, batch)
            if cand["graph"] is not None:
                R.chunk_release(cand["graph"])
            cand["graph"] = None

        def run_graph():
            if cand["graph"] is None:
                cand["graph"] = R.chunk_capture(desc())
            R.chunk_launch(cand["graph"])
        best, table = autotune(run_graph, set_tiling, TILE_SHAPES, BATCHES, reps=5)
        log(f"[bench] autotune best {best}")
    R.set_tiling(best[0], best[1])

    # ---- batched: one graph launch per chunk
    d = desc()
    graph = R.chunk_capture(d)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        R.chunk_launch(graph)
    torch.cuda.synchronize()
    assert R.status() == 0, f"status {R.status()}"
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        R.chunk_launch(graph)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1) / args.steps
    log(f"[bench] batched {ms:.3f} ms/chunk (wall {1000 * wall / args.steps:.3f})")
    batched_color = img.color.clone()
    batched_dec = decision.clone()

    # ---- the same chunk with the Gaussians in a random index order (the scene stores them in the order a
    # mapper moving along the path would spawn them, which gives every kernel spatially coherent indices)
    perm = torch.from_numpy(np.random.default_rng(17).permutation(N)).to(dev)
    g_sh = GaussianParams(g.means[:, perm].contiguous(), g.log_scales[:, perm].contiguous(),
                          g.quats[:, perm].contiguous(), g.logits[perm].contiguous(), g.sh[:, :, perm].contiguous(),
                          g.sh_degree)
    d_sh = R.chunk_desc(g_sh, cams, None, target, img, dl, loss, grads, pose_grad, stats, tau_err=0.1,
                        zero_accumulators=True, state=state, decision=decision)
    graph_sh = R.chunk_capture(d_sh)
    for _ in range(max(args.warmup, 1)):
        R.chunk_launch(graph_sh)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        R.chunk_launch(graph_sh)
    ev1.record(stream)
    torch.cuda.synchronize()
    assert R.status() == 0, f"status {R.status()}"
    shuffled_ms = ev0.elapsed_time(ev1) / args.steps
    shuffled_same_images = bool(torch.equal(img.color, batched_color))
    log(f"[bench] batched, shuffled index order {shuffled_ms:.3f} ms/chunk (images identical: {shuffled_same_images})")
    del graph_sh, d_sh, g_sh, perm
    torch.cuda.empty_cache()

    # ---- per-stage timing (eager, same stream, HIP events)
    names = ["project", "bin_sort", "render_fwd", "loss", "render_bwd_pixels", "project_bwd", "stats_decide"]
    acc = {k: [] for k in names}
    for _ in range(args.stage_reps):
        grads.means.zero_()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        evs[0].record(stream)
        R.project(g, cams)
        evs[1].record(stream)
        R.bin_sort()
        evs[2].record(stream)
        R.render_fwd(img)
        evs[3].record(stream)
        R.loss_l1(target, img, dl, loss)
        evs[4].record(stream)
        R.render_bwd_pixels(img, dl, None, target, 0.1)
        evs[5].record(stream)
        R.project_bwd(g, cams, None, loss, grads, pose_grad, stats)
        evs[6].record(stream)
        R.accumulate_stats(stats, V, state, reset=False)
        R.decide(state, keep_map=False)
        evs[7].record(stream)
        torch.cuda.synchronize()
        for k, nme in enumerate(names):
            acc[nme].append(evs[k].elapsed_time(evs[k + 1]))
    stage_ms = {k: float(np.median(v)) for k, v in acc.items()}
    log(f"[bench] stages {json.dumps({k: round(v, 3) for k, v in stage_ms.items()})}")
    n_slots, n_pairs = R.counts()
    E = int(img.last.to(torch.int64).sum().item())
    # pairs some pixel of their tile still needs: per (view, tile) the largest 1 + last position
    tw, th = best[0]
    lp = torch.nn.functional.pad(img.last.to(torch.int64), (0, (-W) % tw, 0, (-H) % th))
    P_live = int(lp.view(V, lp.shape[1] // th, th, lp.shape[2] // tw, tw).amax(dim=(2, 4)).sum().item())
    E_b = int(stats.omega_sum.to(torch.int64).sum().item()) // args.stage_reps
    flop = FLOP_TEST * E + FLOP_BLEND * E_b
    t_bwd = stage_ms["render_bwd_pixels"] / 1e3
    achieved = flop / t_bwd / 1e12
    traffic = read_traffic(best[0], best[1])
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_ALU_TFLOPS, 2),
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_ALU_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_render_bwd (compositing backward)", "evaluations": E, "blended": E_b,
                "kernel_ms": round(stage_ms["render_bwd_pixels"], 4)}
    chunk_roof = chunk_roofline(stage_ms, ms, N, n_slots, n_pairs, P_live, E, E_b, V * W * H)
    roofline["chunk_frac"] = chunk_roof["survey"]["frac"]
    roofline["chunk_frac_strict"] = chunk_roof["strict"]["frac"]
    log(f"[bench] chunk roofline: survey {chunk_roof['survey']['t_roof_ms']} ms ({chunk_roof['survey']['frac']}), "
        f"strict {chunk_roof['strict']['t_roof_ms']} ms ({chunk_roof['strict']['frac']}), live pairs {P_live}")

    # ---- plain per-view loop (same library, no graph), with and without a host read of the
    # pair count between projection and sort; timed at 16x16 tiles with batch 128 and at the
    # batched chunk's tiling, and the faster of the two taken
    plain_ms = plain_nr_ms = None
    plain_table = None
    identical = None
    if not args.no_plain:
        P1 = Rasterizer(W, H, 1, N, slot_capacity=int(max_s * 1.25) + 1024,
                        pair_capacity=int(max_p * 1.25) + 4096, tile=(16, 16), batch=128, far_z=FAR)
        pimg = Image.empty(V, H, W)
        pdl = torch.empty_like(pimg.color)
        ploss = torch.empty(V, device=dev)
        pgr = g.zeros_like()
        ppose = torch.zeros(V, 6, device=dev)
        pst = ViewStats.zeros(N)
        pstate = LifecycleState.zeros(N)
        cam_bytes = cams.view(V, -1)

        def plain_chunk(host_read=True):
            for t in (pgr.means, pgr.log_scales, pgr.quats, pgr.logits, pgr.sh, ppose, pst.kappa_sum, pst.omega_sum,
                      pst.gamma_sum, pst.grad_norm_sum, pst.view_count, pst.max_radius):
                t.zero_()
            for v in range(V):
                vi = Image(pimg.color[v:v + 1], pimg.depth[v:v + 1], pimg.t_final[v:v + 1], pimg.last[v:v + 1])
                P1.project(g, cam_bytes[v])
                if host_read:
                    P1.counts()  # host read of the pair count before sorting, as a naive loop would
                P1.bin_sort()
                P1.render_fwd(vi)
                P1.loss_l1(target[v:v + 1], vi, pdl[v:v + 1], ploss[v:v + 1])
                P1.render_bwd(g, cam_bytes[v], None, vi, pdl[v:v + 1], target=target[v:v + 1], tau_err=0.1,
                              view_loss=ploss[v:v + 1], grads=pgr, pose_grad=ppose[v:v + 1], stats=pst)
            P1.accumulate_stats(pst, V, pstate, reset=True)
            return P1.decide(pstate, keep_map=False)[0]

        reps = max(3, args.steps // 4)
        plain_tilings = [((16, 16), 128)]
        if (tuple(best[0]), best[1]) not in plain_tilings:
            plain_tilings.append((tuple(best[0]), best[1]))
        plain_table = {}
        identical = True
        for tiling in plain_tilings:
            P1.set_tiling(*tiling)
            timed = {}
            for host_read in (True, False):
                for _ in range(2):
                    plain_chunk(host_read)
                torch.cuda.synchronize()
                ev0.record(stream)
                for _ in range(reps):
                    pdec = plain_chunk(host_read)
                ev1.record(stream)
                torch.cuda.synchronize()
                timed[host_read] = ev0.elapsed_time(ev1) / reps
            plain_table[f"{tiling[0][0]}x{tiling[0][1]}/{tiling[1]}"] = [round(timed[True], 4), round(timed[False], 4)]
            identical = identical and bool(torch.equal(pimg.color, batched_color)) and bool(torch.equal(pdec, batched_dec))
        plain_ms = min(v[0] for v in plain_table.values())
        plain_nr_ms = min(v[1] for v in plain_table.values())
        log(f"[bench] plain {plain_ms:.3f} ms/chunk ({plain_nr_ms:.3f} without the host read; per tiling, with / "
            f"without: {plain_table}), identical outputs {identical}")
        del P1

    # ---- equal-PSNR fit: 200 Adam steps from the perturbed map, batched graph against the plain loop
    fit_res = None
    if not args.no_fit:
        from paper_2606_30436_amd.fit import fit
        cap = dict(slot_capacity=int(max_s * 1.5) + 1024, pair_capacity=int(max_p * 1.5) + 4096)

        def both(tgt):
            fb = fit(sc, tgt, "batched", iters=args.fit_steps, tile=best[0], batch=best[1], far_z=FAR, **cap)
            fp = fit(sc, tgt, "plain", iters=args.fit_steps, tile=best[0], batch=best[1], far_z=FAR, **cap)
            return {"psnr_start_db": round(fb["psnr_start_db"], 4), "batched_psnr_db": round(fb["psnr_db"], 4),
                    "plain_psnr_db": round(fp["psnr_db"], 4), "delta_db": round(fb["psnr_db"] - fp["psnr_db"], 4),
                    "batched_l1_last_step": round(fb["l1_last_step"], 6), "plain_l1_last_step": round(fp["l1_last_step"], 6),
                    "batched_ms_per_step": round(fb["ms_per_step"], 3), "plain_ms_per_step": round(fp["ms_per_step"], 3)}

        # a keyframe is not exactly the render of any map: the targets carry sensor-like pixel noise
        noise = np.random.default_rng(99).normal(0.0, FIT_NOISE, tuple(target.shape)).astype(np.float32)
        noisy = (target + torch.from_numpy(noise).to(dev)).clamp_(0.0, 1.0)
        del noise
        fit_res = dict(both(noisy), iterations=args.fit_steps,
                       target=f"renders of the unperturbed map + N(0, {FIT_NOISE}^2) pixel noise, clamped to [0, 1]")
        nf = both(target)
        # where the fit reaches ~58 dB the end PSNR is set by rounding: the same batched fit with the other
        # 512-pixel tiles sums its pair terms in another grouping
        alt = (16, 32) if tuple(best[0]) != (16, 32) else (32, 16)
        fa = fit(sc, target, "batched", iters=args.fit_steps, tile=alt, batch=best[1], far_z=FAR, **cap)
        nf["batched_other_tiles"] = {"tile": list(alt), "psnr_db": round(fa["psnr_db"], 4),
                                     "delta_vs_batched_db": round(fa["psnr_db"] - nf["batched_psnr_db"], 4)}
        fit_res["noise_free_target"] = nf
        del noisy
        log(f"[bench] fit {json.dumps(fit_res)}")

    def psnr(a, b):
        mse = float(((a - b) ** 2).mean().item())
        return 10 * math.log10(1.0 / mse) if mse > 0 else float("inf")
    psnr_b = psnr(batched_color.clamp(0, 1), target.clamp(0, 1))

    # ---- the adjacent rows of the mapping step on this chunk, each timed on its own
    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def adjacent_rows():
        adjacent = {}
        # mapping loss (0.8 L1 + 0.2 D-SSIM and the depth L1 against renders of the noise-free map)
        tgt_depth = torch.empty(V, H, W, device=dev)
        R.project(gt, cams)
        R.bin_sort()
        timg = Image(torch.empty_like(img.color), tgt_depth, torch.empty_like(img.t_final), torch.empty_like(img.last))
        R.render_fwd(timg)
        R.project(g, cams)
        R.bin_sort()
        R.render_fwd(img)
        ml_dl, ml_dd = torch.empty_like(img.color), torch.empty_like(img.depth)
        ml_loss, ml_geo = torch.empty(V, device=dev), torch.empty(V, device=dev)
        t_ml = timed(lambda: R.loss_mapping(V, img, target, ml_dl, ml_loss, target_depth=tgt_depth, dl_ddepth=ml_dd,
                                            geo_loss=ml_geo))
        px_ch = 3 * V * W * H
        flop_ml = MAPLOSS_FLOP_PER_PX_CH * px_ch + 3 * V * W * H
        bytes_ml = 12 * px_ch + 12 * V * W * H
        adjacent["mapping_loss"] = {
            "ms": round(t_ml, 4), "bound": "alu", "flop": int(flop_ml), "bytes": int(bytes_ml),
            "achieved_tflops": round(flop_ml / (t_ml / 1e3) / 1e12, 3),
            "frac": round(flop_ml / (t_ml / 1e3) / 1e12 / PEAK_ALU_TFLOPS, 4),
            "photometric_loss_per_view": [round(float(x), 5) for x in ml_loss.cpu().tolist()]}
        iso_loss = torch.empty(1, device=dev)
        iso_grad = torch.zeros(3, N, device=dev)
        t_iso = timed(lambda: R.loss_iso(g, iso_loss, iso_grad))
        adjacent["isotropy"] = {"ms": round(t_iso, 4), "bound": "hbm", "bytes": 36 * N,
                                "frac": round(36 * N / (t_iso / 1e3) / HBM_BYTES_PER_S, 4)}

        def hbm_row(ms_, nbytes, **extra):
            return dict(ms=round(ms_, 4), bound="hbm", bytes=int(nbytes),
                        frac=round(nbytes / (ms_ / 1e3) / HBM_BYTES_PER_S, 4), **extra)

        # probabilistic initialisation on the chunk's keyframes: the noise-free renders as the keyframes, the
        # current map's renders as the rendered map
        from paper_2606_30436_amd.mapping import (Anchors, Initializer, SpawnList, VoxelMap, anchor_stats,
                                                  decode_anchors, gaussians_out)
        init = Initializer(W, H, V)
        spawn_cap = V * W * H
        spawn = SpawnList.empty(spawn_cap)
        uni = torch.from_numpy(np.random.default_rng(9).uniform(size=(V, H, W)).astype(np.float32)).to(dev)
        t_init = timed(lambda: init.spawn(target, tgt_depth, uni, cams, spawn, spawn_cap, rendered=img.color,
                                          rendered_depth=img.depth))
        n_spawn = int(spawn.count.item())
        # 36 B per pixel in (keyframe and render colour and depth, the uniform), the FP64 maps written and read
        # once (40 B), the spawning pixels' records out
        adjacent["init_spawn"] = hbm_row(t_init, (36 + 40) * V * W * H + 40 * n_spawn, spawning_pixels=n_spawn)
        # the keyframes' spawning pixels into an empty voxel map, then their new Gaussians
        vmap = VoxelMap(22, max(n_spawn, 1))
        keys = vmap.keys(spawn.level[:n_spawn], spawn.voxel[:n_spawn])
        n0 = torch.zeros(1, dtype=torch.int32, device=dev)
        n1 = torch.zeros(1, dtype=torch.int32, device=dev)
        anchor_ids = torch.empty(max(n_spawn, 1), dtype=torch.int32, device=dev)
        created = torch.empty(max(n_spawn, 1), dtype=torch.int32, device=dev)

        def map_insert():
            vmap.clear()
            vmap.insert(keys, n0, n1, anchor_ids, created)
        t_ins = timed(map_insert)
        # per candidate: key 8 B, slot read + claim 16 B, index and anchor out 8 B; the 2^22-slot clear
        adjacent["map_insert"] = hbm_row(t_ins, 32 * n_spawn + 16 * (1 << 22), candidates=n_spawn,
                                         new_anchors=int(n1.item()))
        # map maintenance on the chunk's 2M Gaussians: the survivors of the chunk's decision gathered into a
        # compacted map, and every Gaussian moved rigidly with its keyframe's pose update (Gaussian i tied to
        # keyframe i mod V, each keyframe's pose replaced by the next one's)
        from paper_2606_30436_amd import _lib as L
        dec_m, keep_m, nk_m = R.decide(state, keep_map=True)
        n_keep = int(nk_m.item())
        cm = [torch.empty(3, max(n_keep, 1), device=dev), torch.empty(3, max(n_keep, 1), device=dev),
              torch.empty(4, max(n_keep, 1), device=dev), torch.empty(max(n_keep, 1), device=dev),
              torch.empty(16, 3, max(n_keep, 1), device=dev)]
        cm_out = gaussians_out(*cm, sh_degree=3)
        t_cmp = timed(lambda: L.kgs_map_compact(g.c(), dec_m, keep_m, cm_out))
        # decision byte and keep-map entry per Gaussian, 236 B read and 236 B written per survivor
        adjacent["map_compact"] = hbm_row(t_cmp, 5 * N + 2 * 236 * n_keep, survivors=n_keep)
        al_means, al_quats = g.means.clone(), g.quats.clone()
        kf_of = torch.arange(N, device=dev, dtype=torch.int32) % V
        cam_rows = cams.view(V, -1)
        new_poses = torch.cat([cam_rows[1:], cam_rows[:1]]).reshape(-1).contiguous()
        t_al = timed(lambda: L.kgs_map_align(al_means, al_quats, N, kf_of, cams, new_poses, V))
        # mean and quaternion read and written, keyframe index read
        adjacent["map_align"] = hbm_row(t_al, 60 * N, gaussians=N)
        del cm, cm_out, al_means, al_quats
        # decoded Gaussians of 200k voxel anchors with 10 children each (2M Gaussians) for one keyframe, and
        # their per-anchor union footprints after compositing
        asc = scenes.make_anchor_scene()
        A_n, K_n = len(asc["level"]), asc["k"]
        anc = Anchors.from_arrays(asc["p"], asc["feat"], asc["log_l"], asc["offsets"], asc["level"])
        theta_a = torch.from_numpy(asc["theta"]).to(dev)
        acams = device_cameras(asc["cams"]).view(len(asc["cams"]), -1)
        dec = GaussianParams(torch.empty(3, A_n * K_n, device=dev), torch.empty(3, A_n * K_n, device=dev),
                             torch.empty(4, A_n * K_n, device=dev), torch.empty(A_n * K_n, device=dev),
                             torch.empty(1, 3, A_n * K_n, device=dev), 0)
        t_dec = timed(lambda: decode_anchors(anc, theta_a, acams[4], dec))
        # per anchor 276 B in (p, f, log l, 10 offsets, level), per child 56 B out
        adjacent["anchor_decode"] = hbm_row(t_dec, 276 * A_n + 56 * A_n * K_n, anchors=A_n, children=K_n,
                                            view="the fifth keyframe")
        # the anchors re-voxelised (after an alignment moved them): a freshly cleared 2^19-slot table, the
        # lowest index of each voxel kept, survivors renumbered
        rvm = VoxelMap(19, A_n)
        rv_means = torch.from_numpy(np.ascontiguousarray(asc["p"], dtype=np.float32)).to(dev)
        rv_level = torch.from_numpy(np.ascontiguousarray(asc["level"], dtype=np.int32)).to(dev)
        rv_keep = torch.empty(A_n, dtype=torch.uint8, device=dev)
        rv_anchor = torch.empty(A_n, dtype=torch.int32, device=dev)
        rv_n = torch.zeros(1, dtype=torch.int32, device=dev)

        def revoxelize():
            rvm.clear()
            rvm.revoxelize(rv_means, rv_level, rv_keep, rv_anchor, rv_n)
        t_rv = timed(revoxelize)
        # per anchor: mean and level in, the voxel's slot probed and claimed (16 B), keep flag and new index out;
        # the 8 MB table clear
        adjacent["map_revoxelize"] = hbm_row(t_rv, (16 + 16 + 5) * A_n + 16 * (1 << 19), anchors=A_n,
                                             survivors=int(rv_n.item()))
        del rvm
        RA = Rasterizer(W, H, 1, A_n * K_n, slot_capacity=A_n * K_n, pair_capacity=40_000_000, tile=best[0],
                        batch=best[1])
        RA.project(dec, acams[4])
        RA.bin_sort()
        aimg = Image.empty(1, H, W)
        RA.render_fwd(aimg)
        a_of = torch.arange(A_n * K_n, device=dev, dtype=torch.int32) // K_n
        ast = ViewStats.zeros(A_n)
        acounts = torch.zeros(2 * A_n, dtype=torch.int32, device=dev)
        astatus = torch.zeros(2, dtype=torch.int32, device=dev)
        t_ast = timed(lambda: anchor_stats(RA, aimg, a_of, A_n, target[4:5], None, acounts, ast, astatus))
        E_a = int(aimg.last.to(torch.int64).sum().item())
        # every evaluated entry is tested (10 flop) and blended entries update T (6 flop); the ballots and
        # unions are the overhead this count leaves out
        flop_a = FLOP_TEST * E_a
        adjacent["anchor_stats"] = dict(ms=round(t_ast, 4), bound="alu", flop=int(flop_a), evaluations=E_a,
                                        achieved_tflops=round(flop_a / (t_ast / 1e3) / 1e12, 3),
                                        frac=round(flop_a / (t_ast / 1e3) / 1e12 / PEAK_ALU_TFLOPS, 4),
                                        rewalks=int(astatus[1].item()))
        del RA
        return adjacent

    adjacent = {} if args.no_adjacent else adjacent_rows()
    log(f"[bench] adjacent rows {json.dumps(adjacent)}")

    # ---- CPU oracle baseline (the whole chunk, FP64, all host threads)
    cpu = None
    if not args.no_cpu:
        sys.path.insert(0, ROOT)
        import oracle
        from oracle import OracleConfig
        ocfg = OracleConfig(far=FAR)
        tgt = target.cpu().numpy()
        gC = dl.cpu().numpy().astype(np.float64)
        ot0 = time.perf_counter()
        for v in range(V):
            ov = oracle.View(sc, v, ocfg)
            ov.image()
            ov.stats(tgt[v], 0.1)
            ov.backward(gC[v])
            del ov
        ot = time.perf_counter() - ot0
        cpu = {"value": round(V * W * H / ot / 1e6, 4), "unit": "Mpix/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": f"the full workload: all {V} views of the chunk, fwd + stats + bwd, FP64",
               "seconds": round(ot, 2)}
        log(f"[bench] cpu oracle {ot:.1f}s")
        # one core: one view of the chunk (the fourth keyframe), the same three steps
        v1 = 3
        threads = oracle.num_threads()
        oracle.set_num_threads(1)
        ot0 = time.perf_counter()
        ov = oracle.View(sc, v1, ocfg)
        ov.image()
        ov.stats(tgt[v1], 0.1)
        ov.backward(gC[v1])
        del ov
        ot1 = time.perf_counter() - ot0
        oracle.set_num_threads(threads)
        cpu["one_core"] = {"value": round(W * H / ot1 / 1e6, 4), "unit": "Mpix/s", "cores": 1,
                           "sample": f"view {v1} of the chunk ({visible[v1]} visible Gaussians), fwd + stats + bwd, "
                                     "FP64, one thread", "seconds": round(ot1, 2)}
        log(f"[bench] cpu oracle one core, one view {ot1:.1f}s")

    mpix = V * W * H / (ms / 1e3) / 1e6
    out = {
        "metric": METRIC, "value": round(mpix, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched keyframe chunk: 2M Gaussians on a 1 km trajectory, 8 keyframes at "
                               "1242x375, SH3, FP32, one HIP graph per chunk",
                   "n_gaussians": N, "n_views": V, "width": W, "height": H, "far_z": FAR,
                   "tile": list(best[0]), "batch": best[1], "visible_per_view": visible, "slots": n_slots,
                   "pairs": n_pairs, "live_pairs": P_live,
                   "plain_loop": "per view: project, host read of the pair count, sort, fwd, loss, bwd; then "
                                 "stats + decide; no graph; the faster of 16x16 tiles with batch 128 and the "
                                 "batched chunk's tiling",
                   "plain_ms_per_tiling": plain_table,
                   "plain_ms_per_chunk": None if plain_ms is None else round(plain_ms, 4),
                   "speedup_vs_plain": None if plain_ms is None else round(plain_ms / ms, 3),
                   "plain_ms_per_chunk_no_host_read": None if plain_nr_ms is None else round(plain_nr_ms, 4),
                   "speedup_vs_plain_no_host_read": None if plain_nr_ms is None else round(plain_nr_ms / ms, 3),
                   "outputs_identical_to_plain": identical, "psnr_vs_target_db": round(psnr_b, 3),
                   "shuffled_index_order": {"ms_per_chunk": round(shuffled_ms, 4),
                                            "mpix_per_s": round(V * W * H / (shuffled_ms / 1e3) / 1e6, 1),
                                            "images_identical": shuffled_same_images},
                   "equal_psnr_fit": fit_res,
                   "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
                   "autotune_ms": table},
        "roofline": roofline,
        "chunk_roofline": chunk_roof,
        "adjacent_rows": adjacent,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
