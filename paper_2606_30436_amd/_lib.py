"""ctypes binding of libkgs.so (include/kgs.h), argument marshalling only.

The structures mirror the C header field for field; the functions carry the
C names.  Device arrays are passed as torch tensors (their data pointers);
streams default to torch's current stream.  Loading fails loudly when the HIP
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkgs.so")

P = ctypes.POINTER
c_void_p, c_int32, c_int64, c_float, c_double = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double

KGS_OK, KGS_ERR_INVALID_ARG, KGS_ERR_HIP, KGS_ERR_CAPACITY, KGS_ERR_NONFINITE, KGS_ERR_STATE = range(6)
FLAG_SLOT_OVERFLOW, FLAG_PAIR_OVERFLOW, FLAG_NONFINITE = 1, 2, 4
KEEP, DENSIFY, PRUNE = 0, 1, 2


class KgsCamera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("width", c_int32), ("height", c_int32)]


class KgsConfig(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("batch", c_int32), ("sh_degree", c_int32),
                ("alpha_min", c_float), ("alpha_max", c_float), ("t_min", c_float), ("near_z", c_float),
                ("eps2d", c_float), ("guard", c_float), ("rect_margin", c_float), ("far_z", c_float), ("bg", c_float * 3),
                ("width", c_int32), ("height", c_int32), ("max_views", c_int32), ("px_per_lane", c_int32),
                ("max_gaussians", c_int64), ("slot_capacity", c_int64), ("pair_capacity", c_int64)]


class KgsGaussians(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacity_logits", c_void_p),
                ("sh", c_void_p), ("n", c_int64), ("sh_degree", c_int32), ("pad_", c_int32)]


class KgsImage(ctypes.Structure):
    _fields_ = [("color", c_void_p), ("depth", c_void_p), ("t_final", c_void_p), ("last", c_void_p)]


class KgsGrads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacity_logits", c_void_p),
                ("sh", c_void_p), ("pose_xi", c_void_p)]


class KgsViewStats(ctypes.Structure):
    _fields_ = [("kappa_sum", c_void_p), ("omega_sum", c_void_p), ("gamma_sum", c_void_p),
                ("grad_norm_sum", c_void_p), ("view_count", c_void_p), ("max_radius", c_void_p)]


class KgsLifecycleState(ctypes.Structure):
    _fields_ = [("densify", c_void_p), ("prune_score", c_void_p)]


class KgsSpawnList(ctypes.Structure):
    _fields_ = [("pixel", c_void_p), ("level", c_void_p), ("voxel", c_void_p), ("point", c_void_p),
                ("color", c_void_p), ("count", c_void_p), ("capacity", c_int64)]


class KgsGaussiansOut(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacity_logits", c_void_p),
                ("sh", c_void_p), ("n", c_int64), ("sh_degree", c_int32), ("pad_", c_int32)]


class KgsAnchors(ctypes.Structure):
    _fields_ = [("p", c_void_p), ("feat", c_void_p), ("log_l", c_void_p), ("offsets", c_void_p), ("level", c_void_p),
                ("n", c_int64), ("k", c_int32), ("pad_", c_int32)]


def decoder_params(K: int) -> int:
    return 32 * 36 + 32 + 14 * K * 32 + 14 * K


class KgsBuffers(ctypes.Structure):
    _fields_ = [("n_slots", c_void_p), ("n_pairs", c_void_p), ("slot_rec", c_void_p), ("slot_gid", c_void_p),
                ("slot_view", c_void_p), ("slot_pix", c_void_p), ("slot_pairoff", c_void_p), ("keys", c_void_p),
                ("sorted_slot", c_void_p), ("ranges", c_void_p), ("tiles_x", c_int32), ("tiles_y", c_int32),
                ("tile_bits", c_int32), ("n_views", c_int32)]


class KgsChunkDesc(ctypes.Structure):
    _fields_ = [("gaussians", KgsGaussians), ("cams", c_void_p), ("pose_xi", c_void_p), ("n_views", c_int32),
                ("tau_err", c_float), ("target", c_void_p), ("image", KgsImage), ("dl_dcolor", c_void_p),
                ("view_loss", c_void_p), ("grads", KgsGrads), ("stats", KgsViewStats),
                ("zero_accumulators", c_int32), ("tau_d", c_float), ("state", KgsLifecycleState),
                ("decision", c_void_p), ("tau_p", c_double)]


_SIGS = {
    "kgs_config_default": (None, [P(KgsConfig), c_int32, c_int32]),
    "kgs_workspace_size": (c_int32, [P(KgsConfig), P(ctypes.c_size_t)]),
    "kgs_create": (c_int32, [P(KgsConfig), c_void_p, ctypes.c_size_t, P(c_void_p)]),
    "kgs_destroy": (c_int32, [c_void_p]),
    "kgs_set_tiling": (c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    "kgs_project": (c_int32, [c_void_p, P(KgsGaussians), c_void_p, c_int32, c_void_p, c_void_p]),
    "kgs_bin_sort": (c_int32, [c_void_p, c_void_p]),
    "kgs_render_fwd": (c_int32, [c_void_p, P(KgsImage), c_void_p]),
    "kgs_loss_l1": (c_int32, [c_void_p, c_void_p, P(KgsImage), c_void_p, c_void_p, c_void_p]),
    "kgs_loss_mapping": (c_int32, [c_void_p, c_int32, P(KgsImage), c_void_p, c_void_p, c_float, c_float, c_float,
                                   c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "kgs_loss_iso": (c_int32, [c_void_p, P(KgsGaussians), c_float, c_void_p, c_void_p, c_void_p]),
    "kgs_init_workspace_size": (c_int32, [c_int32, c_int32, c_int32, P(ctypes.c_size_t)]),
    "kgs_adam": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_float, c_float, c_float,
                           c_float, c_void_p]),
    "kgs_anchor_decode": (c_int32, [P(KgsAnchors), c_void_p, c_void_p, P(KgsGaussiansOut), c_void_p]),
    "kgs_anchor_stats": (c_int32, [c_void_p, P(KgsImage), c_void_p, c_int64, c_void_p, c_float, c_void_p, c_void_p,
                                   P(KgsViewStats), c_void_p, c_void_p]),
    "kgs_map_table_bytes": (c_int32, [c_int32, P(ctypes.c_size_t)]),
    "kgs_map_table_clear": (c_int32, [c_void_p, c_int32, c_void_p]),
    "kgs_map_workspace_size": (c_int32, [c_int64, P(ctypes.c_size_t)]),
    "kgs_map_voxel_keys": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "kgs_map_insert": (c_int32, [c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, ctypes.c_size_t, c_void_p]),
    "kgs_map_spawn": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64,
                                P(KgsGaussiansOut), c_void_p, c_void_p]),
    "kgs_map_densify_points": (c_int32, [P(KgsGaussians), c_void_p, P(c_double), c_int64, c_void_p, c_void_p,
                                         c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_size_t, c_void_p]),
    "kgs_map_compact": (c_int32, [P(KgsGaussians), c_void_p, c_void_p, P(KgsGaussiansOut), c_void_p]),
    "kgs_map_align": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "kgs_map_revoxelize": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, ctypes.c_size_t, c_void_p]),
    "kgs_init_spawn": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                 c_int32, c_void_p, ctypes.c_size_t, c_void_p, P(KgsSpawnList), c_void_p]),
    "kgs_render_bwd": (c_int32, [c_void_p, P(KgsGaussians), c_void_p, c_int32, c_void_p, P(KgsImage), c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_float, c_void_p, P(KgsGrads), P(KgsViewStats),
                                 c_void_p]),
    "kgs_render_bwd_pixels": (c_int32, [c_void_p, P(KgsImage), c_void_p, c_void_p, c_void_p, c_void_p, c_float,
                                        c_void_p]),
    "kgs_project_bwd": (c_int32, [c_void_p, P(KgsGaussians), c_void_p, c_int32, c_void_p, c_void_p, P(KgsGrads),
                                  P(KgsViewStats), c_void_p]),
    "kgs_accumulate_stats": (c_int32, [c_void_p, P(KgsViewStats), c_int64, c_int32, P(KgsLifecycleState), c_float,
                                       c_int32, c_void_p]),
    "kgs_accumulate_stats_static": (c_int32, [P(KgsViewStats), c_int64, c_int32, P(KgsLifecycleState), c_float,
                                              c_int32, c_void_p]),
    "kgs_densify_prune_decide": (c_int32, [c_void_p, P(KgsLifecycleState), c_int64, c_double, c_void_p, c_void_p,
                                           c_void_p, c_void_p]),
    "kgs_chunk_run": (c_int32, [c_void_p, P(KgsChunkDesc), c_void_p]),
    "kgs_chunk_capture": (c_int32, [c_void_p, P(KgsChunkDesc), P(c_void_p)]),
    "kgs_chunk_launch": (c_int32, [c_void_p, c_void_p]),
    "kgs_graph_destroy": (c_int32, [c_void_p]),
    "kgs_status_read": (c_int32, [c_void_p, P(ctypes.c_uint32)]),
    "kgs_status_clear": (c_int32, [c_void_p, c_void_p]),
    "kgs_counts_read": (c_int32, [c_void_p, P(c_int64), P(c_int64)]),
    "kgs_get_buffers": (c_int32, [c_void_p, P(KgsBuffers)]),
    "kgs_status_string": (ctypes.c_char_p, [c_int32]),
    "kgs_head_workspace_size": (c_int32, [P(ctypes.c_size_t)]),
    "kgs_head_features": (c_int32, [c_void_p, P(KgsGaussians), P(KgsViewStats), c_int32, c_void_p, c_void_p,
                                    c_void_p]),
    "kgs_head_forward": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "kgs_head_loss_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, ctypes.c_size_t,
                                     c_void_p, c_void_p, c_void_p]),
    "kgs_head_adam": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_float, c_float, c_float, c_float,
                                c_void_p]),
}

EXPORTED = tuple(_SIGS)

_lib = None


class KgsError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {_status_string(code)} ({code})")


def load(path: str = LIB_PATH):
    """Load libkgs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build the HIP library first "
                               "(python -m paper_2606_30436_amd.build_lib); there is no fallback")
        L = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _status_string(code: int) -> str:
    try:
        return load().kgs_status_string(code).decode()
    except Exception:  # pragma: no cover
        return "status"


def check(code: int, where: str):
    if code != KGS_OK:
        raise KgsError(code, where)


def ptr(t) -> int | None:
    """Device pointer of a tensor (None passes NULL)."""
    if t is None:
        return None
    return t.data_ptr()


def stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ wrappers
def kgs_config_default(width: int, height: int) -> KgsConfig:
    c = KgsConfig()
    load().kgs_config_default(ctypes.byref(c), width, height)
    return c


def kgs_workspace_size(cfg: KgsConfig) -> int:
    n = ctypes.c_size_t()
    check(load().kgs_workspace_size(ctypes.byref(cfg), ctypes.byref(n)), "kgs_workspace_size")
    return n.value


def kgs_create(cfg: KgsConfig, workspace, nbytes: int) -> int:
    h = c_void_p()
    check(load().kgs_create(ctypes.byref(cfg), ctypes.c_void_p(workspace.data_ptr()), nbytes, ctypes.byref(h)),
          "kgs_create")
    return h.value


def kgs_destroy(ctx: int):
    load().kgs_destroy(ctypes.c_void_p(ctx))


def kgs_set_tiling(ctx: int, tile_w: int, tile_h: int, batch: int):
    check(load().kgs_set_tiling(ctypes.c_void_p(ctx), tile_w, tile_h, batch), "kgs_set_tiling")


def kgs_project(ctx, g: KgsGaussians, cams, n_views, pose_xi=None, stream=None):
    check(load().kgs_project(ctypes.c_void_p(ctx), ctypes.byref(g), ptr(cams), n_views, ptr(pose_xi),
                             stream_handle(stream)), "kgs_project")


def kgs_bin_sort(ctx, stream=None):
    check(load().kgs_bin_sort(ctypes.c_void_p(ctx), stream_handle(stream)), "kgs_bin_sort")


def kgs_render_fwd(ctx, img: KgsImage, stream=None):
    check(load().kgs_render_fwd(ctypes.c_void_p(ctx), ctypes.byref(img), stream_handle(stream)), "kgs_render_fwd")


def kgs_loss_l1(ctx, target, img: KgsImage, dl_dcolor, view_loss, stream=None):
    check(load().kgs_loss_l1(ctypes.c_void_p(ctx), ptr(target), ctypes.byref(img), ptr(dl_dcolor), ptr(view_loss),
                             stream_handle(stream)), "kgs_loss_l1")


def kgs_loss_mapping(ctx, n_views, img: KgsImage, target, target_depth, w_l1, w_ssim, lambda_g, dl_dcolor, dl_ddepth,
                     view_loss, geo_loss, stream=None):
    check(load().kgs_loss_mapping(ctypes.c_void_p(ctx), int(n_views), ctypes.byref(img), ptr(target), ptr(target_depth),
                                  float(w_l1), float(w_ssim), float(lambda_g), ptr(dl_dcolor), ptr(dl_ddepth),
                                  ptr(view_loss), ptr(geo_loss), stream_handle(stream)), "kgs_loss_mapping")


def kgs_loss_iso(ctx, g: KgsGaussians, lambda_iso, grad_log_scales, loss, stream=None):
    check(load().kgs_loss_iso(ctypes.c_void_p(ctx), ctypes.byref(g), float(lambda_iso), ptr(grad_log_scales), ptr(loss),
                              stream_handle(stream)), "kgs_loss_iso")


def kgs_init_workspace_size(width, height, n_views) -> int:
    n = ctypes.c_size_t()
    check(load().kgs_init_workspace_size(int(width), int(height), int(n_views), ctypes.byref(n)),
          "kgs_init_workspace_size")
    return int(n.value)


def kgs_init_spawn(color, depth, rendered, rendered_depth, uniforms, cams, n_views, width, height, workspace,
                   workspace_bytes, p_kf, out: KgsSpawnList, stream=None):
    check(load().kgs_init_spawn(ptr(color), ptr(depth), ptr(rendered), ptr(rendered_depth), ptr(uniforms), ptr(cams),
                                int(n_views), int(width), int(height), ptr(workspace), int(workspace_bytes), ptr(p_kf),
                                ctypes.byref(out), stream_handle(stream)), "kgs_init_spawn")


def kgs_adam(theta, m, v, grad, n, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(load().kgs_adam(ptr(theta), ptr(m), ptr(v), ptr(grad), int(n), int(step), float(lr), float(beta1),
                          float(beta2), float(eps), stream_handle(stream)), "kgs_adam")


def kgs_anchor_decode(a: KgsAnchors, theta, camera, out: KgsGaussiansOut, stream=None):
    check(load().kgs_anchor_decode(ctypes.byref(a), ptr(theta), ptr(camera), ctypes.byref(out), stream_handle(stream)),
          "kgs_anchor_decode")


def kgs_anchor_stats(ctx, img: KgsImage, anchor_of, n_anchors, target, tau_err, view_loss, counts,
                     stats: KgsViewStats, status, stream=None):
    check(load().kgs_anchor_stats(ctypes.c_void_p(ctx), ctypes.byref(img), ptr(anchor_of), int(n_anchors), ptr(target),
                                  float(tau_err), ptr(view_loss), ptr(counts), ctypes.byref(stats), ptr(status),
                                  stream_handle(stream)), "kgs_anchor_stats")


def kgs_map_table_bytes(log2_capacity) -> int:
    n = ctypes.c_size_t()
    check(load().kgs_map_table_bytes(int(log2_capacity), ctypes.byref(n)), "kgs_map_table_bytes")
    return int(n.value)


def kgs_map_table_clear(table, log2_capacity, stream=None):
    check(load().kgs_map_table_clear(ptr(table), int(log2_capacity), stream_handle(stream)), "kgs_map_table_clear")


def kgs_map_workspace_size(max_items) -> int:
    n = ctypes.c_size_t()
    check(load().kgs_map_workspace_size(int(max_items), ctypes.byref(n)), "kgs_map_workspace_size")
    return int(n.value)


def kgs_map_voxel_keys(level, voxel, n, keys, stream=None):
    check(load().kgs_map_voxel_keys(ptr(level), ptr(voxel), int(n), ptr(keys), stream_handle(stream)),
          "kgs_map_voxel_keys")


def kgs_map_insert(table, log2_capacity, keys, n, n_in, anchor, created, n_out, status, workspace, ws_bytes,
                   stream=None):
    check(load().kgs_map_insert(ptr(table), int(log2_capacity), ptr(keys), int(n), ptr(n_in), ptr(anchor), ptr(created),
                                ptr(n_out), ptr(status), ptr(workspace), int(ws_bytes), stream_handle(stream)),
          "kgs_map_insert")


def kgs_map_spawn(created, n_in, n_out, level, voxel, color, n_candidates, out: KgsGaussiansOut, status, stream=None):
    check(load().kgs_map_spawn(ptr(created), ptr(n_in), ptr(n_out), ptr(level), ptr(voxel), ptr(color),
                               int(n_candidates), ctypes.byref(out), ptr(status), stream_handle(stream)), "kgs_map_spawn")


def kgs_map_densify_points(g: KgsGaussians, decision, centre, capacity, level, voxel, point, source, count, workspace,
                           ws_bytes, stream=None):
    c = (c_double * 3)(*[float(x) for x in centre])
    check(load().kgs_map_densify_points(ctypes.byref(g), ptr(decision), c, int(capacity), ptr(level), ptr(voxel),
                                        ptr(point), ptr(source), ptr(count), ptr(workspace), int(ws_bytes),
                                        stream_handle(stream)), "kgs_map_densify_points")


def kgs_map_compact(g: KgsGaussians, decision, keep_map, out: KgsGaussiansOut, stream=None):
    check(load().kgs_map_compact(ctypes.byref(g), ptr(decision), ptr(keep_map), ctypes.byref(out),
                                 stream_handle(stream)), "kgs_map_compact")


def kgs_map_align(means, quats, n, keyframe_of, old_poses, new_poses, n_keyframes, stream=None):
    check(load().kgs_map_align(ptr(means), ptr(quats), int(n), ptr(keyframe_of), ptr(old_poses), ptr(new_poses),
                               int(n_keyframes), stream_handle(stream)), "kgs_map_align")


def kgs_map_revoxelize(means, level, n, table, log2_capacity, keep, anchor, n_keep, status, workspace, ws_bytes,
                       stream=None):
    check(load().kgs_map_revoxelize(ptr(means), ptr(level), int(n), ptr(table), int(log2_capacity), ptr(keep),
                                    ptr(anchor), ptr(n_keep), ptr(status), ptr(workspace), int(ws_bytes),
                                    stream_handle(stream)), "kgs_map_revoxelize")


def kgs_render_bwd(ctx, g: KgsGaussians, cams, n_views, pose_xi, img: KgsImage, dl_dcolor, dl_ddepth, dl_dtfinal,
                   target, tau_err, view_loss, grads: KgsGrads, stats: KgsViewStats | None, stream=None):
    check(load().kgs_render_bwd(ctypes.c_void_p(ctx), ctypes.byref(g), ptr(cams), n_views, ptr(pose_xi),
                                ctypes.byref(img), ptr(dl_dcolor), ptr(dl_ddepth), ptr(dl_dtfinal), ptr(target),
                                float(tau_err),
                                ptr(view_loss), ctypes.byref(grads),
                                ctypes.byref(stats) if stats is not None else None, stream_handle(stream)),
          "kgs_render_bwd")


def kgs_render_bwd_pixels(ctx, img: KgsImage, dl_dcolor, dl_ddepth, dl_dtfinal, target, tau_err, stream=None):
    check(load().kgs_render_bwd_pixels(ctypes.c_void_p(ctx), ctypes.byref(img), ptr(dl_dcolor), ptr(dl_ddepth),
                                       ptr(dl_dtfinal), ptr(target), float(tau_err), stream_handle(stream)),
          "kgs_render_bwd_pixels")


def kgs_project_bwd(ctx, g: KgsGaussians, cams, n_views, pose_xi, view_loss, grads: KgsGrads,
                    stats: KgsViewStats | None, stream=None):
    check(load().kgs_project_bwd(ctypes.c_void_p(ctx), ctypes.byref(g), ptr(cams), n_views, ptr(pose_xi),
                                 ptr(view_loss), ctypes.byref(grads), ctypes.byref(stats) if stats is not None else None,
                                 stream_handle(stream)), "kgs_project_bwd")


def kgs_accumulate_stats(ctx, stats: KgsViewStats, n, n_views, state: KgsLifecycleState, tau_d, reset=0,
                         stream=None):
    check(load().kgs_accumulate_stats(ctypes.c_void_p(ctx), ctypes.byref(stats), n, n_views, ctypes.byref(state),
                                      float(tau_d), int(reset), stream_handle(stream)), "kgs_accumulate_stats")


ACCUMULATE_STATIC_MAX_N = 16776960


def kgs_accumulate_stats_static(stats: KgsViewStats, n, n_views, state: KgsLifecycleState, tau_d, reset=0,
                                stream=None):
    check(load().kgs_accumulate_stats_static(ctypes.byref(stats), n, n_views, ctypes.byref(state), float(tau_d),
                                             int(reset), stream_handle(stream)), "kgs_accumulate_stats_static")


def kgs_densify_prune_decide(ctx, state: KgsLifecycleState, n, tau_p, decision, keep_map=None, n_keep=None,
                             stream=None):
    check(load().kgs_densify_prune_decide(ctypes.c_void_p(ctx), ctypes.byref(state), n, float(tau_p), ptr(decision),
                                          ptr(keep_map), ptr(n_keep), stream_handle(stream)),
          "kgs_densify_prune_decide")


def kgs_chunk_run(ctx, desc: KgsChunkDesc, stream=None):
    check(load().kgs_chunk_run(ctypes.c_void_p(ctx), ctypes.byref(desc), stream_handle(stream)), "kgs_chunk_run")


def kgs_chunk_capture(ctx, desc: KgsChunkDesc) -> int:
    h = c_void_p()
    check(load().kgs_chunk_capture(ctypes.c_void_p(ctx), ctypes.byref(desc), ctypes.byref(h)), "kgs_chunk_capture")
    return h.value


def kgs_chunk_launch(graph: int, stream=None):
    check(load().kgs_chunk_launch(ctypes.c_void_p(graph), stream_handle(stream)), "kgs_chunk_launch")


def kgs_graph_destroy(graph: int):
    load().kgs_graph_destroy(ctypes.c_void_p(graph))


def kgs_status_read(ctx) -> int:
    f = ctypes.c_uint32()
    check(load().kgs_status_read(ctypes.c_void_p(ctx), ctypes.byref(f)), "kgs_status_read")
    return f.value


def kgs_status_clear(ctx, stream=None):
    check(load().kgs_status_clear(ctypes.c_void_p(ctx), stream_handle(stream)), "kgs_status_clear")


def kgs_counts_read(ctx):
    a, b = c_int64(), c_int64()
    check(load().kgs_counts_read(ctypes.c_void_p(ctx), ctypes.byref(a), ctypes.byref(b)), "kgs_counts_read")
    return a.value, b.value


def kgs_get_buffers(ctx) -> KgsBuffers:
    b = KgsBuffers()
    check(load().kgs_get_buffers(ctypes.c_void_p(ctx), ctypes.byref(b)), "kgs_get_buffers")
    return b


# ---------------------------------------------------------------- learned head
HEAD_FEATURES = 16
HEAD_PARAMS = 5443


def kgs_head_workspace_size() -> int:
    b = ctypes.c_size_t()
    check(load().kgs_head_workspace_size(ctypes.byref(b)), "kgs_head_workspace_size")
    return b.value


def kgs_head_features(ctx, g: KgsGaussians, stats: KgsViewStats, n_views, before, features, stream=None):
    check(load().kgs_head_features(ctypes.c_void_p(ctx), ctypes.byref(g), ctypes.byref(stats), int(n_views),
                                   ctypes.byref(before) if before is not None else None, ptr(features),
                                   stream_handle(stream)), "kgs_head_features")


def kgs_head_forward(theta, features, n, logits=None, decision=None, stream=None):
    check(load().kgs_head_forward(ptr(theta), ptr(features), int(n), ptr(logits), ptr(decision),
                                  stream_handle(stream)), "kgs_head_forward")


def kgs_head_loss_grad(theta, features, labels, n, class_w, workspace, ws_bytes, grad, loss, stream=None):
    check(load().kgs_head_loss_grad(ptr(theta), ptr(features), ptr(labels), int(n), ptr(class_w), ptr(workspace),
                                    int(ws_bytes), ptr(grad), ptr(loss), stream_handle(stream)), "kgs_head_loss_grad")


def kgs_head_adam(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(load().kgs_head_adam(ptr(theta), ptr(m), ptr(v), ptr(grad), int(step), float(lr), float(beta1),
                               float(beta2), float(eps), stream_handle(stream)), "kgs_head_adam")
