"""Python side of the mapping-step entry points next to the rasterizer: the
probabilistic initialisation of new Gaussians (kgs_init_spawn) and the map
maintenance calls.  Argument marshalling only: every step runs in libkgs."""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import _lib as L


@dataclasses.dataclass
class SpawnList:
    """Device outputs of kgs_init_spawn (see kgs_spawn_list in kgs.h)."""
    pixel: torch.Tensor   # int32 [cap][2]: keyframe, y * W + x
    level: torch.Tensor   # int32 [cap]
    voxel: torch.Tensor   # int32 [cap][3]
    point: torch.Tensor   # float32 [cap][3]
    color: torch.Tensor   # float32 [cap][3]
    count: torch.Tensor   # uint32-valued int32 [1]

    @staticmethod
    def empty(capacity: int, device="cuda") -> "SpawnList":
        cap = max(int(capacity), 1)
        i32 = dict(dtype=torch.int32, device=device)
        return SpawnList(torch.empty(cap, 2, **i32), torch.empty(cap, **i32), torch.empty(cap, 3, **i32),
                         torch.empty(cap, 3, device=device), torch.empty(cap, 3, device=device),
                         torch.zeros(1, **i32))

    def c(self, capacity: int) -> L.KgsSpawnList:
        s = L.KgsSpawnList()
        s.pixel, s.level, s.voxel = self.pixel.data_ptr(), self.level.data_ptr(), self.voxel.data_ptr()
        s.point, s.color, s.count = self.point.data_ptr(), self.color.data_ptr(), self.count.data_ptr()
        s.capacity = int(capacity)
        return s


class Initializer:
    """kgs_init_spawn over keyframes of one size, with its workspace."""

    def __init__(self, width: int, height: int, max_views: int, device="cuda"):
        self.W, self.H, self.V = int(width), int(height), int(max_views)
        self.ws_bytes = L.kgs_init_workspace_size(self.W, self.H, self.V)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def spawn(self, color, depth, uniforms, cams, out: SpawnList, capacity: int, rendered=None, rendered_depth=None,
              p_kf=None, stream=None):
        V = int(color.shape[0])
        assert 1 <= V <= self.V and tuple(color.shape[1:]) == (3, self.H, self.W)
        L.kgs_init_spawn(color, depth, rendered, rendered_depth, uniforms, cams, V, self.W, self.H, self.workspace,
                         self.ws_bytes, p_kf, out.c(capacity), stream)


def gaussians_out(means, log_scales, quats, logits, sh, sh_degree: int) -> L.KgsGaussiansOut:
    """Writable structure-of-arrays Gaussians (capacity = the planes' length)."""
    o = L.KgsGaussiansOut()
    o.means, o.log_scales, o.quats = means.data_ptr(), log_scales.data_ptr(), quats.data_ptr()
    o.opacity_logits, o.sh = logits.data_ptr(), sh.data_ptr()
    o.n, o.sh_degree = int(means.shape[-1]), int(sh_degree)
    return o


class VoxelMap:
    """The spatial hash of occupied voxels and the workspace of the map calls."""

    def __init__(self, log2_capacity: int, max_items: int, device="cuda"):
        self.log2 = int(log2_capacity)
        self.table = torch.empty(L.kgs_map_table_bytes(self.log2), dtype=torch.uint8, device=device)
        self.ws_bytes = L.kgs_map_workspace_size(max_items)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.max_items = int(max_items)
        self.clear()

    def clear(self, stream=None):
        L.kgs_map_table_clear(self.table, self.log2, stream)

    def keys(self, level, voxel, stream=None):
        out = torch.empty(int(level.shape[0]), dtype=torch.int64, device=level.device)
        L.kgs_map_voxel_keys(level, voxel, int(level.shape[0]), out, stream)
        return out

    def insert(self, keys, n_in, n_out, anchor=None, created=None, stream=None):
        n = int(keys.shape[0])
        assert n <= self.max_items
        L.kgs_map_insert(self.table, self.log2, keys, n, n_in, anchor, created, n_out, self.status, self.workspace,
                         self.ws_bytes, stream)

    def densify_points(self, g, decision, centre, capacity, level, voxel, point, source, count, stream=None):
        assert g.n <= self.max_items
        L.kgs_map_densify_points(g.c(), decision, centre, capacity, level, voxel, point, source, count,
                                 self.workspace, self.ws_bytes, stream)

    def revoxelize(self, means, level, keep, anchor, n_keep, stream=None):
        n = int(means.shape[-1])
        assert n <= self.max_items
        L.kgs_map_revoxelize(means, level, n, self.table, self.log2, keep, anchor, n_keep, self.status, self.workspace,
                             self.ws_bytes, stream)


@dataclasses.dataclass
class Anchors:
    """Device anchors (kgs_anchors): p [3][A], feat [A][32], log_l [3][A], offsets [K][3][A], level [A]."""
    p: torch.Tensor
    feat: torch.Tensor
    log_l: torch.Tensor
    offsets: torch.Tensor
    level: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.p.shape[1])

    @property
    def k(self) -> int:
        return int(self.offsets.shape[0])

    @staticmethod
    def from_arrays(p, feat, log_l, offsets, level, device="cuda") -> "Anchors":
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return Anchors(f(p), f(feat), f(log_l), f(offsets),
                       torch.from_numpy(np.ascontiguousarray(level, np.int32)).to(device))

    def c(self) -> L.KgsAnchors:
        a = L.KgsAnchors()
        a.p, a.feat, a.log_l = self.p.data_ptr(), self.feat.data_ptr(), self.log_l.data_ptr()
        a.offsets, a.level, a.n, a.k = self.offsets.data_ptr(), self.level.data_ptr(), self.n, self.k
        return a


def decode_anchors(anchors: Anchors, theta, camera, out, stream=None):
    """kgs_anchor_decode into a degree-0 GaussianParams `out` of at least A K Gaussians."""
    o = gaussians_out(out.means, out.log_scales, out.quats, out.logits, out.sh, 0)
    L.kgs_anchor_decode(anchors.c(), theta, camera, o, stream)


def anchor_stats(R, img, anchor_of, n_anchors, target, view_loss, counts, stats, status, tau_err=0.1, stream=None):
    """kgs_anchor_stats for the views R last rendered."""
    L.kgs_anchor_stats(R.ctx, img.c(), anchor_of, n_anchors, target, tau_err, view_loss, counts, stats.c(), status,
                       stream)
