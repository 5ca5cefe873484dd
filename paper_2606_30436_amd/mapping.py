"""Python side of the mapping-step entry points next to the rasterizer: the
probabilistic initialisation of new Gaussians (kgs_init_spawn) and the map
maintenance calls.  Argument marshalling only: every step runs in libkgs."""
from __future__ import annotations

import dataclasses

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
