"""Device-side front end of libkgs: a context over a torch-allocated workspace
and thin methods that marshal torch tensors into the C calls.  Every step
runs in the HIP kernels of libkgs.so; torch only provides memory and streams.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from .scenes import CAMERA_DTYPE

TILE_SHAPES = ((16, 16), (8, 32), (32, 8), (32, 16), (16, 32))
BATCHES = (32, 64, 128)


def tiling_valid(tile, batch) -> bool:
    """The library's rule: 512-pixel tiles stage at most 64 records at a time."""
    return tuple(tile) in TILE_SHAPES and batch in BATCHES and not (tile[0] * tile[1] == 512 and batch > 64)


@dataclasses.dataclass
class GaussianParams:
    """SoA Gaussian parameters on the device (float32, contiguous)."""
    means: torch.Tensor        # [3, N]
    log_scales: torch.Tensor   # [3, N]
    quats: torch.Tensor        # [4, N]
    logits: torch.Tensor       # [N]
    sh: torch.Tensor           # [K, 3, N]
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def c(self) -> L.KgsGaussians:
        g = L.KgsGaussians()
        g.means, g.log_scales, g.quats = self.means.data_ptr(), self.log_scales.data_ptr(), self.quats.data_ptr()
        g.opacity_logits, g.sh = self.logits.data_ptr(), self.sh.data_ptr()
        g.n, g.sh_degree = self.n, self.sh_degree
        return g

    @staticmethod
    def from_scene(scene, device="cuda") -> "GaussianParams":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return GaussianParams(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.logits), t(scene.sh),
                              scene.sh_degree)

    def zeros_like(self) -> "GaussianParams":
        return GaussianParams(torch.zeros_like(self.means), torch.zeros_like(self.log_scales),
                              torch.zeros_like(self.quats), torch.zeros_like(self.logits), torch.zeros_like(self.sh),
                              self.sh_degree)


def device_cameras(cams: np.ndarray, device="cuda") -> torch.Tensor:
    """CAMERA_DTYPE records as raw device bytes laid out as kgs_camera."""
    assert cams.dtype == CAMERA_DTYPE
    return torch.from_numpy(np.ascontiguousarray(cams).view(np.uint8).copy()).to(device)


@dataclasses.dataclass
class Image:
    color: torch.Tensor    # [V, 3, H, W]
    depth: torch.Tensor    # [V, H, W]
    t_final: torch.Tensor  # [V, H, W]
    last: torch.Tensor     # [V, H, W] int32

    def c(self) -> L.KgsImage:
        im = L.KgsImage()
        im.color, im.depth = self.color.data_ptr(), self.depth.data_ptr()
        im.t_final, im.last = self.t_final.data_ptr(), self.last.data_ptr()
        return im

    @staticmethod
    def empty(V, H, W, device="cuda") -> "Image":
        return Image(torch.empty(V, 3, H, W, device=device), torch.empty(V, H, W, device=device),
                     torch.empty(V, H, W, device=device), torch.empty(V, H, W, dtype=torch.int32, device=device))


@dataclasses.dataclass
class ViewStats:
    """Per-Gaussian chunk accumulators (kgs_view_stats)."""
    kappa_sum: torch.Tensor
    omega_sum: torch.Tensor
    gamma_sum: torch.Tensor
    grad_norm_sum: torch.Tensor
    view_count: torch.Tensor
    max_radius: torch.Tensor

    @staticmethod
    def zeros(n, device="cuda") -> "ViewStats":
        return ViewStats(torch.zeros(n, dtype=torch.int32, device=device), torch.zeros(n, dtype=torch.int32, device=device),
                         torch.zeros(n, dtype=torch.float64, device=device), torch.zeros(n, device=device),
                         torch.zeros(n, dtype=torch.int32, device=device), torch.zeros(n, dtype=torch.int32, device=device))

    def c(self) -> L.KgsViewStats:
        s = L.KgsViewStats()
        s.kappa_sum, s.omega_sum, s.gamma_sum = self.kappa_sum.data_ptr(), self.omega_sum.data_ptr(), self.gamma_sum.data_ptr()
        s.grad_norm_sum, s.view_count, s.max_radius = (self.grad_norm_sum.data_ptr(), self.view_count.data_ptr(),
                                                       self.max_radius.data_ptr())
        return s


@dataclasses.dataclass
class LifecycleState:
    densify: torch.Tensor      # uint8 [N]
    prune_score: torch.Tensor  # float64 [N]

    @staticmethod
    def zeros(n, device="cuda") -> "LifecycleState":
        return LifecycleState(torch.zeros(n, dtype=torch.uint8, device=device),
                              torch.zeros(n, dtype=torch.float64, device=device))

    def c(self) -> L.KgsLifecycleState:
        s = L.KgsLifecycleState()
        s.densify, s.prune_score = self.densify.data_ptr(), self.prune_score.data_ptr()
        return s


def grads_c(g: Optional[GaussianParams], pose: Optional[torch.Tensor]) -> L.KgsGrads:
    out = L.KgsGrads()
    if g is not None:
        out.means, out.log_scales, out.quats = g.means.data_ptr(), g.log_scales.data_ptr(), g.quats.data_ptr()
        out.opacity_logits, out.sh = g.logits.data_ptr(), g.sh.data_ptr()
    if pose is not None:
        out.pose_xi = pose.data_ptr()
    return out


class Rasterizer:
    """One libkgs context and its workspace."""

    def __init__(self, width: int, height: int, max_views: int, max_gaussians: int, slot_capacity: int = 0,
                 pair_capacity: int = 0, tile=(16, 16), batch: int = 64, device="cuda", **overrides):
        cfg = L.kgs_config_default(width, height)
        cfg.tile_w, cfg.tile_h = tile
        cfg.batch = batch
        cfg.max_views = max_views
        cfg.max_gaussians = max_gaussians
        cfg.slot_capacity = slot_capacity or max(1, max_views * max_gaussians)
        cfg.pair_capacity = pair_capacity or min(2 ** 32 - 1, max(1024, 8 * cfg.slot_capacity))
        for k, v in overrides.items():
            if k == "bg":
                for i in range(3):
                    cfg.bg[i] = float(v[i])
            else:
                setattr(cfg, k, v)
        self.cfg = cfg
        self.device = device
        self.ws_bytes = L.kgs_workspace_size(cfg)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.ctx = L.kgs_create(cfg, self.workspace, self.ws_bytes)
        self.graphs = []
        self.generation = 0  # bumped by every project(): the workspace then holds new records

    def close(self):
        for g in self.graphs:
            L.kgs_graph_destroy(g)
        self.graphs = []
        if getattr(self, "ctx", None):
            L.kgs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def width(self):
        return self.cfg.width

    @property
    def height(self):
        return self.cfg.height

    def set_tiling(self, tile, batch):
        L.kgs_set_tiling(self.ctx, tile[0], tile[1], batch)
        self.cfg.tile_w, self.cfg.tile_h = tile
        self.cfg.batch = batch

    # ---------------------------------------------------------- the steps
    def project(self, g: GaussianParams, cams: torch.Tensor, pose_xi: Optional[torch.Tensor] = None, stream=None):
        V = cams.numel() // CAMERA_DTYPE.itemsize
        L.kgs_project(self.ctx, g.c(), cams, V, pose_xi, stream)
        self.generation += 1
        return V

    def bin_sort(self, stream=None):
        L.kgs_bin_sort(self.ctx, stream)

    def render_fwd(self, img: Image, stream=None):
        L.kgs_render_fwd(self.ctx, img.c(), stream)

    def loss_l1(self, target, img: Image, dl_dcolor, view_loss, stream=None):
        L.kgs_loss_l1(self.ctx, target, img.c(), dl_dcolor, view_loss, stream)

    def loss_mapping(self, n_views, img: Image, target, dl_dcolor, view_loss, target_depth=None, dl_ddepth=None,
                     geo_loss=None, w_l1=0.8, w_ssim=0.2, lambda_g=0.01, stream=None):
        L.kgs_loss_mapping(self.ctx, n_views, img.c(), target, target_depth, w_l1, w_ssim, lambda_g, dl_dcolor,
                           dl_ddepth, view_loss, geo_loss, stream)

    def loss_iso(self, g: GaussianParams, loss, grad_log_scales=None, lambda_iso=10.0, stream=None):
        L.kgs_loss_iso(self.ctx, g.c(), lambda_iso, grad_log_scales, loss, stream)

    def render_bwd(self, g: GaussianParams, cams, pose_xi, img: Image, dl_dcolor, dl_ddepth=None, target=None,
                   tau_err=0.1, view_loss=None, grads: Optional[GaussianParams] = None, pose_grad=None,
                   stats: Optional[ViewStats] = None, stream=None, dl_dtfinal=None):
        V = cams.numel() // CAMERA_DTYPE.itemsize
        L.kgs_render_bwd(self.ctx, g.c(), cams, V, pose_xi, img.c(), dl_dcolor, dl_ddepth, dl_dtfinal, target, tau_err,
                         view_loss, grads_c(grads, pose_grad), stats.c() if stats is not None else None, stream)

    def render_bwd_pixels(self, img: Image, dl_dcolor, dl_ddepth=None, target=None, tau_err=0.1, stream=None,
                          dl_dtfinal=None):
        L.kgs_render_bwd_pixels(self.ctx, img.c(), dl_dcolor, dl_ddepth, dl_dtfinal, target, tau_err, stream)

    def project_bwd(self, g: GaussianParams, cams, pose_xi, view_loss=None, grads: Optional[GaussianParams] = None,
                    pose_grad=None, stats: Optional[ViewStats] = None, stream=None):
        V = cams.numel() // CAMERA_DTYPE.itemsize
        L.kgs_project_bwd(self.ctx, g.c(), cams, V, pose_xi, view_loss, grads_c(grads, pose_grad),
                          stats.c() if stats is not None else None, stream)

    def accumulate_stats(self, stats: ViewStats, n_views: int, state: LifecycleState, tau_d=5.0, reset=True,
                         stream=None):
        L.kgs_accumulate_stats(self.ctx, stats.c(), stats.kappa_sum.numel(), n_views, state.c(), tau_d,
                               int(reset), stream)

    def decide(self, state: LifecycleState, tau_p=0.99, keep_map=True, stream=None):
        n = state.densify.numel()
        dec = torch.empty(n, dtype=torch.uint8, device=self.device)
        km = torch.empty(n, dtype=torch.int32, device=self.device) if keep_map else None
        nk = torch.zeros(1, dtype=torch.int32, device=self.device) if keep_map else None
        L.kgs_densify_prune_decide(self.ctx, state.c(), n, tau_p, dec, km, nk, stream)
        return dec, km, nk

    # ---------------------------------------------------------- readback
    def counts(self):
        return L.kgs_counts_read(self.ctx)

    def status(self) -> int:
        return L.kgs_status_read(self.ctx)

    def status_clear(self, stream=None):
        L.kgs_status_clear(self.ctx, stream)

    def buffers(self) -> dict:
        """Copies of the slot and pair buffers of the last project/bin_sort."""
        b = L.kgs_get_buffers(self.ctx)
        ns, npairs = self.counts()
        dev = torch.device(self.device)

        def grab(addr, count, dtype, width=1):
            if count == 0:
                return torch.empty((0, width) if width > 1 else (0,), dtype=dtype)
            nbytes = count * width * torch.tensor([], dtype=dtype).element_size()
            u8 = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            torch.cuda.synchronize()
            _copy_device(u8.data_ptr(), addr, nbytes)
            t = u8.view(dtype)
            return (t.view(count, width) if width > 1 else t).cpu()
        out = dict(n_slots=ns, n_pairs=npairs,
                   slot_rec=grab(b.slot_rec, ns, torch.float32, 16), slot_gid=grab(b.slot_gid, ns, torch.int32),
                   slot_view=grab(b.slot_view, ns, torch.int32), slot_pix=grab(b.slot_pix, ns, torch.int32, 4),
                   slot_pairoff=grab(b.slot_pairoff, ns, torch.int32), keys=grab(b.keys, npairs, torch.int32),
                   sorted_slot=grab(b.sorted_slot, npairs, torch.int32),
                   ranges=grab(b.ranges, b.n_views * b.tiles_x * b.tiles_y, torch.int32, 2),
                   tiles_x=b.tiles_x, tiles_y=b.tiles_y, tile_bits=b.tile_bits, n_views=b.n_views)
        return out

    # ---------------------------------------------------------- chunk
    def chunk_desc(self, g: GaussianParams, cams, pose_xi, target, img: Image, dl_dcolor, view_loss,
                   grads: Optional[GaussianParams], pose_grad, stats: Optional[ViewStats], tau_err=0.1,
                   zero_accumulators=False, state: Optional[LifecycleState] = None, decision=None, tau_d=5.0,
                   tau_p=0.99):
        d = L.KgsChunkDesc()
        d.gaussians = g.c()
        d.cams = cams.data_ptr()
        d.pose_xi = pose_xi.data_ptr() if pose_xi is not None else None
        d.n_views = cams.numel() // CAMERA_DTYPE.itemsize
        d.tau_err = tau_err
        d.target = target.data_ptr()
        d.image = img.c()
        d.dl_dcolor = dl_dcolor.data_ptr()
        d.view_loss = view_loss.data_ptr()
        d.grads = grads_c(grads, pose_grad)
        d.stats = stats.c() if stats is not None else L.KgsViewStats()
        d.zero_accumulators = int(bool(zero_accumulators))
        d.tau_d = tau_d
        d.state = state.c() if state is not None else L.KgsLifecycleState()
        d.decision = decision.data_ptr() if decision is not None else None
        d.tau_p = tau_p
        return d

    def chunk_run(self, desc, stream=None):
        L.kgs_chunk_run(self.ctx, desc, stream)

    def chunk_capture(self, desc) -> int:
        h = L.kgs_chunk_capture(self.ctx, desc)
        self.graphs.append(h)
        return h

    def chunk_launch(self, graph: int, stream=None):
        L.kgs_chunk_launch(graph, stream)

    def chunk_release(self, graph: int):
        """Destroy one captured chunk (e.g. after a tiling change made it stale)."""
        self.graphs.remove(graph)
        L.kgs_graph_destroy(graph)


def _copy_device(dst: int, src: int, nbytes: int):
    """Device-to-device byte copy through torch (marshalling of workspace views)."""
    import ctypes
    hip = _hip()
    r = hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes), 3)
    if r != 0:
        raise RuntimeError(f"hipMemcpy failed ({r})")


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        import ctypes
        _hip_lib = ctypes.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.restype = ctypes.c_int
        _hip_lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _hip_lib
