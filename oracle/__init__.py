"""FP64 CPU oracle of the rasterizer and of the lifecycle statistics.

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  It shares no code with the HIP path
(paper_2606_30436_amd); both read the same seeded scenes.

Modules
  kgs_oracle.c   projection, binning contract, compositing, analytic backward,
                 per-view footprint / error statistics (C, FP64, OpenMP)
  lifecycle.py   chunk scores, global OR / max rules and the decision (NumPy FP64)
  brute.py       tile-free compositing in plain PyTorch FP64 with autograd
  mlp.py         the prune/keep/densify network with BF16 rounding, FP64 GEMMs
  mapping_loss.py  the mapping loss (L1 + D-SSIM, depth L1, isotropy) and its
                 gradients in plain PyTorch FP64
  init_prob.py   probabilistic initialisation (DoG, depth gradient, residual
                 against the render, 3x3 suppression, unprojection, level and
                 voxel quantisation) in NumPy FP64
  map_maint.py   map maintenance: voxel keys and the spatial-hash insertion of
                 new anchors, their attributes, densify points, prune
                 compaction, rigid alignment and re-voxelisation
  anchors.py     anchor decoding (the decoder network with BF16 rounding
                 points, position and scale composition, the level-of-detail
                 opacity mask); the per-anchor union footprint statistics are
                 View.anchor_stats in the C oracle
  optim.py       Adam with bias correction (the map's gradient steps)

Every function cites the passage of the paper it follows; readings of passages
the paper leaves open are the constants of OracleConfig.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kgs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class _Cfg(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("t_min", ctypes.c_double), ("near_z", ctypes.c_double), ("eps2d", ctypes.c_double),
                ("guard", ctypes.c_double), ("rect_margin", ctypes.c_double), ("far_z", ctypes.c_double),
                ("bg", ctypes.c_double * 3), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32)]


P = ctypes.POINTER
_d = P(ctypes.c_double)
_f = P(ctypes.c_float)
_i32 = P(ctypes.c_int32)
_i64 = P(ctypes.c_int64)
_u32 = P(ctypes.c_uint32)
_u64 = P(ctypes.c_uint64)
_u8 = P(ctypes.c_uint8)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = ctypes.CDLL(build())
            L.orc_view_create.restype = ctypes.c_void_p
            L.orc_view_create.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d, _d, _d,
                                          P(_Camera), _d, P(_Cfg)]
            L.orc_view_free.argtypes = [ctypes.c_void_p]
            L.orc_view_n_visible.restype = ctypes.c_int64
            L.orc_view_n_visible.argtypes = [ctypes.c_void_p]
            L.orc_view_n_pairs.restype = ctypes.c_int64
            L.orc_view_n_pairs.argtypes = [ctypes.c_void_p]
            L.orc_view_image.argtypes = [ctypes.c_void_p, _d, _d, _d, _i32, _i32, _d]
            L.orc_view_gauss_margins.argtypes = [ctypes.c_void_p, _d]
            L.orc_view_proj.argtypes = [ctypes.c_void_p, _d, _i64, _d]
            L.orc_view_pairs.argtypes = [ctypes.c_void_p, _i32, _i64]
            L.orc_view_stats.argtypes = [ctypes.c_void_p, _f, ctypes.c_double, _i32, _i32, _u8, _d]
            L.orc_view_anchor_stats.argtypes = [ctypes.c_void_p, _i64, ctypes.c_int64, _f, ctypes.c_double, _i64,
                                                _i64]
            L.orc_view_backward.argtypes = [ctypes.c_void_p, _d, _d, _d, _d, _d, _d, _d, _d, _d]
            L.orc_se3_exp.argtypes = [_d, _d]
            L.orc_se3_exp_deriv.argtypes = [_d, ctypes.c_int, _d]
            L.orc_sh_eval.argtypes = [ctypes.c_int, _d, _d, _d]
            L.orc_bin_keys.restype = ctypes.c_int64
            L.orc_bin_keys.argtypes = [ctypes.c_int64, _i32, _i64, _i64, _i64, _i64, _i64, _u32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       _u64, _i64, ctypes.c_int64]
            L.orc_num_threads.restype = ctypes.c_int
            L.orc_set_num_threads.argtypes = [ctypes.c_int]
            _lib = L
    return _lib


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


@dataclasses.dataclass
class OracleConfig:
    """Rasterizer constants.  The paper states none of them (it inherits the
    rasterizer from 3DGS); these are the readings used throughout."""
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    near: float = 0.2
    eps2d: float = 0.3
    guard: float = 1.3
    rect_margin: float = 1.0 / 256.0
    far: float = 1e30
    bg: tuple = (0.0, 0.0, 0.0)
    tile_w: int = 16
    tile_h: int = 16

    def c(self) -> _Cfg:
        c = _Cfg()
        c.alpha_min, c.alpha_max, c.t_min = self.alpha_min, self.alpha_max, self.t_min
        c.near_z, c.eps2d, c.guard, c.rect_margin = self.near, self.eps2d, self.guard, self.rect_margin
        c.far_z = self.far
        for k in range(3):
            c.bg[k] = self.bg[k]
        c.tile_w, c.tile_h = self.tile_w, self.tile_h
        return c

    @staticmethod
    def smooth(**kw) -> "OracleConfig":
        """Thresholds switched off (for finite differences): no alpha floor or
        clamp, no transmittance stop, no low-pass term needed."""
        base = dict(alpha_min=1e-12, alpha_max=1.0, t_min=0.0)
        base.update(kw)
        return OracleConfig(**base)


def _camera(rec) -> _Camera:
    c = _Camera()
    for k in range(9):
        c.R[k] = float(rec["R"][k])
    for k in range(3):
        c.t[k] = float(rec["t"][k])
    c.fx, c.fy, c.cx, c.cy = float(rec["fx"]), float(rec["fy"]), float(rec["cx"]), float(rec["cy"])
    c.width, c.height = int(rec["width"]), int(rec["height"])
    return c


class View:
    """One view of a scene rendered by the oracle: projection + per-tile lists +
    compositing happen at construction."""

    def __init__(self, scene, v: int, cfg: OracleConfig = OracleConfig(), params=None):
        p = params or {}
        # parameters are taken in FP64 (float32 scene arrays convert exactly)
        self.means = np.ascontiguousarray(p.get("means", scene.means), np.float64)
        self.log_scales = np.ascontiguousarray(p.get("log_scales", scene.log_scales), np.float64)
        self.quats = np.ascontiguousarray(p.get("quats", scene.quats), np.float64)
        self.logits = np.ascontiguousarray(p.get("logits", scene.logits), np.float64)
        self.sh = np.ascontiguousarray(p.get("sh", scene.sh), np.float64)
        self.xi = np.ascontiguousarray(p.get("pose_xi", scene.pose_xi)[v], np.float64)
        self.degree = scene.sh_degree
        self.n = int(self.means.shape[1])
        self.cam = _camera(scene.cams[v])
        self.W, self.H = int(scene.cams[v]["width"]), int(scene.cams[v]["height"])
        self.cfg = cfg
        self._c = cfg.c()
        L = lib()
        self._h = L.orc_view_create(self.n, self.degree, _ptr(self.means, _d), _ptr(self.log_scales, _d),
                                    _ptr(self.quats, _d), _ptr(self.logits, _d), _ptr(self.sh, _d),
                                    ctypes.byref(self.cam), _ptr(self.xi, _d), ctypes.byref(self._c))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_view_free(h)
            self._h = None

    @property
    def n_visible(self) -> int:
        return int(lib().orc_view_n_visible(self._h))

    @property
    def n_pairs(self) -> int:
        return int(lib().orc_view_n_pairs(self._h))

    def image(self) -> dict:
        """Colour, depth, final transmittance, last blended position, blended
        count, and four decision-margin planes per pixel (relative distance of
        alpha from alpha_min, of a candidate T from T_min, of alpha from the
        alpha_max clamp, and the smallest relative depth gap)."""
        H, W = self.H, self.W
        out = dict(color=np.empty((3, H, W)), depth=np.empty((H, W)), tfinal=np.empty((H, W)),
                   last=np.empty((H, W), np.int32), nblend=np.empty((H, W), np.int32),
                   margins=np.empty((4, H, W)))
        lib().orc_view_image(self._h, _ptr(out["color"], _d), _ptr(out["depth"], _d),
                             _ptr(out["tfinal"], _d), _ptr(out["last"], _i32), _ptr(out["nblend"], _i32),
                             _ptr(out["margins"], _d))
        return out

    def gauss_margins(self) -> np.ndarray:
        """[N][3]: each Gaussian's own alpha-vs-alpha_min margin, alpha_max
        margin, and the T_min margin where it ends a pixel's sequence."""
        out = np.empty((self.n, 3))
        lib().orc_view_gauss_margins(self._h, _ptr(out, _d))
        return out

    def proj(self) -> dict:
        rec = np.empty((self.n, 10))
        irec = np.empty((self.n, 9), np.int64)
        misc = np.empty((self.n, 9))
        lib().orc_view_proj(self._h, _ptr(rec, _d), _ptr(irec, _i64), _ptr(misc, _d))
        return dict(mu=rec[:, 0:2], conic=rec[:, 2:5], opacity=rec[:, 5], color=rec[:, 6:9],
                    depth=rec[:, 9], visible=irec[:, 0].astype(bool), fxi=irec[:, 1], fyi=irec[:, 2],
                    rx=irec[:, 3], ry=irec[:, 4], rect=irec[:, 5:9], margins=misc)

    def pairs(self):
        n = self.n_pairs
        tile = np.empty(n, np.int32)
        gid = np.empty(n, np.int64)
        lib().orc_view_pairs(self._h, _ptr(tile, _i32), _ptr(gid, _i64))
        return tile, gid

    def stats(self, target: np.ndarray, tau_err: float = 0.1) -> dict:
        """Footprint |Omega_v(i)|, high-error count kappa_v(i) and the error
        mask M_v (appendix, densification score: error mask and kappa)."""
        t = np.ascontiguousarray(target, np.float32)
        omega = np.empty(self.n, np.int32)
        kappa = np.empty(self.n, np.int32)
        mask = np.empty((self.H, self.W), np.uint8)
        mm = np.empty((self.H, self.W))
        lib().orc_view_stats(self._h, _ptr(t, _f), float(tau_err), _ptr(omega, _i32), _ptr(kappa, _i32),
                             _ptr(mask, _u8), _ptr(mm, _d))
        return dict(omega=omega, kappa=kappa, mask=mask.astype(bool), mask_margin=mm)

    def anchor_stats(self, anchor_of, n_anchor: int, target: np.ndarray, tau_err: float = 0.1) -> dict:
        """Per-anchor |Omega_v(a)| and kappa_v(a): the union of the blended pixels of
        the Gaussians g with anchor_of[g] == a (appendix, densification and
        pruning scores of an anchor)."""
        a = np.ascontiguousarray(anchor_of, np.int64)
        t = np.ascontiguousarray(target, np.float32)
        om = np.zeros(int(n_anchor), np.int64)
        ka = np.zeros(int(n_anchor), np.int64)
        lib().orc_view_anchor_stats(self._h, _ptr(a, _i64), int(n_anchor), _ptr(t, _f), float(tau_err),
                                    _ptr(om, _i64), _ptr(ka, _i64))
        return dict(omega=om, kappa=ka)

    def backward(self, dLdC: np.ndarray, dLdD=None) -> dict:
        """Gradients of L with dL/dC (3,H,W) and dL/dD (H,W) given; exact
        derivative with thresholds held fixed."""
        n, K = self.n, (self.degree + 1) ** 2
        gC = np.ascontiguousarray(dLdC, np.float64)
        gD = None if dLdD is None else np.ascontiguousarray(dLdD, np.float64)
        out = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
                   logits=np.zeros(n), sh=np.zeros((K, 3, n)), pose_xi=np.zeros(6),
                   g2=np.zeros((n, 10)))
        lib().orc_view_backward(self._h, _ptr(gC, _d), _ptr(gD, _d), _ptr(out["means"], _d),
                                _ptr(out["log_scales"], _d), _ptr(out["quats"], _d),
                                _ptr(out["logits"], _d), _ptr(out["sh"], _d), _ptr(out["pose_xi"], _d),
                                _ptr(out["g2"], _d))
        return out


def se3_exp(xi) -> np.ndarray:
    x = np.ascontiguousarray(xi, np.float64)
    T = np.empty(16)
    lib().orc_se3_exp(_ptr(x, _d), _ptr(T, _d))
    return T.reshape(4, 4)


def se3_exp_deriv(xi, k: int) -> np.ndarray:
    x = np.ascontiguousarray(xi, np.float64)
    D = np.empty(16)
    lib().orc_se3_exp_deriv(_ptr(x, _d), int(k), _ptr(D, _d))
    return D.reshape(4, 4)


def sh_eval(degree: int, d) -> tuple:
    d = np.ascontiguousarray(d, np.float64)
    Y = np.zeros(16)
    dY = np.zeros((16, 3))
    lib().orc_sh_eval(int(degree), _ptr(d, _d), _ptr(Y, _d), _ptr(dY, _d))
    K = (degree + 1) ** 2
    return Y[:K], dY[:K]


def bin_keys(view, gid, fxi, fyi, rx, ry, depth_bits, W, H, TW, TH, cap=None):
    """Sorted (key, gaussian) list of the integer binning contract."""
    n = len(view)
    a = [np.ascontiguousarray(x, t) for x, t in
         ((view, np.int32), (gid, np.int64), (fxi, np.int64), (fyi, np.int64), (rx, np.int64),
          (ry, np.int64), (depth_bits, np.uint32))]
    if cap is None:
        TX, TY = -(-W // TW), -(-H // TH)
        cap = int(np.sum((np.minimum(TX, (a[2] + a[4]) // TW + 1) - np.maximum(0, (a[2] - a[4]) // TW)).clip(0)
                         * (np.minimum(TY, (a[3] + a[5]) // TH + 1) - np.maximum(0, (a[3] - a[5]) // TH)).clip(0)))
    keys = np.empty(max(cap, 1), np.uint64)
    gids = np.empty(max(cap, 1), np.int64)
    m = lib().orc_bin_keys(n, _ptr(a[0], _i32), _ptr(a[1], _i64), _ptr(a[2], _i64), _ptr(a[3], _i64),
                           _ptr(a[4], _i64), _ptr(a[5], _i64), _ptr(a[6], _u32), W, H, TW, TH,
                           _ptr(keys, _u64), _ptr(gids, _i64), cap)
    if m < 0:
        raise ValueError("capacity too small")
    return keys[:m], gids[:m]


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP regions from now on (for timing)."""
    lib().orc_set_num_threads(int(n))
