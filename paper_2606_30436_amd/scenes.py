"""Seeded synthetic scenes: the only module shared by the HIP path and the oracle.

It holds random draws and scene geometry (camera placement along a trajectory)
and nothing of the method's arithmetic: no projection, no compositing, no
statistics.  Every array is float32 (int32 for image sizes) and every scene is
a pure function of its seed.

Layouts (structure of arrays, Gaussian index fastest):
  means        [3][N]     world position (x right, y down, z forward at s = 0)
  log_scales   [3][N]     natural log of the three axis scales
  quats        [4][N]     (w, x, y, z), not necessarily unit length
  logits       [N]        opacity logits
  sh           [K][3][N]  K = (degree + 1)^2 real SH coefficients per colour channel
  cams         [V]        CAMERA_DTYPE records: world->camera R (row major), t,
                          pinhole fx, fy, cx, cy, image width, height
  pose_xi      [V][6]     tangent perturbation (rho, phi) applied on the left

The workloads stand in for the driving sequences of the paper's experiments
(Sec. 4: Waymo, KITTI, KITTI-360): forward-moving cameras at road height,
1242x375 images, keyframes every few metres, chunks of 100 keyframes
(hyper-parameter table).  No dataset content is reproduced.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

CAMERA_DTYPE = np.dtype([
    ("R", "<f4", (9,)), ("t", "<f4", (3,)),
    ("fx", "<f4"), ("fy", "<f4"), ("cx", "<f4"), ("cy", "<f4"),
    ("width", "<i4"), ("height", "<i4"),
], align=False)
assert CAMERA_DTYPE.itemsize == 72

# sqrt(pi): a uniform DC coefficient on [-sqrt(pi), sqrt(pi)] makes the degree-0
# colour uniform on [0, 1] under the real-SH colour model with a +0.5 offset.
SQRT_PI = math.sqrt(math.pi)


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    logits: np.ndarray
    sh: np.ndarray
    sh_degree: int
    cams: np.ndarray
    pose_xi: np.ndarray
    target: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def n_views(self) -> int:
        return int(self.cams.shape[0])

    @property
    def width(self) -> int:
        return int(self.cams["width"][0])

    @property
    def height(self) -> int:
        return int(self.cams["height"][0])

    def subset(self, idx: np.ndarray) -> "Scene":
        idx = np.asarray(idx)
        return dataclasses.replace(
            self, means=np.ascontiguousarray(self.means[:, idx]),
            log_scales=np.ascontiguousarray(self.log_scales[:, idx]),
            quats=np.ascontiguousarray(self.quats[:, idx]),
            logits=np.ascontiguousarray(self.logits[idx]),
            sh=np.ascontiguousarray(self.sh[:, :, idx]), meta=dict(self.meta))

    def views(self, vidx) -> "Scene":
        vidx = np.atleast_1d(np.asarray(vidx))
        return dataclasses.replace(
            self, cams=np.ascontiguousarray(self.cams[vidx]),
            pose_xi=np.ascontiguousarray(self.pose_xi[vidx]),
            target=None if self.target is None else np.ascontiguousarray(self.target[vidx]),
            meta=dict(self.meta))


def make_camera(R, t, fx, fy, cx, cy, width, height) -> np.ndarray:
    c = np.zeros((), CAMERA_DTYPE)
    c["R"] = np.asarray(R, np.float32).reshape(9)
    c["t"] = np.asarray(t, np.float32).reshape(3)
    c["fx"], c["fy"], c["cx"], c["cy"] = fx, fy, cx, cy
    c["width"], c["height"] = width, height
    return c


def stack_cameras(cams) -> np.ndarray:
    out = np.zeros(len(cams), CAMERA_DTYPE)
    for i, c in enumerate(cams):
        out[i] = c
    return out


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    return (q / np.linalg.norm(q, axis=0, keepdims=True)).astype(np.float32)


def _sh_coeffs(rng, n, degree, hi_sigma=0.05):
    k = (degree + 1) ** 2
    sh = np.zeros((k, 3, n), np.float32)
    sh[0] = rng.uniform(-SQRT_PI, SQRT_PI, (3, n))
    if k > 1:
        sh[1:] = rng.normal(0.0, hi_sigma, (k - 1, 3, n))
    return sh


# --------------------------------------------------------------------------- C1
def make_c1(seed: int = 1, n: int = 10_000, target_seed: int = 101) -> Scene:
    """Plain single view: 10k Gaussians uniform in the volume of a 60-degree
    frustum between 2 and 20 m, camera at the origin looking down +z, 320x240."""
    rng = np.random.default_rng(seed)
    W, H = 320, 240
    f = (W / 2) / math.tan(math.radians(30.0))
    z = np.cbrt(8.0 + rng.uniform(0.0, 1.0, n) * (8000.0 - 8.0))
    x = (2 * rng.uniform(0.0, 1.0, n) - 1) * z * math.tan(math.radians(30.0))
    y = (2 * rng.uniform(0.0, 1.0, n) - 1) * z * (H / 2) / f
    means = np.stack([x, y, z]).astype(np.float32)
    log_scales = rng.normal(-3.0, 0.5, (3, n)).astype(np.float32)
    quats = _unit_quats(rng, n)
    logits = rng.normal(0.0, 1.0, n).astype(np.float32)
    sh = np.zeros((1, 3, n), np.float32)
    sh[0] = rng.uniform(-SQRT_PI, SQRT_PI, (3, n))
    cam = make_camera(np.eye(3), np.zeros(3), f, f, W / 2, H / 2, W, H)
    trng = np.random.default_rng(target_seed)
    target = trng.uniform(0.0, 1.0, (1, 3, H, W)).astype(np.float32)
    return Scene(means, log_scales, quats, logits, sh, 0, stack_cameras([cam]),
                 np.zeros((1, 6), np.float32), target,
                 {"name": "c1", "seed": seed, "target_seed": target_seed})


# --------------------------------------------------------------- road layout
def _road_layout(rng, n):
    """Lateral offset and height of road-like structure: 40% road surface 1.65 m
    below the camera, 40% facades 8-12 m to either side, 20% clutter."""
    kind = rng.choice(3, size=n, p=[0.4, 0.4, 0.2])
    lat = np.empty(n)
    y = np.empty(n)
    m = kind == 0
    lat[m] = rng.uniform(-7.0, 7.0, m.sum())
    y[m] = 1.65 + rng.normal(0.0, 0.03, m.sum())
    m = kind == 1
    side = rng.choice([-1.0, 1.0], size=m.sum())
    lat[m] = side * rng.uniform(8.0, 12.0, m.sum())
    y[m] = rng.uniform(-8.0, 1.65, m.sum())
    m = kind == 2
    lat[m] = rng.uniform(-12.0, 12.0, m.sum())
    y[m] = rng.uniform(-4.0, 1.65, m.sum())
    return lat, y, kind


# --------------------------------------------------------------------------- C2
def make_c2(seed: int = 2, n: int = 500_000, target_seed: int = 102) -> Scene:
    """Single view of a 200 m road corridor: depth log-uniform on [2, 80] m,
    SH degree 3, 1242x375, f = 720."""
    rng = np.random.default_rng(seed)
    W, H, f = 1242, 375, 720.0
    z = np.exp(rng.uniform(math.log(2.0), math.log(80.0), n))
    lat, y, _ = _road_layout(rng, n)
    means = np.stack([lat, y, z]).astype(np.float32)
    log_scales = (rng.normal(-3.0, 0.5, (3, n)) + np.log(np.maximum(1.0, z / 10.0))).astype(np.float32)
    quats = _unit_quats(rng, n)
    logits = rng.normal(0.0, 1.0, n).astype(np.float32)
    sh = _sh_coeffs(rng, n, 3)
    cam = make_camera(np.eye(3), np.zeros(3), f, f, W / 2, H / 2, W, H)
    trng = np.random.default_rng(target_seed)
    target = trng.uniform(0.0, 1.0, (1, 3, H, W)).astype(np.float32)
    return Scene(means, log_scales, quats, logits, sh, 3, stack_cameras([cam]),
                 np.zeros((1, 6), np.float32), target,
                 {"name": "c2", "seed": seed, "target_seed": target_seed})


# ------------------------------------------------------------------ trajectory
def _heading(s):
    return 0.4 * np.sin(2.0 * math.pi * s / 700.0)


def trajectory(length: float, ds: float = 0.25):
    """Planar path at camera height: heading theta(s) = 0.4 sin(2 pi s / 700)."""
    s = np.arange(0.0, length + ds, ds)
    th = _heading(s)
    x = np.concatenate([[0.0], np.cumsum(np.sin(th[:-1]) * ds)])
    z = np.concatenate([[0.0], np.cumsum(np.cos(th[:-1]) * ds)])
    return s, x, z, th


def _path_frame(s_query, s, x, z):
    px = np.interp(s_query, s, x)
    pz = np.interp(s_query, s, z)
    th = _heading(s_query)
    return px, pz, th


def trajectory_cameras(s_views, length, W=1242, H=375, f=720.0):
    s, x, z, _ = trajectory(length)
    px, pz, th = _path_frame(np.asarray(s_views, np.float64), s, x, z)
    cams = []
    for cx_w, cz_w, t in zip(px, pz, th):
        right = np.array([math.cos(t), 0.0, -math.sin(t)])
        down = np.array([0.0, 1.0, 0.0])
        fwd = np.array([math.sin(t), 0.0, math.cos(t)])
        R = np.stack([right, down, fwd])
        c = np.array([cx_w, 0.0, cz_w])
        cams.append(make_camera(R, -R @ c, f, f, W / 2, H / 2, W, H))
    return stack_cameras(cams)


def _sample_arclength(rng, n, edges, density):
    """Arc lengths from a piecewise-constant density (Gaussians per metre)."""
    edges = np.asarray(edges, np.float64)
    w = np.asarray(density, np.float64) * np.diff(edges)
    seg = rng.choice(len(w), size=n, p=w / w.sum())
    return edges[seg] + rng.uniform(0.0, 1.0, n) * (edges[seg + 1] - edges[seg])


def trajectory_gaussians(rng, n, length, edges, density, degree=3):
    """Gaussians along the trajectory, stored in insertion order: a mapping
    system spawns them at the keyframes as the camera moves (Sec. 3.3,
    probabilistic initialisation at incoming keyframes), so the map's index
    order follows the arc length."""
    s, x, z, _ = trajectory(length)
    sg = np.sort(_sample_arclength(rng, n, edges, density))
    px, pz, th = _path_frame(sg, s, x, z)
    lat, y, kind = _road_layout(rng, n)
    gx = px + lat * np.cos(th)
    gz = pz - lat * np.sin(th)
    means = np.stack([gx, y, gz]).astype(np.float32)
    # creation distance: finer Gaussians near the keyframe that spawned them,
    # coarser ones far away (the paper's level-of-detail idea, Sec. 3.2).
    z0 = np.exp(rng.uniform(math.log(2.0), math.log(80.0), n))
    log_scales = (rng.normal(-3.0, 0.5, (3, n)) + np.log(np.maximum(1.0, z0 / 10.0))).astype(np.float32)
    quats = _unit_quats(rng, n)
    logits = rng.normal(0.0, 1.0, n).astype(np.float32)
    sh = _sh_coeffs(rng, n, degree)
    return means, log_scales, quats, logits, sh, sg, kind


# Keyframes every 3 m; a chunk holds C = 100 keyframes (hyper-parameter table);
# the views of a chunk are sampled uniformly from it.
KEYFRAME_SPACING = 3.0
CHUNK_KEYFRAMES = 100


def chunk_view_arclengths(chunk: int, n_views: int) -> np.ndarray:
    k = np.floor((np.arange(n_views) + 0.5) * CHUNK_KEYFRAMES / n_views)
    return (chunk * CHUNK_KEYFRAMES + k) * KEYFRAME_SPACING


# density profile of the 1 km trajectory: a sparse start, a dense block and a
# tail, so that the 8 views of the first chunk see very different numbers of
# Gaussians (about 50k to 600k).
C3_EDGES = [0.0, 130.0, 170.0, 250.0, 290.0, 360.0, 1080.0]
C3_DENSITY = [800.0, 3000.0, 9000.0, 3000.0, 1200.0, 1183.0]


def make_c3(seed: int = 3, n: int = 2_000_000, n_views: int = 8, perturb: bool = True) -> Scene:
    """Batched chunk: 2M Gaussians along a 1 km trajectory, 8 keyframes of the
    first chunk at 1242x375, SH degree 3.  `meta['true']` holds the unperturbed
    parameters (targets are rendered from them); the returned parameters carry
    5 cm mean noise and colour noise of 0.05 (in DC-coefficient units 0.05*2*sqrt(pi))."""
    rng = np.random.default_rng(seed)
    length = 1080.0
    means, ls, q, lg, sh, sg, kind = trajectory_gaussians(rng, n, length, C3_EDGES, C3_DENSITY)
    cams = trajectory_cameras(chunk_view_arclengths(0, n_views), length)
    true = {"means": means.copy(), "sh": sh.copy()}
    if perturb:
        means = (means + rng.normal(0.0, 0.05 / math.sqrt(3.0), means.shape)).astype(np.float32)
        sh = sh.copy()
        sh[0] = sh[0] + rng.normal(0.0, 0.05 * 2.0 * SQRT_PI, sh[0].shape).astype(np.float32)
    return Scene(means, ls, q, lg, sh, 3, cams, np.zeros((n_views, 6), np.float32), None,
                 {"name": "c3", "seed": seed, "true": true, "arclength": sg, "kind": kind})


def random_pose_perturbation(rng, n_views, angle_deg=0.5, trans=0.2) -> np.ndarray:
    """Tangent perturbations with |phi| = angle exactly (random axis) and
    |rho| = trans exactly (random direction)."""
    a = rng.standard_normal((n_views, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    d = rng.standard_normal((n_views, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    xi = np.concatenate([d * trans, a * math.radians(angle_deg)], axis=1)
    return xi.astype(np.float32)


C4_EDGES = [0.0, 100.0, 200.0, 300.0, 360.0, 1600.0]
C4_DENSITY = [3000.0, 9000.0, 14000.0, 6000.0, 2250.0]


def make_c4(seed: int = 4, n: int = 5_000_000, n_views: int = 16) -> Scene:
    """Differentiable pose + map: 5M Gaussians, 16 keyframes of one chunk, each
    pose perturbed by 0.5 degrees and 0.2 m (the tangent vector is pose_xi; the
    cameras are the true poses the targets are rendered at)."""
    rng = np.random.default_rng(seed)
    length = 1600.0
    means, ls, q, lg, sh, sg, kind = trajectory_gaussians(rng, n, length, C4_EDGES, C4_DENSITY)
    cams = trajectory_cameras(chunk_view_arclengths(0, n_views), length)
    xi = random_pose_perturbation(rng, n_views)
    return Scene(means, ls, q, lg, sh, 3, cams, xi, None,
                 {"name": "c4", "seed": seed, "arclength": sg, "kind": kind})


def make_c5(seed: int = 5, n: int = 5_000_000, n_chunks: int = 32, views_per_chunk: int = 16,
            floater_frac: float = 0.05, n_holes: int = 64) -> Scene:
    """Learned-head workload: 5M Gaussians along a ~10 km trajectory, 32 chunks
    of 16 keyframes.  The returned map has 5% injected floaters (large, faint,
    in the air) and `n_holes` 5 m stretches of facade removed:
    `meta['struct_index']` selects the structure-only scene the targets are
    rendered from (facade in the holes included, no floaters) and
    `meta['map_index']` the map (floaters included, the holes' facade
    Gaussians left out)."""
    rng = np.random.default_rng(seed)
    length = n_chunks * CHUNK_KEYFRAMES * KEYFRAME_SPACING + 120.0
    n_float = int(round(n * floater_frac))
    n_struct = n - n_float
    means, ls, q, lg, sh, sg, kind = trajectory_gaussians(
        rng, n_struct, length, [0.0, length], [1.0])
    # floaters
    s, x, z, _ = trajectory(length)
    fs = rng.uniform(0.0, length, n_float)
    px, pz, th = _path_frame(fs, s, x, z)
    lat = rng.uniform(-10.0, 10.0, n_float)
    fy = rng.uniform(-6.0, 1.0, n_float)
    fmeans = np.stack([px + lat * np.cos(th), fy, pz - lat * np.sin(th)]).astype(np.float32)
    fls = rng.normal(-1.0, 0.3, (3, n_float)).astype(np.float32)
    fq = _unit_quats(rng, n_float)
    flg = rng.normal(-3.0, 0.5, n_float).astype(np.float32)
    fsh = _sh_coeffs(rng, n_float, 3)
    # holes: facade Gaussians in short stretches are removed from the map
    hole_start = rng.uniform(0.0, length - 5.0, n_holes)
    in_hole = np.zeros(n_struct, bool)
    for h in hole_start:
        in_hole |= (sg >= h) & (sg < h + 5.0) & (kind == 1)
    all_means = np.concatenate([means, fmeans], axis=1)
    all_ls = np.concatenate([ls, fls], axis=1)
    all_q = np.concatenate([q, fq], axis=1)
    all_lg = np.concatenate([lg, flg])
    all_sh = np.concatenate([sh, fsh], axis=2)
    is_floater = np.concatenate([np.zeros(n_struct, bool), np.ones(n_float, bool)])
    struct_index = np.nonzero(~is_floater)[0]
    map_index = np.nonzero(~np.concatenate([in_hole, np.zeros(n_float, bool)]))[0]
    s_views = np.concatenate([chunk_view_arclengths(c, views_per_chunk) for c in range(n_chunks)])
    cams = trajectory_cameras(s_views, length)
    return Scene(all_means, all_ls, all_q, all_lg, all_sh, 3, cams,
                 np.zeros((len(cams), 6), np.float32), None,
                 {"name": "c5", "seed": seed, "is_floater": is_floater, "in_hole": in_hole,
                  "struct_index": struct_index, "map_index": map_index,
                  "n_chunks": n_chunks, "views_per_chunk": views_per_chunk})


# --------------------------------------------------------------- tiny scenes
def tiny_scene(seed: int = 0, n: int = 24, W: int = 40, H: int = 32, degree: int = 1,
               n_views: int = 1, depth=(2.0, 6.0), log_scale_mu: float = -2.0,
               log_scale_sigma: float = 0.3, spread: float = 0.6, pose_sigma: float = 0.0,
               with_target: bool = True) -> Scene:
    """A handful of Gaussians in front of small cameras; used for brute-force,
    autograd and finite-difference pins."""
    rng = np.random.default_rng(seed)
    f = 0.9 * W
    z = rng.uniform(depth[0], depth[1], n)
    x = rng.uniform(-spread, spread, n) * z * (W / 2) / f
    y = rng.uniform(-spread, spread, n) * z * (H / 2) / f
    means = np.stack([x, y, z]).astype(np.float32)
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, (3, n)).astype(np.float32)
    quats = rng.standard_normal((4, n)).astype(np.float32)  # unnormalised on purpose
    logits = rng.normal(0.5, 1.0, n).astype(np.float32)
    sh = _sh_coeffs(rng, n, degree, hi_sigma=0.2)
    cams = []
    for v in range(n_views):
        ang = 0.05 * v
        R = np.array([[math.cos(ang), 0.0, -math.sin(ang)], [0.0, 1.0, 0.0],
                      [math.sin(ang), 0.0, math.cos(ang)]])
        t = np.array([0.05 * v, -0.02 * v, 0.1 * v])
        cams.append(make_camera(R, t, f, f * 1.05, W / 2 + 0.3, H / 2 - 0.2, W, H))
    cams = stack_cameras(cams)
    xi = (rng.normal(0.0, pose_sigma, (n_views, 6)) if pose_sigma > 0
          else np.zeros((n_views, 6))).astype(np.float32)
    target = rng.uniform(0.0, 1.0, (n_views, 3, H, W)).astype(np.float32) if with_target else None
    return Scene(means, log_scales, quats, logits, sh, degree, cams, xi, target,
                 {"name": "tiny", "seed": seed})


def random_target(seed: int, n_views: int, H: int, W: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, (n_views, 3, H, W)).astype(np.float32)


# Spawn-time levels of the anchor scene: the band of the distance from which the
# anchor was first seen (10, 25, 100, 500 m: voxels of 0.1, 0.25, 1, 5, 25 m).
ANCHOR_LEVEL_EDGES = (10.0, 25.0, 100.0, 500.0)
ANCHOR_VOXEL = (0.1, 0.25, 1.0, 5.0, 25.0)


def make_anchor_scene(seed: int = 6, n_anchors: int = 200_000, k: int = 10, n_views: int = 8) -> dict:
    """Voxel anchors along the 1 km trajectory (Scaffold-style map, appendix
    'Voxelized Representation and MLP Decoding'): positions laid out like the
    trajectory Gaussians, each anchor seen first from a keyframe 3-60 m behind
    it, which sets its level and its local scale (the level's voxel size); a
    32-dim feature N(0, 0.5^2), k offsets N(0, 1) in units of the local scale,
    and a decoder whose output biases give opacity tanh(1), rotation near the
    identity and half-scale children.  Cameras: the first chunk's keyframes."""
    rng = np.random.default_rng(seed)
    length = 1080.0
    means, _, _, _, _, sg, _ = trajectory_gaussians(rng, n_anchors, length, C3_EDGES, C3_DENSITY, degree=0)
    s, x, z, _ = trajectory(length)
    s_seen = np.maximum(sg - rng.uniform(3.0, 60.0, n_anchors), 0.0)
    px, pz, _ = _path_frame(s_seen, s, x, z)
    dist = np.sqrt((means[0] - px) ** 2 + (means[1] - 0.0) ** 2 + (means[2] - pz) ** 2)
    level = np.searchsorted(np.array(ANCHOR_LEVEL_EDGES), dist, side="right").astype(np.int32)
    log_l = (np.log(np.array(ANCHOR_VOXEL)[level])[None, :] + rng.normal(0.0, 0.2, (3, n_anchors))).astype(np.float32)
    feat = rng.normal(0.0, 0.5, (n_anchors, 32)).astype(np.float32)
    offsets = rng.normal(0.0, 1.0, (k, 3, n_anchors)).astype(np.float32)
    W1 = rng.normal(0.0, 1.0 / math.sqrt(36.0), (32, 36))
    W1[:, 35] *= 0.01                                    # the distance input reaches 1 km: weight it like a
    b1 = rng.normal(0.0, 0.1, 32)                        # metre-scale input of the other columns' size
    W2 = rng.normal(0.0, 0.5 / math.sqrt(32.0), (14 * k, 32))
    child = np.array([1.0, 0, 0, 0, 1.0, 0, 0, 0, 0, 0, 0, 0, 0, 0])
    b2 = np.tile(child, k) + rng.normal(0.0, 0.05, 14 * k)
    theta = np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(np.float32)
    cams = trajectory_cameras(chunk_view_arclengths(0, n_views), length)
    return dict(p=means, feat=feat, log_l=log_l, offsets=offsets, level=level, theta=theta, k=k, cams=cams,
                width=1242, height=375)
