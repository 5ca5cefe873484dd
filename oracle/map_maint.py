"""Map maintenance in plain Python / NumPy FP64.  TEST INFRASTRUCTURE ONLY (see
oracle/__init__.py).

Follows the appendix sections "Dynamic Map Expansion" (a new 3D point x is
assigned a level l by its camera distance, its voxel index is
idx = floor(x / eps_l), and a new anchor is created at p = idx eps_l only if
that voxel is not occupied yet, looked up in a spatial hash table) and "Global
Map Alignment" (after loop closure every anchor spawned at keyframe m moves
rigidly, p_new = T_new^(m) (T_old^(m))^-1 p, in batches; then the map is
re-voxelised and hashed again so that overlapping regions merge), with the
densify / prune decisions of Sec. 3.3 acting on the map.

Readings where the paper is silent:
  * A voxel is the pair (level, idx); its key packs the level (3 bits) and
    the three indices offset by 2^19 (20 bits each).  A batch of candidate
    points creates one anchor per new voxel, numbered after the existing ones
    in the order of each voxel's first candidate.
  * With explicit Gaussians an anchor is one Gaussian.  A new one gets the mean
    idx eps_l (the paper's p), isotropic log-scales ln(eps_l), the identity
    rotation, opacity 0.1 and the colour of the pixel that spawned it (SH
    degree-0 coefficient (c - 0.5) / Y_00, higher bands zero).
  * Densifying Gaussian i proposes the two points mu_i +- s_max a_max (its
    largest scale along that axis); their level comes from the distance to a
    given camera centre, and they enter the map through the same hash.
  * Pruning keeps the survivors in index order (the keep map of the decision).
  * Poses T are world->camera (R, t) as everywhere here, so
    p_new = R_new^T (R_old p + t_old - t_new) and the rotation of the Gaussian
    is left-multiplied by R_new^T R_old; anchors with keyframe -1 stay.
  * Re-voxelisation keeps, of the anchors that share a voxel after the move,
    the one with the lowest index; the others are merged away (pruned).
"""
from __future__ import annotations

import math

import numpy as np

EPS = (0.1, 0.25, 1.0, 5.0, 25.0)
DMAX = tuple(100.0 * e for e in EPS[:-1]) + (math.inf,)
IDX_OFFSET = 1 << 19
Y00 = 0.28209479177387814
SPAWN_OPACITY = 0.1


def level_of(distance: float) -> int:
    for l, dm in enumerate(DMAX):
        if distance < dm:
            return l
    return len(DMAX) - 1


def voxel_key(level: int, idx) -> int:
    """(level, idx) -> 63-bit key: level in bits 60..62, x, y, z offset by 2^19 in 20 bits each."""
    x, y, z = (int(v) + IDX_OFFSET for v in idx)
    assert 0 <= x < (1 << 20) and 0 <= y < (1 << 20) and 0 <= z < (1 << 20) and 0 <= level < 8
    return (int(level) << 60) | (x << 40) | (y << 20) | z


def insert(table: dict, keys, n_anchors: int):
    """Insert candidate voxel keys into the map's table {key: anchor}.  Returns the
    anchor of every candidate, the candidates that created an anchor (first
    occurrence of a new key, in candidate order) and the new anchor count."""
    anchor = np.empty(len(keys), np.int64)
    created = []
    for i, k in enumerate(keys):
        k = int(k)
        if k not in table:
            table[k] = n_anchors + len(created)
            created.append(i)
        anchor[i] = table[k]
    return anchor, np.array(created, np.int64), n_anchors + len(created)


def spawn_params(level, voxel, color):
    """Explicit Gaussians for new anchors (arrays over the new anchors)."""
    level = np.asarray(level, np.int64)
    eps = np.array(EPS)[level]
    n = len(level)
    means = (np.asarray(voxel, np.float64) * eps[:, None]).T
    log_scales = np.tile(np.log(eps), (3, 1))
    quats = np.zeros((4, n))
    quats[0] = 1.0
    logits = np.full(n, math.log(SPAWN_OPACITY / (1.0 - SPAWN_OPACITY)))
    sh0 = ((np.asarray(color, np.float64) - 0.5) / Y00).T
    return dict(means=means, log_scales=log_scales, quats=quats, logits=logits, sh0=sh0)


def quat_to_rot(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def densify_points(means, log_scales, quats, decision, centre, densify_code=1):
    """Candidate points of the Gaussians marked for densification, in Gaussian
    order, the + point before the - point; with their level and voxel."""
    pts, src = [], []
    c = np.asarray(centre, np.float64)
    for i in np.flatnonzero(np.asarray(decision) == densify_code):
        s = np.exp(np.asarray(log_scales, np.float64)[:, i])
        k = int(np.argmax(s))
        a = quat_to_rot(np.asarray(quats, np.float64)[:, i])[:, k]
        mu = np.asarray(means, np.float64)[:, i]
        for sign in (1.0, -1.0):
            pts.append(mu + sign * s[k] * a)
            src.append(i)
    pts = np.array(pts).reshape(-1, 3)
    lev = np.array([level_of(float(np.linalg.norm(p - c))) for p in pts], np.int64)
    eps = np.array(EPS)[lev] if len(lev) else np.zeros(0)
    vox = np.floor(pts / eps[:, None]).astype(np.int64) if len(lev) else np.zeros((0, 3), np.int64)
    return dict(point=pts, source=np.array(src, np.int64), level=lev, voxel=vox)


def compact(arrays: dict, decision, prune_code=2) -> dict:
    """Survivors of the prune decision, in index order (Gaussian index is the last axis)."""
    keep = np.asarray(decision) != prune_code
    return {k: np.asarray(v)[..., keep] for k, v in arrays.items()}


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def rot_to_quat(R):
    """Unit quaternion (w, x, y, z) of a rotation matrix, w >= 0 (Shepperd's method)."""
    R = np.asarray(R, np.float64)
    tr = np.trace(R)
    cands = [1 + tr, 1 + 2 * R[0, 0] - tr, 1 + 2 * R[1, 1] - tr, 1 + 2 * R[2, 2] - tr]
    k = int(np.argmax(cands))
    r = math.sqrt(cands[k])
    if k == 0:
        q = [r / 2, (R[2, 1] - R[1, 2]) / (2 * r), (R[0, 2] - R[2, 0]) / (2 * r), (R[1, 0] - R[0, 1]) / (2 * r)]
    elif k == 1:
        q = [(R[2, 1] - R[1, 2]) / (2 * r), r / 2, (R[0, 1] + R[1, 0]) / (2 * r), (R[0, 2] + R[2, 0]) / (2 * r)]
    elif k == 2:
        q = [(R[0, 2] - R[2, 0]) / (2 * r), (R[0, 1] + R[1, 0]) / (2 * r), r / 2, (R[1, 2] + R[2, 1]) / (2 * r)]
    else:
        q = [(R[1, 0] - R[0, 1]) / (2 * r), (R[0, 2] + R[2, 0]) / (2 * r), (R[1, 2] + R[2, 1]) / (2 * r), r / 2]
    q = np.array(q)
    return q if q[0] >= 0 else -q


def align(means, quats, keyframe_of, R_old, t_old, R_new, t_new):
    """p_new = T_new^(m) (T_old^(m))^-1 p with world->camera poses, i.e.
    R_new^T (R_old p + t_old - t_new); the rotation becomes (R_new^T R_old) R(q).
    keyframe_of [N] (-1: not moved); R_* [K][3][3], t_* [K][3]."""
    means = np.array(means, np.float64)
    quats = np.array(quats, np.float64)
    for i, m in enumerate(np.asarray(keyframe_of)):
        if m < 0:
            continue
        Ro, to, Rn, tn = (np.asarray(a[m], np.float64) for a in (R_old, t_old, R_new, t_new))
        means[:, i] = Rn.T @ (Ro @ means[:, i] + to - tn)
        qr = rot_to_quat(Rn.T @ Ro)
        quats[:, i] = quat_mul(qr, quats[:, i])
    return means, quats


def revoxelize(means, level):
    """Keys of every anchor at its level after a move, and the keep mask that
    merges anchors sharing a voxel into the one with the lowest index."""
    means = np.asarray(means, np.float64)
    keys, keep, seen = [], np.ones(means.shape[1], bool), set()
    for i in range(means.shape[1]):
        eps = EPS[int(level[i])]
        k = voxel_key(int(level[i]), np.floor(means[:, i] / eps).astype(np.int64))
        keys.append(k)
        if k in seen:
            keep[i] = False
        seen.add(k)
    return np.array(keys, np.uint64), keep
