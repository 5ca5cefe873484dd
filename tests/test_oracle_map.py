"""Pins of the map-maintenance oracle (appendix "Dynamic Map Expansion" and
"Global Map Alignment"; Sec. 3.3 decisions acting on the map) against
hand-worked cases, scipy's rotations and geometric invariants.  CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import map_maint as mm


def test_voxel_key_layout_and_injectivity():
    assert mm.voxel_key(2, (0, 0, 0)) == (2 << 60) | ((1 << 19) << 40) | ((1 << 19) << 20) | (1 << 19)
    assert mm.voxel_key(0, (-(1 << 19), 0, (1 << 19) - 1)) == ((1 << 19) << 20) | ((1 << 20) - 1)
    keys = {mm.voxel_key(l, (x, y, z)) for l in range(5) for x in (-2, 0, 3) for y in (-1, 1) for z in (-7, 7)}
    assert len(keys) == 5 * 3 * 2 * 2
    with pytest.raises(AssertionError):
        mm.voxel_key(0, (1 << 19, 0, 0))


def test_insert_hand_worked():
    """Keys a b a c b into an empty map holding 10 anchors: a -> 10, b -> 11, c -> 12, created by candidates
    0, 1, 3; then c d: c is occupied (12), d is new (13)."""
    a, b, c, d = (mm.voxel_key(0, (i, 0, 0)) for i in range(4))
    table = {}
    anc, created, n = mm.insert(table, [a, b, a, c, b], 10)
    assert list(anc) == [10, 11, 10, 12, 11] and list(created) == [0, 1, 3] and n == 13
    anc, created, n = mm.insert(table, [c, d], n)
    assert list(anc) == [12, 13] and list(created) == [1] and n == 14


def test_spawn_params_closed_form():
    p = mm.spawn_params([0, 3], [[3, -13, 80], [1, 2, -1]], [[0.2, 0.5, 0.9], [1.0, 0.0, 0.25]])
    assert np.allclose(p["means"].T, [[0.3, -1.3, 8.0], [5.0, 10.0, -5.0]], rtol=1e-15)
    assert np.allclose(p["log_scales"], np.log([[0.1, 5.0]] * 3))
    assert np.allclose(p["sh0"] * mm.Y00 + 0.5, np.array([[0.2, 0.5, 0.9], [1.0, 0.0, 0.25]]).T, atol=1e-15)
    assert np.allclose(1 / (1 + np.exp(-p["logits"])), 0.1) and np.array_equal(p["quats"][0], [1, 1])


def test_densify_points_along_the_major_axis():
    """Scales (0.1, 0.5, 0.2): the points are mu +- 0.5 along the rotated y axis; rotating by 90 degrees about z
    takes y to -x."""
    q = np.array([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)])   # 90 degrees about z
    means = np.array([[1.0, 4.0], [2.0, 0.0], [3.0, 1.0]])
    ls = np.log(np.array([[0.1, 0.3], [0.5, 0.1], [0.2, 0.1]]))
    quats = np.stack([[1, 0, 0, 0], q], 1)
    out = mm.densify_points(means, ls, quats, [1, 1], centre=[0, 0, 0])
    assert np.allclose(out["point"], [[1, 2.5, 3], [1, 1.5, 3], [4, 0.3, 1], [4, -0.3, 1]], atol=1e-12)
    assert list(out["source"]) == [0, 0, 1, 1] and list(out["level"]) == [0, 0, 0, 0]
    assert np.array_equal(out["voxel"][0], [10, 25, 30])  # 1 / 0.1 and 3 / 0.1 round to 10 and 30 in FP64
    assert mm.densify_points(means, ls, quats, [0, 2], centre=[0, 0, 0])["point"].shape == (0, 3)


def test_compact_is_boolean_indexing():
    rng = np.random.default_rng(0)
    arr = {"means": rng.normal(size=(3, 9)), "logits": rng.normal(size=9)}
    dec = np.array([0, 2, 1, 2, 0, 0, 2, 1, 0])
    out = mm.compact(arr, dec)
    keep = dec != 2
    assert np.array_equal(out["means"], arr["means"][:, keep]) and np.array_equal(out["logits"], arr["logits"][keep])


def test_rotation_quaternion_round_trip_against_scipy():
    for R in Rotation.random(20, random_state=1).as_matrix():
        q = mm.rot_to_quat(R)
        ref = Rotation.from_matrix(R).as_quat()          # (x, y, z, w)
        ref = np.r_[ref[3], ref[:3]]
        ref = ref if ref[0] >= 0 else -ref
        assert np.allclose(q, ref, atol=1e-12)
        assert np.allclose(mm.quat_to_rot(q), R, atol=1e-12)


def _pose(seed):
    R = Rotation.random(random_state=seed).as_matrix()
    return R, np.random.default_rng(seed).normal(size=3) * 5


def test_alignment_keeps_every_anchor_fixed_in_its_keyframe():
    """Moving the anchors of keyframe m with T_new T_old^-1 leaves their camera-frame coordinates and
    orientations in keyframe m unchanged: R_new p_new + t_new = R_old p + t_old and R_new R(q_new) = R_old R(q);
    anchors of keyframe -1 stay; T_new = T_old is the identity."""
    rng = np.random.default_rng(2)
    n, K = 12, 3
    means = rng.normal(size=(3, n)) * 10
    quats = rng.normal(size=(4, n))
    quats /= np.linalg.norm(quats, axis=0)
    kf = rng.integers(-1, K, n)
    Ro, to = zip(*[_pose(10 + k) for k in range(K)])
    Rn, tn = zip(*[_pose(20 + k) for k in range(K)])
    m2, q2 = mm.align(means, quats, kf, Ro, to, Rn, tn)
    for i in range(n):
        m = kf[i]
        if m < 0:
            assert np.array_equal(m2[:, i], means[:, i]) and np.array_equal(q2[:, i], quats[:, i])
            continue
        assert np.allclose(Rn[m] @ m2[:, i] + tn[m], Ro[m] @ means[:, i] + to[m], atol=1e-9)
        assert np.allclose(Rn[m] @ mm.quat_to_rot(q2[:, i]), Ro[m] @ mm.quat_to_rot(quats[:, i]), atol=1e-12)
    m3, q3 = mm.align(means, quats, kf, Ro, to, Ro, to)
    assert np.allclose(m3, means, atol=1e-12)


def test_revoxelize_merges_into_the_lowest_index():
    means = np.array([[0.31, 5.0, 0.39, 0.31], [0.0, 0.0, 0.01, 0.0], [1.0, 1.0, 1.05, 1.0]])
    keys, keep = mm.revoxelize(means, [0, 0, 0, 1])
    # anchors 0 and 2 share level-0 voxel (3, 0, 10); anchor 3 sits at level 1 (another grid)
    assert list(keep) == [True, True, False, True]
    assert keys[0] == keys[2] != keys[3]
