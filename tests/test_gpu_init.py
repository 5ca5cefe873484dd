"""Probabilistic initialisation on the GPU (kgs_init_spawn, through the C ABI)
against the FP64 oracle of Sec. 3.3's initialisation and Sec. 3.2's voxel rule.
Both sides take every decision in FP64; the spawning set must be identical
except at pixels whose decision the oracle finds within 1e-12 (relative) of
its threshold -- a P_kf next to a neighbour's in the suppression, or to the
pixel's uniform -- and the level and voxel of every spawned pixel identical
except within 1e-12 of a band edge or a voxel face.  The excluded counts are
printed and bounded."""
import numpy as np
import pytest
import scipy.ndimage
import torch

from oracle import init_prob as ip
from paper_2606_30436_amd import scenes
from paper_2606_30436_amd.mapping import Initializer, SpawnList
from paper_2606_30436_amd.rasterizer import GaussianParams, Image, Rasterizer, device_cameras
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _inputs(seed, V, H, W):
    rng = np.random.default_rng(seed)
    col = np.stack([scipy.ndimage.gaussian_filter(rng.uniform(size=(3, H, W)), (0, 1.2, 1.2)) for _ in range(V)])
    col[:, :, : H // 3, : W // 3] = 0.5                      # a flat patch
    dep = np.stack([scipy.ndimage.gaussian_filter(rng.uniform(2, 80, size=(H, W)), 2.0) for _ in range(V)])
    dep[:, -1, :3] = 0.0                                     # no depth there: never spawns
    ren = np.clip(col + rng.normal(0, 0.02, col.shape), 0, 1)
    rdep = dep * (1 + rng.normal(0, 0.01, dep.shape))
    u = rng.uniform(size=(V, H, W)) * 0.3                     # a third of the range: many spawn
    cams = []
    for v in range(V):
        a = 0.3 * v
        R = np.array([[np.cos(a), 0, -np.sin(a)], [0, 1, 0], [np.sin(a), 0, np.cos(a)]])
        cams.append(scenes.make_camera(R, np.array([0.5 * v, -1.0, 2.0]), 0.9 * W, 0.9 * W, W / 2, H / 2, W, H))
    f = np.float32
    return col.astype(f), dep.astype(f), ren.astype(f), rdep.astype(f), u.astype(f), scenes.stack_cameras(cams)


def _run(col, dep, u, cams, ren=None, rdep=None, capacity=None):
    V, _, H, W = col.shape
    I = Initializer(W, H, V)
    cap = capacity if capacity is not None else V * H * W
    out = SpawnList.empty(cap)
    pk = torch.full((V, H, W), float("nan"), device="cuda")
    t = lambda a: None if a is None else torch.from_numpy(a).cuda()
    I.spawn(t(col), t(dep), t(u), device_cameras(cams), out, cap, rendered=t(ren), rendered_depth=t(rdep), p_kf=pk)
    torch.cuda.synchronize()
    n = int(out.count.cpu().numpy().view(np.uint32)[0])
    m = min(n, cap)
    return dict(n=n, pixel=out.pixel[:m].cpu().numpy(), level=out.level[:m].cpu().numpy(),
                voxel=out.voxel[:m].cpu().numpy(), point=out.point[:m].cpu().numpy(),
                color=out.color[:m].cpu().numpy(), p_kf=pk.cpu().numpy())


def _compare(g, col, dep, u, cams, ren=None, rdep=None):
    V, _, H, W = col.shape
    got = {(int(a), int(b)): k for k, (a, b) in enumerate(g["pixel"])}
    assert len(got) == len(g["pixel"]) == g["n"]
    order = [(int(a), int(b)) for a, b in g["pixel"]]
    assert order == sorted(order)                             # (keyframe, row, column) order
    excluded = n_ref = 0
    for v in range(V):
        o = ip.spawn_candidates(col[v], dep[v], cams[v], u[v], None if ren is None else ren[v],
                                None if rdep is None else rdep[v])
        assert np.abs(g["p_kf"][v] - o["P_kf"]).max() <= 1e-7
        # a tie in the suppression flags both pixels (the margin is symmetric)
        near = (o["margin_nms"] <= 1e-12) | (o["margin_u"] <= 1e-12)
        mine = np.zeros(H * W, bool)
        mine[[p for (vv, p) in got if vv == v]] = True
        diff = (mine != o["spawn"].reshape(-1)) & ~near.reshape(-1)
        assert not diff.any(), np.flatnonzero(diff)[:8]
        excluded += int((near.reshape(-1) & (mine != o["spawn"].reshape(-1))).sum())
        n_ref += len(o["pixel"])
        for j, p in enumerate(o["pixel"]):
            k = got.get((v, int(p)))
            if k is None:
                continue
            if o["margin_level"][j] > 1e-12:
                assert g["level"][k] == o["level"][j]
            if o["margin_floor"][j] > 1e-12 and g["level"][k] == o["level"][j]:
                assert np.array_equal(g["voxel"][k], o["voxel"][j]), (v, p)
            assert np.allclose(g["point"][k], o["point"][j], rtol=1e-6, atol=1e-6)
            assert np.array_equal(g["color"][k], col[v][:, p // W, p % W])
    say(f"  spawned {g['n']} (oracle {n_ref}); differing at a margin: {excluded}")
    assert excluded <= max(2, 1e-3 * n_ref)
    return n_ref


@pytest.mark.parametrize("render", [False, True])
@pytest.mark.parametrize("V,H,W", [(2, 45, 70), (1, 1, 1), (3, 17, 300)])
def test_spawn_matches_oracle(V, H, W, render):
    """Ragged sizes (tiles of 32x16 and row segments of 256 pixels partly outside the image), a single pixel,
    a first keyframe (no render) and later ones (residual against the render)."""
    say(f"[gpu] init spawn V={V} {W}x{H} render={render}")
    col, dep, ren, rdep, u, cams = _inputs(V * 100 + H, V, H, W)
    g = _run(col, dep, u, cams, ren if render else None, rdep if render else None)
    _compare(g, col, dep, u, cams, ren if render else None, rdep if render else None)


def test_spawn_capacity():
    """A list shorter than the spawning pixels: the count is the full number and the first entries are the
    first pixels in order."""
    col, dep, ren, rdep, u, cams = _inputs(7, 2, 45, 70)
    full = _run(col, dep, u, cams)
    cut = _run(col, dep, u, cams, capacity=10)
    assert cut["n"] == full["n"] > 10
    assert np.array_equal(cut["pixel"], full["pixel"][:10]) and np.array_equal(cut["voxel"], full["voxel"][:10])


def test_spawn_full_size_keyframes():
    """Eight keyframes at 1242x375 along the 1 km trajectory: the input images and depth priors are renders of
    the noise-free 2M-Gaussian map, the rendered map is the perturbed one, as a mapping step would see."""
    sc = scenes.make_c3()
    V, H, W = sc.n_views, sc.height, sc.width
    say(f"[gpu] init spawn, full size V={V} {W}x{H}")
    true = scenes.Scene(sc.meta["true"]["means"], sc.log_scales, sc.quats, sc.logits, sc.meta["true"]["sh"], 3,
                        sc.cams, sc.pose_xi)
    R = Rasterizer(W, H, max_views=V, max_gaussians=sc.n, slot_capacity=3_000_000, pair_capacity=30_000_000,
                   far_z=80.0)
    cams = device_cameras(sc.cams)
    imgs = []
    for s in (true, sc):
        img = Image.empty(V, H, W)
        R.project(GaussianParams.from_scene(s), cams)
        R.bin_sort()
        R.render_fwd(img)
        torch.cuda.synchronize()
        imgs.append((img.color.cpu().numpy(), img.depth.cpu().numpy()))
    R.close()
    (col, dep), (ren, rdep) = imgs
    u = np.random.default_rng(9).uniform(size=(V, H, W)).astype(np.float32)
    g = _run(col, dep, u, sc.cams, ren, rdep)
    n_ref = _compare(g, col, dep, u, sc.cams, ren, rdep)
    assert n_ref > 100
