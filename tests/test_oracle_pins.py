"""Pins of the FP64 oracle against mathematics it does not share code with:
textbook closed forms, library routines, brute force, invariants and finite
differences.  CPU only."""
import math

import numpy as np
import pytest
import scipy.special
import torch

import oracle
from oracle import OracleConfig, brute
from paper_2606_30436_amd import scenes

CFG = OracleConfig()


# ------------------------------------------------------------------ pose
def _skew(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


def test_se3_exp_identity_and_inverse():
    assert np.allclose(oracle.se3_exp(np.zeros(6)), np.eye(4), atol=0, rtol=0)
    rng = np.random.default_rng(0)
    for _ in range(5):
        xi = rng.normal(0, 0.7, 6)
        assert np.allclose(oracle.se3_exp(xi) @ oracle.se3_exp(-xi), np.eye(4), atol=1e-13)


def test_se3_exp_rotation_is_rodrigues():
    rng = np.random.default_rng(1)
    for _ in range(5):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        th = rng.uniform(0.01, 2.5)
        K = _skew(axis)
        R = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K  # Rodrigues
        T = oracle.se3_exp(np.concatenate([np.zeros(3), axis * th]))
        assert np.allclose(T[:3, :3], R, atol=1e-13)
        assert np.allclose(T[:3, 3], 0.0, atol=0)
    rho = np.array([0.3, -0.2, 0.7])
    T = oracle.se3_exp(np.concatenate([rho, np.zeros(3)]))
    assert np.allclose(T[:3, :3], np.eye(3), atol=0) and np.allclose(T[:3, 3], rho, atol=1e-15)


def test_se3_exp_deriv_matches_central_differences():
    rng = np.random.default_rng(2)
    xi = rng.normal(0, 0.4, 6)
    h = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        fd = (oracle.se3_exp(xi + e) - oracle.se3_exp(xi - e)) / (2 * h)
        assert np.allclose(oracle.se3_exp_deriv(xi, k), fd, atol=1e-8)


# ------------------------------------------------------- spherical harmonics
def _scipy_real_sh(degree, d):
    """Real SH from scipy's complex Y_l^m (Condon-Shortley phase included):
    sqrt2 Re Y_l^m for m > 0, sqrt2 Im Y_l^|m| for m < 0."""
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0])
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = scipy.special.sph_harm(abs(m), l, phi, theta)
            if m > 0:
                out.append(math.sqrt(2) * Y.real)
            elif m < 0:
                out.append(math.sqrt(2) * Y.imag)
            else:
                out.append(Y.real)
    return np.array(out)


@pytest.mark.filterwarnings("ignore::DeprecationWarning")
def test_sh_matches_scipy_and_polynomials():
    rng = np.random.default_rng(3)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ref = _scipy_real_sh(3, d)
        Y, _ = oracle.sh_eval(3, d)
        assert np.allclose(Y, ref, atol=1e-12)
        Yt = brute.real_sh_polys(torch.tensor(d)[None], 3)[0].numpy()
        assert np.allclose(Yt, ref, atol=1e-12)


def test_sh_gradient_tangential_fd():
    rng = np.random.default_rng(4)
    for _ in range(10):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        _, dY = oracle.sh_eval(3, d)
        P = np.eye(3) - np.outer(d, d)
        h = 1e-6
        for r in range(3):
            e = np.zeros(3)
            e[r] = h
            dp, dm = d + e, d - e
            fd = (oracle.sh_eval(3, dp / np.linalg.norm(dp))[0] - oracle.sh_eval(3, dm / np.linalg.norm(dm))[0]) / (2 * h)
            # derivative of Y(v/|v|) at |v| = 1 is P dY
            assert np.allclose((dY @ P)[:, r], fd, atol=1e-7)


def test_sh_orthonormal_on_sphere():
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 6 products exactly
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    G = np.zeros((16, 16))
    for z, w in zip(xg, wg):
        for j in range(nphi):
            ph = 2 * math.pi * j / nphi
            s = math.sqrt(1 - z * z)
            Y, _ = oracle.sh_eval(3, np.array([s * math.cos(ph), s * math.sin(ph), z]))
            G += w * (2 * math.pi / nphi) * np.outer(Y, Y)
    assert np.allclose(G, np.eye(16), atol=1e-12)


# ------------------------------------------------------------- projection
def _one_gaussian(mean, log_scales, quat, logit, rgb=(0.7, 0.4, 0.2), W=64, H=48, f=50.0, cx=None, cy=None,
                  R=np.eye(3), t=np.zeros(3)):
    sh = np.zeros((1, 3, 1), np.float32)
    sh[0, :, 0] = (np.asarray(rgb) - 0.5) * 2 * math.sqrt(math.pi)
    cam = scenes.make_camera(R, t, f, f, W / 2 if cx is None else cx, H / 2 if cy is None else cy, W, H)
    return scenes.Scene(np.asarray(mean, np.float32).reshape(3, 1), np.asarray(log_scales, np.float32).reshape(3, 1),
                        np.asarray(quat, np.float32).reshape(4, 1), np.asarray([logit], np.float32), sh, 0,
                        scenes.stack_cameras([cam]), np.zeros((1, 6), np.float32))


def test_degree0_colour_is_rgb_and_on_axis_covariance_closed_form():
    # rotation about the optical axis by angle th: Sigma2D = (f/z)^2 R2 diag(s1^2, s2^2) R2^T + eps I
    th, z, f = 0.6, 5.0, 50.0
    s = np.array([0.08, 0.03, 0.05])
    q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
    sc = _one_gaussian([0, 0, z], np.log(s), q, 2.0, f=f)
    p = oracle.View(sc, 0, CFG).proj()
    assert p["visible"][0]
    assert np.allclose(p["color"][0], [0.7, 0.4, 0.2], atol=1e-6)  # float32 inputs
    R2 = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    S = (f / z) ** 2 * R2 @ np.diag(s[:2] ** 2) @ R2.T + CFG.eps2d * np.eye(2)
    a, b, c = p["conic"][0]
    assert np.allclose(np.array([[a, b], [b, c]]) @ S, np.eye(2), atol=1e-5)  # scales are float32
    # rotation about x by angle th: the y-z block rotates, the image sees its yy entry
    q = [math.cos(th / 2), math.sin(th / 2), 0, 0]
    sc = _one_gaussian([0, 0, z], np.log(s), q, 2.0, f=f)
    p = oracle.View(sc, 0, CFG).proj()
    Rx = np.array([[1, 0, 0], [0, math.cos(th), -math.sin(th)], [0, math.sin(th), math.cos(th)]])
    Sw = Rx @ np.diag(s ** 2) @ Rx.T
    S = (f / z) ** 2 * Sw[:2, :2] + CFG.eps2d * np.eye(2)
    a, b, c = p["conic"][0]
    assert np.allclose(np.array([[a, b], [b, c]]) @ S, np.eye(2), atol=1e-5)
    assert p["depth"][0] == pytest.approx(z)


def test_jacobian_is_pinhole_fd_and_guard_band_clamps():
    # tiny isotropic Gaussian off axis: Sigma2D - eps I = s^2 J J^T, J = d pi / d t by FD
    f, z = 60.0, 4.0
    t = np.array([0.7, -0.4, z])
    s = 1e-3
    sc = _one_gaussian(t, np.log([s, s, s]), [1, 0, 0, 0], 3.0, f=f, W=80, H=60)
    p = oracle.View(sc, 0, OracleConfig(eps2d=0.0)).proj()
    tt = sc.means[:, 0].astype(np.float64)
    ss = math.exp(float(np.float32(np.log(s))))

    def pi(v):
        return np.array([f * v[0] / v[2] + 40.0, f * v[1] / v[2] + 30.0])
    J = np.stack([(pi(tt + h) - pi(tt - h)) / 2e-7 for h in np.eye(3) * 1e-7], axis=1)
    S = ss * ss * J @ J.T
    a, b, c = p["conic"][0]
    assert np.allclose(np.linalg.inv(np.array([[a, b], [b, c]])), S, rtol=1e-6, atol=1e-15)
    assert np.allclose(p["mu"][0], pi(tt), atol=1e-9)
    # far outside the frustum in x: J uses the clamped x/z = g W / (2 f)
    t2 = np.array([5.0 * z, 0.0, z])
    sc = _one_gaussian(t2, np.log([0.5, 0.5, 0.5]), [1, 0, 0, 0], 3.0, f=f, W=80, H=60)
    p = oracle.View(sc, 0, OracleConfig(eps2d=0.0)).proj()
    ux = CFG.guard * 40.0 / f
    J = np.array([[f / z, 0, -f * ux / z], [0, f / z, 0]])
    ss = math.exp(float(np.float32(np.log(0.5))))
    S = ss * ss * J @ J.T
    a, b, c = p["conic"][0]
    assert np.allclose(np.linalg.inv(np.array([[a, b], [b, c]])), S, rtol=1e-9)


def test_single_isotropic_gaussian_image_closed_form():
    """Camera-facing isotropic Gaussian on the axis: C(p) = c alpha(p),
    alpha = min(0.99, o exp(-|p - mu|^2 / (2 sigma^2))), sigma^2 = s^2 f^2 / z^2 + eps,
    zero where o exp(.) < 1/255; depth = alpha z; T = 1 - alpha."""
    z, f, W, H = 6.0, 50.0, 48, 40
    ls = np.float32(math.log(0.25))
    logit = np.float32(1.3)
    sc = _one_gaussian([0, 0, z], [ls] * 3, [0.3, -0.5, 0.1, 0.8], logit, f=f, W=W, H=H, cx=W / 2 + 0.25, cy=H / 2 - 0.4)
    img = oracle.View(sc, 0, CFG).image()
    s2 = math.exp(2 * float(ls))
    sig2 = s2 * f * f / (z * z) + CFG.eps2d
    o = 1 / (1 + math.exp(-float(logit)))
    py, px = np.mgrid[0:H, 0:W] + 0.5
    r2 = (px - (W / 2 + 0.25)) ** 2 + (py - (H / 2 - 0.4)) ** 2
    raw = o * np.exp(-r2 / (2 * sig2))
    alpha = np.where(raw >= 1 / 255, np.minimum(0.99, raw), 0.0)
    assert alpha.max() > 0.5 and (alpha == 0).any()
    for ch, c in enumerate([0.7, 0.4, 0.2]):
        assert np.allclose(img["color"][ch], np.float32(c) * 0 + c * alpha, atol=2e-7)
    assert np.allclose(img["depth"], alpha * z, atol=1e-12)
    assert np.allclose(img["tfinal"], 1 - alpha, atol=1e-15)
    # footprint = pixel centres inside the ellipse q <= 2 ln(255 o)
    st = oracle.View(sc, 0, CFG).stats(np.zeros((3, H, W), np.float32))
    assert st["omega"][0] == int((r2 / sig2 <= 2 * math.log(255 * o)).sum())


def _stack_scene(n, logit, W=32, H=32):
    """n Gaussians centred exactly on pixel (16, 16)'s centre at increasing depth."""
    cx = 16.5
    means = np.stack([np.zeros(n), np.zeros(n), np.linspace(3.0, 4.0, n)]).astype(np.float32)
    sh = np.zeros((1, 3, n), np.float32)
    sh[0] = ((1.0 - 0.5) * 2 * math.sqrt(math.pi))
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 40.0, 40.0, cx, cx, W, H)
    return scenes.Scene(means, np.full((3, n), -2.5, np.float32), np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)),
                        np.full(n, logit, np.float32), sh, 0, scenes.stack_cameras([cam]), np.zeros((1, 6), np.float32))


@pytest.mark.parametrize("alpha,kstar", [(0.5, 13), (0.8, 5)])
def test_transmittance_cutoff_stack(alpha, kstar):
    """k* = max{k : (1 - alpha)^k >= T_min}: the Gaussian that would push T below
    1e-4 is not blended."""
    logit = np.float32(math.log(alpha / (1 - alpha)))
    a = 1 / (1 + math.exp(-float(logit)))
    assert kstar == max(k for k in range(40) if (1 - a) ** k >= 1e-4)
    sc = _stack_scene(20, logit)
    v = oracle.View(sc, 0, CFG)
    img = v.image()
    c = float(v.proj()["color"][0, 0])
    assert c == pytest.approx(1.0, abs=1e-6)
    assert img["nblend"][16, 16] == kstar
    assert img["color"][0, 16, 16] == pytest.approx(c * (1 - (1 - a) ** kstar), rel=1e-12)
    assert img["last"][16, 16] == kstar


def test_alpha_max_clamp_single():
    """o -> 1 clamps alpha at 0.99: T = 0.01 after one Gaussian."""
    sc1 = _stack_scene(1, np.float32(20.0))
    img = oracle.View(sc1, 0, CFG).image()
    assert img["tfinal"][16, 16] == pytest.approx(0.01, rel=1e-12)


@pytest.mark.parametrize("sign", [+1, -1])
def test_alpha_min_threshold(sign):
    """A pixel whose alpha is 1/255 * (1 +- 1e-3) is blended or skipped."""
    z, f = 5.0, 40.0
    ls = np.float32(math.log(0.1))
    logit = np.float32(0.0)
    o = 0.5
    sig2 = math.exp(2 * float(ls)) * f * f / (z * z) + CFG.eps2d
    target = (1 / 255) * (1 + sign * 1e-3)
    r2 = -2 * sig2 * math.log(target / o)
    dx = math.sqrt(r2)
    # pixel (0, 10) centre at (0.5, 10.5); put the mean dx to its right on the same row
    cx = 0.5 + dx
    sc = _one_gaussian([0, 0, z], [ls] * 3, [1, 0, 0, 0], logit, f=f, W=64, H=21, cx=cx, cy=10.5)
    img = oracle.View(sc, 0, CFG).image()
    val = img["color"][0, 10, 0]
    if sign > 0:
        assert val == pytest.approx(0.7 * target, rel=1e-5)
    else:
        assert val == 0.0


# ------------------------------------------------------------ far plane
@pytest.mark.parametrize("mean_z,t_z,kept", [
    (9.999, 0.0, True),          # just inside the mask
    (10.0, 0.0, False),          # exactly at far: culled (the mask keeps z < far)
    (10.001, 0.0, False),        # beyond
    (10.0, -2.0 ** -30, True)])  # FP64 z = far - 2^-30 is kept; its FP32 rounding equals far
def test_far_plane_cull_closed_form(mean_z, t_z, kept):
    """Single-level distance mask (appendix, LoD mask): a Gaussian is rendered
    only while its camera depth is below far, decided on the FP64 camera point.
    A kept Gaussian's image is the closed form of a camera-facing isotropic
    Gaussian; a culled one leaves the image empty.  The tile-free renderer,
    which has its own far-plane test, agrees."""
    far, f, W, H = 10.0, 300.0, 40, 32
    ls = np.float32(math.log(0.05))
    logit = np.float32(0.7)
    cfg = OracleConfig(far=far)
    sc = _one_gaussian([0, 0, mean_z], [ls] * 3, [1, 0, 0, 0], logit, f=f, W=W, H=H, t=np.array([0.0, 0.0, t_z]))
    z = float(np.float32(mean_z)) + float(np.float32(t_z))
    assert (z < far) == kept
    v = oracle.View(sc, 0, cfg)
    img = v.image()
    assert bool(v.proj()["visible"][0]) == kept
    o = 1 / (1 + math.exp(-float(logit)))
    sig2 = math.exp(2 * float(ls)) * f * f / (z * z) + cfg.eps2d
    py, px = np.mgrid[0:H, 0:W] + 0.5
    raw = o * np.exp(-((px - W / 2) ** 2 + (py - H / 2) ** 2) / (2 * sig2))
    alpha = np.where(raw >= 1 / 255, np.minimum(0.99, raw), 0.0) if kept else np.zeros((H, W))
    assert alpha.max() > 0.3 or not kept
    assert np.allclose(img["color"][0], 0.7 * alpha, atol=2e-7)
    assert np.allclose(img["depth"], alpha * z, atol=1e-12)
    C, D, _ = brute.render(_torch_params(sc), sc.cams[0], 0, cfg, torch.zeros(6, dtype=torch.float64))
    assert np.allclose(C.detach().numpy(), img["color"], atol=1e-12)
    assert np.allclose(D.detach().numpy(), img["depth"], atol=1e-12)


def test_zero_opacity_invariance():
    sc = scenes.tiny_scene(seed=5, n=20, degree=2)
    v0 = oracle.View(sc, 0, CFG)
    img0 = v0.image()
    rng = np.random.default_rng(0)
    g0 = v0.backward(rng.normal(size=(3, sc.height, sc.width)), rng.normal(size=(sc.height, sc.width)))
    extra = scenes.tiny_scene(seed=6, n=10, degree=2)
    both = scenes.Scene(np.concatenate([sc.means, extra.means], 1), np.concatenate([sc.log_scales, extra.log_scales], 1),
                        np.concatenate([sc.quats, extra.quats], 1), np.concatenate([sc.logits, np.full(10, -20, np.float32)]),
                        np.concatenate([sc.sh, extra.sh], 2), 2, sc.cams, sc.pose_xi)
    v1 = oracle.View(both, 0, CFG)
    img1 = v1.image()
    for k in ("color", "depth", "tfinal", "nblend"):
        assert np.array_equal(img0[k], img1[k])
    rng = np.random.default_rng(0)
    g1 = v1.backward(rng.normal(size=(3, sc.height, sc.width)), rng.normal(size=(sc.height, sc.width)))
    # FP64 gradient sums are accumulated by several threads, so compare to 1e-12
    assert np.allclose(g1["means"][:, :20], g0["means"], rtol=1e-12, atol=0) and not g1["means"][:, 20:].any()
    assert not g1["logits"][20:].any() and np.allclose(g1["pose_xi"], g0["pose_xi"], rtol=1e-12, atol=0)
    st = v1.stats(sc.target[0])
    assert not st["omega"][20:].any()


# ----------------------------------------------------------- brute force
def _torch_params(sc):
    return {k: torch.tensor(getattr(sc, k).astype(np.float64), requires_grad=True)
            for k in ("means", "log_scales", "quats", "logits", "sh")}


BG = (0.2, 0.55, 0.9)


@pytest.mark.parametrize("seed,degree,pose,far,bg", [
    (0, 0, 0.0, 1e30, (0.0, 0.0, 0.0)), (1, 1, 0.02, 1e30, (0.0, 0.0, 0.0)), (2, 3, 0.05, 1e30, (0.0, 0.0, 0.0)),
    (3, 2, 0.0, 1e30, (0.0, 0.0, 0.0)),
    # a non-zero background: C = sum T_j alpha_j c_j + T_final bg, and its share of dL/dalpha
    (4, 1, 0.03, 1e30, BG), (5, 3, 0.0, 1e30, BG),
    # the distance mask in the middle of the depth range (2-6 m), with a background
    (6, 2, 0.02, 4.0, BG), (7, 0, 0.0, 3.5, (0.0, 0.0, 0.0))])
def test_oracle_matches_tile_free_autograd(seed, degree, pose, far, bg):
    cfg = OracleConfig(far=far, bg=bg)
    sc = scenes.tiny_scene(seed=seed, n=18, degree=degree, n_views=2, pose_sigma=pose)
    rng = np.random.default_rng(seed)
    if far < 1e29:
        z = sc.means[2]
        assert (z < far - 0.1).sum() >= 3 and (z > far + 0.1).sum() >= 3  # both sides of the mask are populated
    for v in range(2):
        wC = rng.normal(size=(3, sc.height, sc.width))
        wD = rng.normal(size=(sc.height, sc.width))
        ov = oracle.View(sc, v, cfg)
        img = ov.image()
        P = _torch_params(sc)
        xi = torch.tensor(sc.pose_xi[v].astype(np.float64), requires_grad=True)
        C, D, _ = brute.render(P, sc.cams[v], degree, cfg, xi)
        assert np.allclose(C.detach().numpy(), img["color"], atol=1e-10)
        assert np.allclose(D.detach().numpy(), img["depth"], atol=1e-9)
        L = (C * torch.tensor(wC)).sum() + (D * torch.tensor(wD)).sum()
        L.backward()
        g = ov.backward(wC, wD)
        for k in ("means", "log_scales", "quats", "logits", "sh"):
            ref = P[k].grad.numpy()
            assert np.allclose(g[k], ref, rtol=1e-7, atol=1e-9 * (1 + np.abs(ref).max())), k
        assert np.allclose(g["pose_xi"], xi.grad.numpy(), rtol=1e-7, atol=1e-9 * (1 + np.abs(xi.grad.numpy()).max()))


@pytest.mark.parametrize("tile", [(8, 32), (32, 8), (32, 16), (16, 32)])
def test_oracle_image_is_tile_shape_invariant(tile):
    sc = scenes.tiny_scene(seed=7, n=40, degree=1, W=72, H=56)
    a = oracle.View(sc, 0, CFG).image()
    b = oracle.View(sc, 0, OracleConfig(tile_w=tile[0], tile_h=tile[1])).image()
    for k in ("color", "depth", "tfinal", "nblend"):
        assert np.array_equal(a[k], b[k])


# ---------------------------------------------------- finite differences
def _loss(sc, v, cfg, params, wC, wD):
    img = oracle.View(sc, v, cfg, params).image()
    return float((img["color"] * wC).sum() + (img["depth"] * wD).sum())


@pytest.mark.parametrize("seed,bg", [(11, (0.0, 0.0, 0.0)), (12, (0.0, 0.0, 0.0)), (13, (0.8, 0.3, 0.6))])
def test_backward_matches_fp64_central_differences(seed, bg):
    """Smooth configuration (thresholds off): analytic gradient == central FD.
    The background case checks the T_final * bg term of dL/dalpha."""
    cfg = OracleConfig.smooth(bg=bg)
    sc = scenes.tiny_scene(seed=seed, n=6, degree=3, W=24, H=20, n_views=1, pose_sigma=0.03,
                           log_scale_mu=-1.6)
    rng = np.random.default_rng(seed)
    wC = rng.normal(size=(3, sc.height, sc.width))
    wD = rng.normal(size=(sc.height, sc.width)) * 0.1
    g = oracle.View(sc, 0, cfg).backward(wC, wD)
    base = {k: getattr(sc, k).astype(np.float64) for k in ("means", "log_scales", "quats", "logits", "sh", "pose_xi")}
    checks = [("means", (0, 1)), ("means", (2, 3)), ("log_scales", (1, 2)), ("quats", (0, 4)), ("quats", (3, 0)),
              ("logits", (5,)), ("sh", (0, 1, 2)), ("sh", (5, 0, 3)), ("sh", (13, 2, 1))]
    checks += [("pose_xi", (0, k)) for k in range(6)]
    for name, idx in checks:
        h = 1e-6 * max(1.0, abs(base[name][idx]))
        vals = []
        for sgn in (1, -1):
            pp = {k: v.copy() for k, v in base.items()}
            pp[name][idx] += sgn * h
            vals.append(_loss(sc, 0, cfg, pp, wC, wD))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = g[name][idx[1:]] if name == "pose_xi" else g[name][idx]
        assert an == pytest.approx(fd, rel=2e-5, abs=2e-6 * (1 + abs(fd))), (name, idx)



def test_translation_identity():
    """Moving every Gaussian by d and the camera with them leaves the image
    unchanged:  sum_i dL/dmu_i = R'^T dL/drho  (at xi = 0)."""
    sc = scenes.tiny_scene(seed=21, n=25, degree=2, W=40, H=32)
    rng = np.random.default_rng(1)
    g = oracle.View(sc, 0, CFG).backward(rng.normal(size=(3, 32, 40)), rng.normal(size=(32, 40)))
    R = sc.cams[0]["R"].reshape(3, 3).astype(np.float64)
    assert np.allclose(g["means"].sum(axis=1), R.T @ g["pose_xi"][:3], rtol=1e-9, atol=1e-12)


# ------------------------------------------------------------ statistics
def test_stats_brute_force_counts_and_invariants():
    sc = scenes.tiny_scene(seed=31, n=30, degree=1, W=48, H=40)
    v = oracle.View(sc, 0, CFG)
    img = v.image()
    st = v.stats(sc.target[0], 0.1)
    pr = v.proj()
    # brute force: every visible Gaussian at every pixel, no tiles, (fp32 depth, index) order
    vis = np.nonzero(pr["visible"])[0]
    order = sorted(vis, key=lambda i: (np.float32(pr["depth"][i]), i))
    omega = np.zeros(sc.n, int)
    kappa = np.zeros(sc.n, int)
    err = np.abs(sc.target[0].astype(np.float64) - img["color"]).sum(0)
    for py in range(40):
        for px in range(48):
            T = 1.0
            for i in order:
                dx, dy = px + 0.5 - pr["mu"][i, 0], py + 0.5 - pr["mu"][i, 1]
                a, b, c = pr["conic"][i]
                raw = pr["opacity"][i] * math.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
                if raw < CFG.alpha_min:
                    continue
                Tn = T * (1 - min(raw, CFG.alpha_max))
                if Tn < CFG.t_min:
                    break
                omega[i] += 1
                kappa[i] += err[py, px] > 0.1
                T = Tn
    assert np.array_equal(st["omega"], omega) and np.array_equal(st["kappa"], kappa)
    assert (st["kappa"] <= st["omega"]).all()
    assert st["omega"].sum() == img["nblend"].sum()
    assert np.array_equal(st["mask"], err > 0.1)


# ------------------------------------------------------------ binning
def test_bin_keys_match_python_sorted():
    rng = np.random.default_rng(9)
    n = 300
    W, H, TW, TH = 100, 70, 16, 16
    view = rng.integers(0, 3, n)
    gid = rng.permutation(n).astype(np.int64)
    fxi = rng.integers(-30, 130, n)
    fyi = rng.integers(-30, 100, n)
    rx = rng.integers(0, 25, n)
    ry = rng.integers(0, 25, n)
    depth = rng.uniform(1, 3, n).astype(np.float32)
    depth[:40] = depth[40:80]  # equal depths: ties broken by index
    db = depth.view(np.uint32)
    keys, gids = oracle.bin_keys(view, gid, fxi, fyi, rx, ry, db, W, H, TW, TH)
    TX, TY = -(-W // TW), -(-H // TH)
    ref = []
    for s in range(n):
        for ty in range(max(0, (fyi[s] - ry[s]) // TH), min(TY, (fyi[s] + ry[s]) // TH + 1)):
            for tx in range(max(0, (fxi[s] - rx[s]) // TW), min(TX, (fxi[s] + rx[s]) // TW + 1)):
                ref.append((int(view[s]) * TX * TY + ty * TX + tx, int(db[s]), int(gid[s])))
    ref.sort()
    assert len(ref) == len(keys)
    assert all(int(k) == (r[0] << 32 | r[1]) and g == r[2] for k, g, r in zip(keys, gids, ref))


def test_oracle_tile_lists_follow_the_binning_contract():
    sc = scenes.tiny_scene(seed=41, n=35, degree=0, W=70, H=45)
    v = oracle.View(sc, 0, CFG)
    pr = v.proj()
    vis = np.nonzero(pr["visible"])[0]
    keys, gids = oracle.bin_keys(np.zeros(len(vis)), vis, pr["fxi"][vis], pr["fyi"][vis], pr["rx"][vis],
                                 pr["ry"][vis], pr["depth"][vis].astype(np.float32).view(np.uint32), 70, 45, 16, 16)
    tile, gid = v.pairs()
    assert np.array_equal(keys >> np.uint64(32), tile.astype(np.uint64)) and np.array_equal(gids, gid)


@pytest.mark.parametrize("gap_ulps,t_z,hazard", [(1, 0.0, True), (0, 0.0, True), (2, 0.0, False),
                                                 (1, 2.0 ** -25, True)])
def test_depth_order_hazard_margin(gap_ulps, t_z, hazard):
    """The image's fourth margin plane flags a pixel only where two consecutive
    contributing Gaussians have FP32 depth keys equal or one unit apart, and then
    measures how close either FP64 depth lies to an FP32 rounding boundary.  At
    depth 4 the float spacing is 2^-22 below and 2^-21 above, so a float-exact 4
    sits 2^-23 from the boundary below; a camera shift of 2^-25 moves it."""
    z0 = np.float32(4.0)
    z1 = z0
    for _ in range(gap_ulps):
        z1 = np.nextafter(z1, np.float32(np.inf))
    sh = np.zeros((1, 3, 2), np.float32)
    cam = scenes.make_camera(np.eye(3), np.array([0.0, 0.0, t_z]), 40.0, 40.0, 16.5, 16.5, 32, 32)
    sc = scenes.Scene(np.array([[0.0, 0.0], [0.0, 0.0], [z0, z1]], np.float32), np.full((3, 2), -2.5, np.float32),
                      np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, 2)), np.full(2, 0.0, np.float32), sh, 0,
                      scenes.stack_cameras([cam]), np.zeros((1, 6), np.float32))
    m3 = oracle.View(sc, 0, CFG).image()["margins"][3][16, 16]
    if not hazard:
        assert m3 == np.inf
        return
    d0, d1 = float(z0) + t_z, float(z1) + t_z
    # distance from the nearest rounding boundary, by hand from the float spacing around 4
    def margin(d):
        f = np.float32(d)
        lo, hi = float(np.nextafter(f, np.float32(0))), float(np.nextafter(f, np.float32(np.inf)))
        return min(abs(d - (float(f) + hi) / 2), abs(d - (float(f) + lo) / 2)) / d
    assert m3 == pytest.approx(min(margin(d0), margin(d1)), rel=1e-12)
    if t_z == 0.0:
        assert m3 == pytest.approx(2.0 ** -23 / 4.0, rel=1e-12)  # half of the 2^-22 spacing below 4
