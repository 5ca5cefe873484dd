"""The map's gradient steps on the GPU: kgs_adam (through the C ABI) against the
FP64 Adam of the oracle, and the equal-PSNR check of the batched chunk against
the plain per-view loop (the same fit run both ways ends at the same PSNR)."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle.optim import adam_step
from paper_2606_30436_amd import _lib as L
from paper_2606_30436_amd import scenes
from paper_2606_30436_amd.fit import fit
from paper_2606_30436_amd.rasterizer import GaussianParams, Image, Rasterizer, device_cameras
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1_000_003, 1, 0])
def test_adam_matches_oracle(n):
    """Four steps on FP32 buffers against the FP64 definition fed the same FP32 state and constants: every
    update within 1e-5 of its own size plus 1e-6 lr and an ulp of theta (FP32 rounding of the moments, the
    square root and the quotient), the moments to 1e-6 of the magnitudes they add."""
    say(f"[gpu] adam n={n}")
    rng = np.random.default_rng(n + 5)
    th = rng.normal(size=n).astype(np.float32)
    dev = {k: torch.from_numpy(x).cuda() for k, x in
           dict(th=th, m=np.zeros(n, np.float32), v=np.zeros(n, np.float32)).items()}
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    # the entry point takes its constants as FP32: the oracle computes with the same values
    lr, b1, b2, eps = (float(np.float32(c)) for c in (3e-3, 0.9, 0.999, 1e-8))
    for t in range(1, 5):
        g = (rng.normal(size=n) * np.exp(rng.uniform(-8, 3, n))).astype(np.float32)
        if n > 10:
            g[::97] = 0.0
        prev = dev["th"].cpu().numpy()
        L.kgs_adam(dev["th"], dev["m"], dev["v"], torch.from_numpy(g).cuda(), n, t, lr, b1, b2, eps)
        torch.cuda.synchronize()
        ref_th, ref_m, ref_v = adam_step(prev, m, v, g, t, lr, b1, b2, eps)
        got_th, got_m, got_v = (dev[k].cpu().numpy() for k in ("th", "m", "v"))
        step_ref = ref_th - prev.astype(np.float64)
        step_got = got_th.astype(np.float64) - prev
        # theta is FP32: its own rounding (half an ulp of theta) comes on top of the update's error
        ulp = np.spacing(np.abs(got_th)).astype(np.float64)
        assert (np.abs(step_got - step_ref) <= 1e-5 * np.abs(step_ref) + 1e-6 * lr + ulp).all(), t
        # m may cancel (gradients of both signs): bound its rounding by the magnitudes it adds
        m_mag = b1 * np.abs(m.astype(np.float64)) + (1 - b1) * np.abs(g.astype(np.float64))
        assert (np.abs(got_m - ref_m) <= 1e-6 * m_mag).all(), t
        assert np.allclose(got_v, ref_v, rtol=1e-6, atol=1e-37)
        m, v = got_m, got_v


def test_equal_psnr_fit():
    """A map whose means and colours were perturbed, fitted 60 Adam steps towards renders of the unperturbed
    map: once with the chunk as one graph, once view by view; both must end within 0.05 dB, above the start."""
    true = scenes.tiny_scene(seed=11, n=600, W=160, H=96, degree=1, n_views=4, spread=0.8, log_scale_mu=-2.3)
    rng = np.random.default_rng(12)
    start = dataclasses.replace(true, means=(true.means + rng.normal(0, 0.02, true.means.shape)).astype(np.float32),
                                sh=(true.sh + rng.normal(0, 0.05, true.sh.shape)).astype(np.float32))
    V, H, W = true.n_views, true.height, true.width
    R = Rasterizer(W, H, V, true.n)
    R.project(GaussianParams.from_scene(true), device_cameras(true.cams))
    R.bin_sort()
    img = Image.empty(V, H, W)
    R.render_fwd(img)
    torch.cuda.synchronize()
    assert R.status() == 0
    target = img.color.clone()
    say("[gpu] equal-PSNR fit, batched")
    fb = fit(start, target, "batched", iters=60, tile=(16, 16), batch=64, far_z=100.0)
    say("[gpu] equal-PSNR fit, plain")
    fp = fit(start, target, "plain", iters=60, tile=(16, 16), batch=64, far_z=100.0)
    say(f"  start {fb['psnr_start_db']:.3f} dB, batched {fb['psnr_db']:.4f} dB, plain {fp['psnr_db']:.4f} dB")
    assert fb["psnr_start_db"] == fp["psnr_start_db"]
    assert abs(fb["psnr_db"] - fp["psnr_db"]) <= 0.05
    assert fb["psnr_db"] > fb["psnr_start_db"] + 0.5
