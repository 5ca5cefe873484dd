"""The allocation-free chunk close (kgs_accumulate_stats_static, for callers
that cannot allocate) against the context entry point kgs_accumulate_stats on
the same statistics, and both against the FP64 chunk rules: two calls in a row,
the second on fewer Gaussians, so the static partials hold the first call's
values when the second starts."""
import numpy as np
import pytest
import torch

from oracle import lifecycle
from paper_2606_30436_amd import _lib as L
from paper_2606_30436_amd.rasterizer import LifecycleState, Rasterizer, ViewStats
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _stats(rng, n, V):
    om = (rng.integers(0, 60, n) * (rng.uniform(size=n) < 0.6)).astype(np.int32)
    ka = np.minimum(om, rng.integers(0, 12 * V, n)).astype(np.int32)
    ka[: n // 50] = 5 * V  # exactly at the densify threshold
    gam = om * rng.uniform(0.02, 0.3, n)
    st = ViewStats.zeros(n)
    st.kappa_sum.copy_(torch.from_numpy(ka))
    st.omega_sum.copy_(torch.from_numpy(om))
    st.gamma_sum.copy_(torch.from_numpy(gam))
    return st, ka, om, gam


def _state(rng, n):
    s = LifecycleState.zeros(n)
    s.densify.copy_(torch.from_numpy((rng.uniform(size=n) < 0.1).astype(np.uint8)))
    s.prune_score.copy_(torch.from_numpy(rng.uniform(0, 0.6, n)))
    return s


def _clone_stats(st):
    return ViewStats(*(t.clone() for t in (st.kappa_sum, st.omega_sum, st.gamma_sum, st.grad_norm_sum,
                                           st.view_count, st.max_radius)))


def test_static_chunk_close_equals_the_context_entry_point():
    rng = np.random.default_rng(77)
    R = Rasterizer(64, 32, max_views=1, max_gaussians=400_000)
    for call, (n, V) in enumerate([(300_001, 7), (1_000, 15)]):
        say(f"[gpu] static chunk close, call {call}: n={n} V={V}")
        st_a, ka, om, gam = _stats(rng, n, V)
        st_b = _clone_stats(st_a)
        s_a = _state(rng, n)
        s_b = LifecycleState(s_a.densify.clone(), s_a.prune_score.clone())
        D0, P0 = s_a.densify.cpu().numpy().astype(bool), s_a.prune_score.cpu().numpy()
        L.kgs_accumulate_stats(R.ctx, st_a.c(), n, V, s_a.c(), 5.0, 1, None)
        L.kgs_accumulate_stats_static(st_b.c(), n, V, s_b.c(), 5.0, 1, None)
        torch.cuda.synchronize()
        # the same kernels on the same inputs: identical bits
        assert torch.equal(s_a.densify, s_b.densify) and torch.equal(s_a.prune_score, s_b.prune_score)
        for t in (st_b.kappa_sum, st_b.omega_sum, st_b.gamma_sum):
            assert not t.any()  # reset
        ref = lifecycle.chunk_scores_from_sums(ka, om, gam, V)
        D, P = lifecycle.global_update(D0, P0, ref["sd"], ref["sp"], 5.0)
        assert np.array_equal(s_b.densify.cpu().numpy().astype(bool), D)
        assert np.abs(s_b.prune_score.cpu().numpy() - P).max() <= 1e-12
    R.close()


def test_static_chunk_close_rejects_sizes_beyond_its_array():
    st = ViewStats.zeros(16)
    s = LifecycleState.zeros(16)
    with pytest.raises(L.KgsError) as e:
        L.kgs_accumulate_stats_static(st.c(), L.ACCUMULATE_STATIC_MAX_N + 1, 4, s.c(), 5.0, 0, None)
    assert e.value.code == L.KGS_ERR_INVALID_ARG
    L.kgs_accumulate_stats_static(st.c(), 0, 4, s.c(), 5.0, 0, None)  # empty: nothing to do
