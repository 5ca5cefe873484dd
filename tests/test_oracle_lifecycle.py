"""Pins of the lifecycle-statistics oracle: the paper's hyper-parameters, a
hand-built truth table of the global rules, and invariants of the chunk scores.
CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import OracleConfig, lifecycle
from paper_2606_30436_amd import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_thresholds_are_the_papers():
    hp = json.load(open(os.path.join(GOLD, "hyperparameters.json")))
    assert lifecycle.TAU_ERR == hp["tau_err"] and lifecycle.TAU_D == hp["tau_d"] and lifecycle.TAU_P == hp["tau_p"]
    assert scenes.CHUNK_KEYFRAMES == hp["chunk_size_C"]


def _truth_rows():
    rows = []
    for line in open(os.path.join(GOLD, "decide_truth_table.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        sd, sp, want = (x.strip() for x in line.split("|"))
        rows.append(([float(x) for x in sd.split(",")], [float(x) for x in sp.split(",")], int(want)))
    return rows


@pytest.mark.parametrize("sd,sp,want", _truth_rows())
def test_truth_table(sd, sp, want):
    D, P = np.zeros(1, bool), np.zeros(1)
    for a, b in zip(sd, sp):
        D, P = lifecycle.global_update(D, P, np.array([a]), np.array([b]))
    assert lifecycle.decide(D, P)[0] == want


def test_chunk_score_invariants():
    rng = np.random.default_rng(0)
    V, N = 8, 500
    omega = rng.integers(0, 40, (V, N)) * (rng.uniform(size=(V, N)) < 0.4)
    kappa = np.minimum(omega, rng.integers(0, 40, (V, N)))
    loss = rng.uniform(0.05, 0.3, V)
    s = lifecycle.chunk_scores(kappa, omega, loss)
    act = s["active"]
    assert act.any() and (s["sp"] >= 0).all() and (s["sp"] <= 1).all()
    assert s["sp"][act].min() == 0.0 and s["sp"][act].max() == 1.0
    assert not s["sp"][~act].any()
    # every non-degenerate chunk prunes its arg-max (1 > tau_p)
    dec = lifecycle.decide(np.zeros(N, bool), s["sp"])
    assert dec[np.argmax(np.where(act, s["L"], -np.inf))] == lifecycle.PRUNE
    # identical views: S_d == kappa of one view
    s1 = lifecycle.chunk_scores(np.tile(kappa[:1], (V, 1)), np.tile(omega[:1], (V, 1)), np.full(V, loss[0]))
    assert np.array_equal(s1["sd"], kappa[0].astype(float))
    # min-max normalisation is invariant to the log base / positive scaling of L
    Ls = np.log1p((loss[:, None] * omega).sum(0))
    assert np.allclose(s["L"], Ls)
    # sums form == per-view form
    s2 = lifecycle.chunk_scores_from_sums(kappa.sum(0), omega.sum(0), (loss[:, None] * omega).sum(0), V)
    assert np.allclose(s2["sp"], s["sp"]) and np.allclose(s2["sd"], s["sd"])


def test_degenerate_chunk_gives_zero_prune_score():
    omega = np.array([[3, 3, 0]])
    s = lifecycle.chunk_scores(np.zeros_like(omega), omega, np.array([0.2]))
    assert not s["sp"].any()


def test_decisions_invariant_to_chunk_order():
    rng = np.random.default_rng(1)
    N, C = 200, 6
    chunks = []
    for c in range(C):
        omega = rng.integers(0, 30, (4, N)) * (rng.uniform(size=(4, N)) < 0.5)
        kappa = np.minimum(omega, rng.integers(0, 30, (4, N)))
        chunks.append(lifecycle.chunk_scores(kappa, omega, rng.uniform(0.05, 0.3, 4)))
    outs = []
    for order in (range(C), reversed(range(C)), rng.permutation(C)):
        D, P = np.zeros(N, bool), np.zeros(N)
        for c in order:
            D, P = lifecycle.global_update(D, P, chunks[c]["sd"], chunks[c]["sp"])
        outs.append(lifecycle.decide(D, P))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_keep_map():
    dec = np.array([0, 2, 1, 2, 0], np.uint8)
    km, n = lifecycle.keep_map(dec)
    assert n == 3 and list(km) == [0, 1, 1, 2, 2]


def test_view_statistics_feed_the_chunk_scores():
    """End to end on the oracle: two views of a tiny scene -> S_d, S_p."""
    sc = scenes.tiny_scene(seed=3, n=30, degree=1, n_views=2)
    kap, om, loss = [], [], []
    for v in range(2):
        ov = oracle.View(sc, v, OracleConfig())
        img = ov.image()
        st = ov.stats(sc.target[v], lifecycle.TAU_ERR)
        kap.append(st["kappa"])
        om.append(st["omega"])
        loss.append(np.abs(img["color"] - sc.target[v]).mean())
    s = lifecycle.chunk_scores(np.array(kap), np.array(om), np.array(loss))
    assert np.allclose(s["sd"], (kap[0] + kap[1]) / 2)
    assert np.allclose(s["s_tilde"], loss[0] * om[0] + loss[1] * om[1])


def test_chunk_scores_hand_worked_example():
    """Two chunks of two views and five Gaussians, worked out by hand from the
    appendix's score definitions (arithmetic in the fixture's comments)."""
    ex = json.load(open(os.path.join(GOLD, "chunk_scores_worked.json")))
    D, P = np.zeros(5, bool), np.zeros(5)
    for ch in ex["chunks"]:
        s = lifecycle.chunk_scores(np.array(ch["kappa"]), np.array(ch["omega"]), np.array(ch["view_loss"]))
        assert np.array_equal(s["sd"], ch["sd"])
        assert np.allclose(s["s_tilde"], ch["s_tilde"], rtol=1e-15, atol=1e-15)
        assert np.array_equal(s["active"], np.array(ch["active"], bool))
        assert np.allclose(s["sp"], ch["sp"], rtol=1e-14, atol=1e-15)
        # the same scores from per-Gaussian sums over the views
        ss = lifecycle.chunk_scores_from_sums(np.sum(ch["kappa"], 0), np.sum(ch["omega"], 0),
                                              (np.array(ch["view_loss"])[:, None] * np.array(ch["omega"])).sum(0),
                                              len(ch["view_loss"]))
        assert np.allclose(ss["sp"], ch["sp"], rtol=1e-14, atol=1e-15) and np.array_equal(ss["sd"], ch["sd"])
        D, P = lifecycle.global_update(D, P, s["sd"], s["sp"])
    assert np.array_equal(D, np.array(ex["densify"], bool))
    assert np.allclose(P, ex["prune_score"], rtol=1e-14, atol=1e-15)
    assert np.array_equal(lifecycle.decide(D, P), ex["decision"])
