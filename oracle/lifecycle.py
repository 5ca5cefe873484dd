"""Chunk scores, global aggregation rules and the densify / prune decision in
NumPy FP64.  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the appendix section "Details for Lifecycle-Managed Gaussian Mapping"
(densification score, pruning score) and the global rules of Sec. 3.3
("Global Densification Rules", "Global Pruning Rules"); thresholds from the
hyper-parameter table: tau_err = 0.1, tau_d = 5, tau_p = 0.99, C = 100.

Readings where the paper is silent:
  * |V_c| is the number of views passed for the chunk.
  * The active set A_c is every Gaussian with a non-empty footprint in some
    view of the chunk; inactive Gaussians get S_p = 0.
  * When max L == min L over A_c the normalisation is undefined; S_p = 0.
  * A Gaussian both marked for densification and over the prune threshold is
    pruned.
  * Both threshold tests are strict (">"), as written.
"""
from __future__ import annotations

import numpy as np

KEEP, DENSIFY, PRUNE = 0, 1, 2
TAU_ERR, TAU_D, TAU_P = 0.1, 5.0, 0.99


def chunk_scores(kappa: np.ndarray, omega: np.ndarray, view_loss: np.ndarray) -> dict:
    """kappa, omega: [V][N] per-view high-error counts and footprint sizes;
    view_loss: [V] photometric loss of each view.

    S_d^(i,c) = (1/|V_c|) sum_v kappa_v(i)                (densification score)
    gamma_v(i) = L_photo^(v) |Omega_v(i)|;  S~ = sum_v gamma_v(i)
    L = log(1 + S~);  S_p = (L - min_A L) / (max_A L - min_A L)  (pruning score)
    """
    kappa = np.asarray(kappa, np.float64)
    omega = np.asarray(omega, np.float64)
    loss = np.asarray(view_loss, np.float64)
    V = kappa.shape[0]
    sd = kappa.sum(axis=0) / V
    s_tilde = (loss[:, None] * omega).sum(axis=0)
    L = np.log1p(s_tilde)
    active = omega.sum(axis=0) > 0
    sp = np.zeros_like(L)
    if active.any():
        lo, hi = L[active].min(), L[active].max()
        if hi > lo:
            sp[active] = (L[active] - lo) / (hi - lo)
    return dict(sd=sd, s_tilde=s_tilde, L=L, active=active, sp=sp,
                lmin=L[active].min() if active.any() else 0.0,
                lmax=L[active].max() if active.any() else 0.0)


def chunk_scores_from_sums(kappa_sum, omega_sum, gamma_sum, n_views: int) -> dict:
    """Same scores from per-Gaussian sums over the chunk's views."""
    sd = np.asarray(kappa_sum, np.float64) / n_views
    L = np.log1p(np.asarray(gamma_sum, np.float64))
    active = np.asarray(omega_sum) > 0
    sp = np.zeros_like(L)
    if active.any():
        lo, hi = L[active].min(), L[active].max()
        if hi > lo:
            sp[active] = (L[active] - lo) / (hi - lo)
    return dict(sd=sd, L=L, active=active, sp=sp)


def global_update(D: np.ndarray, P: np.ndarray, sd: np.ndarray, sp: np.ndarray, tau_d: float = TAU_D):
    """S_d(i) = OR_c [S_d^(i,c) > tau_d];  S_p(i) = max_c S_p^(i,c)."""
    return np.logical_or(D, sd > tau_d), np.maximum(P, sp)


def decide(D: np.ndarray, P: np.ndarray, tau_p: float = TAU_P) -> np.ndarray:
    """PRUNE if S_p(i) > tau_p, else DENSIFY if S_d(i), else KEEP."""
    out = np.full(D.shape, KEEP, np.uint8)
    out[np.asarray(D, bool)] = DENSIFY
    out[np.asarray(P) > tau_p] = PRUNE
    return out


def keep_map(decision: np.ndarray):
    """Exclusive prefix count of the Gaussians that survive (not pruned)."""
    keep = (decision != PRUNE).astype(np.int64)
    return np.concatenate([[0], np.cumsum(keep)[:-1]]).astype(np.uint32), int(keep.sum())
