"""Anchor decoding (Scaffold-GS style) with the level-of-detail opacity mask,
in NumPy FP64 with the GPU's BF16 rounding points made explicit.  TEST
INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the appendix sections "Voxelized Representation and MLP Decoding":

    (c_k, alpha_k, q_k, ds_k, dO_k) = MLP(f_i, d_hat_iv, d_iv),  k = 1..K
    x_k = p_i + (O_k + dO_k) * l_i,    s_k = l_i * ds_k

with d_iv = ||p_i - c_v|| and d_hat_iv = (p_i - c_v) / d_iv for the camera
centre c_v, and "Level-of-Detail (LoD) Mask Computation": alpha~ = alpha M_l(d),
M_l = 1 on [D_min^l, D_max^l) and 0 elsewhere.

Readings where the paper is silent:
  * One MLP: 36 inputs (f in R^32, d_hat, d) -> 32 ReLU units -> 14 K outputs;
    child k takes outputs 14k .. 14k + 13 as (alpha, c (3), q (4), ds (3), dO (3)).
    alpha = tanh, c = sigmoid, ds = sigmoid, q and dO as they come (q is
    normalised by the projection).  The local scale is stored as log l.
  * Bands as in the initialisation: D_max^l = 100 eps_l for eps = (0.1, 0.25,
    1, 5, 25), D_min^l = D_max^(l-1) (0 for the finest), the last unbounded.
  * The decoded Gaussian enters the rasterizer with SH degree 0 (its colour is
    already view dependent): coefficient (c - 0.5) / Y_00; opacity logit
    ln(alpha~ / (1 - alpha~)), and a child with alpha~ <= 0 gets the logit -100
    (fully transparent, culled).  Inside the band alpha~ = tanh(y), and the
    logit is formed from y as ln((e^{2y} - 1) / 2), the same number without the
    cancellation of 1 - tanh y near 1 (see tanh_logit).
  * Child k of anchor a is Gaussian a K + k.
  * The network runs on the matrix cores with BF16 operands: the 36 inputs, both
    weight matrices and the 32 hidden activations are rounded to BF16 (nearest,
    ties to even); sums and biases are exact here (FP64).
"""
from __future__ import annotations

import math

import numpy as np

from .mlp import bf16

IN, HID, OUTC = 36, 32, 14
EPS = (0.1, 0.25, 1.0, 5.0, 25.0)
DMAX = tuple(100.0 * e for e in EPS[:-1]) + (math.inf,)
Y00 = 0.28209479177387814
N_PARAMS = lambda K: HID * IN + HID + OUTC * K * HID + OUTC * K


def unpack(theta, K):
    """theta = W1 [32][36], b1 [32], W2 [14K][32], b2 [14K] (row-major, concatenated)."""
    t = np.asarray(theta, np.float64)
    o = 0
    W1 = t[o:o + HID * IN].reshape(HID, IN); o += HID * IN
    b1 = t[o:o + HID]; o += HID
    W2 = t[o:o + OUTC * K * HID].reshape(OUTC * K, HID); o += OUTC * K * HID
    b2 = t[o:o + OUTC * K]
    return W1, b1, W2, b2


def tanh_logit(y):
    """ln(a / (1 - a)) for a = tanh(y), y > 0.  Since 1 - tanh y = 2 / (e^{2y} + 1), the ratio is
    (e^{2y} - 1) / 2 exactly; this form keeps its precision where tanh y rounds to 1."""
    y = np.maximum(np.asarray(y, np.float64), 1e-300)
    with np.errstate(over="ignore", divide="ignore"):
        return np.where(y < 0.5, np.log(0.5 * np.expm1(2.0 * y)), 2.0 * y - math.log(2.0) + np.log1p(-np.exp(-2.0 * y)))


def lod_mask(distance, level):
    """1 where the camera distance lies in its level's band, else 0."""
    level = np.asarray(level, np.int64)
    hi = np.array(DMAX)[level]
    lo = np.where(level > 0, np.array((0.0,) + DMAX[:-1])[level], 0.0)
    return ((distance >= lo) & (distance < hi)).astype(np.float64)


def decode(anchors: dict, theta, K: int, centre) -> dict:
    """anchors: p [3][A], f [A][32], log_l [3][A], O [K][3][A], level [A] (any float
    type; taken in FP64).  Returns the decoded Gaussians of one view (means
    [3][AK], log_scales [3][AK], quats [4][AK], logits [AK], sh [1][3][AK]), the raw
    network outputs, alpha~ and, per anchor, how close its hidden activations and
    inputs came to a BF16 rounding boundary (relative), for comparisons with an
    FP32 accumulation."""
    p = np.asarray(anchors["p"], np.float64)
    f = np.asarray(anchors["f"], np.float64)
    log_l = np.asarray(anchors["log_l"], np.float64)
    O = np.asarray(anchors["O"], np.float64)
    level = np.asarray(anchors["level"], np.int64)
    A = p.shape[1]
    c = np.asarray(centre, np.float64).reshape(3, 1)
    dv = p - c
    d = np.sqrt((dv * dv).sum(0))
    dhat = dv / d
    x = np.concatenate([f, dhat.T, d[:, None]], axis=1)          # [A][36]
    W1, b1, W2, b2 = unpack(theta, K)
    z1 = bf16(x) @ bf16(W1).T + b1                                # [A][32]
    h = np.maximum(z1, 0.0)
    y = bf16(h) @ bf16(W2).T + b2                                 # [A][14K]
    # sums of the magnitudes of what each accumulation adds (bounds another arithmetic's rounding)
    z1_abs = np.abs(bf16(x)) @ np.abs(bf16(W1)).T + np.abs(b1)
    y_abs = np.abs(bf16(h)) @ np.abs(bf16(W2)).T + np.abs(b2)
    yk = y.reshape(A, K, OUTC)
    alpha = np.tanh(yk[..., 0])
    col = 1.0 / (1.0 + np.exp(-yk[..., 1:4]))
    q = yk[..., 4:8]
    ds = 1.0 / (1.0 + np.exp(-yk[..., 8:11]))
    dO = yk[..., 11:14]
    l = np.exp(log_l).T                                           # [A][3]
    Ok = np.transpose(O, (2, 0, 1))                               # [A][K][3]
    xk = p.T[:, None, :] + (Ok + dO) * l[:, None, :]
    log_s = log_l.T[:, None, :] + np.log(ds)
    at = alpha * lod_mask(d, level)[:, None]
    logit = np.where(at > 0, tanh_logit(yk[..., 0]), -100.0)
    n = A * K
    out = dict(means=xk.reshape(n, 3).T.copy(), log_scales=log_s.reshape(n, 3).T.copy(),
               quats=q.reshape(n, 4).T.copy(), logits=logit.reshape(n), sh=((col.reshape(n, 3).T - 0.5) / Y00)[None],
               raw=y, alpha_masked=at, distance=d, z1=z1, z1_abs=z1_abs, y_abs=y_abs)
    # BF16 rounding margins: distance of each rounded value from a rounding boundary, relative
    out["margin_hidden"] = _bf16_margin(h).min(axis=1)
    out["margin_input"] = _bf16_margin(x).min(axis=1)
    return out


def _bf16_margin(v):
    """Relative distance of each value from the nearest BF16 rounding boundary (inf for 0)."""
    v = np.abs(np.asarray(v, np.float64))
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.floor(np.log2(np.where(v > 0, v, 1.0)))
        ulp = np.exp2(e - 7)                                      # BF16 keeps 8 significant bits
        r = v / ulp - np.floor(v / ulp)
        m = np.abs(r - 0.5) * ulp / np.where(v > 0, v, 1.0)
    return np.where(v > 0, m, np.inf)
