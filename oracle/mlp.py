"""The prune / keep / densify network in NumPy FP64, with the BF16 roundings of
the GPU path made explicit.  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The learned part replaces the plain multi-view criterion of Sec. 3.3 / App. D
with a small classifier over per-Gaussian statistics; the criterion's decision
(KEEP 0, DENSIFY 1, PRUNE 2) is its training label and the reference for its
agreement.  The paper does not state the network, its activation or its loss.
Readings:
  * MLP 16 -> 64 -> 64 -> 3, ReLU after the two hidden layers, logits out;
  * loss: class-weighted softmax cross-entropy, averaged with the weights
    (sum_n w_{y_n} CE_n / sum_n w_{y_n});
  * precision: every GEMM operand is rounded to BF16 (round to nearest even,
    from the FP32 value the GPU holds), products are exact and accumulate in a
    wider type; biases and the loss stay FP32 / FP64.  With bf16=False the same
    functions run in plain FP64 (used for the finite-difference pin).

Parameter vector (FP32, 5443 entries, this order): W1 [64][16], b1 [64],
W2 [64][64], b2 [64], W3 [3][64], b3 [3].
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 16, 64, 3
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_OUT, N_H)),
         ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], np.float64).reshape(shape)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in SIZES])


def bf16_bits(x) -> np.ndarray:
    """BF16 bit patterns of x: first to FP32 (nearest even), then the upper 16
    bits with round to nearest, ties to even (finite inputs)."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return ((u >> 16) & 0xFFFF).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16(x) -> np.ndarray:
    """Round to BF16 and return the value in FP64."""
    return from_bf16_bits(bf16_bits(x))


def _r(x, on):
    return bf16(x) if on else np.asarray(x, np.float64)


def forward(x: np.ndarray, theta: np.ndarray, bf16_ops: bool = True) -> dict:
    """x: [N][16] features.  Returns logits [N][3] and the intermediates."""
    p = unpack(theta)
    xb = _r(x, bf16_ops)
    W1, W2, W3 = _r(p["W1"], bf16_ops), _r(p["W2"], bf16_ops), _r(p["W3"], bf16_ops)
    z1 = xb @ W1.T + p["b1"]
    a1 = np.maximum(z1, 0.0)
    h1 = _r(a1, bf16_ops)
    z2 = h1 @ W2.T + p["b2"]
    a2 = np.maximum(z2, 0.0)
    h2 = _r(a2, bf16_ops)
    logits = h2 @ W3.T + p["b3"]
    return dict(x=xb, W1=W1, W2=W2, W3=W3, z1=z1, h1=h1, z2=z2, h2=h2, logits=logits)


def class_weights(labels: np.ndarray) -> np.ndarray:
    """Balanced weights N / (3 count_c) (0 for an absent class)."""
    cnt = np.bincount(np.asarray(labels, np.int64), minlength=N_OUT).astype(np.float64)
    w = np.zeros(N_OUT)
    nz = cnt > 0
    w[nz] = cnt.sum() / (N_OUT * cnt[nz])
    return w


def loss_and_grad(x: np.ndarray, labels: np.ndarray, cw: np.ndarray, theta: np.ndarray, bf16_ops: bool = True):
    """Weighted mean cross-entropy and its gradient in the parameter order.
    The backward rounds, like the GPU, the operands of its GEMMs: dlogits,
    the masked dh2 and dh1 (and uses the rounded forward activations)."""
    f = forward(x, theta, bf16_ops)
    y = np.asarray(labels, np.int64)
    n = len(y)
    lg = f["logits"]
    m = lg.max(axis=1, keepdims=True)
    e = np.exp(lg - m)
    s = e.sum(axis=1, keepdims=True)
    logp = lg - m - np.log(s)
    wy = np.asarray(cw, np.float64)[y]
    wsum = wy.sum()
    loss = float(-(wy * logp[np.arange(n), y]).sum() / wsum)
    prob = e / s
    onehot = np.zeros_like(prob)
    onehot[np.arange(n), y] = 1.0
    dlog = (prob - onehot) * (wy / wsum)[:, None]
    dl = _r(dlog, bf16_ops)
    dh2 = dl @ f["W3"]
    dz2 = _r(dh2 * (f["z2"] > 0), bf16_ops)
    dh1 = dz2 @ f["W2"]
    dz1 = _r(dh1 * (f["z1"] > 0), bf16_ops)
    g = dict(W3=dl.T @ f["h2"], b3=dl.sum(axis=0), W2=dz2.T @ f["h1"], b2=dz2.sum(axis=0),
             W1=dz1.T @ f["x"], b1=dz1.sum(axis=0))
    return loss, pack(g)


def predict(x: np.ndarray, theta: np.ndarray, bf16_ops: bool = True) -> np.ndarray:
    return np.argmax(forward(x, theta, bf16_ops)["logits"], axis=1).astype(np.uint8)


def adam(theta, m, v, grad, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma & Ba) with bias correction; returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (FP32 values)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shape[1])
            p[name] = rng.uniform(-lim, lim, shape)
        else:
            p[name] = np.zeros(shape)
    return pack(p).astype(np.float32)
