"""The learned prune / keep / densify head on the GPU (thin wrapper over the
C ABI): features from a chunk's statistics, BF16 MFMA forward, the weighted
cross-entropy gradient and Adam, all in libkgs kernels."""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from .rasterizer import GaussianParams, LifecycleState, Rasterizer, ViewStats

KEEP, DENSIFY, PRUNE = 0, 1, 2
N_PARAMS = L.HEAD_PARAMS
N_FEATURES = L.HEAD_FEATURES
# parameter blocks: W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [3][64], b3 [3]
BLOCKS = [("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (3, 64)), ("b3", (3,))]


def he_init(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (FP32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in BLOCKS:
        if name.startswith("W"):
            lim = math.sqrt(6.0 / shape[1])
            parts.append(rng.uniform(-lim, lim, shape).reshape(-1))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float32)


def features(R: Rasterizer, g: GaussianParams, stats: ViewStats, n_views: int,
             before: Optional[LifecycleState] = None, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """[N][16] BF16 features of every Gaussian from a chunk's statistics."""
    if out is None:
        out = torch.empty(g.n, N_FEATURES, dtype=torch.bfloat16, device=g.means.device)
    L.kgs_head_features(R.ctx, g.c(), stats.c(), n_views, before.c() if before is not None else None, out, stream)
    return out


class PruneHead:
    """FP32 master parameters with Adam moments; BF16 MFMA kernels."""

    def __init__(self, theta=None, seed: int = 0, device="cuda"):
        t = he_init(seed) if theta is None else np.asarray(theta, np.float32)
        self.theta = torch.from_numpy(t.copy()).to(device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.grad = torch.zeros_like(self.theta)
        self.loss = torch.zeros(1, device=device)
        self.step_count = 0
        self.ws_bytes = L.kgs_head_workspace_size()
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def forward(self, feats: torch.Tensor, logits=True, decision=True, stream=None):
        n = feats.shape[0]
        lg = torch.empty(n, 3, device=feats.device) if logits else None
        dec = torch.empty(n, dtype=torch.uint8, device=feats.device) if decision else None
        L.kgs_head_forward(self.theta, feats, n, lg, dec, stream)
        return lg, dec

    def loss_grad(self, feats: torch.Tensor, labels: torch.Tensor, class_w: torch.Tensor, stream=None):
        L.kgs_head_loss_grad(self.theta, feats, labels, feats.shape[0], class_w, self.workspace, self.ws_bytes,
                             self.grad, self.loss, stream)
        return self.loss, self.grad

    def adam(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        L.kgs_head_adam(self.theta, self.m, self.v, self.grad, self.step_count, lr, beta1, beta2, eps, stream)

    def train_step(self, feats, labels, class_w, lr: float, stream=None):
        self.loss_grad(feats, labels, class_w, stream)
        self.adam(lr, stream=stream)
        return self.loss
