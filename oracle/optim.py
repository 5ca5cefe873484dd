"""Adam, written out from its published definition (Kingma and Ba, 2015), in
NumPy FP64.  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The sliding-window optimisation (Sec. 3.2) updates the map by gradient steps
and names no optimiser; Adam with bias correction is the reading.  Per
parameter, for step t = 1, 2, ...:
    m_t = b1 m_{t-1} + (1 - b1) g_t
    v_t = b2 v_{t-1} + (1 - b2) g_t^2
    theta_t = theta_{t-1} - lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps)
"""
from __future__ import annotations

import numpy as np


def adam_step(theta, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One step; returns new (theta, m, v) in FP64 (inputs are not modified)."""
    g = np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return np.asarray(theta, np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
