"""Pins of the Adam oracle: closed forms of its first steps and of a constant
gradient, and torch.optim.Adam (the same published update) on the CPU."""
import numpy as np
import pytest
import torch

from oracle.optim import adam_step


def test_first_step_closed_form():
    """Step 1: m_hat = g and v_hat = g^2, so theta moves by lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = adam_step(np.ones(4), np.zeros(4), np.zeros(4), g, 1, lr=0.1, eps=1e-8)
    assert np.allclose(th, 1.0 - 0.1 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_constant_gradient_closed_form():
    """A constant gradient keeps m_hat = g and v_hat = g^2 at every step (the bias corrections are exact), so
    after t steps theta has moved t lr g / (|g| + eps)."""
    g = np.array([2.0, -0.25])
    th, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, 51):
        th, m, v = adam_step(th, m, v, g, t, lr=0.01, b1=0.8, b2=0.99, eps=1e-6)
    assert np.allclose(th, -50 * 0.01 * g / (np.abs(g) + 1e-6), rtol=1e-12, atol=0)


def test_against_torch_adam():
    rng = np.random.default_rng(3)
    th0 = rng.normal(size=257)
    p = torch.nn.Parameter(torch.from_numpy(th0.copy()))
    opt = torch.optim.Adam([p], lr=0.05, betas=(0.85, 0.995), eps=1e-7)
    th, m, v = th0.copy(), np.zeros(257), np.zeros(257)
    for t in range(1, 8):
        g = rng.normal(size=257) * (1 + t)
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        th, m, v = adam_step(th, m, v, g, t, lr=0.05, b1=0.85, b2=0.995, eps=1e-7)
    assert np.allclose(p.detach().numpy(), th, rtol=1e-12, atol=1e-14)


def test_mutation_wrong_bias_correction_fails():
    """Without the second-moment bias correction the first step is lr g / (sqrt(1 - b2) |g|): far from the pin."""
    g = np.array([1.0])
    th, _, _ = adam_step(np.zeros(1), np.zeros(1), np.zeros(1), g, 1, lr=1.0)
    wrong = -1.0 * (0.1 * g) / 0.1 / (np.sqrt(0.001 * g * g) + 1e-8)
    assert not np.allclose(th, wrong)
    assert th[0] == pytest.approx(-1.0, abs=1e-7)
