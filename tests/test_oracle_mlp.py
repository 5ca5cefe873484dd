"""Pins of the network oracle (oracle/mlp.py): BF16 rounding against hand-picked
ties and torch's bfloat16, the FP64 forward against an explicit loop and
torch, the analytic gradient against central differences and torch autograd,
the class weights, and Adam against torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp


@pytest.mark.parametrize("value,bits", [
    (1.0, 0x3F80),
    (1.0 + 2.0 ** -8, 0x3F80),                 # tie between 1 and 1 + 2^-7: even mantissa wins
    (1.0 + 3 * 2.0 ** -8, 0x3F82),             # tie between 0x3F81 and 0x3F82: even wins
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 0x3F81),    # just above the tie
    (1.0 + 2.0 ** -7, 0x3F81),                 # exact
    (-2.5, 0xC020),
    (0.0, 0x0000),
    (-0.0, 0x8000),
    (3.0e38, 0x7F62),
    (1.0e-40, 0x0001),                         # FP32 subnormal, kept
])
def test_bf16_round_to_nearest_even(value, bits):
    assert int(mlp.bf16_bits(np.array([value]))[0]) == bits


def test_bf16_matches_torch_on_random_values():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e4, 2000), rng.normal(0, 1e-4, 2000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(mlp.bf16_bits(x), ref)


def _case(n=37, seed=1):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (n, 16))
    theta = mlp.init_params(seed).astype(np.float64)
    theta[1024:1088] = rng.normal(0, 0.1, 64)          # non-zero biases
    theta[5184:5248] = rng.normal(0, 0.1, 64)
    theta[5440:] = rng.normal(0, 0.1, 3)
    y = rng.integers(0, 3, n)
    return x, theta, y


def test_fp64_forward_is_the_textbook_network():
    x, theta, _ = _case(5)
    p = mlp.unpack(theta)
    out = np.zeros((5, 3))
    for n in range(5):
        h1 = [max(0.0, sum(p["W1"][o, i] * x[n, i] for i in range(16)) + p["b1"][o]) for o in range(64)]
        h2 = [max(0.0, sum(p["W2"][o, i] * h1[i] for i in range(64)) + p["b2"][o]) for o in range(64)]
        for o in range(3):
            out[n, o] = sum(p["W3"][o, i] * h2[i] for i in range(64)) + p["b3"][o]
    got = mlp.forward(x, theta, bf16_ops=False)["logits"]
    assert np.allclose(got, out, rtol=1e-12, atol=1e-12)
    t = {k: torch.from_numpy(v) for k, v in p.items()}
    ref = torch.nn.functional.linear(
        torch.relu(torch.nn.functional.linear(torch.relu(torch.nn.functional.linear(torch.from_numpy(x), t["W1"], t["b1"])),
                                              t["W2"], t["b2"])), t["W3"], t["b3"])
    assert np.allclose(got, ref.numpy(), rtol=1e-12, atol=1e-12)


def test_fp64_gradient_matches_central_differences():
    x, theta, y = _case(23, seed=2)
    cw = np.array([0.7, 1.9, 1.3])
    loss, g = mlp.loss_and_grad(x, y, cw, theta, bf16_ops=False)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(1024, 12, replace=False), 1024 + rng.choice(64, 4, replace=False),
                          1088 + rng.choice(4096, 12, replace=False), 5184 + rng.choice(64, 4, replace=False),
                          5248 + rng.choice(192, 8, replace=False), [5440, 5441, 5442]])
    for k in idx:
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mlp.loss_and_grad(x, y, cw, tp, False)[0] - mlp.loss_and_grad(x, y, cw, tm, False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * (abs(fd) + 1e-3), (k, fd, g[k])


def test_fp64_gradient_matches_torch_autograd():
    x, theta, y = _case(41, seed=4)
    cw = mlp.class_weights(y)
    loss, g = mlp.loss_and_grad(x, y, cw, theta, bf16_ops=False)
    th = torch.tensor(theta, requires_grad=True)
    p = {}
    o = 0
    for name, shape in mlp.SIZES:
        k = int(np.prod(shape))
        p[name] = th[o:o + k].reshape(shape)
        o += k
    xt = torch.from_numpy(x)
    h1 = torch.relu(xt @ p["W1"].T + p["b1"])
    h2 = torch.relu(h1 @ p["W2"].T + p["b2"])
    lg = h2 @ p["W3"].T + p["b3"]
    lt = torch.nn.functional.cross_entropy(lg, torch.from_numpy(y), weight=torch.from_numpy(cw))
    lt.backward()
    assert abs(float(lt.detach()) - loss) < 1e-12
    assert np.allclose(th.grad.numpy(), g, rtol=1e-10, atol=1e-13)


def test_bf16_mode_rounds_every_gemm_operand():
    x, theta, y = _case(19, seed=5)
    f = mlp.forward(x, theta, bf16_ops=True)
    for k in ("x", "W1", "W2", "W3", "h1", "h2"):
        assert np.array_equal(mlp.bf16(f[k]), f[k]), k
    # the rounded network differs from the exact one only by rounding-sized amounts
    g = mlp.forward(x, theta, bf16_ops=False)
    assert np.abs(f["logits"] - g["logits"]).max() < 0.05 * np.abs(g["logits"]).max()


def test_class_weights_balance_the_classes():
    y = np.array([0] * 60 + [1] * 30 + [2] * 10)
    w = mlp.class_weights(y)
    assert np.allclose(w * np.bincount(y), [100 / 3] * 3)
    assert mlp.class_weights(np.array([0, 0, 2]))[1] == 0.0


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    theta = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    tt = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([tt], lr=3e-3)
    for step in range(1, 6):
        g = rng.normal(size=50)
        theta, m, v = mlp.adam(theta, m, v, g, step, 3e-3)
        opt.zero_grad()
        tt.grad = torch.from_numpy(g)
        opt.step()
    assert np.allclose(theta, tt.detach().numpy(), rtol=1e-12, atol=1e-12)
