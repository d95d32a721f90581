"""Pins for the fp64 MLP reference: central finite differences, torch autograd
(an independent implementation), and a hand-computed tiny case."""
import numpy as np
import torch

from oracle import mlp


def test_param_count():
    assert mlp.N_PARAMS == 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5313


def test_gradient_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init(1) + rng.normal(0, 0.05, mlp.N_PARAMS)
    x = rng.normal(size=(12, 16))
    t = rng.normal(size=12)
    loss, g = mlp.loss_and_grad(theta, x, t)
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(theta + e, x, t)[0] - mlp.loss_and_grad(theta - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_gradient_vs_torch_autograd():
    rng = np.random.default_rng(1)
    theta = mlp.init(2)
    x = rng.normal(size=(33, 16))
    t = rng.normal(size=33)
    loss, g = mlp.loss_and_grad(theta, x, t)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    o = 0
    parts = {}
    for name, shape in mlp.SIZES:
        n = int(np.prod(shape))
        parts[name] = th[o:o + n].reshape(shape)
        o += n
    X = torch.tensor(x)
    a1 = torch.relu(X @ parts["W1"].T + parts["b1"])
    a2 = torch.relu(a1 @ parts["W2"].T + parts["b2"])
    y = (a2 @ parts["W3"].T + parts["b3"])[:, 0]
    L = ((y - torch.tensor(t)) ** 2).mean()
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    np.testing.assert_allclose(th.grad.numpy(), g, rtol=1e-10, atol=1e-12)


def test_hand_computed_forward():
    # W1 routes x[0] to hidden unit 0 and -x[0] to unit 1; W2 sums them; W3 = 2; b3 = 0.5
    p = {n: np.zeros(s) for n, s in mlp.SIZES}
    p["W1"][0, 0] = 1.0
    p["W1"][1, 0] = -1.0
    p["W2"][0, 0] = 1.0
    p["W2"][0, 1] = 1.0
    p["W3"][0, 0] = 2.0
    p["b3"][0] = 0.5
    theta = mlp.pack(p)
    x = np.zeros((3, 16))
    x[:, 0] = [3.0, -2.0, 0.0]
    y, _ = mlp.forward(theta, x)
    # relu(x)+relu(-x) = |x|; y = 2|x| + 0.5
    np.testing.assert_allclose(y, [6.5, 4.5, 0.5])


def test_adam_decreases_loss():
    rng = np.random.default_rng(2)
    theta = mlp.init(3)
    x = rng.normal(size=(64, 16))
    t = np.abs(x[:, 0]) - x[:, 1]
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss_and_grad(theta, x, t)[0]
    for k in range(1, 201):
        _, g = mlp.loss_and_grad(theta, x, t)
        theta, m, v = mlp.adam_step(theta, g, m, v, k, lr=3e-3)
    assert mlp.loss_and_grad(theta, x, t)[0] < 0.1 * l0
