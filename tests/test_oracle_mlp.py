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


def test_adam_first_step_is_bias_corrected():
    """At t = 1 the bias-corrected moments are m^ = g and v^ = g^2 exactly, so
    every coordinate moves by lr * g / (|g| + eps): almost exactly lr against
    the sign of its gradient, whatever the gradient's size.  Without the bias
    correction the step would be lr * (1 - b1) / sqrt(1 - b2) ~ 3.16 lr."""
    lr = 0.1
    theta0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(theta0, g, np.zeros(4), np.zeros(4), 1, lr=lr)
    step = theta0 - th
    np.testing.assert_allclose(step[:3], lr * np.sign(g[:3]), rtol=1e-5)
    assert step[3] == 0.0
    # the raw moments are the first exponential-average terms
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_second_step_after_a_sign_flip():
    """Gradient +1 at t = 1 and -1 at t = 2.  Worked by hand with b1 = 0.9,
    b2 = 0.999: m2 = b1 (1-b1) - (1-b1) = -(1-b1)^2 = -0.01 and the correction
    1 - b1^2 = 0.19 give m^ = -1/19; v2 = b2 (1-b2) + (1-b2) = 1 - b2^2, so
    v^ = 1.  The second step therefore raises theta by lr/19 / (1 + eps).
    Swapping b1 and b2 would give m^ = -(1-b2)^2/(1-b2^2), about -5e-4."""
    lr = 0.05
    th, m, v = mlp.adam_step(np.array([0.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr=lr)
    np.testing.assert_allclose(th, [-lr], rtol=1e-7)
    th2, m2, v2 = mlp.adam_step(th, np.array([-1.0]), m, v, 2, lr=lr)
    np.testing.assert_allclose(m2, [-0.01], rtol=1e-12)
    np.testing.assert_allclose(v2, [1 - 0.999 ** 2], rtol=1e-12)
    np.testing.assert_allclose(th2 - th, [lr / 19 / (1 + 1e-8)], rtol=1e-12)


def test_adam_constant_gradient_gives_constant_steps():
    """With a constant gradient the bias-corrected averages equal g and g^2 at
    every step, so each step is the same lr * g / (|g| + eps)."""
    lr = 0.01
    g = np.array([3.0, -0.25])
    th = np.zeros(2)
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 30):
        nth, m, v = mlp.adam_step(th, g, m, v, t, lr=lr)
        np.testing.assert_allclose(th - nth, lr * g / (np.abs(g) + 1e-8), rtol=1e-9)
        th = nth
