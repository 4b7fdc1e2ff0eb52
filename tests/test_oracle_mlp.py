"""Pins of the FP64 MLP reference: gradients against central finite differences,
Adam's first step against its closed form, and a hand-built network whose output
is known exactly."""
import numpy as np

from oracle import mlp

F, H = 6, 8


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = rng.normal(scale=0.5, size=mlp.n_params(F, H))
    X = rng.normal(size=(7, F))
    t = rng.normal(size=7)
    L, g = mlp.grad(theta, X, t, F, H)
    assert abs(L - mlp.loss(theta, X, t, F, H)) < 1e-14
    h = 1e-6
    for k in rng.choice(theta.size, 60, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mlp.loss(tp, X, t, F, H) - mlp.loss(tm, X, t, F, H)) / (2 * h)
        assert abs(g[k] - fd) < 1e-7 * max(1.0, abs(fd)), k


def test_adam_first_step_closed_form():
    # After one step from m = v = 0: mhat = g, vhat = g^2, so the update is lr * g / (|g| + eps).
    rng = np.random.default_rng(1)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    assert np.allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_hand_built_network():
    # W1 copies x into the first F hidden units, other layers pass them through,
    # W4 sums them: y = sum(relu(x)) + b4.
    W1 = np.zeros((F, H)); W1[np.arange(F), np.arange(F)] = 1
    I = np.eye(H)
    W4 = np.ones((H, 1))
    theta = mlp.pack([W1, np.zeros(H), I, np.zeros(H), I, np.zeros(H), W4, [0.25]])
    X = np.array([[1, -2, 3, -4, 5, -6], [0.5, 0.5, -1, 0, 0, 2]], float)
    y, _ = mlp.forward(theta, X, F, H)
    assert np.allclose(y, [9.25, 3.25])


def test_training_decreases_loss():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(256, F))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2
    theta = rng.normal(scale=0.3, size=mlp.n_params(F, H))
    m = np.zeros_like(theta); v = np.zeros_like(theta)
    L0 = mlp.loss(theta, X, t, F, H)
    for step in range(1, 301):
        _, g = mlp.grad(theta, X, t, F, H)
        theta, m, v = mlp.adam_step(theta, g, m, v, step, lr=0.01)
    assert mlp.loss(theta, X, t, F, H) < 0.2 * L0
