"""Pins of the FP64 reference of the learned PP switch (CPU only)."""

import numpy as np

from oracle import mlp


def _data(B=37, D=9, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, D))
    y = (rng.random(B) < 0.4).astype(float)
    return X, y


def test_gradient_matches_central_differences():
    D, H = 9, 7
    X, y = _data(D=D)
    theta = mlp.init_params(D, H, 1) + 0.05 * np.random.default_rng(2).standard_normal(mlp.n_params(D, H))
    g = mlp.grad(theta, X, y, D, H)
    h = 1e-6
    num = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        num[i] = (mlp.loss(theta + e, X, y, D, H) - mlp.loss(theta - e, X, y, D, H)) / (2 * h)
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-9)


def test_forward_matches_per_sample_loop():
    D, H = 5, 4
    X, _ = _data(B=6, D=D)
    theta = mlp.init_params(D, H, 4)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(theta, D, H)
    p, _ = mlp.forward(theta, X, D, H)
    for b in range(X.shape[0]):
        h1 = [np.tanh(sum(X[b, d] * W1[d, j] for d in range(D)) + b1[j]) for j in range(H)]
        h2 = [np.tanh(sum(h1[i] * W2[i, j] for i in range(H)) + b2[j]) for j in range(H)]
        z = sum(h2[j] * w3[j] for j in range(H)) + b3
        assert abs(p[b] - 1.0 / (1.0 + np.exp(-z))) < 1e-14


def test_first_adam_step_moves_every_coordinate_by_lr():
    # with m0 = v0 = 0 and t = 1 the bias-corrected step is lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(th[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert th[3] == 0.0


def test_training_fits_a_separable_rule():
    D, H = 3, 8
    rng = np.random.default_rng(0)
    X = rng.standard_normal((200, D))
    y = (X[:, 0] - 0.5 * X[:, 1] > 0).astype(float)
    theta = mlp.init_params(D, H, 5)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, y, D, H)
    for t in range(1, 401):
        theta, m, v = mlp.adam_step(theta, mlp.grad(theta, X, y, D, H), m, v, t, lr=0.02)
    assert mlp.loss(theta, X, y, D, H) < 0.2 * l0
    p, _ = mlp.forward(theta, X, D, H)
    assert np.mean((p > 0.5) == (y > 0.5)) > 0.95
