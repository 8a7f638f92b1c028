"""FP64 reference of the learned PP switch: a perceptron D -> H -> H -> 1 with
tanh hidden units and a sigmoid output, trained on binary cross-entropy with
Adam (Kingma & Ba, "Adam: A Method for Stochastic Optimization", Alg. 1).
Not part of the paper: the paper decides with the hand threshold of Alg. 2;
this network replaces that threshold.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Parameter vector layout (shared with the GPU kernels' documentation, not
code): W1 (D x H, row-major, input index slowest), b1 (H), W2 (H x H), b2 (H),
w3 (H), b3 (1).

Pins: gradients against central finite differences; the forward pass against
a per-sample loop; the Adam step against its closed form after one step
(|delta| = lr for every coordinate with a nonzero gradient).
"""

import numpy as np


def n_params(D, H):
    return D * H + H + H * H + H + H + 1


def unpack(theta, D, H):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + D * H].reshape(D, H); o += D * H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def forward(theta, X, D, H):
    """Probabilities p (B,) and the hidden activations."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, D, H)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    z = h2 @ w3 + b3
    p = 1.0 / (1.0 + np.exp(-z))
    return p, (h1, h2, z)


def loss(theta, X, y, D, H):
    """Mean binary cross-entropy, written with log-sigmoid for stability."""
    _, (_, _, z) = forward(theta, X, D, H)
    y = np.asarray(y, dtype=np.float64)
    # -[y log s(z) + (1-y) log(1-s(z))] = softplus(z) - y z
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def grad(theta, X, y, D, H):
    """Gradient of the mean BCE with respect to theta (backpropagation)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, D, H)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    B = X.shape[0]
    p, (h1, h2, z) = forward(theta, X, D, H)
    dz = (p - y) / B                       # d loss / d z
    g_w3 = h2.T @ dz
    g_b3 = dz.sum()
    dh2 = np.outer(dz, w3) * (1.0 - h2 * h2)
    g_W2 = h1.T @ dh2
    g_b2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (1.0 - h1 * h1)
    g_W1 = X.T @ dh1
    g_b1 = dh1.sum(axis=0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])


def adam_step(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(D, H, seed):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    def glorot(a, b):
        lim = np.sqrt(6.0 / (a + b))
        return rng.uniform(-lim, lim, size=(a, b))
    return np.concatenate([glorot(D, H).ravel(), np.zeros(H), glorot(H, H).ravel(), np.zeros(H),
                           glorot(H, 1).ravel(), [0.0]])
