"""FP64 reference of the learned chemical-potential network (oracle; test infrastructure only).

The network is not in the paper: it maps Chebyshev trace moments to the
scaled chemical potential so that the trace-based mu search can start from
a close guess.  Its architecture is a design choice ("parity unpinned" as a
choice); its arithmetic is pinned by central finite differences (backward)
and by a two-step hand-checked case (forward and Adam).

Layout of the flat parameter vector (float32 on the device, float64 here):
    W1 (H1 x IN, row-major), b1 (H1), W2 (H2 x H1), b2 (H2), w3 (H2), b3 (1)
with IN = 64, H1 = H2 = 256: 82,689 parameters.
    y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3,  loss = mean_b (y_b - t_b)^2.
Features (64): tau_1..tau_62 divided by n, N_e / n, log(beta') / 4.
"""
from __future__ import annotations

import numpy as np

IN, H1, H2 = 64, 256, 256
N_PARAMS = H1 * IN + H1 + H2 * H1 + H2 + H2 + 1


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0

    def take(n, shape):
        nonlocal o
        v = w[o:o + n].reshape(shape)
        o += n
        return v

    W1 = take(H1 * IN, (H1, IN))
    b1 = take(H1, (H1,))
    W2 = take(H2 * H1, (H2, H1))
    b2 = take(H2, (H2,))
    w3 = take(H2, (H2,))
    b3 = take(1, (1,))
    return W1, b1, W2, b2, w3, b3


def init_params(seed: int = 0):
    """He-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (H1, IN)) * np.sqrt(6.0 / IN)
    W2 = rng.uniform(-1, 1, (H2, H1)) * np.sqrt(6.0 / H1)
    w3 = rng.uniform(-1, 1, H2) * np.sqrt(6.0 / H2) * 0.1
    return np.concatenate([W1.ravel(), np.zeros(H1), W2.ravel(), np.zeros(H2), w3, np.zeros(1)])


def features(tau, n, n_elec, beta_s):
    """64 inputs: tau_1..tau_62 / n, N_e / n, log(beta') / 4 (rows = problems)."""
    tau = np.atleast_2d(np.asarray(tau, dtype=np.float64))
    n = np.asarray(n, dtype=np.float64).reshape(-1, 1)
    out = np.empty((tau.shape[0], IN))
    out[:, :62] = tau[:, 1:63] / n
    out[:, 62] = np.asarray(n_elec, dtype=np.float64) / n[:, 0]
    out[:, 63] = np.log(np.asarray(beta_s, dtype=np.float64)) / 4.0
    return out


def forward(w, X):
    W1, b1, W2, b2, w3, b3 = unpack(w)
    Z1 = X @ W1.T + b1
    A1 = np.maximum(Z1, 0.0)
    Z2 = A1 @ W2.T + b2
    A2 = np.maximum(Z2, 0.0)
    y = A2 @ w3 + b3[0]
    return y, (X, Z1, A1, Z2, A2)


def loss(w, X, t):
    y, _ = forward(w, X)
    return float(np.mean((y - t) ** 2))


def backward(w, X, t):
    """Loss and its gradient (flat, same layout as w) by the chain rule."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    y, (X, Z1, A1, Z2, A2) = forward(w, X)
    B = X.shape[0]
    dy = 2.0 * (y - t) / B
    g_w3 = A2.T @ dy
    g_b3 = np.array([dy.sum()])
    dZ2 = np.outer(dy, w3) * (Z2 > 0)
    g_W2 = dZ2.T @ A1
    g_b2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * (Z1 > 0)
    g_W1 = dZ1.T @ X
    g_b1 = dZ1.sum(axis=0)
    g = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, g_b3])
    return float(np.mean((y - t) ** 2)), g


def adam_step(w, g, m, v, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1); returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v
