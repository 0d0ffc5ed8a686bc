"""Pins for the oracle's MLP: finite differences, a hand-checked tiny case, Adam's first step."""
import numpy as np

from oracle import mlp


def test_param_count():
    assert mlp.N_PARAMS == 82689


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    w = mlp.init_params(1)
    w[mlp.H1 * mlp.IN: mlp.H1 * mlp.IN + mlp.H1] = rng.normal(0, 0.1, mlp.H1)   # non-zero biases
    X = rng.normal(0, 1, (5, mlp.IN))
    t = rng.normal(0, 0.1, 5)
    L, g = mlp.backward(w, X, t)
    assert abs(L - mlp.loss(w, X, t)) < 1e-15
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 40, replace=False), [mlp.N_PARAMS - 1]])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss(wp, X, t) - mlp.loss(wm, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_forward_by_hand():
    # one active unit per layer: y = w3[0] * relu(W2[0,0] * relu(W1[0] . x + b1[0]) + b2[0]) + b3
    w = np.zeros(mlp.N_PARAMS)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(w)   # views into w
    W1[0, 0], W1[0, 1], b1[0] = 2.0, -1.0, 0.5
    W2[0, 0], b2[0] = 3.0, -1.0
    w3[0], b3[0] = 0.25, 0.125
    x = np.zeros((2, mlp.IN))
    x[0, 0], x[0, 1] = 1.0, 1.0      # z1 = 1.5, z2 = 3.5, y = 0.875 + 0.125
    x[1, 0] = -1.0                   # z1 = -1.5 -> 0, z2 = -1 -> 0, y = 0.125
    y, _ = mlp.forward(w, x)
    np.testing.assert_allclose(y, [1.0, 0.125], rtol=0, atol=1e-15)


def test_adam_first_step_is_sign_times_lr():
    g = np.array([0.3, -2.0, 0.0, 1e-3])
    w, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-300)
    np.testing.assert_allclose(w[[0, 1, 3]], [-0.01, 0.01, -0.01], rtol=1e-12)


def test_features_layout():
    tau = np.arange(70, dtype=float)[None, :]
    f = mlp.features(tau, [10.0], [4.0], [np.e ** 8])
    np.testing.assert_allclose(f[0, :62], np.arange(1, 63) / 10.0)
    assert f[0, 62] == 0.4 and abs(f[0, 63] - 2.0) < 1e-15
