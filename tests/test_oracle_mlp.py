"""Pins for the oracle's rank-predictor MLP (forward, pinball-loss backward,
Adam) and block features.  CPU only."""
import numpy as np

import synth


def _init(orc, seed=0):
    rng = np.random.default_rng(seed)
    P = orc.mlp_nparams()
    w = np.empty(P)
    sizes = [(64, 8), (64,), (64, 64), (64,), (64, 64), (64,), (1, 64), (1,)]
    o = 0
    for s in sizes:
        k = int(np.prod(s))
        fan_in = s[1] if len(s) == 2 else 64
        w[o:o + k] = rng.standard_normal(k) * np.sqrt(2.0 / fan_in) if len(s) == 2 else 0.1 * rng.standard_normal(k)
        o += k
    assert o == P == 8961
    return w


def _numpy_forward(w, X):
    W1, b1 = w[:512].reshape(64, 8), w[512:576]
    W2, b2 = w[576:4672].reshape(64, 64), w[4672:4736]
    W3, b3 = w[4736:8832].reshape(64, 64), w[8832:8896]
    W4, b4 = w[8896:8960], w[8960]
    a = np.maximum(X @ W1.T + b1, 0)
    a = np.maximum(a @ W2.T + b2, 0)
    a = np.maximum(a @ W3.T + b3, 0)
    return a @ W4 + b4


def test_forward_matches_matrix_form(orc):
    w = _init(orc)
    X = np.random.default_rng(1).standard_normal((50, 8))
    assert np.allclose(orc.mlp_forward(w, X), _numpy_forward(w, X), rtol=1e-12, atol=1e-12)


def test_gradient_central_differences(orc):
    w = _init(orc, 2)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 8))
    y = rng.standard_normal(40) * 3
    loss, g = orc.mlp_loss_grad(w, X, y, 0.9)
    # the pinball loss as a function of the predictions (numpy)
    u = y - _numpy_forward(w, X)
    assert abs(loss - np.mean(u * (0.9 - (u < 0)))) < 1e-12
    h = 1e-6
    idx = rng.choice(w.shape[0], 60, replace=False)
    idx = np.concatenate([idx, [0, 511, 512, 4735, 8895, 8960]])
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (orc.mlp_loss_grad(wp, X, y, 0.9)[0] - orc.mlp_loss_grad(wm, X, y, 0.9)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_gradient_closed_form_bias_only(orc):
    """Zero weights: the prediction is b4 and dL/db4 = -mean(q - [y < b4])."""
    w = np.zeros(orc.mlp_nparams())
    w[-1] = 0.5
    y = np.array([0.0, 1.0, 2.0, 0.2, 0.7])
    loss, g = orc.mlp_loss_grad(w, np.ones((5, 8)), y, 0.8)
    assert abs(g[-1] + np.mean(0.8 - (y < 0.5))) < 1e-15
    assert np.count_nonzero(g[:-1]) == 0


def test_adam_first_step_closed_form(orc):
    """From zero moments the bias-corrected first step is lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w = np.ones(4)
    m, v = np.zeros(4), np.zeros(4)
    orc.mlp_adam(w, m, v, g, 1, lr=0.01, eps=1e-8)
    assert np.allclose(w, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_training_reduces_loss(orc):
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (256, 8))
    y = 3.0 + 2.0 * X[:, 0] - X[:, 1] ** 2 + 0.1 * rng.standard_normal(256)
    w = _init(orc, 5)
    m, v = np.zeros_like(w), np.zeros_like(w)
    l0 = orc.mlp_loss_grad(w, X, y, 0.9)[0]
    for t in range(1, 201):
        _, g = orc.mlp_loss_grad(w, X, y, 0.9)
        orc.mlp_adam(w, m, v, g, t, lr=3e-3)
    l1 = orc.mlp_loss_grad(w, X, y, 0.9)[0]
    assert l1 < 0.3 * l0
    # quantile 0.9: about 90% of the targets lie below the fit
    assert 0.75 <= np.mean(y <= orc.mlp_forward(w, X)) <= 0.99


def test_features(orc):
    f = orc.features([0, 0], [3, 4], [10, 0], [11, 1], 64, 128, 0.5)
    assert np.allclose(f, [6, 7, 10, np.sqrt(2) / 0.5, 14.0, np.sqrt(2) / 7, 2, np.log10(0.25)])
    # touching boxes: distance floor
    f = orc.features([0, 0, 0], [1, 1, 1], [1, 0, 0], [2, 1, 1], 8, 8, 1.0)
    assert f[4] == 0.0 and f[5] == np.sqrt(3) / 1e-12
