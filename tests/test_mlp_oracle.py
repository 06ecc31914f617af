"""Pins of the FP64 warm-start reference (network, Adam, summary statistics).

The network and features are the library's own component (not in the paper),
so they are pinned by finite differences and closed forms only."""
import numpy as np
from scipy.special import erf

import oracle as O

SHAPE = (6, 8, 2, 3)  # in, hidden, layers, out


def _params(seed):
    _, n = O.mlp_shapes(*SHAPE)
    return np.random.default_rng(seed).normal(0, 0.5, n)


def test_forward_matches_layerwise_numpy():
    p = _params(0)
    X = np.random.default_rng(1).normal(size=(5, 6))
    offs, _ = O.mlp_shapes(*SHAPE)
    h = X
    for li, (o, dout, din) in enumerate(offs):
        W = p[o:o + dout * din].reshape(dout, din)
        b = p[o + dout * din:o + dout * din + dout]
        h = h @ W.T + b
        if li < len(offs) - 1:
            h = 0.5 * h * (1 + erf(h / np.sqrt(2)))
    assert np.allclose(O.mlp_forward(p, X, *SHAPE), h, rtol=1e-13, atol=1e-13)


def test_backprop_matches_central_differences():
    p = _params(2)
    rng = np.random.default_rng(3)
    X, Y = rng.normal(size=(7, 6)), rng.normal(size=(7, 3))
    loss, g = O.mlp_loss_grad(p, X, Y, *SHAPE)
    pred = O.mlp_forward(p, X, *SHAPE)
    assert abs(loss - np.mean((pred - Y) ** 2)) < 1e-13
    h = 1e-6
    for i in range(0, len(p), 7):
        e = np.zeros_like(p)
        e[i] = h
        fd = (O.mlp_loss_grad(p + e, X, Y, *SHAPE)[0] - O.mlp_loss_grad(p - e, X, Y, *SHAPE)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_is_signed_learning_rate():
    # with bias correction the first step is lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m, v = np.zeros(3), np.zeros(3)
    O.mlp_adam(p, g, m, v, 1, 0.01, eps=0.0)
    assert np.allclose(p, np.array([1.0, -2.0, 0.5]) - 0.01 * np.sign(g), rtol=0, atol=1e-15)


def test_features_closed_form_for_a_linear_field():
    """d = 1, y = w x: the scaled semivariance is exactly w^2 dx^2 / (2 var y),
    so every rank's fit has intercept 0, slope w^2/(2 var y) and R^2 = 1."""
    rng = np.random.default_rng(4)
    x = rng.random((400, 1))
    y = 3.0 * x[:, 0]
    f = O.features(x, y, np.arange(400))
    var = np.var(y)
    assert abs(f[0] - np.log(var)) < 1e-12
    for r in range(5):
        c0, c1, r2 = f[2 + 3 * r: 5 + 3 * r]
        assert abs(c0) < 1e-8 and abs(c1 - 9.0 / (2 * var)) < 1e-8 * c1 and abs(r2 - 1) < 1e-9
    assert len(f) == 4 + 5 * 3
