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


def test_adam_bias_correction_over_several_steps():
    """Kingma & Ba, Algorithm 1, worked by hand.  With a constant gradient g
    the corrected moments are exactly g and g^2, so every step is
    lr * sign(g) (eps = 0).  With the gradient alternating g, -g, g the
    corrected first moments are g, -(1 - b1)/(1 + b1) g and
    (1 - b1 + b1^2)/(1 + b1 + b1^2) g while the corrected second moment stays
    g^2.  A bias correction with a fixed exponent (1 - b1 for every t) fails
    both from t = 2 on."""
    b1, b2, lr = 0.9, 0.999, 0.01
    g = np.array([0.3, -4.0, 2e-3])
    p, m, v = np.array([1.0, -2.0, 0.5]), np.zeros(3), np.zeros(3)
    for t in range(1, 6):
        O.mlp_adam(p, g, m, v, t, lr, b1, b2, eps=0.0)
        assert np.allclose(p, np.array([1.0, -2.0, 0.5]) - t * lr * np.sign(g), rtol=0, atol=1e-14)
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    steps = [1.0, -(1 - b1) / (1 + b1), (1 - b1 + b1 ** 2) / (1 + b1 + b1 ** 2)]
    expect = np.zeros(3)
    for t, sgn in enumerate([1.0, -1.0, 1.0], start=1):
        O.mlp_adam(p, sgn * g, m, v, t, lr, b1, b2, eps=0.0)
        expect = expect - lr * steps[t - 1] * np.sign(g)
        assert np.allclose(p, expect, rtol=0, atol=1e-14)


def test_nearest_neighbour_semivariance_feature_closed_form():
    """f1 = log of the mean over points of (y_i - y_nn(i))^2 / 2.  For a
    linear field y = w x on an evenly spaced grid in d = 1 (spacing h, points
    in shuffled order) every nearest neighbour is one grid step away, so
    f1 = log(w^2 h^2 / 2) exactly (up to rounding)."""
    n, h, w = 500, 1.0 / 500, 2.5
    x = (np.random.default_rng(6).permutation(n) * h)[:, None]
    y = w * x[:, 0]
    f = O.features(x, y, np.arange(n))
    assert abs(f[1] - np.log(0.5 * w * w * h * h)) < 1e-9
    # the same field with a different slope moves f1 by log of the slope ratio squared
    f2 = O.features(x, 3.0 * y, np.arange(n))
    assert abs((f2[1] - f[1]) - np.log(9.0)) < 1e-9
