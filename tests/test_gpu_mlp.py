"""GPU warm-start kernels against the FP64 reference: forward, loss and
gradient of the hand-written FP32 kernels (relative 1e-4), a short training
run that must reduce the loss, save/load, and the feature kernel."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbv():
    from paper_2504_12004_amd import sbv as S
    return S


@pytest.mark.parametrize("shape", [(64, 256, 3, 12), (20, 40, 2, 5), (7, 33, 1, 3)])
def test_loss_and_gradient_match_reference(sbv, shape):
    m = sbv.sbv_mlp_create(*shape, seed=3)
    p = sbv.sbv_mlp_get_params(m).astype(np.float64)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(70, shape[0])).astype(np.float32)
    Y = rng.normal(size=(70, shape[3])).astype(np.float32)
    loss, g = sbv.sbv_mlp_loss_grad(m, X, Y)
    rl, rg = O.mlp_loss_grad(p, X.astype(np.float64), Y.astype(np.float64), *shape)
    assert abs(loss - rl) <= 1e-4 * abs(rl)
    assert np.max(np.abs(g - rg)) <= 1e-4 * np.max(np.abs(rg))


def test_training_reduces_loss_and_roundtrips(sbv, tmp_path):
    rng = np.random.default_rng(6)
    X = rng.normal(size=(2048, 16)).astype(np.float32)
    W = rng.normal(size=(16, 4))
    Y = np.tanh(X @ W).astype(np.float32)
    m = sbv.sbv_mlp_create(16, 64, 2, 4, seed=1)
    l0 = sbv.sbv_mlp_train(m, X, Y, epochs=1, batch=256, lr=1e-3, seed=2)
    l1 = sbv.sbv_mlp_train(m, X, Y, epochs=40, batch=256, lr=1e-3, seed=3)
    assert l1 < 0.5 * l0
    pred = sbv.sbv_mlp_predict(m, X[:100])
    path = tmp_path / "net.bin"
    sbv.sbv_mlp_save(m, path)
    m2 = sbv.sbv_mlp_load(path, 4)
    assert np.array_equal(sbv.sbv_mlp_predict(m2, X[:100]), pred)


def test_features_match_reference(sbv):
    rng = np.random.default_rng(7)
    X = rng.random((3000, 10))
    y = np.sin(6 * X[:, 0]) + 0.3 * X[:, 3] ** 2 + 0.01 * rng.normal(size=3000)
    f = sbv.sbv_features(X, y, sub_n=5000, seed=0)  # n <= sub_n: every point used
    ref = O.features(X, y, np.arange(3000))
    assert len(f) == 64
    assert np.max(np.abs(f - ref) / np.maximum(1.0, np.abs(ref))) < 1e-9
