"""GPU gradient of the SBV log-likelihood (adjoint kernels) against the oracle's
block-inverse gradient and against central differences of the GPU value.

Bar (per component k): |g_gpu - g_oracle| <= 1e-8 * max(||g_oracle||_inf, 1)
in FP64; FD: |g - g_fd| <= 1e-5 * max(|g|, 1) + 10 eps |l| / h with h = 1e-5.
"""
import numpy as np
import pytest

import oracle as O
from helpers import problem, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbv():
    from paper_2504_12004_amd import sbv as S
    return S


def _cmp(sbv, X, y, th, S, two_nu, prec=0, tol=1e-8):
    ref_l, ref_g = O.sbv_loglik(X, y, S, th, two_nu, grad=True)
    B = to_gpu(sbv, X, y, S)
    l, g = sbv.sbv_loglik_grad(B, th, two_nu, prec)
    scale = max(1.0, np.max(np.abs(ref_g)))
    err = np.max(np.abs(g - ref_g)) / scale
    print(f"l {l[0]!r} ref {ref_l!r}; grad max rel err {err:.3e}", flush=True)
    assert abs(l[0] - ref_l) <= (1e-10 if prec == 0 else 1e-4) * abs(ref_l)
    assert err <= tol
    return B, g


@pytest.mark.parametrize("two_nu", [1, 3, 5, 7])
def test_grad_small(sbv, two_nu):
    X, y, th, S = problem(1500, 4, K=100, m=30, seed=41, two_nu=two_nu, tau2=1e-3)
    _cmp(sbv, X, y, th, S, two_nu)


def test_grad_large_joint_sizes(sbv):
    X, y, th, S = problem(5000, 10, K=250, m=230, seed=42, tau2=1e-4, max_bs=30)
    assert (np.diff(S.nn_ptr) + np.diff(S.block_ptr)).max() > 192
    _cmp(sbv, X, y, th, S, 5)


def test_grad_blocks_wider_than_one_chunk(sbv):
    # blocks of up to 60 points: the adjoint right-hand sides span two chunks
    X, y, th, S = problem(3000, 5, K=60, m=100, seed=43, tau2=1e-3, min_bs=35, max_bs=60)
    assert np.diff(S.block_ptr).max() > 32
    _cmp(sbv, X, y, th, S, 5)


def test_grad_central_differences(sbv):
    X, y, th, S = problem(2000, 6, K=100, m=40, seed=44, tau2=1e-3)
    B, g = _cmp(sbv, X, y, th, S, 5)
    h = 1e-5
    l0 = sbv.sbv_loglik(B, th, 5)[0]
    for k in range(len(th)):
        e = np.zeros_like(th)
        e[k] = h
        fd = (sbv.sbv_loglik(B, th + e, 5)[0] - sbv.sbv_loglik(B, th - e, 5)[0]) / (2 * h)
        assert abs(g[k] - fd) <= 1e-5 * max(abs(g[k]), 1.0) + 10 * 2.2e-16 * abs(l0) / h


def test_grad_fp32(sbv):
    X, y, th, S = problem(3000, 10, K=150, m=120, seed=45, tau2=1e-4)
    _cmp(sbv, X, y, th, S, 5, prec=1, tol=1e-3)
