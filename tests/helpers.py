"""Shared helpers of the test-suite: seeded problems built and sampled with the
oracle (observations are never produced by the GPU path)."""
import numpy as np

import oracle as O
from paper_2504_12004_amd import synth


def problem(n, d, K, m, seed, two_nu=5, sigma2=1.0, tau2=1e-4, beta=None, lloyd_iters=5, min_bs=0,
            max_bs=0, m_gen=None):
    """X, theta from the synthetic generator; y from the oracle's Vecchia
    sampler on an independent generating structure; evaluation structure from
    the oracle builder."""
    X, theta, xi = synth.random_spd_problem(n, d, seed, beta=beta, sigma2=sigma2, tau2=tau2)
    bb = np.exp(theta[:d])
    Sg = O.build(X, bb, K=K, m=m_gen if m_gen is not None else 2 * max(m, 10), lloyd_iters=1, seed=seed + 7919)
    y = O.sample(X, Sg, theta, two_nu, xi)
    S = O.build(X, bb, K=K, m=m, lloyd_iters=lloyd_iters, min_bs=min_bs, max_bs=max_bs, seed=seed)
    return X, y, theta, S


def to_gpu(sbv, X, y, S):
    return sbv.sbv_blocks_import(X, y, S.block_ptr, S.block_pts, S.nn_ptr, S.nn_idx)


def block_tolerance(lb_ref, ud_ref, tol):
    """Per-block bound tol * (|l_i| + |d_i| + u_i): l_i = -(u_i + d_i + b_i log 2 pi)/2
    is a signed sum that can cancel to near 0, so its error is measured
    against the size of its parts (u_i = v^T v, d_i = 2 log det L')."""
    return tol * (np.abs(lb_ref) + np.abs(ud_ref[:, 1]) + ud_ref[:, 0])
