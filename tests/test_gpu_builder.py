"""GPU block builder (sbv_build_blocks) against brute force and the oracle.

Several clusterings are valid (k-means local optima), so the builder is
checked by invariants: the blocks partition the points, size bounds hold, every
neighbour set is exactly the m nearest points of strictly earlier blocks to the
block centroid (numpy brute force), and Lloyd passes follow the same rule as the
oracle's builder -- on these inputs both produce the same structure.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbv():
    from paper_2504_12004_amd import sbv as S
    return S


def _structure(sbv, B):
    bp, pts, npt, nid = sbv.sbv_blocks_export(B)
    return O.Structure(B.n, B.d, 0, bp, pts, npt, nid)


def _check_knn(X, bb, S, m):
    Z = X / bb
    for r in range(S.K):
        Bk, J = S.block(r)
        earlier = S.block_pts[:S.block_ptr[r]]
        assert len(J) == min(m, len(earlier))
        if len(J) == 0:
            continue
        c = Z[Bk].mean(0)
        d2 = ((Z[earlier] - c) ** 2).sum(1)
        kth = np.sort(d2)[len(J) - 1]
        dj = ((Z[J] - c) ** 2).sum(1)
        assert np.all(dj <= kth * (1 + 1e-12)), r
        assert set(J.tolist()) <= set(earlier.tolist())


@pytest.mark.parametrize("method,iters", [(0, 6), (1, 0)])
def test_builder_invariants_and_oracle_agreement(sbv, method, iters):
    rng = np.random.default_rng(31)
    X = rng.random((4000, 6))
    bb = np.array([0.1, 0.3, 0.5, 1.0, 2.0, 3.0])
    B = sbv.sbv_build_blocks(X, None, bb, 200, 40, method=method, lloyd_iters=iters, min_bs=5, max_bs=40, seed=5)
    S = _structure(sbv, B)
    assert np.array_equal(np.sort(S.block_pts), np.arange(4000))
    sizes = np.diff(S.block_ptr)
    assert sizes.min() >= 5 and sizes.max() <= 40
    _check_knn(X, bb, S, 40)
    R = O.build(X, bb, K=200, m=40, lloyd_iters=iters, min_bs=5, max_bs=40, seed=5)
    assert np.array_equal(R.block_ptr, S.block_ptr)
    assert np.array_equal(R.block_pts, S.block_pts)
    assert np.array_equal(R.nn_ptr, S.nn_ptr)
    assert np.array_equal(R.nn_idx, S.nn_idx)
    B.free()


def test_builder_then_loglik_matches_oracle(sbv):
    from helpers import problem
    X, y, th, _ = problem(5000, 10, K=250, m=100, seed=32, tau2=1e-4)
    bb = np.exp(th[:10])
    B = sbv.sbv_build_blocks(X, y, bb, 250, 100, lloyd_iters=5, seed=9)
    S = _structure(sbv, B)
    _check_knn(X, bb, S, 100)
    got = sbv.sbv_loglik(B, th, 5)[0]
    ref = O.sbv_loglik(X, y, S, th, 5)
    assert abs(got - ref) <= 1e-10 * abs(ref)


def test_builder_rejects_bad_arguments(sbv):
    X = np.random.default_rng(0).random((100, 3))
    with pytest.raises(sbv.SBVError):
        sbv.sbv_build_blocks(X, None, [1.0, 1.0, -1.0], 10, 5)
    with pytest.raises(sbv.SBVError):
        sbv.sbv_build_blocks(X, None, [1.0, 1.0, 1.0], 200, 5)
    Xn = X.copy()
    Xn[3, 1] = np.nan
    with pytest.raises(sbv.SBVError):
        sbv.sbv_build_blocks(Xn, None, [1.0, 1.0, 1.0], 10, 5)
