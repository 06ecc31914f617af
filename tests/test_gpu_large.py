"""GPU parity of the large-block path (joint sizes 273..512: the prefix kernel
plus the register kernel with streamed prefix updates) against the FP64 oracle.

The oracle runs Alg. 5 on the whole joint set; the GPU splits it into a
prefix of conditioning points and the trailing 17 tiles (block Cholesky), so
agreement to the FP64 tolerance checks the split itself.
"""
import numpy as np
import pytest

import oracle as O
from helpers import block_tolerance, problem, to_gpu
from paper_2504_12004_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbv():
    from paper_2504_12004_amd import sbv as S
    return S


def _compare(sbv, X, y, th, S, two_nu, prec, tol):
    ref, lb_ref, ud_ref = O.sbv_loglik(X, y, S, th, two_nu, blocks=True, parts=True)
    B = to_gpu(sbv, X, y, S)
    got = sbv.sbv_loglik(B, th, two_nu, prec)[0]
    lb = sbv.sbv_blocks_terms(B)
    worst = np.max(np.abs(lb - lb_ref) / (np.abs(lb_ref) + np.abs(ud_ref[:, 1]) + ud_ref[:, 0]))
    print(f"ref {ref!r} got {got!r} rel {abs(got - ref) / abs(ref):.3e} worst block {worst:.3e}", flush=True)
    assert abs(got - ref) <= tol * abs(ref)
    assert np.all(np.abs(lb - lb_ref) <= block_tolerance(lb_ref, ud_ref, tol))
    return B


def _explicit(n, d, sizes, targets, seed):
    """Consecutive blocks of the given sizes; block r conditions on the
    targets[r] points just before it (all in earlier blocks)."""
    X, th, _ = synth.random_spd_problem(n, d, seed, beta=np.full(d, 0.3), sigma2=1.0, tau2=1e-4)
    rng = np.random.default_rng(seed + 1)
    y = rng.standard_normal(n)
    bp = np.r_[0, np.cumsum(sizes)]
    assert bp[-1] == n
    nn_ptr, nn_idx = [0], []
    for r in range(len(sizes)):
        m = min(targets[r], bp[r])
        nn_idx.extend(range(bp[r] - m, bp[r]))
        nn_ptr.append(len(nn_idx))
    S = O.Structure(n, d, 0, bp, np.arange(n), np.array(nn_ptr), np.array(nn_idx, dtype=np.int64))
    return X, y, th, S


def test_fp64_m400_builder_structure(sbv):
    # k-means blocks of 5..60 points conditioned on m = 400 neighbours: joint
    # sizes up to 460 (prefix lengths up to 12) next to small early blocks
    X, y, th, S = problem(4000, 10, K=200, m=400, seed=31, tau2=1e-4, min_bs=5, max_bs=60, m_gen=60)
    sizes = np.diff(S.nn_ptr) + np.diff(S.block_ptr)
    assert sizes.max() > 400 and (sizes > 272).sum() > 50 and sizes.min() < 100
    B = _compare(sbv, X, y, th, S, 5, sbv.SBV_FP64, 1e-10)
    B.free()


def test_fp64_prefix_extremes(sbv):
    # joint sizes at both ends of the large path: 273 (one prefix tile),
    # 512 (fifteen), a ragged last tile, and register-path neighbours
    sizes = [32] * 24 + [60, 32, 17, 32, 5, 32]
    targets = [0] * 8 + [241, 480, 452, 300, 256, 257, 399, 400, 480, 272, 240, 16] + [0] * 4 + \
              [452, 241, 470, 480, 507, 400]
    n = int(np.sum(sizes))
    X, y, th, S = _explicit(n, 5, sizes, targets, seed=32)
    joint = np.diff(S.nn_ptr) + np.diff(S.block_ptr)
    assert joint.max() == 512 and 273 in joint and (joint > 272).sum() >= 12
    B = _compare(sbv, X, y, th, S, 3, sbv.SBV_FP64, 1e-10)
    B.free()


def test_fp32_large(sbv):
    # sigma^2 = 4: with sigma^2 = 1 the per-point terms of this small dataset
    # take both signs and the total (|l| ~ 100-500) is mostly cancellation, which
    # makes a relative bound on it meaningless; here |l| ~ 3400
    X, y, th, S = problem(4000, 10, K=200, m=400, seed=33, sigma2=4.0, tau2=1e-4, min_bs=5, max_bs=60, m_gen=60)
    B = _compare(sbv, X, y, th, S, 5, sbv.SBV_FP32, 1e-4)
    B.free()


def test_windows_and_fallback(sbv, monkeypatch):
    # several workspace windows with a ragged last one, in FP64 and in FP32
    # with every block sent back to FP64 by the pivot test
    monkeypatch.setenv("SBV_LARGE_WINDOW", "7")
    X, y, th, S = problem(3000, 10, K=150, m=400, seed=34, tau2=1e-4, min_bs=5, max_bs=60, m_gen=60)
    joint = np.diff(S.nn_ptr) + np.diff(S.block_ptr)
    assert (joint > 272).sum() > 20
    B = _compare(sbv, X, y, th, S, 5, sbv.SBV_FP64, 1e-10)
    B.free()
    monkeypatch.setenv("SBV_PIV_TAU", "2.0")  # every pivot is below twice the diagonal
    B = _compare(sbv, X, y, th, S, 5, sbv.SBV_FP32, 1e-10)
    assert sbv.sbv_blocks_fallback_count(B) == S.K
    B.free()


def test_large_rejections(sbv):
    # a block above 272 whose prefix would reach into its own points
    sizes = [32] * 10 + [280]
    targets = [0] * 10 + [0]
    X, y, th, S = _explicit(600, 3, sizes, targets, seed=35)
    with pytest.raises(sbv.SBVError):
        to_gpu(sbv, X, y, S)
    # the conditional simulator stays within the register path
    X, y, th, S = problem(1500, 5, K=60, m=300, seed=36, tau2=1e-3, m_gen=40)
    B = to_gpu(sbv, X, y, S)
    with pytest.raises(sbv.SBVError):
        sbv.sbv_sample(B, th, 5, np.zeros(X.shape[0]))
    B.free()


def _grad_cmp(sbv, X, y, th, S, two_nu, prec, tol):
    ref_l, ref_g = O.sbv_loglik(X, y, S, th, two_nu, grad=True)
    B = to_gpu(sbv, X, y, S)
    l, g = sbv.sbv_loglik_grad(B, th, two_nu, prec)
    scale = max(1.0, np.max(np.abs(ref_g)))
    err = np.max(np.abs(g - ref_g)) / scale
    print(f"l {l[0]!r} ref {ref_l!r}; grad max rel err {err:.3e}", flush=True)
    assert abs(l[0] - ref_l) <= 1e-10 * abs(ref_l)
    assert err <= tol
    return B


def test_grad_large_fp64(sbv):
    # every component of the gradient through the prefix adjoint and the
    # streamed contraction, blocks of up to 60 points (two right-hand-side chunks)
    X, y, th, S = problem(2000, 10, K=100, m=400, seed=37, tau2=1e-4, min_bs=5, max_bs=60, m_gen=60)
    joint = np.diff(S.nn_ptr) + np.diff(S.block_ptr)
    assert (joint > 272).sum() > 30 and np.diff(S.block_ptr).max() > 32
    B = _grad_cmp(sbv, X, y, th, S, 5, sbv.SBV_FP64, 1e-8)
    B.free()


def test_grad_large_extremes_and_fallback(sbv, monkeypatch):
    sizes = [32] * 24 + [60, 32, 17, 32, 5, 32]
    targets = [0] * 8 + [241, 480, 452, 300, 256, 257, 399, 400, 480, 272, 240, 16] + [0] * 4 + \
              [452, 241, 470, 480, 507, 400]
    X, y, th, S = _explicit(int(np.sum(sizes)), 5, sizes, targets, seed=38)
    monkeypatch.setenv("SBV_LARGE_WINDOW", "5")
    B = _grad_cmp(sbv, X, y, th, S, 3, sbv.SBV_FP64, 1e-8)
    B.free()
    # FP32 with every block sent back to FP64: the FP64 bar applies
    monkeypatch.setenv("SBV_PIV_TAU", "2.0")
    B = _grad_cmp(sbv, X, y, th, S, 3, sbv.SBV_FP32, 1e-8)
    assert sbv.sbv_blocks_fallback_count(B) == S.K
    B.free()


def test_grad_m400_workload_subset(sbv):
    # the generator of the n = 5e6, m = 400 workload at n = 2e4 with its own
    # structure (K = 1000, k-means blocks of 5..60 points, m = 400)
    w = synth.dataset("grad_5m", n=20000)
    X, th, xi = w["X"], w["theta"], w["xi"]
    bb = np.exp(th[:10])
    Sg = O.build(X, bb, K=1000, m=100, lloyd_iters=1, seed=w["seed"] + 7919)
    y = O.sample(X, Sg, th, 5, xi)
    S = O.build(X, bb, K=1000, m=400, lloyd_iters=5, min_bs=5, max_bs=60, seed=w["seed"])
    assert (np.diff(S.nn_ptr) + np.diff(S.block_ptr)).max() > 400
    B = _grad_cmp(sbv, X, y, th, S, 5, sbv.SBV_FP64, 1e-8)
    B.free()
