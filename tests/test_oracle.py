"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test names the invariant it checks; none retypes the oracle's formula:
library routines (scipy Bessel K, scipy multivariate normal, numpy Cholesky),
closed-form limits, brute force and finite differences are the references.
"""
import numpy as np
import pytest
from scipy.special import gamma, kv
from scipy.stats import multivariate_normal

import oracle as O

TWO_NU = (1, 3, 5, 7)


def _theta(beta, s2, t2):
    return np.r_[np.log(beta), np.log(s2), np.log(t2)]


def _data(n, d, seed, beta, s2=1.0, t2=1e-2, two_nu=5):
    rng = np.random.default_rng(seed)
    X = rng.random((n, d))
    th = _theta(beta, s2, t2)
    S = O.cov_matrix(X, X, th, two_nu, True)
    y = np.linalg.cholesky(S) @ rng.standard_normal(n)
    return X, y, th


# --- Matern closed forms: Sec. 4.4 Eq. (maternkernel), literal in r --------
@pytest.mark.parametrize("two_nu", TWO_NU)
def test_matern_closed_form_matches_bessel(two_nu):
    nu = two_nu / 2
    r = np.linspace(1e-3, 8.0, 300)
    ref = 2 ** (1 - nu) / gamma(nu) * r ** nu * kv(nu, r)
    got = np.array([O.rho(x, two_nu) for x in r])
    assert np.max(np.abs(got - ref)) < 5e-15
    assert O.rho(0.0, two_nu) == 1.0


@pytest.mark.parametrize("two_nu", TWO_NU)
def test_matern_derivative_matches_fd(two_nu):
    # -rho'(r)/r against central differences of the Bessel-K definition
    nu = two_nu / 2
    f = lambda r: 2 ** (1 - nu) / gamma(nu) * r ** nu * kv(nu, r)
    for r in (0.05, 0.3, 1.0, 2.5, 6.0):
        h = 1e-6 * max(r, 1.0)
        fd = -(f(r + h) - f(r - h)) / (2 * h) / r
        assert abs(O.mdrho_over_r(r, two_nu) - fd) < 1e-7 * max(1.0, abs(fd))


def test_nugget_on_diagonal_only():
    rng = np.random.default_rng(1)
    X = rng.random((5, 2))
    X[3] = X[1]  # duplicate location, distinct observation
    th = _theta([0.5, 0.5], 2.0, 0.25)
    S = O.cov_matrix(X, X, th, 3, True)
    assert np.allclose(np.diag(S), 2.25)
    assert S[1, 3] == pytest.approx(2.0)  # sigma^2 rho(0), no nugget off the diagonal


# --- Exact GP, Eq. (1) -------------------------------------------------------
@pytest.mark.parametrize("two_nu", TWO_NU)
def test_exact_loglik_matches_scipy_mvn(two_nu):
    X, y, th = _data(150, 3, 2, [0.3, 0.6, 1.2], two_nu=two_nu)
    S = O.cov_matrix(X, X, th, two_nu, True)
    ref = multivariate_normal(np.zeros(len(y)), S).logpdf(y)
    assert abs(O.exact_loglik(X, y, th, two_nu) - ref) < 1e-10 * abs(ref)


def test_exact_gradient_matches_fd():
    X, y, th = _data(120, 3, 3, [0.3, 0.6, 1.2])
    _, g = O.exact_loglik(X, y, th, 5, grad=True)
    h = 1e-5
    for k in range(len(th)):
        e = np.zeros_like(th)
        e[k] = h
        fd = (O.exact_loglik(X, y, th + e, 5) - O.exact_loglik(X, y, th - e, 5)) / (2 * h)
        assert abs(g[k] - fd) < 1e-5 * max(1.0, abs(fd))


# --- Block Vecchia: chain rule (Sec. 4.2) ------------------------------------
@pytest.mark.parametrize("two_nu", TWO_NU)
def test_full_conditioning_is_exact(two_nu):
    """P1: when every block conditions on all earlier points the block product is
    the exact chain-rule factorisation, so l_SBV = l_exact (values and gradients)."""
    X, y, th = _data(240, 4, 4, [0.2, 0.5, 1.0, 2.0], two_nu=two_nu)
    S = O.build(X, np.exp(th[:4]), K=25, m=10 ** 6, lloyd_iters=4, seed=7)
    ll, g = O.sbv_loglik(X, y, S, th, two_nu, grad=True)
    ex, gex = O.exact_loglik(X, y, th, two_nu, grad=True)
    assert abs(ll - ex) < 1e-11 * abs(ex)
    assert np.max(np.abs(g - gex)) < 1e-9 * max(1.0, np.max(np.abs(gex)))


def test_single_block_is_exact():
    """P2: K = 1 is one unconditioned block, i.e. Eq. (1)."""
    X, y, th = _data(90, 3, 5, [0.3, 0.4, 0.5])
    S = O.build(X, np.exp(th[:3]), K=1, m=50, lloyd_iters=0, seed=0)
    assert S.K == 1 and len(S.nn_idx) == 0
    assert abs(O.sbv_loglik(X, y, S, th, 5) - O.exact_loglik(X, y, th, 5)) < 1e-12 * 200


def test_block_term_is_joint_minus_conditioning_logpdf():
    """P3: each Alg. 5 block term equals log N(y_A; Sigma_A) - log N(y_J; Sigma_J)."""
    X, y, th = _data(400, 3, 6, [0.2, 0.3, 0.9])
    S = O.build(X, np.exp(th[:3]), K=40, m=25, lloyd_iters=5, seed=2)
    _, lb = O.sbv_loglik(X, y, S, th, 5, blocks=True)
    for r in range(S.K):
        B, J = S.block(r)
        A = np.r_[J, B]
        SA = O.cov_matrix(X[A], X[A], th, 5, True)
        ref = multivariate_normal(np.zeros(len(A)), SA).logpdf(y[A])
        if len(J):
            SJ = O.cov_matrix(X[J], X[J], th, 5, True)
            ref -= multivariate_normal(np.zeros(len(J)), SJ).logpdf(y[J])
        assert abs(lb[r] - ref) < 1e-11 * max(1.0, abs(ref))


def test_nugget_only_limit():
    """P4: with sigma^2 -> 0 every observation is independent N(0, tau^2)."""
    X, y, _ = _data(300, 3, 7, [0.2, 0.3, 0.9])
    th = _theta([0.2, 0.3, 0.9], np.exp(-60.0), 0.3)
    S = O.build(X, [0.2, 0.3, 0.9], K=30, m=20, seed=1)
    ref = -0.5 * len(y) * np.log(2 * np.pi * 0.3) - y @ y / (2 * 0.3)
    assert abs(O.sbv_loglik(X, y, S, th, 5) - ref) < 1e-12 * abs(ref)


def test_no_conditioning_is_independent_blocks():
    """P5: m = 0 gives a product of independent block densities."""
    X, y, th = _data(200, 2, 8, [0.2, 0.4])
    S = O.build(X, np.exp(th[:2]), K=20, m=0, seed=3)
    ref = 0.0
    for r in range(S.K):
        B, J = S.block(r)
        assert len(J) == 0
        ref += multivariate_normal(np.zeros(len(B)), O.cov_matrix(X[B], X[B], th, 5, True)).logpdf(y[B])
    assert abs(O.sbv_loglik(X, y, S, th, 5) - ref) < 1e-12 * abs(ref)


def test_ou_markov_exactness():
    """P6: d = 1, nu = 1/2, no nugget (Ornstein-Uhlenbeck, Markov): contiguous
    interval blocks ordered left to right with m >= 1 are exact, because the
    nearest earlier point to each block centroid is its predecessor."""
    rng = np.random.default_rng(9)
    n = 400
    x = np.sort(rng.random(n))[:, None]
    th = _theta([0.3], 1.5, 1e-300)
    S0 = O.cov_matrix(x, x, th, 1, True)
    y = np.linalg.cholesky(S0) @ rng.standard_normal(n)
    bs = 8
    bp = np.arange(0, n + 1, bs)
    pts = np.arange(n)
    K = len(bp) - 1
    nn_ptr = np.r_[0, 0, np.arange(1, K)]
    nn_idx = bp[1:-1] - 1  # predecessor point of every block after the first
    S = O.Structure(n, 1, 1, bp, pts, nn_ptr, nn_idx)
    ex = O.exact_loglik(x, y, th, 1)
    assert abs(O.sbv_loglik(x, y, S, th, 1) - ex) < 1e-11 * abs(ex)


def test_kl_nonnegative_and_nonincreasing_in_m():
    """P7 / Eq. (kldivergence): KL = l_exact(0) - l_SBV(0) >= 0, and larger
    nested conditioning sets cannot increase it."""
    X, _, th = _data(300, 4, 10, [0.1, 0.3, 1.0, 3.0])
    y0 = np.zeros(300)
    ex0 = O.exact_loglik(X, y0, th, 7)
    kls = []
    for m in (0, 5, 10, 20, 40, 80, 300):
        S = O.build(X, np.exp(th[:4]), K=30, m=m, lloyd_iters=5, seed=11)
        kls.append(ex0 - O.sbv_loglik(X, y0, S, th, 7))
    assert all(k >= -1e-9 for k in kls)
    assert all(a >= b - 1e-9 for a, b in zip(kls, kls[1:]))
    assert abs(kls[-1]) < 1e-9


def test_quadratic_form_expectation_tiny():
    """P8: with y drawn from the exact GP, E[sum_i u_i] = tr(S_vecchia^{-1} S) and for
    m >= n this is exactly n; checked through E over y of -2(l(y) - l(0))."""
    X, _, th = _data(60, 2, 12, [0.3, 0.5])
    S = O.build(X, np.exp(th[:2]), K=6, m=60, seed=1)
    Sig = O.cov_matrix(X, X, th, 5, True)
    # -2(l(y)-l(0)) = y^T Q y with Q the Vecchia precision; E = tr(Q Sig) = n.
    # Recover Q columnwise from the oracle (polarisation), then the trace.
    n = 60
    l0 = O.sbv_loglik(X, np.zeros(n), S, th, 5)
    q = lambda v: -2.0 * (O.sbv_loglik(X, v, S, th, 5) - l0)
    E = np.eye(n)
    diag = np.array([q(E[i]) for i in range(n)])
    tr = 0.0
    for i in range(n):
        for j in range(n):
            qij = diag[i] if i == j else 0.5 * (q(E[i] + E[j]) - diag[i] - diag[j])
            tr += qij * Sig[j, i]
    assert abs(tr - n) < 1e-8 * n


def test_invariances():
    """P9: scaling x and beta jointly, translating x, permuting dimensions with
    beta, and permuting points inside blocks and conditioning sets."""
    X, y, th = _data(200, 3, 13, [0.2, 0.5, 1.1])
    S = O.build(X, np.exp(th[:3]), K=20, m=15, seed=4)
    base = O.sbv_loglik(X, y, S, th, 5)
    th2 = th.copy()
    th2[:3] += np.log(3.0)
    assert abs(O.sbv_loglik(3.0 * X, y, S, th2, 5) - base) < 1e-12 * abs(base)
    assert abs(O.sbv_loglik(X + 7.25, y, S, th, 5) - base) < 1e-11 * abs(base)
    p = [2, 0, 1]
    th3 = np.r_[th[:3][p], th[3:]]
    assert abs(O.sbv_loglik(X[:, p], y, S, th3, 5) - base) < 1e-12 * abs(base)
    rng = np.random.default_rng(0)
    pts, nidx = S.block_pts.copy(), S.nn_idx.copy()
    for r in range(S.K):
        a, b = S.block_ptr[r], S.block_ptr[r + 1]
        pts[a:b] = rng.permutation(pts[a:b])
        a, b = S.nn_ptr[r], S.nn_ptr[r + 1]
        nidx[a:b] = rng.permutation(nidx[a:b])
    S2 = O.Structure(S.n, S.d, S.m, S.block_ptr, pts, S.nn_ptr, nidx)
    assert abs(O.sbv_loglik(X, y, S2, th, 5) - base) < 1e-12 * abs(base)


def test_sigma2_gradient_identity_without_nugget():
    """P10: with tau^2 = 0 the model is sigma^2 times a fixed correlation, so
    dl/dlog sigma^2 = (sum_i u_i - n)/2 with sum_i u_i = 2(l(0) - l(y))."""
    X, y, _ = _data(180, 3, 14, [0.3, 0.6, 1.0])
    th = _theta([0.3, 0.6, 1.0], 1.7, 1e-300)
    S = O.build(X, [0.3, 0.6, 1.0], K=18, m=12, seed=5)
    ll, g = O.sbv_loglik(X, y, S, th, 5, grad=True)
    u = 2.0 * (O.sbv_loglik(X, np.zeros_like(y), S, th, 5) - ll)
    assert abs(g[3] - (u - len(y)) / 2) < 1e-9 * max(1.0, abs(g[3]))


@pytest.mark.parametrize("two_nu", TWO_NU)
def test_sbv_gradient_matches_fd(two_nu):
    """P12: block-inverse gradient against central differences (h = 1e-5)."""
    X, y, th = _data(220, 3, 15, [0.2, 0.5, 1.1], two_nu=two_nu)
    S = O.build(X, np.exp(th[:3]), K=22, m=14, seed=6)
    ll, g = O.sbv_loglik(X, y, S, th, two_nu, grad=True)
    h = 1e-5
    for k in range(len(th)):
        e = np.zeros_like(th)
        e[k] = h
        fd = (O.sbv_loglik(X, y, S, th + e, two_nu) - O.sbv_loglik(X, y, S, th - e, two_nu)) / (2 * h)
        assert abs(g[k] - fd) < 1e-5 * max(1.0, abs(g[k])) + 10 * 2.2e-16 * abs(ll) / h


def test_neighbours_are_exact_brute_force():
    """P13: J_i are the m nearest points of strictly earlier blocks to the block
    centroid in beta_build-scaled space (brute force with numpy)."""
    rng = np.random.default_rng(16)
    X = rng.random((500, 3))
    bb = np.array([0.1, 0.4, 2.0])
    S = O.build(X, bb, K=50, m=30, lloyd_iters=3, seed=8)
    Z = X / bb
    rank_of = np.empty(500, np.int64)
    for r in range(S.K):
        rank_of[S.block_pts[S.block_ptr[r]:S.block_ptr[r + 1]]] = r
    for r in range(S.K):
        B, J = S.block(r)
        c = Z[B].mean(0)
        earlier = S.block_pts[:S.block_ptr[r]]
        assert len(J) == min(30, len(earlier))
        if len(J) == 0:
            continue
        assert np.all(rank_of[J] < r)
        d2 = ((Z[earlier] - c) ** 2).sum(1)
        kth = np.sort(d2)[len(J) - 1]
        dj = ((Z[J] - c) ** 2).sum(1)
        assert np.all(dj <= kth * (1 + 1e-12))
        assert np.all(np.diff(dj) >= -1e-15)


def test_kmeans_objective_and_bounds():
    """P14: Lloyd passes never increase the k-means objective; RAC is zero passes;
    size bounds hold; blocks partition the points."""
    rng = np.random.default_rng(17)
    X = rng.random((3000, 4))
    S = O.build(X, np.ones(4), K=150, m=10, lloyd_iters=8, min_bs=5, max_bs=60, seed=9)
    obj = S.kmeans_obj
    assert len(obj) >= 2 and np.all(np.diff(obj) <= 1e-9 * obj[0])
    sizes = np.diff(S.block_ptr)
    assert sizes.min() >= 5 and sizes.max() <= 60
    assert np.array_equal(np.sort(S.block_pts), np.arange(3000))
    R = O.build(X, np.ones(4), K=150, m=10, lloyd_iters=0, seed=9)
    assert len(R.kmeans_obj) == 1


def test_sampler_with_full_conditioning_is_cholesky_draw():
    """O6: visiting blocks in rank order and drawing y_B = mu + L' xi_B with every
    earlier point conditioned on reproduces y = chol(Sigma) xi in that order."""
    rng = np.random.default_rng(18)
    n = 150
    X = rng.random((n, 3))
    th = _theta([0.3, 0.5, 0.8], 1.2, 1e-3)
    S = O.build(X, [0.3, 0.5, 0.8], K=15, m=n, seed=3)
    xi = rng.standard_normal(n)
    y = O.sample(X, S, th, 5, xi)
    P = S.block_pts
    L = np.linalg.cholesky(O.cov_matrix(X[P], X[P], th, 5, True))
    assert np.max(np.abs(y[P] - L @ xi[P])) < 1e-10


# --- Alg. 1 Step 5: the total is a compensated sum ------------------------
def test_total_is_compensated_where_plain_summation_fails():
    """One block term near -1e16 followed by 2,000 terms of -log(2 pi)/2:
    plain left-to-right FP64 summation drops every small term (each is below
    half an ulp of 1e16), the compensated total must keep them.  The
    reference is math.fsum (exactly rounded) of the oracle's own block terms;
    the blocks are single points with no conditioning (m = 0), so each term
    is -(y_i^2/s + log s + log 2 pi)/2 with s = sigma^2 + tau^2."""
    import math
    K = 2001
    rng = np.random.default_rng(7)
    X = rng.random((K, 1))
    y = np.zeros(K)
    y[0] = np.sqrt(2e16)  # s = 1: first term about -1e16
    th = _theta([0.3], 1.0 - 1e-6, 1e-6)
    ar = np.arange(K + 1)
    S = O.Structure(K, 1, 0, ar, ar[:-1], np.zeros(K + 1, np.int64), np.zeros(0, np.int64))
    tot, lb = O.sbv_loglik(X, y, S, th, 5, blocks=True)
    exact = math.fsum(lb)
    naive = 0.0
    for v in lb:
        naive += v
    assert abs(naive - exact) > 1000.0  # plain summation is far off here
    assert abs(tot - exact) <= 2.0 * np.spacing(abs(exact))
    # the small terms are the closed form of a single-point block
    assert np.allclose(lb[1:], -0.5 * np.log(2 * np.pi), rtol=0, atol=1e-15)


def test_block_parts_recombine_to_the_term():
    """u_i = v^T v and d_i = 2 log det L' that the oracle reports give back
    l_i = -(u_i + d_i + b_i log 2 pi)/2 (Alg. 5 Step 2 with the constant of
    Eq. (1)), and for a block without conditioning they are the quadratic form
    and log-determinant of its own covariance (numpy Cholesky)."""
    X, y, th = _data(300, 3, 41, [0.3, 0.5, 0.8], t2=1e-2)
    S = O.build(X, np.exp(th[:3]), K=20, m=25, lloyd_iters=2, seed=3)
    tot, lb, ud = O.sbv_loglik(X, y, S, th, 5, blocks=True, parts=True)
    b = np.diff(S.block_ptr)
    assert np.allclose(lb, -0.5 * (ud[:, 0] + ud[:, 1] + b * np.log(2 * np.pi)), rtol=1e-14, atol=1e-12)
    B0, J0 = S.block(0)
    assert len(J0) == 0
    C0 = O.cov_matrix(X[B0], X[B0], th, 5, True)
    L0 = np.linalg.cholesky(C0)
    w = np.linalg.solve(L0, y[B0])
    assert abs(ud[0, 0] - w @ w) < 1e-10 * max(1.0, w @ w)
    assert abs(ud[0, 1] - 2 * np.sum(np.log(np.diag(L0)))) < 1e-10 * max(1.0, abs(ud[0, 1]))


# --- Prediction: Sec. 5.5 with the block-conditional product of Sec. 4.2 --
def _exact_conditional(X, y, Xp, th, two_nu):
    """Dense GP conditional of new noisy observations given all observations
    (the joint normal of the new and observed outputs, numpy solves)."""
    K = O.cov_matrix(X, X, th, two_nu, True)
    Kx = O.cov_matrix(Xp, X, th, two_nu, False)
    Kp = O.cov_matrix(Xp, Xp, th, two_nu, True)
    A = np.linalg.solve(K, Kx.T)
    return Kx @ np.linalg.solve(K, y), np.diag(Kp - Kx @ A)


def test_prediction_with_all_observations_is_the_exact_conditional():
    X, y, th = _data(300, 3, 81, [0.3, 0.5, 0.8], t2=1e-2)
    Xp = np.random.default_rng(82).random((45, 3))
    P = O.pred_structure(X, Xp, np.exp(th[:3]), K=9, m=300, lloyd_iters=2, seed=4)
    assert np.all(np.diff(P.nn_ptr) == 300)
    mean, var = O.predict(X, y, Xp, P, th, 5)
    em, ev = _exact_conditional(X, y, Xp, th, 5)
    assert np.max(np.abs(mean - em)) < 1e-10 * max(1.0, np.max(np.abs(em)))
    assert np.max(np.abs(var - ev) / ev) < 1e-9


def test_prediction_neighbours_are_brute_force_and_variance_shrinks_with_m():
    X, y, th = _data(400, 4, 83, [0.2, 0.4, 0.6, 1.0], t2=1e-3)
    Xp = np.random.default_rng(84).random((60, 4))
    bb = np.exp(th[:4])
    Z, Zp = X / bb, Xp / bb
    prev = None
    for m in (5, 20, 60):
        P = O.pred_structure(X, Xp, bb, K=12, m=m, lloyd_iters=3, seed=5)
        for r in range(P.K):
            Bp, J = P.block(r)
            c = Zp[Bp].mean(0)
            d2 = ((Z - c) ** 2).sum(1)
            assert set(J.tolist()) == set(np.argsort(d2, kind="stable")[:m].tolist())
        mean, var = O.predict(X, y, Xp, P, th, 5)
        s2, t2 = np.exp(th[4]), np.exp(th[5])
        assert np.all(var >= t2 * (1 - 1e-9)) and np.all(var <= (s2 + t2) * (1 + 1e-12))
        if prev is not None:  # nested conditioning sets: the conditional variance cannot grow
            assert np.all(var <= prev * (1 + 1e-10))
        prev = var


def test_prediction_draw_summaries_converge():
    """Draw summaries: with 40,000 draws the sample mean and variance are within
    a few standard errors of the mean and variance they were drawn from."""
    rng = np.random.default_rng(85)
    mean, var = rng.normal(size=50), rng.uniform(0.1, 2.0, 50)
    N = 40000
    xi = rng.standard_normal((N, 50))
    m, v, lo, hi = O.pred_draws(mean, var, xi)
    assert np.all(np.abs(m - mean) < 6 * np.sqrt(var / N))
    assert np.all(np.abs(v - var) < 6 * var * np.sqrt(2.0 / N))
    assert np.allclose(hi - lo, 2 * 1.959963984540054 * np.sqrt(v), rtol=1e-12)
