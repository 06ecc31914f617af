"""Learned warm start for the MLE (the network is the library's own FP32 MLP
with device training and inference kernels).

  1. training data: datasets simulated by the library itself (inputs uniform on
     [0,1]^d, theta from the prior below, observations from the Vecchia
     conditional simulator), each summarised by sbv_features;
  2. the network maps the summary statistics to log theta (standardised inputs
     and targets, Adam, early stopping on held-out sets);
  3. for a new dataset the network's prediction is completed by a nugget
     profile on the same 2e4-point subsample the features use: the library's
     SBV log-likelihood at the predicted ranges and variance over a grid of
     log tau^2, refined by a parabola through the best three grid points.  The
     summary statistics carry little information on the nugget (it only
     shows at distances below the nearest-neighbour spacing of a 2e4-point
     sample in 10 dimensions), the likelihood does.

The prior: beta_k ~ logU[0.05, 3], sigma^2 ~ logU[0.5, 2], tau^2 ~ logU[1e-6, 1e-2],
nu = 5/2; the cold start the warm start is compared with: beta_k = 1,
sigma^2 = var(y), tau^2 = 1e-3 var(y).
"""
import time

import numpy as np

from . import sbv, synth


def prior(g, d):
    beta = synth.log_uniform(g, 0.05, 3.0, d)
    return synth.theta_vector(beta, synth.log_uniform(g, 0.5, 2.0), synth.log_uniform(g, 1e-6, 1e-2))


def cold_start(y, d):
    v = float(np.var(y))
    return np.r_[np.zeros(d), np.log(v), np.log(1e-3 * v)]


def training_sets(n_sets, n_pts, d, seed, two_nu=5, blocks=None, m_gen=100, log=None):
    """Summary statistics and log theta of n_sets simulated datasets."""
    g = np.random.default_rng(seed)
    nf = 4 + 5 * (d + 2)
    feats = np.empty((n_sets, nf), np.float32)
    targ = np.empty((n_sets, d + 2), np.float32)
    K = blocks or max(1, n_pts // 20)
    t0 = time.perf_counter()
    for j in range(n_sets):
        X = g.random((n_pts, d))
        th = prior(g, d)
        xi = g.standard_normal(n_pts)
        Bg = sbv.sbv_build_blocks(X, None, np.exp(th[:d]), K, m_gen, method=sbv.SBV_KMEANS, lloyd_iters=1,
                                  seed=1000003 + j + seed * 7919)
        y = sbv.sbv_sample(Bg, th, two_nu, xi)
        Bg.free()
        feats[j] = sbv.sbv_features(X, y, min(n_pts, 20000), seed=j)
        targ[j] = th
        if log and (j + 1) % 256 == 0:
            log(f"training sets: {j + 1}/{n_sets} ({time.perf_counter() - t0:.0f} s)")
    return feats, targ


def train(feats, targ, n_val, epochs=200, seed=5, hidden=256, layers=3):
    """The 64-256-256-256-12 GELU network trained on all but the last n_val
    sets; the parameters with the lowest validation error are kept."""
    ntr = len(feats) - n_val
    mlp = sbv.sbv_mlp_create(feats.shape[1], hidden, layers, targ.shape[1], seed=seed)
    best, best_p, best_ep = np.inf, None, 0
    for ep in range(10, epochs + 1, 10):
        sbv.sbv_mlp_train(mlp, feats[:ntr], targ[:ntr], 10, batch=256, lr=1e-3, seed=seed + ep)
        err = float(np.mean((sbv.sbv_mlp_predict(mlp, feats[ntr:]) - targ[ntr:]) ** 2))
        if err < best:
            best, best_p, best_ep = err, sbv.sbv_mlp_get_params(mlp), ep
    sbv.sbv_mlp_set_params(mlp, best_p)
    return mlp, best_ep


def refine_nugget(X, y, theta, two_nu, sub_n=20000, seed=11, m=60, grid=None):
    """Nugget profile on a subsample: log tau^2 over a grid (default 13 values
    from log(1e-7 var y) to log(1e-1 var y)) at theta's ranges and variance,
    the best point refined by the parabola through it and its neighbours."""
    n, d = X.shape
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, size=min(n, sub_n), replace=False))
    Xs, ys = X[idx], y[idx]
    v = float(np.var(ys))
    if grid is None:
        grid = np.linspace(np.log(1e-7 * v), np.log(1e-1 * v), 13)
    B = sbv.sbv_build_blocks(Xs, ys, np.exp(theta[:d]), max(1, len(idx) // 20), m, method=sbv.SBV_KMEANS,
                             lloyd_iters=2, seed=seed)
    ll = []
    for gv in grid:
        t = theta.copy()
        t[d + 1] = gv
        try:
            ll.append(sbv.sbv_loglik(B, t, two_nu)[0])
        except sbv.SBVError:
            ll.append(-np.inf)
    B.free()
    ll = np.array(ll)
    i = int(np.argmax(ll))
    best = grid[i]
    if 0 < i < len(grid) - 1 and np.all(np.isfinite(ll[i - 1:i + 2])):
        a, b, c = ll[i - 1], ll[i], ll[i + 1]
        den = a - 2 * b + c
        if den < 0:
            best = grid[i] + 0.5 * (grid[1] - grid[0]) * (a - c) / den
    out = theta.copy()
    out[d + 1] = best
    return out


def predict(mlp, X, y, two_nu, sub_n=20000, seed=11):
    """Warm start for one dataset: the network's prediction from the summary
    statistics, with the nugget from the likelihood profile."""
    d = X.shape[1]
    f = sbv.sbv_features(X, y, sub_n, seed=seed)
    th = sbv.sbv_mlp_predict(mlp, f[None, :].astype(np.float32))[0].astype(np.float64)
    return refine_nugget(X, y, th, two_nu, sub_n=sub_n, seed=seed), th
