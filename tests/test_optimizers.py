"""The MLE driver's optimisers (host code of libsbv.so), run on the CPU through
sbv_minimize: textbook test functions, an MLE with the oracle as objective,
and checkpoint/resume following the uninterrupted trajectory exactly."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2504_12004_amd import sbv
from paper_2504_12004_amd import synth


def rosen(x, want_grad):
    f = np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1 - x[:-1]) ** 2)
    if not want_grad:
        return f
    g = np.zeros_like(x)
    g[:-1] = -400.0 * x[:-1] * (x[1:] - x[:-1] ** 2) - 2 * (1 - x[:-1])
    g[1:] += 200.0 * (x[1:] - x[:-1] ** 2)
    return f, g


@pytest.mark.parametrize("n", [2, 5])
def test_lbfgs_rosenbrock(n):
    o = sbv.make_fit_opts(optimizer=sbv.SBV_LBFGS, max_evals=2000, ftol=0.0, gtol=1e-9)
    x, f, ne, conv = sbv.sbv_minimize(sbv.SBV_LBFGS, -np.ones(n) * 1.2, rosen, o)
    assert conv and np.max(np.abs(x - 1)) < 1e-6, (x, ne)


def test_nelder_mead_rosenbrock():
    o = sbv.make_fit_opts(optimizer=sbv.SBV_NELDER_MEAD, max_evals=5000, ftol=1e-14, init_step=0.5)
    x, f, ne, conv = sbv.sbv_minimize(sbv.SBV_NELDER_MEAD, np.array([-1.2, 1.0]), rosen, o)
    assert conv and np.max(np.abs(x - 1)) < 1e-4, (x, ne)


def _mle_problem():
    X, th, xi = synth.random_spd_problem(400, 3, seed=61, beta=[0.3, 0.6, 1.2], sigma2=1.3, tau2=1e-2)
    S = O.build(X, np.exp(th[:3]), K=40, m=20, seed=2)
    y = O.sample(X, O.build(X, np.exp(th[:3]), K=40, m=400, seed=5), th, 5, xi)

    def negll(t, want_grad):
        if want_grad:
            ll, g = O.sbv_loglik(X, y, S, t, 5, grad=True)
            return (-ll if np.isfinite(ll) else np.inf), -g
        ll = O.sbv_loglik(X, y, S, t, 5)
        return -ll if np.isfinite(ll) else np.inf
    return th, negll


def test_mle_with_oracle_objective_agrees_between_optimisers():
    th, negll = _mle_problem()
    x0 = th + 0.3
    ol = sbv.make_fit_opts(optimizer=sbv.SBV_LBFGS, max_evals=400, ftol=1e-13, gtol=1e-7)
    xl, fl, nl, cl = sbv.sbv_minimize(sbv.SBV_LBFGS, x0, negll, ol)
    on = sbv.make_fit_opts(optimizer=sbv.SBV_NELDER_MEAD, max_evals=4000, ftol=1e-12, init_step=0.3)
    xn, fn, nn, cn = sbv.sbv_minimize(sbv.SBV_NELDER_MEAD, x0, negll, on)
    assert cl and cn
    assert abs(fl - fn) <= 1e-6 * abs(fl)
    _, g = negll(xl, True)
    assert np.max(np.abs(g)) < 1e-4


@pytest.mark.parametrize("method", [sbv.SBV_LBFGS, sbv.SBV_NELDER_MEAD])
def test_checkpoint_resume_follows_the_same_trajectory(tmp_path, method):
    th, negll = _mle_problem()
    x0 = th + 0.25
    full = sbv.make_fit_opts(optimizer=method, max_evals=150, ftol=1e-13, gtol=1e-7)
    xa, fa, na, _ = sbv.sbv_minimize(method, x0, negll, full)
    ck = str(tmp_path / "state.json")
    part = sbv.make_fit_opts(optimizer=method, max_evals=40, ftol=1e-13, gtol=1e-7, checkpoint_path=ck)
    sbv.sbv_minimize(method, x0, negll, part)
    assert os.path.exists(ck)
    rest = sbv.make_fit_opts(optimizer=method, max_evals=150, ftol=1e-13, gtol=1e-7, checkpoint_path=ck)
    xb, fb, nb, _ = sbv.sbv_minimize(method, x0, negll, rest)
    assert np.array_equal(xa, xb) and fa == fb


@pytest.mark.parametrize("method", [sbv.SBV_LBFGS, sbv.SBV_NELDER_MEAD])
def test_non_finite_objective_is_backed_away_from(method):
    """An objective that is +inf (or NaN) outside its domain, as the
    log-likelihood is at a point where a block is not positive definite:
    both optimisers treat such points as worse than any finite value and still
    reach the minimum inside the domain (the first L-BFGS step from x0 = 0
    overshoots the boundary just past the minimum)."""
    calls = {"bad": 0}

    def f(x, want_grad):
        if x[0] > 0.9 or x[1] < -1.0:
            calls["bad"] += 1
            v = np.inf if x[0] > 0.9 else np.nan
            return (v, np.zeros(2)) if want_grad else v
        v = 1.0 + 100.0 * (x[0] - 0.85) ** 2 + (x[1] - 0.5) ** 2
        if want_grad:
            return v, np.array([200.0 * (x[0] - 0.85), 2.0 * (x[1] - 0.5)])
        return v
    o = sbv.make_fit_opts(optimizer=method, max_evals=3000, ftol=1e-13, gtol=1e-9, init_step=4.0)
    x, fb, ne, conv = sbv.sbv_minimize(method, np.zeros(2), f, o)
    assert conv and calls["bad"] > 0 and abs(fb - 1.0) < 1e-9
    assert np.max(np.abs(x - [0.85, 0.5])) < 1e-5, x
