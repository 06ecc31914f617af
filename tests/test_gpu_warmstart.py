"""What the learned warm start gains: a network trained on datasets the
library simulates (its own training kernels) predicts log theta from summary
statistics; completed by the nugget profile, its prediction starts the FP64
L-BFGS MLE of fresh datasets, which then needs fewer objective evaluations
in total than the same fits from the cold start, at the same optimum."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_needs_fewer_evaluations_than_the_cold_start():
    from paper_2504_12004_amd import sbv
    from paper_2504_12004_amd import warmstart as W
    d = 10
    F, T = W.training_sets(512, 3000, d, seed=1, blocks=150, m_gen=100)
    mlp, _ = W.train(F, T, 64, epochs=200)
    # the network beats the mean predictor on the ranges and the variance
    pred = sbv.sbv_mlp_predict(mlp, F[-64:])
    rmse = np.sqrt(np.mean((pred - T[-64:]) ** 2, axis=0))
    base = np.sqrt(np.mean((T[:-64].mean(0) - T[-64:]) ** 2, axis=0))
    print("validation RMSE", rmse.round(2), "mean predictor", base.round(2), flush=True)
    assert np.all(rmse[:d + 1] < base[:d + 1])
    g = np.random.default_rng(99)
    evals = {"cold": 0, "warm": 0}
    o = sbv.make_fit_opts(optimizer=sbv.SBV_LBFGS, max_evals=2000, ftol=1e-12, gtol=1e-5)
    for k in range(6):
        n = 5000
        X = g.random((n, d))
        th = W.prior(g, d)
        xi = g.standard_normal(n)
        Bg = sbv.sbv_build_blocks(X, None, np.exp(th[:d]), 250, 120, lloyd_iters=1, seed=500 + k)
        y = sbv.sbv_sample(Bg, th, 5, xi)
        Bg.free()
        warm, _ = W.predict(mlp, X, y, 5, sub_n=n, seed=k)
        B = sbv.sbv_build_blocks(X, y, np.exp(th[:d]), 250, 60, lloyd_iters=2, min_bs=5, max_bs=40, seed=7 + k)
        out = {}
        for name, x0 in (("cold", W.cold_start(y, d)), ("warm", warm)):
            t, l64, ne, sec, conv = sbv.sbv_fit(B, x0, 5, o)
            assert conv
            out[name] = l64
            evals[name] += ne
        print(k, out, flush=True)
        assert abs(out["warm"] - out["cold"]) <= 1e-6 * abs(out["cold"])  # the same optimum
        B.free()
    print(evals, flush=True)
    assert evals["warm"] < evals["cold"]
    mlp.free()
