"""Accuracy study of Sec. 7.1 (synthetic data simulation) on the GPU.

    python -m paper_2504_12004_amd.accuracy --out results/accuracy.json

Data: inputs uniform on [0,1]^10, a zero-mean GP with the Matern kernel at
nu = 7/2, sigma^2 = 1, ranges 0.05 for the two relevant dimensions and 5 for
the eight others; observations of n training and n_test test points drawn
jointly and exactly (dense covariance from the library's covariance kernel,
Cholesky factor from torch on the device; data generation, not the method).
The nugget is 1e-6 instead of the paper's 0: without it the dense factor of
this very smooth kernel is numerically singular.

Four Vecchia settings at the true parameters, as in the paper's comparison:
  CV   blocks of one point, neighbours by unscaled distance
  BV   blocks of bs = 10 points (k-means), unscaled
  SV   blocks of one point, inputs scaled by the ranges before ordering,
       clustering and neighbour search
  SBV  blocks of bs = 10 points, scaled
For each conditioning size m the study reports
  - the KL divergence of Eq. (kldivergence), exact minus approximate
    log-likelihood at y = 0 (the exact one from the dense factor);
  - the mean squared prediction error of the predictive means at the test
    points (prediction blocks of the method's block size, m_pred = m);
then KL of SBV for block sizes 12, 25 and 50, and the relative error of the
log-likelihood at the observed y against the exact one for k-means and for
random anchor clustering (RAC) over five anchor seeds.
"""
import argparse
import json
import math
import os
import time

import numpy as np


def log(*a):
    print("[acc]", *a, flush=True)


def _draw(sbv, torch, dev, n_all, d, theta, two_nu, seed):
    from . import synth
    g = synth.rng(seed)
    X = g.random((n_all, d))
    z = g.standard_normal(n_all)
    Xd = torch.tensor(X, dtype=torch.float64, device=dev)
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    S = torch.empty((n_all, n_all), dtype=torch.float64, device=dev)
    sbv.sbv_cov_matrix_dev(Xd, Xd, th, two_nu, S, same=True)
    L = torch.linalg.cholesky(S)
    del S
    y = (L @ torch.tensor(z, dtype=torch.float64, device=dev)).cpu().numpy()
    return X, y, L


def _exact_terms(torch, L, y, n):
    """Exact log-likelihood of the first n points (Eq. (1)) at y and at y = 0
    from the leading block of the joint Cholesky factor."""
    Ln = L[:n, :n]
    logdet = 2.0 * torch.log(torch.diagonal(Ln)).sum().item()
    w = torch.linalg.solve_triangular(Ln, torch.tensor(y[:n], dtype=torch.float64, device=L.device)[:, None],
                                      upper=False)
    q = float((w * w).sum().item())
    c = n * math.log(2 * math.pi)
    return -0.5 * (q + logdet + c), -0.5 * (logdet + c)


SETTINGS = {  # name: (block size, scaled)
    "CV": (1, False),
    "BV": (10, False),
    "SV": (1, True),
    "SBV": (10, True),
}


def study(out_path, n=10000, n_test=1000, ms=(10, 20, 30, 40, 60), seed=11, bs_sweep=(12, 25, 50),
          rac_seeds=5):
    import torch

    from . import sbv

    dev = torch.device("cuda:0")
    d, two_nu = 10, 7
    beta = np.r_[0.05, 0.05, np.full(8, 5.0)]
    theta = np.r_[np.log(beta), 0.0, np.log(1e-6)]
    t0 = time.perf_counter()
    X_all, y_all, L = _draw(sbv, torch, dev, n + n_test, d, theta, two_nu, seed)
    X, y, Xt, yt = X_all[:n], y_all[:n], X_all[n:], y_all[n:]
    l_exact, l0_exact = _exact_terms(torch, L, y_all, n)
    del L
    torch.cuda.empty_cache()
    log(f"data n={n} n_test={n_test} drawn in {time.perf_counter() - t0:.1f}s; exact l = {l_exact:.6f}")
    res = {"config": {"n": n, "n_test": n_test, "d": d, "nu": 3.5, "beta": beta.tolist(), "sigma2": 1.0,
                      "tau2": 1e-6, "ms": list(ms), "seed": seed},
           "exact_loglik": l_exact, "exact_loglik_y0": l0_exact, "kl": {}, "mspe": {}, "bs_kl": {},
           "rac_vs_kmeans": {}}
    zeros = np.zeros(n)

    def build(bs, scaled, m, method=sbv.SBV_KMEANS, aseed=seed):
        bb = beta if scaled else np.ones(d)
        return sbv.sbv_build_blocks(X, y, bb, n // bs, m, method=method,
                                    lloyd_iters=0 if method == sbv.SBV_RAC else 5, seed=aseed), bb

    for name, (bs, scaled) in SETTINGS.items():
        res["kl"][name], res["mspe"][name] = [], []
        for m in ms:
            B, bb = build(bs, scaled, m)
            ly = sbv.sbv_loglik(B, theta, two_nu)[0]
            sbv.sbv_blocks_set_y(B, zeros)
            l0 = sbv.sbv_loglik(B, theta, two_nu)[0]
            sbv.sbv_blocks_set_y(B, y)
            P = sbv.sbv_pred_build(B, Xt, bb, n_test // bs, m, lloyd_iters=5, seed=seed)
            mu, _ = sbv.sbv_predict(P, theta, two_nu)
            mspe = float(np.mean((mu - yt) ** 2))
            res["kl"][name].append(l0_exact - l0)
            res["mspe"][name].append(mspe)
            log(f"{name} m={m}: KL {l0_exact - l0:.4f}, MSPE {mspe:.6f}, l(y) {ly:.4f}")
            P.free()
            B.free()
    for bs in bs_sweep:
        res["bs_kl"][str(bs)] = []
        for m in ms:
            B, _ = build(bs, True, m)
            sbv.sbv_blocks_set_y(B, zeros)
            kl = l0_exact - sbv.sbv_loglik(B, theta, two_nu)[0]
            res["bs_kl"][str(bs)].append(kl)
            log(f"SBV bs={bs} m={m}: KL {kl:.4f}")
            B.free()
    for m in ms:
        B, _ = build(10, True, m)
        km = abs(sbv.sbv_loglik(B, theta, two_nu)[0] - l_exact) / abs(l_exact)
        B.free()
        rac = []
        for s in range(rac_seeds):
            B, _ = build(10, True, m, method=sbv.SBV_RAC, aseed=seed + 100 + s)
            rac.append(abs(sbv.sbv_loglik(B, theta, two_nu)[0] - l_exact) / abs(l_exact))
            B.free()
        res["rac_vs_kmeans"][str(m)] = {"kmeans_rel_err": km, "rac_rel_err_mean": float(np.mean(rac)),
                                        "rac_rel_err_sd": float(np.std(rac, ddof=1))}
        log(f"m={m}: k-means rel err {km:.3e}, RAC {np.mean(rac):.3e} +- {np.std(rac, ddof=1):.1e}")
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    log(f"wrote {out_path}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--n-test", type=int, default=1000)
    a = ap.parse_args()
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    study(a.out, n=a.n, n_test=a.n_test)


if __name__ == "__main__":
    main()
