"""Larger measurements beyond the benchmark's default run.

    python -m paper_2504_12004_amd.experiments c4 --out results/c4.json

c4: n = 5e6, d = 10, Matern-5/2, 250,000 k-means blocks of 5..60 points,
m = 400 (joint sets up to 460, the large path).  Observations from the
Vecchia conditional simulator on an independent generating structure
(m_gen = 200, the simulator's joint-size limit being 272).  Reports
log-likelihood and log-likelihood + gradient evaluations per second in FP64
and FP32, the gradient against central differences of the GPU value at the
generating theta (h = 1e-5, 24 extra evaluations), and L-BFGS fits from the
cold start (beta_k = 1, sigma^2 = var(y), tau^2 = 1e-3 var(y)) in FP64 and in
FP32 with an FP64 polish, each judged by one FP64 evaluation.

Every step prints a progress line; fits rewrite a checkpoint file per
iteration next to the output.
"""
import argparse
import json
import os
import time

import numpy as np


def log(*a):
    print("[exp]", *a, flush=True)


def _rates(sbv, B, theta, two_nu, reps):
    out = {}
    for name, prec in (("fp64", sbv.SBV_FP64), ("fp32", sbv.SBV_FP32)):
        sbv.sbv_loglik(B, theta, two_nu, prec)
        t0 = time.perf_counter()
        for _ in range(reps):
            sbv.sbv_loglik(B, theta, two_nu, prec)
        tl = (time.perf_counter() - t0) / reps
        sbv.sbv_loglik_grad(B, theta, two_nu, prec)
        t0 = time.perf_counter()
        for _ in range(reps):
            l, g = sbv.sbv_loglik_grad(B, theta, two_nu, prec)
        tg = (time.perf_counter() - t0) / reps
        out[name] = {"loglik_evals_per_s": 1.0 / tl, "loglik_grad_evals_per_s": 1.0 / tg,
                     "loglik_ms": 1e3 * tl, "loglik_grad_ms": 1e3 * tg,
                     "fallback_blocks": int(sbv.sbv_blocks_fallback_count(B)) if prec == sbv.SBV_FP32 else 0}
        log(f"{name}: loglik {1e3 * tl:.1f} ms, loglik+grad {1e3 * tg:.1f} ms")
    return out


def _fd_check(sbv, B, theta, two_nu, h=1e-5):
    l0, g = sbv.sbv_loglik_grad(B, theta, two_nu, sbv.SBV_FP64)
    fd = np.empty_like(g)
    for k in range(len(theta)):
        e = np.zeros_like(theta)
        e[k] = h
        lp = sbv.sbv_loglik(B, theta + e, two_nu)[0]
        lm = sbv.sbv_loglik(B, theta - e, two_nu)[0]
        fd[k] = (lp - lm) / (2 * h)
    err = np.abs(g - fd) / np.maximum(np.abs(g), 1.0)
    noise = 10 * np.finfo(float).eps * abs(l0[0]) / h
    log(f"gradient vs central differences: max rel err {err.max():.2e} (FD noise ~{noise:.1e})")
    return {"h": h, "grad": g.tolist(), "fd": fd.tolist(), "max_rel_err": float(err.max()),
            "fd_noise_abs": noise}


def _fits(sbv, B, x0, two_nu, n, ckpt):
    out = {}
    legs = [("lbfgs_fp64", sbv.SBV_FP64, False), ("lbfgs_fp32_polish64", sbv.SBV_FP32, True)]
    for name, prec, polish in legs:
        if os.path.exists(ckpt):
            os.remove(ckpt)
        o = sbv.make_fit_opts(optimizer=sbv.SBV_LBFGS, prec=prec, fp64_polish=polish, max_evals=400, ftol=1e-12,
                              gtol=1e-6 * n, checkpoint_path=ckpt)
        log(f"fit {name} from the cold start")
        th, l64, ne, sec, conv = sbv.sbv_fit(B, x0, two_nu, o)
        out[name] = {"seconds": sec, "evals": ne, "loglik_fp64": l64, "converged": conv, "theta": th.tolist()}
        log(f"fit {name}: {sec:.1f} s, {ne} evals, l64 {l64:.6f}, converged {conv}")
    if os.path.exists(ckpt):
        os.remove(ckpt)
    a, b = out["lbfgs_fp64"]["loglik_fp64"], out["lbfgs_fp32_polish64"]["loglik_fp64"]
    out["rel_gap_fp32_vs_fp64"] = (b - a) / abs(a)
    return out


def c4(out_path, reps=3, fits=True):
    import torch  # the HIP runtime bundled with torch must load first
    torch.cuda.init()
    from paper_2504_12004_amd import sbv, synth
    w = synth.dataset("grad_5m")
    X, theta, xi = w["X"], w["theta"], w["xi"]
    n, d = X.shape
    two_nu = w["two_nu"]
    beta = np.exp(theta[:d])
    res = {"workload": "c4: n=5e6 d=10 Matern-5/2 tau2=1e-4 kmeans K=2.5e5 (5..60) m=400", "n": n}
    t0 = time.perf_counter()
    Bg = sbv.sbv_build_blocks(X, None, beta, w["K"], 200, method=sbv.SBV_KMEANS, lloyd_iters=1,
                              min_bs=w["min_bs"], max_bs=w["max_bs"], seed=w["seed"] + 7919)
    log(f"generating structure built in {time.perf_counter() - t0:.1f} s")
    y = sbv.sbv_sample(Bg, theta, two_nu, xi)
    Bg.free()
    log("observations simulated")
    t0 = time.perf_counter()
    B = sbv.sbv_build_blocks(X, y, beta, w["K"], w["m"], method=sbv.SBV_KMEANS, lloyd_iters=w["lloyd_iters"],
                             min_bs=w["min_bs"], max_bs=w["max_bs"], seed=w["seed"])
    res["build_seconds"] = time.perf_counter() - t0
    log(f"evaluation structure built in {res['build_seconds']:.1f} s, K = {B.K}")
    flops, _ = sbv.sbv_plan_flops(B, two_nu)
    res["algorithmic_tflop_per_eval"] = float(np.sum(flops)) / 1e12
    res["rates"] = _rates(sbv, B, theta, two_nu, reps)
    res["loglik_at_theta"] = float(sbv.sbv_loglik(B, theta, two_nu)[0])
    res["fd"] = _fd_check(sbv, B, theta, two_nu)
    if fits:
        var_y = float(np.var(y))
        x0 = np.r_[np.zeros(d), np.log(var_y), np.log(1e-3 * var_y)]
        res["fits"] = _fits(sbv, B, x0, two_nu, n, out_path + ".ckpt")
    B.free()
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    log(f"wrote {out_path}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["c4"])
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--no-fits", action="store_true")
    a = ap.parse_args()
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    if a.what == "c4":
        c4(a.out, a.reps, not a.no_fits)


if __name__ == "__main__":
    main()
