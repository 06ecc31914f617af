"""Larger measurements beyond the benchmark's default run.

    python -m paper_2504_12004_amd.experiments c2fits --out results/c2fits.json
    python -m paper_2504_12004_amd.experiments c3 --out results/c3.json
    python -m paper_2504_12004_amd.experiments c4 --out results/c4.json
    python -m paper_2504_12004_amd.experiments c5 --out results/c5.json
    python -m paper_2504_12004_amd.experiments accuracy --out results/accuracy.json

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


def c5(out_path, n_train=4096, n_val=512, n_app=20_000_000, epochs=200, nm_evals=100, stage="all",
       mlp_path=None, legs=None):
    """Learned warm start (paper_2504_12004_amd/warmstart.py).  Training:
    n_train datasets of n = 2e4 points in [0,1]^10, theta from the prior,
    observations from the simulator (1000 k-means blocks, m_gen = 100); 64
    summary statistics each; the 64-256-256-256-12 GELU network trained with
    Adam (lr 1e-3, batch 256) on all but n_val sets, early stopping.
    Application: a fresh dataset of n_app = 2e7 points (theta* from the prior,
    observations from the simulator on an independent generating structure,
    m_gen = 250 with blocks of at most 22 points); the warm start is the
    network's prediction with the nugget from the likelihood profile on a
    2e4-point subsample; one evaluation structure (m = 400, blocks of 5..60
    points, built at the warm start's ranges) is shared by every fit:
    FP32 L-BFGS with an FP64 polish from the warm and from the cold start,
    FP64 L-BFGS from the cold start, and plain FP64 Nelder-Mead from the cold
    start with an evaluation cap (nm_evals); every optimum is judged by one
    FP64 evaluation.  stage = "train" stops after saving the network
    (mlp_path), stage = "apply" loads it; legs selects fits by name."""
    import torch
    torch.cuda.init()
    from paper_2504_12004_amd import sbv, workloads
    from paper_2504_12004_amd import warmstart as W
    d, two_nu = 10, 5
    res = {}
    mlp_path = mlp_path or out_path + ".mlp"
    if stage in ("all", "train"):
        t0 = time.perf_counter()
        F, T = W.training_sets(n_train, 20000, d, seed=5, blocks=1000, m_gen=100, log=log)
        res["training_sets"], res["data_seconds"] = n_train, time.perf_counter() - t0
        t0 = time.perf_counter()
        mlp, ep = W.train(F, T, n_val, epochs=epochs)
        res["train_seconds"], res["epochs_kept"] = time.perf_counter() - t0, ep
        ntr = n_train - n_val
        pred = sbv.sbv_mlp_predict(mlp, F[ntr:])
        res["val_rmse_log_theta"] = np.sqrt(np.mean((pred - T[ntr:]) ** 2, axis=0)).tolist()
        res["val_rmse_mean_predictor"] = np.sqrt(np.mean((T[:ntr].mean(0) - T[ntr:]) ** 2, axis=0)).tolist()
        log(f"network: epoch {ep}, validation RMSE {np.round(res['val_rmse_log_theta'], 2)} vs mean predictor "
            f"{np.round(res['val_rmse_mean_predictor'], 2)}")
        sbv.sbv_mlp_save(mlp, mlp_path)
        if stage == "train":
            with open(out_path, "w") as f:
                json.dump(res, f, indent=1)
            return
    else:
        mlp = sbv.sbv_mlp_load(mlp_path, d + 2)
    dev = torch.device("cuda:0")
    ga = np.random.default_rng(6)
    X = ga.random((n_app, d))
    th_true = W.prior(ga, d)
    xi = ga.standard_normal(n_app)
    t0 = time.perf_counter()
    wgen = dict(seed=6, m_gen=250, gen_bs_mean=10, gen_max_bs=22)
    y = workloads.simulate(sbv, torch, dev, X, th_true, xi, two_nu, wgen).cpu().numpy()
    log(f"application observations simulated in {time.perf_counter() - t0:.0f} s")
    t0 = time.perf_counter()
    th_warm, th_net = W.predict(mlp, X, y, two_nu, sub_n=20000, seed=11)
    t_warm = time.perf_counter() - t0
    mlp.free()
    th_cold = W.cold_start(y, d)
    K = n_app // 20
    app = {"n": n_app, "K": K, "m": 400, "theta_true": th_true.tolist(), "theta_net": th_net.tolist(),
           "theta_warm": th_warm.tolist(), "theta_cold": th_cold.tolist(), "warm_start_seconds": t_warm,
           "warm_abs_err": np.abs(th_warm - th_true).tolist(), "cold_abs_err": np.abs(th_cold - th_true).tolist()}
    t0 = time.perf_counter()
    B = sbv.sbv_build_blocks(X, y, np.exp(th_warm[:d]), K, 400, method=sbv.SBV_KMEANS, lloyd_iters=2, min_bs=5,
                             max_bs=60, seed=8)
    app["build_seconds"] = time.perf_counter() - t0
    log(f"application structure: n = {n_app}, K = {B.K}, built in {app['build_seconds']:.1f} s")
    del X
    for prec in (sbv.SBV_FP32, sbv.SBV_FP64):
        sbv.sbv_autotune([B], th_warm, two_nu, prec, reps=1)
    app["loglik_fp64_at_true"] = float(sbv.sbv_loglik(B, th_true, two_nu)[0])
    all_legs = [("lbfgs_fp32_warm_polish64", sbv.SBV_LBFGS, sbv.SBV_FP32, True, th_warm, 400),
                ("lbfgs_fp32_cold_polish64", sbv.SBV_LBFGS, sbv.SBV_FP32, True, th_cold, 400),
                ("lbfgs_fp64_cold", sbv.SBV_LBFGS, sbv.SBV_FP64, False, th_cold, 400),
                ("nm_fp64_cold", sbv.SBV_NELDER_MEAD, sbv.SBV_FP64, False, th_cold, nm_evals)]
    fits = {}
    for name, opt, prec, polish, x0, me in all_legs:
        if legs and name not in legs:
            continue
        o = sbv.make_fit_opts(optimizer=opt, prec=prec, fp64_polish=polish, max_evals=me, ftol=1e-12,
                              gtol=1e-6 * n_app)
        log(f"fit {name}")
        th, l64, ne, sec, conv = sbv.sbv_fit(B, x0, two_nu, o)
        fits[name] = {"seconds": sec, "evals": ne, "loglik_fp64": l64, "converged": conv, "theta": th.tolist()}
        log(f"fit {name}: {sec:.1f} s, {ne} evals, l64 {l64:.6f}, converged {conv}")
    app["fits"] = fits
    res["application"] = app
    B.free()
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    log(f"wrote {out_path}")


def c3(out_path, reps=3):
    """Batched evaluation of 64 datasets (n_j in 5e4..4e5, d_j in {5, 10, 20},
    nu_j in {3/2, 5/2}, m_j in {100, 200, 400}, 20-point k-means blocks bounded
    to 5..60; y from the simulator on an independent structure with m_gen = 60).
    One evaluation of all 64 = one replay of the captured graph of the
    combined plan (size buckets shared across datasets, autotuned), against
    64 per-dataset evaluations queued one after the other on the same stream,
    in FP32 (FP64 accumulation, FP64 fallback) and in FP64."""
    import torch
    torch.cuda.init()
    from paper_2504_12004_amd import sbv, synth
    recipes = synth.multi_datasets(64, 3)
    hs, ths, tns = [], [], []
    t0 = time.perf_counter()
    for j, r in enumerate(recipes):
        X, xi = synth.inputs_for(r)
        th, d = r["theta"], r["d"]
        beta = np.exp(th[:d])
        Bg = sbv.sbv_build_blocks(X, None, beta, r["K"], 60, method=sbv.SBV_KMEANS, lloyd_iters=1,
                                  min_bs=r["min_bs"], max_bs=r["max_bs"], seed=r["seed"] + 7919)
        y = sbv.sbv_sample(Bg, th, r["two_nu"], xi)
        Bg.free()
        hs.append(sbv.sbv_build_blocks(X, y, beta, r["K"], r["m"], method=sbv.SBV_KMEANS, lloyd_iters=2,
                                       min_bs=r["min_bs"], max_bs=r["max_bs"], seed=r["seed"]))
        ths.append(th)
        tns.append(r["two_nu"])
        if (j + 1) % 8 == 0:
            log(f"datasets built: {j + 1}/64 ({time.perf_counter() - t0:.0f} s)")
    res = {"datasets": 64, "total_points": int(sum(r["n"] for r in recipes)),
           "build_seconds": time.perf_counter() - t0}
    flops, _ = sbv.sbv_plan_flops(hs, tns)
    res["algorithmic_tflop_per_eval"] = float(np.sum(flops)) / 1e12
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    th_all = torch.tensor(np.concatenate(ths), dtype=torch.float64, device=dev)
    offs = np.r_[0, np.cumsum([len(t) for t in ths])]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for name, prec in (("fp32", sbv.SBV_FP32), ("fp64", sbv.SBV_FP64)):
        out_b = torch.empty(64, dtype=torch.float64, device=dev)
        out_s = torch.empty(64, dtype=torch.float64, device=dev)

        def batched():
            sbv.sbv_eval_graph_dev(hs, th_all, tns, out_b, prec, stream=stream)

        def seq():
            for j in range(64):
                sbv.sbv_loglik_dev(hs[j], th_all[offs[j]:offs[j + 1]], tns[j], out_s[j:j + 1], prec, stream)
        # 1. the same kernel for every block in both runs (default variants):
        #    the batched values must equal the per-dataset ones bit for bit
        t_b0, t_s0 = timed(batched), timed(seq)
        ob, os_ = out_b.cpu().numpy(), out_s.cpu().numpy()
        bitwise = bool(np.array_equal(ob, os_))
        # 2. both autotuned (the combined plan and every per-dataset plan)
        tiles = sbv.sbv_autotune(hs, ths, tns, prec, reps=2)
        for j in range(64):
            sbv.sbv_autotune([hs[j]], [ths[j]], [tns[j]], prec, reps=2)
        t_b, t_s = timed(batched), timed(seq)
        ob2, os2 = out_b.cpu().numpy(), out_s.cpu().numpy()
        res[name] = {"default_variants": {"batched_graph_ms": t_b0, "sequential_ms": t_s0, "speedup": t_s0 / t_b0,
                                          "bitwise_equal": bitwise},
                     "autotuned": {"batched_graph_ms": t_b, "sequential_ms": t_s, "speedup": t_s / t_b,
                                   "max_rel_diff_batched_vs_sequential":
                                       float(np.max(np.abs(ob2 - os2) / np.abs(os2)))},
                     "batched_algorithmic_tflops": float(np.sum(flops)) / (t_b * 1e-3) / 1e12,
                     "autotuned_tiles": [int(t) for t in tiles]}
        log(f"{name}: default variants batched {t_b0:.1f} ms vs sequential {t_s0:.1f} ms (bitwise {bitwise}); "
            f"autotuned batched {t_b:.1f} ms vs sequential {t_s:.1f} ms, "
            f"{res[name]['batched_algorithmic_tflops']:.2f} TFLOP/s")
    for b in hs:
        b.free()
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    log(f"wrote {out_path}")


def c2fits(out_path, nm_evals=20000):
    """MLE fits on the n = 1e6, m = 200 benchmark workload (observations from
    the simulator on an independent generating structure, as in the
    benchmark), all from the cold start (beta_k = 1, sigma^2 = var(y),
    tau^2 = 1e-3 var(y)) on one shared structure built at the generating
    ranges: plain FP64 Nelder-Mead run to convergence (ftol 1e-10, up to
    nm_evals evaluations), FP32 Nelder-Mead with an FP64 polish, FP64 L-BFGS,
    FP32 L-BFGS with an FP64 polish.  Every optimum is judged by one FP64
    evaluation; the report gives wall times, evaluations, the FP64
    log-likelihood gap to the converged Nelder-Mead (nats and relative), and
    the distance of theta_hat from the generating theta."""
    import torch
    torch.cuda.init()
    from paper_2504_12004_amd import sbv, synth, workloads
    w = synth.dataset("uneven_1m")
    X, th_true, xi = w["X"], w["theta"], w["xi"]
    n, d = X.shape
    dev = torch.device("cuda:0")
    B = sbv.sbv_build_blocks(X, None, np.exp(th_true[:d]), w["K"], w["m"], method=sbv.SBV_KMEANS,
                             lloyd_iters=w["lloyd_iters"], min_bs=w["min_bs"], max_bs=w["max_bs"], seed=w["seed"])
    y = workloads.simulate(sbv, torch, dev, X, th_true, xi, w["two_nu"], w)
    sbv.sbv_blocks_set_y_dev(B, y)
    torch.cuda.synchronize()
    for prec in (sbv.SBV_FP64, sbv.SBV_FP32):
        sbv.sbv_autotune([B], th_true, w["two_nu"], prec, reps=3)
    var_y = float(torch.var(y).item())
    x0 = np.r_[np.zeros(d), np.log(var_y), np.log(1e-3 * var_y)]
    res = {"n": n, "K": B.K, "m": w["m"], "theta_true": th_true.tolist(), "theta_cold": x0.tolist(),
           "loglik_fp64_at_true": float(sbv.sbv_loglik(B, th_true, w["two_nu"])[0])}
    legs = [("nm_fp64", sbv.SBV_NELDER_MEAD, sbv.SBV_FP64, False, nm_evals, 1e-10),
            ("nm_fp32_polish64", sbv.SBV_NELDER_MEAD, sbv.SBV_FP32, True, nm_evals, 1e-10),
            ("lbfgs_fp64", sbv.SBV_LBFGS, sbv.SBV_FP64, False, 1000, 1e-12),
            ("lbfgs_fp32_polish64", sbv.SBV_LBFGS, sbv.SBV_FP32, True, 1000, 1e-12)]
    fits = {}
    for name, opt, prec, polish, me, ftol in legs:
        o = sbv.make_fit_opts(optimizer=opt, prec=prec, fp64_polish=polish, max_evals=me, ftol=ftol, gtol=1e-3,
                              init_step=0.5)
        log(f"fit {name}")
        th, l64, ne, sec, conv = sbv.sbv_fit(B, x0, w["two_nu"], o)
        fits[name] = {"seconds": sec, "evals": ne, "loglik_fp64": l64, "converged": conv, "theta": th.tolist(),
                      "max_abs_log_theta_err": float(np.max(np.abs(th - th_true)))}
        log(f"fit {name}: {sec:.2f} s, {ne} evals, l64 {l64:.6f}, converged {conv}, "
            f"max |theta - theta*| {fits[name]['max_abs_log_theta_err']:.3f}")
    base = fits["nm_fp64"]["loglik_fp64"]
    for k in fits:
        fits[k]["gap_nats_vs_nm_fp64"] = fits[k]["loglik_fp64"] - base
        fits[k]["rel_gap_vs_nm_fp64"] = (fits[k]["loglik_fp64"] - base) / abs(base)
        fits[k]["speedup_vs_nm_fp64"] = fits["nm_fp64"]["seconds"] / fits[k]["seconds"]
    res["fits"] = fits
    B.free()
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    log(f"wrote {out_path}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["c2fits", "c3", "c4", "c5", "accuracy"])
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--no-fits", action="store_true")
    ap.add_argument("--train-sets", type=int, default=4096)
    ap.add_argument("--app-n", type=int, default=20_000_000)
    ap.add_argument("--stage", choices=["all", "train", "apply"], default="all")
    ap.add_argument("--mlp", default=None)
    ap.add_argument("--legs", default=None, help="comma-separated fit names (C5)")
    a = ap.parse_args()
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    if a.what == "c4":
        c4(a.out, a.reps, not a.no_fits)
    elif a.what == "c3":
        c3(a.out, a.reps)
    elif a.what == "c5":
        c5(a.out, n_train=a.train_sets, n_app=a.app_n, stage=a.stage, mlp_path=a.mlp,
           legs=a.legs.split(",") if a.legs else None)
    elif a.what == "c2fits":
        c2fits(a.out)
    elif a.what == "accuracy":
        from . import accuracy
        accuracy.study(a.out)


if __name__ == "__main__":
    main()
