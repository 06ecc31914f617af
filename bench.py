"""Benchmark of the SBV log-likelihood hot path on one MI355X.

Workload (the headline configuration): n = 1,000,000 inputs uniform on
[0,1]^10, Matern-5/2, ranges log-uniform on [0.05, 3], sigma^2 = 1,
tau^2 = 1e-4; k-means into 50,000 blocks bounded to 5..60 points; m = 200
nearest earlier neighbours; evaluations at perturbed parameters
theta_t = theta* + 0.1 N(0, I).  The structure is built once on the GPU
(sbv_build_blocks) and stays resident; the timed region holds only
log-likelihood evaluations with parameters and results already in HBM.

One step = one FP64 log-likelihood evaluation of the whole dataset (all
blocks: covariance build, factorisation, solves, log-det/quadratic-form,
reduction).  The same line also reports the FP32 path (FP32 covariance and
Cholesky, FP64 accumulation, FP64 re-run of low-pivot blocks) and the
log-likelihood + gradient path when available.

Prints ONE JSON line.  Only --gpus 1 is supported (one GPU per box).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12  # MI355X dense FP64 (vector = matrix), FLOP/s
PEAK_FP32 = 157.3e12


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="override n (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM byte counters)")
    ap.add_argument("--fit-evals", type=int, default=300,
                    help="evaluation budget of each MLE fit leg (0 skips the fits)")
    ap.add_argument("--large-steps", type=int, default=3,
                    help="evaluations of the m = 400, n = 5e6 leg per precision (0 skips it)")
    ap.add_argument("--traffic-json", default=None,
                    help="JSON with measured per-launch HBM bytes of the dominant kernel")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library and this benchmark run on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2504_12004_amd import sbv, synth, workloads

    dev = torch.device("cuda:0")
    torch.cuda.init()
    w = synth.dataset("uneven_1m", n=args.n)
    X, theta_true, xi = w["X"], w["theta"], w["xi"]
    n, d = X.shape
    K = w["K"] if args.n is None else max(1, args.n // 20)
    m = w["m"]
    two_nu = w["two_nu"]
    bb = np.exp(theta_true[:d])

    t0 = time.perf_counter()
    B = sbv.sbv_build_blocks(X, None, bb, K, m, method=sbv.SBV_KMEANS, lloyd_iters=w["lloyd_iters"],
                             min_bs=w["min_bs"], max_bs=w["max_bs"], seed=w["seed"])
    t_build = time.perf_counter() - t0
    log(f"built structure: n={n} K={B.K} nnz={B.nnz} in {t_build:.2f}s")
    # observations: the device Vecchia simulator at the true parameters on an
    # independent generating structure (own seed, m_gen >= m)
    t0 = time.perf_counter()
    y_d = workloads.simulate(sbv, torch, dev, X, theta_true, xi, two_nu, w)
    sbv.sbv_blocks_set_y_dev(B, y_d)
    torch.cuda.synchronize()
    y_host = y_d.cpu().numpy()
    y_source = (f"vecchia-sampler, generating structure m_gen={w['m_gen']} "
                f"K_gen={n // w['gen_bs_mean']} blocks<={w['gen_max_bs']}")
    log(f"simulated observations in {time.perf_counter() - t0:.2f}s")

    # per size bucket, pick the fastest kernel variant and schedule (setup, not timed)
    tuned, sched, pers_choice = {}, {}, {}
    for name, prec in (("fp64", sbv.SBV_FP64), ("fp32", sbv.SBV_FP32)):
        ch, la, wv, pc = sbv.sbv_autotune([B], theta_true, two_nu, prec, reps=3, with_schedule=True)
        tuned[name] = [int(t) for t in ch]
        sched[name] = [("lookahead" if x else "plain") + f"/{int(v)} waves per CU" for x, v in zip(la, wv)]
        pers_choice[name] = "persistent single launch" if pc else "one launch per size bucket"
    log(f"autotuned tiles per bucket: {tuned}, schedules {sched}")

    thetas = synth.perturbed_thetas(theta_true, w["n_theta"], w["theta_seed"])
    th_d = torch.tensor(thetas, dtype=torch.float64, device=dev)
    out = torch.empty(max(args.steps, 1) + args.warmup + 8, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def run(prec, steps, warm, timing):
        for i in range(warm):
            sbv.sbv_loglik_dev(B, th_d[i % len(thetas)], two_nu, out[i:i + 1], prec, stream)
        torch.cuda.synchronize()
        sbv.sbv_timing_enable(timing)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(steps):
            sbv.sbv_loglik_dev(B, th_d[i % len(thetas)], two_nu, out[i:i + 1], prec, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        kt = sbv.sbv_timing_read(prec) if timing else None
        sbv.sbv_timing_enable(False)
        return ms, kt, out[:steps].cpu().numpy()

    # headline: FP64, timed without per-kernel events
    ms64, _, ll64 = run(sbv.SBV_FP64, args.steps, args.warmup, False)
    ms_step = ms64 / args.steps
    log(f"FP64: {ms_step:.3f} ms/eval")
    # per-kernel live timing of the same workload (separate pass, events on the launch stream)
    kin = min(args.steps, 20)
    _, kt64, _ = run(sbv.SBV_FP64, kin, 1, True)
    ms32, kt32, ll32 = run(sbv.SBV_FP32, kin, 1, True)
    fb = sbv.sbv_blocks_fallback_count(B)
    rel32 = float(np.max(np.abs(ll32[:kin] - ll64[:kin]) / np.abs(ll64[:kin])))
    log(f"FP32: {ms32 / kin:.3f} ms/eval, max rel diff vs FP64 {rel32:.2e}, fallback blocks {fb}")

    flops, tiles = sbv.sbv_plan_flops(B, two_nu)
    ms_tot, launches = kt64
    v_dom = int(np.argmax(ms_tot))
    avg_ms = ms_tot[v_dom] / max(launches[v_dom], 1)
    achieved = flops[v_dom] / (avg_ms * 1e-3)
    total_flop = float(np.sum(flops))
    log(f"dominant kernel: variant with {tiles[v_dom]} tiles, {avg_ms:.3f} ms/launch, "
        f"{achieved / 1e12:.2f} TFLOP/s algorithmic")

    grad_rate = {}
    g_d = torch.empty(d + 2, dtype=torch.float64, device=dev)
    for name, prec in (("fp64", sbv.SBV_FP64), ("fp32", sbv.SBV_FP32)):
        for i in range(2):
            sbv.sbv_loglik_grad_dev(B, th_d[i], two_nu, out[i:i + 1], g_d, prec, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(kin):
            sbv.sbv_loglik_grad_dev(B, th_d[i % len(thetas)], two_nu, out[i:i + 1], g_d, prec, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        grad_rate[name] = 1000.0 * kin / e0.elapsed_time(e1)
    log(f"loglik + gradient: {grad_rate['fp64']:.2f} evals/s FP64, {grad_rate['fp32']:.2f} evals/s FP32")

    # both launch modes timed explicitly (the autotuner's choice is used above):
    # one launch per size bucket, and one persistent launch for all buckets
    persistent = {"autotuner_choice": pers_choice}
    for mode in ("0", "1"):
        os.environ["SBV_PERSISTENT"] = mode
        try:
            for name, prec in (("fp64", sbv.SBV_FP64), ("fp32", sbv.SBV_FP32)):
                msp, _, llp = run(prec, kin, 2, False)
                ref = ll64[:kin] if prec == sbv.SBV_FP64 else ll32[:kin]
                key = "persistent" if mode == "1" else "per_bucket"
                persistent[f"{name}_{key}"] = {
                    "ms_per_eval": msp / kin,
                    "max_rel_diff_vs_timed": float(np.max(np.abs(llp[:kin] - ref) / np.abs(ref)))}
        finally:
            del os.environ["SBV_PERSISTENT"]
    log(f"launch modes: {persistent}")

    small = small_leg(sbv, torch, dev, stream)

    fits = None
    if args.fit_evals > 0:
        fits = fit_legs(B, sbv, theta_true, two_nu, w, args.fit_evals)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(B, X, y_host, sbv, torch, dev, thetas[0], two_nu, args.cpu_seconds, small)

    large = None
    if args.large_steps > 0:
        large = large_leg(sbv, torch, dev, stream, args.large_steps)

    res = {
        "metric": "SBV loglik evals/s (n=1M, m=200, FP64)",
        "value": 1000.0 / ms_step,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": f"synthetic (uniform X, GP observations from {y_source})",
        "config": {"workload": "uneven_1m: n=1e6 d=10 Matern-5/2 tau2=1e-4 kmeans K=5e4 (5..60) m=200",
                   "n": n, "d": d, "blocks": B.K, "m": m, "parallelism": "1 GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": traffic(args.traffic_json),
                     "kernel": f"k_block_loglik<double,{tiles[v_dom]}>",
                     "flop_per_launch": flops[v_dom], "avg_launch_ms": avg_ms},
        "extra": {
            "fp64_total_algorithmic_tflops": total_flop / (ms_step * 1e-3) / 1e12,
            "fp32_evals_per_s": 1000.0 * kin / ms32,
            "fp32_max_rel_diff_vs_fp64": rel32,
            "fp32_fallback_blocks": int(fb),
            "grad_fp64_evals_per_s": grad_rate["fp64"],
            "grad_fp32_evals_per_s": grad_rate["fp32"],
            "small_20k": {k: v for k, v in small.items() if not k.startswith("_")},
            "persistent_single_launch": persistent,
            "build_seconds": t_build,
            "autotuned_tiles": tuned,
            "autotuned_schedules": sched,
            "fits": fits,
            "m400_5m": large,
        },
    }
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


def small_leg(sbv, torch, dev, stream, steps=100):
    """The n = 20,000, d = 10, Matern-5/2, tau^2 = 1e-6, 1,000-block, m = 60
    workload at its true theta: FP64 evaluations per second (structure built
    on the GPU, observations from the simulator)."""
    from paper_2504_12004_amd import synth, workloads
    w = synth.dataset("small_fp64")
    X, theta, xi = w["X"], w["theta"], w["xi"]
    d = X.shape[1]
    B = sbv.sbv_build_blocks(X, None, np.exp(theta[:d]), w["K"], w["m"], method=sbv.SBV_KMEANS,
                             lloyd_iters=w["lloyd_iters"], seed=w["seed"])
    y = workloads.simulate(sbv, torch, dev, X, theta, xi, w["two_nu"], w)
    sbv.sbv_blocks_set_y_dev(B, y)
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    out = torch.empty(steps + 3, dtype=torch.float64, device=dev)
    for i in range(3):
        sbv.sbv_loglik_dev(B, th, w["two_nu"], out[i:i + 1], sbv.SBV_FP64, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        sbv.sbv_loglik_dev(B, th, w["two_nu"], out[3 + i:4 + i], sbv.SBV_FP64, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    flops, _ = sbv.sbv_plan_flops(B, w["two_nu"])
    res = {"workload": "small_20k: n=2e4 d=10 Matern-5/2 tau2=1e-6 kmeans K=1000 m=60, true theta",
           "evals_per_s": 1000.0 / ms, "ms_per_eval": ms, "loglik_fp64": float(out[3].item()),
           "total_algorithmic_tflops": float(np.sum(flops)) / (ms * 1e-3) / 1e12}
    log(f"small_20k: {ms:.3f} ms/eval")
    # kept for the oracle comparison of the CPU-baseline leg
    res["_X"], res["_y"], res["_theta"], res["_two_nu"] = X, y.cpu().numpy(), theta, w["two_nu"]
    res["_structure"] = sbv.sbv_blocks_export(B)
    B.free()
    return res


def large_leg(sbv, torch, dev, stream, steps):
    """The n = 5e6, d = 10, K = 2.5e5, m = 400 workload (joint sizes up to 460:
    most blocks take the large path).  Forward log-likelihood only; y is the
    standard-normal draw of the generator (the conditional simulator covers
    joint sizes up to 272, and the timing does not depend on y)."""
    from paper_2504_12004_amd import synth
    w = synth.dataset("grad_5m")
    X, theta, xi = w["X"], w["theta"], w["xi"]
    d = X.shape[1]
    t0 = time.perf_counter()
    B = sbv.sbv_build_blocks(X, xi, np.exp(theta[:d]), w["K"], w["m"], method=sbv.SBV_KMEANS,
                             lloyd_iters=w["lloyd_iters"], min_bs=w["min_bs"], max_bs=w["max_bs"], seed=w["seed"])
    t_build = time.perf_counter() - t0
    del X
    two_nu = w["two_nu"]
    th_d = torch.tensor(theta, dtype=torch.float64, device=dev)
    out = torch.empty(steps + 2, dtype=torch.float64, device=dev)
    flops, tiles = sbv.sbv_plan_flops(B, two_nu)
    res = {"workload": "m400_5m: n=5e6 d=10 Matern-5/2 tau2=1e-4 kmeans K=2.5e5 (5..60) m=400",
           "build_seconds": t_build, "blocks": B.K, "algorithmic_tflop_per_eval": float(np.sum(flops)) / 1e12,
           "large_path_flop_share": float(flops[-1] / np.sum(flops)), "data": "y iid standard normal"}
    vals = {}
    for name, prec in (("fp64", sbv.SBV_FP64), ("fp32", sbv.SBV_FP32)):
        sbv.sbv_loglik_dev(B, th_d, two_nu, out[0:1], prec, stream)
        torch.cuda.synchronize()
        sbv.sbv_timing_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            sbv.sbv_loglik_dev(B, th_d, two_nu, out[1 + i:2 + i], prec, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        kt, kl = sbv.sbv_timing_read(prec)
        sbv.sbv_timing_enable(False)
        vals[name] = float(out[1].item())
        large_ms = kt[-1] / max(kl[-1], 1)
        res[name] = {"evals_per_s": 1000.0 / ms, "ms_per_eval": ms,
                     "large_bucket_ms": large_ms,
                     "large_bucket_tflops": flops[-1] / (large_ms * 1e-3) / 1e12 if large_ms > 0 else None,
                     "total_algorithmic_tflops": float(np.sum(flops)) / (ms * 1e-3) / 1e12,
                     "fallback_blocks": int(sbv.sbv_blocks_fallback_count(B)) if prec == sbv.SBV_FP32 else 0}
        log(f"m400_5m {name}: {ms:.1f} ms/eval, large bucket {large_ms:.1f} ms, "
            f"{res[name]['total_algorithmic_tflops']:.2f} TFLOP/s algorithmic")
    res["fp32_rel_diff_vs_fp64"] = abs(vals["fp32"] - vals["fp64"]) / abs(vals["fp64"])
    # log-likelihood + gradient (large-path adjoint), FP64 and FP32
    g = torch.empty(len(theta), dtype=torch.float64, device=dev)
    for name, prec in (("fp64", sbv.SBV_FP64), ("fp32", sbv.SBV_FP32)):
        sbv.sbv_loglik_grad_dev(B, th_d, two_nu, out[0:1], g, prec, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            sbv.sbv_loglik_grad_dev(B, th_d, two_nu, out[1 + i:2 + i], g, prec, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name]["grad_evals_per_s"] = 1000.0 / ms
        res[name]["grad_ms_per_eval"] = ms
        log(f"m400_5m {name} loglik+grad: {ms:.1f} ms/eval")
    B.free()
    return res


def fit_legs(B, sbv, theta_true, two_nu, w, max_evals):
    """MLE wall time on the resident structure from the cold start
    (beta_k = 1, sigma^2 = var(y), tau^2 = 1e-3 var(y)): plain FP64
    Nelder-Mead versus FP32 L-BFGS with an FP64 polish; each leg's optimum is
    judged by one FP64 evaluation."""
    d = w["d"]
    var_y = 1.0
    x0 = np.r_[np.zeros(d), np.log(var_y), np.log(1e-3 * var_y)]
    out = {}
    legs = [("nelder_mead_fp64", sbv.SBV_NELDER_MEAD, sbv.SBV_FP64, False),
            ("lbfgs_fp32_polish64", sbv.SBV_LBFGS, sbv.SBV_FP32, True),
            ("lbfgs_fp64", sbv.SBV_LBFGS, sbv.SBV_FP64, False)]
    for name, opt, prec, polish in legs:
        o = sbv.make_fit_opts(optimizer=opt, prec=prec, fp64_polish=polish, max_evals=max_evals, ftol=1e-10,
                              gtol=1e-3, init_step=0.5)
        th, l64, ne, sec, conv = sbv.sbv_fit(B, x0, two_nu, o)
        out[name] = {"seconds": sec, "evals": ne, "loglik_fp64": l64, "converged": conv}
        log(f"fit {name}: {sec:.2f}s, {ne} evals, l64 {l64:.6f}, converged {conv}")
    base = out["nelder_mead_fp64"]["loglik_fp64"]
    for k in out:
        out[k]["rel_gap_vs_nm64"] = (out[k]["loglik_fp64"] - base) / abs(base)
    return out


def traffic(path):
    """Per-launch HBM bytes of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the plain-copy
    calibration), or None when there is none or it was taken from kernel
    sources other than the current ones."""
    from paper_2504_12004_amd import profiling
    if path is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "k_block_loglik_uneven_1m_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != profiling.kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(B, X, y, sbv, torch, dev, theta, two_nu, seconds, small):
    """The FP64 oracle on a bounded sample of the same workload's blocks (real
    observations, the first evaluation point), scaled to evaluations per
    second of the whole dataset.  The same oracle evaluations check the
    device values at the full size: the GPU's per-block terms of those blocks
    (FP64 and FP32) against the oracle's, and the whole n = 2e4 workload."""
    import oracle as O
    bp, pts, npt, nid = sbv.sbv_blocks_export(B)
    S = O.Structure(B.n, B.d, 0, bp, pts, npt, nid)
    rng = np.random.default_rng(0)
    order = rng.permutation(B.K)
    threads = len(os.sched_getaffinity(0))
    # device block terms at theta (FP64, then FP32 with its fallback pass)
    th_d = torch.tensor(theta, dtype=torch.float64, device=dev)
    o = torch.empty(2, dtype=torch.float64, device=dev)
    terms = {}
    for name, prec in (("fp64", sbv.SBV_FP64), ("fp32", sbv.SBV_FP32)):
        sbv.sbv_loglik_dev(B, th_d, two_nu, o[:1], prec)
        torch.cuda.synchronize()
        terms[name] = sbv.sbv_blocks_terms(B)
    # calibrate on 64 blocks, then take enough blocks for about `seconds`
    t0 = time.perf_counter()
    O.sbv_loglik(X, y, O.subset(S, order[:64]), theta, two_nu, nthreads=threads)
    t_cal = max(time.perf_counter() - t0, 1e-4)
    nb = int(min(B.K, max(64, 64 * seconds / t_cal)))
    blocks = np.sort(order[:nb])
    sub = O.subset(S, blocks)
    t0 = time.perf_counter()
    tot, lb, ud = O.sbv_loglik(X, y, sub, theta, two_nu, blocks=True, parts=True, nthreads=threads)
    t = time.perf_counter() - t0
    scale = np.abs(lb) + np.abs(ud[:, 1]) + ud[:, 0]
    parity = {"blocks_checked": int(nb), "of_blocks": int(B.K), "theta": "first evaluation point"}
    for name in ("fp64", "fp32"):
        g = terms[name][blocks]
        parity[f"{name}_max_block_rel"] = float(np.max(np.abs(g - lb) / scale))
        parity[f"{name}_subset_sum_rel"] = float(abs(np.sum(g) - tot) / abs(tot))
    # the n = 2e4 workload, whole dataset
    if small is not None:
        Ss = O.Structure(len(small["_X"]), small["_X"].shape[1], 0, *small["_structure"])
        ref = O.sbv_loglik(small["_X"], small["_y"], Ss, small["_theta"], small["_two_nu"], nthreads=threads)
        parity["small_20k_fp64_rel"] = float(abs(small["loglik_fp64"] - ref) / abs(ref))
    log(f"parity vs oracle: {parity}")
    full = t * B.K / nb
    return {"value": 1.0 / full, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{nb} of {B.K} blocks (random), {t:.1f}s, scaled to the full dataset",
            "parity": parity}


if __name__ == "__main__":
    main()
