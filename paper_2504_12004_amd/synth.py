"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws random numbers only (numpy PCG64 via default_rng); it holds
none of the method's arithmetic, so both the GPU path and the CPU oracle can
consume exactly the same bytes.  Draw order inside one recipe is fixed:
inputs X, then parameters, then the standard-normal innovations xi.

Workloads (inputs uniform on [0,1]^d as in Sec. 7.1 and Sec. 8):
  small_fp64   n = 20,000, d = 10, Matern-5/2, sigma^2 = 1, tau^2 = 1e-6,
               ranges (0.05,0.1,0.2,0.3,0.5,0.8,1,1.5,2,3), 1,000 k-means
               blocks, m = 60 (seed 0)
  uneven_1m    n = 1,000,000, d = 10, Matern-5/2, ranges log-uniform on
               [0.05, 3], sigma^2 = 1, tau^2 = 1e-4, 50,000 k-means blocks
               bounded to 5..60 points, m = 200, 100 perturbed theta (seed 1/2)
  (m_gen, gen_bs_mean, gen_max_bs: the independent generating structure of the
  observations -- conditioning count, mean and largest block size)
  multi64      64 datasets, n ~ U[50k, 400k], d in {5,10,20}, nu in {3/2,5/2},
               m in {100,200,400} (seed 3)
  grad_5m      n = 5,000,000, d = 10, 250,000 blocks, m = 400 (seed 4)
  warm_20m     n = 20,000,000, d = 10, m = 400; training sets n = 20,000 (seeds 5/6)
"""
import numpy as np

SMALL_BETA = np.array([0.05, 0.1, 0.2, 0.3, 0.5, 0.8, 1.0, 1.5, 2.0, 3.0])

WORKLOADS = {
    "small_fp64": dict(seed=0, n=20_000, d=10, two_nu=5, sigma2=1.0, tau2=1e-6, K=1_000, m=60,
                       lloyd_iters=10, min_bs=0, max_bs=0, m_gen=120, gen_bs_mean=20, gen_max_bs=40),
    "uneven_1m": dict(seed=1, n=1_000_000, d=10, two_nu=5, sigma2=1.0, tau2=1e-4, K=50_000, m=200,
                      lloyd_iters=10, min_bs=5, max_bs=60, n_theta=100, theta_seed=2,
                      m_gen=250, gen_bs_mean=10, gen_max_bs=22),
    "grad_5m": dict(seed=4, n=5_000_000, d=10, two_nu=5, sigma2=1.0, tau2=1e-4, K=250_000, m=400,
                    lloyd_iters=5, min_bs=5, max_bs=60),
    "warm_20m": dict(seed=6, n=20_000_000, d=10, two_nu=5, K=1_000_000, m=400, lloyd_iters=2,
                     min_bs=5, max_bs=60),
}


def rng(seed):
    return np.random.default_rng(seed)


def log_uniform(g, lo, hi, size=None):
    return np.exp(g.uniform(np.log(lo), np.log(hi), size))


def theta_vector(beta, sigma2, tau2):
    """Pack [log beta_1..d, log sigma^2, log tau^2] (the parameter vector order)."""
    return np.r_[np.log(np.asarray(beta, dtype=np.float64)), np.log(sigma2), np.log(tau2)]


def dataset(name, n=None):
    """Inputs X, true theta and innovations xi of one named workload.
    `n` overrides the size (a prefix-consistent subsample of the same stream is
    NOT implied; a smaller n is a fresh draw with the same seed)."""
    w = dict(WORKLOADS[name])
    if n is not None:
        w["n"] = int(n)
    g = rng(w["seed"])
    X = g.random((w["n"], w["d"]))
    if name == "small_fp64":
        beta = SMALL_BETA[: w["d"]].copy()
        s2, t2 = w["sigma2"], w["tau2"]
    elif name == "warm_20m":
        beta = log_uniform(g, 0.05, 3.0, w["d"])
        s2 = log_uniform(g, 0.5, 2.0)
        t2 = log_uniform(g, 1e-6, 1e-2)
    else:
        beta = log_uniform(g, 0.05, 3.0, w["d"])
        s2, t2 = w["sigma2"], w["tau2"]
    xi = g.standard_normal(w["n"])
    return dict(X=X, theta=theta_vector(beta, s2, t2), xi=xi, **w)


def perturbed_thetas(theta, count, seed, scale=0.1):
    """theta_t = theta + scale * N(0, I), the evaluation points of a benchmark."""
    g = rng(seed)
    return theta[None, :] + scale * g.standard_normal((count, len(theta)))


def multi_datasets(count=64, seed=3):
    """Per-dataset recipes of the 64-set batching workload (sizes, d, nu, m, theta)."""
    g = rng(seed)
    out = []
    for j in range(count):
        n = int(g.integers(50_000, 400_001))
        d = int(g.choice([5, 10, 20]))
        two_nu = int(g.choice([3, 5]))
        m = int(g.choice([100, 200, 400]))
        beta = log_uniform(g, 0.05, 3.0, d)
        out.append(dict(n=n, d=d, two_nu=two_nu, m=m, theta=theta_vector(beta, 1.0, 1e-4),
                        K=max(1, round(n / 20)), min_bs=5, max_bs=60, seed=1000 + j))
    return out


def inputs_for(recipe):
    """X and xi of one multi-dataset recipe."""
    g = rng(recipe["seed"])
    X = g.random((recipe["n"], recipe["d"]))
    xi = g.standard_normal(recipe["n"])
    return X, xi


def random_spd_problem(n, d, seed, beta=None, sigma2=1.0, tau2=1e-2, two_nu=5):
    """Small random problem for tests: X uniform, theta fixed or drawn."""
    g = rng(seed)
    X = g.random((n, d))
    if beta is None:
        beta = log_uniform(g, 0.1, 2.0, d)
    xi = g.standard_normal(n)
    return X, theta_vector(beta, sigma2, tau2), xi
