"""Observations for the synthetic workloads, drawn by the library itself.

The inputs and the standard-normal innovations come from `synth` (random
numbers only); the observations are the library's Vecchia conditional
simulation at the true parameters on a generating structure that is built
independently of any evaluation structure.
"""
import numpy as np


def simulate(sbv, torch, dev, X, theta, xi, two_nu, w):
    """Observations at the true parameters: the device conditional simulator on
    a generating structure built independently of the evaluation structure
    (its own seed, m_gen conditioning points, blocks of at most gen_max_bs
    points so that every joint set fits the simulator).  Returns y (device,
    original point order)."""
    n, d = X.shape
    G = sbv.sbv_build_blocks(X, None, np.exp(theta[:d]), max(1, n // w["gen_bs_mean"]), w["m_gen"],
                             method=sbv.SBV_KMEANS, lloyd_iters=1, min_bs=0, max_bs=w["gen_max_bs"],
                             seed=w["seed"] + 7919)
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    xi_d = torch.tensor(xi, dtype=torch.float64, device=dev)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    sbv.sbv_sample_dev(G, th, two_nu, xi_d, y)
    torch.cuda.synchronize()
    G.free()
    return y
