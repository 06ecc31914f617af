"""The allocation-free log-likelihood entry point against sbv_loglik_dev.

Two calls in a row on the same device (a larger handle, then a smaller one)
must each reproduce sbv_loglik_dev's value bit for bit (same kernels, buckets
and reduction), in FP64 and in FP32 with its FP64 fallback pass, and the FP64
value must match the oracle."""
import numpy as np
import pytest

import oracle as O
from helpers import problem, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cases():
    # larger first: two size buckets (early blocks with few candidates take
    # the smallest variant), ragged block sizes 5..60
    big = problem(3000, 6, 150, 90, seed=21, min_bs=5, max_bs=60)
    small = problem(700, 6, 35, 40, seed=22)
    return [big, small]


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_loglik_dev_twice(cases, prec):
    import torch
    from paper_2504_12004_amd import sbv
    dev = torch.device("cuda:0")
    for X, y, theta, S in cases:
        print(f"noalloc case n={X.shape[0]} K={S.K} prec={prec}", flush=True)
        B = to_gpu(sbv, X, y, S)
        th = torch.tensor(theta, dtype=torch.float64, device=dev)
        ref = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
        got = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream()
        sbv.sbv_loglik_dev(B, th, 5, ref, prec=prec, stream=stream)
        sbv.sbv_loglik_noalloc_dev(B, th, 5, got, prec=prec, stream=stream)
        torch.cuda.synchronize()
        r, g = ref.item(), got.item()
        assert np.isfinite(g)
        assert g == r, (g, r)
        if prec == 0:
            o = O.sbv_loglik(X, y, S, theta, 5)
            assert abs(g - o) <= 1e-10 * abs(o)
        B.free()


def test_noalloc_rejects_oversized_and_bad_arguments(cases):
    import torch
    from paper_2504_12004_amd import sbv
    X, y, theta, S = cases[1]
    B = to_gpu(sbv, X, y, S)
    th = torch.tensor(theta, dtype=torch.float64, device="cuda:0")
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sbv.SBVError) as e:
        sbv.sbv_loglik_noalloc_dev(B, th, 4, out)
    assert e.value.status == sbv.SBV_E_INVAL
    with pytest.raises(sbv.SBVError) as e:
        sbv.sbv_loglik_noalloc_dev(B, th, 5, out, prec=7)
    assert e.value.status == sbv.SBV_E_INVAL
    B.free()
    # joint sizes above 272 need the large-set workspace: refused
    Xl, yl, thl, Sl = problem(1200, 4, 40, 300, seed=23)
    Bl = to_gpu(sbv, Xl, yl, Sl)
    thl_d = torch.tensor(thl, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sbv.SBVError) as e:
        sbv.sbv_loglik_noalloc_dev(Bl, thl_d, 5, out)
    assert e.value.status == sbv.SBV_E_INVAL and "joint sizes" in str(e.value)
    Bl.free()
    # more blocks than the scratch array holds: refused
    K = (1 << 18) + 1
    Xs = np.random.default_rng(5).random((K, 2))
    ar = np.arange(K + 1, dtype=np.int64)
    Bs = sbv.sbv_blocks_import(Xs, np.zeros(K), ar, ar[:-1], np.zeros(K + 1, np.int64), np.zeros(0, np.int64))
    ths = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sbv.SBVError) as e:
        sbv.sbv_loglik_noalloc_dev(Bs, ths, 5, out)
    assert e.value.status == sbv.SBV_E_INVAL and "blocks" in str(e.value)
    Bs.free()
