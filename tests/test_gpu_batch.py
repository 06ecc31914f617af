"""Batching across datasets: one plan over several datasets (different d, nu,
sizes) equals the per-dataset evaluations; the captured graph's replays equal
the eager evaluation, replay after replay with eager work in between; the
autotuner's choice leaves the values unchanged."""
import numpy as np
import pytest

from helpers import problem, to_gpu
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sbv():
    from paper_2504_12004_amd import sbv as S
    return S


@pytest.fixture(scope="module")
def batch(sbv):
    specs = [(2000, 5, 100, 40, 3), (3000, 10, 150, 120, 5), (1500, 7, 60, 200, 5), (2500, 3, 125, 60, 1)]
    hs, ths, tns, refs = [], [], [], []
    for i, (n, d, K, m, tn) in enumerate(specs):
        X, y, th, S = problem(n, d, K=K, m=m, seed=70 + i, two_nu=tn, tau2=1e-3, max_bs=40)
        hs.append(to_gpu(sbv, X, y, S))
        ths.append(th)
        tns.append(tn)
        refs.append(O.sbv_loglik(X, y, S, th, tn))
    return hs, ths, tns, np.array(refs)


def test_batched_equals_separate_and_oracle(sbv, batch):
    hs, ths, tns, refs = batch
    joint = sbv.sbv_loglik(hs, ths, tns)
    sep = np.array([sbv.sbv_loglik(h, t, tn)[0] for h, t, tn in zip(hs, ths, tns)])
    assert np.array_equal(joint, sep)
    assert np.all(np.abs(joint - refs) <= 1e-10 * np.abs(refs))


def test_graph_replays_equal_eager(sbv, batch):
    import torch
    hs, ths, tns, _ = batch
    dev = torch.device("cuda:0")
    th = torch.tensor(np.concatenate(ths), dtype=torch.float64, device=dev)
    out_e = torch.empty(len(hs), dtype=torch.float64, device=dev)
    out_g = torch.empty(len(hs), dtype=torch.float64, device=dev)
    for prec in (sbv.SBV_FP64, sbv.SBV_FP32):
        sbv.sbv_loglik_dev(hs, th, tns, out_e, prec)
        torch.cuda.synchronize()
        eager = out_e.cpu().numpy().copy()
        for rep in range(4):
            sbv.sbv_eval_graph_dev(hs, th, tns, out_g, prec)
            torch.cuda.synchronize()
            assert np.array_equal(out_g.cpu().numpy(), eager), (prec, rep)
            # eager work in between replays
            sbv.sbv_loglik_dev(hs, th, tns, out_e, prec)
            torch.cuda.synchronize()
            assert np.array_equal(out_e.cpu().numpy(), eager)


def test_graph_gradient_replays_equal_eager(sbv, batch):
    import torch
    hs, ths, tns, _ = batch
    dev = torch.device("cuda:0")
    th = torch.tensor(np.concatenate(ths), dtype=torch.float64, device=dev)
    l_e = torch.empty(len(hs), dtype=torch.float64, device=dev)
    g_e = torch.empty(len(th), dtype=torch.float64, device=dev)
    l_g = torch.empty_like(l_e)
    g_g = torch.empty_like(g_e)
    sbv.sbv_loglik_grad_dev(hs, th, tns, l_e, g_e)
    torch.cuda.synchronize()
    for _ in range(3):
        sbv.sbv_eval_graph_dev(hs, th, tns, l_g, sbv.SBV_FP64, grad_dev=g_g)
        torch.cuda.synchronize()
        assert torch.equal(l_g, l_e) and torch.equal(g_g, g_e)


def test_autotune_keeps_values(sbv, batch):
    hs, ths, tns, _ = batch
    before = sbv.sbv_loglik(hs, ths, tns)
    chosen = sbv.sbv_autotune(hs, ths, tns, reps=2)
    assert len(chosen) >= 1
    after = sbv.sbv_loglik(hs, ths, tns)
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before))


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-4)])
def test_persistent_single_launch(sbv, batch, prec, tol, monkeypatch):
    """SBV_PERSISTENT=1: every register-path block of every set goes through
    one launch whose workgroups take blocks from a device counter, longest
    first; values match the oracle, and its captured graph replays equal the
    eager evaluation (the counter is reset by a kernel inside the graph)."""
    import torch
    hs, ths, tns, refs = batch
    monkeypatch.setenv("SBV_PERSISTENT", "1")
    got = sbv.sbv_loglik(hs, ths, tns, prec)
    assert np.all(np.abs(got - refs) <= tol * np.abs(refs))
    dev = torch.device("cuda:0")
    th = torch.tensor(np.concatenate(ths), dtype=torch.float64, device=dev)
    out_e = torch.empty(len(hs), dtype=torch.float64, device=dev)
    out_g = torch.empty(len(hs), dtype=torch.float64, device=dev)
    sbv.sbv_loglik_dev(hs, th, tns, out_e, prec)
    torch.cuda.synchronize()
    eager = out_e.cpu().numpy().copy()
    assert np.array_equal(eager, got)
    # a graph captured in persistent mode (its own plan: a fresh handle list order)
    order = [3, 2, 1, 0]
    hs2 = [hs[i] for i in order]
    th2 = torch.tensor(np.concatenate([ths[i] for i in order]), dtype=torch.float64, device=dev)
    tn2 = [tns[i] for i in order]
    sbv.sbv_loglik_dev(hs2, th2, tn2, out_e, prec)
    torch.cuda.synchronize()
    eager2 = out_e.cpu().numpy().copy()
    assert np.all(np.abs(eager2 - refs[order]) <= tol * np.abs(refs[order]))
    for rep in range(3):
        sbv.sbv_eval_graph_dev(hs2, th2, tn2, out_g, prec)
        torch.cuda.synchronize()
        assert np.array_equal(out_g.cpu().numpy(), eager2), rep
        sbv.sbv_loglik_dev(hs, th, tns, out_e, prec)  # eager work of another plan in between
        torch.cuda.synchronize()
