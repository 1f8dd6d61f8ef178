"""GPU checks of the GCP-Adam driver (gcp_adam_fit, Alg. 4).

With FP64 factors the device fit must follow the oracle's fit on the same
sample streams: the same accept/undo decisions, the same loss estimates and
the same final factors up to summation order.  An overshooting step size must
leave the start untouched (every epoch undone).  In FP32 the fit must recover
the factors of a noisy low-rank tensor (score >= 0.9, App. E).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1906_01687_amd as gcp
from pins import cp_score, full_model, tiny_sparse

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def gaussian_problem(dims=(20, 15, 10), r=3, seed=42, noise=0.1):
    rng = np.random.default_rng(seed)
    A_true = [rng.standard_normal((n, r)) for n in dims]
    X = full_model(A_true) + noise * rng.standard_normal(dims)
    A0 = [rng.standard_normal((n, r)) for n in dims]
    return X, A_true, A0


def test_fit_matches_oracle_fp64_dense():
    announce("gcp_adam_fit FP64 dense Gaussian vs oracle.adam_fit")
    X, _, A0 = gaussian_problem()
    dev = torch.device("cuda:0")
    Xt = gcp.dense_tensor(torch.as_tensor(X).to(dev))
    M = gcp.Factors(X.shape, 3, torch.float64, dev, init=A0)
    opts = dict(lr=0.01, tau=100, kappa=1, max_epochs=6)
    res = gcp.adam_fit(0, Xt, M, gcp.sampling("uniform", s=300, seed=5), gcp.sampling("uniform", s=3000, seed=6),
                       **opts)
    A, hist, acc, alpha = oracle.adam_fit(oracle.GAUSSIAN, X.shape, A0, dense=X,
                                          grad_cfg=dict(sampler=0, s=300, seed=5), est_cfg=dict(sampler=0, s=3000, seed=6),
                                          alpha=0.01, tau=100, kappa=1, max_epochs=6)
    torch.cuda.synchronize()
    assert res.accepted == acc and res.epochs == len(hist) - 1 and res.alpha == alpha
    np.testing.assert_allclose(res.history, hist, rtol=1e-9)
    for a_dev, a_orc in zip(M.A, A):
        a_dev = a_dev.cpu().numpy()
        assert np.linalg.norm(a_dev - a_orc) <= 1e-8 * np.linalg.norm(a_orc)


def test_fit_matches_oracle_fp64_stratified():
    announce("gcp_adam_fit FP64 sparse binary, stratified gradients and estimate, vs oracle")
    X, coo, val, A0 = tiny_sparse("binary", dims=(12, 10, 9), r=3, seed=29)
    dev = torch.device("cuda:0")
    Xt = gcp.coo_tensor(X.shape, torch.as_tensor(coo.astype(np.uint32).view(np.int32)).to(dev),
                        torch.as_tensor(val).to(torch.float64).to(dev))
    M = gcp.Factors(X.shape, 3, torch.float64, dev, init=A0)
    g = gcp.sampling("stratified", p=60, q=60, seed=11, iteration=3)
    e = gcp.sampling("stratified", p=400, q=400, seed=12)
    res = gcp.adam_fit(1, Xt, M, g, e, lr=0.01, lower=0.0, tau=50, kappa=1, max_epochs=5)
    A, hist, acc, alpha = oracle.adam_fit(oracle.BERNOULLI_ODDS, X.shape, A0, coo_idx=coo, coo_val=val,
                                          grad_cfg=dict(sampler=1, p=60, q=60, seed=11, iteration=3),
                                          est_cfg=dict(sampler=1, p=400, q=400, seed=12),
                                          alpha=0.01, lower=0.0, tau=50, kappa=1, max_epochs=5)
    torch.cuda.synchronize()
    assert res.accepted == acc and res.epochs == len(hist) - 1
    np.testing.assert_allclose(res.history, hist, rtol=1e-9)
    for a_dev, a_orc in zip(M.A, A):
        a_dev = a_dev.cpu().numpy()
        assert np.linalg.norm(a_dev - a_orc) <= 1e-8 * np.linalg.norm(a_orc)


def test_fit_undo_restores_the_start():
    announce("gcp_adam_fit: overshooting steps are undone exactly")
    X, _, A0 = gaussian_problem(dims=(6, 5, 4), r=2, seed=43, noise=0.0)
    dev = torch.device("cuda:0")
    Xt = gcp.dense_tensor(torch.as_tensor(X).to(dev))
    M = gcp.Factors(X.shape, 2, torch.float32, dev, init=A0)
    start = M.flat.clone()
    res = gcp.adam_fit(0, Xt, M, gcp.sampling("uniform", s=40, seed=7), gcp.sampling("uniform", s=500, seed=8),
                       lr=50.0, nu=0.5, tau=5, kappa=2, max_epochs=10)
    torch.cuda.synchronize()
    assert res.accepted == [True, False, False, False] and res.epochs == 3
    assert abs(res.alpha - 50.0 * 0.125) < 1e-12
    assert torch.equal(M.flat, start)
    assert int(res.adam.state[0].item()) == 0          # the step count was wound back
    assert float(res.adam.B.abs().max()) == 0.0


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_fit_recovers_low_rank_factors(dtype):
    announce(f"gcp_adam_fit recovery, {dtype}")
    X, A_true, A0 = gaussian_problem()
    dev = torch.device("cuda:0")
    Xt = gcp.dense_tensor(torch.as_tensor(X).to(torch.float32).to(dev))
    M = gcp.Factors(X.shape, 3, dtype, dev, init=A0)
    res = gcp.adam_fit(0, Xt, M, gcp.sampling("uniform", s=300, seed=5), gcp.sampling("uniform", s=3000, seed=6),
                       lr=0.01, tau=500, kappa=3, max_epochs=40)
    torch.cuda.synchronize()
    A = [a.detach().to(torch.float64).cpu().numpy() for a in (M.A if M.master is None else M._views(M.master))]
    score = cp_score(A_true, A)
    print(f"[result] recovery {dtype}: score {score:.4f} after {res.epochs} epochs, final estimate "
          f"{res.history[-1]:.4g}", flush=True)
    assert score >= 0.9


def test_fit_recovers_gamma_factors():
    """GCP-Adam with the Gamma loss on the App. C test problem (U(0,1) factors,
    shape-1 Gamma data), nonnegative projection, FP32."""
    announce("gcp_adam_fit recovery, Gamma loss")
    import synth
    dims, r = (30, 25, 20, 15), 3
    X, A_true = synth.dense_gamma(dims, r, seed=71)
    rng = np.random.default_rng(72)
    A0 = [rng.random((n, r)) for n in dims]
    dev = torch.device("cuda:0")
    Xt = gcp.dense_tensor(torch.as_tensor(X).to(torch.float32).to(dev))
    M = gcp.Factors(dims, r, torch.float32, dev, init=A0)
    res = gcp.adam_fit("gamma", Xt, M, gcp.sampling("uniform", s=500, seed=5),
                       gcp.sampling("uniform", s=20000, seed=6), lr=0.01, lower=0.0, tau=500, kappa=3,
                       max_epochs=40)
    torch.cuda.synchronize()
    A = [a.detach().to(torch.float64).cpu().numpy() for a in M.A]
    score = cp_score(A_true, A)
    print(f"[result] Gamma recovery: score {score:.4f} after {res.epochs} epochs", flush=True)
    assert score >= 0.9
    assert min(float(a.min()) for a in A) >= 0.0
