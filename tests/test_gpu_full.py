"""GPU checks of the FULL sampler (every entry once, weight 1: the exact
gradient and loss) against the oracle's enumeration, and of the estimator
statistics of the sampler comparison (variance.gradient_moments)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1906_01687_amd as gcp
from paper_1906_01687_amd import variance
from gpu_cases import TORCH_DT, check_grad, grad_scale, host_rounded, rel_fro, small_dense, small_sparse

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dense_of(w):
    if w.dense is not None:
        return np.asarray(w.dense, dtype=np.float64)
    X = np.zeros(w.dims)
    X[tuple(np.asarray(w.coo_idx, dtype=np.int64).T)] = w.coo_val
    return X


CASES = [("dense_f64", lambda: small_dense(dtype="f64", loss=synth.POISSON), "f64", None),
         ("dense_f32_gamma", lambda: small_dense(rank=6, loss=synth.GAMMA), "f32", None),
         ("counts_hash_f32", lambda: small_sparse("counts", rank=10), "f32", False),
         ("binary_bitmap_f32", lambda: small_sparse("binary"), "f32", True)]


@pytest.mark.parametrize("name,make,dtype,bitmap", CASES, ids=[c[0] for c in CASES])
def test_full_gradient_is_the_enumeration(name, make, dtype, bitmap):
    announce(f"FULL sampler vs enumeration, {name}")
    w = make()
    dev = torch.device("cuda:0")
    vdt = torch.float64 if dtype == "f64" else torch.float32
    if w.dense is not None:
        X = gcp.dense_tensor(torch.as_tensor(w.dense).to(vdt).to(dev))
    else:
        X = gcp.coo_tensor(w.dims, torch.as_tensor(np.ascontiguousarray(w.coo_idx).view(np.int32)).to(dev),
                           torch.as_tensor(w.coo_val).to(vdt).to(dev), bitmap=bitmap)
    M = gcp.Factors(w.dims, w.rank, TORCH_DT[dtype], dev, init=w.A_init)
    cfg = gcp.sampling("full")
    G, fs = gcp.sampled_grad(w.loss, X, M, cfg, with_loss=True)
    dense = torch.as_tensor(dense_of(w)).to(vdt).to(torch.float64).numpy()
    Gref, Fref = oracle.full_grad(w.loss, host_rounded(w.A_init, dtype), dense)
    idx, xv, st = gcp.sample(X, cfg)
    torch.cuda.synchronize()
    tol = 1e-12 if dtype == "f64" else 1e-5
    omega = int(np.prod(w.dims))
    ref_idx = np.stack(np.unravel_index(np.arange(omega), w.dims), axis=1)
    enum = oracle.Samples(ref_idx, dense.reshape(-1), np.zeros(omega, np.int32), np.arange(omega), omega)
    E = grad_scale(w.loss, w.dims, host_rounded(w.A_init, dtype), enum, s=omega)
    check_grad(G, Gref, E, tol, f"FULL {name}")
    assert abs(fs.item() - Fref) <= 10 * tol * max(1.0, abs(Fref))
    # the materialised enumeration: entry c in row-major order, its value, weight-1 stratum
    assert np.array_equal(idx.cpu().numpy().astype(np.int64), ref_idx)
    assert np.array_equal(xv.cpu().to(torch.float64).numpy(), dense.reshape(-1))
    assert int(st.max()) == 0


def test_sampler_statistics_order():
    """On an App. D binary tensor the three samplers are unbiased (the mean of
    N draws sits within the 3 tr(Sigma)/N band of the exact gradient) and the
    stratified and semi-stratified variances are below the uniform one."""
    announce("sampler statistics on an App. D tensor 60x50x40x30")
    dims, r = (60, 50, 40, 30), 5
    coo, val, A_true = synth.sparse_binary_appd(dims, r, seed=11)
    dev = torch.device("cuda:0")
    X = gcp.coo_tensor(dims, torch.as_tensor(coo.view(np.int32)).to(dev), torch.as_tensor(val).float().to(dev))
    rng = np.random.default_rng(12)
    A0 = [rng.random((n, r)) * 0.3 for n in dims]
    out = {}
    for name, A in (("start", A0), ("truth", A_true)):
        M = gcp.Factors(dims, r, torch.float32, dev, init=A)
        exact = variance.exact_gradient(synth.BERNOULLI_ODDS, X, M)
        stats = {}
        for sname, cfg in (("uniform", gcp.sampling("uniform", s=1000, seed=5)),
                           ("stratified", gcp.sampling("stratified", p=500, q=500, seed=5)),
                           ("semi", gcp.sampling("semi_stratified", p=500, q=500, seed=5))):
            mo = variance.gradient_moments(synth.BERNOULLI_ODDS, X, M, cfg, 400, exact=exact)
            assert mo.bias ** 2 <= 3.0 * mo.variance / mo.draws, (name, sname, mo)
            stats[sname] = mo
        assert stats["stratified"].variance < stats["uniform"].variance
        assert stats["semi"].variance < stats["uniform"].variance
        out[name] = {k: (v.bias, v.variance) for k, v in stats.items()}
    print(f"[result] sampler statistics (bias, variance): {out}", flush=True)
