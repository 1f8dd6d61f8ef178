"""GPU parity of the weighted objective (eq. wgcp): entry weights on dense and
COO tensors (w_zero for the entries a COO tensor does not store), in the fused
and unfused paths, the Adam step and batches, against the oracle's weighted
gradient on the same samples (element by element and in relative Frobenius
norm: 1e-5 in FP32, 1e-12 in FP64; gpu_cases.check_grad).  Stored weights of
exactly 0 are included: a corrected semi-stratified nonzero of weight 0 still
carries its -(eta/p) w_zero g(0, m) term (Sec. 4.3, eq. wgcp)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1906_01687_amd as gcp
from gpu_cases import TORCH_DT, check_grad, grad_scale, host_rounded, rel_fro, small_dense, small_sparse

pytestmark = pytest.mark.gpu
TOL = {"f64": 1e-12, "f32": 1e-5}


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def weighted_problem(kind, dtype="f32", w_zero=0.3, seed=5, zero_frac=0.0):
    """(workload, DataTensor with weights, host weights for the oracle); a
    fraction ``zero_frac`` of the stored weights of a COO tensor is 0."""
    dev = torch.device("cuda:0")
    vdt = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(seed)
    if kind == "dense":
        w = small_dense(dims=(13, 17, 11), rank=6, s=4000, dtype=dtype, loss=synth.POISSON)
        W = rng.uniform(0.2, 2.0, size=w.dims)
        W[rng.random(w.dims) < 0.3] = 0.0            # missing entries
        X = gcp.dense_tensor(torch.as_tensor(w.dense).to(vdt).to(dev),
                             weights=torch.as_tensor(W).to(vdt).to(dev))
        host = dict(dense_w=torch.as_tensor(W).to(vdt).to(torch.float64).numpy())
        return w, X, host, 1.0
    sampler = {"strat": synth.STRATIFIED, "semi": synth.SEMI_STRATIFIED, "uniform": synth.UNIFORM}[kind]
    w = small_sparse("counts", rank=7, dtype=dtype, sampler=sampler)
    if sampler == synth.UNIFORM:
        w.s = 5000
    cw = rng.uniform(0.2, 2.0, size=w.nnz)
    cw[rng.random(w.nnz) < zero_frac] = 0.0
    X = gcp.coo_tensor(w.dims, torch.as_tensor(np.ascontiguousarray(w.coo_idx).view(np.int32)).to(dev),
                       torch.as_tensor(w.coo_val).to(vdt).to(dev), weights=torch.as_tensor(cw).to(vdt).to(dev),
                       w_zero=w_zero)
    host = dict(coo_idx=np.asarray(w.coo_idx, dtype=np.int64),
                coo_w=torch.as_tensor(cw).to(vdt).to(torch.float64).numpy(), w_zero=w_zero)
    return w, X, host, w_zero


def oracle_weighted(w, host, w_zero, dtype, iteration):
    if w.dense is not None:
        vdt = torch.float64 if dtype == "f64" else torch.float32
        dense64 = torch.as_tensor(w.dense).to(vdt).to(torch.float64).numpy()
        smp = oracle.sample(w.sampler, w.dims, dense=dense64, s=w.s, seed=w.seed, iteration=iteration)
    else:
        vdt = torch.float64 if dtype == "f64" else torch.float32
        val64 = torch.as_tensor(w.coo_val).to(vdt).to(torch.float64).numpy()
        smp = oracle.sample(w.sampler, w.dims, coo_idx=np.asarray(w.coo_idx, dtype=np.int64), coo_val=val64,
                            s=w.s, p=w.p, q=w.q, seed=w.seed, iteration=iteration)
    wg = oracle.entry_weights(w.dims, smp, **host)
    A64 = host_rounded(w.A_init, dtype)
    G, F = oracle.grad(w.loss, w.dims, A64, smp, nnz=w.nnz, s=w.s, p=w.p, q=w.q, wgt=wg, w_zero=w_zero)
    E = grad_scale(w.loss, w.dims, A64, smp, nnz=w.nnz, s=w.s, p=w.p, q=w.q, ew=wg, w_zero=w_zero)
    return G, F, E


CASES = [("dense", "f32", 0.0), ("dense", "f64", 0.0), ("uniform", "f32", 0.0), ("strat", "f32", 0.0),
         ("semi", "f32", 0.0), ("semi", "f64", 0.0),
         # stored weights of 0 (missing entries kept in the list)
         ("semi", "f32", 0.3), ("semi", "f64", 0.3), ("strat", "f32", 0.3), ("uniform", "f32", 0.3)]


@pytest.mark.parametrize("kind,dtype,zero_frac", CASES, ids=[f"{k}_{d}_w0{z}" for k, d, z in CASES])
def test_weighted_fused_and_unfused(kind, dtype, zero_frac):
    announce(f"weighted objective, {kind}, {dtype}, stored weights 0: {zero_frac}")
    w, X, host, wz = weighted_problem(kind, dtype, zero_frac=zero_frac)
    dev = torch.device("cuda:0")
    M = gcp.Factors(w.dims, w.rank, TORCH_DT[dtype], dev, init=w.A_init)
    cfg = gcp.sampling(w.sampler, s=w.s, p=w.p, q=w.q, seed=w.seed, iteration=2)
    G, fs = gcp.sampled_grad(w.loss, X, M, cfg, with_loss=True)
    idx, xv, st = gcp.sample(X, cfg)
    y, fs2 = gcp.loss_grad(w.loss, X, cfg, M, idx, xv, st, with_loss=True)
    G2 = gcp.mttkrp(X, M, idx, y)
    Gref, Fref, E = oracle_weighted(w, host, wz, dtype, 2)
    torch.cuda.synchronize()
    tol = TOL[dtype]
    check_grad(G, Gref, E, tol, f"weighted fused {kind} {dtype}")
    check_grad(G2, Gref, E, tol, f"weighted unfused {kind} {dtype}")
    assert abs(fs.item() - Fref) <= 10 * tol * max(1.0, abs(Fref))
    assert abs(fs2.item() - Fref) <= 10 * tol * max(1.0, abs(Fref))


def test_unit_weights_equal_unweighted():
    announce("weights of 1 everywhere equal the unweighted gradient")
    w = small_sparse("counts", rank=7, sampler=synth.SEMI_STRATIFIED)
    dev = torch.device("cuda:0")
    ci = torch.as_tensor(np.ascontiguousarray(w.coo_idx).view(np.int32)).to(dev)
    cv = torch.as_tensor(w.coo_val).to(torch.float32).to(dev)
    Xw = gcp.coo_tensor(w.dims, ci, cv, weights=torch.ones_like(cv), w_zero=1.0)
    Xu = gcp.coo_tensor(w.dims, ci, cv)
    M = gcp.Factors(w.dims, w.rank, torch.float32, dev, init=w.A_init)
    cfg = gcp.sampling(w.sampler, p=w.p, q=w.q, seed=w.seed)
    Gw = gcp.sampled_grad(w.loss, Xw, M, cfg)
    Gu = gcp.sampled_grad(w.loss, Xu, M, cfg)
    torch.cuda.synchronize()
    assert max(rel_fro(Gw, [g.to(torch.float64).cpu().numpy() for g in Gu])) <= 1e-6


def test_weighted_batch_and_adam():
    announce("weighted problems in a batch and in the fused Adam step")
    dev = torch.device("cuda:0")
    wa, Xa, ha, wza = weighted_problem("dense", seed=7)
    wb, Xb, hb, wzb = weighted_problem("semi", seed=8, zero_frac=0.3)
    probs = []
    for b, (w, X) in enumerate(((wa, Xa), (wb, Xb))):
        M = gcp.Factors(w.dims, w.rank, torch.float32, dev, init=w.A_init)
        cfg = gcp.sampling(w.sampler, s=w.s, p=w.p, q=w.q, seed=w.seed, problem_id=0)
        probs.append(gcp.Problem(w.loss, X, M, cfg, lower=w.lower, keep_grad=True))
    batch = gcp.Batch(probs)
    batch.grad()
    torch.cuda.synchronize()
    for (w, h, wz), p in zip(((wa, ha, wza), (wb, hb, wzb)), probs):
        Gref, _, E = oracle_weighted(w, h, wz, "f32", 0)
        check_grad(p.M.grad_views(p.G), Gref, E, 1e-5, "weighted batch")
    batch.close()
    # fused step: the Adam update follows the weighted gradient
    M = gcp.Factors(wb.dims, wb.rank, torch.float32, dev, init=wb.A_init)
    adam = gcp.Adam(M, lr=0.01, lower=0.0)
    cfg = gcp.sampling(wb.sampler, p=wb.p, q=wb.q, seed=wb.seed, iteration=4)
    step = gcp.SampledAdamStep(wb.loss, Xb, M, cfg, adam, keep_grad=True)
    step()
    torch.cuda.synchronize()
    Gref, _, E = oracle_weighted(wb, hb, wzb, "f32", 4)
    check_grad(M.grad_views(step.gbuf), Gref, E, 1e-5, "weighted fused Adam step")


def test_missing_entries_by_observed_list():
    """Missing data without zero weights: nonzero picks over the list of
    observed entries (observed zeros stored explicitly) with q = 0."""
    announce("missing data: sampling the observed list")
    dev = torch.device("cuda:0")
    w = small_dense(dims=(13, 17, 11), rank=5, s=1, loss=synth.GAUSSIAN)
    rng = np.random.default_rng(3)
    obs = np.argwhere(rng.random(w.dims) < 0.6).astype(np.uint32)
    val = w.dense[tuple(obs.astype(np.int64).T)]
    X = gcp.coo_tensor(w.dims, torch.as_tensor(obs.view(np.int32)).to(dev), torch.as_tensor(val).float().to(dev))
    M = gcp.Factors(w.dims, w.rank, torch.float32, dev, init=w.A_init)
    cfg = gcp.sampling("stratified", p=3000, q=0, seed=9)
    G = gcp.sampled_grad(w.loss, X, M, cfg)
    smp = oracle.sample(oracle.STRATIFIED, w.dims, coo_idx=obs.astype(np.int64),
                        coo_val=torch.as_tensor(val).float().double().numpy(), p=3000, q=0, seed=9)
    A64 = host_rounded(w.A_init, "f32")
    Gref, _ = oracle.grad(w.loss, w.dims, A64, smp, nnz=obs.shape[0], p=3000, q=0)
    torch.cuda.synchronize()
    check_grad(G, Gref, grad_scale(w.loss, w.dims, A64, smp, nnz=obs.shape[0], p=3000, q=0), 1e-5,
               "observed list")
