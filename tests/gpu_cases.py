"""Shared set-up for the GPU parity tests: seeded problems on the device and the
oracle's answers for them.  The oracle always gets the same input values the
device gets (FP32/BF16 factors are rounded on the host, then widened)."""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import torch

import oracle
import synth
import paper_1906_01687_amd as gcp

TORCH_DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def host_rounded(mats, dtype: str) -> List[np.ndarray]:
    """The factor values the device stores, widened to float64 on the host."""
    out = []
    for a in mats:
        t = torch.as_tensor(np.asarray(a, dtype=np.float64))
        if dtype == "f32":
            t = t.to(torch.float32)
        elif dtype == "bf16":
            t = t.to(torch.float32).to(torch.bfloat16)
        out.append(t.to(torch.float64).numpy())
    return out


@dataclasses.dataclass
class Problem:
    w: synth.Workload
    X: gcp.DataTensor
    M: gcp.Factors
    A64: List[np.ndarray]          # oracle view of the factors
    dense64: Optional[np.ndarray]  # oracle view of dense X
    coo64: Optional[np.ndarray]
    val64: Optional[np.ndarray]


def to_device(w: synth.Workload, vdtype=None, dtype: Optional[str] = None, bitmap: Optional[bool] = None) -> Problem:
    dev = torch.device("cuda:0")
    dtype = dtype or w.dtype
    if vdtype is None:
        vdtype = torch.float64 if dtype == "f64" else torch.float32
    if w.dense is not None:
        Xd = torch.as_tensor(np.ascontiguousarray(w.dense)).to(vdtype).to(dev)
        X = gcp.dense_tensor(Xd)
        dense64 = torch.as_tensor(np.asarray(w.dense)).to(vdtype).to(torch.float64).numpy()
        coo64 = val64 = None
    else:
        ci = torch.as_tensor(np.ascontiguousarray(w.coo_idx).view(np.int32)).to(dev)
        cv = torch.as_tensor(np.asarray(w.coo_val)).to(vdtype).to(dev)
        X = gcp.coo_tensor(w.dims, ci, cv, bitmap=bitmap)
        dense64 = None
        coo64 = np.asarray(w.coo_idx, dtype=np.int64)
        val64 = torch.as_tensor(np.asarray(w.coo_val)).to(vdtype).to(torch.float64).numpy()
    M = gcp.Factors(w.dims, w.rank, TORCH_DT[dtype], dev, init=w.A_init)
    return Problem(w, X, M, host_rounded(w.A_init, dtype), dense64, coo64, val64)


def oracle_samples(pb: Problem, iteration: int = 0, problem_id: int = 0, **over):
    w = pb.w
    kw = dict(s=over.get("s", w.s), p=over.get("p", w.p), q=over.get("q", w.q))
    if pb.dense64 is not None:
        return oracle.sample(w.sampler, w.dims, dense=pb.dense64, seed=w.seed, problem_id=problem_id,
                             iteration=iteration, **kw)
    return oracle.sample(w.sampler, w.dims, coo_idx=pb.coo64, coo_val=pb.val64, seed=w.seed,
                         problem_id=problem_id, iteration=iteration, **kw)


def oracle_grad(pb: Problem, smp, **over):
    w = pb.w
    return oracle.grad(w.loss, w.dims, pb.A64, smp, nnz=w.nnz, s=over.get("s", w.s),
                       p=over.get("p", w.p), q=over.get("q", w.q), want_ytilde=True)


def cfg_for(pb: Problem, iteration: int = 0, problem_id: int = 0, rho: float = 0.0, **over):
    w = pb.w
    return gcp.sampling(w.sampler, s=over.get("s", w.s), p=over.get("p", w.p), q=over.get("q", w.q),
                        seed=w.seed, problem_id=problem_id, iteration=iteration, rho=rho)


def rel_fro(gpu_list, ref_list) -> List[float]:
    out = []
    for g, r in zip(gpu_list, ref_list):
        g = g.detach().to(torch.float64).cpu().numpy()
        den = float(np.linalg.norm(r))
        out.append(float(np.linalg.norm(g - r)) / (den if den > 0 else 1.0))
    return out


# ---------------------------------------------------------------------------
# small seeded problems with ragged sizes
# ---------------------------------------------------------------------------

def small_dense(dims=(13, 17, 11), rank=5, s=3001, dtype="f32", loss=synth.GAUSSIAN, seed=501):
    X, _ = synth.dense_gaussian(dims, rank, seed=seed)
    A0 = synth.gaussian_start(dims, rank, seed=seed + 1)
    if loss in (synth.GAMMA, synth.BETA_HALF):
        X = np.abs(X) + 0.05
        A0 = [np.abs(a) + 0.05 for a in A0]
    elif loss != synth.GAUSSIAN:
        X = np.round(np.abs(X)) if loss == synth.POISSON else (np.abs(X) > 1.0).astype(float)
        A0 = [np.abs(a) + 0.05 for a in A0]
    return synth.Workload(f"dense{dims}", tuple(dims), rank, loss, synth.UNIFORM, dtype, s=s, dense=X,
                          A_init=A0, seed=seed + 2, lr=1e-3)


def small_sparse(kind="binary", dims=(61, 47, 33), rank=7, p=2111, q=3333, sampler=None, dtype="f32",
                 seed=601, loss=None):
    loss_override = loss
    if kind == "binary":
        coo, val, _, scale = synth.sparse_binary(dims, rank, 0.03, seed=seed, subsample=50000)
        A0 = synth.nonneg_start(dims, rank, seed + 1, "uniform", scale)
        loss = synth.BERNOULLI_ODDS
        sampler = synth.STRATIFIED if sampler is None else sampler
    else:
        omega = math.prod(dims)
        coo, val, _, scale = synth.sparse_counts(dims, rank, 0.04 * omega, seed=seed, subsample=50000)
        A0 = synth.nonneg_start(dims, rank, seed + 1, "gamma", scale)
        loss = synth.POISSON
        sampler = synth.SEMI_STRATIFIED if sampler is None else sampler
    return synth.Workload(f"{kind}{dims}", tuple(dims), rank, loss if loss_override is None else loss_override,
                          sampler, dtype, p=p, q=q, coo_idx=coo, coo_val=val, A_init=A0, seed=seed + 2, lower=0.0)
