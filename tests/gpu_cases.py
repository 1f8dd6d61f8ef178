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


# ---------------------------------------------------------------------------
# element-wise parity
#
# Every element G_k[i, j] is a sum over the samples c with i_k = i of the term
# ytilde_c * prod_{k' != k} A_k'[i_k', j] (eq. Gks).  The device forms each
# term in its compute precision (FP32 for FP32 and BF16 factors, FP64 for
# FP64): m_c with d - 1 products and a tree sum over at most 64 lanes, so its
# error is a few ulp of mabs_c = sum_j prod_k |A_k[i_k, j]|; ytilde_c = W_c g
# with g = base(m) - t(x, m) rounds to a few ulp of W_c (|base| + |t|) and
# inherits W_c (|base'| + |t'|) times the error of m; the scatter product adds
# d more roundings.  So the error of an element is a small multiple of the
# unit roundoff u times
#     E_k[i, j] = sum_c W_c (|base| + |t| + (|base'| + |t'|) mabs_c) prod_{k' != k} |A_k'[i_k', j]|
# plus the rounding of the accumulation (FP64 in LDS, or FP32 for the
# partials and device rows that do not fit, where the sum of n terms of
# random sign stays near sqrt(n) u of the sum of their magnitudes).  The test
# bar is |G_dev - G_oracle| <= tol * E_k element by element, with tol = 1e-5
# for FP32 arithmetic (u = 6e-8: ~20 roundings per term leave a margin of 8)
# and 1e-12 for FP64 (u = 1.1e-16).  Elements no sample touches (E = 0) must be
# exactly 0.  The per-mode relative Frobenius error stays a second bar.
# ---------------------------------------------------------------------------

def _loss_magnitudes(loss: int, x: np.ndarray, m: np.ndarray, eps: float):
    """|base| + |t| and |base'| + |t'| of g = base(m) - t(x, m) for each loss."""
    u = m + eps
    ax = np.abs(x)
    if loss == synth.GAUSSIAN:
        return 2 * np.abs(m) + 2 * ax, np.full_like(m, 2.0)
    if loss == synth.BERNOULLI_ODDS:
        return np.abs(1 / (m + 1)) + ax / np.abs(u), 1 / (m + 1) ** 2 + ax / u ** 2
    if loss == synth.POISSON:
        return 1 + ax / np.abs(u), ax / u ** 2
    if loss == synth.GAMMA:
        return 1 / np.abs(u) + ax / u ** 2, 1 / u ** 2 + 2 * ax / np.abs(u) ** 3
    if loss == synth.BETA_HALF:
        return u ** -0.5 + ax * u ** -1.5, 0.5 * u ** -1.5 + 1.5 * ax * u ** -2.5
    raise ValueError(loss)


def grad_scale(loss: int, dims, A64, smp, *, nnz: int = 0, s: int = 0, p: int = 0, q: int = 0, ew=None,
               w_zero: float = 1.0, eps: float = oracle.LOSS_EPS) -> List[np.ndarray]:
    """E_k of the element-wise bar above, for the oracle's samples ``smp`` and
    entry weights ``ew`` (None: unweighted)."""
    d = len(dims)
    r = A64[0].shape[1]
    S = len(smp)
    if S == 0:
        return [np.zeros((n, r)) for n in dims]
    omega = float(math.prod(int(n) for n in dims))
    eta = float(nnz)
    st = np.asarray(smp.stratum)
    sw = np.zeros(S)
    sw[st == oracle.S_UNIFORM] = omega / max(s, 1)
    sw[st == oracle.S_NZ] = eta / max(p, 1)
    sw[st == oracle.S_ZERO] = (omega - eta) / max(q, 1)
    sw[st == oracle.S_NZ_CORR] = eta / max(p, 1)
    sw[st == oracle.S_SEMI_ZERO] = omega / max(q, 1)
    e = np.ones(S) if ew is None else np.abs(np.asarray(ew, dtype=np.float64))
    W = sw * e
    corr = st == oracle.S_NZ_CORR
    W[corr] = sw[corr] * (e[corr] + (abs(w_zero) if ew is not None else 1.0))
    idx = np.asarray(smp.idx, dtype=np.int64)
    rows = [np.asarray(A64[k], dtype=np.float64)[idx[:, k]] for k in range(d)]
    prod = np.ones((S, r))
    for k in range(d):
        prod *= rows[k]
    m = prod.sum(axis=1)
    mabs = np.abs(prod).sum(axis=1)
    mag, sens = _loss_magnitudes(loss, np.asarray(smp.xval, dtype=np.float64), m, eps)
    Y = W * (mag + sens * mabs)
    cols = np.arange(r)
    out = []
    for k in range(d):
        z = np.ones((S, r))
        for k2 in range(d):
            if k2 != k:
                z *= np.abs(rows[k2])
        lin = (idx[:, k][:, None] * r + cols[None, :]).reshape(-1)
        out.append(np.bincount(lin, weights=(Y[:, None] * z).reshape(-1), minlength=int(dims[k]) * r)
                   .reshape(int(dims[k]), r))
    return out


def check_grad(gpu_list, ref_list, scale, tol: float, label: str = "") -> None:
    """The element-wise bar |G_dev - G_oracle| <= tol * E_k plus the per-mode
    relative Frobenius bar; prints max-abs, relative Frobenius and the largest
    error-to-scale ratio of every mode."""
    for k, (g, ref, E) in enumerate(zip(gpu_list, ref_list, scale)):
        g = (g.detach().to(torch.float64).cpu().numpy() if torch.is_tensor(g) else np.asarray(g, np.float64))
        g = g.reshape(ref.shape)
        diff = np.abs(g - ref)
        den = float(np.linalg.norm(ref))
        rf = float(np.linalg.norm(g - ref)) / (den if den > 0 else 1.0)
        touched = E > 0
        ratio = float(np.max(diff[touched] / E[touched])) if touched.any() else 0.0
        untouched = float(np.max(diff[~touched])) if (~touched).any() else 0.0
        print(f"[parity] {label} mode {k}: max-abs {float(diff.max()):.3e} (max |G| {float(np.abs(ref).max()):.3e}), "
              f"rel-fro {rf:.2e}, max err/scale {ratio:.2e}", flush=True)
        assert untouched == 0.0, (label, k, "untouched element differs", untouched)
        assert ratio <= tol, (label, k, "element-wise", ratio)
        assert rf <= tol, (label, k, "relative Frobenius", rf)


def oracle_scale(pb: "Problem", smp, **over) -> List[np.ndarray]:
    w = pb.w
    return grad_scale(w.loss, w.dims, pb.A64, smp, nnz=w.nnz, s=over.get("s", w.s), p=over.get("p", w.p),
                      q=over.get("q", w.q))


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


def with_zero_factors(w: synth.Workload, seed: int = 17) -> synth.Workload:
    """The same workload at a start holding exact zeros, as the projection onto
    A >= 0 of Alg. 4 leaves them: a fifth of the rows of every mode and one
    whole column of the first mode set to 0.  Samples whose rows are all zero
    have m = 0 exactly, so x / (m + eps) reaches x / eps = 1e10 x."""
    rng = np.random.default_rng(seed)
    A = [np.array(a, dtype=np.float64, copy=True) for a in w.A_init]
    for a in A:
        a[rng.random(a.shape[0]) < 0.2, :] = 0.0
    A[0][:, 0] = 0.0
    return dataclasses.replace(w, name=w.name + "_zeros", A_init=A)

