"""Seeded synthetic inputs shaped like the paper's workloads.

This module only makes inputs: data tensors, true factors and starting
factors.  It holds none of the sampled-gradient arithmetic (no sampling, no
loss derivative, no MTTKRP, no Adam); both the HIP path and the oracle consume
what it returns.  Every array comes from numpy's PCG64 with a fixed seed and a
fixed traversal order, so the same call gives the same bytes on any machine.

Workloads (dims, rank, loss, sampler; data recipe):

* ``dense_gaussian_30x40x50`` -- 30x40x50, rank 4, FP64.  X = [[A1,A2,A3]] with
  N(0,1) factor entries plus 0.1*N(0,1) noise; Gaussian loss; uniform sampling,
  s = 2000; evaluated at an independent N(0,1) start.
* ``sparse_binary_1000x800x600`` -- binary, rank 8, FP32.  Factor entries
  U(0,1); the model is scaled by lambda so that the mean odds-probability
  lambda*m/(1+lambda*m) is 0.002; every entry is drawn Bernoulli(lambda*m/(1+lambda*m))
  (the odds link of the paper's binary recipe).  Bernoulli-odds loss,
  stratified sampling p = q = 1e5.
* ``sparse_count_6000x24x77x32`` -- counts, rank 10, FP32.  Factor entries
  Gamma(0.5, 1); the model is scaled so that the expected number of nonzeros
  sum(1 - exp(-lambda*m)) is 5e6; entries are Poisson(lambda*m).  Poisson loss,
  semi-stratified sampling p = q = 5e5.  Stands in for the Chicago crime
  tensor (6186x24x77x32, 5.3M nonzeros, rank 10), which is not available.
* ``dense_gaussian_200x200x200x200`` -- 200^4, rank 32, FP32 data (6.4 GB,
  generated in slabs).  X = [[A1..A4]] with N(0,1) factor entries plus
  0.1*N(0,1) noise; Gaussian loss; uniform sampling, s = 1e6; factors stored
  in FP32 or BF16 (``_bf16``); evaluated at an independent N(0,1) start.
* ``dense_gamma_200x150x100x50`` -- the Gamma test problem of App. C at the
  shape and rank of the paper's Gamma study (Sec. 5.2): U(0,1) factors, rank
  5, entries Gamma(shape 1, mean m); FP32 data (600 MB); uniform sampling.
* ``batch_of_cubes`` -- 64 dense cubes, sides round(exp(U(ln 20, ln 300))),
  ranks uniform over {4, 8, 16, 32}, losses b mod 3 with the data of the
  recipes above, s = ceil(2% of the entries) uniform samples each.

Seeds: data 1000c+1, start 1000c+2, samples 1000c+3 for workload c = 1..4.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
import os
from typing import List, Optional

import numpy as np

GAUSSIAN, BERNOULLI_ODDS, POISSON, GAMMA, BETA_HALF = 0, 1, 2, 3, 4
UNIFORM, STRATIFIED, SEMI_STRATIFIED = 0, 1, 2

_CACHE = os.environ.get("GCP_DATA_CACHE",
                        os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                     "data_cache"))


@dataclasses.dataclass
class Workload:
    name: str
    dims: tuple
    rank: int
    loss: int
    sampler: int
    dtype: str                       # factor storage: "f64", "f32" or "bf16"
    s: int = 0                       # uniform samples
    p: int = 0                       # nonzero samples
    q: int = 0                       # zero samples
    dense: Optional[np.ndarray] = None        # row-major dense X
    coo_idx: Optional[np.ndarray] = None      # [nnz, d] uint32, sorted by row-major linear index
    coo_val: Optional[np.ndarray] = None      # [nnz]
    A_true: Optional[List[np.ndarray]] = None
    A_init: Optional[List[np.ndarray]] = None
    seed: int = 0                    # sample stream seed
    lower: float = -np.inf           # projection bound of the Adam step
    lr: float = 0.01

    @property
    def d(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return 0 if self.coo_idx is None else int(self.coo_idx.shape[0])

    @property
    def omega(self) -> int:
        return int(np.prod(np.array(self.dims, dtype=object)))

    @property
    def n_samples(self) -> int:
        return self.s if self.sampler == UNIFORM else self.p + self.q


# ---------------------------------------------------------------------------
# small building blocks
# ---------------------------------------------------------------------------

def _full(A: List[np.ndarray]) -> np.ndarray:
    """Dense tensor of a CP model (data construction only)."""
    d = len(A)
    letters = "abcdefgh"[:d]
    spec = ",".join(f"{c}z" for c in letters) + "->" + letters
    return np.einsum(spec, *A, optimize=True)


def dense_gaussian(dims, rank, seed, noise=0.1, dtype=np.float64):
    """X = [[A_1..A_d]] + noise*N(0,1), factors N(0,1); returns (X, A_true)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = [rng.standard_normal((n, rank)) for n in dims]
    X = _full(A) + noise * rng.standard_normal(tuple(dims))
    return X.astype(dtype), [a.astype(dtype) for a in A]


def gaussian_start(dims, rank, seed, dtype=np.float64):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal((n, rank)).astype(dtype) for n in dims]


def _slab_models(A, lam):
    """Yield (slab index, lambda * model values of that mode-0 slab)."""
    rest = A[1:]
    for i0 in range(A[0].shape[0]):
        B = [rest[0] * A[0][i0]] + rest[1:]
        yield i0, lam * _full(B)


def _subsample_models(A, count, rng):
    idx = [rng.integers(0, a.shape[0], size=count) for a in A]
    prod = np.ones((count, A[0].shape[1]))
    for k, a in enumerate(A):
        prod *= a[idx[k]]
    return prod.sum(axis=1)


def _bisect_scale(target, func, lo=1e-12, hi=1e12, iters=80):
    """Scale lambda (geometric bisection) with func(lambda) = target, func increasing."""
    for _ in range(iters):
        mid = np.sqrt(lo * hi)
        if func(mid) < target:
            lo = mid
        else:
            hi = mid
    return np.sqrt(lo * hi)


def sparse_binary(dims, rank, density, seed, subsample=2_000_000):
    """Binary tensor, entries Bernoulli(lam*m/(1+lam*m)); factors U(0,1).

    lambda is chosen on a seeded subsample of entries so that the mean
    probability is ``density``; factors are returned scaled by lambda^(1/d).
    Returns (coo_idx uint32 [nnz, d], coo_val float64 ones, A_true, lambda^(1/d)).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    d = len(dims)
    A = [rng.random((n, rank)) for n in dims]
    msub = _subsample_models(A, subsample, rng)
    lam = _bisect_scale(density, lambda l: float(np.mean(l * msub / (1.0 + l * msub))))
    coords = []
    for i0, m in _slab_models(A, lam):
        u = rng.random(m.shape)
        hit = np.nonzero(u < m / (1.0 + m))
        if hit[0].size:
            c = np.empty((hit[0].size, d), dtype=np.uint32)
            c[:, 0] = i0
            for k in range(1, d):
                c[:, k] = hit[k - 1]
            coords.append(c)
    coo = np.concatenate(coords) if coords else np.zeros((0, d), dtype=np.uint32)
    scale = lam ** (1.0 / d)
    return coo, np.ones(coo.shape[0]), [a * scale for a in A], scale


def _poisson_inverse_cdf(mu, v):
    """Smallest k >= 1 with CDF_Poisson(mu)(k) >= v, for v > exp(-mu) (vectorised)."""
    pmf = np.exp(-mu)
    cdf = pmf.copy()
    k = np.zeros(mu.shape, dtype=np.int64)
    todo = np.ones(mu.shape, dtype=bool)
    while todo.any():
        k[todo] += 1
        pmf[todo] = pmf[todo] * mu[todo] / k[todo]
        cdf[todo] += pmf[todo]
        todo &= cdf < v
        todo &= k < 10_000
    return k


def sparse_counts(dims, rank, nnz_target, seed, subsample=2_000_000):
    """Count tensor, entries Poisson(lam*m); factors Gamma(0.5, 1).

    lambda is chosen on a seeded subsample so that the expected number of
    nonzeros sum(1 - exp(-lam*m)) is ``nnz_target``.  Each entry uses one
    uniform v: it is zero when v <= exp(-lam*m), else the Poisson inverse CDF
    at v.  Returns (coo_idx uint32 [nnz, d], coo_val float64, A_true scaled
    by lambda^(1/d), lambda^(1/d)).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    d = len(dims)
    A = [rng.gamma(0.5, 1.0, size=(n, rank)) for n in dims]
    omega = float(np.prod(np.array(dims, dtype=np.float64)))
    msub = _subsample_models(A, subsample, rng)
    lam = _bisect_scale(nnz_target / omega, lambda l: float(np.mean(-np.expm1(-l * msub))))
    coords, vals = [], []
    for i0, m in _slab_models(A, lam):
        v = rng.random(m.shape)
        hit = np.nonzero(v > np.exp(-m))
        if hit[0].size:
            c = np.empty((hit[0].size, d), dtype=np.uint32)
            c[:, 0] = i0
            for k in range(1, d):
                c[:, k] = hit[k - 1]
            coords.append(c)
            vals.append(_poisson_inverse_cdf(m[hit], v[hit]).astype(np.float64))
    coo = np.concatenate(coords) if coords else np.zeros((0, d), dtype=np.uint32)
    val = np.concatenate(vals) if vals else np.zeros(0)
    scale = lam ** (1.0 / d)
    return coo, val, [a * scale for a in A], scale


def nonneg_start(dims, rank, seed, kind, scale):
    """Positive start: same distribution and scale as the true factors, new seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "uniform":
        return [rng.random((n, rank)) * scale for n in dims]
    return [rng.gamma(0.5, 1.0, size=(n, rank)) * scale for n in dims]


# ---------------------------------------------------------------------------
# cache (numpy .npz, no pickles)
# ---------------------------------------------------------------------------

def _cached(key: str, make):
    os.makedirs(_CACHE, exist_ok=True)
    h = hashlib.sha1(key.encode()).hexdigest()[:16]
    path = os.path.join(_CACHE, f"{h}.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            return {k: z[k] for k in z.files}
    out = make()
    tmp = path + f".tmp{os.getpid()}.npz"
    np.savez(tmp, **out)
    os.replace(tmp, path)
    return out


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def dense_gaussian_30x40x50() -> Workload:
    dims, r = (30, 40, 50), 4
    X, A_true = dense_gaussian(dims, r, seed=1001)
    A0 = gaussian_start(dims, r, seed=1002)
    return Workload("dense_gaussian_30x40x50", dims, r, GAUSSIAN, UNIFORM, "f64", s=2000,
                    dense=X, A_true=A_true, A_init=A0, seed=1003, lr=1e-3)


def sparse_binary_workload(dims=(1000, 800, 600), rank=8, density=0.002, p=100_000, q=100_000,
                           seed_base=2000, name=None, cache=True) -> Workload:
    d = len(dims)

    def make():
        coo, val, A_true, scale = sparse_binary(dims, rank, density, seed=seed_base + 1)
        out = {"coo": coo, "val": val, "scale": np.array(scale)}
        for k, a in enumerate(A_true):
            out[f"A{k}"] = a
        return out

    key = f"sparse_binary:{dims}:{rank}:{density}:{seed_base}:v3"
    z = _cached(key, make) if cache else make()
    A_true = [z[f"A{k}"] for k in range(d)]
    A0 = nonneg_start(dims, rank, seed_base + 2, "uniform", float(z["scale"]))
    return Workload(name or f"sparse_binary_{'x'.join(map(str, dims))}", tuple(dims), rank,
                    BERNOULLI_ODDS, STRATIFIED, "f32", p=p, q=q, coo_idx=z["coo"],
                    coo_val=z["val"], A_true=A_true, A_init=A0, seed=seed_base + 3, lower=0.0)


def sparse_count_workload(dims=(6000, 24, 77, 32), rank=10, nnz_target=5.0e6, p=500_000,
                          q=500_000, seed_base=3000, name=None, cache=True) -> Workload:
    d = len(dims)

    def make():
        coo, val, A_true, scale = sparse_counts(dims, rank, nnz_target, seed=seed_base + 1)
        out = {"coo": coo, "val": val, "scale": np.array(scale)}
        for k, a in enumerate(A_true):
            out[f"A{k}"] = a
        return out

    key = f"sparse_counts:{dims}:{rank}:{nnz_target}:{seed_base}:v3"
    z = _cached(key, make) if cache else make()
    A_true = [z[f"A{k}"] for k in range(d)]
    A0 = nonneg_start(dims, rank, seed_base + 2, "gamma", float(z["scale"]))
    return Workload(name or f"sparse_count_{'x'.join(map(str, dims))}", tuple(dims), rank,
                    POISSON, SEMI_STRATIFIED, "f32", p=p, q=q, coo_idx=z["coo"], coo_val=z["val"],
                    A_true=A_true, A_init=A0, seed=seed_base + 3, lower=0.0)


def dense_gaussian_4way_f32(dims=(200, 200, 200, 200), rank=32, noise=0.1, seed=4001, chunk_rows=1000):
    """FP32 X = [[A_1..A_4]] + noise*N(0,1) with N(0,1) factors, generated in
    slabs of the (n_1 n_2) x (n_3 n_4) matricization: the model part as a
    float64 product of Khatri-Rao factors rounded to float32, the noise from
    one sequential float32 normal stream.  Returns (X, A_true)."""
    assert len(dims) == 4
    rng = np.random.Generator(np.random.PCG64(seed))
    A = [rng.standard_normal((n, rank)) for n in dims]
    left = (A[0][:, None, :] * A[1][None, :, :]).reshape(dims[0] * dims[1], rank)
    right = (A[2][:, None, :] * A[3][None, :, :]).reshape(dims[2] * dims[3], rank)
    X = np.empty((dims[0] * dims[1], dims[2] * dims[3]), dtype=np.float32)
    for r0 in range(0, X.shape[0], chunk_rows):
        r1 = min(r0 + chunk_rows, X.shape[0])
        X[r0:r1] = left[r0:r1] @ right.T
        X[r0:r1] += np.float32(noise) * rng.standard_normal((r1 - r0, X.shape[1]), dtype=np.float32)
    return X.reshape(dims), A


def dense_gaussian_200x200x200x200(dtype="f32", s=1_000_000) -> Workload:
    """200^4 Gaussian, rank 32, FP32 data (6.4 GB), uniform s = 1e6; factors in
    FP32 or BF16 storage (BF16: FP32 master, BF16 copy for the gathers)."""
    dims, r = (200, 200, 200, 200), 32
    X, A_true = dense_gaussian_4way_f32(dims, r, seed=4001)
    A0 = gaussian_start(dims, r, seed=4002)
    name = "dense_gaussian_200x200x200x200" + ("_bf16" if dtype == "bf16" else "")
    return Workload(name, dims, r, GAUSSIAN, UNIFORM, dtype, s=s, dense=X, A_true=A_true, A_init=A0,
                    seed=4003, lr=1e-3)


def kruskal_norm(A) -> float:
    """Frobenius norm of the CP model [[A_1, ..., A_d]] from the Gram
    matrices: ||M||^2 = sum over component pairs of the product over modes of
    (A_k^T A_k)."""
    G = np.ones((A[0].shape[1], A[0].shape[1]))
    for a in A:
        G *= a.T @ a
    return float(math.sqrt(max(G.sum(), 0.0)))


def sparse_binary_appd(dims, rank, delta=0.15, p_high=0.9, p_low=0.002, seed=0):
    """Binary test problem of the paper's App. D (odds link): components 1..r-1
    have sparse factor columns (each entry nonzero with probability delta,
    value |N(c_high, 0.5)| with c_high = (p_high / (1 - p_high))^(1/d)); the
    last component is dense with every entry c_low = (p_low / (1 - p_low))^(1/d),
    so away from the sparse components a one has probability p_low.  Entries
    inside some sparse component's support get their exact probability
    m/(1+m) and one Bernoulli draw each; the p_low ones elsewhere are drawn in
    bulk (a binomial count of distinct uniform keys outside those supports).
    Returns (coo_idx uint32 [nnz, d] sorted by linear key, values ones, A_true)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = len(dims)
    dims = tuple(int(n) for n in dims)
    c_high = (p_high / (1.0 - p_high)) ** (1.0 / d)
    c_low = (p_low / (1.0 - p_low)) ** (1.0 / d)
    A = []
    for n in dims:
        a = np.zeros((n, rank))
        for j in range(rank - 1):
            hit = rng.random(n) < delta
            a[hit, j] = np.abs(rng.normal(c_high, 0.5, size=int(hit.sum())))
        a[:, rank - 1] = c_low
        A.append(a)
    strides = np.ones(d, dtype=np.int64)
    for k in range(d - 2, -1, -1):
        strides[k] = strides[k + 1] * dims[k + 1]
    keys = []
    for j in range(rank - 1):
        sup = [np.nonzero(A[k][:, j])[0].astype(np.int64) for k in range(d)]
        grid = np.zeros(1, dtype=np.int64)
        for k in range(d):
            grid = (grid[:, None] + (sup[k] * strides[k])[None, :]).reshape(-1)
        keys.append(grid)
    cand = np.unique(np.concatenate(keys)) if keys else np.zeros(0, dtype=np.int64)
    idx = np.stack([(cand // strides[k]) % dims[k] for k in range(d)], axis=1)
    m = np.full(cand.shape[0], c_low ** d)
    for j in range(rank - 1):
        prod = np.ones(cand.shape[0])
        for k in range(d):
            prod *= A[k][idx[:, k], j]
        m += prod
    ones_c = cand[rng.random(cand.shape[0]) < m / (1.0 + m)]
    omega = int(np.prod(np.array(dims, dtype=object)))
    n_noise = int(rng.binomial(omega - cand.shape[0], p_low))
    noise = np.zeros(0, dtype=np.int64)
    while noise.shape[0] < n_noise:
        draw = rng.integers(0, omega, size=(n_noise - noise.shape[0]) * 11 // 10 + 16, dtype=np.int64)
        draw = draw[~np.isin(draw, cand)]
        noise = np.unique(np.concatenate([noise, draw]))
    noise = rng.permutation(noise)[:n_noise]
    nz = np.sort(np.concatenate([ones_c, noise]))
    coo = np.stack([(nz // strides[k]) % dims[k] for k in range(d)], axis=1).astype(np.uint32)
    return coo, np.ones(coo.shape[0]), A


def sparse_binary_400x300x200x100(cache=True):
    """The sampler-comparison tensor of the paper's Sec. 5.4 (Table 1): App. D
    recipe with delta = 0.15, p_high = 0.9, p_low = 0.002, rank 5."""
    dims, r = (400, 300, 200, 100), 5

    def make():
        coo, val, A = sparse_binary_appd(dims, r, 0.15, 0.9, 0.002, seed=7001)
        out = {"coo": coo, "val": val}
        for k, a in enumerate(A):
            out[f"A{k}"] = a
        return out

    z = _cached(f"appd:{dims}:{r}:7001:v1", make) if cache else make()
    A_true = [z[f"A{k}"] for k in range(len(dims))]
    # start (Sec. 5.4): U(0,1) factors scaled so that the model's Frobenius
    # norm equals the data's, sqrt(nnz) for a binary tensor
    rng = np.random.Generator(np.random.PCG64(7002))
    A0 = [rng.random((n, r)) for n in dims]
    A0 = [a * (math.sqrt(z["coo"].shape[0]) / kruskal_norm(A0)) ** (1.0 / len(dims)) for a in A0]
    return Workload("sparse_binary_400x300x200x100", dims, r, BERNOULLI_ODDS, STRATIFIED, "f32", p=500, q=500,
                    coo_idx=z["coo"], coo_val=z["val"], A_true=A_true, A_init=A0, seed=7003, lower=0.0)


def dense_gamma(dims, rank, seed):
    """Gamma test problem of the paper's App. C: factor entries U(0,1); every
    entry x ~ Gamma(shape 1, mean m) (exponential with mean m).  Returns
    (X float64, A_true)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = [rng.random((n, rank)) for n in dims]
    M = _full(A)
    X = rng.exponential(1.0, size=M.shape) * M
    return X, A


def dense_gamma_200x150x100x50(s=2000) -> Workload:
    """The shape and rank of the paper's Gamma study (Sec. 5.2): 200x150x100x50,
    rank 5, FP32 data (600 MB), uniform sampling, nonnegative factors."""
    dims, r = (200, 150, 100, 50), 5
    X, A_true = dense_gamma(dims, r, seed=6001)
    rng = np.random.Generator(np.random.PCG64(6002))
    A0 = [rng.random((n, r)) for n in dims]
    return Workload("dense_gamma_200x150x100x50", dims, r, GAMMA, UNIFORM, "f32", s=s, dense=X.astype(np.float32),
                    A_true=A_true, A_init=A0, seed=6003, lower=0.0)


def sparse_binary_1000x800x600() -> Workload:
    return sparse_binary_workload()


def sparse_count_6000x24x77x32() -> Workload:
    return sparse_count_workload()


WORKLOADS = {
    "dense_gaussian_30x40x50": dense_gaussian_30x40x50,
    "sparse_binary_1000x800x600": sparse_binary_1000x800x600,
    "sparse_count_6000x24x77x32": sparse_count_6000x24x77x32,
    "dense_gaussian_200x200x200x200": dense_gaussian_200x200x200x200,
    "dense_gaussian_200x200x200x200_bf16": lambda: dense_gaussian_200x200x200x200("bf16"),
    "dense_gamma_200x150x100x50": dense_gamma_200x150x100x50,
}


# ---------------------------------------------------------------------------
# batches of dense problems
# ---------------------------------------------------------------------------

def dense_problem(n_dims, rank, loss, seed, density=None):
    """A dense problem with the recipe of its loss: Gaussian N(0,1) factors plus
    0.1 noise; Poisson counts from Gamma(0.5,1) factors scaled to `density`
    nonzeros; Bernoulli(odds) from U(0,1) factors scaled to mean probability
    `density`; Gamma and beta-divergence: shape-1 Gamma data with mean m from
    U(0,1) factors.  Returns (X float64 dense, start factors, projection bound)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = tuple(n_dims)
    d = len(dims)
    if loss == GAUSSIAN:
        A = [rng.standard_normal((n, rank)) for n in dims]
        X = _full(A) + 0.1 * rng.standard_normal(dims)
        A0 = [rng.standard_normal((n, rank)) for n in dims]
        return X, A0, -np.inf
    if loss in (GAMMA, BETA_HALF):
        # positive data: shape-1 Gamma with mean m from U(0,1) factors (App. C)
        A = [rng.random((n, rank)) for n in dims]
        X = rng.exponential(1.0, size=dims) * _full(A)
        A0 = [rng.random((n, rank)) for n in dims]
        return X, A0, 0.0
    if loss == POISSON:
        A = [rng.gamma(0.5, 1.0, size=(n, rank)) for n in dims]
        M = _full(A)
        sub = rng.choice(M.reshape(-1), size=min(M.size, 200_000), replace=False)
        target = density if density is not None else 5.0e6 / (6000 * 24 * 77 * 32)
        lam = _bisect_scale(target, lambda l: float(np.mean(-np.expm1(-l * sub))))
        X = rng.poisson(lam * M).astype(np.float64)
        scale = lam ** (1.0 / d)
        A0 = [rng.gamma(0.5, 1.0, size=(n, rank)) * scale for n in dims]
        return X, A0, 0.0
    A = [rng.random((n, rank)) for n in dims]
    M = _full(A)
    sub = rng.choice(M.reshape(-1), size=min(M.size, 200_000), replace=False)
    target = density if density is not None else 0.002
    lam = _bisect_scale(target, lambda l: float(np.mean(l * sub / (1.0 + l * sub))))
    X = (rng.random(dims) < lam * M / (1.0 + lam * M)).astype(np.float64)
    scale = lam ** (1.0 / d)
    A0 = [rng.random((n, rank)) * scale for n in dims]
    return X, A0, 0.0


def batch_of_cubes(count=64, side_lo=20, side_hi=300, ranks=(4, 8, 16, 32), frac=0.02, seed_base=5000,
                   cache=True):
    """`count` dense 3-way cubes: side round(exp(U(ln lo, ln hi))), rank uniform
    over `ranks`, loss b mod 3 (Gaussian, Poisson, Bernoulli-odds), uniform
    sampling of ceil(frac * side^3) entries, FP32.  Problem b draws with seed
    seed_base + 3 and problem_id b."""
    rng = np.random.Generator(np.random.PCG64(seed_base + 4))
    sides = np.rint(np.exp(rng.uniform(np.log(side_lo), np.log(side_hi), size=count))).astype(int)
    rks = rng.choice(np.array(ranks), size=count)
    out = []
    for b in range(count):
        n, r, loss = int(sides[b]), int(rks[b]), [GAUSSIAN, POISSON, BERNOULLI_ODDS][b % 3]

        def make(n=n, r=r, loss=loss, b=b):
            X, A0, lower = dense_problem((n, n, n), r, loss, seed=seed_base * 1000 + 1 + 7 * b)
            z = {"X": X.astype(np.float32), "lower": np.array(lower)}
            for k, a in enumerate(A0):
                z[f"A{k}"] = a
            return z

        key = f"cube:{n}:{r}:{loss}:{seed_base}:{b}:v2"
        z = _cached(key, make) if cache else make()
        s = int(np.ceil(frac * n ** 3))
        w = Workload(f"cube{b}_{n}_r{r}", (n, n, n), r, loss, UNIFORM, "f32", s=s, dense=z["X"],
                     A_init=[z[f"A{k}"] for k in range(3)], seed=seed_base + 3, lower=float(z["lower"]))
        w.problem_id = b
        out.append(w)
    return out
