"""Independent checks ("pins") for the FP64 oracle.

Each ``pin_*`` function computes something the paper or the mathematics fixes
by a route other than the oracle's own code, compares, and returns
``(ok, detail)``.  ``tests/test_oracle_pins.py`` asserts every pin holds;
``tests/test_oracle_mutations.py`` plants each deliberate mistake in the oracle
and asserts that at least one pin catches it.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special
import scipy.stats

import oracle
import synth

MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# independent re-derivations
# ---------------------------------------------------------------------------

def numpy_philox_block(key, counter):
    """Philox4x64-10 block at ``counter`` via numpy (which increments first)."""
    c = [int(x) for x in counter]
    pred = (c[0] | (c[1] << 64) | (c[2] << 128) | (c[3] << 192)) - 1
    pred &= (1 << 256) - 1
    words = np.array([(pred >> (64 * t)) & MASK64 for t in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([int(key[0]), int(key[1])], dtype=np.uint64), counter=words)
    return bg.random_raw(4)


def numpy_index(seed, pid, j, iteration, purpose, dims):
    """Mode indices of draw j: word k -> floor(w_k * n_k / 2^64), exact integers."""
    out = []
    blocks = {}
    for k, n in enumerate(dims):
        b = k // 4
        if b not in blocks:
            blocks[b] = numpy_philox_block((seed, pid), (j, iteration, purpose, b))
        w = int(blocks[b][k % 4])
        out.append((w * int(n)) >> 64)
    return tuple(out)


def khatri_rao(mats, r=None):
    """Column-wise Kronecker product; the first matrix varies slowest.  The
    product of no matrices is the 1 x r row of ones (a one-way model has
    m_i = sum_j a_ij, so its leave-one-out factor is 1)."""
    if not mats:
        return np.ones((1, r))
    out = mats[0]
    for m in mats[1:]:
        out = (out[:, None, :] * m[None, :, :]).reshape(-1, out.shape[1])
    return out


def unfold(T, k):
    """Mode-k unfolding; remaining modes in order, last fastest (row-major)."""
    return np.moveaxis(T, k, 0).reshape(T.shape[k], -1)


def full_model(A):
    d = len(A)
    letters = "abcdefgh"[:d]
    return np.einsum(",".join(f"{c}z" for c in letters) + "->" + letters, *A)


def exact_gradient(loss, X, A, eps=oracle.LOSS_EPS, W=None):
    """G_k = Y_(k) Z_k (eqs. Y, Gk) with explicit unfolding and Khatri-Rao
    product; with entry weights W, y_i = w_i g(x_i, m_i) (eq. wgcp)."""
    M = full_model(A)
    gvec = np.vectorize(lambda x, m: oracle.loss_g(loss, float(x), float(m), eps))
    Y = gvec(X, M)
    if W is not None:
        Y = Y * W
    G = []
    for k in range(len(A)):
        Z = khatri_rao([A[j] for j in range(len(A)) if j != k], A[k].shape[1])
        G.append(unfold(Y, k) @ Z)
    return G


def exact_loss(loss, X, A, eps=oracle.LOSS_EPS, W=None):
    """F(X, M) = sum_i f(x_i, m_i) over every entry (eq. gcp); with entry
    weights W, sum_i w_i f(x_i, m_i) (eq. wgcp)."""
    M = full_model(A)
    fvec = np.vectorize(lambda x, m: oracle.loss_f(loss, float(x), float(m), eps))
    Fm = fvec(X, M)
    if W is not None:
        Fm = Fm * W
    return float(Fm.sum())


def enumeration_samples(dims, X):
    """Every index once, uniform stratum, in row-major order (s = number of entries)."""
    grids = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    idx = np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.int64)
    S = idx.shape[0]
    return oracle.Samples(idx, np.asarray(X, dtype=np.float64).reshape(-1),
                          np.zeros(S, dtype=np.int32), np.arange(S), S)


def rel_err(a_list, b_list):
    num = sum(float(np.sum((np.asarray(a) - np.asarray(b)) ** 2)) for a, b in zip(a_list, b_list))
    den = sum(float(np.sum(np.asarray(b) ** 2)) for b in b_list)
    return math.sqrt(num / max(den, 1e-300))


# ---------------------------------------------------------------------------
# tiny test problems
# ---------------------------------------------------------------------------

def tiny_dense(dims=(3, 4, 5), r=3, seed=11):
    X, _ = synth.dense_gaussian(dims, r, seed=seed)
    A = synth.gaussian_start(dims, r, seed=seed + 1)
    return X, A


def tiny_sparse(kind, dims=(6, 5, 4), r=3, seed=21):
    """Tiny binary or count tensor, its dense form, COO and a positive start."""
    if kind == "binary":
        coo, val, A_true, scale = synth.sparse_binary(dims, r, 0.2, seed=seed, subsample=20000)
        A = synth.nonneg_start(dims, r, seed + 1, "uniform", scale)
    else:
        omega = int(np.prod(dims))
        coo, val, A_true, scale = synth.sparse_counts(dims, r, 0.25 * omega, seed=seed, subsample=20000)
        A = synth.nonneg_start(dims, r, seed + 1, "gamma", scale)
    X = np.zeros(dims)
    for e in range(coo.shape[0]):
        X[tuple(int(t) for t in coo[e])] = val[e]
    return X, coo.astype(np.int64), val, A


# ---------------------------------------------------------------------------
# pins
# ---------------------------------------------------------------------------

def pin_philox_numpy(n=200, seed=5):
    """P0: oracle Philox4x64-10 == numpy.random.Philox on many keys/counters."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cases = [((0, 0), (0, 0, 0, 0)), ((MASK64, MASK64), (MASK64, MASK64, MASK64, MASK64)),
             ((1, 2), (MASK64, 0, 0, 0)), ((3, 4), (0, MASK64, 7, 1))]
    for _ in range(n):
        cases.append((tuple(int(x) for x in rng.integers(0, 2**63, 2, dtype=np.int64)),
                      tuple(int(x) for x in rng.integers(0, 2**63, 4, dtype=np.int64))))
    for key, ctr in cases:
        a = oracle.philox4x64_10(key, ctr)
        b = numpy_philox_block(key, ctr)
        if not np.array_equal(a, b):
            return False, f"key={key} ctr={ctr}: {a} != {b}"
    return True, f"{len(cases)} blocks"


def pin_randi_exact(n=2000, seed=6):
    """randi(n) == floor(w n / 2^64) in exact integer arithmetic, in range."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ws = [0, 1, MASK64, 1 << 63] + [int(x) * 2 + 1 for x in rng.integers(0, 2**63, n, dtype=np.int64)]
    ns = [1, 2, 3, 1000, 959756, 2**32 + 15, 2**63 - 25]
    for w in ws:
        for m in ns:
            got = oracle.randi(w, m)
            if got != (w * m) >> 64 or not (0 <= got < m):
                return False, f"w={w} n={m}: {got}"
    return True, "ok"


def pin_sample_streams(iteration=3, seed=77, pid=2):
    """Sample indices == the counter contract recomputed with numpy's Philox.

    Uniform (purpose 0), nonzero picks (purpose 1, xi = randi(eta)), stratified
    rejection (purpose 2, first q non-members in counter order) and semi
    "zeros" (purpose 0, no rejection) -- Alg. 1, 2, 3 sampling lines.
    """
    X, coo, val, _ = tiny_sparse("binary")
    dims = X.shape
    nz = {tuple(int(t) for t in c) for c in coo}
    eta = coo.shape[0]
    # uniform on the dense form
    smp = oracle.sample(oracle.UNIFORM, dims, dense=X, s=40, seed=seed, problem_id=pid, iteration=iteration)
    for c in range(40):
        ii = numpy_index(seed, pid, c, iteration, 0, dims)
        if tuple(smp.idx[c]) != ii or smp.xval[c] != X[ii]:
            return False, f"uniform sample {c}: {tuple(smp.idx[c])} vs {ii}"
    # stratified
    p, q = 15, 25
    smp = oracle.sample(oracle.STRATIFIED, dims, coo_idx=coo, coo_val=val, p=p, q=q, seed=seed,
                        problem_id=pid, iteration=iteration)
    for c in range(p):
        w = int(numpy_philox_block((seed, pid), (c, iteration, 1, 0))[0])
        e = (w * eta) >> 64
        if tuple(smp.idx[c]) != tuple(int(t) for t in coo[e]) or smp.stratum[c] != oracle.S_NZ:
            return False, f"nonzero pick {c}"
    accepted, j = [], 0
    while len(accepted) < q:
        ii = numpy_index(seed, pid, j, iteration, 2, dims)
        if ii not in nz:
            accepted.append((j, ii))
        j += 1
    if smp.examined != j:
        return False, f"candidates examined {smp.examined} != {j}"
    for c, (jj, ii) in enumerate(accepted):
        o = p + c
        if tuple(smp.idx[o]) != ii or smp.cand[o] != jj or smp.xval[o] != 0.0 or smp.stratum[o] != oracle.S_ZERO:
            return False, f"zero sample {c}: oracle {tuple(smp.idx[o])}@{smp.cand[o]} vs {ii}@{jj}"
    # semi-stratified
    smp = oracle.sample(oracle.SEMI_STRATIFIED, dims, coo_idx=coo, coo_val=val, p=p, q=q, seed=seed,
                        problem_id=pid, iteration=iteration)
    for c in range(q):
        ii = numpy_index(seed, pid, c, iteration, 0, dims)
        o = p + c
        if tuple(smp.idx[o]) != ii or smp.xval[o] != 0.0 or smp.stratum[o] != oracle.S_SEMI_ZERO:
            return False, f"semi zero {c}"
    for c in range(p):
        if smp.stratum[c] != oracle.S_NZ_CORR:
            return False, "semi nonzero stratum"
    return True, "ok"


def pin_stratified_zeros_are_zeros():
    """P5: stratified zero samples never hit a nonzero; x = 0 there."""
    X, coo, val, _ = tiny_sparse("binary")
    for it in range(20):
        smp = oracle.sample(oracle.STRATIFIED, X.shape, coo_idx=coo, coo_val=val, p=5, q=60,
                            seed=9, iteration=it)
        for o in range(5, 65):
            if X[tuple(smp.idx[o])] != 0.0:
                return False, f"iteration {it}: zero sample {o} hit a nonzero"
    return True, "ok"


def pin_index_uniformity(seed=1234):
    """P5: per-mode histograms of uniform draws pass a chi-square test; E[count] = s/n."""
    dims = (7, 11, 5)
    X = np.zeros(dims)
    smp = oracle.sample(oracle.UNIFORM, dims, dense=X, s=20000, seed=seed)
    for k, n in enumerate(dims):
        h = np.bincount(smp.idx[:, k], minlength=n)
        pval = scipy.stats.chisquare(h).pvalue
        if pval < 1e-4:
            return False, f"mode {k} chi-square p={pval}"
    lin = np.ravel_multi_index(tuple(smp.idx.T), dims)
    h = np.bincount(lin, minlength=int(np.prod(dims)))
    pval = scipy.stats.chisquare(h).pvalue
    if pval < 1e-4:
        return False, f"joint chi-square p={pval}"
    return True, "ok"


def pin_enumeration_equals_unfolding(losses=(oracle.GAUSSIAN, oracle.BERNOULLI_ODDS, oracle.POISSON)):
    """P1: the sampled gradient over every index once (weight omega/s = 1) equals
    Y_(k) Z_k computed by explicit unfolding and Khatri-Rao products (eq. Gk)."""
    for dims in [(3, 4, 5), (2, 3, 4, 5), (7,), (3, 4), (2, 3, 2, 3, 2)]:
        for loss in losses:
            if loss == oracle.GAUSSIAN:
                X, A = tiny_dense(dims)
            else:
                X, _ = tiny_dense(dims)
                X = (np.abs(X) > 1.0).astype(float) if loss == oracle.BERNOULLI_ODDS else np.round(np.abs(X))
                A = [np.abs(a) + 0.1 for a in synth.gaussian_start(dims, 3, seed=5)]
            smp = enumeration_samples(dims, X)
            G, _ = oracle.grad(loss, dims, A, smp, s=len(smp))
            Gx = exact_gradient(loss, X, A)
            e = rel_err(G, Gx)
            if e > 1e-12:
                return False, f"dims={dims} loss={loss}: rel err {e:.3e}"
            Gf, _ = oracle.full_grad(loss, A, X)
            e = rel_err(Gf, Gx)
            if e > 1e-12:
                return False, f"full_grad dims={dims} loss={loss}: rel err {e:.3e}"
    return True, "ok"


def pin_gaussian_closed_form():
    """P2: Gaussian (standard CP) gradient in closed form (App. A):
    G_k = 2 (A_k (hadamard_{j != k} A_j^T A_j) - X_(k) Z_k), on the 30x40x50 workload."""
    w = synth.dense_gaussian_30x40x50()
    A, X = w.A_init, w.dense
    smp = enumeration_samples(w.dims, X)
    G, _ = oracle.grad(oracle.GAUSSIAN, w.dims, A, smp, s=len(smp))
    Gc = []
    for k in range(w.d):
        others = [A[j] for j in range(w.d) if j != k]
        gram = np.ones((w.rank, w.rank))
        for a in others:
            gram *= a.T @ a
        Gc.append(2.0 * (A[k] @ gram - unfold(X, k) @ khatri_rao(others)))
    e = rel_err(G, Gc)
    return e <= 1e-10, f"rel err {e:.3e}"


def pin_poisson_closed_form():
    """P3: Poisson gradient in closed form (App. A): G_k = 1 (hadamard_{j != k} 1^T A_j)
    - V_(k) Z_k with v = x / (m + eps) on the nonzeros only."""
    X, coo, val, A = tiny_sparse("counts", dims=(7, 6, 5, 4), r=3)
    dims = X.shape
    smp = enumeration_samples(dims, X)
    G, _ = oracle.grad(oracle.POISSON, dims, A, smp, s=len(smp))
    M = full_model(A)
    V = np.where(X != 0, X / (M + oracle.LOSS_EPS), 0.0)
    Gc = []
    for k in range(len(dims)):
        others = [A[j] for j in range(len(dims)) if j != k]
        colsum = np.ones(A[0].shape[1])
        for a in others:
            colsum = colsum * a.sum(axis=0)
        Gc.append(np.outer(np.ones(dims[k]), colsum) - unfold(V, k) @ khatri_rao(others))
    e = rel_err(G, Gc)
    return e <= 1e-11, f"rel err {e:.3e}"


def pin_loss_likelihoods():
    """Losses from their likelihoods: Bernoulli with odds m has P(x=1) = m/(1+m);
    Poisson f = -log pmf(x; m) - log x!; Gaussian f = (x - m)^2; shape-1 Gamma
    f = -log density of the exponential with mean m; beta = 1/2 f = the
    beta-divergence d(x|m) plus a term free of m.  Derivatives by central
    differences of f."""
    for m in [0.01, 0.3, 1.0, 4.5]:
        if abs(oracle.loss_f(oracle.BERNOULLI_ODDS, 1.0, m, 0.0) + math.log(m / (1 + m))) > 1e-12:
            return False, "bernoulli x=1"
        if abs(oracle.loss_f(oracle.BERNOULLI_ODDS, 0.0, m, 0.0) + math.log(1 / (1 + m))) > 1e-12:
            return False, "bernoulli x=0"
        for x in [0, 1, 3, 7]:
            ref = -scipy.stats.poisson.logpmf(x, m) - scipy.special.gammaln(x + 1)
            if abs(oracle.loss_f(oracle.POISSON, float(x), m, 0.0) - ref) > 1e-10 * max(1, abs(ref)):
                return False, f"poisson x={x} m={m}"
        for x in [-1.5, 0.0, 2.0]:
            if abs(oracle.loss_f(oracle.GAUSSIAN, x, m, 0.0) - (x - m) ** 2) > 1e-14:
                return False, "gaussian"
    for m in [0.05, 0.7, 2.5]:
        for x in [0.01, 0.4, 3.0]:
            # shape-1 Gamma (exponential with mean m): f = -log density
            ref = -scipy.stats.expon.logpdf(x, scale=m)
            if abs(oracle.loss_f(oracle.GAMMA, x, m, 0.0) - ref) > 1e-12 * max(1, abs(ref)):
                return False, f"gamma x={x} m={m}"
            # beta-divergence, beta = 1/2: d(x|m) = (x^b + (b-1) m^b - b x m^(b-1)) / (b (b-1));
            # f differs from it by 4 sqrt(x), which does not depend on m
            b = 0.5
            dbeta = (x ** b + (b - 1) * m ** b - b * x * m ** (b - 1)) / (b * (b - 1))
            if abs(oracle.loss_f(oracle.BETA_HALF, x, m, 0.0) - dbeta - 4 * math.sqrt(x)) > 1e-12 * max(1, abs(dbeta)):
                return False, f"beta x={x} m={m}"
    for loss in (oracle.GAUSSIAN, oracle.BERNOULLI_ODDS, oracle.POISSON, oracle.GAMMA, oracle.BETA_HALF):
        for x in [0.0, 1.0, 2.0]:
            for m in [0.2, 1.3, 3.0]:
                h = 1e-5
                fd = (oracle.loss_f(loss, x, m + h) - oracle.loss_f(loss, x, m - h)) / (2 * h)
                g = oracle.loss_g(loss, x, m)
                if abs(fd - g) > 1e-7 * max(1.0, abs(g)):
                    return False, f"derivative loss={loss} x={x} m={m}: {g} vs fd {fd}"
    return True, "ok"


def _mean_and_trace(draw, N):
    vals = [np.concatenate([g.reshape(-1) for g in draw(t)]) for t in range(N)]
    V = np.stack(vals)
    return V.mean(axis=0), float(V.var(axis=0, ddof=1).sum())


def pin_unbiased(sampler, loss, N=2000):
    """P4: mean of N sampled gradients -> exact gradient; ||mean - g||^2 <= 3 tr(Sigma)/N
    (E||mean - g||^2 = tr(Sigma)/N), for the three samplers (Sec. 4.1-4.3)."""
    if sampler == oracle.UNIFORM:
        X, A = tiny_dense((4, 3, 5), r=2)
        coo = val = None
        nnz = 0
    else:
        X, coo, val, A = tiny_sparse("binary" if loss == oracle.BERNOULLI_ODDS else "counts")
        nnz = coo.shape[0]
    dims = X.shape
    Gx = np.concatenate([g.reshape(-1) for g in exact_gradient(loss, X, A)])
    s, p, q = 12, 6, 8

    def draw(t):
        if sampler == oracle.UNIFORM:
            smp = oracle.sample(sampler, dims, dense=X, s=s, seed=31, iteration=t)
        else:
            smp = oracle.sample(sampler, dims, coo_idx=coo, coo_val=val, p=p, q=q, seed=31, iteration=t)
        G, _ = oracle.grad(loss, dims, A, smp, nnz=nnz, s=s, p=p, q=q)
        return G

    mean, tr = _mean_and_trace(draw, N)
    dev = float(np.sum((mean - Gx) ** 2))
    return dev <= 3.0 * tr / N, f"||mean-g||^2={dev:.4g} bound={3.0 * tr / N:.4g}"


def _weighted_case(seed=61):
    """Tiny counts tensor with a weight per stored entry and w_zero for the rest."""
    X, coo, val, A = tiny_sparse("counts", seed=seed)
    rng = np.random.default_rng(seed)
    coo_w = rng.uniform(0.2, 2.0, size=coo.shape[0])
    w_zero = 0.3
    W = np.full(X.shape, w_zero)
    for e in range(coo.shape[0]):
        W[tuple(int(t) for t in coo[e])] = coo_w[e]
    return X, coo, val, A, coo_w, w_zero, W


def pin_weighted_unbiased(sampler, N=2000):
    """Weighted GCP (eq. wgcp): every sampler's estimate, with entry weights
    folded into ytilde, is unbiased for the exact weighted gradient
    Y_(k) Z_k with y_i = w_i g(x_i, m_i) (per-entry weights on stored
    entries, w_zero elsewhere; dense: a weight per entry)."""
    loss = oracle.POISSON
    if sampler == oracle.UNIFORM:
        X, A = tiny_dense((4, 3, 5), r=2)
        X = np.round(np.abs(X))
        A = [np.abs(a) + 0.1 for a in A]
        W = np.random.default_rng(62).uniform(0.0, 2.0, size=X.shape)
        data, wkw = dict(dense=X), dict(dense_w=W)
        nnz = 0
    else:
        X, coo, val, A, coo_w, w_zero, W = _weighted_case()
        data, wkw = dict(coo_idx=coo, coo_val=val), dict(coo_idx=coo, coo_w=coo_w, w_zero=w_zero)
        nnz = coo.shape[0]
    dims = X.shape
    Gx = np.concatenate([g.reshape(-1) for g in exact_gradient(loss, X, A, W=W)])
    # enough samples per draw that a wrong weight on the corrected terms
    # (a fixed bias) stands out of the 3 tr(Sigma)/N band
    s, p, q = 40, 60, 80

    def draw(t):
        smp = oracle.sample(sampler, dims, s=s, p=p, q=q, seed=37, iteration=t, **data)
        wg = oracle.entry_weights(dims, smp, **wkw)
        G, _ = oracle.grad(loss, dims, A, smp, nnz=nnz, s=s, p=p, q=q, wgt=wg, w_zero=wkw.get("w_zero", 1.0))
        return G

    mean, tr = _mean_and_trace(draw, N)
    dev = float(np.sum((mean - Gx) ** 2))
    return dev <= 3.0 * tr / N, f"||mean-g||^2={dev:.4g} bound={3.0 * tr / N:.4g}"


def pin_weighted_ones_is_unweighted():
    """All weights 1 (stored entries and w_zero) give the unweighted estimate
    exactly, for the corrected semi-stratified terms too."""
    X, coo, val, A = tiny_sparse("counts")
    dims = X.shape
    for sampler in (oracle.STRATIFIED, oracle.SEMI_STRATIFIED):
        smp = oracle.sample(sampler, dims, coo_idx=coo, coo_val=val, p=9, q=11, seed=5)
        wg = oracle.entry_weights(dims, smp, coo_idx=coo, coo_w=np.ones(coo.shape[0]), w_zero=1.0)
        G1, F1 = oracle.grad(oracle.POISSON, dims, A, smp, nnz=coo.shape[0], p=9, q=11, wgt=wg, w_zero=1.0)
        G0, F0 = oracle.grad(oracle.POISSON, dims, A, smp, nnz=coo.shape[0], p=9, q=11)
        if F1 != F0 or any(not np.array_equal(a, b) for a, b in zip(G1, G0)):
            return False, f"sampler {sampler}"
    return True, "ok"


def pin_missing_data(N=3000):
    """Missing entries (Sec. 4.4): zero weights on a dense tensor's missing
    entries under uniform sampling, and nonzero picks over the list of observed
    entries (observed zeros stored explicitly, q = 0), both estimate the
    gradient of the loss over the observed entries only."""
    X, A = tiny_dense((4, 3, 5), r=2)
    rng = np.random.default_rng(71)
    mask = (rng.random(X.shape) < 0.6).astype(float)
    dims = X.shape
    Gx = np.concatenate([g.reshape(-1) for g in exact_gradient(oracle.GAUSSIAN, X, A, W=mask)])
    obs = np.argwhere(mask > 0)
    obs_val = X[tuple(obs.T)]

    def draw_uniform(t):
        smp = oracle.sample(oracle.UNIFORM, dims, dense=X, s=20, seed=41, iteration=t)
        wg = oracle.entry_weights(dims, smp, dense_w=mask)
        return oracle.grad(oracle.GAUSSIAN, dims, A, smp, s=20, wgt=wg)[0]

    def draw_observed(t):
        smp = oracle.sample(oracle.STRATIFIED, dims, coo_idx=obs, coo_val=obs_val, p=20, q=0, seed=43, iteration=t)
        return oracle.grad(oracle.GAUSSIAN, dims, A, smp, nnz=obs.shape[0], p=20, q=0)[0]

    for draw, name in ((draw_uniform, "zero weights"), (draw_observed, "observed list")):
        mean, tr = _mean_and_trace(draw, N)
        dev = float(np.sum((mean - Gx) ** 2))
        if not dev <= 3.0 * tr / N:
            return False, f"{name}: ||mean-g||^2={dev:.4g} bound={3.0 * tr / N:.4g}"
    return True, "ok"


def pin_semi_zero_half_poisson(N=2000):
    """P6: with p = 0 the semi-stratified estimate for Poisson (g(0,m) = 1) has
    expectation the all-ones MTTKRP, 1 (hadamard_{j != k} 1^T A_j)."""
    X, coo, val, A = tiny_sparse("counts")
    dims = X.shape
    r = A[0].shape[1]
    want = []
    for k in range(len(dims)):
        colsum = np.ones(r)
        for j in range(len(dims)):
            if j != k:
                colsum = colsum * A[j].sum(axis=0)
        want.append(np.outer(np.ones(dims[k]), colsum))
    Gx = np.concatenate([g.reshape(-1) for g in want])

    def draw(t):
        smp = oracle.sample(oracle.SEMI_STRATIFIED, dims, coo_idx=coo, coo_val=val, p=0, q=10, seed=8,
                            iteration=t)
        G, _ = oracle.grad(oracle.POISSON, dims, A, smp, nnz=coo.shape[0], p=0, q=10)
        return G

    mean, tr = _mean_and_trace(draw, N)
    dev = float(np.sum((mean - Gx) ** 2))
    return dev <= 3.0 * tr / N, f"||mean-g||^2={dev:.4g} bound={3.0 * tr / N:.4g}"


def pin_adam_closed_forms():
    """P7: first step (t = 1) gives Bhat = G, Chat = G^2, so dA = -alpha G / sqrt(G^2 + eps)
    (eps inside the root, Alg. 4) or -alpha G / (|G| + eps); a constant gradient keeps
    Bhat = G and Chat = G^2 at every t (bias correction); G = 0 leaves A; projection clamps."""
    rng = np.random.Generator(np.random.PCG64(3))
    P = 257
    G = rng.standard_normal(P) * 10.0 ** rng.uniform(-6, 2, P)
    G[:5] = 0.0
    alpha, eps = 0.01, 1e-8
    for mode in (0, 1):
        A = rng.standard_normal(P)
        A0 = A.copy()
        B = np.zeros(P)
        C = np.zeros(P)
        for t in range(1, 6):
            oracle.adam(A, G, B, C, t, alpha=alpha, eps=eps, eps_mode=mode)
            den = np.sqrt(G * G + eps) if mode == 0 else np.abs(G) + eps
            expect = A0 - t * alpha * G / den
            err = np.max(np.abs(A - expect) / (1 + np.abs(expect)))
            if err > 1e-12:
                return False, f"eps_mode={mode} t={t}: err {err:.3e}"
        if not np.array_equal(A[:5], A0[:5]):
            return False, "zero-gradient entries moved"
    A = np.full(P, 0.001)
    B = np.zeros(P)
    C = np.zeros(P)
    oracle.adam(A, np.abs(G) + 1.0, B, C, 1, alpha=alpha, eps=eps, lower=0.0)
    if not (np.all(A >= 0.0) and np.any(A == 0.0)):
        return False, "projection"
    return True, "ok"


def pin_finite_differences(loss, h=None):
    """P8: the sampled gradient is the exact gradient of the sampled loss estimate on
    a fixed sample set (eqs. Fhat, Fhat-strat); central differences in single
    coordinates (the model is linear in each, so Gaussian differences are exact)."""
    if loss == oracle.GAUSSIAN:
        X, A = tiny_dense((4, 3, 5), r=3)
        dims = X.shape
        smp = oracle.sample(oracle.UNIFORM, dims, dense=X, s=30, seed=4)
        kw = dict(s=30)
        h = h or 1e-3
    elif loss == oracle.GAMMA:
        X, A = tiny_dense((4, 3, 5), r=3)
        X = np.abs(X) + 0.1
        A = [np.abs(a) + 0.2 for a in A]
        dims = X.shape
        smp = oracle.sample(oracle.UNIFORM, dims, dense=X, s=30, seed=4)
        kw = dict(s=30)
        h = h or 1e-6
    elif loss == oracle.BETA_HALF:
        X, coo, val, A = tiny_sparse("counts")
        dims = X.shape
        smp = oracle.sample(oracle.SEMI_STRATIFIED, dims, coo_idx=coo, coo_val=val, p=9, q=11, seed=4)
        kw = dict(nnz=coo.shape[0], p=9, q=11)
        h = h or 1e-6
    else:
        X, coo, val, A = tiny_sparse("binary" if loss == oracle.BERNOULLI_ODDS else "counts")
        dims = X.shape
        sampler = oracle.STRATIFIED if loss == oracle.BERNOULLI_ODDS else oracle.SEMI_STRATIFIED
        smp = oracle.sample(sampler, dims, coo_idx=coo, coo_val=val, p=9, q=11, seed=4)
        kw = dict(nnz=coo.shape[0], p=9, q=11)
        h = h or 1e-6
    G, _ = oracle.grad(loss, dims, A, smp, **kw)
    worst = 0.0
    for k in range(len(dims)):
        for i in range(dims[k]):
            for j in range(A[0].shape[1]):
                Ap = [a.copy() for a in A]
                Am = [a.copy() for a in A]
                Ap[k][i, j] += h
                Am[k][i, j] -= h
                _, fp = oracle.grad(loss, dims, Ap, smp, **kw)
                _, fm = oracle.grad(loss, dims, Am, smp, **kw)
                fd = (fp - fm) / (2 * h)
                worst = max(worst, abs(fd - G[k][i, j]) / max(1.0, abs(G[k][i, j])))
    tol = 1e-8 if loss == oracle.GAUSSIAN else 1e-5
    return worst <= tol, f"worst rel {worst:.3e}"


def cp_score(A_true, A_est):
    """Cosine similarity score of App. E: mean over components of the product
    over modes of column cosines, under the best column matching."""
    from scipy.optimize import linear_sum_assignment
    r = A_true[0].shape[1]
    S = np.ones((r, r))
    for a, b in zip(A_true, A_est):
        an = a / np.linalg.norm(a, axis=0)
        bn = b / np.linalg.norm(b, axis=0)
        S *= an.T @ bn
    ri, ci = linear_sum_assignment(-S)
    return float(S[ri, ci].mean())


def pin_cp_score():
    """The score is 1 for the same model up to column order, column scaling and
    sign flips in pairs of modes, and near 0 for unrelated factors."""
    rng = np.random.default_rng(9)
    A = [rng.standard_normal((n, 4)) for n in (9, 8, 7)]
    perm = np.array([2, 0, 3, 1])
    scale = [np.array([2.0, 0.5, 3.0, 1.0]), np.array([1.0, 4.0, 0.25, 1.0]), np.array([0.5, 0.5, 1.0, 1.0])]
    B = [a[:, perm] * s_ for a, s_ in zip(A, scale)]
    B[0][:, 1] *= -1
    B[2][:, 1] *= -1
    if abs(cp_score(A, B) - 1.0) > 1e-12:
        return False, "equivalent model"
    C = [rng.standard_normal(a.shape) for a in A]
    sc = cp_score(A, C)
    return sc < 0.3, f"unrelated score {sc:.3f}"


def pin_adam_fit_recovers():
    """GCP-Adam (Alg. 4) with the oracle's gradients recovers the factors of a
    noisy rank-3 Gaussian tensor from a random start (score >= 0.9, App. E),
    and the accepted estimates never rise."""
    dims, r = (20, 15, 10), 3
    rng = np.random.default_rng(41)
    A_true = [rng.standard_normal((n, r)) for n in dims]
    X = full_model(A_true) + 0.1 * rng.standard_normal(dims)
    A0 = [rng.standard_normal((n, r)) for n in dims]
    A, hist, acc, _ = oracle.adam_fit(oracle.GAUSSIAN, dims, A0, dense=X,
                                      grad_cfg=dict(sampler=oracle.UNIFORM, s=300, seed=5),
                                      est_cfg=dict(sampler=oracle.UNIFORM, s=3000, seed=6),
                                      alpha=0.01, tau=500, kappa=3, max_epochs=40)
    kept = [h for h, a in zip(hist, acc) if a]
    mono = all(b <= a for a, b in zip(kept, kept[1:]))
    sc = cp_score(A_true, A)
    return sc >= 0.9 and mono, f"score {sc:.4f}, kept estimates non-increasing {mono}"


def pin_adam_fit_undo():
    """An epoch that raises the estimate is undone exactly: with a step size
    that overshoots, every epoch is undone, so the fit returns the start
    unchanged after kappa + 1 epochs with the rate scaled by nu^(kappa+1)."""
    dims, r = (6, 5, 4), 2
    rng = np.random.default_rng(43)
    A_true = [rng.standard_normal((n, r)) for n in dims]
    X = full_model(A_true)
    A0 = [rng.standard_normal((n, r)) for n in dims]
    A, hist, acc, alpha = oracle.adam_fit(oracle.GAUSSIAN, dims, A0, dense=X,
                                          grad_cfg=dict(sampler=oracle.UNIFORM, s=40, seed=7),
                                          est_cfg=dict(sampler=oracle.UNIFORM, s=500, seed=8),
                                          alpha=50.0, nu=0.5, tau=5, kappa=2, max_epochs=10)
    same = all(np.array_equal(a, b) for a, b in zip(A, A0))
    ok = same and acc == [True, False, False, False] and len(hist) == 4 and abs(alpha - 50.0 * 0.125) < 1e-12
    return ok, f"unchanged {same}, accepted {acc}, alpha {alpha}"


def pin_loss_estimate_unbiased(sampler, weighted=False, N=4000):
    """The oracle's loss estimate -- eq. Fhat (uniform), eq. Fhat-strat
    (stratified), and for semi-stratified sampling the correction reading
    sum_nz (eta/p)[f(x, m) - f(0, m)] + sum_zero (omega/q) f(0, m) -- has
    mean F(X, M) = sum_i f(x_i, m_i) over every entry (eq. gcp), or the
    weighted sum_i w_i f(x_i, m_i) (eq. wgcp): the mean of N estimates lies
    within 3 standard errors of the enumerated value."""
    loss = {oracle.UNIFORM: oracle.GAUSSIAN, oracle.STRATIFIED: oracle.BERNOULLI_ODDS,
            oracle.SEMI_STRATIFIED: oracle.POISSON}[sampler]
    W = None
    if sampler == oracle.UNIFORM:
        X, A = tiny_dense((4, 3, 5), r=2)
        data, nnz = dict(dense=X), 0
        if weighted:
            W = np.random.default_rng(62).uniform(0.0, 2.0, size=X.shape)
            wkw = dict(dense_w=W)
    elif weighted:
        loss = oracle.POISSON if sampler == oracle.SEMI_STRATIFIED else oracle.BERNOULLI_ODDS
        X, coo, val, A, coo_w, w_zero, W = _weighted_case()
        data, nnz = dict(coo_idx=coo, coo_val=val), coo.shape[0]
        wkw = dict(coo_idx=coo, coo_w=coo_w, w_zero=w_zero)
    else:
        X, coo, val, A = tiny_sparse("binary" if loss == oracle.BERNOULLI_ODDS else "counts")
        data, nnz = dict(coo_idx=coo, coo_val=val), coo.shape[0]
    dims = X.shape
    F_exact = exact_loss(loss, X, A, W=W)
    s, p, q = 30, 20, 25
    est = np.empty(N)
    for t in range(N):
        smp = oracle.sample(sampler, dims, s=s, p=p, q=q, seed=53, iteration=t, **data)
        kw = dict(nnz=nnz, s=s, p=p, q=q)
        if weighted:
            kw.update(wgt=oracle.entry_weights(dims, smp, **wkw), w_zero=wkw.get("w_zero", 1.0))
        est[t] = oracle.grad(loss, dims, A, smp, **kw)[1]
    se = float(est.std(ddof=1)) / math.sqrt(N)
    dev = abs(float(est.mean()) - F_exact)
    return dev <= 3.0 * se, f"|mean - F| = {dev:.4g}, 3 s.e. = {3.0 * se:.4g} (F = {F_exact:.6g})"


def _fit_by_alg4(loss, dims, A0, X, gcfg, ecfg, alpha, nu, tau, kappa, max_epochs, beta1=0.9, beta2=0.999,
                 eps=1e-8):
    """Alg. 4 written out independently of oracle.adam_fit: after an epoch whose
    estimate rose, A, B, C and the step count t go back to their values at the
    start of the epoch (t <- t - tau) and the rate is scaled by nu."""
    d = len(dims)
    r = A0[0].shape[1]
    A = [np.array(a, dtype=np.float64) for a in A0]
    B = [np.zeros_like(a) for a in A]
    C = [np.zeros_like(a) for a in A]
    est_smp = oracle.sample(ecfg["sampler"], dims, dense=X, s=ecfg["s"], seed=ecfg["seed"])
    F = oracle.grad(loss, dims, A, est_smp, s=ecfg["s"])[1]
    t, draws, bad, accepted = 0, 0, 0, [True]
    for _ in range(max_epochs):
        if bad > kappa:
            break
        A_keep, B_keep, C_keep = [a.copy() for a in A], [b.copy() for b in B], [c.copy() for c in C]
        for _ in range(tau):
            smp = oracle.sample(gcfg["sampler"], dims, dense=X, s=gcfg["s"], seed=gcfg["seed"], iteration=draws)
            draws += 1
            G, _ = oracle.grad(loss, dims, A, smp, s=gcfg["s"])
            t += 1
            flatA = np.concatenate([a.reshape(-1) for a in A])
            flatB = np.concatenate([b.reshape(-1) for b in B])
            flatC = np.concatenate([c.reshape(-1) for c in C])
            oracle.adam(flatA, np.concatenate([g.reshape(-1) for g in G]), flatB, flatC, t, alpha=alpha,
                        beta1=beta1, beta2=beta2, eps=eps)
            off = 0
            for k in range(d):
                n = dims[k] * r
                A[k] = flatA[off:off + n].reshape(dims[k], r)
                B[k] = flatB[off:off + n].reshape(dims[k], r)
                C[k] = flatC[off:off + n].reshape(dims[k], r)
                off += n
        F_new = oracle.grad(loss, dims, A, est_smp, s=ecfg["s"])[1]
        if F_new > F:
            A, B, C = A_keep, B_keep, C_keep
            t -= tau
            alpha *= nu
            bad += 1
            accepted.append(False)
        else:
            F = F_new
            accepted.append(True)
    return A, accepted


def pin_adam_fit_rewind():
    """Alg. 4's undo winds the step count back (t <- t - tau), so the bias
    corrections of the epoch after an undone one are those of a fresh epoch:
    with a rate that overshoots in the first epoch only, oracle.adam_fit
    (undo, then kept epochs) equals the loop written out here bit for bit."""
    dims, r = (6, 5, 4), 2
    rng = np.random.default_rng(43)
    A_true = [rng.standard_normal((n, r)) for n in dims]
    X = full_model(A_true) + 0.05 * rng.standard_normal(dims)
    A0 = [rng.standard_normal((n, r)) for n in dims]
    gcfg = dict(sampler=oracle.UNIFORM, s=40, seed=7)
    ecfg = dict(sampler=oracle.UNIFORM, s=500, seed=8)
    A, _, acc, _ = oracle.adam_fit(oracle.GAUSSIAN, dims, A0, dense=X, grad_cfg=gcfg, est_cfg=ecfg, alpha=3.0,
                                   nu=0.1, tau=10, kappa=2, max_epochs=4)
    A_ref, acc_ref = _fit_by_alg4(oracle.GAUSSIAN, dims, A0, X, gcfg, ecfg, alpha=3.0, nu=0.1, tau=10, kappa=2,
                                  max_epochs=4)
    pattern = acc_ref[:3] == [True, False, True]
    same = acc == acc_ref and all(np.array_equal(a, b) for a, b in zip(A, A_ref))
    return pattern and same, f"accepted {acc} (written-out loop {acc_ref}), factors equal {same}"


ALL_PINS = {
    "philox_numpy": pin_philox_numpy,
    "randi_exact": pin_randi_exact,
    "sample_streams": pin_sample_streams,
    "stratified_zeros_are_zeros": pin_stratified_zeros_are_zeros,
    "index_uniformity": pin_index_uniformity,
    "enumeration_equals_unfolding": pin_enumeration_equals_unfolding,
    "gaussian_closed_form": pin_gaussian_closed_form,
    "poisson_closed_form": pin_poisson_closed_form,
    "loss_likelihoods": pin_loss_likelihoods,
    "unbiased_uniform_gaussian": lambda: pin_unbiased(oracle.UNIFORM, oracle.GAUSSIAN),
    "unbiased_stratified_bernoulli": lambda: pin_unbiased(oracle.STRATIFIED, oracle.BERNOULLI_ODDS),
    "unbiased_semi_poisson": lambda: pin_unbiased(oracle.SEMI_STRATIFIED, oracle.POISSON),
    "unbiased_semi_bernoulli": lambda: pin_unbiased(oracle.SEMI_STRATIFIED, oracle.BERNOULLI_ODDS),
    "unbiased_semi_beta_half": lambda: pin_unbiased(oracle.SEMI_STRATIFIED, oracle.BETA_HALF),
    "unbiased_stratified_gamma": lambda: pin_unbiased(oracle.STRATIFIED, oracle.GAMMA),
    "semi_zero_half_poisson": pin_semi_zero_half_poisson,
    "adam_closed_forms": pin_adam_closed_forms,
    "fd_gaussian": lambda: pin_finite_differences(oracle.GAUSSIAN),
    "fd_bernoulli_stratified": lambda: pin_finite_differences(oracle.BERNOULLI_ODDS),
    "fd_poisson_semi": lambda: pin_finite_differences(oracle.POISSON),
    "fd_gamma_uniform": lambda: pin_finite_differences(oracle.GAMMA),
    "fd_beta_half_semi": lambda: pin_finite_differences(oracle.BETA_HALF),
    "weighted_unbiased_uniform": lambda: pin_weighted_unbiased(oracle.UNIFORM),
    "weighted_unbiased_stratified": lambda: pin_weighted_unbiased(oracle.STRATIFIED),
    "weighted_unbiased_semi": lambda: pin_weighted_unbiased(oracle.SEMI_STRATIFIED),
    "weighted_ones_is_unweighted": pin_weighted_ones_is_unweighted,
    "missing_data": pin_missing_data,
    "cp_score": pin_cp_score,
    "adam_fit_recovers": pin_adam_fit_recovers,
    "adam_fit_undo": pin_adam_fit_undo,
    "adam_fit_rewind": pin_adam_fit_rewind,
    "loss_estimate_uniform": lambda: pin_loss_estimate_unbiased(oracle.UNIFORM),
    "loss_estimate_stratified": lambda: pin_loss_estimate_unbiased(oracle.STRATIFIED),
    "loss_estimate_semi": lambda: pin_loss_estimate_unbiased(oracle.SEMI_STRATIFIED),
    "loss_estimate_weighted_uniform": lambda: pin_loss_estimate_unbiased(oracle.UNIFORM, weighted=True),
    "loss_estimate_weighted_stratified": lambda: pin_loss_estimate_unbiased(oracle.STRATIFIED, weighted=True),
    "loss_estimate_weighted_semi": lambda: pin_loss_estimate_unbiased(oracle.SEMI_STRATIFIED, weighted=True),
}
