"""CPU checks of the seeded input generators that stand in for the paper's
binary test tensors (App. D recipe) and of the Sec. 5.4 starting point."""
import math

import numpy as np

import synth


def test_appd_binary_recipe():
    dims, r, delta, p_high, p_low = (40, 30, 20, 10), 5, 0.15, 0.9, 0.002
    coo, val, A = synth.sparse_binary_appd(dims, r, delta, p_high, p_low, seed=3)
    d = len(dims)
    c_low = (p_low / (1 - p_low)) ** (1 / d)
    # factor structure: r-1 sparse nonnegative columns, one constant column
    for a, n in zip(A, dims):
        assert a.shape == (n, r) and (a >= 0).all()
        assert np.allclose(a[:, r - 1], c_low)
        frac = (a[:, : r - 1] > 0).mean()
        assert 0.02 < frac < 0.4
    # COO: unique, sorted by row-major key, in range, values one
    keys = np.ravel_multi_index(tuple(coo.astype(np.int64).T), dims)
    assert (np.diff(keys) > 0).all()
    assert (val == 1).all()
    # away from every sparse component the model is c_low^d, whose odds
    # probability is p_low: the ones there come at that rate
    inside = np.zeros(dims, dtype=bool)
    for j in range(r - 1):
        sup = [A[k][:, j] > 0 for k in range(d)]
        inside |= np.einsum("i,j,k,l->ijkl", *[s.astype(np.int8) for s in sup]).astype(bool)
    X = np.zeros(dims, dtype=bool)
    X[tuple(coo.astype(np.int64).T)] = True
    out = ~inside
    rate = X[out].sum() / out.sum()
    sd = math.sqrt(p_low * (1 - p_low) / out.sum())
    assert abs(rate - p_low) < 5 * sd
    # inside the supports, ones follow m/(1+m) on average
    M = np.einsum("ir,jr,kr,lr->ijkl", *A)
    prob = M / (1 + M)
    assert abs(X[inside].sum() - prob[inside].sum()) < 5 * math.sqrt((prob[inside] * (1 - prob[inside])).sum())


def test_kruskal_norm_and_norm_matched_start():
    rng = np.random.default_rng(4)
    A = [rng.random((n, 3)) for n in (5, 4, 6, 3)]
    M = np.einsum("ir,jr,kr,lr->ijkl", *A)
    assert abs(synth.kruskal_norm(A) - np.linalg.norm(M)) < 1e-12 * np.linalg.norm(M)


def test_table1_workload_start_has_the_data_norm():
    """Sec. 5.4: random positive starts scaled so the model's norm equals the
    tensor's (sqrt(nnz) for binary data); about 0.38 % dense."""
    w = synth.sparse_binary_400x300x200x100()
    assert w.dims == (400, 300, 200, 100) and w.rank == 5
    assert all((a > 0).all() for a in w.A_init)
    assert abs(synth.kruskal_norm(w.A_init) - math.sqrt(w.nnz)) < 1e-9 * math.sqrt(w.nnz)
    assert 0.0035 < w.nnz / w.omega < 0.0041
