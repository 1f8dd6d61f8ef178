"""Checkpoint and resume of the oracle's Alg. 4 inner loop (CPU).

The state of a run of sampled Adam steps is (A, B, C, t) plus the position of
the sample stream.  Samples are keyed by (seed, problem_id, iteration), so a
run of 2k steps equals k steps, a save and load of that state through a file,
and k more steps, bit for bit.
"""
import numpy as np

import oracle
import pins


def _steps(state, X, coo, val, nnz, A_shapes, k, p=9, q=11, seed=19):
    A, B, C, t, it = state
    dims = X.shape
    for _ in range(k):
        smp = oracle.sample(oracle.STRATIFIED, dims, coo_idx=coo, coo_val=val, p=p, q=q, seed=seed, iteration=it)
        it += 1
        off, mats = 0, []
        for (n, r) in A_shapes:
            mats.append(A[off:off + n * r].reshape(n, r))
            off += n * r
        G, _ = oracle.grad(oracle.BERNOULLI_ODDS, dims, mats, smp, nnz=nnz, p=p, q=q)
        t += 1
        oracle.adam(A, np.concatenate([g.reshape(-1) for g in G]), B, C, t, alpha=0.01, lower=0.0)
    return A, B, C, t, it


def test_oracle_resume_is_bit_exact(tmp_path):
    X, coo, val, A0 = pins.tiny_sparse("binary")
    shapes = [a.shape for a in A0]
    flat = np.concatenate([a.reshape(-1) for a in A0]).astype(np.float64)
    start = (flat.copy(), np.zeros_like(flat), np.zeros_like(flat), 0, 100)
    k = 7
    whole = _steps(tuple(x.copy() if isinstance(x, np.ndarray) else x for x in start), X, coo, val,
                   coo.shape[0], shapes, 2 * k)
    half = _steps(tuple(x.copy() if isinstance(x, np.ndarray) else x for x in start), X, coo, val,
                  coo.shape[0], shapes, k)
    path = tmp_path / "ckpt.npz"
    np.savez(path, A=half[0], B=half[1], C=half[2], t=half[3], it=half[4])
    z = np.load(path)
    resumed = _steps((z["A"].copy(), z["B"].copy(), z["C"].copy(), int(z["t"]), int(z["it"])), X, coo, val,
                     coo.shape[0], shapes, k)
    for a, b in zip(whole[:3], resumed[:3]):
        assert np.array_equal(a, b)
    assert whole[3:] == resumed[3:] == (2 * k, 100 + 2 * k)
    # and the run really moved: a different stream position gives other factors
    other = _steps((flat.copy(), np.zeros_like(flat), np.zeros_like(flat), 0, 101), X, coo, val, coo.shape[0],
                   shapes, 2 * k)
    assert not np.array_equal(other[0], whole[0])
