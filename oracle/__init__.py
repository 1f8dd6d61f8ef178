"""FP64 CPU oracle for the sampled GCP gradient -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It loads ``liboracle.so``, built by gcc from
``gcp_oracle.c`` in this folder, and shares no code with the HIP library.

Every function here is argument marshalling around the C oracle: the
arithmetic (Philox draws, sampling, model entries, loss derivatives, the
sparse MTTKRP and the Adam step) all lives in ``gcp_oracle.c`` and follows
Kolda & Hong, Alg. 1-4 and eqs. Y, Gks, Fhat, Fhat-strat.  ``adam_fit`` (the
GCP-Adam epoch loop of Alg. 4) is plain Python control flow over those calls.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gcp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

GAUSSIAN, BERNOULLI_ODDS, POISSON, GAMMA, BETA_HALF = 0, 1, 2, 3, 4
UNIFORM, STRATIFIED, SEMI_STRATIFIED = 0, 1, 2
S_UNIFORM, S_NZ, S_ZERO, S_NZ_CORR, S_SEMI_ZERO = 0, 1, 2, 3, 4
LOSS_EPS = 1e-10

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, no threads)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    """The loaded oracle; GCP_ORACLE_LIB names another build of gcp_oracle.c
    (the sanitizer test loads an instrumented one)."""
    global _lib
    if _lib is None:
        path = os.environ.get("GCP_ORACLE_LIB")
        if not path:
            path = _LIB_PATH
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
        L = ctypes.CDLL(path)
        u64, i64, i32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        P = ctypes.c_void_p
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_philox4x64_10.restype = None
        L.orc_randi.argtypes = [u64, u64]
        L.orc_randi.restype = u64
        L.orc_loss_f.argtypes = [ctypes.c_int, dbl, dbl, dbl]
        L.orc_loss_f.restype = dbl
        L.orc_loss_g.argtypes = [ctypes.c_int, dbl, dbl, dbl]
        L.orc_loss_g.restype = dbl
        L.orc_sample.argtypes = [ctypes.c_int, ctypes.c_int, P, P, i64, P, P, i64, i64, i64,
                                 u64, u64, u64, P, P, P, P]
        L.orc_sample.restype = i64
        L.orc_grad.argtypes = [ctypes.c_int, ctypes.c_int, P, i64, P, i64, P, P, P,
                               i64, i64, i64, i64, dbl, P, P]
        L.orc_grad.restype = dbl
        L.orc_grad_weighted.argtypes = [ctypes.c_int, ctypes.c_int, P, i64, P, i64, P, P, P, P, dbl,
                                        i64, i64, i64, i64, dbl, P, P]
        L.orc_grad_weighted.restype = dbl
        L.orc_entry_weights.argtypes = [ctypes.c_int, P, P, i64, P, P, dbl, i64, P, P, P]
        L.orc_entry_weights.restype = ctypes.c_int
        L.orc_full_grad.argtypes = [ctypes.c_int, ctypes.c_int, P, i64, P, P, dbl, P]
        L.orc_full_grad.restype = dbl
        L.orc_adam.argtypes = [i64, P, P, P, P, i64, dbl, dbl, dbl, dbl, dbl, ctypes.c_int]
        L.orc_adam.restype = None
        L.orc_set_mutation.argtypes = [ctypes.c_int]
        L.orc_set_mutation.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


_mutation = 0


def set_mutation(m: int) -> None:
    """Plant deliberate mistake ``m`` (0 = none); used only by the pin tests.
    Mistakes 1-8 live in the C code, 9 in adam_fit below."""
    global _mutation
    _mutation = int(m)
    lib().orc_set_mutation(int(m))


def philox4x64_10(key, counter) -> np.ndarray:
    k = np.ascontiguousarray(key, dtype=np.uint64)
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(k), _ptr(c), _ptr(out))
    return out


def randi(w: int, n: int) -> int:
    return int(lib().orc_randi(int(w), int(n)))


def loss_f(loss: int, x: float, m: float, eps: float = LOSS_EPS) -> float:
    return lib().orc_loss_f(loss, x, m, eps)


def loss_g(loss: int, x: float, m: float, eps: float = LOSS_EPS) -> float:
    return lib().orc_loss_g(loss, x, m, eps)


class Samples:
    """One sample set: idx [S, d] int64, xval [S] f64, stratum [S] int32, cand [S] int64."""

    def __init__(self, idx, xval, stratum, cand, examined):
        self.idx, self.xval, self.stratum, self.cand, self.examined = idx, xval, stratum, cand, examined

    def __len__(self):
        return len(self.xval)


def sample(sampler: int, dims, *, dense=None, coo_idx=None, coo_val=None,
           s: int = 0, p: int = 0, q: int = 0, seed: int = 0, problem_id: int = 0,
           iteration: int = 0) -> Samples:
    """Draw one gradient's samples (Alg. 1 / 2 / 3 sampling lines)."""
    d = len(dims)
    dims_a = np.ascontiguousarray(dims, dtype=np.int64)
    S = s if sampler == UNIFORM else p + q
    idx = np.zeros((max(S, 1), d), dtype=np.int64)
    xval = np.zeros(max(S, 1), dtype=np.float64)
    st = np.zeros(max(S, 1), dtype=np.int32)
    cand = np.zeros(max(S, 1), dtype=np.int64)
    keep = []
    if dense is not None:
        dense_a = np.ascontiguousarray(dense, dtype=np.float64).reshape(-1)
        keep.append(dense_a)
        dense_p, nnz, ci_p, cv_p = _ptr(dense_a), 0, None, None
    else:
        ci = np.ascontiguousarray(coo_idx, dtype=np.int64).reshape(-1, d)
        cv = np.ascontiguousarray(coo_val, dtype=np.float64).reshape(-1)
        keep += [ci, cv]
        dense_p, nnz, ci_p, cv_p = None, ci.shape[0], _ptr(ci), _ptr(cv)
    examined = lib().orc_sample(sampler, d, _ptr(dims_a), dense_p, nnz, ci_p, cv_p, s, p, q,
                                seed, problem_id, iteration, _ptr(idx), _ptr(xval), _ptr(st), _ptr(cand))
    if examined < 0:
        raise ValueError("oracle sample: bad arguments")
    return Samples(idx[:S], xval[:S], st[:S], cand[:S], examined)


def _factor_ptrs(A):
    A64 = [np.ascontiguousarray(a, dtype=np.float64) for a in A]
    arr = (ctypes.c_void_p * len(A64))(*[a.ctypes.data for a in A64])
    return A64, arr


def entry_weights(dims, smp: Samples, *, dense_w=None, coo_idx=None, coo_w=None, w_zero: float = 1.0):
    """The weight w_i of eq. wgcp at every sample: a stored entry's own weight,
    w_zero for entries a COO tensor does not store (and for zero samples)."""
    d = len(dims)
    dims_a = np.ascontiguousarray(dims, dtype=np.int64)
    S = len(smp)
    idx = np.ascontiguousarray(smp.idx, dtype=np.int64).reshape(-1)
    st = np.ascontiguousarray(smp.stratum, dtype=np.int32)
    out = np.zeros(max(S, 1), dtype=np.float64)
    keep = []
    if dense_w is not None:
        wd = np.ascontiguousarray(dense_w, dtype=np.float64).reshape(-1)
        keep.append(wd)
        rc = lib().orc_entry_weights(d, _ptr(dims_a), _ptr(wd), 0, None, None, float(w_zero), S, _ptr(idx),
                                     _ptr(st), _ptr(out))
    else:
        ci = np.ascontiguousarray(coo_idx, dtype=np.int64).reshape(-1, d)
        cw = np.ascontiguousarray(coo_w, dtype=np.float64).reshape(-1)
        keep += [ci, cw]
        rc = lib().orc_entry_weights(d, _ptr(dims_a), None, ci.shape[0], _ptr(ci), _ptr(cw), float(w_zero), S,
                                     _ptr(idx), _ptr(st), _ptr(out))
    if rc != 0:
        raise ValueError("oracle entry_weights: bad arguments")
    return out[:S]


def grad(loss: int, dims, A, smp: Samples, *, nnz: int = 0, s: int = 0, p: int = 0, q: int = 0,
         eps: float = LOSS_EPS, want_ytilde: bool = False, wgt=None, w_zero: float = 1.0):
    """Sampled gradient G_k (list of n_k x r float64) and the loss estimate;
    with ``wgt`` (entry weights per sample, see entry_weights) that of the
    weighted objective of eq. wgcp."""
    d = len(dims)
    r = A[0].shape[1]
    dims_a = np.ascontiguousarray(dims, dtype=np.int64)
    A64, Ap = _factor_ptrs(A)
    G = [np.zeros((n, r), dtype=np.float64) for n in dims]
    Gp = (ctypes.c_void_p * d)(*[g.ctypes.data for g in G])
    S = len(smp)
    idx = np.ascontiguousarray(smp.idx, dtype=np.int64).reshape(-1)
    xv = np.ascontiguousarray(smp.xval, dtype=np.float64)
    st = np.ascontiguousarray(smp.stratum, dtype=np.int32)
    yt = np.zeros(max(S, 1), dtype=np.float64)
    if wgt is None:
        F = lib().orc_grad(loss, d, _ptr(dims_a), r, Ap, S, _ptr(idx), _ptr(xv), _ptr(st),
                           nnz, s, p, q, eps, _ptr(yt), Gp)
    else:
        wg = np.ascontiguousarray(wgt, dtype=np.float64)
        F = lib().orc_grad_weighted(loss, d, _ptr(dims_a), r, Ap, S, _ptr(idx), _ptr(xv), _ptr(st), _ptr(wg),
                                    float(w_zero), nnz, s, p, q, eps, _ptr(yt), Gp)
    if want_ytilde:
        return G, F, yt[:S]
    return G, F


def full_grad(loss: int, A, dense, eps: float = LOSS_EPS):
    """Full gradient by enumerating every entry (eqs. Y, Gk); tiny tensors only."""
    dense_a = np.ascontiguousarray(dense, dtype=np.float64)
    dims = dense_a.shape
    d = len(dims)
    r = A[0].shape[1]
    dims_a = np.ascontiguousarray(dims, dtype=np.int64)
    A64, Ap = _factor_ptrs(A)
    G = [np.zeros((n, r), dtype=np.float64) for n in dims]
    Gp = (ctypes.c_void_p * d)(*[g.ctypes.data for g in G])
    F = lib().orc_full_grad(loss, d, _ptr(dims_a), r, Ap, _ptr(dense_a.reshape(-1)), eps, Gp)
    return G, F


def adam(A, G, B, C, t: int, alpha=0.01, beta1=0.9, beta2=0.999, eps=1e-8,
         lower=-np.inf, eps_mode: int = 0):
    """One Adam step (Alg. 4) in place on flat float64 arrays A, B, C; t >= 1."""
    for a in (A, B, C):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    G64 = np.ascontiguousarray(G, dtype=np.float64)
    lib().orc_adam(A.size, _ptr(A), _ptr(G64), _ptr(B), _ptr(C), int(t), alpha, beta1, beta2,
                   eps, lower, eps_mode)


def adam_fit(loss: int, dims, A0, *, dense=None, coo_idx=None, coo_val=None, grad_cfg: dict, est_cfg: dict,
             alpha=0.01, beta1=0.9, beta2=0.999, eps=1e-8, lower=-np.inf, eps_mode: int = 0, nu=0.1,
             tau=1000, kappa=1, max_epochs=100, loss_eps: float = LOSS_EPS):
    """GCP-Adam (Alg. 4) in FP64.

    ``grad_cfg`` and ``est_cfg`` are dicts with keys sampler, s, p, q, seed,
    problem_id and (gradient draws only) iteration: the j-th Adam step of the
    fit draws with iteration grad_cfg["iteration"] + j; the estimation set (EstObj, eqs. Fhat and
    Fhat-strat) is drawn once and reused.  After each epoch of ``tau`` steps
    the estimate is recomputed; if it rose, the epoch is undone (factors,
    moments and step count), the learning rate is multiplied by ``nu`` and the
    count of bad epochs grows; the loop ends when that count exceeds ``kappa``
    or after ``max_epochs`` epochs.  Control flow only: every draw, gradient,
    loss and Adam update is one of the calls above.

    Returns (A, history, accepted, alpha): history[0] is the first estimate,
    history[e] the estimate after epoch e; accepted[e] says if epoch e was kept.
    """
    d = len(dims)
    data = dict(dense=dense) if dense is not None else dict(coo_idx=coo_idx, coo_val=coo_val)
    nnz = 0 if coo_idx is None else int(np.asarray(coo_idx).shape[0])
    sizes = [int(dims[k]) * int(A0[0].shape[1]) for k in range(d)]
    A = np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in A0])
    B = np.zeros_like(A)
    C = np.zeros_like(A)
    r = A0[0].shape[1]

    def mats(flat):
        out, off = [], 0
        for k in range(d):
            out.append(flat[off:off + sizes[k]].reshape(dims[k], r))
            off += sizes[k]
        return out

    def wkw(c):
        return dict(nnz=nnz, s=c.get("s", 0), p=c.get("p", 0), q=c.get("q", 0))

    est = est_cfg
    est_smp = sample(est["sampler"], dims, s=est.get("s", 0), p=est.get("p", 0), q=est.get("q", 0),
                     seed=est["seed"], problem_id=est.get("problem_id", 0), iteration=est.get("iteration", 0), **data)

    def estimate():
        return grad(loss, dims, mats(A), est_smp, eps=loss_eps, **wkw(est))[1]

    F = estimate()
    history, accepted = [F], [True]
    bad, t, step, epoch = 0, 0, 0, 0
    while bad <= kappa and epoch < max_epochs:
        saved = (A.copy(), B.copy(), C.copy(), t)
        F_old = F
        for _ in range(tau):
            g = grad_cfg
            smp = sample(g["sampler"], dims, s=g.get("s", 0), p=g.get("p", 0), q=g.get("q", 0),
                         seed=g["seed"], problem_id=g.get("problem_id", 0),
                         iteration=g.get("iteration", 0) + step, **data)
            step += 1
            G, _ = grad(loss, dims, mats(A), smp, eps=loss_eps, **wkw(g))
            t += 1
            adam(A, np.concatenate([g.reshape(-1) for g in G]), B, C, t, alpha=alpha, beta1=beta1,
                 beta2=beta2, eps=eps, lower=lower, eps_mode=eps_mode)
        F = estimate()
        epoch += 1
        history.append(F)
        if F > F_old:
            A[:], B[:], C[:] = saved[0], saved[1], saved[2]
            if _mutation != 9:                       # 9 planted: the step count is not wound back
                t = saved[3]
            F = F_old
            alpha *= nu
            bad += 1
            accepted.append(False)
        else:
            accepted.append(True)
    return mats(A), history, accepted, alpha

