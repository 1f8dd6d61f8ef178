"""Torch-facing binding of libgcp: argument marshalling only.

Every step of the sampled GCP gradient runs in the HIP kernels behind the C
ABI (include/gcp.h).  torch supplies device memory (tensors, workspaces) and
the current HIP stream; nothing here computes any part of the method.

Index tensors hold the ABI's uint32 mode indices in torch.int32 storage.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import (BF16, COO, DENSE, F32, F64, GcpFactors, GcpSampling, GcpTensor, check, lib)

LOSSES = {"gaussian": _lib.GAUSSIAN, "bernoulli_odds": _lib.BERNOULLI_ODDS, "poisson": _lib.POISSON,
          "gamma": _lib.GAMMA, "beta_half": _lib.BETA_HALF}
SAMPLERS = {"uniform": _lib.UNIFORM, "stratified": _lib.STRATIFIED, "semi_stratified": _lib.SEMI_STRATIFIED,
            "full": _lib.FULL}
LOSS_EPS = 1e-10

_TORCH_DTYPE = {F32: torch.float32, F64: torch.float64, BF16: torch.bfloat16}
_CODE = {torch.float32: F32, torch.float64: F64, torch.bfloat16: BF16}


def _stream(stream: Optional[torch.cuda.Stream] = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _loss_code(loss) -> int:
    return LOSSES[loss] if isinstance(loss, str) else int(loss)


def _sampler_code(sampler) -> int:
    return SAMPLERS[sampler] if isinstance(sampler, str) else int(sampler)


# ---------------------------------------------------------------------------
# data tensor
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class DataTensor:
    """Device description of X: dense row-major values or COO (indices + values)."""
    dims: tuple
    values: torch.Tensor
    coo_idx: Optional[torch.Tensor] = None      # [nnz, d] int32 (uint32 bits)
    nz_table: Optional[torch.Tensor] = None     # uint8 bytes of the nonzero hash
    nz_slots: int = 0
    nz_bitmap: Optional[torch.Tensor] = None    # int32 words of the membership bitmap
    weights: Optional[torch.Tensor] = None      # entry weights (eq. wgcp), same dtype and layout as values
    w_zero: float = 1.0                         # COO with weights: weight of the entries not stored

    @property
    def d(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return 0 if self.coo_idx is None else int(self.coo_idx.shape[0])

    @property
    def is_dense(self) -> bool:
        return self.coo_idx is None

    @property
    def omega(self) -> int:
        return math.prod(int(n) for n in self.dims)

    def struct(self) -> GcpTensor:
        t = GcpTensor()
        t.d = self.d
        t.format = DENSE if self.is_dense else COO
        t.vdtype = _CODE[self.values.dtype]
        for k, n in enumerate(self.dims):
            t.dims[k] = int(n)
        t.values = _ptr(self.values)
        t.coo_idx = _ptr(self.coo_idx)
        t.nnz = self.nnz
        t.nz_table = _ptr(self.nz_table)
        t.nz_slots = int(self.nz_slots)
        t.nz_bitmap = _ptr(self.nz_bitmap)
        t.weights = _ptr(self.weights)
        t.w_zero = float(self.w_zero)
        return t


def _check_weights(weights: Optional[torch.Tensor], values: torch.Tensor) -> Optional[torch.Tensor]:
    if weights is None:
        return None
    if weights.dtype != values.dtype or weights.shape != values.shape or weights.device != values.device:
        raise ValueError("weights must match the values in dtype, shape and device")
    return weights.contiguous()


def dense_tensor(X: torch.Tensor, weights: Optional[torch.Tensor] = None) -> DataTensor:
    """Dense row-major X; ``weights`` (same shape) gives the entry weights of
    the weighted objective (eq. wgcp), e.g. 0 for missing entries."""
    if X.dtype not in (torch.float32, torch.float64) or not X.is_contiguous():
        raise ValueError("dense X must be a contiguous float32/float64 tensor")
    return DataTensor(tuple(X.shape), X, weights=_check_weights(weights, X))


BITMAP_LIMIT_BYTES = 1 << 30


def coo_tensor(dims: Sequence[int], coo_idx: torch.Tensor, values: torch.Tensor,
               build_index: bool = True, bitmap: Optional[bool] = None, stream=None,
               weights: Optional[torch.Tensor] = None, w_zero: float = 1.0) -> DataTensor:
    """COO tensor; builds the nonzero hash (gcp_nz_index_build) unless told not
    to, and the membership bitmap (gcp_nz_bitmap_build) when ``bitmap`` is True,
    or when it is None and the bitmap takes at most BITMAP_LIMIT_BYTES.
    ``weights`` (one per stored entry) and ``w_zero`` (every other entry) give
    the weighted objective of eq. wgcp."""
    if coo_idx.dtype != torch.int32 or coo_idx.dim() != 2 or coo_idx.shape[1] != len(dims):
        raise ValueError("coo_idx must be an [nnz, d] int32 tensor")
    X = DataTensor(tuple(int(n) for n in dims), values.contiguous(), coo_idx.contiguous(),
                   weights=_check_weights(weights, values), w_zero=float(w_zero))
    if build_index:
        L = lib()
        slots = int(L.gcp_nz_table_slots(X.nnz))
        table = torch.empty(int(L.gcp_nz_table_bytes(slots)), dtype=torch.uint8, device=values.device)
        t = X.struct()
        check(L.gcp_nz_index_build(ctypes.byref(t), _ptr(table), slots, _stream(stream)))
        X.nz_table, X.nz_slots = table, slots
    t = X.struct()
    nbytes = int(lib().gcp_nz_bitmap_bytes(ctypes.byref(t)))
    if bitmap or (bitmap is None and 0 < nbytes <= BITMAP_LIMIT_BYTES):
        bm = torch.empty((nbytes + 3) // 4, dtype=torch.int32, device=values.device)
        check(lib().gcp_nz_bitmap_build(ctypes.byref(t), _ptr(bm), nbytes, _stream(stream)))
        X.nz_bitmap = bm
    return X


# ---------------------------------------------------------------------------
# factors and sampling configuration
# ---------------------------------------------------------------------------

class Factors:
    """A_1..A_d in one flat buffer (row-major n_k x r blocks), as the Adam step wants.

    dtype float64/float32: ``flat`` is the parameter vector.  bfloat16: ``master``
    (float32) is updated by Adam and ``flat`` is its bf16 copy used for gathers.
    """

    def __init__(self, dims: Sequence[int], rank: int, dtype: torch.dtype, device, init=None):
        self.dims = tuple(int(n) for n in dims)
        self.rank = int(rank)
        self.dtype = dtype
        self.sizes = [n * self.rank for n in self.dims]
        self.P = sum(self.sizes)
        self.flat = torch.zeros(self.P, dtype=dtype, device=device)
        self.master = torch.zeros(self.P, dtype=torch.float32, device=device) if dtype == torch.bfloat16 else None
        if init is not None:
            self.load(init)

    def _views(self, buf: torch.Tensor) -> List[torch.Tensor]:
        out, off = [], 0
        for n, sz in zip(self.dims, self.sizes):
            out.append(buf[off:off + sz].view(n, self.rank))
            off += sz
        return out

    @property
    def A(self) -> List[torch.Tensor]:
        return self._views(self.flat)

    def load(self, mats) -> None:
        src = torch.cat([torch.as_tensor(m).reshape(-1).to(torch.float64) for m in mats])
        if self.master is not None:
            self.master.copy_(src.to(torch.float32))
            self.flat.copy_(self.master.to(torch.bfloat16))
        else:
            self.flat.copy_(src.to(self.dtype))

    def grad_buffer(self) -> torch.Tensor:
        gdt = torch.float64 if self.dtype == torch.float64 else torch.float32
        return torch.zeros(self.P, dtype=gdt, device=self.flat.device)

    def grad_views(self, buf: torch.Tensor) -> List[torch.Tensor]:
        return self._views(buf)

    def struct(self) -> GcpFactors:
        m = GcpFactors()
        m.dtype = _CODE[self.dtype]
        m.rank = self.rank
        for k, a in enumerate(self.A):
            m.A[k] = _ptr(a)
        return m


def sampling(sampler="uniform", s=0, p=0, q=0, seed=0, problem_id=0, iteration=0, rho=0.0,
             iteration_counter: Optional[torch.Tensor] = None) -> GcpSampling:
    """A gcp_sampling struct.  ``iteration_counter`` (a 1-element int64 device
    tensor the caller keeps alive) makes each call draw with iteration +
    counter and then advance the counter on the device."""
    c = GcpSampling()
    c.sampler = _sampler_code(sampler)
    c.s, c.p, c.q = int(s), int(p), int(q)
    c.seed, c.problem_id, c.iteration = int(seed), int(problem_id), int(iteration)
    c.rho = float(rho)
    if iteration_counter is not None:
        if iteration_counter.dtype != torch.int64 or iteration_counter.numel() < 1 or not iteration_counter.is_cuda:
            raise ValueError("iteration_counter must be an int64 device tensor")
        c.iteration_counter = _ptr(iteration_counter)
    return c


def n_samples(cfg: GcpSampling, X: Optional["DataTensor"] = None) -> int:
    """Samples one draw yields (FULL: every entry of X)."""
    if cfg.sampler == _lib.FULL:
        if X is None:
            raise ValueError("the FULL sampler's sample count needs the tensor")
        return X.omega
    return cfg.s if cfg.sampler == _lib.UNIFORM else cfg.p + cfg.q


def _ptr_array(tensors) -> ctypes.Array:
    return (ctypes.c_void_p * len(tensors))(*[_ptr(t) for t in tensors])


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def set_cols_per_lane(cpl: int) -> None:
    """gcp_set_cols_per_lane: rank columns per lane of the gradient kernels
    (1, 2 or 4; 0 picks by rank) for every later single-problem call."""
    check(lib().gcp_set_cols_per_lane(int(cpl)))


def _rejection_status(X: DataTensor, M: Optional["Factors"], cfg: GcpSampling, ws: torch.Tensor) -> int:
    """The rejection status word of a finished call (0: all q zeros drawn; 1:
    the device refill stopped at its cap); 0 for calls without rejection."""
    t = X.struct()
    m = M.struct() if M is not None else None
    off = int(lib().gcp_rejection_status_offset(ctypes.byref(t), ctypes.byref(m) if m is not None else None,
                                                ctypes.byref(cfg)))
    if off < 0:
        return 0
    return int(ws[off:off + 4].cpu().view(torch.int32)[0].item())


def sample(X: DataTensor, cfg: GcpSampling, stream=None, check_status: bool = False):
    """gcp_sample: (idx [S, d] int32, xval [S], stratum [S] uint8).  With
    check_status, waits for the call and raises if the rejection refill
    stopped at its cap."""
    L = lib()
    dev = X.values.device
    S = n_samples(cfg, X)
    idx = torch.empty((max(S, 1), X.d), dtype=torch.int32, device=dev)
    xval = torch.empty(max(S, 1), dtype=X.values.dtype, device=dev)
    st = torch.empty(max(S, 1), dtype=torch.uint8, device=dev)
    t = X.struct()
    nbytes = int(L.gcp_sample_workspace_bytes(ctypes.byref(t), ctypes.byref(cfg)))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    check(L.gcp_sample(ctypes.byref(t), ctypes.byref(cfg), _ptr(idx), _ptr(xval), _ptr(st),
                       _ptr(ws), nbytes, _stream(stream)))
    if check_status and _rejection_status(X, None, cfg, ws) != 0:
        raise _lib.GcpError(2, "stratified rejection stopped at its refill cap")
    return idx[:S], xval[:S], st[:S]


def loss_grad(loss, X: DataTensor, cfg: GcpSampling, M: Factors, idx, xval, stratum,
              eps: float = LOSS_EPS, with_loss: bool = False, stream=None):
    """gcp_loss_grad: ytilde [S] (and the loss estimate as a device double)."""
    L = lib()
    S = int(idx.shape[0])
    ydt = torch.float64 if M.dtype == torch.float64 else torch.float32
    y = torch.empty(max(S, 1), dtype=ydt, device=X.values.device)
    fs = torch.zeros(1, dtype=torch.float64, device=X.values.device) if with_loss else None
    t, m = X.struct(), M.struct()
    check(L.gcp_loss_grad(_loss_code(loss), ctypes.byref(t), ctypes.byref(cfg), ctypes.byref(m),
                          _ptr(idx), _ptr(xval), _ptr(stratum), S, float(eps), _ptr(y), _ptr(fs),
                          _stream(stream)))
    return (y[:S], fs) if with_loss else y[:S]


def mttkrp(X: DataTensor, M: Factors, idx, ytilde, out: Optional[List[torch.Tensor]] = None,
           accumulate: bool = False, stream=None) -> List[torch.Tensor]:
    """gcp_mttkrp: G_k for every mode (list of n_k x r tensors)."""
    L = lib()
    if out is None:
        out = M.grad_views(M.grad_buffer())
    t, m = X.struct(), M.struct()
    nbytes = int(L.gcp_mttkrp_workspace_bytes(ctypes.byref(t), ctypes.byref(m), int(idx.shape[0])))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=X.values.device)
    check(L.gcp_mttkrp(ctypes.byref(t), ctypes.byref(m), _ptr(idx), _ptr(ytilde), int(idx.shape[0]),
                       _ptr_array(out), int(bool(accumulate)), _ptr(ws), nbytes, _stream(stream)))
    return out


class SampledGrad:
    """Reusable gcp_sampled_grad call: descriptors and workspace set up once."""

    def __init__(self, loss, X: DataTensor, M: Factors, cfg: GcpSampling, eps: float = LOSS_EPS,
                 out: Optional[List[torch.Tensor]] = None, with_loss: bool = False):
        L = lib()
        self.loss = _loss_code(loss)
        self.X, self.M, self.cfg, self.eps = X, M, cfg, float(eps)
        self.t, self.m = X.struct(), M.struct()
        self.gbuf = None
        if out is None:
            self.gbuf = M.grad_buffer()
            out = M.grad_views(self.gbuf)
        self.out = out
        self.out_ptrs = _ptr_array(out)
        self.nbytes = int(L.gcp_sampled_grad_workspace_bytes(ctypes.byref(self.t), ctypes.byref(self.m),
                                                              ctypes.byref(cfg)))
        self.ws = torch.empty(max(self.nbytes, 1), dtype=torch.uint8, device=X.values.device)
        self.loss_sum = torch.zeros(1, dtype=torch.float64, device=X.values.device) if with_loss else None

    def __call__(self, iteration: Optional[int] = None, stream=None) -> List[torch.Tensor]:
        if iteration is not None:
            self.cfg.iteration = int(iteration)
        check(lib().gcp_sampled_grad(self.loss, ctypes.byref(self.t), ctypes.byref(self.m),
                                     ctypes.byref(self.cfg), self.eps, self.out_ptrs, _ptr(self.loss_sum),
                                     _ptr(self.ws), self.nbytes, _stream(stream)))
        return self.out

    def rejection_status(self) -> int:
        """Status word of the last call's rejection step (waits for it)."""
        return _rejection_status(self.X, self.M, self.cfg, self.ws)


def sampled_grad(loss, X: DataTensor, M: Factors, cfg: GcpSampling, eps: float = LOSS_EPS,
                 out=None, with_loss: bool = False, stream=None):
    """gcp_sampled_grad in one call: G_k (and the loss estimate if asked)."""
    call = SampledGrad(loss, X, M, cfg, eps, out, with_loss)
    G = call(stream=stream)
    return (G, call.loss_sum) if with_loss else G


class SampledAdamStep:
    """gcp_sampled_adam_step: sampled gradient and Adam update in one call (Alg. 4 inner loop)."""

    def __init__(self, loss, X: DataTensor, M: Factors, cfg: GcpSampling, adam: "Adam",
                 eps: float = LOSS_EPS, keep_grad: bool = False, with_loss: bool = False):
        L = lib()
        if adam.M is not M:
            raise ValueError("adam must belong to the same Factors")
        self.loss = _loss_code(loss)
        self.X, self.M, self.cfg, self.adam, self.eps = X, M, cfg, adam, float(eps)
        self.t, self.m = X.struct(), M.struct()
        self.gbuf = M.grad_buffer() if keep_grad else None
        self.out_ptrs = _ptr_array(M.grad_views(self.gbuf)) if keep_grad else None
        self.nbytes = int(L.gcp_sampled_grad_workspace_bytes(ctypes.byref(self.t), ctypes.byref(self.m),
                                                              ctypes.byref(cfg)))
        self.ws = torch.empty(max(self.nbytes, 1), dtype=torch.uint8, device=X.values.device)
        self.loss_sum = torch.zeros(1, dtype=torch.float64, device=X.values.device) if with_loss else None

    def __call__(self, iteration: Optional[int] = None, stream=None) -> None:
        if iteration is not None:
            self.cfg.iteration = int(iteration)
        a, M = self.adam, self.M
        check(lib().gcp_sampled_adam_step(
            self.loss, ctypes.byref(self.t), ctypes.byref(self.m), ctypes.byref(self.cfg), self.eps,
            _ptr(M.flat), _ptr(M.master), _ptr(a.B), _ptr(a.C), _ptr(a.state), float(a.lr), float(a.beta1),
            float(a.beta2), float(a.eps), float(a.lower), int(a.eps_mode), self.out_ptrs, _ptr(self.loss_sum),
            _ptr(self.ws), self.nbytes, _stream(stream)))

    def rejection_status(self) -> int:
        """Status word of the last call's rejection step (waits for it)."""
        return _rejection_status(self.X, self.M, self.cfg, self.ws)


class Adam:
    """Adam moments B, C and the device step counter for a Factors set (Alg. 4)."""

    def __init__(self, M: Factors, lr: float = 0.01, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, lower: float = -math.inf, eps_mode: int = _lib.EPS_INSIDE_SQRT):
        self.M = M
        mdt = torch.float64 if M.dtype == torch.float64 else torch.float32
        dev = M.flat.device
        self.B = torch.zeros(M.P, dtype=mdt, device=dev)
        self.C = torch.zeros(M.P, dtype=mdt, device=dev)
        self.state = torch.zeros(2, dtype=torch.int64, device=dev)
        self.lr, self.beta1, self.beta2, self.eps, self.lower = lr, beta1, beta2, eps, lower
        self.eps_mode = eps_mode

    def step(self, G_flat: torch.Tensor, stream=None) -> None:
        M = self.M
        check(lib().gcp_adam_step(M.P, _CODE[M.dtype], _ptr(M.flat), _ptr(M.master), _ptr(G_flat),
                                  _ptr(self.B), _ptr(self.C), _ptr(self.state), float(self.lr),
                                  float(self.beta1), float(self.beta2), float(self.eps), float(self.lower),
                                  int(self.eps_mode), _stream(stream)))


@dataclasses.dataclass
class FitResult:
    history: List[float]      # [0] first estimate, [e] estimate after epoch e
    accepted: List[bool]      # epoch e kept (False: undone)
    epochs: int
    alpha: float              # final learning rate
    adam: "Adam"


def adam_fit(loss, X: DataTensor, M: Factors, grad: GcpSampling, est: GcpSampling, *, lr: float = 0.01,
             beta1: float = 0.9, beta2: float = 0.999, adam_eps: float = 1e-8, lower: float = -math.inf,
             nu: float = 0.1, tau: int = 1000, kappa: int = 1, max_epochs: int = 100,
             eps_mode: int = _lib.EPS_INSIDE_SQRT, eps: float = LOSS_EPS, adam: Optional["Adam"] = None,
             stream=None) -> FitResult:
    """gcp_adam_fit: GCP-Adam (Alg. 4) on M in place, with the loss estimated on
    the fixed sample set ``est`` once per epoch."""
    L = lib()
    adam = adam or Adam(M, lr=lr, beta1=beta1, beta2=beta2, eps=adam_eps, lower=lower, eps_mode=eps_mode)
    o = _lib.GcpFitOptions()
    o.grad, o.est = grad, est
    o.alpha, o.beta1, o.beta2, o.adam_eps = float(lr), float(beta1), float(beta2), float(adam_eps)
    o.lower, o.nu, o.eps_mode = float(lower), float(nu), int(eps_mode)
    o.tau, o.kappa, o.max_epochs = int(tau), int(kappa), int(max_epochs)
    t, m = X.struct(), M.struct()
    nbytes = int(L.gcp_adam_fit_workspace_bytes(ctypes.byref(t), ctypes.byref(m), ctypes.byref(o)))
    if nbytes == 0:
        raise _lib.GcpError(1, L.gcp_last_error().decode())
    ws = torch.empty(nbytes, dtype=torch.uint8, device=X.values.device)
    hist = (ctypes.c_double * (max_epochs + 1))()
    acc = (ctypes.c_int8 * (max_epochs + 1))()
    ep, alpha = ctypes.c_int32(), ctypes.c_double()
    check(L.gcp_adam_fit(_loss_code(loss), ctypes.byref(t), ctypes.byref(m), ctypes.byref(o), float(eps),
                         _ptr(M.flat), _ptr(M.master), _ptr(adam.B), _ptr(adam.C), _ptr(adam.state), hist, acc,
                         ctypes.byref(ep), ctypes.byref(alpha), _ptr(ws), nbytes, _stream(stream)))
    n = ep.value
    return FitResult([hist[i] for i in range(n + 1)], [bool(acc[i]) for i in range(n + 1)], n, alpha.value, adam)


# ---------------------------------------------------------------------------
# batches of independent problems (gcp_batched_*)
# ---------------------------------------------------------------------------

class Problem:
    """One problem of a batch: data, factors, sampling, loss and Adam buffers."""

    def __init__(self, loss, X: DataTensor, M: Factors, cfg: GcpSampling, eps: float = LOSS_EPS,
                 lower: float = -math.inf, keep_grad: bool = False):
        self.loss = _loss_code(loss)
        self.X, self.M, self.cfg = X, M, cfg
        self.eps, self.lower = float(eps), float(lower)
        mdt = torch.float64 if M.dtype == torch.float64 else torch.float32
        dev = M.flat.device
        self.B = torch.zeros(M.P, dtype=mdt, device=dev)
        self.C = torch.zeros(M.P, dtype=mdt, device=dev)
        self.G = torch.zeros(M.P, dtype=mdt, device=dev) if keep_grad else None

    def struct(self, with_grad: bool = True) -> _lib.GcpProblem:
        pr = _lib.GcpProblem()
        pr.X = self.X.struct()
        pr.M = self.M.struct()
        pr.cfg = self.cfg
        pr.loss = self.loss
        pr.eps = self.eps
        pr.lower = self.lower
        pr.A = _ptr(self.M.flat)
        pr.A_master = _ptr(self.M.master)
        pr.B = _ptr(self.B)
        pr.C = _ptr(self.C)
        pr.G = _ptr(self.G) if with_grad else None
        return pr


class Batch:
    """A planned and prepared batch: one gradient launch and one reduction (+ Adam)
    advance every problem.  ``tune`` = (threads, unit_items[, schedule[,
    cols_per_lane]]) or None for defaults; schedule is BATCH_CONTIGUOUS
    (default) or BATCH_LPT; cols_per_lane is 1, 2, 4 or 0 (by rank)."""

    def __init__(self, problems: Sequence[Problem], tune=None, with_grad: bool = True):
        L = lib()
        self.problems = list(problems)
        arr = (_lib.GcpProblem * len(self.problems))(*[p.struct(with_grad) for p in self.problems])
        t = _lib.GcpBatchTuning()
        if tune is not None:
            t.threads, t.unit_items = int(tune[0]), int(tune[1])
            t.schedule = int(tune[2]) if len(tune) > 2 else _lib.BATCH_CONTIGUOUS
            t.cols_per_lane = int(tune[3]) if len(tune) > 3 else 0
        self.tune = tune
        h = ctypes.c_void_p()
        check(L.gcp_batched_create(arr, len(self.problems), ctypes.byref(t), ctypes.byref(h)))
        self.handle = h
        dev = self.problems[0].M.flat.device
        self.nbytes = int(L.gcp_batched_workspace_bytes(h))
        self.ws = torch.empty(max(self.nbytes, 1), dtype=torch.uint8, device=dev)
        check(L.gcp_batched_prepare(h, _ptr(self.ws), self.nbytes, _stream(None)))
        self.state = torch.zeros(2, dtype=torch.int64, device=dev)
        self.counter = torch.zeros(1, dtype=torch.int64, device=dev)

    def plan(self):
        """The host plan: (block_ptr, unit_problem, unit_items[n_units, 2]) as numpy arrays."""
        import numpy as np
        L = lib()
        nb, nu = ctypes.c_int64(), ctypes.c_int64()
        check(L.gcp_batched_plan(self.handle, ctypes.byref(nb), ctypes.byref(nu), None, None, None))
        bp = np.zeros(nb.value + 1, dtype=np.int64)
        up = np.zeros(max(1, nu.value), dtype=np.int32)
        ui = np.zeros((max(1, nu.value), 2), dtype=np.int64)
        check(L.gcp_batched_plan(self.handle, None, None, bp.ctypes.data, up.ctypes.data, ui.ctypes.data))
        return bp, up[:nu.value], ui[:nu.value]

    def grad(self, stream=None) -> None:
        check(lib().gcp_batched_grad(self.handle, _ptr(self.counter), _stream(stream)))

    def adam_step(self, lr: float = 0.01, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                  eps_mode: int = _lib.EPS_INSIDE_SQRT, stream=None) -> None:
        check(lib().gcp_batched_adam_step(self.handle, _ptr(self.state), _ptr(self.counter), float(lr),
                                          float(beta1), float(beta2), float(eps), int(eps_mode), _stream(stream)))

    def capture_adam_steps(self, steps: int, lr: float = 0.01, beta1: float = 0.9, beta2: float = 0.999,
                           eps: float = 1e-8, eps_mode: int = _lib.EPS_INSIDE_SQRT) -> None:
        """gcp_batched_graph_capture: `steps` batched Adam steps recorded into a
        graph the batch owns (each step draws the next samples through the
        batch's iteration counter); replay with graph_launch()."""
        check(lib().gcp_batched_graph_capture(self.handle, int(steps), _ptr(self.state), _ptr(self.counter),
                                              float(lr), float(beta1), float(beta2), float(eps), int(eps_mode)))

    def graph_launch(self, stream=None) -> None:
        """gcp_batched_graph_launch: replay the captured steps on the stream."""
        check(lib().gcp_batched_graph_launch(self.handle, _stream(stream)))

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().gcp_batched_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
