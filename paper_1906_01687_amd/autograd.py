"""The sampled GCP loss as a differentiable torch function.

F(A) = sum_i w_i f(x_i, m_i) over one sample set (the estimate of eqs. Fhat
and Fhat-strat; for the corrected nonzeros of semi-stratified sampling
w (f(x,m) - f(0,m))).  Its gradient with respect to A_k is the sparse MTTKRP
of ytilde_i = w_i g(x_i, m_i) (eqs. mttkrp, Gks), so:

* forward  = gcp_sample (draws, data lookup, strata) + gcp_loss_grad (model
  entries, ytilde and the loss estimate);
* backward = gcp_mttkrp_scaled of the saved ytilde at the saved indices,
  scaled on the device by the incoming gradient.

The differentiable input is a flat parameter vector laid out like a
``Factors`` set: normally ``flat`` itself for FP64 and FP32 storage and the
FP32 ``master`` for BF16 storage.  The kernels read the Factors storage, so a
forward on another tensor first copies it there (FP64/FP32), and for BF16
storage every forward refreshes the BF16 gather copy ``flat`` from the
parameter with gcp_bf16_round.  The parameter is saved for backward, so an
in-place change between forward and backward raises instead of giving the
gradient at other factors.  Gradients come back in the parameter's dtype (FP32
accumulation for FP32 and BF16 storage, FP64 for FP64).

With ``cfg.iteration_counter`` set, every forward draws a fresh sample set and
advances the counter on the device; without it the samples are fixed by
``cfg.iteration`` (what a finite-difference check needs).
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import GcpSampling, check, lib
from .api import (LOSS_EPS, DataTensor, Factors, _loss_code, _ptr, _ptr_array, _stream, n_samples)


class _SampledLossFn(torch.autograd.Function):

    @staticmethod
    def forward(ctx, param: torch.Tensor, sl: "SampledLoss"):
        M = sl.M
        want = torch.float32 if M.master is not None else M.dtype
        if param.dtype != want or param.numel() != M.P or param.device != M.flat.device:
            raise ValueError(f"param must be a {want} vector of {M.P} values on {M.flat.device}")
        if M.master is not None:
            # BF16 storage: the gathers read the rounded copy of the FP32 parameter
            check(lib().gcp_bf16_round(M.P, _ptr(param.detach()), _ptr(M.flat), _stream(None)))
        elif param.data_ptr() != M.flat.data_ptr():
            M.flat.copy_(param.detach())
        idx, y, fs = sl._forward()
        ctx.sl = sl
        ctx.save_for_backward(param, idx, y)
        return fs.view(())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        _, idx, y = ctx.saved_tensors
        scale = grad_out.detach().to(torch.float64).reshape(1).contiguous()
        G = ctx.sl._backward(idx, y, scale=scale)
        return G, None


class SampledLoss:
    """Callable F(param) for data X, factors M, sampling cfg and a loss."""

    def __init__(self, loss, X: DataTensor, M: Factors, cfg: GcpSampling, eps: float = LOSS_EPS):
        L = lib()
        self.loss = _loss_code(loss)
        self.X, self.M, self.cfg, self.eps = X, M, cfg, float(eps)
        self.t, self.m = X.struct(), M.struct()
        self.S = n_samples(cfg, X)
        dev = X.values.device
        self.dev = dev
        self.sample_bytes = int(L.gcp_sample_workspace_bytes(ctypes.byref(self.t), ctypes.byref(cfg)))
        self.sample_ws = torch.empty(max(self.sample_bytes, 1), dtype=torch.uint8, device=dev)
        self.mttkrp_bytes = int(L.gcp_mttkrp_workspace_bytes(ctypes.byref(self.t), ctypes.byref(self.m), self.S))
        self.mttkrp_ws = torch.empty(max(self.mttkrp_bytes, 1), dtype=torch.uint8, device=dev)
        self.ydtype = torch.float64 if M.dtype == torch.float64 else torch.float32

    def parameter(self) -> torch.Tensor:
        """The leaf tensor to optimise (requires_grad set)."""
        p = self.M.master if self.M.master is not None else self.M.flat
        return p.requires_grad_(True)

    def __call__(self, param: Optional[torch.Tensor] = None) -> torch.Tensor:
        if param is None:
            param = self.parameter()
        return _SampledLossFn.apply(param, self)

    # -- the two halves -----------------------------------------------------
    def _forward(self, stream=None):
        L = lib()
        S, d = self.S, self.X.d
        idx = torch.empty((max(S, 1), d), dtype=torch.int32, device=self.dev)
        xval = torch.empty(max(S, 1), dtype=self.X.values.dtype, device=self.dev)
        st = torch.empty(max(S, 1), dtype=torch.uint8, device=self.dev)
        y = torch.empty(max(S, 1), dtype=self.ydtype, device=self.dev)
        fs = torch.zeros(1, dtype=torch.float64, device=self.dev)
        s = _stream(stream)
        check(L.gcp_sample(ctypes.byref(self.t), ctypes.byref(self.cfg), _ptr(idx), _ptr(xval), _ptr(st),
                           _ptr(self.sample_ws), self.sample_bytes, s))
        check(L.gcp_loss_grad(self.loss, ctypes.byref(self.t), ctypes.byref(self.cfg), ctypes.byref(self.m),
                              _ptr(idx), _ptr(xval), _ptr(st), S, self.eps, _ptr(y), _ptr(fs), s))
        return idx, y, fs

    def _backward(self, idx: torch.Tensor, y: torch.Tensor, scale: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
        L = lib()
        G = self.M.grad_buffer()
        check(L.gcp_mttkrp_scaled(ctypes.byref(self.t), ctypes.byref(self.m), _ptr(idx), _ptr(y), self.S,
                                  _ptr_array(self.M.grad_views(G)), 0, _ptr(scale), _ptr(self.mttkrp_ws),
                                  self.mttkrp_bytes, _stream(stream)))
        return G


def sampled_loss(loss, X: DataTensor, M: Factors, cfg: GcpSampling, eps: float = LOSS_EPS) -> torch.Tensor:
    """One differentiable evaluation of the sampled loss at M's parameters."""
    sl = SampledLoss(loss, X, M, cfg, eps)
    return sl(sl.parameter())
