"""Empirical bias and variance of the stochastic gradient (the quantities of
the paper's sampler comparison, Sec. 5.4, Table 1).

For N draws g_1..g_N of the vectorised gradient [vec(G_1); ...; vec(G_d)]
(iterations cfg.iteration + 0..N-1 of the sample stream):

* empirical bias     = || mean - g ||_2, g the exact gradient (the FULL sampler);
* empirical variance = (1/N) sum_xi || g_xi - mean ||_2^2.

Every gradient is one fused gcp_sampled_grad call; the running sums are
accumulated in FP64 on the device.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import _lib
from .api import LOSS_EPS, DataTensor, Factors, GcpSampling, SampledGrad, sampling


@dataclasses.dataclass
class Moments:
    bias: Optional[float]      # || mean - exact ||, None without the exact gradient
    variance: float            # (1/N) sum || g_xi - mean ||^2
    grad_norm: Optional[float] # || exact ||
    mean_norm: float
    draws: int


def exact_gradient(loss, X: DataTensor, M: Factors, eps: float = LOSS_EPS) -> torch.Tensor:
    """The full gradient (every entry once, weight 1) as one flat FP64 vector."""
    sg = SampledGrad(loss, X, M, sampling("full"), eps)
    sg()
    return sg.gbuf.to(torch.float64)


def gradient_moments(loss, X: DataTensor, M: Factors, cfg: GcpSampling, N: int,
                     exact: Optional[torch.Tensor] = None, eps: float = LOSS_EPS) -> Moments:
    sg = SampledGrad(loss, X, M, cfg, eps)
    base = int(cfg.iteration)
    total = torch.zeros(M.P, dtype=torch.float64, device=X.values.device)
    total_sq = torch.zeros_like(total)
    for xi in range(N):
        sg(iteration=base + xi)
        g = sg.gbuf.to(torch.float64)
        total += g
        total_sq += g * g
    mean = total / N
    # (1/N) sum ||g - mean||^2 = (1/N) sum ||g||^2 - ||mean||^2
    var = float((total_sq / N).sum() - (mean * mean).sum())
    cfg.iteration = base
    bias = float((mean - exact).norm()) if exact is not None else None
    gnorm = float(exact.norm()) if exact is not None else None
    return Moments(bias, var, gnorm, float(mean.norm()), N)
