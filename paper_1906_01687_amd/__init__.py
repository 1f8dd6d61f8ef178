"""MI355X-native sampled GCP gradient (Kolda & Hong, Stochastic Gradients for
Large-Scale Tensor Decomposition): hand-written HIP kernels for gfx950 behind
the C ABI in include/gcp.h, with a thin torch binding in ``api``."""
from . import _lib
from ._lib import BATCH_CONTIGUOUS, BATCH_LPT
from .autograd import SampledLoss, sampled_loss
from .score import factor_match_score
from .api import (Adam, Batch, FitResult, adam_fit, DataTensor, Factors, LOSSES, Problem, SAMPLERS, SampledAdamStep, SampledGrad, set_cols_per_lane,
                  coo_tensor, dense_tensor, loss_grad, mttkrp, n_samples, sample, sampled_grad, sampling)

__all__ = ["BATCH_CONTIGUOUS", "BATCH_LPT", "Adam", "Batch", "DataTensor", "Factors", "LOSSES", "Problem", "SAMPLERS", "SampledAdamStep",
           "SampledGrad", "coo_tensor", "dense_tensor", "loss_grad", "mttkrp", "n_samples", "sample",
           "sampled_grad", "sampling", "set_cols_per_lane", "SampledLoss", "sampled_loss", "FitResult", "adam_fit", "factor_match_score"]
