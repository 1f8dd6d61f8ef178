"""The allocation-free entry point gcp_sampled_grad_noalloc, through the C ABI:
its gradient equals gcp_sampled_grad's (with a caller workspace) and the
oracle's on the same samples, on two calls in a row whose second problem is
smaller than the first (the shared static scratch keeps the first call's
contents, so whatever must start at zero has to be cleared by each call)."""
import ctypes
import sys

import pytest
import torch

import synth
import paper_1906_01687_amd as gcp
from paper_1906_01687_amd import _lib
from gpu_cases import cfg_for, check_grad, oracle_grad, oracle_samples, oracle_scale, rel_fro, small_dense, \
    small_sparse, to_device

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _noalloc(pb, cfg, with_loss=True):
    L = _lib.lib()
    t, m = pb.X.struct(), pb.M.struct()
    G = pb.M.grad_views(pb.M.grad_buffer())
    Gp = (ctypes.c_void_p * len(G))(*[g.data_ptr() for g in G])
    fs = torch.zeros(1, dtype=torch.float64, device="cuda") if with_loss else None
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(L.gcp_sampled_grad_noalloc(gcp.api._loss_code(pb.w.loss), ctypes.byref(t), ctypes.byref(m),
                                          ctypes.byref(cfg), 1e-10, Gp,
                                          ctypes.c_void_p(fs.data_ptr()) if fs is not None else None, stream))
    return G, fs


def test_noalloc_equals_workspace_entry_point():
    # the first problem is the larger one: stratified rejection, a long mode
    # that takes device atomics (an accumulator the call must clear), FP32
    # LDS partials; the second is a small dense problem
    cases = [("counts 6000x7x5 semi-stratified (device atomics)",
              small_sparse("counts", dims=(6000, 7, 5), rank=8, p=20000, q=30000)),
             ("binary 61x47x33 stratified (rejection)", small_sparse("binary", rank=8)),
             ("dense 13x17x11 uniform", small_dense(rank=5))]
    for rep in range(2):
        for name, w in cases:
            announce(f"no-alloc call {rep}: {name}")
            pb = to_device(w)
            cfg = cfg_for(pb, iteration=3 + rep)
            G_ws, fs_ws = gcp.sampled_grad(w.loss, pb.X, pb.M, cfg, with_loss=True)
            G_na, fs_na = _noalloc(pb, cfg)
            torch.cuda.synchronize()
            assert max(rel_fro(G_na, [g.double().cpu().numpy() for g in G_ws])) <= 1e-6
            smp = oracle_samples(pb, iteration=3 + rep)
            Gref, Fref, _ = oracle_grad(pb, smp)
            check_grad(G_na, Gref, oracle_scale(pb, smp), 1e-5, f"no-alloc {name}")
            assert abs(fs_na.item() - Fref) <= 1e-4 * max(1.0, abs(Fref))
            assert abs(fs_na.item() - fs_ws.item()) <= 1e-6 * max(1.0, abs(fs_ws.item()))
