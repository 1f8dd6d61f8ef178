"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: sample indices, values and strata bit-exact; gradients element by
element within tol times the element's error scale (gpu_cases.check_grad) and
within tol in relative Frobenius norm per mode, tol = 1e-12 for FP64 factors
and 1e-5 for FP32 (and BF16 storage, the oracle on the rounded values); Adam
within the same bars.  Every case prints its name before it runs.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1906_01687_amd as gcp
from gpu_cases import (cfg_for, check_grad, oracle_grad, oracle_samples, oracle_scale, small_dense,
                       small_sparse, to_device, with_zero_factors)

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5}  # bf16: the oracle sees the bf16-rounded factors


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def u32(t):
    return t.to(torch.int64).cpu().numpy() & 0xFFFFFFFF


def check_samples(pb, smp_gpu, smp_orc):
    idx, xval, st = smp_gpu
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(idx), smp_orc.idx)
    np.testing.assert_array_equal(st.cpu().numpy().astype(np.int32), smp_orc.stratum)
    np.testing.assert_array_equal(xval.to(torch.float64).cpu().numpy(), smp_orc.xval)


# ---------------------------------------------------------------------------
# sampling: bit-exact indices
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("it", [0, 7])
def test_sample_uniform_dense_workload(it):
    announce(f"sample uniform dense 30x40x50 f64 it={it}")
    pb = to_device(synth.dense_gaussian_30x40x50())
    check_samples(pb, gcp.sample(pb.X, cfg_for(pb, iteration=it)), oracle_samples(pb, iteration=it))


@pytest.mark.parametrize("dims", [(13, 17, 11), (5, 9), (7, 3, 4, 6, 5), (1000,), (3, 2, 4, 2, 3, 2, 2, 3)])
def test_sample_uniform_dense_shapes(dims):
    announce(f"sample uniform dense {dims}")
    pb = to_device(small_dense(dims=dims, rank=3, s=2049))
    check_samples(pb, gcp.sample(pb.X, cfg_for(pb, iteration=3, problem_id=5)),
                  oracle_samples(pb, iteration=3, problem_id=5))


def test_sample_uniform_coo_lookup():
    announce("sample uniform on COO (hash value lookup)")
    w = small_sparse("counts", dims=(9, 8, 7), p=0, q=0)
    w.sampler, w.s = synth.UNIFORM, 5000
    pb = to_device(w)
    smp = oracle_samples(pb, iteration=2)
    assert np.count_nonzero(smp.xval) > 100
    check_samples(pb, gcp.sample(pb.X, cfg_for(pb, iteration=2)), smp)


@pytest.mark.parametrize("membership", ["bitmap", "hash"])
@pytest.mark.parametrize("p,q", [(2111, 3333), (0, 1025), (1024, 0), (1, 1), (64, 65537)])
def test_sample_stratified(p, q, membership):
    announce(f"sample stratified p={p} q={q} ({membership})")
    pb = to_device(small_sparse("binary", p=p, q=q), bitmap=membership == "bitmap")
    assert (pb.X.nz_bitmap is not None) == (membership == "bitmap")
    for it in (0, 11):
        check_samples(pb, gcp.sample(pb.X, cfg_for(pb, iteration=it)), oracle_samples(pb, iteration=it))


@pytest.mark.parametrize("membership", ["bitmap", "hash"])
@pytest.mark.parametrize("rho", [0.01, 0.5, 1.0, 3.0])
def test_sample_stratified_refill_independent_of_rho(rho, membership):
    announce(f"sample stratified rho={rho} (device-side refill, {membership})")
    w = small_sparse("binary", dims=(20, 19, 18), p=100, q=5000)
    pb = to_device(w, bitmap=membership == "bitmap")
    smp = oracle_samples(pb, iteration=4)
    check_samples(pb, gcp.sample(pb.X, cfg_for(pb, iteration=4, rho=rho)), smp)


@pytest.mark.parametrize("membership", ["bitmap", "hash"])
@pytest.mark.parametrize("rho", [0.01, 1.0])
def test_fused_stratified_refill(rho, membership):
    announce(f"fused stratified gradient, rho={rho} ({membership})")
    w = small_sparse("binary", dims=(20, 19, 18), p=700, q=5000)
    pb = to_device(w, bitmap=membership == "bitmap")
    G = gcp.sampled_grad(w.loss, pb.X, pb.M, cfg_for(pb, iteration=6, rho=rho))
    smp = oracle_samples(pb, iteration=6)
    Gref, _, _ = oracle_grad(pb, smp)
    torch.cuda.synchronize()
    check_grad(G, Gref, oracle_scale(pb, smp), 1e-5, f"refill rho={rho}")


def test_sample_stratified_dense_nonzeros():
    announce("sample stratified, 60% nonzeros (many rejections)")
    w = small_sparse("binary", dims=(12, 10, 9), p=300, q=4000)
    w2 = synth.sparse_binary((12, 10, 9), 7, 0.6, seed=77, subsample=20000)
    w.coo_idx, w.coo_val = w2[0], w2[1]
    pb = to_device(w)
    smp = oracle_samples(pb, iteration=1)
    assert smp.examined > 1.5 * 4000
    check_samples(pb, gcp.sample(pb.X, cfg_for(pb, iteration=1)), smp)


@pytest.mark.parametrize("dims", [(61, 47, 33), (30, 7, 11, 13), (6, 5, 4, 3, 7)])
def test_sample_semi_stratified(dims):
    announce(f"sample semi-stratified {dims}")
    pb = to_device(small_sparse("counts", dims=dims, p=1500, q=2500))
    check_samples(pb, gcp.sample(pb.X, cfg_for(pb, iteration=9)), oracle_samples(pb, iteration=9))


# ---------------------------------------------------------------------------
# derivative and MTTKRP, unfused ABI path
# ---------------------------------------------------------------------------

def _unfused(pb, cfg):
    idx, xval, st = gcp.sample(pb.X, cfg)
    y, fs = gcp.loss_grad(pb.w.loss, pb.X, cfg, pb.M, idx, xval, st, with_loss=True)
    G = gcp.mttkrp(pb.X, pb.M, idx, y)
    return idx, y, fs, G


CASES = [
    ("dense_30x40x50_f64", lambda: synth.dense_gaussian_30x40x50()),
    ("dense_f32_r5", lambda: small_dense()),
    ("dense_f32_poisson_r10", lambda: small_dense(rank=10, loss=synth.POISSON)),
    ("dense_f32_bernoulli_r1", lambda: small_dense(rank=1, loss=synth.BERNOULLI_ODDS)),
    # three modes, FP64 LDS partial, rows of 2 or 4 chunks: the swizzled
    # partial layout (each rank gives it a different shift and mask)
    ("dense_f32_r16_swizzled", lambda: small_dense(rank=16, loss=synth.POISSON)),
    ("dense_f32_r32_swizzled", lambda: small_dense(rank=32)),
    ("dense_f64_r8_swizzled", lambda: small_dense(rank=8, dtype="f64", loss=synth.BERNOULLI_ODDS)),
    # ranks 3 and 4: lane pairs at two columns per lane, a lane per sample at four
    ("dense_f32_r4", lambda: small_dense(rank=4, loss=synth.POISSON)),
    ("counts_strat_r3", lambda: small_sparse("counts", rank=3, sampler=synth.STRATIFIED)),
    ("binary_strat_r7", lambda: small_sparse("binary")),
    ("binary_semi_r8", lambda: small_sparse("binary", rank=8, sampler=synth.SEMI_STRATIFIED)),
    ("counts_semi_r10", lambda: small_sparse("counts", rank=10)),
    ("counts_strat_r33", lambda: small_sparse("counts", rank=33, sampler=synth.STRATIFIED)),
    ("counts_semi_r64_d4", lambda: small_sparse("counts", dims=(30, 7, 11, 13), rank=64)),
    ("dense_f32_d5_r16", lambda: small_dense(dims=(7, 3, 4, 6, 5), rank=16, s=1111)),
    ("dense_f64_d2_r2", lambda: small_dense(dims=(40, 31), rank=2, s=777, dtype="f64")),
    # one mode (the leave-one-out product is empty: every column of a row gets
    # the same w g) and six and eight modes
    ("dense_f32_d1_r6", lambda: small_dense(dims=(300,), rank=6, s=500)),
    ("dense_f64_d1_poisson_r5", lambda: small_dense(dims=(900,), rank=5, s=700, dtype="f64", loss=synth.POISSON)),
    ("dense_f32_d6_r9", lambda: small_dense(dims=(4, 3, 5, 2, 3, 4), rank=9, s=1500)),
    ("dense_f64_d8_r3", lambda: small_dense(dims=(3, 2, 4, 2, 3, 2, 2, 3), rank=3, s=900, dtype="f64")),
    ("dense_f32_gamma_r6", lambda: small_dense(rank=6, loss=synth.GAMMA)),
    ("dense_f64_beta_r4", lambda: small_dense(rank=4, loss=synth.BETA_HALF, dtype="f64")),
    ("counts_semi_beta_r10", lambda: small_sparse("counts", rank=10, loss=synth.BETA_HALF)),
    ("counts_strat_gamma_r5", lambda: small_sparse("counts", rank=5, sampler=synth.STRATIFIED, loss=synth.GAMMA)),
    # all modes (3012 x 8) fit in LDS only as FP32 partials (compare-and-swap adds)
    ("counts_semi_fp32_lds", lambda: small_sparse("counts", dims=(3000, 7, 5), rank=8, p=20000, q=30000)),
    ("dense_f32_r64_fp32_lds", lambda: small_dense(dims=(120, 110, 100), rank=64, s=5000)),
    ("dense_bf16_r64_fp32_lds", lambda: small_dense(dims=(120, 110, 100), rank=64, s=5000, dtype="bf16")),
    # mode 0 (6000 x 8) exceeds the LDS budget even in FP32: device-atomic fallback
    ("counts_semi_long_mode", lambda: small_sparse("counts", dims=(6000, 7, 5), rank=8, p=20000, q=30000)),
    # device accumulator rows padded to sector bounds: FP32 rows of 10 at a
    # 16-element stride, FP32 rows of 33 at 48, FP64 rows of 5 at 8
    ("counts_semi_long_mode_r10", lambda: small_sparse("counts", dims=(6000, 7, 5), rank=10, p=20000, q=30000)),
    ("counts_strat_long_mode_r33", lambda: small_sparse("counts", dims=(1500, 6, 5), rank=33, p=9000, q=7000,
                                                        sampler=synth.STRATIFIED)),
    ("dense_f64_long_mode_r5", lambda: small_dense(dims=(5000, 9, 7), rank=5, s=20000, dtype="f64")),
    # FP32 factors, but over 1024 adds per element of the long mode: FP64 accumulator
    ("dense_f32_long_mode_many_adds", lambda: small_dense(dims=(700, 5, 4), rank=64, s=800000)),
    # exact zeros at the projection bound: m = 0 for samples on a zero row, so
    # the Bernoulli-odds and Poisson derivatives reach 1e10 x
    ("binary_strat_zero_factors", lambda: with_zero_factors(small_sparse("binary", rank=8))),
    ("counts_semi_zero_factors", lambda: with_zero_factors(small_sparse("counts", rank=10))),
    ("dense_f32_bernoulli_zero_factors", lambda: with_zero_factors(small_dense(rank=6, loss=synth.BERNOULLI_ODDS))),
    ("dense_f32_poisson_zero_factors", lambda: with_zero_factors(small_dense(rank=4, loss=synth.POISSON))),
    # ranks above one wave's 64 lanes: 2 or 4 columns per lane, with wide
    # loads (r a multiple of the chunk) and with one load per column
    ("dense_f32_r100", lambda: small_dense(dims=(23, 19, 17), rank=100, s=3000)),
    ("dense_f64_r65", lambda: small_dense(dims=(11, 9, 8), rank=65, s=1500, dtype="f64")),
    ("counts_semi_r130", lambda: small_sparse("counts", dims=(30, 7, 11, 13), rank=130, p=900, q=1100)),
    ("dense_bf16_r256", lambda: small_dense(dims=(9, 8, 7), rank=256, s=700, dtype="bf16")),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_unfused_parity(name, make):
    announce(f"unfused sample->loss_grad->mttkrp {name}")
    w = make()
    pb = to_device(w)
    cfg = cfg_for(pb, iteration=5)
    idx, y, fs, G = _unfused(pb, cfg)
    smp = oracle_samples(pb, iteration=5)
    Gref, Fref, yref = oracle_grad(pb, smp)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(idx), smp.idx)
    tol = TOL[w.dtype]
    yg = y.to(torch.float64).cpu().numpy()
    assert np.linalg.norm(yg - yref) <= tol * np.linalg.norm(yref)
    assert abs(fs.item() - Fref) <= tol * max(1.0, abs(Fref)) * 10
    check_grad(G, Gref, oracle_scale(pb, smp), tol, f"unfused {name}")


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_fused_parity(name, make):
    announce(f"fused gcp_sampled_grad {name}")
    w = make()
    pb = to_device(w)
    for it in (0, 3):
        cfg = cfg_for(pb, iteration=it)
        G, fs = gcp.sampled_grad(w.loss, pb.X, pb.M, cfg, with_loss=True)
        smp = oracle_samples(pb, iteration=it)
        Gref, Fref, _ = oracle_grad(pb, smp)
        torch.cuda.synchronize()
        tol = TOL[w.dtype]
        check_grad(G, Gref, oracle_scale(pb, smp), tol, f"fused {name} it={it}")
        assert abs(fs.item() - Fref) <= 10 * tol * max(1.0, abs(Fref))


def test_fused_bf16_storage():
    announce("fused gcp_sampled_grad bf16 factors")
    w = small_sparse("counts", dims=(30, 7, 11, 13), rank=16)
    pb = to_device(w, dtype="bf16")
    cfg = cfg_for(pb, iteration=2)
    G = gcp.sampled_grad(w.loss, pb.X, pb.M, cfg)
    smp = oracle_samples(pb, iteration=2)
    Gref, _, _ = oracle_grad(pb, smp)          # oracle on the bf16-rounded values
    torch.cuda.synchronize()
    check_grad(G, Gref, oracle_scale(pb, smp), 1e-5, "bf16 storage")


def test_empty_sample_sets():
    announce("empty sample sets")
    pb = to_device(small_dense(s=0))
    G = gcp.sampled_grad(pb.w.loss, pb.X, pb.M, cfg_for(pb))
    torch.cuda.synchronize()
    assert all(float(g.abs().max()) == 0.0 for g in G)
    pb = to_device(small_sparse("binary", p=0, q=0))
    G = gcp.sampled_grad(pb.w.loss, pb.X, pb.M, cfg_for(pb))
    idx, xval, st = gcp.sample(pb.X, cfg_for(pb))
    torch.cuda.synchronize()
    assert idx.shape[0] == 0 and all(float(g.abs().max()) == 0.0 for g in G)


def test_mttkrp_accumulate():
    announce("gcp_mttkrp accumulate flag")
    pb = to_device(small_dense(rank=6))
    cfg = cfg_for(pb, iteration=1)
    idx, xval, st = gcp.sample(pb.X, cfg)
    y = gcp.loss_grad(pb.w.loss, pb.X, cfg, pb.M, idx, xval, st)
    G1 = [g.clone() for g in gcp.mttkrp(pb.X, pb.M, idx, y)]
    G2 = gcp.mttkrp(pb.X, pb.M, idx, y, out=[g.clone() for g in G1], accumulate=True)
    torch.cuda.synchronize()
    for a, b in zip(G1, G2):
        torch.testing.assert_close(b, 2 * a, rtol=1e-6, atol=0)


# ---------------------------------------------------------------------------
# Adam
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("eps_mode", [0, 1])
def test_adam_steps(dtype, eps_mode):
    announce(f"adam dtype={dtype} eps_mode={eps_mode}")
    w = small_sparse("counts", rank=10, dtype="f32")
    pb = to_device(w, dtype=dtype)
    adam = gcp.Adam(pb.M, lr=0.01, lower=0.0, eps_mode=eps_mode)
    A64 = np.concatenate([a.reshape(-1) for a in pb.A64])
    if dtype == "bf16":   # the master copy is float32 of the original values
        A64 = np.concatenate([np.float32(a).astype(np.float64).reshape(-1) for a in w.A_init])
    B = np.zeros_like(A64)
    C = np.zeros_like(A64)
    call = gcp.SampledGrad(w.loss, pb.X, pb.M, cfg_for(pb))
    tol = 1e-12 if dtype == "f64" else 1e-5
    for t in range(1, 4):
        call(iteration=t)
        gflat = call.gbuf
        g_host = gflat.to(torch.float64).cpu().numpy()     # the GPU gradient, fed to both updates
        A_before = A64.copy()
        adam.step(gflat)
        oracle.adam(A64, g_host, B, C, t, alpha=0.01, lower=0.0, eps_mode=eps_mode)
        torch.cuda.synchronize()
        assert int(adam.state[0].item()) == t and int(adam.state[1].item()) == 0
        got = (pb.M.master if dtype == "bf16" else pb.M.flat).to(torch.float64).cpu().numpy()
        # the step dA, relative Frobenius, as the acceptance bar states it
        d_ref = A64 - A_before
        d_got = got - A_before
        err = np.linalg.norm(d_got - d_ref) / np.linalg.norm(d_ref)
        assert err <= tol, (t, err)
        if dtype == "bf16":
            shadow = pb.M.flat.to(torch.float32).cpu().numpy()
            want = pb.M.master.cpu().to(torch.bfloat16).to(torch.float32).numpy()
            np.testing.assert_array_equal(shadow, want)
        # continue both from the device values so every step is compared from one start
        A64 = got.copy()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_sampled_adam_step_matches_two_calls(dtype):
    announce(f"gcp_sampled_adam_step vs gcp_sampled_grad + gcp_adam_step ({dtype})")
    w = small_sparse("binary", rank=8)
    pa, pb = to_device(w, dtype=dtype), to_device(w, dtype=dtype)
    adam_a = gcp.Adam(pa.M, lr=0.01, lower=0.0)
    adam_b = gcp.Adam(pb.M, lr=0.01, lower=0.0)
    fused = gcp.SampledAdamStep(w.loss, pa.X, pa.M, cfg_for(pa), adam_a, keep_grad=True)
    grad = gcp.SampledGrad(w.loss, pb.X, pb.M, cfg_for(pb))
    tol = 1e-12 if dtype == "f64" else 1e-5
    for it in range(4):
        before = (pb.M.master if dtype == "bf16" else pb.M.flat).to(torch.float64).clone()
        fused(iteration=it)
        grad(iteration=it)
        adam_b.step(grad.gbuf)
        torch.cuda.synchronize()
        ga, gb = fused.gbuf.to(torch.float64), grad.gbuf.to(torch.float64)
        assert float((ga - gb).norm() / gb.norm()) <= tol
        xa = (pa.M.master if dtype == "bf16" else pa.M.flat).to(torch.float64)
        xb = (pb.M.master if dtype == "bf16" else pb.M.flat).to(torch.float64)
        assert float((xa - xb).norm() / (xb - before).norm()) <= tol, it
        assert int(adam_a.state[0]) == it + 1 and int(adam_a.state[1]) == 0
        if dtype == "bf16":
            torch.testing.assert_close(pa.M.flat, pa.M.master.to(torch.bfloat16), rtol=0, atol=0)


@pytest.mark.parametrize("kind", ["binary", "counts"])
def test_graph_replay_with_device_iteration_counter(kind):
    announce(f"hipGraph replay of gcp_sampled_adam_step with a device iteration counter ({kind})")
    w = small_sparse(kind, rank=8)
    pa, pb = to_device(w), to_device(w)
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    cfg_a = gcp.sampling(w.sampler, p=w.p, q=w.q, seed=w.seed, iteration=100, iteration_counter=counter)
    adam_a = gcp.Adam(pa.M, lr=0.01, lower=0.0)
    adam_b = gcp.Adam(pb.M, lr=0.01, lower=0.0)
    step_a = gcp.SampledAdamStep(w.loss, pa.X, pa.M, cfg_a, adam_a, keep_grad=True)
    step_b = gcp.SampledAdamStep(w.loss, pb.X, pb.M, cfg_for(pb), adam_b, keep_grad=True)
    step_a()                                   # eager: iteration 100 + 0
    step_b(iteration=100)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step_a()
    for rep in range(1, 5):
        graph.replay()                         # iteration 100 + rep
        step_b(iteration=100 + rep)
        torch.cuda.synchronize()
        assert int(counter.item()) == rep + 1
        torch.testing.assert_close(step_a.gbuf, step_b.gbuf, rtol=1e-5, atol=1e-6 * float(step_b.gbuf.abs().max()))
        torch.testing.assert_close(pa.M.flat, pb.M.flat, rtol=1e-5, atol=1e-7)
        assert int(adam_a.state[0]) == int(adam_b.state[0]) == rep + 1
        _ = (pa.M.flat * 2).sum().item()        # unrelated eager work between replays


def test_sample_iteration_counter():
    announce("gcp_sample with a device iteration counter")
    pb = to_device(small_sparse("binary", p=300, q=500))
    counter = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    w = pb.w
    cfg = gcp.sampling(w.sampler, p=w.p, q=w.q, seed=w.seed, iteration=3, iteration_counter=counter)
    for rep in range(3):
        got = gcp.sample(pb.X, cfg)
        check_samples(pb, got, oracle_samples(pb, iteration=3 + 7 + rep))
        assert int(counter.item()) == 8 + rep


# ---------------------------------------------------------------------------
# full-size workloads
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("make", [synth.sparse_binary_1000x800x600, synth.sparse_count_6000x24x77x32],
                         ids=["binary_1000x800x600", "counts_6000x24x77x32"])
def test_full_size_workload(make):
    w = make()
    announce(f"full-size {w.name}: fused vs oracle, unfused indices bit-exact")
    pb = to_device(w)
    cfg = cfg_for(pb, iteration=1)
    G = gcp.sampled_grad(w.loss, pb.X, pb.M, cfg)
    Gg = [g.clone() for g in G]
    idx, xval, st = gcp.sample(pb.X, cfg)
    smp = oracle_samples(pb, iteration=1)
    Gref, _, _ = oracle_grad(pb, smp)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(idx), smp.idx)
    np.testing.assert_array_equal(xval.to(torch.float64).cpu().numpy(), smp.xval)
    check_grad(Gg, Gref, oracle_scale(pb, smp), 1e-5, f"full-size {w.name}")


VARIANT_CASES = [c for c in CASES if c[0] in (
    "dense_f32_r5", "binary_strat_r7", "binary_semi_r8", "counts_semi_r10", "counts_strat_r33", "dense_f32_d5_r16",
    "dense_f64_d2_r2", "counts_semi_fp32_lds", "dense_bf16_r64_fp32_lds", "counts_semi_long_mode_r10",
    "dense_f64_long_mode_r5", "counts_strat_gamma_r5", "dense_f32_r16_swizzled", "dense_f32_r32_swizzled",
    "dense_f64_r8_swizzled", "dense_f32_r4", "counts_strat_r3")]


@pytest.mark.parametrize("cpl", [1, 2, 4])
@pytest.mark.parametrize("name,make", VARIANT_CASES, ids=[c[0] for c in VARIANT_CASES])
def test_cols_per_lane_variants(name, make, cpl):
    """Every lane layout (1, 2 or 4 rank columns per lane, where it fits the
    rank) gives the oracle's gradient, fused and unfused."""
    announce(f"cols_per_lane={cpl}: {name}")
    w = make()
    pb = to_device(w)
    gcp.set_cols_per_lane(cpl)
    try:
        cfg = cfg_for(pb, iteration=4)
        G, fs = gcp.sampled_grad(w.loss, pb.X, pb.M, cfg, with_loss=True)
        G = [g.clone() for g in G]
        idx, y, fs2, G2 = _unfused(pb, cfg)
        smp = oracle_samples(pb, iteration=4)
        Gref, Fref, yref = oracle_grad(pb, smp)
        torch.cuda.synchronize()
    finally:
        gcp.set_cols_per_lane(0)
    tol = TOL[w.dtype]
    E = oracle_scale(pb, smp)
    check_grad(G, Gref, E, tol, f"fused cpl={cpl} {name}")
    check_grad(G2, Gref, E, tol, f"unfused cpl={cpl} {name}")
    yg = y.to(torch.float64).cpu().numpy()
    assert np.linalg.norm(yg - yref) <= tol * np.linalg.norm(yref)
    assert abs(fs.item() - Fref) <= 10 * tol * max(1.0, abs(Fref))
