"""GPU parity of batches (gcp_batched_*): one launch pair advances many problems.

Every problem of a batch draws the samples it would draw alone, so its batched
gradient and Adam step must agree with the single-problem calls and with the
oracle: element by element and in relative Frobenius norm (gpu_cases.check_grad),
1e-5 for FP32 factors, 1e-12 for FP64.  The 64-cube batch of dense problems
(sides 20-300, ranks 4-32, three losses, 2 % of the entries per problem) is
checked whole, at the launch shape the autotuner picks.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_1906_01687_amd as gcp
from paper_1906_01687_amd import autotune
from gpu_cases import TORCH_DT, check_grad, grad_scale, host_rounded, rel_fro, small_sparse

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def make_problem(w, pid, dtype=None, keep_grad=True):
    dev = torch.device("cuda:0")
    dtype = dtype or w.dtype
    vdt = torch.float64 if dtype == "f64" else torch.float32
    if w.dense is not None:
        X = gcp.dense_tensor(torch.as_tensor(np.ascontiguousarray(w.dense)).to(vdt).to(dev))
    else:
        X = gcp.coo_tensor(w.dims, torch.as_tensor(np.ascontiguousarray(w.coo_idx).view(np.int32)).to(dev),
                           torch.as_tensor(w.coo_val).to(vdt).to(dev))
    M = gcp.Factors(w.dims, w.rank, TORCH_DT[dtype], dev, init=w.A_init)
    cfg = gcp.sampling(w.sampler, s=w.s, p=w.p, q=w.q, seed=w.seed, problem_id=pid)
    return gcp.Problem(w.loss, X, M, cfg, lower=w.lower, keep_grad=keep_grad)


def mixed_workloads(dtype="f32"):
    """Dense cubes of several sides, ranks and losses plus sparse semi-stratified problems."""
    out = []
    losses = [synth.GAUSSIAN, synth.POISSON, synth.BERNOULLI_ODDS, synth.GAMMA, synth.BETA_HALF]
    specs = [(9, 1, 0), (17, 4, 1), (23, 7, 2), (31, 16, 0), (12, 33, 1), (40, 8, 2), (26, 5, 0), (15, 6, 3),
             (21, 3, 4)]
    for b, (n, r, loss) in enumerate(specs):
        X, A0, lower = synth.dense_problem((n, n, n), r, losses[loss], seed=900 + b,
                                           density=0.05 if loss in (1, 2) else None)
        out.append(synth.Workload(f"cube{b}", (n, n, n), r, losses[loss], synth.UNIFORM, dtype,
                                  s=max(37, int(0.03 * n ** 3)), dense=X, A_init=A0, seed=77, lower=lower))
    out.append(small_sparse("counts", dims=(41, 23, 17), rank=10, p=1500, q=2100, dtype=dtype))
    out.append(small_sparse("binary", dims=(33, 29, 18), rank=6, p=900, q=1300, dtype=dtype,
                            sampler=synth.SEMI_STRATIFIED))
    return out


def oracle_gradient(w, pid, iteration, dtype):
    A64 = host_rounded(w.A_init, dtype)
    if w.dense is not None:
        dense = torch.as_tensor(np.asarray(w.dense)).to(torch.float64 if dtype == "f64" else torch.float32)
        smp = oracle.sample(w.sampler, w.dims, dense=dense.to(torch.float64).numpy(), s=w.s, seed=w.seed,
                            problem_id=pid, iteration=iteration)
    else:
        smp = oracle.sample(w.sampler, w.dims, coo_idx=np.asarray(w.coo_idx, dtype=np.int64),
                            coo_val=np.asarray(w.coo_val, dtype=np.float64), p=w.p, q=w.q, seed=w.seed,
                            problem_id=pid, iteration=iteration)
    G, _ = oracle.grad(w.loss, w.dims, A64, smp, nnz=w.nnz, s=w.s, p=w.p, q=w.q)
    return G, grad_scale(w.loss, w.dims, A64, smp, nnz=w.nnz, s=w.s, p=w.p, q=w.q)


@pytest.mark.parametrize("tune", [None, (256, 0, gcp.BATCH_CONTIGUOUS), (512, 0, gcp.BATCH_CONTIGUOUS),
                                  (256, 8, gcp.BATCH_LPT), (512, 1, gcp.BATCH_LPT), (1024, 200, gcp.BATCH_LPT),
                                  (1024, 64, gcp.BATCH_LPT, 1), (512, 16, gcp.BATCH_LPT, 2),
                                  (1024, 0, gcp.BATCH_CONTIGUOUS, 4)])
def test_batched_grad_matches_single_problem_calls(tune):
    announce(f"batched gradient vs single-problem calls and the oracle, tune={tune}")
    ws = mixed_workloads()
    probs = [make_problem(w, b) for b, w in enumerate(ws)]
    batch = gcp.Batch(probs, tune=tune)
    for it in range(2):
        batch.grad()
        torch.cuda.synchronize()
        assert int(batch.counter.item()) == it + 1
        for b, (w, p) in enumerate(zip(ws, probs)):
            cfg = gcp.sampling(w.sampler, s=w.s, p=w.p, q=w.q, seed=w.seed, problem_id=b, iteration=it)
            single = gcp.sampled_grad(w.loss, p.X, p.M, cfg)
            torch.cuda.synchronize()
            Gb = p.M.grad_views(p.G)
            err = max(rel_fro(Gb, [s.detach().to(torch.float64).cpu().numpy() for s in single]))
            assert err <= 1e-5, (b, it, err)
            if it == 0:
                check_grad(Gb, *oracle_gradient(w, b, it, "f32"), 1e-5, f"batched problem {b}")
    batch.close()


@pytest.mark.parametrize("cpl", [0, 2])
def test_batched_high_ranks(cpl):
    """Ranks 64-256 (two or four rank columns per lane, 32 or 64 lanes per
    sample) in one FP32 batch, with the automatic layout and with two columns
    per lane asked for (rank 256 falls back to four): every problem against
    its single-problem call and the oracle."""
    announce(f"batched gradient, ranks 64-256, cols_per_lane={cpl}")
    specs = [(11, 64, 0), (9, 100, 1), (8, 256, 0), (13, 130, 2), (10, 17, 1)]
    losses = [synth.GAUSSIAN, synth.POISSON, synth.BERNOULLI_ODDS]
    ws = []
    for b, (n, r, loss) in enumerate(specs):
        X, A0, lower = synth.dense_problem((n, n + 1, n + 2), r, losses[loss], seed=980 + b,
                                           density=0.05 if loss else None)
        ws.append(synth.Workload(f"hr{b}", (n, n + 1, n + 2), r, losses[loss], synth.UNIFORM, "f32",
                                 s=max(64, n ** 3 // 4), dense=X, A_init=A0, seed=81, lower=lower))
    probs = [make_problem(w, b) for b, w in enumerate(ws)]
    batch = gcp.Batch(probs, tune=(1024, 0, gcp.BATCH_CONTIGUOUS, cpl) if cpl else None)
    batch.grad()
    torch.cuda.synchronize()
    for b, (w, p) in enumerate(zip(ws, probs)):
        cfg = gcp.sampling(w.sampler, s=w.s, seed=w.seed, problem_id=b)
        single = gcp.sampled_grad(w.loss, p.X, p.M, cfg)
        torch.cuda.synchronize()
        Gb = p.M.grad_views(p.G)
        err = max(rel_fro(Gb, [s_.detach().to(torch.float64).cpu().numpy() for s_ in single]))
        assert err <= 1e-5, (b, err)
        check_grad(Gb, *oracle_gradient(w, b, 0, "f32"), 1e-5, f"batched rank {w.rank}")
    batch.close()


@pytest.mark.parametrize("dims_list", [[(37,), (120,)], [(30, 20), (9, 41), (50, 3)],
                                       [(7, 8, 9, 10), (5, 12, 6, 9)], [(4, 5, 6, 3, 7), (6, 3, 5, 4, 4)]],
                         ids=["d1", "d2", "d4", "d5"])
def test_batched_other_tensor_orders(dims_list):
    """Batches of 1-, 2-, 4- and 5-way dense problems (one order per batch):
    every problem against its single-problem call and the oracle."""
    d = len(dims_list[0])
    announce(f"batched gradient, {d}-way problems")
    losses = [synth.GAUSSIAN, synth.POISSON, synth.BERNOULLI_ODDS]
    ws = []
    for b, dims in enumerate(dims_list):
        loss = losses[b % 3]
        r = [3, 8, 5][b % 3]
        X, A0, lower = synth.dense_problem(dims, r, loss, seed=990 + 10 * d + b,
                                           density=0.1 if loss != synth.GAUSSIAN else None)
        ws.append(synth.Workload(f"o{d}_{b}", dims, r, loss, synth.UNIFORM, "f32",
                                 s=max(50, math.prod(dims) // 3), dense=X, A_init=A0, seed=82, lower=lower))
    probs = [make_problem(w, b) for b, w in enumerate(ws)]
    batch = gcp.Batch(probs)
    batch.grad()
    torch.cuda.synchronize()
    for b, (w, p) in enumerate(zip(ws, probs)):
        cfg = gcp.sampling(w.sampler, s=w.s, seed=w.seed, problem_id=b)
        single = gcp.sampled_grad(w.loss, p.X, p.M, cfg)
        torch.cuda.synchronize()
        Gb = p.M.grad_views(p.G)
        err = max(rel_fro(Gb, [s_.detach().to(torch.float64).cpu().numpy() for s_ in single]))
        assert err <= 1e-5, (b, err)
        check_grad(Gb, *oracle_gradient(w, b, 0, "f32"), 1e-5, f"batched {d}-way problem {b}")
    batch.close()


def test_batched_fp64():
    announce("batched gradient, FP64 factors")
    ws = mixed_workloads(dtype="f64")[:5]
    probs = [make_problem(w, b, dtype="f64") for b, w in enumerate(ws)]
    batch = gcp.Batch(probs)
    batch.grad()
    torch.cuda.synchronize()
    for b, (w, p) in enumerate(zip(ws, probs)):
        check_grad(p.M.grad_views(p.G), *oracle_gradient(w, b, 0, "f64"), 1e-12, f"batched FP64 problem {b}")
    batch.close()


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
def test_batched_adam_matches_single_problem_steps(dtype):
    """BF16 factors: the Adam step updates the float master copy and rounds it
    to the BF16 factors; the master copies are compared.  FP64: the two
    gradients differ only in the order of FP64 additions, hence 1e-10."""
    announce(f"batched Adam steps vs single-problem gcp_sampled_adam_step, {dtype}")
    ws = mixed_workloads(dtype=dtype)
    pa = [make_problem(w, b) for b, w in enumerate(ws)]
    pb = [make_problem(w, b) for b, w in enumerate(ws)]
    params = (lambda p: p.M.master) if dtype == "bf16" else (lambda p: p.M.flat)
    batch = gcp.Batch(pa)
    singles = []
    for b, (w, p) in enumerate(zip(ws, pb)):
        adam = gcp.Adam(p.M, lr=0.01, lower=w.lower)
        cfg = gcp.sampling(w.sampler, s=w.s, p=w.p, q=w.q, seed=w.seed, problem_id=b)
        singles.append((gcp.SampledAdamStep(w.loss, p.X, p.M, cfg, adam), adam))
    for it in range(3):
        before = [params(p).to(torch.float64).clone() for p in pb]
        batch.adam_step(lr=0.01)
        for step, _ in singles:
            step(iteration=it)
        torch.cuda.synchronize()
        assert int(batch.state[0]) == it + 1
        for b in range(len(ws)):
            xa, xb = params(pa[b]).to(torch.float64), params(pb[b]).to(torch.float64)
            err = float((xa - xb).norm() / (xb - before[b]).norm().clamp_min(1e-30))
            assert err <= (1e-10 if dtype == "f64" else 1e-5), (b, it, err)
            if dtype == "bf16":  # the factors are the master copy rounded to BF16
                assert torch.equal(pa[b].M.flat, pa[b].M.master.to(torch.bfloat16)), (b, it)
    batch.close()


def test_batched_graph_replay():
    announce("hipGraph replay of a batched Adam step")
    ws = mixed_workloads()[:6]
    pa = [make_problem(w, b) for b, w in enumerate(ws)]
    pb = [make_problem(w, b) for b, w in enumerate(ws)]
    ba, bb = gcp.Batch(pa), gcp.Batch(pb)
    ba.adam_step()
    bb.adam_step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ba.adam_step()
    for rep in range(3):
        graph.replay()
        bb.adam_step()
        torch.cuda.synchronize()
        for b in range(len(ws)):
            torch.testing.assert_close(pa[b].M.flat, pb[b].M.flat, rtol=1e-5, atol=1e-7)
        _ = sum(float(p.M.flat.sum()) for p in pa)   # unrelated eager work between replays
    ba.close()
    bb.close()


def test_library_graph_replay_equals_eager_steps():
    """gcp_batched_graph_capture / _launch: a library-owned graph of 3 batched
    Adam steps, replayed twice with eager work in between, equals 6 eager
    steps (the iteration counter gives every replayed step fresh samples)."""
    announce("library-owned graph of batched Adam steps vs eager steps")
    ws = mixed_workloads()[:7]
    pa = [make_problem(w, b) for b, w in enumerate(ws)]
    pb = [make_problem(w, b) for b, w in enumerate(ws)]
    ba, bb = gcp.Batch(pa), gcp.Batch(pb)
    ba.capture_adam_steps(3, lr=0.02)
    torch.cuda.synchronize()
    assert int(ba.counter.item()) == 0 and int(ba.state[0].item()) == 0     # capture ran nothing
    for rep in range(2):
        ba.graph_launch()
        for _ in range(3):
            bb.adam_step(lr=0.02)
        torch.cuda.synchronize()
        assert int(ba.counter.item()) == int(bb.counter.item()) == 3 * (rep + 1)
        assert int(ba.state[0].item()) == int(bb.state[0].item()) == 3 * (rep + 1)
        for b in range(len(ws)):
            torch.testing.assert_close(pa[b].M.flat, pb[b].M.flat, rtol=1e-5, atol=1e-7)
        _ = sum(float(p.M.flat.sum()) for p in pa)   # unrelated eager work between replays
    ba.capture_adam_steps(1, lr=0.02)                # a new capture replaces the graph
    ba.graph_launch()
    bb.adam_step(lr=0.02)
    torch.cuda.synchronize()
    for b in range(len(ws)):
        torch.testing.assert_close(pa[b].M.flat, pb[b].M.flat, rtol=1e-5, atol=1e-7)
    ba.close()
    bb.close()


def test_batched_reduction_table_longer_than_its_grid():
    """A batch whose reduction has more blocks of 256 parameters than the
    reduction grid holds (65536): (600000 + 2 + 2) x 32 parameters make 75001
    blocks, so some workgroups take two.  Adam steps against the
    single-problem calls."""
    announce("batched: reduction block table longer than the grid")
    specs = [((600_000, 2, 2), 32, 20_000), ((23, 23, 23), 7, 400)]
    ws = []
    for b, (dims, r, s_) in enumerate(specs):
        X, A0, _ = synth.dense_problem(dims, r, synth.GAUSSIAN, seed=970 + b)
        ws.append(synth.Workload(f"long{b}", dims, r, synth.GAUSSIAN, synth.UNIFORM, "f32", s=s_, dense=X,
                                 A_init=A0, seed=80))
    assert (600_004 * 32 + 255) // 256 > 65536
    pa = [make_problem(w, b) for b, w in enumerate(ws)]
    pb = [make_problem(w, b) for b, w in enumerate(ws)]
    batch = gcp.Batch(pa)
    singles = []
    for b, (w, p) in enumerate(zip(ws, pb)):
        adam = gcp.Adam(p.M, lr=0.01, lower=w.lower)
        cfg = gcp.sampling(w.sampler, s=w.s, seed=w.seed, problem_id=b)
        singles.append(gcp.SampledAdamStep(w.loss, p.X, p.M, cfg, adam))
    for it in range(2):
        before = [p.M.flat.to(torch.float64).clone() for p in pb]
        batch.adam_step(lr=0.01)
        for step in singles:
            step(iteration=it)
        torch.cuda.synchronize()
        for b in range(len(ws)):
            xa, xb = pa[b].M.flat.to(torch.float64), pb[b].M.flat.to(torch.float64)
            err = float((xa - xb).norm() / (xb - before[b]).norm().clamp_min(1e-30))
            assert err <= 1e-5, (b, it, err)
    batch.close()


def test_batched_large_problems_use_fp32_lds_and_atomics():
    announce("batched: problems beyond the FP64 LDS budget (FP32 LDS, device atomics)")
    # (700+20+15) x 32: 188 KB in FP64 -> FP32 LDS; (1500+35) x 32: 196 KB even in FP32 -> atomics
    specs = [(700, 32), (1500, 32), (50, 4)]
    ws = []
    for b, (n, r) in enumerate(specs):
        dims = (n, 20, 15)
        X, A0, lower = synth.dense_problem(dims, r, synth.GAUSSIAN, seed=950 + b)
        ws.append(synth.Workload(f"big{b}", dims, r, synth.GAUSSIAN, synth.UNIFORM, "f32", s=40_000, dense=X,
                                 A_init=A0, seed=78))
    probs = [make_problem(w, b) for b, w in enumerate(ws)]
    batch = gcp.Batch(probs)
    batch.grad()
    torch.cuda.synchronize()
    for b, (w, p) in enumerate(zip(ws, probs)):
        check_grad(p.M.grad_views(p.G), *oracle_gradient(w, b, 0, "f32"), 1e-5, f"batched large problem {b}")
    batch.close()


def test_batch_of_64_cubes_full_size():
    """The 64-problem batch at its own size (3.34e6 samples per step), at the
    autotuned launch shape: every problem against the oracle and against its
    single-problem call on the same samples."""
    ws = synth.batch_of_cubes(64)
    announce(f"64-cube batch, {sum(w.s for w in ws)} samples, sides {min(w.dims[0] for w in ws)}-"
             f"{max(w.dims[0] for w in ws)}")
    probs = [make_problem(w, w.problem_id) for w in ws]
    best, _ = autotune.tune_batch(probs, steps=3, cache_path=None)
    announce(f"64-cube batch at the autotuned shape {best}")
    batch = gcp.Batch(probs, tune=best)
    batch.grad()
    torch.cuda.synchronize()
    for w, p in zip(ws, probs):
        b = w.problem_id
        cfg = gcp.sampling(w.sampler, s=w.s, seed=w.seed, problem_id=b, iteration=0)
        single = gcp.sampled_grad(w.loss, p.X, p.M, cfg)
        torch.cuda.synchronize()
        Gb = p.M.grad_views(p.G)
        err = max(rel_fro(Gb, [t.detach().to(torch.float64).cpu().numpy() for t in single]))
        assert err <= 1e-5, (b, err)
        check_grad(Gb, *oracle_gradient(w, b, 0, "f32"), 1e-5, f"64-cube batch problem {b} ({w.name})")
    batch.close()


def test_autotune_picks_a_candidate(tmp_path):
    announce("autotune over two launch shapes")
    ws = mixed_workloads()[:4]
    probs = [make_problem(w, b) for b, w in enumerate(ws)]
    before = [p.M.flat.clone() for p in probs]
    cache = str(tmp_path / "tune.json")
    cands = [(256, 8, gcp.BATCH_LPT), (1024, 0, gcp.BATCH_CONTIGUOUS)]
    best, times = autotune.tune_batch(probs, candidates=cands, steps=3, cache_path=cache)
    assert best in cands and len(times) == 2
    best2, _ = autotune.tune_batch(probs, candidates=[(512, 16, gcp.BATCH_LPT)], cache_path=cache)   # cached
    assert best2 == best
    torch.cuda.synchronize()
    for p, a in zip(probs, before):
        assert torch.equal(p.M.flat, a)          # tuning leaves the parameters alone
