"""Benchmark: sampled GCP gradient + Adam step on one MI355X.

A step is one pass of the whole hot path over one fresh sample set: index
draws (stratified: nonzero picks plus zeros by rejection), model entries,
weighted loss derivatives, the MTTKRP scatter into every mode, and the Adam
update -- the library's gcp_sampled_adam_step, with all inputs resident in
HBM.  The default workload is the sparse binary tensor
1000x800x600 (about 1e6 nonzeros, rank 8, FP32 factors, Bernoulli-odds loss,
stratified sampling p = q = 1e5).

Prints one JSON line.  `value` is sampled entries per second over the timed
steps; `roofline` prices the dominant kernel (the fused gradient kernel) by
its algorithmic bytes against MI355X's 8 TB/s; `cpu_baseline` times the FP64
oracle on a bounded sample of the same workload on one host core.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sparse_binary_1000x800x600",
                    help="sparse_binary_1000x800x600 | sparse_count_6000x24x77x32 | dense_gaussian_30x40x50 | "
                         "dense_gaussian_200x200x200x200[_bf16] | batched_64_cubes")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="bound on the oracle timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch every step eagerly")
    ap.add_argument("--autograd", action="store_true",
                    help="also time the step as SampledLoss forward + backward + Adam")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--study", choices=["variance"], default=None,
                    help="variance: the sampler comparison of Sec. 5.4 (empirical bias and variance, Table 1) "
                         "on the 400x300x200x100 binary tensor instead of the throughput bench")
    ap.add_argument("--draws", type=int, default=1000, help="stochastic gradients per sampler and model (study)")
    ap.add_argument("--fit-epochs", type=int, default=60, help="GCP-Adam epoch cap for the fitted model (study)")
    return ap.parse_args()


def algorithmic_bytes(w) -> float:
    """Bytes a cacheless fused kernel must move for one gradient of workload w.

    Per sample: d rows of r factor values (b_f each), a read-modify-write of d
    gradient rows of r values at 4 + 4 bytes (FP32 accumulation), and the data
    bytes its stratum reads: uniform dense x (b_v); nonzero pick a COO row
    (4 d) plus its value (b_v); stratified zero the 8-byte key of its
    membership probe; semi-stratified zero nothing.
    """
    d, r = w.d, w.rank
    bf = {"f64": 8, "f32": 4, "bf16": 2}[w.dtype]
    bv = 8 if w.dtype == "f64" else 4
    rmw = 16 if w.dtype == "f64" else 8
    per = d * r * bf + d * r * rmw
    if w.sampler == 0:
        return w.s * (per + bv)
    zero_data = 8 if w.sampler == 1 else 0
    return w.p * (per + 4 * d + bv) + w.q * (per + zero_data)


KERNEL_SOURCES = ["paper_1906_01687_amd/csrc/grad.hip", "paper_1906_01687_amd/csrc/grad_device.hpp",
                  "paper_1906_01687_amd/csrc/device.hpp", "paper_1906_01687_amd/csrc/common.hpp"]


def kernel_source_hash(read=None) -> str:
    """SHA-256 of the gradient kernel's sources with comments and whitespace
    removed, so that a comment edit does not retire a profile but any code
    change does.  ``read(rel)`` returns a source's text (default: the tree)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
                text = fh.read()
        else:
            text = read(rel)
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update("".join(text.split()).encode())
    return h.hexdigest()


def profiled_traffic(workload: str):
    """HBM bytes per launch of the gradient kernel from the committed PMC summary
    (FETCH_SIZE + WRITE_SIZE, calibrated on a copy), or None when there is no
    summary for this workload or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"grad_kernel_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ", "`")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if "traffic_bytes_per_launch" not in fields or "kernel_source_sha256" not in fields:
        return None
    h = kernel_source_hash()
    if h != fields["kernel_source_sha256"]:
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_baseline(w, seconds: float):
    import oracle
    samples, t0, iters = 0, time.perf_counter(), 0
    kw = dict(s=w.s, p=w.p, q=w.q)
    huge = w.dense is not None and w.dense.size > 100_000_000
    while True:
        if huge:
            # the oracle's uniform draws need no data; x is read from the same
            # FP32 array (an FP64 copy of a 6.4 GB tensor per gradient would
            # dominate the timing)
            smp = oracle.sample(w.sampler, w.dims, coo_idx=np.zeros((0, w.d), dtype=np.int64),
                                coo_val=np.zeros(0), seed=w.seed, iteration=iters, **kw)
            smp.xval = w.dense[tuple(smp.idx.T)].astype(np.float64)
        elif w.dense is not None:
            smp = oracle.sample(w.sampler, w.dims, dense=w.dense, seed=w.seed, iteration=iters, **kw)
        else:
            smp = oracle.sample(w.sampler, w.dims, coo_idx=w.coo_idx.astype(np.int64), coo_val=w.coo_val,
                                seed=w.seed, iteration=iters, **kw)
        A64 = [np.float32(a).astype(np.float64) for a in w.A_init] if w.dtype == "f32" else w.A_init
        if w.dtype == "bf16":
            import torch
            A64 = [torch.as_tensor(a).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
                   for a in w.A_init]
        oracle.grad(w.loss, w.dims, A64, smp, nnz=w.nnz, **kw)
        samples += len(smp)
        iters += 1
        el = time.perf_counter() - t0
        if el >= seconds or iters >= 50:
            break
    return {"value": samples / el, "unit": "entries/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} full gradients of {w.name} (oracle sample + grad, FP64, 1 thread), "
                      f"{samples} entries in {el:.1f} s"}


def run_batched(args):
    """64 dense cubes (sides 20..300, ranks 4..32, mixed losses, s = 2%): one
    batched step (gradient + reduction/Adam) per step, against 64 single-problem
    gcp_sampled_adam_step calls; both replayed as HIP graphs."""
    import torch
    import synth
    import paper_1906_01687_amd as gcp
    from paper_1906_01687_amd import _lib, autotune

    ws = synth.batch_of_cubes(64)
    dev = torch.device("cuda:0")

    def problems():
        out = []
        for b, w in enumerate(ws):
            X = gcp.dense_tensor(torch.as_tensor(w.dense).to(dev))
            M = gcp.Factors(w.dims, w.rank, torch.float32, dev, init=w.A_init)
            cfg = gcp.sampling("uniform", s=w.s, seed=w.seed, problem_id=b)
            out.append(gcp.Problem(w.loss, X, M, cfg, lower=w.lower))
        return out

    probs = problems()
    tune, times = autotune.tune_batch(probs, cache_path=os.path.join("/tmp", "gcp_batch_tuning.json"), verbose=True)
    print(f"[bench] autotuned launch shape (threads, unit items, schedule) = {tune}", file=sys.stderr, flush=True)
    batch = gcp.Batch(probs, tune=tune, with_grad=False)
    samples = sum(w.s for w in ws)
    for _ in range(args.warmup):
        batch.adam_step(lr=0.01)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(args.steps):
            batch.adam_step(lr=0.01)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    graph.replay()
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    L = _lib.lib()
    _lib.check(L.gcp_timing_start(args.steps))
    for _ in range(args.steps):
        batch.adam_step(lr=0.01)
    torch.cuda.synchronize()
    kms, kn = ctypes.c_double(), ctypes.c_int64()
    _lib.check(L.gcp_timing_stop(ctypes.byref(kms), ctypes.byref(kn)))
    kernel_ms = kms.value / max(1, kn.value)

    # the same 64 problems as single-problem steps, also one graph
    plain = problems()
    steps = []
    for b, (w, p) in enumerate(zip(ws, plain)):
        adam = gcp.Adam(p.M, lr=0.01, lower=w.lower)
        counter = torch.zeros(1, dtype=torch.int64, device=dev)
        cfg = gcp.sampling("uniform", s=w.s, seed=w.seed, problem_id=b, iteration_counter=counter)
        steps.append((gcp.SampledAdamStep(w.loss, p.X, p.M, cfg, adam), counter))
    for st, _ in steps:
        st()
    torch.cuda.synchronize()
    pgraph = torch.cuda.CUDAGraph()
    plain_steps = max(1, min(args.steps, 20))
    with torch.cuda.graph(pgraph):
        for _ in range(plain_steps):
            for st, _ in steps:
                st()
    torch.cuda.synchronize()
    start.record()
    pgraph.replay()
    stop.record()
    torch.cuda.synchronize()
    plain_ms = start.elapsed_time(stop) / plain_steps

    ms_per_step = total_ms / args.steps
    bpp = {"f32": 4}
    balg = sum(w.s * (3 * w.rank * 4 + 3 * w.rank * 8 + 4) for w in ws)
    achieved = balg / (kernel_ms / 1e3) / 1e9
    print(f"[bench] batched: step {ms_per_step * 1e3:.1f} us (gradient kernel {kernel_ms * 1e3:.1f} us); "
          f"64 single-problem steps: {plain_ms * 1e3:.1f} us", file=sys.stderr, flush=True)
    out = {
        "metric": "sampled gradient entries/sec & HBM GB/s (% peak)",
        "value": samples * args.steps / (total_ms / 1e3),
        "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_64_cubes", "problems": 64, "samples_per_step": samples,
                   "sides": [w.dims[0] for w in ws], "ranks": [w.rank for w in ws],
                   "launch_shape": list(tune), "parallelism": "single_gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "batched_grad_kernel", "kernel_us": kernel_ms * 1e3,
                     "algorithmic_bytes_per_launch": balg},
        "plain_per_problem": {"ms_per_step": plain_ms, "value": samples / (plain_ms / 1e3),
                              "speedup_of_batched": plain_ms / ms_per_step},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: only single-GPU runs are supported (asked for --gpus {args.gpus}); "
              f"the sample stream shards by counter range across GPUs, but that path is not built.",
              file=sys.stderr)
        sys.exit(2)

    if args.study == "variance":
        return run_variance_study(args)
    if args.workload == "batched_64_cubes":
        return run_batched(args)

    import torch
    import synth
    import paper_1906_01687_amd as gcp
    from paper_1906_01687_amd import _lib

    w = synth.WORKLOADS[args.workload]()
    dev = torch.device("cuda:0")
    vdt = torch.float64 if w.dtype == "f64" else torch.float32
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[w.dtype]
    if w.dense is not None:
        X = gcp.dense_tensor(torch.as_tensor(np.ascontiguousarray(w.dense)).to(vdt).to(dev))
    else:
        X = gcp.coo_tensor(w.dims, torch.as_tensor(np.ascontiguousarray(w.coo_idx).view(np.int32)).to(dev),
                           torch.as_tensor(w.coo_val).to(vdt).to(dev))
    M = gcp.Factors(w.dims, w.rank, tdt, dev, init=w.A_init)
    sampler_name = {0: "uniform", 1: "stratified", 2: "semi_stratified"}[w.sampler]
    # the device-side counter advances the sample stream on every step, so a
    # captured graph of one step draws fresh samples on every replay
    counter = torch.zeros(1, dtype=torch.int64, device=dev)
    cfg = gcp.sampling(sampler_name, s=w.s, p=w.p, q=w.q, seed=w.seed, iteration_counter=counter)
    adam = gcp.Adam(M, lr=w.lr, lower=w.lower)
    step_call = gcp.SampledAdamStep(w.loss, X, M, cfg, adam)
    torch.cuda.synchronize()
    print(f"[bench] {w.name}: {w.n_samples} samples/step, nnz={w.nnz}", file=sys.stderr, flush=True)

    for it in range(args.warmup):
        step_call()
    torch.cuda.synchronize()

    L = _lib.lib()
    kms, kn = ctypes.c_double(), ctypes.c_int64()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if args.no_graph:
        _lib.check(L.gcp_timing_start(args.steps))
        torch.cuda.synchronize()
        start.record()
        for it in range(args.steps):
            step_call()
        stop.record()
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(stop)
        _lib.check(L.gcp_timing_stop(ctypes.byref(kms), ctypes.byref(kn)))
    else:
        # the K timed steps as one HIP graph, replayed once in the timed region
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for it in range(args.steps):
                step_call()
        torch.cuda.synchronize()
        start.record()
        graph.replay()
        stop.record()
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(stop)
        # the gradient kernel's own duration: event pairs around it in K eager steps
        _lib.check(L.gcp_timing_start(args.steps))
        for it in range(args.steps):
            step_call()
        torch.cuda.synchronize()
        _lib.check(L.gcp_timing_stop(ctypes.byref(kms), ctypes.byref(kn)))
    kernel_ms = kms.value / max(1, kn.value)
    ms_per_step = total_ms / args.steps
    samples = w.n_samples
    value = samples * args.steps / (total_ms / 1e3)
    balg = algorithmic_bytes(w)
    achieved = balg / (kernel_ms / 1e3) / 1e9
    print(f"[bench] {'eager' if args.no_graph else 'graph'}: step {ms_per_step * 1e3:.1f} us, gradient kernel "
          f"{kernel_ms * 1e3:.1f} us ({kn.value} timed), {achieved:.0f} GB/s algorithmic", file=sys.stderr,
          flush=True)

    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    autograd = None
    if args.autograd:
        autograd = time_autograd(args, w, X, M, sampler_name, ms_per_step)

    traffic = profiled_traffic(w.name)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {
        "metric": "sampled gradient entries/sec & HBM GB/s (% peak)",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16": "bf16"}[w.dtype],
        "data": "synthetic",
        "config": {"workload": w.name, "dims": list(w.dims), "rank": w.rank, "nnz": w.nnz,
                   "loss": ["gaussian", "bernoulli_odds", "poisson", "gamma", "beta_half"][w.loss], "sampler": sampler_name,
                   "samples_per_step": samples, "p": w.p, "q": w.q, "s": w.s, "parallelism": "single_gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "grad_kernel (fused draws + model + derivative + MTTKRP scatter)",
                     "kernel_us": kernel_ms * 1e3, "algorithmic_bytes_per_launch": balg},
        "cpu_baseline": cpu,
    }
    if autograd is not None:
        out["autograd_step"] = autograd
    print(json.dumps(out), flush=True)


def run_variance_study(args):
    """The sampler comparison of Sec. 5.4 at its full size: App. D binary tensor
    400x300x200x100, rank 5, Bernoulli-odds loss.  At the initial guess and at a
    GCP-Adam fit (stratified s = 1000 gradients, 200,000-entry stratified loss
    estimate, alpha = 0.01, tau = 1000, kappa = 1, lower bound 0), N stochastic
    gradients per sampler (uniform s = 1000; stratified and semi-stratified
    p = q = 500) give the empirical bias ||mean - g|| and variance
    (1/N) sum ||g_xi - mean||^2 against the exact gradient g (FULL sampler).
    FP64 factors for the moments; one JSON line."""
    import torch
    import synth
    import paper_1906_01687_amd as gcp
    from paper_1906_01687_amd import variance

    t_gen = time.time()
    w = synth.sparse_binary_400x300x200x100()
    dev = torch.device("cuda:0")
    X = gcp.coo_tensor(w.dims, torch.as_tensor(np.ascontiguousarray(w.coo_idx).view(np.int32)).to(dev),
                       torch.as_tensor(w.coo_val).float().to(dev), bitmap=True)
    torch.cuda.synchronize()
    print(f"[study] data {w.dims}, nnz {w.nnz} ({w.nnz / w.omega * 100:.2f}% dense), "
          f"ready in {time.time() - t_gen:.1f} s", file=sys.stderr, flush=True)

    # the fitted model: GCP-Adam from the initial guess, FP32 factors
    Mfit = gcp.Factors(w.dims, w.rank, torch.float32, dev, init=w.A_init)
    grad = gcp.sampling("stratified", p=500, q=500, seed=w.seed)
    est = gcp.sampling("stratified", p=100000, q=100000, seed=w.seed + 1)
    t0 = time.time()
    fit = gcp.adam_fit(w.loss, X, Mfit, grad, est, lr=0.01, lower=0.0, tau=1000, kappa=1,
                       max_epochs=args.fit_epochs)
    torch.cuda.synchronize()
    fit_s = time.time() - t0
    A_fit = [a.detach().double().cpu().numpy() for a in Mfit.A]
    score_fit = gcp.factor_match_score(w.A_true, A_fit)
    print(f"[study] GCP-Adam: {fit.epochs} epochs in {fit_s:.1f} s, estimate {fit.history[0]:.6e} -> "
          f"{fit.history[-1]:.6e}, score vs truth {score_fit:.3f}", file=sys.stderr, flush=True)

    samplers = [("uniform", gcp.sampling("uniform", s=1000, seed=101)),
                ("stratified", gcp.sampling("stratified", p=500, q=500, seed=102)),
                ("semi_stratified", gcp.sampling("semi_stratified", p=500, q=500, seed=103))]
    table = {}
    for model, A in (("initial", w.A_init), ("fitted", A_fit), ("truth", w.A_true)):
        M = gcp.Factors(w.dims, w.rank, torch.float64, dev, init=A)
        torch.cuda.synchronize()
        t0 = time.time()
        exact = variance.exact_gradient(w.loss, X, M)
        torch.cuda.synchronize()
        t_exact = time.time() - t0
        row = {"grad_norm": float(exact.norm()), "exact_seconds": t_exact}
        for name, cfg in samplers:
            t0 = time.time()
            mo = variance.gradient_moments(w.loss, X, M, cfg, args.draws, exact=exact)
            torch.cuda.synchronize()
            row[name] = {"bias": mo.bias, "variance": mo.variance, "seconds": time.time() - t0}
            print(f"[study] {model:8s} {name:16s} bias {mo.bias:.3e} variance {mo.variance:.3e} "
                  f"(||g|| {row['grad_norm']:.3e})", file=sys.stderr, flush=True)
        table[model] = row
        del M

    out = {"study": "sampler_variance", "workload": "sparse_binary_400x300x200x100", "dims": list(w.dims),
           "rank": w.rank, "nnz": w.nnz, "loss": "bernoulli_odds", "draws": args.draws,
           "samples_per_gradient": 1000, "data": "synthetic (App. D recipe)",
           "fit": {"epochs": fit.epochs, "seconds": fit_s, "estimate_first": fit.history[0],
                   "estimate_last": fit.history[-1], "score_vs_truth": score_fit},
           "table": table}
    print(json.dumps(out), flush=True)


def time_autograd(args, w, X, M, sampler_name, plain_ms):
    """The same step as a torch.autograd graph: F = SampledLoss(param) (gcp_sample +
    gcp_loss_grad), F.backward() (gcp_mttkrp adjoint), then gcp_adam_step on the
    gradient; timed over K eager steps against the plain fused step."""
    import torch
    import paper_1906_01687_amd as gcp

    dev = X.values.device
    counter = torch.zeros(1, dtype=torch.int64, device=dev)
    cfg = gcp.sampling(sampler_name, s=w.s, p=w.p, q=w.q, seed=w.seed, iteration_counter=counter)
    sl = gcp.SampledLoss(w.loss, X, M, cfg)
    param = sl.parameter()
    adam = gcp.Adam(M, lr=w.lr, lower=w.lower)

    def step():
        F = sl(param)
        F.backward()
        adam.step(param.grad.detach())
        param.grad = None

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    print(f"[bench] autograd step (forward + MTTKRP backward + Adam): {ms * 1e3:.1f} us; "
          f"plain fused step {plain_ms * 1e3:.1f} us", file=sys.stderr, flush=True)
    return {"ms_per_step": ms, "value": w.n_samples / (ms / 1e3), "unit": "entries/s",
            "plain_ms_per_step": plain_ms, "plain_over_autograd": ms / plain_ms,
            "launch": "eager (forward, backward and Adam as separate calls)"}


if __name__ == "__main__":
    main()
