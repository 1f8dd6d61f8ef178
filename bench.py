"""Benchmark: sampled GCP gradient + Adam step on one MI355X.

A step is one pass of the whole hot path over one fresh sample set: index
draws, data lookups, model entries, weighted loss derivatives, the MTTKRP
scatter into every mode, and the Adam update, with all inputs resident in HBM.

Default workload: 64 independent dense 3-way problems in one persistent
launch pair (gcp_batched_adam_step) -- cubes with sides log-uniform in
[20, 300], ranks in {4, 8, 16, 32}, Gaussian / Poisson / Bernoulli-odds
losses, 2 % of each cube's entries sampled per step (3.34e6 samples).  The
same 64 problems are also timed as 64 single-problem fused steps (the plain
launch).  `--workload` selects a single-problem workload instead: the sparse
binary 1000x800x600 tensor (stratified sampling), the count tensor
6000x24x77x32 (semi-stratified), the dense 30x40x50 and 200^4 Gaussian
tensors (uniform).

Prints one JSON line.  `value` is sampled entries per second over the timed
steps; `roofline` prices the dominant kernel by its algorithmic bytes against
MI355X's 8 TB/s, with the HBM traffic rocprofv3 measured for it; `issue`
gives the same kernel's VALU and LDS instruction rates against the chip's
issue peaks (from the committed counter summary); `cpu_baseline` times the
FP64 oracle on a bounded sample of the same workload on the host's cores
(one process per core), with the one-thread rate beside it.
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
    ap.add_argument("--workload", default="batched_64_cubes",
                    help="batched_64_cubes | sparse_binary_1000x800x600 | sparse_count_6000x24x77x32 | "
                         "dense_gaussian_30x40x50 | dense_gaussian_200x200x200x200[_bf16]")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="bound on the oracle timing")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes for the CPU baseline (0: the usable cores, at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch every step eagerly")
    ap.add_argument("--launch-shape", default="",
                    help="batched workload: threads,unit_items,schedule,cols_per_lane instead of autotuning")
    ap.add_argument("--cols-per-lane", type=int, default=0,
                    help="rank columns per lane of the gradient kernels (1, 2, 4; 0 = by rank)")
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


_CSRC = "paper_1906_01687_amd/csrc/"
# sources whose code decides what the single-problem gradient kernel executes
KERNEL_SOURCES = [_CSRC + f for f in ("grad_kernels.hpp", "grad_device.hpp", "device.hpp", "kernels.hpp",
                                      "common.hpp", "grad.hip")]
# the same for the batched gradient kernel
BATCH_KERNEL_SOURCES = [_CSRC + f for f in ("batched_kernels.hpp", "batched.hip", "grad_device.hpp", "device.hpp",
                                            "kernels.hpp", "common.hpp")]

# MI355X issue peaks (256 CUs at 2.4 GHz): a wave64 VALU instruction occupies
# one of a CU's four 16-lane SIMDs for 4 cycles; the LDS takes one instruction
# per CU per cycle.  In G wave-instructions per second.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4 / 1e9
LDS_ISSUE_PEAK = 256 * 2.4e9 / 1e9
# LDS FP64 atomic adds: a 64-lane ds_add_f64 with the scatter's address
# pattern occupies a CU's LDS for about 24 cycles (measured on MI355X), so
# 256 CUs add at most 256 * 64 / 24 * 2.4e9 elements per second (G adds/s).
LDS_ATOMIC_PEAK = 256 * 64 / 24 * 2.4e9 / 1e9


def kernel_source_hash(read=None, sources=None) -> str:
    """SHA-256 of a kernel's sources with comments and whitespace removed, so
    that a comment edit does not retire a profile but any code change does.
    ``read(rel)`` returns a source's text (default: the tree)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in (sources or KERNEL_SOURCES):
        if read is None:
            with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
                text = fh.read()
        else:
            text = read(rel)
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update("".join(text.split()).encode())
    return h.hexdigest()


def profiled(name: str, sources):
    """The ``key: value`` figures of profiles/<name>.md (HBM bytes and
    instruction counts per launch from rocprofv3 PMC passes), or None when
    there is no summary or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{name}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ", "`")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_hash(sources=sources):
        return None
    return fields


def issue_rates(fields, kernel_us: float, scatter_adds: float):
    """The kernel against the on-chip resources that bind it: its MTTKRP
    scatter's element adds per second (sum over samples of d r, from the
    workload) against the LDS FP64 atomic rate, and its VALU and LDS
    wave-instruction rates (counts per launch from its profile, over the live
    kernel duration) against the issue peaks."""
    adds = scatter_adds / (kernel_us * 1e-6) / 1e9
    out = {"scatter_adds": {"achieved": adds, "peak": LDS_ATOMIC_PEAK, "frac": adds / LDS_ATOMIC_PEAK,
                            "unit": "G element adds/s", "per_launch": scatter_adds}}
    if fields and "sq_insts_valu_per_launch" in fields:
        valu = float(fields["sq_insts_valu_per_launch"]) / (kernel_us * 1e-6) / 1e9
        lds = float(fields["sq_insts_lds_per_launch"]) / (kernel_us * 1e-6) / 1e9
        out.update({"unit": "G wave-instructions/s",
                    "valu": {"achieved": valu, "peak": VALU_ISSUE_PEAK, "frac": valu / VALU_ISSUE_PEAK},
                    "lds": {"achieved": lds, "peak": LDS_ISSUE_PEAK, "frac": lds / LDS_ISSUE_PEAK},
                    "source": "SQ_INSTS_VALU, SQ_INSTS_LDS per launch (rocprofv3 --pmc, profiles/)"})
    return out


def roofline_of(hbm: dict, issue: dict) -> dict:
    """The kernel's roofline: the algorithmic byte model against HBM while
    that model is a ceiling (fraction at most 1); above 1 it is not one (it
    charges every factor and gradient row to HBM, and these rows stay in L2
    and in the LDS partial), so the roofline is then the tightest on-chip
    ceiling of `issue`, the LDS atomic add rate or VALU issue, and the byte
    model is kept beside it."""
    if hbm["frac"] <= 1.0:
        return hbm
    cands = [("scatter_adds", "LDS FP64 atomic adds of the MTTKRP scatter")]
    if "valu" in issue:
        cands.append(("valu", "VALU wave-instruction issue"))
    key, what = max(cands, key=lambda c: issue[c[0]]["frac"])
    e = issue[key]
    out = {"bound": "alu", "resource": what, "achieved": e["achieved"], "peak": e["peak"],
           "unit": e.get("unit", issue.get("unit")), "frac": e["frac"]}
    out.update({k: hbm[k] for k in ("traffic", "traffic_unit", "kernel", "kernel_us")})
    out["hbm_byte_model"] = {k: hbm[k] for k in ("achieved", "peak", "unit", "frac", "algorithmic_bytes_per_launch")}
    return out


def usable_cores(limit: int = 16) -> int:
    """Host cores this process may run on, capped at the GPU machine's share."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, limit))


def copy_calibration(mib: int, dev) -> None:
    """One device-to-device copy of `mib` MiB: the known byte count against
    which a profiler's FETCH_SIZE and WRITE_SIZE are calibrated."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


# Workloads the oracle workers read; set before the worker processes are forked
# (copy-on-write, nothing is pickled) and before this process touches the GPU.
_CPU_WORKLOADS: list = []


def _oracle_gradient(w, iteration: int) -> int:
    """One full sampled gradient of workload w by the FP64 oracle (sample +
    grad), on the factor values the device stores; returns its sample count."""
    import oracle
    kw = dict(s=w.s, p=w.p, q=w.q)
    if w.dense is not None and w.sampler == 0:
        # uniform draws need no data; x is read from the same FP32 array the
        # device holds (an FP64 copy of a large cube per gradient would
        # dominate the timing)
        smp = oracle.sample(w.sampler, w.dims, coo_idx=np.zeros((0, w.d), dtype=np.int64), coo_val=np.zeros(0),
                            seed=w.seed, problem_id=getattr(w, "problem_id", 0), iteration=iteration, **kw)
        smp.xval = np.asarray(w.dense)[tuple(smp.idx.T)].astype(np.float64)
    elif w.dense is not None:
        smp = oracle.sample(w.sampler, w.dims, dense=w.dense, seed=w.seed, iteration=iteration, **kw)
    else:
        smp = oracle.sample(w.sampler, w.dims, coo_idx=w.coo_idx.astype(np.int64), coo_val=w.coo_val,
                            seed=w.seed, iteration=iteration, **kw)
    if w.dtype == "bf16":
        import torch
        A64 = [torch.as_tensor(a).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy() for a in w.A_init]
    elif w.dtype == "f32":
        A64 = [np.float32(a).astype(np.float64) for a in w.A_init]
    else:
        A64 = w.A_init
    oracle.grad(w.loss, w.dims, A64, smp, nnz=w.nnz, **kw)
    return len(smp)


def _oracle_worker(task):
    """Worker `wi` of `nw`: full oracle gradients for `seconds`; with several
    workloads it walks them in turn from its own offset, every gradient on a
    fresh iteration of the sample stream."""
    wi, nw, seconds = task
    ws = _CPU_WORKLOADS
    t0, n, k = time.perf_counter(), 0, 0
    while True:
        j = wi + k * nw
        w = ws[j % len(ws)]
        n += _oracle_gradient(w, j // len(ws))
        k += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return n, el, k


def cpu_baseline(workloads, name: str, seconds: float, workers: int = 0):
    """The FP64 oracle on the host: one process per usable core (fork, before
    the GPU is touched), each computing whole gradients of the workload(s) for
    about `seconds`, plus the same on one thread.  entries/s = samples over
    the slowest worker's wall time."""
    import multiprocessing as mp
    global _CPU_WORKLOADS
    _CPU_WORKLOADS = list(workloads)
    nw = workers if workers > 0 else usable_cores()
    per_worker = max(1.5, seconds / nw)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(processes=nw) as pool:
        res = pool.map(_oracle_worker, [(i, nw, per_worker) for i in range(nw)])
    wall = time.perf_counter() - t0
    samples = sum(r[0] for r in res)
    grads = sum(r[2] for r in res)
    slowest = max(r[1] for r in res)
    one = _oracle_worker((0, 1, min(seconds, 6.0)))
    return {"value": samples / slowest, "unit": "entries/s", "cores": nw, "kind": "oracle",
            "single_thread_value": one[0] / one[1],
            "sample": f"{grads} full gradients of {name} (oracle sample + grad, FP64) by {nw} processes, "
                      f"{samples} entries in {slowest:.1f} s per process ({wall:.1f} s wall); one thread: "
                      f"{one[2]} gradients, {one[0]} entries in {one[1]:.1f} s"}


def run_batched(args, ws, cpu):
    """64 dense cubes (sides 20..300, ranks 4..32, mixed losses, s = 2%): one
    batched step (gradient + reduction/Adam) per step, against 64 single-problem
    gcp_sampled_adam_step calls; both replayed as HIP graphs."""
    import torch
    import paper_1906_01687_amd as gcp
    from paper_1906_01687_amd import _lib, autotune

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
    if args.launch_shape:
        tune = tuple(int(v) for v in args.launch_shape.split(","))
        print(f"[bench] launch shape (threads, unit items, schedule, cols per lane) = {tune}", file=sys.stderr,
              flush=True)
    else:
        tune, times = autotune.tune_batch(probs, cache_path=os.path.join("/tmp", "gcp_batch_tuning.json"))
        print(f"[bench] autotuned launch shape (threads, unit items, schedule, cols per lane) = {tune} "
              f"of {len(times)} candidates", file=sys.stderr, flush=True)
    batch = gcp.Batch(probs, tune=tune, with_grad=False)
    samples = sum(w.s for w in ws)
    for _ in range(args.warmup):
        batch.adam_step(lr=0.01)
    # the K timed steps as one graph the library owns (gcp_batched_graph_capture)
    batch.capture_adam_steps(args.steps, lr=0.01)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    batch.graph_launch()
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

    if args.copy_mib > 0:
        copy_calibration(args.copy_mib, dev)

    ms_per_step = total_ms / args.steps
    # algorithmic bytes per sample of a dense FP32 problem (d = 3): three
    # factor rows (4 r each), three gradient rows read and written (8 r each),
    # and the 4-byte data value
    balg = sum(w.s * (3 * w.rank * 4 + 3 * w.rank * 8 + 4) for w in ws)
    achieved = balg / (kernel_ms / 1e3) / 1e9
    prof = profiled("batched_grad_kernel_batched_64_cubes", BATCH_KERNEL_SOURCES)
    traffic = int(prof["traffic_bytes_per_launch"]) if prof and "traffic_bytes_per_launch" in prof else None
    print(f"[bench] batched: step {ms_per_step * 1e3:.1f} us (gradient kernel {kernel_ms * 1e3:.1f} us); "
          f"64 single-problem steps: {plain_ms * 1e3:.1f} us", file=sys.stderr, flush=True)
    issue = issue_rates(prof, kernel_ms * 1e3, sum(w.s * 3 * w.rank for w in ws))
    out = {
        "metric": "sampled gradient entries/sec & HBM GB/s (% peak); batched vs plain at 1e-5 rel",
        "value": samples * args.steps / (total_ms / 1e3),
        "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_64_cubes", "problems": 64, "samples_per_step": samples,
                   "sides": [w.dims[0] for w in ws], "ranks": [w.rank for w in ws],
                   "losses": [["gaussian", "bernoulli_odds", "poisson"][w.loss] for w in ws],
                   "launch_shape": {"threads": tune[0], "unit_items": tune[1], "schedule": tune[2],
                                    "cols_per_lane": tune[3] if len(tune) > 3 else 0},
                   "parallelism": "single_gpu"},
        "roofline": roofline_of(
            {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
             "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
             "kernel": "batched_grad_kernel (64 problems: draws + model + derivative + MTTKRP scatter)",
             "kernel_us": kernel_ms * 1e3, "algorithmic_bytes_per_launch": balg}, issue),
        "issue": issue,
        "batched_launch": "2 kernels per step (gradient, reduction + Adam); K steps replayed as one "
                          "library-owned HIP graph (gcp_batched_graph_capture / _launch)",
        "plain_per_problem": {"ms_per_step": plain_ms, "value": samples / (plain_ms / 1e3),
                              "speedup_of_batched": plain_ms / ms_per_step,
                              "launch": "64 gcp_sampled_adam_step calls per step, one HIP graph"},
        "cpu_baseline": cpu,
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

    # host-side inputs and the oracle baseline first: the oracle's worker
    # processes are forked before this process touches the GPU
    import synth
    if args.workload == "batched_64_cubes":
        ws = synth.batch_of_cubes(64)
        cpu = None if args.no_cpu_baseline else cpu_baseline(ws, "the 64-cube batch", args.cpu_seconds,
                                                             args.cpu_workers)
        if cpu:
            print(f"[bench] oracle: {cpu['value']:.3g} entries/s on {cpu['cores']} processes, "
                  f"{cpu['single_thread_value']:.3g} on one", file=sys.stderr, flush=True)
        if args.cols_per_lane:
            import paper_1906_01687_amd as gcp
            gcp.set_cols_per_lane(args.cols_per_lane)
        return run_batched(args, ws, cpu)
    w = synth.WORKLOADS[args.workload]()
    cpu = None if args.no_cpu_baseline else cpu_baseline([w], w.name, args.cpu_seconds, args.cpu_workers)

    import torch
    import paper_1906_01687_amd as gcp
    from paper_1906_01687_amd import _lib

    if args.cols_per_lane:
        gcp.set_cols_per_lane(args.cols_per_lane)
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
        # the gradient kernel's own duration: event pairs around it in K eager
        # steps, after K untimed eager steps (the first eager block of a
        # process issues slower, and its events then read about 1.5 us more
        # per launch than every later block)
        for it in range(args.steps):
            step_call()
        torch.cuda.synchronize()
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
        copy_calibration(args.copy_mib, dev)

    autograd = None
    if args.autograd:
        autograd = time_autograd(args, w, X, M, sampler_name, ms_per_step)

    prof = profiled(f"grad_kernel_{w.name}", KERNEL_SOURCES)
    traffic = int(prof["traffic_bytes_per_launch"]) if prof and "traffic_bytes_per_launch" in prof else None
    issue = issue_rates(prof, kernel_ms * 1e3, float(samples) * w.d * w.rank)

    out = {
        "metric": "sampled gradient entries/sec & HBM GB/s (% peak); batched vs plain at 1e-5 rel",
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
        "roofline": roofline_of(
            {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
             "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
             "kernel": "grad_kernel (fused draws + model + derivative + MTTKRP scatter)",
             "kernel_us": kernel_ms * 1e3, "algorithmic_bytes_per_launch": balg}, issue),
        "issue": issue,
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
