"""Launch-shape autotuner for batches (gcp_batched_*).

The tunables are the gradient workgroup size (256, 512 or 1024 threads), the
schedule (one contiguous run of items per workgroup, or longest-processing-
time dealing of units), for the latter the work-unit size (64-sample items
per unit: small units balance load across workgroups, large ones let a
workgroup hold more of one problem, so fewer LDS partials are flushed), and
the rank-chunk shape: how many rank columns each lane of a sample's lane
group carries (1, 2 or 4, or by rank).  Each candidate is planned and prepared as a separate batch whose
problems publish no gradient and take no Adam step, timed over a few
gradient-only steps with the library's dispatch-stamped kernel events, and the
fastest is kept.  Results are cached in a JSON file keyed by the batch's shape
signature (dims, ranks, losses, samplers, sample counts, dtypes, device).
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
import sys
from typing import Dict, Iterable, Optional, Sequence, Tuple

import torch

from . import _lib
from .api import Batch, Problem

DEFAULT_CANDIDATES: Tuple[Tuple[int, int, int, int], ...] = tuple(
    [(t, 0, _lib.BATCH_CONTIGUOUS, c) for t in (512, 1024) for c in (0, 1, 2, 4)]
    + [(t, u, _lib.BATCH_LPT, c) for t in (256, 512, 1024) for u in (16, 64, 256) for c in (0, 1, 2, 4)]
    + [(1024, u, _lib.BATCH_LPT, c) for u in (32, 128) for c in (0, 1, 2, 4)])
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gcp_mi355x", "batch_tuning.json")


def signature(problems: Sequence[Problem]) -> str:
    h = hashlib.sha256(b"candidates with cols_per_lane")
    dev = problems[0].M.flat.device
    h.update(torch.cuda.get_device_properties(dev).gcnArchName.encode())
    for p in problems:
        c = p.cfg
        h.update(repr((p.X.dims, p.M.rank, str(p.M.dtype), str(p.X.values.dtype), p.X.is_dense, p.loss,
                       c.sampler, c.s, c.p, c.q)).encode())
    return h.hexdigest()[:32]


def _time_candidate(problems: Sequence[Problem], tune, steps: int, warmup: int) -> float:
    L = _lib.lib()
    batch = Batch(problems, tune=tune, with_grad=False)
    try:
        for _ in range(warmup):
            batch.grad()
        torch.cuda.synchronize()
        _lib.check(L.gcp_timing_start(steps))
        for _ in range(steps):
            batch.grad()
        torch.cuda.synchronize()
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _lib.check(L.gcp_timing_stop(ctypes.byref(ms), ctypes.byref(n)))
        return ms.value / max(1, n.value)
    finally:
        batch.close()


def tune_batch(problems: Sequence[Problem], candidates: Optional[Iterable[Tuple[int, ...]]] = None,
               steps: int = 10, warmup: int = 2, cache_path: Optional[str] = DEFAULT_CACHE,
               verbose: bool = False, finalists: int = 4) -> Tuple[Tuple[int, ...], Dict[str, float]]:
    """Best (threads, unit_items, schedule, cols_per_lane) for this batch and the timings (ms)
    of all candidates; a cached answer for the same signature is returned
    untimed.  The `finalists` fastest candidates of the first round are timed
    again over three times as many steps and the best of that round is kept:
    shapes within a few percent of each other are otherwise told apart by a
    few launches (their timings then are those of the second round)."""
    sig = signature(problems)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if sig in cache:
        entry = cache[sig]
        return tuple(entry["best"]), entry.get("times", {})
    times: Dict[str, float] = {}
    best, best_ms = None, float("inf")
    cands = [tuple(t) for t in (candidates or DEFAULT_CANDIDATES)]
    for tune in cands:
        ms = _time_candidate(problems, tune, steps, warmup)
        times["x".join(str(v) for v in tune)] = ms
        if verbose:
            print(f"[autotune] threads={tune[0]} unit_items={tune[1]} schedule={tune[2] if len(tune) > 2 else 0} "
                  f"cols_per_lane={tune[3] if len(tune) > 3 else 0}: "
                  f"{ms * 1e3:.1f} us", file=sys.stderr, flush=True)
        if ms < best_ms:
            best, best_ms = tuple(tune), ms
    keys = {"x".join(str(v) for v in t): t for t in cands}
    ranked = sorted(times, key=times.get)[:max(1, finalists)]
    if len(ranked) > 1:
        best, best_ms = None, float("inf")
        for key in ranked:
            ms = _time_candidate(problems, keys[key], 3 * steps, warmup)
            times[key] = ms
            if verbose:
                print(f"[autotune] finalist {key}: {ms * 1e3:.1f} us", file=sys.stderr, flush=True)
            if ms < best_ms:
                best, best_ms = keys[key], ms
    if cache_path:
        cache[sig] = {"best": list(best), "times": times}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + f".tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return best, times
