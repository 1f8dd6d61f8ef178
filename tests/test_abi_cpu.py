"""Host-only checks of the C-ABI library: it loads, exports every function that
include/gcp.h declares, and its host-side queries and argument checks behave
(no kernel is launched without a GPU)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gcp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gcp_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_1906_01687_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgcp.so not built")
    return _lib


def test_every_declared_symbol_is_exported():
    m = _lib()
    raw = ctypes.CDLL(m.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    assert sorted(m.EXPORTS) == names


def test_struct_layouts_match_header():
    m = _lib()
    assert ctypes.sizeof(m.GcpTensor) == 144
    assert ctypes.sizeof(m.GcpFactors) == 80
    assert ctypes.sizeof(m.GcpSampling) == 72
    assert ctypes.sizeof(m.GcpFitOptions) == 208


def test_host_queries():
    m = _lib()
    L = m.lib()
    assert L.gcp_abi_version() == 1
    assert L.gcp_nz_table_slots(0) == 64
    assert L.gcp_nz_table_slots(959756) == 1 << 21
    s = L.gcp_nz_table_slots(5_000_000)
    assert s >= 10_000_000 and s & (s - 1) == 0
    assert L.gcp_nz_table_bytes(1 << 21) == 12 << 21
    t = m.GcpTensor()
    t.d, t.format = 3, m.COO
    for k, n in enumerate((1000, 800, 600)):
        t.dims[k] = n
    assert L.gcp_nz_bitmap_bytes(ctypes.byref(t)) == 480_000_000 // 8
    t.dims[2] = 601                                  # 480.8e6 bits -> whole 64-bit words
    assert L.gcp_nz_bitmap_bytes(ctypes.byref(t)) == -(-480_800_000 // 64) * 8
    t.format = m.DENSE
    assert L.gcp_nz_bitmap_bytes(ctypes.byref(t)) == 0


def _dense_struct(m, dims, values=0x1000):
    t = m.GcpTensor()
    t.d = len(dims)
    t.format = m.DENSE
    t.vdtype = m.F32
    for k, n in enumerate(dims):
        t.dims[k] = n
    t.values = values
    return t


def test_argument_errors_are_reported_without_launching():
    m = _lib()
    L = m.lib()
    t = _dense_struct(m, (30, 40, 50))
    cfg = m.GcpSampling()
    cfg.sampler = m.STRATIFIED          # needs a COO tensor
    cfg.p, cfg.q = 10, 10
    st = L.gcp_sample(ctypes.byref(t), ctypes.byref(cfg), 0x10, 0x10, 0x10, None, 0, None)
    assert st == 1 and b"COO" in L.gcp_last_error()
    # FULL on a COO tensor looks every entry up in the nonzero table, so the
    # table is required even when the tensor stores no entries
    t.format = m.COO
    t.nnz = 0
    cfg.sampler = m.FULL
    st = L.gcp_sample(ctypes.byref(t), ctypes.byref(cfg), 0x10, 0x10, 0x10, None, 0, None)
    assert st == 1 and b"nz_table" in L.gcp_last_error()
    t.format = m.DENSE
    t.d = 9
    cfg.sampler = m.UNIFORM
    cfg.s = 5
    assert L.gcp_sample(ctypes.byref(t), ctypes.byref(cfg), 0x10, 0x10, 0x10, None, 0, None) == 1
    t = _dense_struct(m, (1 << 32, 2))
    assert L.gcp_sample(ctypes.byref(t), ctypes.byref(cfg), 0x10, 0x10, 0x10, None, 0, None) == 1
    t = _dense_struct(m, (1 << 31, 1 << 31, 4))
    assert L.gcp_sample(ctypes.byref(t), ctypes.byref(cfg), 0x10, 0x10, 0x10, None, 0, None) == 2
    # rank above the supported maximum
    t = _dense_struct(m, (3, 4))
    M = m.GcpFactors()
    M.dtype = m.F32
    M.rank = 257
    M.A[0] = M.A[1] = 0x1000
    G = (ctypes.c_void_p * 2)(0x1000, 0x1000)
    st = L.gcp_sampled_grad(0, ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg), 1e-10, G, None,
                            0x1000, 1 << 20, None)
    assert st == 2
    # a factor block beyond 4 GiB: 2^25 rows x 64 columns x 4 bytes = 8 GiB
    t = _dense_struct(m, (1 << 25, 4))
    M.rank = 64
    st = L.gcp_sampled_grad(0, ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg), 1e-10, G, None,
                            0x1000, 1 << 20, None)
    assert st == 2 and b"4 GiB" in L.gcp_last_error()
    M.dtype = m.BF16                     # 2 bytes per value: exactly 4 GiB is still too large
    st = L.gcp_sampled_grad(0, ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg), 1e-10, G, None,
                            0x1000, 1 << 20, None)
    assert st == 2 and b"4 GiB" in L.gcp_last_error()
    t = _dense_struct(m, ((1 << 25) - 1, 4))   # 4 GiB - 128 bytes passes the size check
    st = L.gcp_sampled_grad(0, ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg), 1e-10, G, None,
                            0x1000, 1 << 20, None)
    assert b"4 GiB" not in L.gcp_last_error()
    M.dtype = m.F32
    t = _dense_struct(m, (3, 4))
    # workspace too small
    M.rank = 4
    need = L.gcp_sampled_grad_workspace_bytes(ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg))
    assert need >= (3 + 4) * 4 * 8
    st = L.gcp_sampled_grad(0, ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg), 1e-10, G, None,
                            0x1000, need - 1, None)
    assert st == 4 and b"workspace" in L.gcp_last_error()
    # Adam argument checks
    st = L.gcp_adam_step(10, m.BF16, 0x10, None, 0x10, 0x10, 0x10, 0x10, 0.01, 0.9, 0.999, 1e-8,
                         -math.inf, 0, None)
    assert st == 1 and b"master" in L.gcp_last_error()
    st = L.gcp_adam_step(10, m.F32, 0x10, None, 0x10, 0x10, 0x10, 0x10, 0.01, 1.0, 0.999, 1e-8,
                         -math.inf, 0, None)
    assert st == 1


def test_stratified_workspace_covers_rejection_scratch():
    m = _lib()
    L = m.lib()
    t = m.GcpTensor()
    t.d, t.format, t.vdtype = 3, m.COO, m.F32
    for k, n in enumerate((1000, 800, 600)):
        t.dims[k] = n
    t.nnz = 959756
    cfg = m.GcpSampling()
    cfg.sampler, cfg.p, cfg.q = m.STRATIFIED, 100_000, 100_000
    ws = L.gcp_sample_workspace_bytes(ctypes.byref(t), ctypes.byref(cfg))
    nchunks = math.ceil(math.ceil(1.1 * 1e5 * 4.8e8 / (4.8e8 - 959756)) / 64)
    assert ws >= nchunks * 12
    M = m.GcpFactors()
    M.dtype, M.rank = m.F32, 8
    ws2 = L.gcp_sampled_grad_workspace_bytes(ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg))
    # every mode fits in LDS: one FP32 partial of 2400 x 8 per gradient workgroup
    assert ws2 >= ws + 2400 * 8 * 4


def test_sampled_adam_step_needs_factor_blocks_of_the_flat_array():
    """The fused step updates the flat array A, so M->A[k] must be its blocks."""
    m = _lib()
    L = m.lib()
    t = _dense_struct(m, (30, 40, 50))
    cfg = m.GcpSampling()
    cfg.sampler, cfg.s = m.UNIFORM, 100
    M = m.GcpFactors()
    M.dtype, M.rank = m.F32, 4
    base = 0x10000
    off = 0
    for k, n in enumerate((30, 40, 50)):
        M.A[k] = base + 4 * off
        off += n * 4
    def call(A):
        return L.gcp_sampled_adam_step(0, ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg), 1e-10,
                                       A, None, 0x40000, 0x50000, 0x60000,          # A, A_master, B, C, state
                                       0.01, 0.9, 0.999, 1e-8, -math.inf, 0,        # Adam parameters
                                       None, None, 0x70000, 0, None)                # G, loss_sum, ws
    assert call(0x90000) == 1 and b"flat parameter array" in L.gcp_last_error()
    # the right array passes the check and only then meets the (too small) workspace
    assert call(base) == 4 and b"workspace" in L.gcp_last_error()


def _problem_struct(m, dims, rank, s, base):
    """A dense FP32 uniform problem with fake (never dereferenced) device pointers."""
    pr = m.GcpProblem()
    pr.X = _dense_struct(m, dims, values=base)
    pr.M.dtype, pr.M.rank = m.F32, rank
    off = 0
    for k, n in enumerate(dims):
        pr.M.A[k] = base + 0x100000 + 4 * off
        off += n * rank
    pr.cfg.sampler, pr.cfg.s = m.UNIFORM, s
    pr.loss, pr.eps, pr.lower = 0, 1e-10, -math.inf
    pr.A, pr.B, pr.C = base + 0x100000, base + 0x200000, base + 0x300000
    return pr


def _plan(m, L, probs, tune):
    arr = (m.GcpProblem * len(probs))(*probs)
    h = ctypes.c_void_p()
    st = L.gcp_batched_create(arr, len(probs), ctypes.byref(tune), ctypes.byref(h))
    assert st == 0, L.gcp_last_error()
    try:
        assert L.gcp_batched_workspace_bytes(h) > 0
        nb, nu = ctypes.c_int64(), ctypes.c_int64()
        assert L.gcp_batched_plan(h, ctypes.byref(nb), ctypes.byref(nu), None, None, None) == 0
        import numpy as np
        bp = np.zeros(nb.value + 1, np.int64)
        up = np.zeros(nu.value, np.int32)
        ui = np.zeros((nu.value, 2), np.int64)
        assert L.gcp_batched_plan(h, None, None, bp.ctypes.data, up.ctypes.data, ui.ctypes.data) == 0
        return bp, up, ui
    finally:
        L.gcp_batched_destroy(h)


@pytest.mark.parametrize("schedule,unit_items", [(0, 0), (1, 1), (1, 7), (1, 64)])
def test_batch_plan_covers_every_item_once(schedule, unit_items):
    """Host planning of a batch: every 64-sample item of every problem lies in
    exactly one unit, each workgroup walks its units in problem order, and the
    contiguous schedule gives every workgroup about the same estimated cost."""
    m = _lib()
    L = m.lib()
    import numpy as np
    rng = np.random.default_rng(3)
    specs = [(int(n), int(r), int(s)) for n, r, s in zip(rng.integers(5, 120, 23), rng.choice([1, 4, 9, 32], 23),
                                                          rng.integers(0, 60_000, 23))]
    specs[5] = (40, 8, 0)                                    # a problem with no samples
    probs = [_problem_struct(m, (n, n + 1, n + 2), r, s, 0x10000000 * (b + 1)) for b, (n, r, s) in enumerate(specs)]
    tune = m.GcpBatchTuning()
    tune.threads, tune.unit_items, tune.schedule = 1024, unit_items, schedule
    bp, up, ui = _plan(m, L, probs, tune)
    nblocks = len(bp) - 1
    assert bp[0] == 0 and bp[-1] == len(up) and np.all(np.diff(bp) >= 0)
    items = [-(-s // 64) for _, _, s in specs]

    def item_cost(r):
        # the planner's estimate per sample (d = 3): a fixed part of 19 and d r
        return 19 + 3 * r
    seen = [np.zeros(n, np.int32) for n in items]
    cost = np.zeros(nblocks)
    for w in range(nblocks):
        units = range(bp[w], bp[w + 1])
        probs_w = [up[u] for u in units]
        assert probs_w == sorted(probs_w)                    # problem order inside a workgroup
        for u in units:
            b, (i0, i1) = up[u], ui[u]
            assert 0 <= i0 < i1 <= items[b]
            seen[b][i0:i1] += 1
            cost[w] += (i1 - i0) * item_cost(specs[b][1])
    for b in range(len(specs)):
        assert np.all(seen[b] == 1), b
    if schedule == 0:
        # a workgroup's cost exceeds the even share by at most one item of the costliest problem
        share = cost.sum() / nblocks
        assert cost.max() <= share + item_cost(32) + 1e-9
        # contiguous runs: (workgroup, problem) pairs are at most workgroups + problems
        pairs = len({(w, up[u]) for w in range(nblocks) for u in range(bp[w], bp[w + 1])})
        assert pairs <= nblocks + len(specs)
    bad = m.GcpBatchTuning()
    bad.schedule = 7
    arr = (m.GcpProblem * 1)(probs[0])
    h = ctypes.c_void_p()
    assert L.gcp_batched_create(arr, 1, ctypes.byref(bad), ctypes.byref(h)) == 1
    assert b"schedule" in L.gcp_last_error()


def test_fit_options_are_checked():
    """gcp_adam_fit validates its options on the host (no launch)."""
    m = _lib()
    L = m.lib()
    t = _dense_struct(m, (30, 40, 50))
    M = m.GcpFactors()
    M.dtype, M.rank = m.F32, 4
    for k in range(3):
        M.A[k] = 0x10000
    o = m.GcpFitOptions()
    o.grad.sampler, o.grad.s = m.UNIFORM, 100
    o.est.sampler, o.est.s = m.UNIFORM, 1000
    o.alpha, o.beta1, o.beta2, o.adam_eps, o.nu = 0.01, 0.9, 0.999, 1e-8, 0.1
    o.tau, o.kappa, o.max_epochs = 10, 1, 5
    assert L.gcp_adam_fit_workspace_bytes(ctypes.byref(t), ctypes.byref(M), ctypes.byref(o)) > 0
    o.tau = 0
    assert L.gcp_adam_fit_workspace_bytes(ctypes.byref(t), ctypes.byref(M), ctypes.byref(o)) == 0
    assert b"tau" in L.gcp_last_error()
    o.tau, o.nu = 10, 0.0
    hist = (ctypes.c_double * 6)()
    acc = (ctypes.c_int8 * 6)()
    ep = ctypes.c_int32()
    st = L.gcp_adam_fit(0, ctypes.byref(t), ctypes.byref(M), ctypes.byref(o), 1e-10, 0x10000, None, 0x20000,
                        0x30000, 0x40000, hist, acc, ctypes.byref(ep), None, 0x50000, 1 << 30, None)
    assert st == 1 and b"nu" in L.gcp_last_error()


def test_factor_match_score():
    """App. E score: 1 for the same model up to component order, column scaling
    and sign flips in pairs of modes; low for unrelated factors; the best
    matching is found, not a greedy one."""
    import numpy as np
    from paper_1906_01687_amd.score import factor_match_score
    rng = np.random.default_rng(21)
    A = [rng.standard_normal((n, 4)) for n in (9, 8, 7)]
    perm = np.array([3, 1, 0, 2])
    scale = [np.array([2.0, 0.5, 3.0, 1.0]), np.array([1.0, 4.0, 0.25, 1.0]), np.array([0.5, 0.5, 1.0, 1.0])]
    B = [a[:, perm] * s for a, s in zip(A, scale)]
    B[1][:, 2] *= -1
    B[2][:, 2] *= -1
    assert abs(factor_match_score(A, B) - 1.0) < 1e-12
    assert factor_match_score(A, [rng.standard_normal(a.shape) for a in A]) < 0.3
    # one mode, similarities [[0.6, 0.5], [0.5, 0.1]]: a greedy pick takes 0.6
    # then 0.1 (mean 0.35); the best matching pairs the 0.5s (mean 0.5)
    e = np.eye(3)
    ref = [np.stack([e[0], e[1]], axis=1)]
    est = [np.stack([0.6 * e[0] + 0.5 * e[1] + np.sqrt(1 - 0.61) * e[2],
                     0.5 * e[0] + 0.1 * e[1] + np.sqrt(1 - 0.26) * e[2]], axis=1)]
    assert abs(factor_match_score(ref, est) - 0.5) < 1e-12


def test_profile_hash_ignores_comments_only():
    """bench.py keeps a committed traffic figure across comment edits of the
    gradient kernel sources and retires it on any code change."""
    import bench
    base = {rel: open(os.path.join(bench.ROOT, rel), encoding="utf-8").read() for rel in bench.KERNEL_SOURCES}
    h0 = bench.kernel_source_hash(lambda rel: base[rel])
    assert h0 == bench.kernel_source_hash()
    first = bench.KERNEL_SOURCES[0]
    commented = dict(base)
    commented[first] = "// a new comment\n/* and a block\n   comment */\n" + base[first].replace("\n", "\n  ", 3)
    assert bench.kernel_source_hash(lambda rel: commented[rel]) == h0
    changed = dict(base)
    changed[first] = base[first] + "\nstatic int gcp_unused_probe = 1;\n"
    assert bench.kernel_source_hash(lambda rel: changed[rel]) != h0


def test_roofline_is_a_ceiling():
    """bench.py's roofline is the byte model against HBM while its fraction is
    at most 1, else the tightest on-chip ceiling (LDS atomic adds or VALU
    issue), with the byte model kept beside it; no roofline fraction exceeds 1."""
    import bench
    fields = {"sq_insts_valu_per_launch": "6.0e7", "sq_insts_lds_per_launch": "3.0e6"}
    issue = bench.issue_rates(fields, 200.0, 1.3e8)
    hbm = {"bound": "hbm", "achieved": 8200.0, "peak": bench.HBM_PEAK_GBS, "unit": "GB/s", "frac": 8200.0 / 8000.0,
           "traffic": 4.9e8, "traffic_unit": "bytes", "kernel": "k", "kernel_us": 200.0,
           "algorithmic_bytes_per_launch": 1.6e9}
    r = bench.roofline_of(hbm, issue)
    assert r["bound"] == "alu" and r["frac"] <= 1.0
    assert r["frac"] == max(issue["scatter_adds"]["frac"], issue["valu"]["frac"])
    assert r["hbm_byte_model"]["frac"] == hbm["frac"] and r["traffic"] == hbm["traffic"]
    low = dict(hbm, achieved=3000.0, frac=3000.0 / 8000.0)
    assert bench.roofline_of(low, issue) is low
    only_adds = bench.issue_rates(None, 200.0, 1.3e8)
    assert bench.roofline_of(hbm, only_adds)["frac"] == only_adds["scatter_adds"]["frac"]


def test_rejection_cap_refused_on_the_host():
    """Stratified rejection whose first batch plus the device refill cap
    (2^22 candidates) cannot cover q omega / zeta plus eight standard
    deviations of the candidate count (Sec. 4.2, App. B) is refused before any
    launch; a larger rho makes the same request acceptable."""
    m = _lib()
    L = m.lib()
    t = m.GcpTensor()
    t.d, t.format, t.vdtype = 2, m.COO, m.F32
    t.dims[0], t.dims[1] = 1 << 20, 1 << 10      # omega = 2^30
    t.nnz = (1 << 30) - (1 << 12)                 # zeta = 2^12 = 2^-18 omega
    t.coo_idx, t.values = 0x1000, 0x1000
    t.nz_bitmap = 0x1000
    cfg = m.GcpSampling()
    cfg.sampler = m.STRATIFIED
    cfg.p, cfg.q = 0, 1000
    cfg.rho = 0.5                                 # first batch: half the mean of 2.6e8 candidates
    st = L.gcp_sample(ctypes.byref(t), ctypes.byref(cfg), 0x10, 0x10, 0x10, None, 0, None)
    assert st == 2 and b"refill cap" in L.gcp_last_error()
    # expected candidates q omega / zeta = 2.6e8, standard deviation 8.3e6:
    # rho = 1.3 covers the mean plus eight deviations
    cfg.rho = 1.3
    assert L.gcp_sample_workspace_bytes(ctypes.byref(t), ctypes.byref(cfg)) > 0
    # the host check passes; only the missing workspace is reported
    st = L.gcp_sample(ctypes.byref(t), ctypes.byref(cfg), 0x10, 0x10, 0x10, None, 0, None)
    assert st == 4 and b"workspace" in L.gcp_last_error(), L.gcp_last_error()
    # the status word lies inside the workspace, for the materialising and the fused call
    off = L.gcp_rejection_status_offset(ctypes.byref(t), None, ctypes.byref(cfg))
    assert 0 <= off < L.gcp_sample_workspace_bytes(ctypes.byref(t), ctypes.byref(cfg))
    M = m.GcpFactors()
    M.dtype, M.rank = m.F32, 4
    offf = L.gcp_rejection_status_offset(ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg))
    assert 0 <= offf < L.gcp_sampled_grad_workspace_bytes(ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg))
    cfg.sampler = m.SEMI_STRATIFIED
    assert L.gcp_rejection_status_offset(ctypes.byref(t), None, ctypes.byref(cfg)) == -1


def test_noalloc_refuses_problems_beyond_its_scratch():
    """gcp_sampled_grad_noalloc refuses, before any launch, a problem whose
    workspace exceeds its static scratch (64 MiB)."""
    m = _lib()
    L = m.lib()
    t = _dense_struct(m, (400000, 200, 30))      # mode 0 takes a 102 MB device accumulator
    M = m.GcpFactors()
    M.dtype, M.rank = m.F32, 64
    for k in range(3):
        M.A[k] = 0x1000
    cfg = m.GcpSampling()
    cfg.sampler = m.UNIFORM
    cfg.s = 50_000_000
    need = L.gcp_sampled_grad_workspace_bytes(ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg))
    assert need > (64 << 20)
    G = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    st = L.gcp_sampled_grad_noalloc(0, ctypes.byref(t), ctypes.byref(M), ctypes.byref(cfg), 1e-10, G, None, None)
    assert st == 4 and b"static" in L.gcp_last_error(), L.gcp_last_error()


def test_cols_per_lane_setter():
    m = _lib()
    L = m.lib()
    for bad in (3, 8, -1):
        assert L.gcp_set_cols_per_lane(bad) == 1
    for ok in (1, 2, 4, 0):
        assert L.gcp_set_cols_per_lane(ok) == 0


def test_stratified_problems_are_refused_in_batches():
    """Batches take uniform and semi-stratified sampling; a stratified problem
    (rejection sampling of zeros, Alg. 2) is refused with GCP_ERR_UNSUPPORTED
    and a message naming the problem, before any device work."""
    m = _lib()
    L = m.lib()
    probs = (m.GcpProblem * 2)()
    for b, sampler in enumerate((m.UNIFORM, m.STRATIFIED)):
        pr = probs[b]
        pr.X.d, pr.X.format, pr.X.vdtype = 3, m.COO, m.F32
        for k, n in enumerate((20, 30, 40)):
            pr.X.dims[k] = n
        pr.X.nnz = 100
        pr.X.coo_idx, pr.X.values, pr.X.nz_bitmap = 0x1000, 0x1000, 0x1000
        pr.X.nz_table, pr.X.nz_slots = 0x1000, 256
        pr.M.dtype, pr.M.rank = m.F32, 4
        off = 0
        for k, n in enumerate((20, 30, 40)):
            pr.M.A[k] = 0x10000 + off * 4
            off += n * 4
        pr.cfg.sampler = sampler
        pr.cfg.s, pr.cfg.p, pr.cfg.q = 500, 50, 50
        pr.A, pr.B, pr.C = 0x10000, 0x20000, 0x30000
        pr.lower = -math.inf
    h = ctypes.c_void_p()
    st = L.gcp_batched_create(probs, 2, None, ctypes.byref(h))
    assert st == 2 and b"problem 1" in L.gcp_last_error() and b"SEMI_STRATIFIED" in L.gcp_last_error()
    assert not h.value
