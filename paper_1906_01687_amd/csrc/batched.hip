// batched.hip -- many independent GCP problems advanced by one persistent
// gradient launch and one reduction + Adam launch.
//
// Each problem's samples are cut into work units of whole 64-sample items and
// the host shares them among the persistent workgroups by estimated cost, so
// problems of very different sizes finish together: either one contiguous run
// of the problem-ordered items per workgroup (a problem then spans few
// workgroups), or units dealt largest first to the least-loaded workgroup
// (longest processing time).  A workgroup walks its units in problem order:
// when a problem starts it clears that
// problem's gradient in LDS (FP64 when it fits, else FP32, else the problem
// scatters straight to device atomics), runs phases A and B of the
// single-problem kernel over the units' items, and when the problem ends it
// adds the non-zero LDS entries into the problem's FP64 accumulator with
// device atomics.  The
// reduction then applies Adam to every problem's parameters and clears the
// accumulators for the next step.  Per step that is two launches for the
// whole batch instead of three per problem.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <queue>
#include <unordered_set>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "grad_device.hpp"
#include "kernels.hpp"

namespace gcp {

// The fixed per-sample cost of the batch planner's estimate, in scattered elements.
constexpr int64_t kSampleFixedCost = 19;

// What the reduction needs per problem.
struct BatchReduceProblem {
    int64_t flat_off;     // first element of the problem in the concatenated accumulator
    int64_t P;            // sum_k n_k r
    int64_t first_block;  // the problem's first reduction workgroup
    void* A;
    float* A_master;
    void* B;
    void* C;
    void* G;
    double lower;
};

struct BatchReduceArgs {
    int adam;
    double* acc;
    int64_t nblk;  // reduction workgroups of all problems (entries of the block table)
    int64_t* state;
    uint64_t* bump_counter;
    double alpha, beta1, beta2, eps;
    int eps_mode;
};


constexpr int kBatchRedThreads = 256;

// Each block of the table covers kBatchRedThreads consecutive elements of one
// problem (a problem gets ceil(P / kBatchRedThreads) blocks), so the problem and
// its record are read with uniform loads through the scalar cache, ahead of the
// element loads, instead of a search over the problem offsets per element.  The
// tables are read-only, non-aliased kernel arguments for that reason.  A
// workgroup takes every gridDim.x-th block (one, unless the table is longer
// than the grid).
template <typename T, int ADAM>
__global__ __launch_bounds__(kBatchRedThreads) void batched_reduce_kernel(
    BatchReduceArgs r, const BatchReduceProblem* __restrict__ probs, const int32_t* __restrict__ blk_prob) {
    __shared__ double bc[2];
    if (r.bump_counter && blockIdx.x == 0 && threadIdx.x == 0) r.bump_counter[0] += 1;
    if (ADAM && threadIdx.x == 0) {
        const double t = (double)r.state[0];  // advanced by the gradient kernel
        bc[0] = 1.0 - pow(r.beta1, t);
        bc[1] = 1.0 - pow(r.beta2, t);
    }
    __syncthreads();
    for (int64_t j = blockIdx.x; j < r.nblk; j += gridDim.x) {
        const BatchReduceProblem& pb = probs[blk_prob[j]];
        const int64_t local = (j - pb.first_block) * kBatchRedThreads + threadIdx.x;
        if (local >= pb.P) continue;
        const int64_t e = pb.flat_off + local;
        const double g = r.acc[e];
        r.acc[e] = 0.0;  // cleared for the next step
        if (pb.G) static_cast<T*>(pb.G)[local] = (T)g;
        if constexpr (ADAM != 0) {
            T* B = static_cast<T*>(pb.B);
            T* C = static_cast<T*>(pb.C);
            const T gt = (T)g;
            const T bm = (T)r.beta1 * B[local] + (T)(1.0 - r.beta1) * gt;
            const T cm = (T)r.beta2 * C[local] + (T)(1.0 - r.beta2) * gt * gt;
            B[local] = bm;
            C[local] = cm;
            const T bhat = bm / (T)bc[0], chat = cm / (T)bc[1];
            const T den = r.eps_mode == GCP_EPS_INSIDE_SQRT ? sqrt(chat + (T)r.eps) : sqrt(chat) + (T)r.eps;
            const T step = (T)r.alpha * bhat / den;
            if constexpr (ADAM == 2) {
                float v = pb.A_master[local] - (float)step;
                v = v < (float)pb.lower ? (float)pb.lower : v;
                pb.A_master[local] = v;
                static_cast<bf16_t*>(pb.A)[local] = to_bf16(v);
            } else {
                T* A = static_cast<T*>(pb.A);
                const T v = A[local] - step;
                A[local] = v < (T)pb.lower ? (T)pb.lower : v;
            }
        }
    }
}

__global__ void fill_zero_f64_kernel(double* __restrict__ p, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

}  // namespace gcp

// ---------------------------------------------------------------------------
// Host side: the opaque batch handle.
// ---------------------------------------------------------------------------
using namespace gcp;

struct gcp_batch {
    int32_t count = 0;
    int d = 0;
    int fdtype = 0;
    int vdtype = 0;
    std::vector<GradArgs> args;
    std::vector<BatchUnit> units;
    std::vector<int64_t> block_ptr;
    std::vector<uint8_t> lds_fp32;
    std::vector<BatchReduceProblem> red;
    std::vector<int64_t> flat_off;
    std::vector<int32_t> red_blk;  // problem of each reduction workgroup
    int threads = 1024;
    int64_t blocks = 1;
    size_t lds_bytes = 0;
    uint32_t stage_off = 0;
    int64_t P_all = 0;
    // workspace layout
    size_t off_args = 0, off_units = 0, off_bptr = 0, off_f32 = 0, off_red = 0, off_rblk = 0, off_acc = 0;
    size_t ws_bytes = 0;
    char* ws = nullptr;
    // graph of captured steps (gcp_batched_graph_capture) and the stream it
    // was recorded on
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t graph_steps = 0;
};

namespace gcp {

constexpr int kXcds = 8;  // accelerator complex dies of an MI355X

gcp_status batch_create(const gcp_problem* problems, int32_t count, const gcp_batch_tuning* tune, gcp_batch** out,
                        gcp_status (*check_problem)(const gcp_problem*, int32_t)) {
    if (!out) return set_error(GCP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!problems || count < 1) return set_error(GCP_ERR_INVALID_ARG, "need at least one problem");
    for (int32_t b = 0; b < count; ++b)
        if (gcp_status st = check_problem(&problems[b], b)) return st;
    const int d = problems[0].X.d, fdt = problems[0].M.dtype, vdt = problems[0].X.vdtype;
    for (int32_t b = 1; b < count; ++b)
        if (problems[b].X.d != d || problems[b].M.dtype != fdt || problems[b].X.vdtype != vdt)
            return set_error(GCP_ERR_UNSUPPORTED, "all problems of a batch need the same d, factor dtype and value dtype");
    int threads = tune && tune->threads ? tune->threads : 1024;
    if (threads != 256 && threads != 512 && threads != 1024)
        return set_error(GCP_ERR_INVALID_ARG, "tune->threads must be 256, 512 or 1024");
    const int64_t unit_items = tune && tune->unit_items > 0 ? tune->unit_items : 64;
    const int schedule = tune ? tune->schedule : GCP_BATCH_CONTIGUOUS;
    if (schedule != GCP_BATCH_CONTIGUOUS && schedule != GCP_BATCH_LPT)
        return set_error(GCP_ERR_INVALID_ARG, "tune->schedule must be GCP_BATCH_CONTIGUOUS or GCP_BATCH_LPT");

    gcp_batch* B = new gcp_batch();
    B->count = count;
    B->d = d;
    B->fdtype = fdt;
    B->vdtype = vdt;
    B->threads = threads;
    B->args.resize(count);
    B->lds_fp32.resize(count);
    B->red.resize(count);
    B->flat_off.resize(count + 1);
    int64_t flat = 0;
    int64_t lds_max = 0;
    // the per-wave sample records sit after the partial; partials get the rest
    const int64_t stage_bytes = (int64_t)threads * stage_record_bytes(d, fdt);
    const int64_t budget = kLdsLimitBytes - stage_bytes - 4096;
    std::vector<double> item_cost(count);
    std::vector<int64_t> items(count);
    int64_t total_items = 0;
    for (int32_t b = 0; b < count; ++b) {
        const gcp_problem& pr = problems[b];
        const int64_t r = pr.M.rank;
        GradArgs a{};
        for (int k = 0; k < d; ++k) a.dims.n[k] = pr.X.dims[k];
        a.loss = pr.loss;
        a.sampler = pr.cfg.sampler;
        a.format = pr.X.format;
        a.r = (int)r;
        a.nnz = pr.X.nnz;
        a.seed = pr.cfg.seed;
        a.pid = pr.cfg.problem_id;
        a.iter = pr.cfg.iteration;
        a.values = pr.X.values;
        a.coo = pr.X.coo_idx;
        if (pr.X.nz_table && pr.X.nz_slots > 0) {
            a.tab.keys = static_cast<const uint64_t*>(pr.X.nz_table);
            a.tab.pos = reinterpret_cast<const uint32_t*>(static_cast<const char*>(pr.X.nz_table) + 8 * pr.X.nz_slots);
            a.tab.mask = (uint64_t)pr.X.nz_slots - 1;
        }
        a.tab.bitmap = pr.X.nz_bitmap;
        if (pr.cfg.sampler == GCP_SAMPLER_UNIFORM || pr.cfg.sampler == GCP_SAMPLER_FULL) {
            a.n_direct = pr.cfg.sampler == GCP_SAMPLER_FULL ? full_count(&pr.X) : pr.cfg.s;
            a.p = 0;
        } else {
            a.n_direct = pr.cfg.p + pr.cfg.q;
            a.p = pr.cfg.p;
        }
        a.n_direct_items = (a.n_direct + kWave - 1) / kWave;
        int64_t off = 0;
        for (int k = 0; k < d; ++k) {
            a.A[k] = pr.M.A[k];
            a.lds_off[k] = off;
            a.acc_off[k] = off;
            off += pr.X.dims[k] * r;
        }
        const int64_t P = off;
        // LDS partial: FP64 if it fits, else FP32, else device atomics only
        if (P * 8 <= budget) {
            a.priv_mask = (1u << d) - 1u;
            a.lds_total = P;
            B->lds_fp32[b] = 0;
            lds_max = std::max(lds_max, P * 8);
        } else if (P * 4 <= budget) {
            a.priv_mask = (1u << d) - 1u;
            a.lds_total = P;
            B->lds_fp32[b] = 1;
            lds_max = std::max(lds_max, P * 4);
        } else {
            a.priv_mask = 0;
            a.lds_total = 0;
            B->lds_fp32[b] = 0;
        }
        a.cpl = cols_per_lane(r, tune ? tune->cols_per_lane : 0, a.priv_mask == 0);
        a.lps = lanes_per_sample(r, a.cpl);
        stratum_weights(&pr.X, &pr.cfg, a.w);
        a.kz = corr_zero_weight(&pr.X, &pr.cfg);
        a.weights = pr.X.weights;
        a.w_zero = zero_weight(&pr.X);
        a.eps = pr.eps;
        B->args[b] = a;
        B->flat_off[b] = flat;
        BatchReduceProblem rp{};
        rp.flat_off = flat;
        rp.P = P;
        rp.first_block = (int64_t)B->red_blk.size();
        B->red_blk.insert(B->red_blk.end(), (size_t)((P + kBatchRedThreads - 1) / kBatchRedThreads), b);
        rp.A = pr.A;
        rp.A_master = pr.A_master;
        rp.B = pr.B;
        rp.C = pr.C;
        rp.G = pr.G;
        rp.lower = pr.lower;
        B->red[b] = rp;
        flat += P;
        // estimated cost of one sample in units of one scattered element: a
        // fixed part (draw, gather, derivative, group sum) and the scatter of
        // its d rows of r entries (fitted to sub-batches of 64 dense cubes by
        // rank on MI355X: about 52, 97 and 194 ps per sample at r = 4, 16, 32)
        item_cost[b] = (double)kWave * (double)(kSampleFixedCost + d * r);
        items[b] = a.n_direct_items;
        total_items += a.n_direct_items;
    }
    B->flat_off[count] = flat;
    B->P_all = flat;
    const int64_t stage_off = (lds_max + 15) / 16 * 16;
    B->stage_off = (uint32_t)stage_off;
    B->lds_bytes = (size_t)(stage_off + stage_bytes);
    for (int32_t b = 0; b < count; ++b) B->args[b].stage_off = (uint32_t)stage_off;
    // persistent grid: as many workgroups as fit at once
    int per_cu = (int)(kLdsLimitBytes / ((int64_t)B->lds_bytes + 1024));
    per_cu = std::min(per_cu, 2048 / threads);
    per_cu = std::max(per_cu, 1);
    int64_t blocks = (int64_t)device_cu_count() * per_cu;
    blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, std::max<int64_t>(1, total_items)));
    std::vector<std::vector<BatchUnit>> per_block(blocks);
    if (schedule == GCP_BATCH_CONTIGUOUS) {
        // cut the problem-ordered item sequence at multiples of total/blocks of
        // the running cost; a workgroup's units are then already in problem order
        double total = 0.0;
        for (int32_t b = 0; b < count; ++b) total += item_cost[b] * (double)items[b];
        const double share = total / (double)blocks;
        double done = 0.0;
        int64_t w = 0;
        for (int32_t b = 0; b < count; ++b) {
            int64_t i0 = 0;
            while (i0 < items[b]) {
                int64_t i1 = items[b];
                if (w < blocks - 1) {
                    const double room = share * (double)(w + 1) - done;
                    const int64_t fit = (int64_t)std::ceil(room / item_cost[b] - 1e-9);
                    i1 = std::min(items[b], i0 + std::max<int64_t>(1, fit));
                }
                per_block[w].push_back(BatchUnit{b, 0, i0, i1});
                done += item_cost[b] * (double)(i1 - i0);
                if (w < blocks - 1 && done >= share * (double)(w + 1) - 1e-9 * share) ++w;
                i0 = i1;
            }
        }
    } else {
        struct Cost {
            double cost;
            BatchUnit unit;
        };
        std::vector<Cost> costs;
        for (int32_t b = 0; b < count; ++b)
            for (int64_t i0 = 0; i0 < items[b]; i0 += unit_items) {
                const int64_t i1 = std::min(i0 + unit_items, items[b]);
                costs.push_back({item_cost[b] * (double)(i1 - i0), BatchUnit{b, 0, i0, i1}});
            }
        // longest processing time first onto the least-loaded workgroup, then
        // each workgroup's units in problem order so it flushes once per
        // problem.  (Dealing each XCD's share of the problem-ordered units over
        // that XCD's workgroups only, for L2 locality, was measured slower on
        // 64 dense cubes, 202 against 195 us: with few problems per workgroup
        // the errors of the cost estimate no longer average out.)
        std::stable_sort(costs.begin(), costs.end(), [](const Cost& x, const Cost& y) { return x.cost > y.cost; });
        using Slot = std::pair<double, int64_t>;
        std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
        for (int64_t w = 0; w < blocks; ++w) heap.push({0.0, w});
        for (const Cost& c : costs) {
            Slot sl = heap.top();
            heap.pop();
            per_block[sl.second].push_back(c.unit);
            heap.push({sl.first + c.cost, sl.second});
        }
        for (auto& v : per_block)
            std::sort(v.begin(), v.end(), [](const BatchUnit& x, const BatchUnit& y) {
                return x.problem != y.problem ? x.problem < y.problem : x.item_begin < y.item_begin;
            });
    }
    B->blocks = blocks;
    // Workgroups are dispatched round-robin over the XCDs (workgroup id mod 8).
    // Contiguous runs w are placed so that each XCD takes one contiguous eighth
    // of the problem-ordered sequence: a problem's factors and data then sit
    // in the L2 of one or two XCDs instead of all eight.
    std::vector<int64_t> run_of(blocks);
    {
        std::vector<int64_t> first(kXcds + 1, 0);
        for (int x = 0; x < kXcds; ++x) first[x + 1] = first[x] + (blocks - x + kXcds - 1) / kXcds;
        for (int64_t id = 0; id < blocks; ++id)
            run_of[id] = schedule == GCP_BATCH_CONTIGUOUS ? first[id % kXcds] + id / kXcds : id;
    }
    B->block_ptr.assign(blocks + 1, 0);
    for (int64_t id = 0; id < blocks; ++id) {
        const std::vector<BatchUnit>& v = per_block[run_of[id]];
        B->block_ptr[id + 1] = B->block_ptr[id] + (int64_t)v.size();
        B->units.insert(B->units.end(), v.begin(), v.end());
    }
    // workspace layout (256-byte aligned regions)
    size_t off = 0;
    auto place = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        const size_t at = off;
        off += bytes;
        return at;
    };
    B->off_args = place(sizeof(GradArgs) * (size_t)count);
    B->off_units = place(sizeof(BatchUnit) * std::max<size_t>(1, B->units.size()));
    B->off_bptr = place(sizeof(int64_t) * ((size_t)blocks + 1));
    B->off_f32 = place((size_t)count);
    B->off_red = place(sizeof(BatchReduceProblem) * (size_t)count);
    B->off_rblk = place(sizeof(int32_t) * B->red_blk.size());
    B->off_acc = place(sizeof(double) * (size_t)std::max<int64_t>(1, flat));
    B->ws_bytes = (off + 255) & ~size_t(255);
    *out = B;
    return GCP_OK;
}

size_t batch_ws_bytes(const gcp_batch* B) { return B ? B->ws_bytes : 0; }

gcp_status batch_prepare(gcp_batch* B, void* ws, size_t ws_bytes, hipStream_t s) {
    if (!B) return set_error(GCP_ERR_INVALID_ARG, "batch is NULL");
    if (!ws || ws_bytes < B->ws_bytes)
        return set_error(GCP_ERR_WORKSPACE, "workspace needs " + std::to_string(B->ws_bytes) + " bytes");
    char* base = static_cast<char*>(ws);
    double* acc = reinterpret_cast<double*>(base + B->off_acc);
    std::vector<GradArgs> args = B->args;
    for (int32_t b = 0; b < B->count; ++b) args[b].acc = acc + B->flat_off[b];
    struct Copy {
        size_t off;
        const void* src;
        size_t bytes;
    };
    const Copy copies[] = {
        {B->off_args, args.data(), sizeof(GradArgs) * args.size()},
        {B->off_units, B->units.data(), sizeof(BatchUnit) * B->units.size()},
        {B->off_bptr, B->block_ptr.data(), sizeof(int64_t) * B->block_ptr.size()},
        {B->off_f32, B->lds_fp32.data(), B->lds_fp32.size()},
        {B->off_red, B->red.data(), sizeof(BatchReduceProblem) * B->red.size()},
        {B->off_rblk, B->red_blk.data(), sizeof(int32_t) * B->red_blk.size()},
    };
    // the tables are small and this is set-up, not the hot path: copy synchronously
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(GCP_ERR_HIP, "hipStreamSynchronize failed");
    for (const Copy& cp : copies)
        if (cp.bytes && hipMemcpy(base + cp.off, cp.src, cp.bytes, hipMemcpyHostToDevice) != hipSuccess)
            return set_error(GCP_ERR_HIP, "uploading the batch tables failed");
    const int64_t n = std::max<int64_t>(1, B->P_all);
    hipLaunchKernelGGL(fill_zero_f64_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, s,
                       acc, n);
    B->ws = base;
    return check_launch("gcp_batched_prepare");
}


gcp_status batch_step(gcp_batch* B, const AdamParams* adam, uint64_t* iteration_counter, hipEvent_t e0, hipEvent_t e1,
                      hipStream_t s) {
    if (!B || !B->ws) return set_error(GCP_ERR_INVALID_ARG, "batch not prepared (call gcp_batched_prepare)");
    char* base = B->ws;
    BatchGradArgs ba{};
    ba.probs = reinterpret_cast<const GradArgs*>(base + B->off_args);
    ba.units = reinterpret_cast<const BatchUnit*>(base + B->off_units);
    ba.block_ptr = reinterpret_cast<const int64_t*>(base + B->off_bptr);
    ba.lds_fp32 = reinterpret_cast<const uint8_t*>(base + B->off_f32);
    ba.iter_ctr = iteration_counter;
    ba.adam_state = adam ? adam->state : nullptr;
    ba.stage_off = B->stage_off;
    const BatchLaunch bl{B->blocks, B->threads, B->lds_bytes, B->fdtype, B->vdtype};
    dispatch_d(B->d, [&](auto dc) { batched_grad_launch<decltype(dc)::value>(bl, ba, s, e0, e1); });
    if (gcp_status st = check_launch("gcp_batched step (gradient)")) return st;
    BatchReduceArgs r{};
    const auto* rprobs = reinterpret_cast<const BatchReduceProblem*>(base + B->off_red);
    const auto* rblk = reinterpret_cast<const int32_t*>(base + B->off_rblk);
    r.acc = reinterpret_cast<double*>(base + B->off_acc);
    r.nblk = (int64_t)B->red_blk.size();
    r.bump_counter = iteration_counter;
    if (adam) {
        r.adam = 1;
        r.state = adam->state;
        r.alpha = adam->alpha;
        r.beta1 = adam->beta1;
        r.beta2 = adam->beta2;
        r.eps = adam->eps;
        r.eps_mode = adam->eps_mode;
    }
    const dim3 g((unsigned)std::min<int64_t>(65536, r.nblk)), t(kBatchRedThreads);
    if (!adam) {
        if (B->fdtype == GCP_F64) hipLaunchKernelGGL((batched_reduce_kernel<double, 0>), g, t, 0, s, r, rprobs, rblk);
        else hipLaunchKernelGGL((batched_reduce_kernel<float, 0>), g, t, 0, s, r, rprobs, rblk);
    } else if (B->fdtype == GCP_F64) {
        hipLaunchKernelGGL((batched_reduce_kernel<double, 1>), g, t, 0, s, r, rprobs, rblk);
    } else if (B->fdtype == GCP_F32) {
        hipLaunchKernelGGL((batched_reduce_kernel<float, 1>), g, t, 0, s, r, rprobs, rblk);
    } else {
        hipLaunchKernelGGL((batched_reduce_kernel<float, 2>), g, t, 0, s, r, rprobs, rblk);
    }
    return check_launch("gcp_batched step (reduction)");
}

void batch_graph_destroy(gcp_batch* B) {
    if (!B) return;
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->graph_steps = 0;
}

gcp_status batch_graph_capture(gcp_batch* B, int32_t steps, const AdamParams* adam, uint64_t* iteration_counter) {
    if (!B || !B->ws) return set_error(GCP_ERR_INVALID_ARG, "batch not prepared (call gcp_batched_prepare)");
    if (steps < 1) return set_error(GCP_ERR_INVALID_ARG, "steps must be >= 1");
    batch_graph_destroy(B);
    // the steps are recorded on a stream of the batch's own (a legacy default
    // stream cannot be captured); replays go to the caller's stream
    if (!B->cap_stream && hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        B->cap_stream = nullptr;
        return check_launch("gcp_batched_graph_capture (stream)");
    }
    if (hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return check_launch("gcp_batched_graph_capture (begin)");
    gcp_status st = GCP_OK;
    for (int32_t i = 0; i < steps && st == GCP_OK; ++i) st = batch_step(B, adam, iteration_counter, nullptr, nullptr, B->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
    if (st != GCP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess || !g) return check_launch("gcp_batched_graph_capture (end)");
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return check_launch("gcp_batched_graph_capture (instantiate)");
    }
    B->graph = g;
    B->exec = x;
    B->graph_steps = steps;
    return GCP_OK;
}

gcp_status batch_graph_launch(gcp_batch* B, hipStream_t s) {
    if (!B || !B->exec) return set_error(GCP_ERR_INVALID_ARG, "the batch holds no captured graph");
    if (hipGraphLaunch(B->exec, s) != hipSuccess) return check_launch("gcp_batched_graph_launch");
    return GCP_OK;
}

void batch_destroy(gcp_batch* B) {
    if (!B) return;
    batch_graph_destroy(B);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    delete B;
}

int64_t batch_blocks(const gcp_batch* B) { return B ? B->blocks : 0; }

gcp_status batch_plan(const gcp_batch* B, int64_t* n_blocks, int64_t* n_units, int64_t* block_ptr,
                      int32_t* unit_problem, int64_t* unit_items) {
    if (!B) return set_error(GCP_ERR_INVALID_ARG, "batch is NULL");
    if (n_blocks) *n_blocks = B->blocks;
    if (n_units) *n_units = (int64_t)B->units.size();
    if (block_ptr) std::copy(B->block_ptr.begin(), B->block_ptr.end(), block_ptr);
    for (size_t u = 0; u < B->units.size(); ++u) {
        if (unit_problem) unit_problem[u] = B->units[u].problem;
        if (unit_items) {
            unit_items[2 * u] = B->units[u].item_begin;
            unit_items[2 * u + 1] = B->units[u].item_end;
        }
    }
    return GCP_OK;
}

}  // namespace gcp
