// common.hpp -- host-side plumbing shared by the libgcp sources: the
// per-thread error message, workspace carving, and the launchers that the
// C ABI (abi.cpp) calls after validating its arguments.
#pragma once

#include <atomic>

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <type_traits>

#include "gcp.h"

namespace gcp {

// Calls f(std::integral_constant<int, D>{}) for the runtime mode count d.
template <typename F>
void dispatch_d(int d, F&& f) {
    switch (d) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
    }
}

// Per-thread last error; set_error returns its status for `return set_error(...)`.
gcp_status set_error(gcp_status st, const std::string& msg);
void clear_error();

// Launch-error check after a kernel launch.
gcp_status check_launch(const char* what);

// Workspace carving: 256-byte aligned regions inside one caller buffer.
struct Carver {
    size_t off = 0;
    template <typename T>
    T* take(void* base, size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(static_cast<char*>(base) + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

// Rejection sampling of stratified zeros: candidates are counted per chunk of
// 64 (one wave), chunk counts are scanned, then ranked per chunk.
constexpr int kRejChunk = 64;
constexpr int kRejThreads = 256;
// Refill loop cap: one wave examines at most this many turns of 64
// candidates beyond the first batch (about 4.2e6 candidates, tens of ms).
// The host refuses a configuration whose first batch plus this cap falls short
// of the expected candidate count q omega / zeta by eight standard deviations,
// so the cap is reached with probability below 1e-15; if it is reached, the
// status word of the rejection scratch reads 1.
constexpr int64_t kRejRefillTurns = int64_t(1) << 16;
constexpr int64_t kRejRefillCandidates = kRejRefillTurns * 64;

// Number of candidates in the first rejection batch.
int64_t rejection_batch(const gcp_tensor* X, const gcp_sampling* cfg);

// Scratch of the rejection pipeline for a first batch of `ncand` candidates.
struct RejScratch {
    uint32_t* chunk_count;   // [nchunks]
    uint64_t* chunk_prefix;  // [nchunks + 1]: exclusive prefixes, then the total (scan)
    uint32_t* group_sum;     // [ngroups]: accepted per 4 chunks (fused path; else NULL)
    uint32_t* zstage;        // [nchunks * 64 * d]: accepted indices per chunk (fused path; else NULL)
    uint32_t* status;        // [1] 0 ok, 1 refill cap reached (cleared by the count kernel)
    int64_t nchunks;
    int64_t ngroups;
};
// staged == true adds group_sum and zstage (the fused gradient path).
RejScratch carve_rejection(Carver& c, void* base, int64_t ncand, bool staged, int d);
// Group count up to which the fused kernel forms chunk prefixes itself
// instead of reading a scan.
constexpr int64_t kMaxGroupsInKernel = 2048;

// Phase-B lane layout: rank columns per lane (1, 2 or 4) and lanes per sample
// (the power of two >= ceil(r / cpl), at most 64).  hint 0 picks by rank and
// scatter (or takes the process-wide choice of gcp_set_cols_per_lane); a hint
// that does not fit r falls back to the automatic choice.  device_atomics:
// some mode is accumulated with device atomics.
int cols_per_lane(int64_t r, int hint, bool device_atomics = false);
int lanes_per_sample(int64_t r, int cpl);
// Whether cpl columns per lane can carry rank r (every sample fits one wave).
bool cols_per_lane_fits(int64_t r, int cpl);
// Swizzle of the single-problem kernel's LDS partial (d modes, elements of
// elem_bytes, rows of r columns handled as cpl chunks of lps): shift and mask
// of lds_swizzle, mask 0 for the plain layout.
void lds_swizzle_params(int d, int64_t r, int lps, int cpl, int elem_bytes, uint32_t* shift, uint32_t* mask);
extern std::atomic<int> g_cols_per_lane;

// Multiprocessor count of the current device (cached per device).
int device_cu_count();

// LDS bytes a gradient workgroup may use for privatised FP64 partials.
constexpr int64_t kLdsBudgetBytes = 156 * 1024;
constexpr int64_t kLdsLimitBytes = 160 * 1024;  // dynamic LDS of one workgroup on gfx950
// FP32 device accumulation while a mode averages at most this many adds per element
constexpr int64_t kAcc32MaxAdds = 1024;

// Bytes of one staged sample record (row offsets of d modes, value, weight),
// padded to 16 like the device struct.
inline int64_t stage_record_bytes(int d, int fdtype) {
    const int64_t raw = 4 * (int64_t)d + 2 * (fdtype == GCP_F64 ? 8 : 4);
    return (raw + 15) / 16 * 16;
}

// How a gradient launch scatters: which modes are privatised in LDS (and
// where), which use device atomics, and the launch shape.
struct ScatterPlan {
    int d;
    int64_t P;                          // sum_k n_k r
    int64_t off[GCP_MAX_D + 1];         // flat element offset of mode k
    uint32_t priv_mask;                 // bit k: mode k accumulated in LDS
    int64_t lds_off[GCP_MAX_D];         // offset of mode k in the LDS partial (elements)
    int64_t lds_total;                  // elements of one partial
    int lds_elem;                       // bytes per LDS element: 8 (FP64) or 4 (FP32, CAS adds)
    uint32_t stage_off;                 // byte offset of the per-wave sample records, or 0xFFFFFFFF
    int64_t shm_bytes;                  // dynamic LDS of one gradient workgroup
    int64_t acc_off[GCP_MAX_D];         // offset of mode k in the atomic accumulator (elements)
    int64_t acc_total;                  // accumulator elements
    int acc_elem;                       // bytes per accumulator element: 8 (FP64) or 4 (FP32)
    uint32_t acc_stride;                // accumulator elements per factor row (>= r)
    uint32_t acc_magic;                 // ceil(2^32 / r) when acc_stride != r, else 0
    int64_t blocks;                     // gradient workgroups (= number of partials)
    int threads;                        // threads per gradient workgroup
};
ScatterPlan plan_scatter(const gcp_tensor* X, const gcp_factors* M, int64_t n_items);
// 8-byte words of the atomic accumulator (what a workspace holds and a clear covers)
inline int64_t acc_words(const ScatterPlan& pl) { return (pl.acc_total * pl.acc_elem + 7) / 8; }
size_t scatter_partials_bytes(const ScatterPlan& pl, int fdtype);
int64_t fused_items(const gcp_tensor* X, const gcp_sampling* cfg, int64_t ncand);

struct AdamParams {
    void* A;
    float* A_master;
    void* B;
    void* C;
    int64_t* state;
    double alpha, beta1, beta2, eps, lower;
    int eps_mode;
};

// Launchers (arguments already validated).
gcp_status launch_nz_build(const gcp_tensor* X, void* table, int64_t slots, hipStream_t s);
gcp_status launch_nz_bitmap(const gcp_tensor* X, uint32_t* bitmap, size_t bytes, hipStream_t s);

// Direct samples c in [0, count) of one kind, written at out_off.
enum SampleKind { kKindUniform = 0, kKindNonzero = 1, kKindSemiZero = 2, kKindFull = 3 };
gcp_status launch_sample_direct(const gcp_tensor* X, const gcp_sampling* cfg, int kind,
                                int64_t count, int64_t out_off, uint32_t* idx, void* xval,
                                uint8_t* stratum, hipStream_t s);

// Chunk counts and their scan for the first rejection batch.
gcp_status launch_rejection_count(const gcp_tensor* X, const gcp_sampling* cfg, int64_t ncand,
                                  const RejScratch& rs, bool scan, hipStream_t s);
// Writes the first q accepted candidates' indices at idx_out + (p_off + rank) * d
// (xval/stratum get 0 / ZERO when given), including the device-side refill.
gcp_status launch_rejection_write(const gcp_tensor* X, const gcp_sampling* cfg, int64_t ncand,
                                  const RejScratch& rs, uint32_t* idx_out, int64_t p_off, void* xval,
                                  uint8_t* stratum, hipStream_t s);

// Adds 1 to the device iteration counter (no-op for NULL).
gcp_status launch_bump_counter(uint64_t* counter, hipStream_t s);

// Stratum weights for X and cfg (omega/s, eta/p, zeta/q, eta/p, omega/q).
void stratum_weights(const gcp_tensor* X, const gcp_sampling* cfg, double w[5]);
double zero_weight(const gcp_tensor* X);
int64_t full_count(const gcp_tensor* X);  // entries of X (the FULL sampler's sample count)
double corr_zero_weight(const gcp_tensor* X, const gcp_sampling* cfg);

gcp_status launch_loss_grad(gcp_loss loss, const gcp_tensor* X, const gcp_sampling* cfg,
                            const gcp_factors* M, const uint32_t* idx, const void* xval,
                            const uint8_t* stratum, int64_t S, double eps, void* ytilde,
                            double* loss_sum, hipStream_t s);

gcp_status launch_fill_zero(double* p, int64_t n, hipStream_t s);

gcp_status launch_grad_list(const gcp_tensor* X, const gcp_factors* M, const uint32_t* idx,
                            const void* ytilde, int64_t S, const ScatterPlan& pl, double* acc,
                            void* partials, hipStream_t s);

// ev_start/ev_stop (nullable): events stamped at the kernel's own start and
// end (launched with hipExtLaunchKernelGGL).
// adam_state (nullable): the gradient kernel advances the Adam step count
// state[0] by one; the reduction that follows reads the new value.
gcp_status launch_grad_fused(gcp_loss loss, const gcp_tensor* X, const gcp_factors* M,
                             const gcp_sampling* cfg, double eps, const ScatterPlan& pl, int64_t ncand,
                             const RejScratch* rs, bool scanned, double* acc, void* partials,
                             double* loss_sum, int64_t* adam_state, hipEvent_t ev_start, hipEvent_t ev_stop,
                             hipStream_t s);

// G[k] (nullable entries) from partials and accumulator; with adam != NULL the
// Adam step is applied to the same elements in the same kernel.
// A non-NULL bump_counter is incremented by the reduction (after every read).
gcp_status launch_reduce(const gcp_factors* M, const ScatterPlan& pl, const double* acc,
                         const void* partials, void* const* G, int accumulate, const AdamParams* adam,
                         uint64_t* bump_counter, hipStream_t s, const double* scale = nullptr);

// Batched problems (batched.hip); check_problem validates one problem.
gcp_status batch_create(const gcp_problem* problems, int32_t count, const gcp_batch_tuning* tune, gcp_batch** out,
                        gcp_status (*check_problem)(const gcp_problem*, int32_t));
size_t batch_ws_bytes(const gcp_batch* b);
gcp_status batch_prepare(gcp_batch* b, void* ws, size_t ws_bytes, hipStream_t s);
gcp_status batch_step(gcp_batch* b, const AdamParams* adam, uint64_t* iteration_counter, hipEvent_t e0, hipEvent_t e1,
                      hipStream_t s);
void batch_destroy(gcp_batch* b);
gcp_status batch_graph_capture(gcp_batch* b, int32_t steps, const AdamParams* adam, uint64_t* iteration_counter);
gcp_status batch_graph_launch(gcp_batch* b, hipStream_t s);
void batch_graph_destroy(gcp_batch* b);
int64_t batch_blocks(const gcp_batch* b);
gcp_status batch_plan(const gcp_batch* b, int64_t* n_blocks, int64_t* n_units, int64_t* block_ptr,
                      int32_t* unit_problem, int64_t* unit_items);

// dst[e] = src[e] rounded to bf16 (nearest even), e < P.
gcp_status launch_bf16_round(int64_t P, const float* src, void* dst, hipStream_t s);
gcp_status launch_adam(int64_t P, gcp_dtype dtype, void* A, float* A_master, const void* G,
                       void* B, void* C, int64_t* state, double alpha, double beta1, double beta2,
                       double eps, double lower, gcp_eps_mode eps_mode, hipStream_t s);

}  // namespace gcp
