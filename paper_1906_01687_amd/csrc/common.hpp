// common.hpp -- host-side plumbing shared by the libgcp sources: the
// per-thread error message, workspace carving, and the launchers that the
// C ABI (abi.cpp) calls after validating its arguments.
#pragma once

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

// Rejection sampling of stratified zeros: 1024 candidates per block.
constexpr int kRejThreads = 256;
constexpr int kRejItems = 4;
constexpr int kRejTile = kRejThreads * kRejItems;
// Refill loop cap (tiles of 1024 candidates beyond the first batch).
constexpr int64_t kRejMaxRefillTiles = int64_t(1) << 22;

// Number of candidates in the first rejection batch.
int64_t rejection_batch(const gcp_tensor* X, const gcp_sampling* cfg);

// Scratch used by the rejection pipeline for a first batch of `ncand`.
struct RejScratch {
    uint32_t* block_count;   // [nblk]
    uint64_t* block_offset;  // [nblk]
    uint64_t* total;         // [1] accepted in the first batch
    uint32_t* status;        // [1] 0 ok, 1 refill cap reached
    int64_t nblk;
};
RejScratch carve_rejection(Carver& c, void* base, int64_t ncand);

// Launchers (arguments already validated).
gcp_status launch_nz_build(const gcp_tensor* X, void* table, int64_t slots, hipStream_t s);

// Direct samples c in [first, first + count) of one kind, written at out_off.
enum SampleKind { kKindUniform = 0, kKindNonzero = 1, kKindSemiZero = 2 };
gcp_status launch_sample_direct(const gcp_tensor* X, const gcp_sampling* cfg, int kind,
                                int64_t count, int64_t out_off, uint32_t* idx, void* xval,
                                uint8_t* stratum, hipStream_t s);

// Rejection pipeline: the first q accepted candidates' indices are written to
// idx_out + (p_off + rank) * d; if xval/stratum are given they get 0 / ZERO.
gcp_status launch_rejection(const gcp_tensor* X, const gcp_sampling* cfg, int64_t ncand,
                            const RejScratch& rs, uint32_t* idx_out, int64_t p_off, void* xval,
                            uint8_t* stratum, hipStream_t s);

// Stratum weights for X and cfg (omega/s, eta/p, zeta/q, eta/p, omega/q).
void stratum_weights(const gcp_tensor* X, const gcp_sampling* cfg, double w[5]);

gcp_status launch_loss_grad(gcp_loss loss, const gcp_tensor* X, const gcp_sampling* cfg,
                            const gcp_factors* M, const uint32_t* idx, const void* xval,
                            const uint8_t* stratum, int64_t S, double eps, void* ytilde,
                            double* loss_sum, hipStream_t s);

// FP64 accumulators for all modes: acc + offset[k], offset[d] = total.
struct AccLayout {
    int64_t offset[GCP_MAX_D + 1];
};
AccLayout acc_layout(const gcp_tensor* X, const gcp_factors* M);

gcp_status launch_fill_zero(double* p, int64_t n, hipStream_t s);
gcp_status launch_finalize(const gcp_tensor* X, const gcp_factors* M, const double* acc,
                           const AccLayout& L, void* const* G, int accumulate, hipStream_t s);

gcp_status launch_mttkrp_list(const gcp_tensor* X, const gcp_factors* M, const uint32_t* idx,
                              const void* ytilde, int64_t S, double* acc, const AccLayout& L,
                              hipStream_t s);

gcp_status launch_fused(gcp_loss loss, const gcp_tensor* X, const gcp_factors* M,
                        const gcp_sampling* cfg, double eps, const uint32_t* zero_list,
                        double* acc, const AccLayout& L, double* loss_sum, hipStream_t s);

gcp_status launch_adam(int64_t P, gcp_dtype dtype, void* A, float* A_master, const void* G,
                       void* B, void* C, int64_t* state, double alpha, double beta1, double beta2,
                       double eps, double lower, gcp_eps_mode eps_mode, hipStream_t s);

}  // namespace gcp
