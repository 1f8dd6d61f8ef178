// kernels.hpp -- argument blocks of the gradient, loss and batched gradient
// kernels and the launch templates that the host launchers (grad.hip,
// batched.hip) call.  The templates are defined in grad_kernels.hpp and
// batched_kernels.hpp and instantiated once per mode count in inst.hip, which
// is compiled separately for d = 1..8.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "grad_device.hpp"

namespace gcp {

// Unfused derivative (gcp_loss_grad): samples, strata and values read from
// memory, ytilde written per sample.
struct LossArgs {
    int loss;
    int r;
    int lps;
    int cpl;
    int64_t S;
    int64_t n[GCP_MAX_D];
    const uint32_t* idx;
    const void* xval;
    const uint8_t* stratum;
    const void* A[GCP_MAX_D];
    double w[5];
    double eps;
    void* ytilde;
    double* loss_sum;
    // weighted objective (eq. wgcp); see GradArgs
    const void* weights;
    double w_zero;
    double kz;
    int format;
    NzTable tab;
};

// One work unit of a batch: a half-open range of one problem's 64-sample items.
struct BatchUnit {
    int32_t problem;
    int32_t reserved;
    int64_t item_begin, item_end;
};

struct BatchGradArgs {
    const GradArgs* probs;
    const BatchUnit* units;
    const int64_t* block_ptr;  // [gridDim.x + 1]
    const uint8_t* lds_fp32;   // per problem: LDS partial held in FP32
    const uint64_t* iter_ctr;
    int64_t* adam_state;
    uint32_t stage_off;  // byte offset of the per-wave sample records in the dynamic LDS
};

// Launch shape of a batched gradient step.
struct BatchLaunch {
    int64_t blocks;
    int threads;
    size_t lds_bytes;
    int fdtype, vdtype;
};

// Lets a kernel take up to 160 KB of dynamic LDS (set once per kernel).
void allow_full_lds(const void* kernel);

// ev_start/ev_stop (nullable): events stamped at the kernel's own start and end.
template <int D, bool LIST>
void grad_launch(const GradArgs& a, const ScatterPlan& pl, int fdtype, int vdtype, hipStream_t s,
                 hipEvent_t ev_start, hipEvent_t ev_stop);
template <int D>
void loss_launch(const LossArgs& a, int fdtype, int vdtype, hipStream_t s);
template <int D>
void batched_grad_launch(const BatchLaunch& bl, const BatchGradArgs& ba, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1);

}  // namespace gcp
