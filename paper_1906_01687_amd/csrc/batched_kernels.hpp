// batched_kernels.hpp -- the persistent gradient kernel of a batch of
// independent problems and its launch template (described at the top of
// batched.hip).  Included only by inst.hip, which instantiates it for one mode
// count per object file.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gcp {

template <typename LT>
__device__ __forceinline__ void clear_lds(LT* lds, int64_t n) {
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) lds[e] = LT(0);
}

template <typename LT>
__device__ __forceinline__ void flush_lds(const LT* lds, int64_t n, double* __restrict__ acc) {
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
        const LT v = lds[e];
        if (v != LT(0)) gadd(acc + e, (double)v);
    }
}

template <int D, typename FT, typename VT>
// The problem table is its own read-only, non-aliased argument: its fields are
// then read with scalar loads through the scalar cache and kept across a
// unit's items, instead of vector loads repeated for every item (device
// atomics in the loop could otherwise alias it).
__global__ __launch_bounds__(1024) void batched_grad_kernel(BatchGradArgs ba, const GradArgs* __restrict__ probs) {
    using T = typename Compute<FT>::type;
    extern __shared__ double lds[];
    // this wave's 64 sample records, after the largest partial
    Sample<D, T>* const stage =
        reinterpret_cast<Sample<D, T>*>(reinterpret_cast<char*>(lds) + ba.stage_off) + (threadIdx.x / kWave) * kWave;
    if (ba.adam_state && blockIdx.x == 0 && threadIdx.x == 0) ba.adam_state[0] += 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wib = threadIdx.x / kWave;
    const int64_t nwib = blockDim.x / kWave;
    // in flight across the first LDS clear and its barrier
    const uint64_t ctr = ba.iter_ctr ? counter_vmem(ba.iter_ctr) : 0;
    T fsum = T(0);
    const int64_t u_end = ba.block_ptr[blockIdx.x + 1];
    int32_t prev = -1;
    for (int64_t u = ba.block_ptr[blockIdx.x]; u < u_end; ++u) {
        const BatchUnit un = ba.units[u];
        const GradArgs& a = probs[un.problem];
        const bool f32 = ba.lds_fp32[un.problem] != 0;
        const int64_t n = a.lds_total;
        // a workgroup's units are sorted by problem: the partial is cleared when
        // a problem starts and flushed when it ends, not per unit
        if (un.problem != prev) {
            if (f32) clear_lds(reinterpret_cast<float*>(lds), n);
            else clear_lds(lds, n);
            __syncthreads();
        }
        const uint64_t iter = a.iter + (uint64_t)uni((int64_t)ctr);
        auto draw = [&](int64_t item) {
            const int64_t c = item * kWave + lane;
            Sample<D, T> smp = no_sample<D, T>();
            if (c < a.n_direct) {
                uint32_t i[D];
                T x, ew;
                int code;
                produce<D, VT, T>(a, iter, c, i, x, code, ew);
                smp = make_sample<D, T>(a, i, x, code, ew);
            }
            return smp;
        };
        int64_t item = un.item_begin + wib;
        Sample<D, T> cur = item < un.item_end ? draw(item) : no_sample<D, T>();
        for (; item < un.item_end; item += nwib) {
            // the next item's gathers are in flight while this one is evaluated
            Sample<D, T> nxt = item + nwib < un.item_end ? draw(item + nwib) : no_sample<D, T>();
            to_rows(a, cur);
            if (f32)
                evaluate_and_scatter<D, FT, false, float, false>(a, reinterpret_cast<float*>(lds), stage, cur, fsum);
            else
                evaluate_and_scatter<D, FT, false, double, false>(a, lds, stage, cur, fsum);
            cur = nxt;
        }
        const int32_t next = u + 1 < u_end ? ba.units[u + 1].problem : -1;
        if (next != un.problem) {
            __syncthreads();
            if (f32) flush_lds(reinterpret_cast<const float*>(lds), n, a.acc);
            else flush_lds(lds, n, a.acc);
            __syncthreads();
        }
        prev = un.problem;
    }
}

template <int D>
void batched_grad_launch(const BatchLaunch& bl, const BatchGradArgs& ba, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
    const dim3 g((unsigned)bl.blocks), t((unsigned)bl.threads);
    auto go = [&](auto kernel) {
        allow_full_lds(reinterpret_cast<const void*>(kernel));
        if (e0 || e1)
            hipExtLaunchKernelGGL(kernel, g, t, (std::uint32_t)bl.lds_bytes, s, e0, e1, 0u, ba, ba.probs);
        else
            hipLaunchKernelGGL(kernel, g, t, bl.lds_bytes, s, ba, ba.probs);
    };
    if (bl.fdtype == GCP_F64) {
        if (bl.vdtype == GCP_F64) go(batched_grad_kernel<D, double, double>);
        else go(batched_grad_kernel<D, double, float>);
    } else if (bl.fdtype == GCP_F32) {
        if (bl.vdtype == GCP_F64) go(batched_grad_kernel<D, float, double>);
        else go(batched_grad_kernel<D, float, float>);
    } else {
        if (bl.vdtype == GCP_F64) go(batched_grad_kernel<D, bf16_t, double>);
        else go(batched_grad_kernel<D, bf16_t, float>);
    }
}

}  // namespace gcp
