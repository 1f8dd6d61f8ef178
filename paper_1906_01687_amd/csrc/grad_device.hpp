// grad_device.hpp -- device code shared by the single-problem and batched
// gradient kernels: the per-problem argument block, phase A (one sample per
// lane) and phase B (lane-group evaluation and scatter).
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace gcp {

struct GradArgs {
    Dims dims;
    int loss;
    int sampler;
    int format;
    int r;
    int lps;
    int64_t nnz;
    uint64_t seed, pid, iter;
    const uint64_t* iter_ctr;
    const void* values;
    const uint32_t* coo;
    NzTable tab;
    // direct items: samples c in [0, n_direct), 64 per item
    int64_t n_direct, n_direct_items, p;
    // stratified zeros: one item per chunk of 64 rejection candidates
    int64_t n_zero_items, ncand, q, ngroups;
    const uint32_t* chunk_count;
    const uint32_t* group_sum;
    const uint32_t* zstage;
    const uint64_t* chunk_prefix;  // non-NULL when a scan provided the prefixes
    // list mode (gcp_mttkrp): indices and ytilde per sample
    const uint32_t* idx;
    const void* ytilde;
    const void* A[GCP_MAX_D];
    // scatter targets
    uint32_t priv_mask;
    int64_t lds_off[GCP_MAX_D];
    int64_t lds_total;
    void* partials;  // [gridDim.x][lds_total], FP64 for FP64 factors, else FP32
    double* acc;
    int64_t acc_off[GCP_MAX_D];
    double w[5];
    double eps;
    double* loss_sum;
    int64_t* adam_state;  // fused step: state[0] += 1 here, read by the reduction
};


// Partial-gradient storage: FP64 for FP64 factors, FP32 otherwise.
template <typename FT> struct Partial { using type = float; };
template <> struct Partial<double> { using type = double; };

template <typename T>
__device__ __forceinline__ T pick_weight(const double (&w)[5], int code) {
    // select chain: no dynamic indexing of the kernel-argument block
    double v = w[0];
    v = code == 1 ? w[1] : v;
    v = code == 2 ? w[2] : v;
    v = code == 3 ? w[3] : v;
    v = code == 4 ? w[4] : v;
    return (T)v;
}

// Phase A for direct items: sample c's indices, data value and stratum.
template <int D, typename VT, typename T>
__device__ __forceinline__ void produce(const GradArgs& a, uint64_t iter, int64_t c, uint32_t (&i)[D], T& x,
                                        int& code) {
    const VT* __restrict__ vals = static_cast<const VT*>(a.values);
    if (a.sampler == GCP_SAMPLER_UNIFORM) {
        draw_index<D>(a.seed, a.pid, (uint64_t)c, iter, kPurposeUniform, a.dims.n, i);
        const uint64_t L = linear_key<D>(i, a.dims.n);
        if (a.format == GCP_DENSE) {
            x = (T)vals[L];
        } else {
            const int64_t e = nz_find(a.tab, L);
            x = e >= 0 ? (T)vals[e] : T(0);
        }
        code = GCP_STRATUM_UNIFORM;
    } else if (c < a.p) {
        const uint64_t e = draw_nonzero(a.seed, a.pid, (uint64_t)c, iter, (uint64_t)a.nnz);
#pragma unroll
        for (int k = 0; k < D; ++k) i[k] = a.coo[e * D + k];
        x = (T)vals[e];
        code = a.sampler == GCP_SAMPLER_SEMI_STRATIFIED ? GCP_STRATUM_NZ_CORR : GCP_STRATUM_NZ;
    } else {
        draw_index<D>(a.seed, a.pid, (uint64_t)(c - a.p), iter, kPurposeUniform, a.dims.n, i);
        x = T(0);
        code = GCP_STRATUM_SEMI_ZERO;
    }
}

// Phase B: the wave's 64 samples (one per lane in i/x/code/ylist) are
// evaluated and scattered into the LDS partial (accumulator type LT) for
// privatised modes and into a.acc with device atomics for the others.  Every
// lane of the wave must call this.  Passes
// are taken kBatch at a time so that the row gathers of a batch are all in
// flight before any of them is consumed.
#ifndef GCP_PASS_BATCH
#define GCP_PASS_BATCH 4
#endif
constexpr int kBatch = GCP_PASS_BATCH;

template <int D, typename FT, bool LIST, typename LT = double>
__device__ __forceinline__ void evaluate_and_scatter(const GradArgs& a, LT* __restrict__ lds,
                                                     const uint32_t (&i)[D],
                                                     typename Compute<FT>::type x, int code,
                                                     typename Compute<FT>::type ylist,
                                                     typename Compute<FT>::type& fsum) {
    using T = typename Compute<FT>::type;
    const int lane = threadIdx.x & (kWave - 1);
    const int lps = a.lps;
    const int spw = kWave / lps;
    const int slot = lane / lps;
    const int j = lane & (lps - 1);
    const int r = a.r;
    const T eps = (T)a.eps;
    for (int p0 = 0; p0 < lps; p0 += kBatch) {
        uint32_t ii[kBatch][D];
        int cc[kBatch];
        T xx[kBatch], yy[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int pass = p0 + u < lps ? p0 + u : 0;
            const int src = pass * spw + slot;
#pragma unroll
            for (int k = 0; k < D; ++k) ii[u][k] = __shfl(i[k], src);
            cc[u] = p0 + u < lps ? __shfl(code, src) : -1;
            if constexpr (LIST) yy[u] = __shfl(ylist, src);
            else xx[u] = __shfl(x, src);
        }
        T av[kBatch][D];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const bool col = cc[u] >= 0 && j < r;
#pragma unroll
            for (int k = 0; k < D; ++k)
                av[u][k] = col ? widen(static_cast<const FT*>(a.A[k])[(size_t)ii[u][k] * r + j]) : T(0);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const bool live = cc[u] >= 0;
            const bool col = live && j < r;
            T pre[D], suf[D];
            pre[0] = T(1);
#pragma unroll
            for (int k = 1; k < D; ++k) pre[k] = pre[k - 1] * av[u][k - 1];
            suf[D - 1] = T(1);
#pragma unroll
            for (int k = D - 2; k >= 0; --k) suf[k] = suf[k + 1] * av[u][k + 1];
            T y;
            if constexpr (LIST) {
                y = yy[u];
            } else {
                T m = pre[D - 1] * av[u][D - 1];
                for (int o = lps >> 1; o > 0; o >>= 1) m += __shfl_xor(m, o);
                const T w = pick_weight<T>(a.w, cc[u]);
                T g = loss_g<T>(a.loss, xx[u], m, eps);
                const bool corr = cc[u] == GCP_STRATUM_NZ_CORR;
                if (corr) g -= loss_g<T>(a.loss, T(0), m, eps);
                y = w * g;
                if (a.loss_sum && live && j == 0) {
                    T f = loss_f<T>(a.loss, xx[u], m, eps);
                    if (corr) f -= loss_f<T>(a.loss, T(0), m, eps);
                    fsum += w * f;
                }
            }
            if (col) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double v = (double)(y * pre[k] * suf[k]);
                    if ((a.priv_mask >> k) & 1u)
                        atomicAdd(&lds[a.lds_off[k] + (int64_t)ii[u][k] * r + j], (LT)v);
                    else
                        unsafeAtomicAdd(&a.acc[a.acc_off[k] + (int64_t)ii[u][k] * r + j], v);
                }
            }
        }
    }
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

}  // namespace gcp
