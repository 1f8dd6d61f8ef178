// grad_kernels.hpp -- the fused and list-mode gradient kernel and the unfused
// derivative kernel (Kolda & Hong, Alg. 1-3 loop bodies and final MTTKRP
// loop; eqs. Mdef, Y, mttkrp, Gks), with their launch templates.  Included only
// by inst.hip, which instantiates them for one mode count per object file; the
// work mapping is described at the top of grad.hip.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gcp {

// Exclusive prefix of zero chunk `chunk` (wave-uniform): from the scan when
// there is one, else from the per-group sums of the count kernel.
__device__ __forceinline__ uint64_t chunk_prefix(const GradArgs& a, int64_t chunk) {
    if (a.chunk_prefix) return a.chunk_prefix[chunk];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t g = chunk / (kRejThreads / kWave);
    uint64_t s = 0;
    // up to 8 loads per lane in flight before they are summed
#pragma unroll 8
    for (int64_t b = lane; b < g; b += kWave) s += a.group_sum[b];
    if (lane < chunk - g * (kRejThreads / kWave)) s += a.chunk_count[g * (kRejThreads / kWave) + lane];
    return wave_sum_u64(s);
}

// Accepted candidates in the whole first batch (wave-uniform).
__device__ __forceinline__ uint64_t batch_total(const GradArgs& a) {
    if (a.chunk_prefix) return a.chunk_prefix[a.n_zero_items];
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t s = 0;
    for (int64_t b = lane; b < a.ngroups; b += kWave) s += a.group_sum[b];
    return wave_sum_u64(s);
}

// Phase A of one item: its 64 samples, one per lane (raw indices; the caller
// applies to_rows before evaluating).  Wave-uniform item index.
template <int D, typename FT, typename VT, bool LIST>
__device__ __forceinline__ Sample<D, typename Compute<FT>::type> item_sample(const GradArgs& a, uint64_t iter,
                                                                             int64_t item) {
    using T = typename Compute<FT>::type;
    const int lane = threadIdx.x & (kWave - 1);
    Sample<D, T> smp = no_sample<D, T>();
    if (item < a.n_direct_items) {
        const int64_t c = item * kWave + lane;
        if (c < a.n_direct) {
            uint32_t i[D];
            if constexpr (LIST) {
#pragma unroll
                for (int k = 0; k < D; ++k) i[k] = a.idx[c * D + k];
                smp = make_sample<D, T>(a, i, static_cast<const T*>(a.ytilde)[c], GCP_STRATUM_UNIFORM);
                smp.w = T(1);
            } else {
                T x, ew;
                int code;
                produce<D, VT, T>(a, iter, c, i, x, code, ew);
                smp = make_sample<D, T>(a, i, x, code, ew);
            }
        }
    } else if constexpr (!LIST) {
        // stratified zeros: the accepted candidates of one 64-candidate chunk,
        // staged in counter order by the count kernel
        // the staged indices and the chunk's count do not depend on the
        // prefix, so their loads go out together with the prefix's (a slot
        // past the count holds stale data and is dropped below)
        const int64_t chunk = item - a.n_direct_items;
        uint32_t i[D];
#pragma unroll
        for (int k = 0; k < D; ++k) i[k] = a.zstage[((int64_t)chunk * kWave + lane) * D + k];
        const uint32_t cnt = a.chunk_count[chunk];
        // the earlier chunks accepted at most 64 each, so the rank of this
        // chunk's accepted candidate l is at most 64 chunk + l: a chunk with
        // 64 chunk + 63 < q lies wholly within the first q zeros and needs no
        // prefix (in practice all but the last few chunks)
        const bool all_in = (uint64_t)chunk * kWave + (kWave - 1) < (uint64_t)a.q;
        const uint64_t rank = all_in ? 0 : chunk_prefix(a, chunk) + (uint64_t)lane;
        if ((uint32_t)lane < cnt && (all_in || rank < (uint64_t)a.q))
            smp = make_sample<D, T>(a, i, T(0), GCP_STRATUM_ZERO);
    }
    return smp;
}

template <int D, typename FT, typename VT, bool LIST, typename LT>
__global__ __launch_bounds__(1024) void grad_kernel(GradArgs a) {
    using T = typename Compute<FT>::type;
    extern __shared__ double lds_raw[];
    LT* const lds = reinterpret_cast<LT*>(lds_raw);
    // this wave's 64 sample records (only used when a.stage_off != kNoStage)
    Sample<D, T>* const stage = reinterpret_cast<Sample<D, T>*>(
                                    reinterpret_cast<char*>(lds_raw) + (a.stage_off == kNoStage ? 0u : a.stage_off)) +
                                (threadIdx.x / kWave) * kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nthreads = blockDim.x;
    // nothing in this kernel reads the step count; the reduction after it does
    if (a.adam_state && blockIdx.x == 0 && threadIdx.x == 0) a.adam_state[0] += 1;

    const int64_t wave = uni((int64_t)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave));
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / kWave;
    const int64_t n_items = a.n_direct_items + a.n_zero_items;
    T fsum = T(0);
    const uint64_t stride = a.item_stride;
    const double inv_items = 1.0 / (double)(n_items > 0 ? n_items : 1);
    auto item_at = [&](int64_t g) -> int64_t {
        if (stride <= 1) return g;
        // (g * stride) mod n without a 64-bit division: g, stride < n < 2^32,
        // so the quotient estimate from the double reciprocal is off by at
        // most 2 and the remainder is corrected into [0, n)
        const uint64_t p = (uint64_t)g * stride;
        const uint64_t q = (uint64_t)((double)p * inv_items);
        int64_t r = (int64_t)(p - q * (uint64_t)n_items);
        while (r < 0) r += n_items;
        while (r >= n_items) r -= n_items;
        return r;
    };

    // the device iteration counter is loaded first and used after the
    // barrier below, so its latency overlaps the LDS clear
    const uint64_t ctr = a.iter_ctr ? counter_vmem(a.iter_ctr) : 0;
    // clear the LDS partial first: after this one barrier every wave runs
    // its draws, gathers and scatter at its own pace (a barrier after the
    // draws would hold each wave back to its workgroup's slowest draw)
    {
        constexpr int per16 = 16 / sizeof(LT);
        uint4* l16 = reinterpret_cast<uint4*>(lds_raw);
        const int64_t n16 = a.lds_total / per16;
        for (int64_t e = threadIdx.x; e < n16; e += nthreads) l16[e] = uint4{0u, 0u, 0u, 0u};
        for (int64_t e = n16 * per16 + threadIdx.x; e < a.lds_total; e += nthreads) lds[e] = LT(0);
    }
    __syncthreads();
    const uint64_t iter = a.iter + (uint64_t)uni((int64_t)ctr);
    Sample<D, T> cur = wave < n_items ? item_sample<D, FT, VT, LIST>(a, iter, item_at(wave)) : no_sample<D, T>();

    for (int64_t g = wave; g < n_items; g += nwave) {
        const int64_t item = item_at(g);
        // the next item's gathers are in flight while this one is evaluated
        const int64_t next = g + nwave;
        Sample<D, T> nxt = next < n_items ? item_sample<D, FT, VT, LIST>(a, iter, item_at(next)) : no_sample<D, T>();
        to_rows(a, cur);
        evaluate_and_scatter<D, FT, LIST>(a, lds, stage, cur, fsum);
        if constexpr (!LIST) {
            if (a.n_zero_items > 0 && item == n_items - 1) {
                // the last zero chunk, and the first batch held fewer than q
                // zeros: continue the counter stream (wave-uniform loop)
                uint64_t filled = batch_total(a);
                uint64_t base = (uint64_t)a.ncand;
                for (int64_t t = 0; t < kRejRefillTurns && filled < (uint64_t)a.q; ++t) {
                    const uint64_t jj = base + lane;
                    uint32_t i[D];
                    const bool ok = candidate_accepted<D>(a.dims, a.tab, a.seed, a.pid, iter, jj, i);
                    const uint64_t b2 = __ballot(ok);
                    const uint64_t rk = filled + __popcll(b2 & ((1ull << lane) - 1ull));
                    const int cz = (ok && rk < (uint64_t)a.q) ? GCP_STRATUM_ZERO : -1;
                    Sample<D, T> z = make_sample<D, T>(a, i, T(0), cz);
                    to_rows(a, z);
                    evaluate_and_scatter<D, FT, false>(a, lds, stage, z, fsum);
                    filled += __popcll(b2);
                    base += kWave;
                }
                if (lane == 0 && filled < (uint64_t)a.q) a.rej_status[0] = 1;
            }
        }
        cur = nxt;
    }
    if constexpr (!LIST) {
        if (a.loss_sum) {
            double f = (double)fsum;
            for (int o = kWave / 2; o > 0; o >>= 1) f += __shfl_xor(f, o);
            if (lane == 0 && f != 0.0) gadd(a.loss_sum, f);
        }
    }
    __syncthreads();
    // one dense partial per workgroup, plain stores (FP32 unless the factors are FP64)
    using PT = typename Partial<FT>::type;
    PT* __restrict__ part = static_cast<PT*>(a.partials) + (int64_t)blockIdx.x * a.lds_total;
    if (a.lds_total % 4 == 0) {
        // four elements per step: 16-byte LDS reads, 16-byte (FP32) or 2 x 16-byte (FP64) stores
        for (int64_t e = threadIdx.x; e < a.lds_total / 4; e += nthreads) {
            LT v[4];
            if constexpr (sizeof(LT) == 8) {
                // four elements are 32 bytes, inside one chunk of the swizzle
                const uint32_t o = lds_swizzle((uint32_t)e * 32u, a.lds_swz_shift, a.lds_swz_mask);
                const double2 u = *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(lds_raw) + o);
                const double2 w = *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(lds_raw) + o + 16);
                v[0] = (LT)u.x, v[1] = (LT)u.y, v[2] = (LT)w.x, v[3] = (LT)w.y;
            } else {
                const float4 u = reinterpret_cast<const float4*>(lds_raw)[e];
                v[0] = (LT)u.x, v[1] = (LT)u.y, v[2] = (LT)u.z, v[3] = (LT)u.w;
            }
            if constexpr (sizeof(PT) == 4) {
                // streamed past the L2: the reduction runs on every XCD, so a
                // partial cached in this XCD's L2 would only have to be
                // written back when the kernel ends
                using f32x4 = float __attribute__((ext_vector_type(4)));
                __builtin_nontemporal_store(f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]},
                                            reinterpret_cast<f32x4*>(part) + e);
            } else {
                using f64x2 = double __attribute__((ext_vector_type(2)));
                __builtin_nontemporal_store(f64x2{(double)v[0], (double)v[1]}, reinterpret_cast<f64x2*>(part) + 2 * e);
                __builtin_nontemporal_store(f64x2{(double)v[2], (double)v[3]}, reinterpret_cast<f64x2*>(part) + 2 * e + 1);
            }
        }
    } else {
        for (int64_t e = threadIdx.x; e < a.lds_total; e += nthreads) {
            const uint32_t o = sizeof(LT) == 8 ? lds_swizzle((uint32_t)e * 8u, a.lds_swz_shift, a.lds_swz_mask)
                                               : (uint32_t)e * (uint32_t)sizeof(LT);
            part[e] = (PT) * reinterpret_cast<const LT*>(reinterpret_cast<const char*>(lds_raw) + o);
        }
    }
}

// ---------------------------------------------------------------------------
// Unfused derivative (gcp_loss_grad).  Same lane layout as the fused kernel:
// lane l of a wave reads sample l of its 64-sample item (indices, value,
// stratum) and stores its record in the wave's LDS slice; in each pass a
// group of lps lanes reads one record, gathers the sample's rows (coalesced),
// forms m with a VALU group sum, and lane 0 of the group writes ytilde and
// adds its weighted loss.
// ---------------------------------------------------------------------------
template <int NB, int CPL, int D, typename FT>
__device__ __forceinline__ void loss_passes(const LossArgs& a, const __amdgpu_buffer_rsrc_t (&rs)[D], int64_t item,
                                            const Sample<D, typename Compute<FT>::type>* stage,
                                            typename Compute<FT>::type& fsum) {
    using T = typename Compute<FT>::type;
    const int lane = threadIdx.x & (kWave - 1);
    const int lps = a.lps, spw = kWave / lps, slot = lane / lps;
    const uint32_t j = (uint32_t)(lane & (lps - 1));
    const T eps = (T)a.eps;
    for (int p0 = 0; p0 < lps; p0 += NB) {
        uint32_t qq[NB][D];
        T xx[NB], ww[NB];
        int src[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            src[u] = (p0 + u < lps ? p0 + u : 0) * spw + slot;
            const Sample<D, T> rec = stage[src[u]];   // broadcast read of the group's record
#pragma unroll
            for (int k = 0; k < D; ++k) qq[u][k] = rec.q[k];
            xx[u] = rec.x;
            ww[u] = rec.w;
        }
        T prod[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            T pc[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) pc[c] = T(1);
#pragma unroll
            for (int k = 0; k < D; ++k) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) pc[c] *= RowLoad<FT>::at(rs[k], qq[u][k] + j + (uint32_t)(c * lps));
            }
            prod[u] = T(0);
#pragma unroll
            for (int c = 0; c < CPL; ++c) prod[u] += ((int)j + c * lps < a.r) ? pc[c] : T(0);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const T m = group_sum(prod[u], lps);
            const int64_t cs = item * kWave + src[u];
            if (j == 0 && p0 + u < lps && cs < a.S) {
                static_cast<T*>(a.ytilde)[cs] = weighted_g(a.loss, xx[u], m, ww[u], eps, (T)a.kz);
                if (a.loss_sum) fsum += weighted_f(a.loss, xx[u], m, ww[u], eps, (T)a.kz);
            }
        }
    }
}

template <int D, typename FT, typename VT>
__global__ __launch_bounds__(256) void loss_grad_kernel(LossArgs a) {
    using T = typename Compute<FT>::type;
    const int lane = threadIdx.x & (kWave - 1);
    __amdgpu_buffer_rsrc_t rs[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint64_t bytes = (uint64_t)a.n[k] * (uint64_t)a.r * sizeof(FT);
        rs[k] = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.A[k]), (short)0,
                                                  (int)(bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes),
                                                  kBufferWord3);
    }
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / kWave;
    const int64_t items = (a.S + kWave - 1) / kWave;
    __shared__ Sample<D, T> stage_all[4][kWave];   // 256 threads: 4 waves
    Sample<D, T>* const stage = stage_all[threadIdx.x / kWave];
    T fsum = T(0);
    for (int64_t item = wave; item < items; item += nwave) {
        const int64_t c = item * kWave + lane;
        Sample<D, T> smp = no_sample<D, T>();
        if (c < a.S) {
            uint32_t i[D];
#pragma unroll
            for (int k = 0; k < D; ++k) i[k] = a.idx[c * D + k];
#pragma unroll
            for (int k = 0; k < D; ++k) smp.q[k] = i[k] * (uint32_t)a.r;
            const int code = a.stratum[c];
            smp.x = (T) static_cast<const VT*>(a.xval)[c];
            T wt = pick_weight<T>(a.w, code);
            if (a.weights && code != GCP_STRATUM_ZERO && code != GCP_STRATUM_SEMI_ZERO) {
                // entry weight of a stored entry (or w_zero for an entry not
                // stored); the zero strata's w_zero is in their stratum weight
                const VT* __restrict__ wts = static_cast<const VT*>(a.weights);
                Dims dm;
#pragma unroll
                for (int k = 0; k < D; ++k) dm.n[k] = a.n[k];
                const uint64_t L = linear_key<D>(i, dm.n);
                if (a.format == GCP_DENSE) {
                    wt *= (T)wts[L];
                } else {
                    const int64_t e = nz_find(a.tab, L);
                    wt *= e >= 0 ? (T)wts[e] : (T)a.w_zero;
                }
            }
            smp.w = code == GCP_STRATUM_NZ_CORR ? -wt : wt;
        }
        // this wave's slice; its ds operations complete in order
        stage[lane] = smp;
        if (a.cpl == 1) {
            constexpr int nb = passes_per_batch<D, T, 1>();
            if (nb == 8 && a.lps <= 4) loss_passes<4, 1, D, FT>(a, rs, item, stage, fsum);
            else loss_passes<nb, 1, D, FT>(a, rs, item, stage, fsum);
        } else if (a.cpl == 2) {
            loss_passes<passes_per_batch<D, T, 2>(), 2, D, FT>(a, rs, item, stage, fsum);
        } else {
            loss_passes<passes_per_batch<D, T, 4>(), 4, D, FT>(a, rs, item, stage, fsum);
        }
    }
    if (a.loss_sum) {
        double f = (double)fsum;
        for (int o = kWave / 2; o > 0; o >>= 1) f += __shfl_xor(f, o);
        if (lane == 0 && f != 0.0) gadd(a.loss_sum, f);
    }
}

template <int D, bool LIST>
void grad_launch(const GradArgs& a, const ScatterPlan& pl, int fdtype, int vdtype, hipStream_t s,
                 hipEvent_t ev_start, hipEvent_t ev_stop) {
    const dim3 g((unsigned)pl.blocks), b((unsigned)pl.threads);
    const size_t shm = (size_t)pl.shm_bytes;
    auto go = [&](auto kernel) {
        allow_full_lds(reinterpret_cast<const void*>(kernel));
        if (ev_start || ev_stop)
            hipExtLaunchKernelGGL(kernel, g, b, (std::uint32_t)shm, s, ev_start, ev_stop, 0u, a);
        else
            hipLaunchKernelGGL(kernel, g, b, shm, s, a);
    };
    const bool f32 = pl.lds_elem == 4;
    if (fdtype == GCP_F64) {
        if (vdtype == GCP_F64) go(grad_kernel<D, double, double, LIST, double>);
        else go(grad_kernel<D, double, float, LIST, double>);
    } else if (fdtype == GCP_F32) {
        if (vdtype == GCP_F64) {
            if (f32) go(grad_kernel<D, float, double, LIST, float>);
            else go(grad_kernel<D, float, double, LIST, double>);
        } else {
            if (f32) go(grad_kernel<D, float, float, LIST, float>);
            else go(grad_kernel<D, float, float, LIST, double>);
        }
    } else {
        if (vdtype == GCP_F64) {
            if (f32) go(grad_kernel<D, bf16_t, double, LIST, float>);
            else go(grad_kernel<D, bf16_t, double, LIST, double>);
        } else {
            if (f32) go(grad_kernel<D, bf16_t, float, LIST, float>);
            else go(grad_kernel<D, bf16_t, float, LIST, double>);
        }
    }
}

template <int D>
void loss_launch(const LossArgs& a, int fdtype, int vdtype, hipStream_t s) {
    // 4 waves per workgroup, one 64-sample item per wave and turn
    const int64_t items = (a.S + kWave - 1) / kWave;
    const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((items + 3) / 4, (int64_t)device_cu_count() * 8))),
        b(256);
    if (fdtype == GCP_F64) {
        if (vdtype == GCP_F64) hipLaunchKernelGGL((loss_grad_kernel<D, double, double>), g, b, 0, s, a);
        else hipLaunchKernelGGL((loss_grad_kernel<D, double, float>), g, b, 0, s, a);
    } else if (fdtype == GCP_F32) {
        if (vdtype == GCP_F64) hipLaunchKernelGGL((loss_grad_kernel<D, float, double>), g, b, 0, s, a);
        else hipLaunchKernelGGL((loss_grad_kernel<D, float, float>), g, b, 0, s, a);
    } else {
        if (vdtype == GCP_F64) hipLaunchKernelGGL((loss_grad_kernel<D, bf16_t, double>), g, b, 0, s, a);
        else hipLaunchKernelGGL((loss_grad_kernel<D, bf16_t, float>), g, b, 0, s, a);
    }
}

}  // namespace gcp
