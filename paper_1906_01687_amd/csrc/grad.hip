// grad.hip -- model entries, weighted loss derivatives and the sparse MTTKRP
// of the sampled GCP gradient (Kolda & Hong, Alg. 1-3 loop bodies and final
// MTTKRP loop; eqs. Mdef, Y, mttkrp, Gks), plus the reduction of per-block
// partial gradients, optionally fused with the Adam step (Alg. 4).
//
// Work mapping (wave64).  The sample set is cut into work items of 64
// samples; persistent waves take items in turn.  Phase A: lane l produces
// sample l of the item -- its Philox draw, data lookup and stratum -- so the
// counter-based generator runs once per sample.  Phase B: the wave walks the
// item in passes; in each pass a group of `lps` lanes (lps = the power of two
// >= r) takes one sample and lane j of the group owns rank column j.  The
// group gathers A_k(i_k, j) for every mode (one coalesced row read per mode),
// forms the Hadamard product, reduces it over the group with DPP and
// permlane swaps to get m_i, evaluates the weighted derivative, and scatters
// ytilde * prod_{k' != k} A_k'(i_k', j) into every mode's gradient.  Leave-one-
// out products come from prefix/suffix products, so no division.
//
// Scatter.  Device-scope atomics on MI355X sustain only ~170 G element-adds/s
// (measured), far below what plain stores reach, so every mode whose rows fit
// is accumulated privately per workgroup in LDS (FP64 ds_add, or FP32 by
// compare-and-swap), and each workgroup writes its dense partial once with
// ordinary stores (rounded to FP32 for FP32/BF16 factors).  A reduction kernel
// then sums the partials in FP64 in a fixed order (deterministic).  Modes too
// long for LDS fall back to device atomics into an accumulator that the call
// clears first: rows padded to 64-byte sectors, FP32 for FP32/BF16 factors
// unless a row averages many adds, else FP64.
//
// Stratified zeros.  The count kernel (sample.hip) has counted the accepted
// candidates of every 64-candidate chunk and a scan has turned the counts
// into exclusive prefixes.  A zero item here is one chunk: its wave redraws
// the 64 candidates, ranks the accepted ones with a ballot, and keeps those
// whose global rank is below q -- exactly the first q accepted in counter
// order.  If the first batch held fewer than q zeros, the wave that owns the
// last chunk keeps drawing candidates until q are found.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <unordered_set>

#include "common.hpp"
#include "device.hpp"
#include "grad_device.hpp"

namespace gcp {

struct ReduceArgs {
    int d;
    int accumulate;
    int64_t P;
    int64_t off[GCP_MAX_D + 1];
    int64_t blk_start[GCP_MAX_D + 1];  // first workgroup of mode k; [d] = grid size
    uint64_t* bump_counter;
    uint32_t priv_mask;
    int64_t lds_off[GCP_MAX_D];
    int64_t lds_total;
    int64_t nparts;
    const void* partials;
    const double* acc;  // FP32 elements when acc_elem == 4
    int64_t acc_off[GCP_MAX_D];
    int64_t r, acc_stride;
    int acc_elem;
    void* G[GCP_MAX_D];
    // Adam (fused variant)
    void* A;
    float* A_master;
    void* B;
    void* C;
    int64_t* state;
    double alpha, beta1, beta2, eps, lower;
    int eps_mode;
};

// Exclusive prefix of zero chunk `chunk` (wave-uniform): from the scan when
// there is one, else from the per-group sums of the count kernel.
__device__ __forceinline__ uint64_t chunk_prefix(const GradArgs& a, int64_t chunk) {
    if (a.chunk_prefix) return a.chunk_prefix[chunk];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t g = chunk / (kRejThreads / kWave);
    uint64_t s = 0;
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
        const int64_t chunk = item - a.n_direct_items;
        const uint64_t rank = chunk_prefix(a, chunk) + (uint64_t)lane;
        const uint32_t cnt = a.chunk_count[chunk];
        if ((uint32_t)lane < cnt && rank < (uint64_t)a.q) {
            uint32_t i[D];
#pragma unroll
            for (int k = 0; k < D; ++k) i[k] = a.zstage[((int64_t)chunk * kWave + lane) * D + k];
            smp = make_sample<D, T>(a, i, T(0), GCP_STRATUM_ZERO);
        }
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

    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / kWave;
    const int64_t n_items = a.n_direct_items + a.n_zero_items;
    const uint64_t iter = effective_iteration(a.iter, a.iter_ctr);
    T fsum = T(0);

    // the first item's draws and gathers are issued before the LDS clear, so
    // the clear runs under their latency
    Sample<D, T> cur = wave < n_items ? item_sample<D, FT, VT, LIST>(a, iter, wave) : no_sample<D, T>();
    {
        constexpr int per16 = 16 / sizeof(LT);
        uint4* l16 = reinterpret_cast<uint4*>(lds_raw);
        const int64_t n16 = a.lds_total / per16;
        for (int64_t e = threadIdx.x; e < n16; e += nthreads) l16[e] = uint4{0u, 0u, 0u, 0u};
        for (int64_t e = n16 * per16 + threadIdx.x; e < a.lds_total; e += nthreads) lds[e] = LT(0);
    }
    __syncthreads();

    for (int64_t item = wave; item < n_items; item += nwave) {
        // the next item's gathers are in flight while this one is evaluated
        const int64_t next = item + nwave;
        Sample<D, T> nxt = next < n_items ? item_sample<D, FT, VT, LIST>(a, iter, next) : no_sample<D, T>();
        to_rows(a, cur);
        evaluate_and_scatter<D, FT, LIST>(a, lds, stage, cur, fsum);
        if constexpr (!LIST) {
            if (a.n_zero_items > 0 && item == n_items - 1) {
                // the last zero chunk, and the first batch held fewer than q
                // zeros: continue the counter stream (wave-uniform loop)
                uint64_t filled = batch_total(a);
                uint64_t base = (uint64_t)a.ncand;
                for (int64_t t = 0; t < kRejMaxRefillTiles * 16 && filled < (uint64_t)a.q; ++t) {
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
            }
        }
        cur = nxt;
    }
    if constexpr (!LIST) {
        if (a.loss_sum) {
            double f = (double)fsum;
            for (int o = kWave / 2; o > 0; o >>= 1) f += __shfl_xor(f, o);
            if (lane == 0 && f != 0.0) unsafeAtomicAdd(a.loss_sum, f);
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
                const double2 u = reinterpret_cast<const double2*>(lds_raw)[2 * e];
                const double2 w = reinterpret_cast<const double2*>(lds_raw)[2 * e + 1];
                v[0] = (LT)u.x, v[1] = (LT)u.y, v[2] = (LT)w.x, v[3] = (LT)w.y;
            } else {
                const float4 u = reinterpret_cast<const float4*>(lds_raw)[e];
                v[0] = (LT)u.x, v[1] = (LT)u.y, v[2] = (LT)u.z, v[3] = (LT)u.w;
            }
            if constexpr (sizeof(PT) == 4) {
                reinterpret_cast<float4*>(part)[e] = float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
            } else {
                reinterpret_cast<double2*>(part)[2 * e] = double2{(double)v[0], (double)v[1]};
                reinterpret_cast<double2*>(part)[2 * e + 1] = double2{(double)v[2], (double)v[3]};
            }
        }
    } else {
        for (int64_t e = threadIdx.x; e < a.lds_total; e += nthreads) part[e] = (PT)lds[e];
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
struct LossArgs {
    int loss;
    int r;
    int lps;
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

template <int NB, int D, typename FT>
__device__ __forceinline__ void loss_passes(const LossArgs& a, const __amdgpu_buffer_rsrc_t (&rs)[D], int64_t item,
                                            const Sample<D, typename Compute<FT>::type>* stage,
                                            typename Compute<FT>::type& fsum) {
    using T = typename Compute<FT>::type;
    const int lane = threadIdx.x & (kWave - 1);
    const int lps = a.lps, spw = kWave / lps, slot = lane / lps;
    const uint32_t j = (uint32_t)(lane & (lps - 1));
    const bool colj = (int)j < a.r;
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
            prod[u] = T(1);
#pragma unroll
            for (int k = 0; k < D; ++k) prod[u] *= RowLoad<FT>::at(rs[k], qq[u][k] + j);
            prod[u] = colj ? prod[u] : T(0);
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
        constexpr int words = D + (2 + D) * (int)(sizeof(T) / 4);
        constexpr int nb = words * 8 <= 64 ? 8 : (words * 4 <= 64 ? 4 : 2);
        if constexpr (nb == 8) {
            if (a.lps <= 4) loss_passes<4, D, FT>(a, rs, item, stage, fsum);
            else loss_passes<8, D, FT>(a, rs, item, stage, fsum);
        } else {
            loss_passes<nb, D, FT>(a, rs, item, stage, fsum);
        }
    }
    if (a.loss_sum) {
        double f = (double)fsum;
        for (int o = kWave / 2; o > 0; o >>= 1) f += __shfl_xor(f, o);
        if (lane == 0 && f != 0.0) unsafeAtomicAdd(a.loss_sum, f);
    }
}

// ---------------------------------------------------------------------------
// Reduction: G = the sum of the per-workgroup partials (fixed order, FP64)
// for privatised modes and the device accumulator for the others, optionally
// followed by the Adam step on the same elements.  Elements are numbered over
// all modes in mode order (the flat parameter layout).  A privatised mode
// gets workgroups of 64 elements whose 8 waves each sum every 8th partial,
// 16 loads in flight per wave (combined in wave order); an accumulator mode
// gets 512 elements per workgroup, one per thread.  Eight waves of sixteen
// loads took the binary 1000x800x600 step from 32.3 to 30.5 us against
// sixteen waves of eight (measured), with the 1024-partial count workload
// within 0.5 %.
// ---------------------------------------------------------------------------
constexpr int kRedWaves = 8;
constexpr int kRedThreads = kRedWaves * kWave;
#ifndef GCP_REDUCE_UNROLL
#define GCP_REDUCE_UNROLL 16
#endif
#ifndef GCP_REDUCE_PREFETCH
#define GCP_REDUCE_PREFETCH 1
#endif

template <typename GT, int ADAM>
__device__ __forceinline__ void finish_element(const ReduceArgs& a, int k, int64_t local, double g, double bc1d,
                                               double bc2d, bool have, GT pb, GT pc, GT pa, float pm) {
    const int64_t e = a.off[k] + local;
    void* gk = a.G[0];
#pragma unroll
    for (int q = 1; q < GCP_MAX_D; ++q)
        if (q == k) gk = a.G[q];
    if (gk) {
        GT* Gp = static_cast<GT*>(gk);
        double v = g;
        if (a.accumulate) v += (double)Gp[local];
        Gp[local] = (GT)v;
    }
    if constexpr (ADAM != 0) {
        using T = GT;  // moment type: double for F64 factors, float otherwise
        T* B = static_cast<T*>(a.B);
        T* C = static_cast<T*>(a.C);
        if (!have) {
            pb = B[e];
            pc = C[e];
            if constexpr (ADAM == 2) pm = a.A_master[e];
            else pa = static_cast<const T*>(a.A)[e];
        }
        const T gt = (T)g;
        const T b1 = (T)a.beta1, b2 = (T)a.beta2;
        const T omb1 = (T)(1.0 - a.beta1), omb2 = (T)(1.0 - a.beta2);
        const T bc1 = (T)bc1d, bc2 = (T)bc2d;
        const T bm = b1 * pb + omb1 * gt;
        const T cm = b2 * pc + omb2 * gt * gt;
        B[e] = bm;
        C[e] = cm;
        const T bhat = bm / bc1, chat = cm / bc2;
        const T den = a.eps_mode == GCP_EPS_INSIDE_SQRT ? sqrt(chat + (T)a.eps) : sqrt(chat) + (T)a.eps;
        const T step = (T)a.alpha * bhat / den;
        if constexpr (ADAM == 2) {
            float v = pm - (float)step;
            v = v < (float)a.lower ? (float)a.lower : v;
            a.A_master[e] = v;
            static_cast<bf16_t*>(a.A)[e] = to_bf16(v);
        } else {
            T v = pa - step;
            static_cast<T*>(a.A)[e] = v < (T)a.lower ? (T)a.lower : v;
        }
    }
}

template <typename GT, int ADAM>
__global__ __launch_bounds__(kRedThreads) void reduce_kernel(ReduceArgs a) {
    __shared__ double wave_sum[kRedWaves][kWave];
    __shared__ int64_t t_shared;
    __shared__ double bc_shared[2];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    int k = 0;
#pragma unroll
    for (int q = 1; q < GCP_MAX_D; ++q)
        if (q < a.d && (int64_t)blockIdx.x >= a.blk_start[q]) k = q;
    const int64_t lb = (int64_t)blockIdx.x - a.blk_start[k];
    const int64_t nk = a.off[k + 1] - a.off[k];
    const bool priv = (a.priv_mask >> k) & 1u;
    // every earlier kernel of the call has read the iteration counter
    if (a.bump_counter && blockIdx.x == 0 && threadIdx.x == 0) a.bump_counter[0] += 1;
    if (ADAM && threadIdx.x == 0) {
        const int64_t t = a.state[0];  // already advanced by the gradient kernel
        t_shared = t;
        bc_shared[0] = 1.0 - pow(a.beta1, (double)t);
        bc_shared[1] = 1.0 - pow(a.beta2, (double)t);
    }
    if (priv) {
        const int64_t local = lb * kWave + lane;
        const bool in = local < nk;
        // wave 0 fetches the Adam operands of its elements before the partials,
        // so their latency overlaps the partial reads
        GT pb = GT(0), pc = GT(0), pa = GT(0);
        float pm = 0.f;
        if (ADAM && GCP_REDUCE_PREFETCH && wv == 0 && in) {
            const int64_t e = a.off[k] + local;
            pb = static_cast<const GT*>(a.B)[e];
            pc = static_cast<const GT*>(a.C)[e];
            if constexpr (ADAM == 2) pm = a.A_master[e];
            else pa = static_cast<const GT*>(a.A)[e];
        }
        double s = 0.0;
        if (in) {
            // U independent partial sums keep U loads in flight; they are
            // combined in a fixed order, so the result does not depend on timing
            const int64_t pe = a.lds_off[k] + local;
            const GT* __restrict__ parts = static_cast<const GT*>(a.partials);  // partial type = gradient type
            constexpr int U = GCP_REDUCE_UNROLL;
            double acc16[U];
#pragma unroll
            for (int u = 0; u < U; ++u) acc16[u] = 0.0;
            // full batches of U loads, then at most one batch that re-reads the
            // last partial past the end and drops those values (issued together,
            // without a branch between the loads); the wave index is made scalar so
            // the partial offsets are scalar arithmetic
            const int64_t wvu = __builtin_amdgcn_readfirstlane(wv);
            int64_t b = wvu;
            for (; b + (U - 1) * kRedWaves < a.nparts; b += U * kRedWaves) {
                GT v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = parts[(b + u * kRedWaves) * a.lds_total + pe];
#pragma unroll
                for (int u = 0; u < U; ++u) acc16[u] += (double)v[u];
            }
            if (b < a.nparts) {
                const int64_t last = a.nparts - 1;
                GT v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t bu = b + u * kRedWaves;
                    v[u] = parts[(bu < last ? bu : last) * a.lds_total + pe];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) acc16[u] += b + u * kRedWaves < a.nparts ? (double)v[u] : 0.0;
            }
#pragma unroll
            for (int w = U / 2; w > 0; w >>= 1)
#pragma unroll
                for (int u = 0; u < w; ++u) acc16[u] += acc16[u + w];
            s = acc16[0];
        }
        wave_sum[wv][lane] = s;
        __syncthreads();
        if (wv == 0 && in) {
            double g = 0.0;
#pragma unroll
            for (int w = 0; w < kRedWaves; ++w) g += wave_sum[w][lane];
            finish_element<GT, ADAM>(a, k, local, g, ADAM ? bc_shared[0] : 1.0, ADAM ? bc_shared[1] : 1.0,
                                     GCP_REDUCE_PREFETCH != 0, pb, pc, pa, pm);
        }
    } else {
        __syncthreads();
        const int64_t local = lb * kRedThreads + threadIdx.x;
        if (local < nk) {
            const int64_t e = a.acc_off[k] + (a.acc_stride == a.r ? local
                                                                   : local / a.r * a.acc_stride + local % a.r);
            const double g = a.acc_elem == 4 ? (double)reinterpret_cast<const float*>(a.acc)[e] : a.acc[e];
            finish_element<GT, ADAM>(a, k, local, g, ADAM ? bc_shared[0] : 1.0, ADAM ? bc_shared[1] : 1.0, false,
                                     GT(0), GT(0), GT(0), 0.f);
        }
    }
}

__global__ void fill_zero_kernel(double* __restrict__ p, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int grid_cap(int64_t n, int threads, int cap) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// Lets a kernel take up to 160 KB of dynamic LDS (set once per kernel).
static void allow_full_lds(const void* kernel) {
    static std::mutex mu;
    static std::unordered_set<const void*> done;
    std::lock_guard<std::mutex> lk(mu);
    if (done.insert(kernel).second)
        (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

static int lanes_per_sample(int64_t r) {
    int l = 1;
    while (l < r) l <<= 1;
    return l;
}

gcp_status launch_fill_zero(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return GCP_OK;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_cap(n, 256, 4096)), dim3(256), 0, s, p, n);
    return check_launch("accumulator clear");
}

ScatterPlan plan_scatter(const gcp_tensor* X, const gcp_factors* M, int64_t n_items) {
    ScatterPlan pl{};
    pl.d = X->d;
    const int64_t r = M->rank;
    // flat element offsets (mode order)
    int64_t off = 0;
    for (int k = 0; k < X->d; ++k) {
        pl.off[k] = off;
        off += X->dims[k] * r;
    }
    for (int k = X->d; k <= GCP_MAX_D; ++k) pl.off[k] = off;
    pl.P = off;
    // privatise the shortest modes first while their partials fit in LDS: in
    // FP64, or for FP32/BF16 factors in FP32 when that holds more of the
    // gradient (FP32 partials are added with compare-and-swap)
    int order[GCP_MAX_D];
    for (int k = 0; k < X->d; ++k) order[k] = k;
    for (int a = 0; a < X->d; ++a)
        for (int b = a + 1; b < X->d; ++b)
            if (X->dims[order[b]] < X->dims[order[a]]) {
                const int t = order[a];
                order[a] = order[b];
                order[b] = t;
            }
    auto privatise = [&](int elem, uint32_t* mask, int64_t* offs) {
        const int64_t budget = kLdsBudgetBytes / elem;
        int64_t lds = 0;
        *mask = 0;
        for (int a = 0; a < X->d; ++a) {
            const int k = order[a];
            const int64_t n = X->dims[k] * r;
            if (lds + n <= budget) {
                *mask |= 1u << k;
                offs[k] = lds;
                lds += n;
            }
        }
        return lds;
    };
    int64_t offs64[GCP_MAX_D] = {0}, offs32[GCP_MAX_D] = {0};
    uint32_t mask64 = 0, mask32 = 0;
    const int64_t n64 = privatise(8, &mask64, offs64);
    const int64_t n32 = M->dtype == GCP_F64 ? 0 : privatise(4, &mask32, offs32);
    const bool use32 = n32 > n64;
    pl.priv_mask = use32 ? mask32 : mask64;
    pl.lds_elem = use32 ? 4 : 8;
    const int64_t lds = use32 ? n32 : n64;
    for (int k = 0; k < X->d; ++k) pl.lds_off[k] = use32 ? offs32[k] : offs64[k];
    // device accumulator of the other modes.  A device atomic costs about one
    // L2 operation per 64-byte sector its row touches (measured: 10 FP32
    // columns at a 40-byte stride take 1.6x the time of the same adds with rows
    // padded to 64 bytes), so rows are padded to a power of two up to 64 bytes
    // and to a multiple of 64 beyond.  FP32 and BF16 factors accumulate in FP32
    // while a mode's rows average at most kAcc32MaxAdds adds per element (the
    // FP32 sum then stays well inside the FP32 gradient's tolerance), else FP64.
    const int64_t samples = n_items * kWave;
    bool acc32 = M->dtype != GCP_F64;
    for (int k = 0; k < X->d; ++k)
        if (!((pl.priv_mask >> k) & 1u) && samples > kAcc32MaxAdds * X->dims[k]) acc32 = false;
    pl.acc_elem = acc32 ? 4 : 8;
    const int64_t row_bytes = r * pl.acc_elem;
    int64_t pad_bytes = row_bytes <= 64 ? 4 : (row_bytes + 63) / 64 * 64;
    while (pad_bytes < row_bytes) pad_bytes <<= 1;
    int64_t stride = pad_bytes / pl.acc_elem;
    // the kernel's row offsets are 32-bit
    for (int k = 0; k < X->d; ++k)
        if (!((pl.priv_mask >> k) & 1u) && X->dims[k] * stride > (int64_t)UINT32_MAX) stride = r;
    pl.acc_stride = (uint32_t)stride;
    // q = i r < 2^32 (a factor block is below 4 GiB), so umulhi(q, ceil(2^32 / r))
    // is exactly i: the product is i 2^32 + i e with e = r ceil(2^32 / r) - 2^32 < r
    pl.acc_magic = stride != r ? (uint32_t)(((1ull << 32) + (uint64_t)r - 1) / (uint64_t)r) : 0u;
    int64_t acc = 0;
    for (int k = 0; k < X->d; ++k)
        if (!((pl.priv_mask >> k) & 1u)) {
            pl.acc_off[k] = acc;
            acc += X->dims[k] * stride;
        }
    pl.lds_total = lds;
    pl.acc_total = acc;
    // launch shape: big LDS footprints get one 1024-thread workgroup per CU
    const int64_t lds_bytes = (lds * pl.lds_elem + 15) / 16 * 16;
    pl.threads = lds_bytes > 40 * 1024 ? 1024 : 512;
    // per-wave sample records for phase B when they fit beside the partial
    const int64_t stage_bytes = (int64_t)pl.threads * stage_record_bytes(X->d, M->dtype);
    if (lds_bytes + stage_bytes <= kLdsLimitBytes) {
        pl.stage_off = (uint32_t)lds_bytes;
        pl.shm_bytes = lds_bytes + stage_bytes;
    } else {
        pl.stage_off = kNoStage;
        pl.shm_bytes = lds_bytes;
    }
    int per_cu = pl.shm_bytes > 0 ? (int)(kLdsLimitBytes / (pl.shm_bytes + 1024)) : 4;
    const int max_per_cu = 2048 / pl.threads;
    if (per_cu > max_per_cu) per_cu = max_per_cu;
    if (per_cu < 1) per_cu = 1;
    const int64_t waves_per_block = pl.threads / kWave;
    int64_t blocks = (int64_t)device_cu_count() * per_cu;
    const int64_t need = (n_items + waves_per_block - 1) / waves_per_block;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    pl.blocks = blocks;
    return pl;
}

size_t scatter_partials_bytes(const ScatterPlan& pl, int fdtype) {
    return (size_t)(pl.blocks * pl.lds_total) * (fdtype == GCP_F64 ? 8u : 4u);
}

template <int D, bool LIST>
static void grad_launch(const GradArgs& a, const ScatterPlan& pl, int fdtype, int vdtype, hipStream_t s,
                        hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr) {
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

static GradArgs base_args(const gcp_tensor* X, const gcp_factors* M, const ScatterPlan& pl, double* acc,
                          void* partials) {
    GradArgs a{};
    for (int k = 0; k < X->d; ++k) a.dims.n[k] = X->dims[k];
    a.format = X->format;
    a.r = (int)M->rank;
    a.lps = lanes_per_sample(M->rank);
    a.nnz = X->nnz;
    a.values = X->values;
    a.coo = X->coo_idx;
    if (X->nz_table && X->nz_slots > 0) {
        a.tab.keys = static_cast<const uint64_t*>(X->nz_table);
        a.tab.pos = reinterpret_cast<const uint32_t*>(static_cast<const char*>(X->nz_table) + 8 * X->nz_slots);
        a.tab.mask = (uint64_t)X->nz_slots - 1;
    }
    a.tab.bitmap = X->nz_bitmap;
    for (int k = 0; k < X->d; ++k) {
        a.A[k] = M->A[k];
        a.lds_off[k] = pl.lds_off[k];
        a.acc_off[k] = pl.acc_off[k];
    }
    a.acc_stride = pl.acc_stride;
    a.acc_magic = pl.acc_magic;
    a.acc32 = pl.acc_elem == 4;
    a.priv_mask = pl.priv_mask;
    a.lds_total = pl.lds_total;
    a.stage_off = pl.stage_off;
    a.weights = X->weights;
    a.w_zero = zero_weight(X);
    a.kz = 1.0;
    a.acc = acc;
    a.partials = partials;
    return a;
}

gcp_status launch_grad_list(const gcp_tensor* X, const gcp_factors* M, const uint32_t* idx, const void* ytilde,
                            int64_t S, const ScatterPlan& pl, double* acc, void* partials, hipStream_t s) {
    GradArgs a = base_args(X, M, pl, acc, partials);
    a.n_direct = S;
    a.n_direct_items = (S + kWave - 1) / kWave;
    a.idx = idx;
    a.ytilde = ytilde;
    dispatch_d(X->d, [&](auto dc) { grad_launch<decltype(dc)::value, true>(a, pl, M->dtype, GCP_F32, s); });
    return check_launch("gcp_mttkrp");
}

int64_t fused_items(const gcp_tensor* X, const gcp_sampling* cfg, int64_t ncand) {
    if (cfg->sampler == GCP_SAMPLER_UNIFORM) return (cfg->s + kWave - 1) / kWave;
    if (cfg->sampler == GCP_SAMPLER_FULL) return (full_count(X) + kWave - 1) / kWave;
    if (cfg->sampler == GCP_SAMPLER_SEMI_STRATIFIED) return (cfg->p + cfg->q + kWave - 1) / kWave;
    const int64_t zero_items = cfg->q > 0 ? (ncand + kWave - 1) / kWave : 0;
    return (cfg->p + kWave - 1) / kWave + zero_items;
}

gcp_status launch_grad_fused(gcp_loss loss, const gcp_tensor* X, const gcp_factors* M, const gcp_sampling* cfg,
                             double eps, const ScatterPlan& pl, int64_t ncand, const RejScratch* rs,
                             bool scanned, double* acc, void* partials, double* loss_sum, int64_t* adam_state,
                             hipEvent_t ev_start, hipEvent_t ev_stop, hipStream_t s) {
    GradArgs a = base_args(X, M, pl, acc, partials);
    a.loss = loss;
    a.sampler = cfg->sampler;
    a.seed = cfg->seed;
    a.pid = cfg->problem_id;
    a.iter = cfg->iteration;
    a.iter_ctr = cfg->iteration_counter;
    stratum_weights(X, cfg, a.w);
    a.kz = corr_zero_weight(X, cfg);
    a.eps = eps;
    a.loss_sum = loss_sum;
    a.adam_state = adam_state;
    if (cfg->sampler == GCP_SAMPLER_UNIFORM || cfg->sampler == GCP_SAMPLER_FULL) {
        a.n_direct = cfg->sampler == GCP_SAMPLER_FULL ? full_count(X) : cfg->s;
        a.p = 0;
    } else if (cfg->sampler == GCP_SAMPLER_SEMI_STRATIFIED) {
        a.n_direct = cfg->p + cfg->q;
        a.p = cfg->p;
    } else {
        a.n_direct = cfg->p;
        a.p = cfg->p;
        a.q = cfg->q;
        a.ncand = ncand;
        if (rs && cfg->q > 0) {
            a.chunk_count = rs->chunk_count;
            a.group_sum = rs->group_sum;
            a.zstage = rs->zstage;
            a.ngroups = rs->ngroups;
            a.chunk_prefix = scanned ? rs->chunk_prefix : nullptr;
            a.n_zero_items = rs->nchunks;
        }
    }
    a.n_direct_items = (a.n_direct + kWave - 1) / kWave;
    // with nothing sampled the single workgroup still publishes a zero partial
    dispatch_d(X->d, [&](auto dc) {
        grad_launch<decltype(dc)::value, false>(a, pl, M->dtype, X->vdtype, s, ev_start, ev_stop);
    });
    return check_launch("gcp_sampled_grad");
}

gcp_status launch_reduce(const gcp_factors* M, const ScatterPlan& pl, const double* acc, const void* partials,
                         void* const* G, int accumulate, const AdamParams* adam, uint64_t* bump_counter,
                         hipStream_t s) {
    ReduceArgs a{};
    a.bump_counter = bump_counter;
    a.d = pl.d;
    a.P = pl.P;
    for (int k = 0; k <= GCP_MAX_D; ++k) a.off[k] = pl.off[k];
    for (int k = 0; k < pl.d; ++k) {
        a.lds_off[k] = pl.lds_off[k];
        a.acc_off[k] = pl.acc_off[k];
        a.G[k] = G ? G[k] : nullptr;
    }
    a.r = M->rank;
    a.acc_stride = pl.acc_stride;
    a.acc_elem = pl.acc_elem;
    a.priv_mask = pl.priv_mask;
    a.lds_total = pl.lds_total;
    a.nparts = pl.blocks;
    a.partials = partials;
    a.acc = acc;
    a.accumulate = accumulate;
    if (adam) {
        a.A = adam->A;
        a.A_master = adam->A_master;
        a.B = adam->B;
        a.C = adam->C;
        a.state = adam->state;
        a.alpha = adam->alpha;
        a.beta1 = adam->beta1;
        a.beta2 = adam->beta2;
        a.eps = adam->eps;
        a.lower = adam->lower;
        a.eps_mode = adam->eps_mode;
    }
    if (pl.P <= 0) return launch_bump_counter(bump_counter, s);
    int64_t nb = 0;
    for (int k = 0; k < pl.d; ++k) {
        a.blk_start[k] = nb;
        const int64_t nk = pl.off[k + 1] - pl.off[k];
        nb += ((pl.priv_mask >> k) & 1u) ? (nk + kWave - 1) / kWave : (nk + kRedThreads - 1) / kRedThreads;
    }
    for (int k = pl.d; k <= GCP_MAX_D; ++k) a.blk_start[k] = nb;
    const dim3 g((unsigned)nb), b(kRedThreads);
    const bool f64 = M->dtype == GCP_F64;
    if (!adam) {
        if (f64) hipLaunchKernelGGL((reduce_kernel<double, 0>), g, b, 0, s, a);
        else hipLaunchKernelGGL((reduce_kernel<float, 0>), g, b, 0, s, a);
    } else if (f64) {
        hipLaunchKernelGGL((reduce_kernel<double, 1>), g, b, 0, s, a);
    } else if (M->dtype == GCP_F32) {
        hipLaunchKernelGGL((reduce_kernel<float, 1>), g, b, 0, s, a);
    } else {
        hipLaunchKernelGGL((reduce_kernel<float, 2>), g, b, 0, s, a);
    }
    return check_launch("gradient reduction");
}

template <int D>
static void loss_launch(const LossArgs& a, int fdtype, int vdtype, hipStream_t s) {
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

gcp_status launch_loss_grad(gcp_loss loss, const gcp_tensor* X, const gcp_sampling* cfg, const gcp_factors* M,
                            const uint32_t* idx, const void* xval, const uint8_t* stratum, int64_t S,
                            double eps, void* ytilde, double* loss_sum, hipStream_t s) {
    if (S <= 0) return GCP_OK;
    LossArgs a{};
    a.loss = loss;
    a.r = (int)M->rank;
    a.lps = lanes_per_sample(M->rank);
    a.S = S;
    for (int k = 0; k < X->d; ++k) a.n[k] = X->dims[k];
    a.idx = idx;
    a.xval = xval;
    a.stratum = stratum;
    for (int k = 0; k < X->d; ++k) a.A[k] = M->A[k];
    stratum_weights(X, cfg, a.w);
    a.kz = corr_zero_weight(X, cfg);
    a.weights = X->weights;
    a.w_zero = zero_weight(X);
    a.format = X->format;
    if (X->nz_table && X->nz_slots > 0) {
        a.tab.keys = static_cast<const uint64_t*>(X->nz_table);
        a.tab.pos = reinterpret_cast<const uint32_t*>(static_cast<const char*>(X->nz_table) + 8 * X->nz_slots);
        a.tab.mask = (uint64_t)X->nz_slots - 1;
    }
    a.eps = eps;
    a.ytilde = ytilde;
    a.loss_sum = loss_sum;
    dispatch_d(X->d, [&](auto dc) { loss_launch<decltype(dc)::value>(a, M->dtype, X->vdtype, s); });
    return check_launch("gcp_loss_grad");
}

}  // namespace gcp
