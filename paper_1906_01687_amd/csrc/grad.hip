// grad.hip -- model entries, weighted loss derivatives and the sparse MTTKRP
// of the sampled GCP gradient (Kolda & Hong, Alg. 1-3 loop bodies and final
// MTTKRP loop; eqs. Mdef, Y, mttkrp, Gks).
//
// Work mapping (wave64).  A wave owns a tile of 64 samples.  Phase A: lane l
// produces sample (tile*64 + l) -- its Philox draw, data lookup and stratum --
// so the counter-based generator runs once per sample.  Phase B: the wave
// walks the tile in passes; in each pass a group of `lps` lanes (lps = the
// power of two >= r) takes one sample, lane j of the group owns rank column
// j.  The group gathers A_k(i_k, j) for every mode (one coalesced row read per
// mode), forms the Hadamard product, reduces it over the group with xor
// shuffles to get m_i, evaluates the weighted derivative, and scatters
// ytilde * prod_{k' != k} A_k'(i_k', j) into every mode's FP64 accumulator.
// Leave-one-out products come from prefix/suffix products, so no division.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "device.hpp"

namespace gcp {

struct GradArgs {
    Dims dims;
    int loss;
    int sampler;
    int format;
    int r;
    int lps;
    int64_t S, p, nnz;
    uint64_t seed, pid, iter;
    const void* values;
    const uint32_t* coo;
    NzTable tab;
    const uint32_t* zero_list;  // stratified zeros, [q][D]
    const uint32_t* idx;        // list mode: [S][D]
    const void* ytilde;         // list mode: [S]
    const void* A[GCP_MAX_D];
    double* acc;
    int64_t acc_off[GCP_MAX_D];
    double w[5];
    double eps;
    double* loss_sum;
};

template <typename T>
__device__ __forceinline__ T pick_weight(const GradArgs& a, int code) {
    // select chain: no dynamic indexing of the kernel-argument block
    double w = a.w[0];
    w = code == 1 ? a.w[1] : w;
    w = code == 2 ? a.w[2] : w;
    w = code == 3 ? a.w[3] : w;
    w = code == 4 ? a.w[4] : w;
    return (T)w;
}

// Phase A: sample c's indices, data value and stratum (Alg. 1, 2, 3 draws).
template <int D, typename VT, typename T>
__device__ __forceinline__ void produce(const GradArgs& a, int64_t c, uint32_t (&i)[D], T& x, int& code) {
    const VT* __restrict__ vals = static_cast<const VT*>(a.values);
    if (a.sampler == GCP_SAMPLER_UNIFORM) {
        draw_index<D>(a.seed, a.pid, (uint64_t)c, a.iter, kPurposeUniform, a.dims.n, i);
        const uint64_t L = linear_key<D>(i, a.dims.n);
        if (a.format == GCP_DENSE) {
            x = (T)vals[L];
        } else {
            const int64_t e = nz_find(a.tab, L);
            x = e >= 0 ? (T)vals[e] : T(0);
        }
        code = GCP_STRATUM_UNIFORM;
    } else if (c < a.p) {
        const uint64_t e = draw_nonzero(a.seed, a.pid, (uint64_t)c, a.iter, (uint64_t)a.nnz);
#pragma unroll
        for (int k = 0; k < D; ++k) i[k] = a.coo[e * D + k];
        x = (T)vals[e];
        code = a.sampler == GCP_SAMPLER_SEMI_STRATIFIED ? GCP_STRATUM_NZ_CORR : GCP_STRATUM_NZ;
    } else if (a.sampler == GCP_SAMPLER_SEMI_STRATIFIED) {
        draw_index<D>(a.seed, a.pid, (uint64_t)(c - a.p), a.iter, kPurposeUniform, a.dims.n, i);
        x = T(0);
        code = GCP_STRATUM_SEMI_ZERO;
    } else {
        const int64_t z = c - a.p;
#pragma unroll
        for (int k = 0; k < D; ++k) i[k] = a.zero_list[z * D + k];
        x = T(0);
        code = GCP_STRATUM_ZERO;
    }
}

template <int D, typename FT, typename VT, bool LIST>
__global__ __launch_bounds__(256) void grad_kernel(GradArgs a) {
    using T = typename Compute<FT>::type;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) / kWave;
    const int lps = a.lps;
    const int spw = kWave / lps;
    const int slot = lane / lps;
    const int j = lane & (lps - 1);
    const int r = a.r;
    const T eps = (T)a.eps;
    T fsum = T(0);

    for (int64_t tile = wave; tile * kWave < a.S; tile += nwave) {
        const int64_t c = tile * kWave + lane;
        uint32_t i[D];
#pragma unroll
        for (int k = 0; k < D; ++k) i[k] = 0;
        T x = T(0), ylist = T(0);
        int code = -1;
        if (c < a.S) {
            if constexpr (LIST) {
#pragma unroll
                for (int k = 0; k < D; ++k) i[k] = a.idx[c * D + k];
                ylist = static_cast<const T*>(a.ytilde)[c];
                code = 0;
            } else {
                produce<D, VT, T>(a, c, i, x, code);
            }
        }
        for (int pass = 0; pass < lps; ++pass) {
            const int src = pass * spw + slot;
            uint32_t ii[D];
#pragma unroll
            for (int k = 0; k < D; ++k) ii[k] = __shfl(i[k], src);
            const int cc = __shfl(code, src);
            const bool live = cc >= 0;
            const bool col = live && j < r;
            T av[D];
#pragma unroll
            for (int k = 0; k < D; ++k)
                av[k] = col ? widen(static_cast<const FT*>(a.A[k])[(size_t)ii[k] * r + j]) : T(0);
            T pre[D], suf[D];
            pre[0] = T(1);
#pragma unroll
            for (int k = 1; k < D; ++k) pre[k] = pre[k - 1] * av[k - 1];
            suf[D - 1] = T(1);
#pragma unroll
            for (int k = D - 2; k >= 0; --k) suf[k] = suf[k + 1] * av[k + 1];
            T y;
            if constexpr (LIST) {
                y = __shfl(ylist, src);
            } else {
                T m = pre[D - 1] * av[D - 1];
                for (int o = lps >> 1; o > 0; o >>= 1) m += __shfl_xor(m, o);
                const T xx = __shfl(x, src);
                const T w = pick_weight<T>(a, cc);
                T g = loss_g<T>(a.loss, xx, m, eps);
                const bool corr = cc == GCP_STRATUM_NZ_CORR;
                if (corr) g -= loss_g<T>(a.loss, T(0), m, eps);
                y = w * g;
                if (a.loss_sum && live && j == 0) {
                    T f = loss_f<T>(a.loss, xx, m, eps);
                    if (corr) f -= loss_f<T>(a.loss, T(0), m, eps);
                    fsum += w * f;
                }
            }
            if (col) {
#pragma unroll
                for (int k = 0; k < D; ++k)
                    unsafeAtomicAdd(&a.acc[a.acc_off[k] + (int64_t)ii[k] * r + j], (double)(y * pre[k] * suf[k]));
            }
        }
    }
    if constexpr (!LIST) {
        if (a.loss_sum) {
            double f = (double)fsum;
            for (int o = kWave / 2; o > 0; o >>= 1) f += __shfl_xor(f, o);
            if (lane == 0 && f != 0.0) unsafeAtomicAdd(a.loss_sum, f);
        }
    }
}

// ---------------------------------------------------------------------------
// Unfused derivative: one thread per sample reads its indices, value and
// stratum, forms m_i and writes ytilde_i (gcp_loss_grad).
// ---------------------------------------------------------------------------
struct LossArgs {
    int loss;
    int r;
    int64_t S;
    const uint32_t* idx;
    const void* xval;
    const uint8_t* stratum;
    const void* A[GCP_MAX_D];
    double w[5];
    double eps;
    void* ytilde;
    double* loss_sum;
};

template <int D, typename FT, typename VT>
__global__ __launch_bounds__(256) void loss_grad_kernel(LossArgs a) {
    using T = typename Compute<FT>::type;
    const int r = a.r;
    const T eps = (T)a.eps;
    double fsum = 0.0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < a.S;
         c += (int64_t)gridDim.x * blockDim.x) {
        uint32_t i[D];
#pragma unroll
        for (int k = 0; k < D; ++k) i[k] = a.idx[c * D + k];
        T m = T(0);
        for (int jj = 0; jj < r; ++jj) {
            T prod = T(1);
#pragma unroll
            for (int k = 0; k < D; ++k) prod *= widen(static_cast<const FT*>(a.A[k])[(size_t)i[k] * r + jj]);
            m += prod;
        }
        const int code = a.stratum[c];
        double wd = a.w[0];
        wd = code == 1 ? a.w[1] : wd;
        wd = code == 2 ? a.w[2] : wd;
        wd = code == 3 ? a.w[3] : wd;
        wd = code == 4 ? a.w[4] : wd;
        const T w = (T)wd;
        const T x = (T) static_cast<const VT*>(a.xval)[c];
        const bool corr = code == GCP_STRATUM_NZ_CORR;
        T g = loss_g<T>(a.loss, x, m, eps);
        if (corr) g -= loss_g<T>(a.loss, T(0), m, eps);
        static_cast<T*>(a.ytilde)[c] = w * g;
        if (a.loss_sum) {
            T f = loss_f<T>(a.loss, x, m, eps);
            if (corr) f -= loss_f<T>(a.loss, T(0), m, eps);
            fsum += (double)(w * f);
        }
    }
    if (a.loss_sum) {
        for (int o = kWave / 2; o > 0; o >>= 1) fsum += __shfl_xor(fsum, o);
        if ((threadIdx.x & (kWave - 1)) == 0 && fsum != 0.0) unsafeAtomicAdd(a.loss_sum, fsum);
    }
}

// ---------------------------------------------------------------------------
// Accumulator clear and final rounding into G.
// ---------------------------------------------------------------------------
__global__ void fill_zero_kernel(double* __restrict__ p, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

struct FinArgs {
    int d;
    int accumulate;
    int64_t off[GCP_MAX_D + 1];
    void* G[GCP_MAX_D];
    const double* acc;
};

template <typename GT>
__global__ void finalize_kernel(FinArgs a) {
    const int64_t total = a.off[a.d];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int k = 0;
#pragma unroll
        for (int t = 1; t < GCP_MAX_D; ++t)
            if (t < a.d && e >= a.off[t]) k = t;
        void* gk = a.G[0];
#pragma unroll
        for (int t = 1; t < GCP_MAX_D; ++t)
            if (t == k) gk = a.G[t];
        GT* G = static_cast<GT*>(gk);
        const int64_t local = e - a.off[k];
        double v = a.acc[e];
        if (a.accumulate) v += (double)G[local];
        G[local] = (GT)v;
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static int grid_cap(int64_t n, int threads, int cap) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

static int lanes_per_sample(int64_t r) {
    int l = 1;
    while (l < r) l <<= 1;
    return l;
}

AccLayout acc_layout(const gcp_tensor* X, const gcp_factors* M) {
    AccLayout L{};
    int64_t off = 0;
    for (int k = 0; k < X->d; ++k) {
        L.offset[k] = off;
        off += X->dims[k] * M->rank;
    }
    for (int k = X->d; k <= GCP_MAX_D; ++k) L.offset[k] = off;
    return L;
}

gcp_status launch_fill_zero(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return GCP_OK;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_cap(n, 256, 4096)), dim3(256), 0, s, p, n);
    return check_launch("accumulator clear");
}

gcp_status launch_finalize(const gcp_tensor* X, const gcp_factors* M, const double* acc, const AccLayout& L,
                           void* const* G, int accumulate, hipStream_t s) {
    FinArgs a{};
    a.d = X->d;
    a.accumulate = accumulate;
    for (int k = 0; k <= GCP_MAX_D; ++k) a.off[k] = L.offset[k];
    for (int k = 0; k < X->d; ++k) a.G[k] = G[k];
    a.acc = acc;
    const int64_t n = L.offset[X->d];
    if (n <= 0) return GCP_OK;
    const dim3 g(grid_cap(n, 256, 4096)), b(256);
    if (M->dtype == GCP_F64) hipLaunchKernelGGL(finalize_kernel<double>, g, b, 0, s, a);
    else hipLaunchKernelGGL(finalize_kernel<float>, g, b, 0, s, a);
    return check_launch("gradient rounding");
}

template <int D, bool LIST>
static void grad_launch(const GradArgs& a, int fdtype, int vdtype, hipStream_t s) {
    const int64_t tiles = (a.S + kWave - 1) / kWave;
    const dim3 g(grid_cap(tiles * kWave, 256, 4096)), b(256);
    if (fdtype == GCP_F64) {
        if (vdtype == GCP_F64) hipLaunchKernelGGL((grad_kernel<D, double, double, LIST>), g, b, 0, s, a);
        else hipLaunchKernelGGL((grad_kernel<D, double, float, LIST>), g, b, 0, s, a);
    } else if (fdtype == GCP_F32) {
        if (vdtype == GCP_F64) hipLaunchKernelGGL((grad_kernel<D, float, double, LIST>), g, b, 0, s, a);
        else hipLaunchKernelGGL((grad_kernel<D, float, float, LIST>), g, b, 0, s, a);
    } else {
        if (vdtype == GCP_F64) hipLaunchKernelGGL((grad_kernel<D, bf16_t, double, LIST>), g, b, 0, s, a);
        else hipLaunchKernelGGL((grad_kernel<D, bf16_t, float, LIST>), g, b, 0, s, a);
    }
}

static GradArgs base_args(const gcp_tensor* X, const gcp_factors* M, double* acc, const AccLayout& L) {
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
    for (int k = 0; k < X->d; ++k) {
        a.A[k] = M->A[k];
        a.acc_off[k] = L.offset[k];
    }
    a.acc = acc;
    return a;
}

gcp_status launch_mttkrp_list(const gcp_tensor* X, const gcp_factors* M, const uint32_t* idx, const void* ytilde,
                              int64_t S, double* acc, const AccLayout& L, hipStream_t s) {
    if (S <= 0) return GCP_OK;
    GradArgs a = base_args(X, M, acc, L);
    a.S = S;
    a.idx = idx;
    a.ytilde = ytilde;
    dispatch_d(X->d, [&](auto dc) { grad_launch<decltype(dc)::value, true>(a, M->dtype, GCP_F32, s); });
    return check_launch("gcp_mttkrp");
}

gcp_status launch_fused(gcp_loss loss, const gcp_tensor* X, const gcp_factors* M, const gcp_sampling* cfg,
                        double eps, const uint32_t* zero_list, double* acc, const AccLayout& L,
                        double* loss_sum, hipStream_t s) {
    GradArgs a = base_args(X, M, acc, L);
    a.loss = loss;
    a.sampler = cfg->sampler;
    a.S = cfg->sampler == GCP_SAMPLER_UNIFORM ? cfg->s : cfg->p + cfg->q;
    a.p = cfg->sampler == GCP_SAMPLER_UNIFORM ? 0 : cfg->p;
    a.seed = cfg->seed;
    a.pid = cfg->problem_id;
    a.iter = cfg->iteration;
    a.zero_list = zero_list;
    stratum_weights(X, cfg, a.w);
    a.eps = eps;
    a.loss_sum = loss_sum;
    if (a.S <= 0) return GCP_OK;
    dispatch_d(X->d, [&](auto dc) { grad_launch<decltype(dc)::value, false>(a, M->dtype, X->vdtype, s); });
    return check_launch("gcp_sampled_grad");
}

template <int D>
static void loss_launch(const LossArgs& a, int fdtype, int vdtype, hipStream_t s) {
    const dim3 g(grid_cap(a.S, 256, 4096)), b(256);
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
    a.S = S;
    a.idx = idx;
    a.xval = xval;
    a.stratum = stratum;
    for (int k = 0; k < X->d; ++k) a.A[k] = M->A[k];
    stratum_weights(X, cfg, a.w);
    a.eps = eps;
    a.ytilde = ytilde;
    a.loss_sum = loss_sum;
    dispatch_d(X->d, [&](auto dc) { loss_launch<decltype(dc)::value>(a, M->dtype, X->vdtype, s); });
    return check_launch("gcp_loss_grad");
}

}  // namespace gcp
