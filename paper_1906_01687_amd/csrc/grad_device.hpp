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
    int lps;  // lanes per sample: the power of two >= ceil(r / cpl)
    int cpl;  // rank columns per lane: 1, 2 or 4
    int64_t nnz;
    uint64_t seed, pid, iter;
    const uint64_t* iter_ctr;
    const void* values;
    const uint32_t* coo;
    NzTable tab;
    // direct items: samples c in [0, n_direct), 64 per item
    int64_t n_direct, n_direct_items, p;
    // waves take items in the order g -> (g * item_stride) mod n_items (a
    // permutation; 0 or 1: in order), so the costlier nonzero items and the
    // zero items of stratified sampling are spread over all CUs
    uint64_t item_stride;
    // stratified zeros: one item per chunk of 64 rejection candidates
    int64_t n_zero_items, ncand, q, ngroups;
    const uint32_t* chunk_count;
    const uint32_t* group_sum;
    const uint32_t* zstage;
    const uint64_t* chunk_prefix;  // non-NULL when a scan provided the prefixes
    uint32_t* rej_status;          // set to 1 if the refill stops at its cap
    // list mode (gcp_mttkrp): indices and ytilde per sample
    const uint32_t* idx;
    const void* ytilde;
    const void* A[GCP_MAX_D];
    // scatter targets
    uint32_t priv_mask;
    int64_t lds_off[GCP_MAX_D];
    int64_t lds_total;
    // FP64 LDS partial of the single-problem kernel only: the element at
    // byte offset o (row-major order from the partial's start) is kept at
    // lds_swizzle(o, lds_swz_shift, lds_swz_mask); mask 0 is the plain layout
    uint32_t lds_swz_shift, lds_swz_mask;
    void* partials;  // [gridDim.x][lds_total], FP64 for FP64 factors, else FP32
    // device accumulator of the modes not privatised: FP64, or FP32 when
    // acc32; row i of mode k starts at element acc_off[k] + i * acc_stride,
    // and the kernel forms i * acc_stride from q = i * r as
    // umulhi(q, acc_magic) * acc_stride when acc_magic != 0
    double* acc;
    int64_t acc_off[GCP_MAX_D];
    uint32_t acc_stride, acc_magic;
    int acc32;
    double w[5];
    double eps;
    double* loss_sum;
    int64_t* adam_state;  // fused step: state[0] += 1 here, read by the reduction
    // weighted objective (eq. wgcp): entry weights (type of values; NULL: all
    // 1), the weight of entries a COO tensor does not store, and (eta/p) times
    // it, the weight of g(0, m) in a corrected nonzero
    const void* weights;
    double w_zero;
    double kz;
    // byte offset in the dynamic LDS of the per-wave sample records (64 per
    // wave, in wave order), or kNoStage when phase B broadcasts with ds_bpermute
    uint32_t stage_off;
};

constexpr uint32_t kNoStage = 0xFFFFFFFFu;

// XOR swizzle of an LDS partial's byte offsets: the chunk bits selected by
// mask are flipped by the row bits `shift` places above them.  Those row bits
// lie above every bit the mask selects, so the map is its own inverse and
// keeps each element in its row.
__device__ __forceinline__ uint32_t lds_swizzle(uint32_t o, uint32_t shift, uint32_t mask) {
    return o ^ ((o >> shift) & mask);
}


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

// Phase A for direct items: sample c's indices, data value, stratum and entry
// weight ew (eq. wgcp; 1 without weights; the zero strata's w_zero is in
// their stratum weight).
template <int D, typename VT, typename T>
__device__ __forceinline__ void produce(const GradArgs& a, uint64_t iter, int64_t c, uint32_t (&i)[D], T& x,
                                        int& code, T& ew) {
    const VT* __restrict__ vals = static_cast<const VT*>(a.values);
    const VT* __restrict__ wts = static_cast<const VT*>(a.weights);
    ew = T(1);
    if (a.sampler == GCP_SAMPLER_UNIFORM || a.sampler == GCP_SAMPLER_FULL) {
        uint64_t L;
        if (a.sampler == GCP_SAMPLER_FULL) {
            // sample c is entry c
            L = (uint64_t)c;
            unravel<D>(L, a.dims.n, i);
        } else {
            draw_index<D>(a.seed, a.pid, (uint64_t)c, iter, kPurposeUniform, a.dims.n, i);
            L = linear_key<D>(i, a.dims.n);
        }
        if (a.format == GCP_DENSE) {
            x = (T)gld(vals + L);
            if (wts) ew = (T)gld(wts + L);
        } else {
            const int64_t e = nz_lookup(a.tab, L);
            x = e >= 0 ? (T)gld(vals + e) : T(0);
            if (wts) ew = e >= 0 ? (T)gld(wts + e) : (T)a.w_zero;
        }
        code = GCP_STRATUM_UNIFORM;
    } else if (c < a.p) {
        const uint64_t e = draw_nonzero(a.seed, a.pid, (uint64_t)c, iter, (uint64_t)a.nnz);
#pragma unroll
        for (int k = 0; k < D; ++k) i[k] = gld(a.coo + e * D + k);
        x = (T)gld(vals + e);
        if (wts) ew = (T)gld(wts + e);
        code = a.sampler == GCP_SAMPLER_SEMI_STRATIFIED ? GCP_STRATUM_NZ_CORR : GCP_STRATUM_NZ;
    } else {
        draw_index<D>(a.seed, a.pid, (uint64_t)(c - a.p), iter, kPurposeUniform, a.dims.n, i);
        x = T(0);
        code = GCP_STRATUM_SEMI_ZERO;
    }
}

// Add into an LDS partial.  FP64 uses the native LDS atomic.  FP32 goes
// through a compare-and-swap loop on the 32-bit word: on gfx950 the native
// LDS FP32 atomic add takes about 190 cycles per wave instruction whatever the
// address pattern, against 14-27 for this loop and 8-21 for the FP64 atomic
// (measured with 16 waves per CU).  The loop compares bit patterns, so it ends
// also when the word holds a NaN.
__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }

__device__ __forceinline__ void lds_add(float* p, float v) {
    unsigned* w = reinterpret_cast<unsigned*>(p);
    unsigned old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    unsigned assumed;
    do {
        assumed = old;
        old = atomicCAS(w, assumed, __float_as_uint(__uint_as_float(assumed) + v));
    } while (old != assumed);
}

// One sample as phase A hands it to phase B.  Phase A fills q with the raw
// indices i_k, which may still be loads in flight; to_rows() turns them into
// row offsets once they are needed, so a prefetched sample's gathers overlap
// the evaluation of the previous one.
template <int D, typename T>
struct alignas(16) Sample {
    uint32_t q[D];  // i_k from phase A; i_k * r after to_rows()
    T x;            // data value (list mode: ytilde)
    T w;            // stratum weight; sign bit set for a corrected nonzero (g(x,m) - g(0,m)); +0: no sample
};

// The sign bit of a sample's weight marks a corrected nonzero (Sec. 4.3), and
// only +0 marks an empty slot: a corrected nonzero whose entry weight is 0
// (eq. wgcp) has w = -0 and still carries its -kz g(0, m) term.
__device__ __forceinline__ bool corrected(float w) { return (__float_as_uint(w) >> 31) != 0u; }
__device__ __forceinline__ bool corrected(double w) { return __double_as_longlong(w) < 0; }
__device__ __forceinline__ bool carries(float w) { return __float_as_uint(w) != 0u; }
__device__ __forceinline__ bool carries(double w) { return __double_as_longlong(w) != 0; }

template <int D, typename T>
__device__ __forceinline__ Sample<D, T> no_sample() {
    Sample<D, T> s;
#pragma unroll
    for (int k = 0; k < D; ++k) s.q[k] = 0;
    s.x = T(0);
    s.w = T(0);
    return s;
}

template <int D, typename T>
__device__ __forceinline__ Sample<D, T> make_sample(const GradArgs& a, const uint32_t (&i)[D], T x, int code,
                                                    T ew = T(1)) {
    Sample<D, T> s;
#pragma unroll
    for (int k = 0; k < D; ++k) s.q[k] = i[k];
    s.x = x;
    if (code < 0) {
        s.w = T(0);
    } else {
        const T w = pick_weight<T>(a.w, code) * ew;
        s.w = code == GCP_STRATUM_NZ_CORR ? -w : w;
    }
    return s;
}

template <int D, typename T>
__device__ __forceinline__ void to_rows(const GradArgs& a, Sample<D, T>& s) {
#pragma unroll
    for (int k = 0; k < D; ++k) s.q[k] *= (uint32_t)a.r;
}

// Cross-lane helpers.  Broadcasts read another lane with ds_bpermute; group
// sums run on the VALU: DPP quad permutations, half-row and row mirrors within
// 16 lanes, then the gfx950 row-pair (permlane16) and half-wave (permlane32)
// swaps, whose two results add to the sum over both rows or halves.
__device__ __forceinline__ uint32_t bcast(uint32_t v, int addr) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)v);
}
__device__ __forceinline__ float bcast(float v, int addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double bcast(double v, int addr) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = bcast((uint32_t)u, addr), hi = bcast((uint32_t)(u >> 32), addr);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int HALF>
__device__ __forceinline__ float swap_sum(float v) {
    const int b = __float_as_int(v);
    const auto p = HALF == 16 ? __builtin_amdgcn_permlane16_swap(b, b, false, false)
                              : __builtin_amdgcn_permlane32_swap(b, b, false, false);
    return __int_as_float((int)p[0]) + __int_as_float((int)p[1]);
}
template <int HALF>
__device__ __forceinline__ double swap_sum(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
    const auto pl = HALF == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                               : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto ph = HALF == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                               : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const double a = __longlong_as_double((long long)(((uint64_t)(uint32_t)ph[0] << 32) | (uint32_t)pl[0]));
    const double b = __longlong_as_double((long long)(((uint64_t)(uint32_t)ph[1] << 32) | (uint32_t)pl[1]));
    return a + b;
}

// Sum over the aligned group of lps lanes (a power of two); every lane of the
// group gets the same bits.  All 64 lanes must be active.
template <typename T>
__device__ __forceinline__ T group_sum(T m, int lps) {
    if (lps >= 2) m += dpp<0xB1>(m);   // quad_perm [1,0,3,2]
    if (lps >= 4) m += dpp<0x4E>(m);   // quad_perm [2,3,0,1]
    if (lps >= 8) m += dpp<0x141>(m);  // row_half_mirror
    if (lps >= 16) m += dpp<0x140>(m); // row_mirror
    if (lps >= 32) m = swap_sum<16>(m);
    if (lps >= 64) m = swap_sum<32>(m);
    return m;
}

// x / y: IEEE division in FP64; reciprocal (1 ulp) and product in FP32.
__device__ __forceinline__ double quot(double x, double y) { return x / y; }
__device__ __forceinline__ float quot(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }
// 1 / sqrt(y): FP64 from the correctly rounded root; FP32 hardware (1 ulp).
__device__ __forceinline__ double rroot(double y) { return 1.0 / sqrt(y); }
__device__ __forceinline__ float rroot(float y) { return __builtin_amdgcn_rsqf(y); }

// w * g(x, m) for the loss's derivative g (Sec. 1, 4.2 and 5.3).  A corrected
// nonzero of semi-stratified sampling (Sec. 4.3, Alg. 3) carries the sign bit
// and gives |w| g(x, m) - kz g(0, m), with kz = (eta/p) w_zero; unweighted,
// |w| = kz and this is |w| (g(x, m) - g(0, m)), only the part of g that
// depends on x.
template <typename T>
__device__ __forceinline__ T weighted_g(int loss, T x, T m, T w, T eps, T kz) {
    const bool corr = corrected(w);
    const T aw = corr ? -w : w;
    // g = base(m) - t(x, m): the x-free part and the part linear in x
    T base, t;
    if (loss == GCP_LOSS_GAUSSIAN) {
        base = T(2) * m;
        t = T(2) * x;
    } else {
        if (loss == GCP_LOSS_GAMMA) {
            const T u = quot(T(1), m + eps);
            base = u;
            t = x * u * u;
        } else if (loss == GCP_LOSS_BETA_HALF) {
            const T u = rroot(m + eps);
            base = u;
            t = x * u * u * u;
        } else {
            t = quot(x, m + eps);
            base = loss == GCP_LOSS_BERNOULLI_ODDS ? quot(T(1), m + T(1)) : T(1);
        }
    }
    // corrected: (|w| - kz) base - |w| t, exact cancellation when unweighted
    return corr ? (aw - kz) * base - aw * t : aw * (base - t);
}

// The weighted loss term matching weighted_g: w f(x, m), or for a corrected
// nonzero |w| f(x, m) - kz f(0, m), written so that it is exactly
// |w| (f(x, m) - f(0, m)) when unweighted.
template <typename T>
__device__ __forceinline__ T weighted_f(int loss, T x, T m, T w, T eps, T kz) {
    if (!corrected(w)) return w * loss_f<T>(loss, x, m, eps);
    const T aw = -w;
    const T f0 = loss_f<T>(loss, T(0), m, eps);
    return aw * (loss_f<T>(loss, x, m, eps) - f0) + (aw - kz) * f0;
}

// Element of a factor block through a buffer resource (32-bit byte offset).
template <typename FT> struct RowLoad;
template <> struct RowLoad<float> {
    static __device__ __forceinline__ float at(__amdgpu_buffer_rsrc_t rs, uint32_t e) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, e * 4u, 0, 0));
    }
};
template <> struct RowLoad<double> {
    static __device__ __forceinline__ double at(__amdgpu_buffer_rsrc_t rs, uint32_t e) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, e * 8u, 0, 0);
        return __longlong_as_double((long long)(((uint64_t)v[1] << 32) | v[0]));
    }
};
template <> struct RowLoad<bf16_t> {
    static __device__ __forceinline__ float at(__amdgpu_buffer_rsrc_t rs, uint32_t e) {
        return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, e * 2u, 0, 0) << 16);
    }
};

constexpr int kBufferWord3 = 0x00020000;  // raw buffer, 32-bit elements, gfx9 family

// The iteration counter through a buffer load, which is a vector-memory load:
// it stays in flight across a barrier that waits only for LDS operations.
__device__ __forceinline__ uint64_t counter_vmem(const uint64_t* p) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint64_t*>(p), (short)0, 8, kBufferWord3);
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, 0u, 0, 0);
    return ((uint64_t)v[1] << 32) | v[0];
}

// Values that are the same on every lane but that the compiler cannot prove
// uniform (fields of an argument block read from global memory) are moved to
// scalar registers, so buffer descriptors and branches built from them stay
// scalar.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
    const uint32_t lo = uni((uint32_t)(uint64_t)v), hi = uni((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename P>
__device__ __forceinline__ P* uni(P* p) {
    return reinterpret_cast<P*>((uintptr_t)uni((int64_t)(uintptr_t)p));
}

// Per-call constants of phase B: lane layout, buffer descriptors of the
// factor blocks and scatter bases of the lane's columns.  A sample takes a
// group of lps lanes; lane j of the group owns columns j, j + lps, ...,
// j + (cpl - 1) lps, so for every column step the group's lanes touch
// consecutive elements of a row (coalesced gathers, conflict-free LDS adds,
// one sector per row for device atomics).  Bit c of cmask says whether
// column j + c lps exists (< r).
template <int D, typename LT>
struct PhaseB {
    int lps, spw, slot, r, loss;
    uint32_t j, cmask, priv;
    uint32_t swz_shift, swz_mask;
    double kz;
    __amdgpu_buffer_rsrc_t rs[D];
    uint32_t lbase[D];
    void* accj[D];
    uint32_t acc_stride, acc_magic;
    bool acc32;
};

// Passes per batch for CPL columns per lane: as many as keep a batch's
// registers (indices, value, weight and gathered entries) within a budget of
// 48 VGPRs for d <= 3 and 32 beyond (the rest of phase B and the prefetched
// next sample share the 128 a 1024-thread workgroup allows; these budgets
// are the largest that compile without spills), and no more than the passes
// an item has at the smallest lane group the host pairs with CPL (CPL > 1
// only for r > 4, so lps >= 8 / CPL).
template <int D, typename T, int CPL>
constexpr int passes_per_batch() {
    constexpr int words = D + (2 + D * CPL) * (int)(sizeof(T) / 4);
    constexpr int budget = D <= 3 ? 48 : 32;
    constexpr int nb = words * 8 <= budget ? 8 : (words * 4 <= budget ? 4 : (words * 2 <= budget ? 2 : 1));
    constexpr int cap = CPL == 1 ? 8 : (CPL == 2 ? 4 : 2);
    return nb < cap ? nb : cap;
}

template <int NB, int CPL, int D, typename FT, bool LIST, typename LT, bool STAGED, bool SWZ>
__device__ __forceinline__ void pass_batches(const GradArgs& a, const PhaseB<D, LT>& b, LT* __restrict__ lds,
                                             const Sample<D, typename Compute<FT>::type>* stage,
                                             const Sample<D, typename Compute<FT>::type>& smp,
                                             typename Compute<FT>::type& fsum) {
    using T = typename Compute<FT>::type;
    const T eps = (T)a.eps;
    for (int p0 = 0; p0 < b.lps; p0 += NB) {
        uint32_t qq[NB][D];
        T xx[NB], ww[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const bool pass_ok = p0 + u < b.lps;
            const int src = (pass_ok ? p0 + u : 0) * b.spw + b.slot;
            T wv;
            if constexpr (STAGED) {
                // one record per lane group: 16-byte broadcast reads
                const Sample<D, T> rec = stage[src];
#pragma unroll
                for (int k = 0; k < D; ++k) qq[u][k] = rec.q[k];
                xx[u] = rec.x;
                wv = rec.w;
            } else {
#pragma unroll
                for (int k = 0; k < D; ++k) qq[u][k] = bcast(smp.q[k], src << 2);
                xx[u] = bcast(smp.x, src << 2);
                wv = bcast(smp.w, src << 2);
            }
            ww[u] = pass_ok ? wv : T(0);
        }
        T av[NB][D][CPL];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const T v = RowLoad<FT>::at(b.rs[k], qq[u][k] + b.j + (uint32_t)(c * b.lps));
                    av[u][k][c] = ((b.cmask >> c) & 1u) ? v : T(0);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            // leave-one-out products of every column from prefix and suffix products
            T pre[D][CPL], suf[D][CPL];
            T part = T(0);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                pre[0][c] = T(1);
#pragma unroll
                for (int k = 1; k < D; ++k) pre[k][c] = pre[k - 1][c] * av[u][k - 1][c];
                suf[D - 1][c] = T(1);
#pragma unroll
                for (int k = D - 2; k >= 0; --k) suf[k][c] = suf[k + 1][c] * av[u][k + 1][c];
                part += pre[D - 1][c] * av[u][D - 1][c];
            }
            const bool live = carries(ww[u]);
            T y;
            if constexpr (LIST) {
                y = xx[u];
            } else {
                const T m = group_sum(part, b.lps);
                y = weighted_g(b.loss, xx[u], m, ww[u], eps, (T)b.kz);
                if (a.loss_sum && live && b.j == 0) fsum += weighted_f(b.loss, xx[u], m, ww[u], eps, (T)b.kz);
            }
            if (live && b.cmask) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    uint32_t row = qq[u][k];
                    if (!((b.priv >> k) & 1u) && b.acc_magic) row = __umulhi(row, b.acc_magic) * b.acc_stride;
                    // byte offset of the lane's first column in the LDS
                    // partial, and the row's swizzle of the chunk bits
                    const uint32_t lrow = b.lbase[k] + qq[u][k] * (uint32_t)sizeof(LT);
                    const uint32_t hs = SWZ ? (lrow >> b.swz_shift) & b.swz_mask : 0u;
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        if (!((b.cmask >> c) & 1u)) continue;
                        const T v = y * (pre[k][c] * suf[k][c]);
                        const uint32_t cc = (uint32_t)(c * b.lps);
                        if ((b.priv >> k) & 1u)
                            lds_add(reinterpret_cast<LT*>(reinterpret_cast<char*>(lds) +
                                                          ((lrow + cc * (uint32_t)sizeof(LT)) ^ hs)),
                                    (LT)v);
                        else if (b.acc32)
                            gadd(static_cast<float*>(b.accj[k]) + (row + cc), (float)v);
                        else
                            gadd(static_cast<double*>(b.accj[k]) + (row + cc), (double)v);
                    }
                }
            }
        }
    }
}

template <int CPL, int D, typename FT, bool LIST, typename LT, bool STAGED, bool SWZ = false>
__device__ __forceinline__ void run_passes(const GradArgs& a, const PhaseB<D, LT>& b, LT* __restrict__ lds,
                                           const Sample<D, typename Compute<FT>::type>* stage,
                                           const Sample<D, typename Compute<FT>::type>& smp,
                                           typename Compute<FT>::type& fsum) {
    using T = typename Compute<FT>::type;
    constexpr int nb = passes_per_batch<D, T, CPL>();
    if constexpr (CPL == 1 && nb == 8) {
        // lane groups of at most 4 lanes have at most 4 passes per item
        if (b.lps <= 4) pass_batches<4, 1, D, FT, LIST, LT, STAGED, SWZ>(a, b, lds, stage, smp, fsum);
        else pass_batches<8, 1, D, FT, LIST, LT, STAGED, SWZ>(a, b, lds, stage, smp, fsum);
    } else {
        pass_batches<nb, CPL, D, FT, LIST, LT, STAGED, SWZ>(a, b, lds, stage, smp, fsum);
    }
}

// Phase B: the wave's 64 samples (one per lane in smp, rows already formed by
// to_rows) are evaluated and scattered into the LDS partial (accumulator type
// LT) for privatised modes and into a.acc with device atomics for the others.
// With a staging slice (64 records of this wave in LDS), each pass reads its
// sample's record with wide broadcast reads; without one it broadcasts with
// ds_bpermute (about six times the LDS time per word, measured).
// A sample takes a group of lps lanes, lane j holding columns j, j + lps, ..
// of its rows, so one pass covers 64/lps samples; the model entry's column
// sum is taken over the lane's columns, then over the group.  Passes are taken 1 to 8 at a time so that the row gathers of a batch
// are all in flight before any of them is consumed.  Every lane of the wave
// must call this.  SINGLE = false (the batched kernel) fixes the device
// accumulator to FP64 rows of r and the LDS partial to the plain layout, so
// neither the padded-row nor the swizzle arithmetic is generated (in the
// batched kernel, measured on MI355X, the swizzle's address arithmetic cost
// more than its LDS adds gained).
template <int D, typename FT, bool LIST, typename LT = double, bool SINGLE = true>
__device__ __forceinline__ void evaluate_and_scatter(const GradArgs& a, LT* __restrict__ lds,
                                                     Sample<D, typename Compute<FT>::type>* stage,
                                                     const Sample<D, typename Compute<FT>::type>& smp,
                                                     typename Compute<FT>::type& fsum) {
    const int lane = threadIdx.x & (kWave - 1);
    PhaseB<D, LT> b;
    b.lps = uni((int32_t)a.lps);
    b.spw = kWave / b.lps;
    b.slot = lane / b.lps;
    b.j = (uint32_t)(lane & (b.lps - 1));
    const int cpl = uni((int32_t)a.cpl);
    b.r = uni((int32_t)a.r);
    b.cmask = 0;
    for (int c = 0; c < cpl; ++c)
        if ((int)b.j + c * b.lps < b.r) b.cmask |= 1u << c;
    b.loss = uni((int32_t)a.loss);
    b.priv = uni(a.priv_mask);
    b.kz = a.kz;
    char* const acc = reinterpret_cast<char*>(uni(a.acc));
    if constexpr (SINGLE) {
        b.swz_shift = uni(a.lds_swz_shift);
        b.swz_mask = uni(a.lds_swz_mask);
        b.acc32 = uni(a.acc32) != 0;
        b.acc_stride = uni(a.acc_stride);
        b.acc_magic = uni(a.acc_magic);
    } else {
        b.swz_shift = 0;
        b.swz_mask = 0;
        b.acc32 = false;
        b.acc_stride = 0;
        b.acc_magic = 0;
    }
    const int64_t acc_elem = b.acc32 ? 4 : 8;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint64_t bytes = (uint64_t)uni(a.dims.n[k]) * (uint64_t)b.r * sizeof(FT);
        b.rs[k] = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(uni(a.A[k])), (short)0,
                                                    (int)(bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes),
                                                    kBufferWord3);
        b.lbase[k] = (uint32_t)((uni(a.lds_off[k]) + (int64_t)b.j) * (int64_t)sizeof(LT));
        b.accj[k] = acc ? acc + (uni(a.acc_off[k]) + (int64_t)b.j) * acc_elem : nullptr;
    }
    // the swizzle (cpl >= 2 and an FP64 partial only) is a separate code
    // path, so launches without it carry none of its address arithmetic; it
    // is compiled for d <= 3 only (at d = 4 its extra path pushed the kernel
    // into register spills that cost more than it gained)
    constexpr bool can_swz = SINGLE && sizeof(LT) == 8 && D <= 3;
    const bool swz = can_swz && b.swz_mask != 0;
    if (uni(a.stage_off) != kNoStage) {
        // the wave's own slice: ds operations of one wave complete in order, so
        // the reads below see these writes and the next item's writes cannot
        // overtake them
        stage[lane] = smp;
        if (cpl == 1) run_passes<1, D, FT, LIST, LT, true>(a, b, lds, stage, smp, fsum);
        else if (cpl == 2 && swz) run_passes<2, D, FT, LIST, LT, true, can_swz>(a, b, lds, stage, smp, fsum);
        else if (cpl == 2) run_passes<2, D, FT, LIST, LT, true>(a, b, lds, stage, smp, fsum);
        else if (swz) run_passes<4, D, FT, LIST, LT, true, can_swz>(a, b, lds, stage, smp, fsum);
        else run_passes<4, D, FT, LIST, LT, true>(a, b, lds, stage, smp, fsum);
    } else {
        if (cpl == 1) run_passes<1, D, FT, LIST, LT, false>(a, b, lds, stage, smp, fsum);
        else if (cpl == 2 && swz) run_passes<2, D, FT, LIST, LT, false, can_swz>(a, b, lds, stage, smp, fsum);
        else if (cpl == 2) run_passes<2, D, FT, LIST, LT, false>(a, b, lds, stage, smp, fsum);
        else if (swz) run_passes<4, D, FT, LIST, LT, false, can_swz>(a, b, lds, stage, smp, fsum);
        else run_passes<4, D, FT, LIST, LT, false>(a, b, lds, stage, smp, fsum);
    }
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

}  // namespace gcp
