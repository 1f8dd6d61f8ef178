// device.hpp -- device helpers of libgcp (gfx950, wave64).
//
// Philox4x64-10 counter-based draws, randi, the five losses, bf16 storage and
// the nonzero hash probe.  Everything here is __device__ code used by the
// sampling and gradient kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gcp.h"

namespace gcp {

constexpr int kWave = 64;

// Mode sizes passed by value to kernels.
struct Dims {
    int64_t n[GCP_MAX_D];
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 64x64
// -> 128-bit multiplies with a Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
struct Philox4 {
    uint64_t w[4];
};

// High and low words of the 128-bit product a * b from four 32 x 32 + 64
// multiply-adds (v_mad_u64_u32); written out because forming the two halves
// separately costs the compiler extra 32-bit multiplies (307 against 238
// VALU instructions per Philox block on gfx950).
__device__ __forceinline__ void mul128(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
    const uint64_t al = (uint32_t)a, ah = a >> 32, bl = (uint32_t)b, bh = b >> 32;
    const uint64_t t0 = al * bl;
    const uint64_t t1 = al * bh + (t0 >> 32);       // < 2^64: (2^32 - 1)^2 + 2^32 - 1
    const uint64_t t2 = ah * bl + (uint32_t)t1;
    hi = ah * bh + (t1 >> 32) + (t2 >> 32);
    lo = (t2 << 32) | (uint32_t)t0;
}

__device__ __forceinline__ Philox4 philox4x64_10(uint64_t k0, uint64_t k1, uint64_t c0,
                                                 uint64_t c1, uint64_t c2, uint64_t c3) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mul128(M0, c0, hi0, lo0);
        mul128(M1, c2, hi1, lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// randi(n), 0-based: floor(w * n / 2^64) -- unbiased to within n / 2^64.
__device__ __forceinline__ uint64_t randi(uint64_t w, uint64_t n) { return __umul64hi(w, n); }

enum Purpose : uint64_t { kPurposeUniform = 0, kPurposeNonzero = 1, kPurposeCandidate = 2 };

// The D mode indices of draw j: word k of the stream is word k % 4 of block k / 4.
template <int D>
__device__ __forceinline__ void draw_index(uint64_t seed, uint64_t pid, uint64_t j, uint64_t iter,
                                           uint64_t purpose, const int64_t* __restrict__ dims,
                                           uint32_t (&i)[D]) {
#pragma unroll
    for (int b = 0; b < (D + 3) / 4; ++b) {
        const Philox4 r = philox4x64_10(seed, pid, j, iter, purpose, (uint64_t)b);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (4 * b + t < D) i[4 * b + t] = (uint32_t)randi(r.w[t], (uint64_t)dims[4 * b + t]);
    }
}

// The iteration a launch draws with: the host value plus, when given, the
// device-side counter (read once per thread; the counter only changes in a
// later kernel of the same call).
__device__ __forceinline__ uint64_t effective_iteration(uint64_t base, const uint64_t* counter) {
    return counter ? base + *counter : base;
}

// Nonzero pick xi = randi(eta) from word 0 of the purpose-1 stream.
__device__ __forceinline__ uint64_t draw_nonzero(uint64_t seed, uint64_t pid, uint64_t j,
                                                 uint64_t iter, uint64_t nnz) {
    const Philox4 r = philox4x64_10(seed, pid, j, iter, kPurposeNonzero, 0);
    return randi(r.w[0], nnz);
}

template <int D>
__device__ __forceinline__ void unravel(uint64_t L, const int64_t* __restrict__ dims, uint32_t (&i)[D]) {
    // row-major: the last mode varies fastest
#pragma unroll
    for (int k = D - 1; k > 0; --k) {
        const uint64_t n = (uint64_t)dims[k];
        i[k] = (uint32_t)(L % n);
        L /= n;
    }
    i[0] = (uint32_t)L;
}

template <int D>
__device__ __forceinline__ uint64_t linear_key(const uint32_t (&i)[D], const int64_t* __restrict__ dims) {
    uint64_t L = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) L = L * (uint64_t)dims[k] + i[k];
    return L;
}

// ---------------------------------------------------------------------------
// Nonzero hash: open addressing with linear probing.  Slot s holds key+1
// (0 = empty) in keys[s] and the COO position in pos[s].  The mixer is the
// splitmix64 finaliser (Steele, Lea, Flood 2014).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Loads and atomic adds through global-address-space pointers.  A pointer
// read from memory (a field of a problem record in device memory) is generic,
// and a generic (flat) memory instruction counts against the LDS counter as
// well as the vector-memory one, so a later wait for an LDS result would also
// wait for it (a gather in flight, or a device atomic).
template <typename V>
__device__ __forceinline__ V gld(const V* p) {
    return *(const __attribute__((address_space(1))) V*)p;
}
template <typename V>
__device__ __forceinline__ void gadd(V* p, V v) {
    auto g = (__attribute__((address_space(1))) V*)p;
    [[clang::atomic(ignore_denormal_mode)]] {
        (void)__hip_atomic_fetch_add(g, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

struct NzTable {
    const uint64_t* keys;
    const uint32_t* pos;
    uint64_t mask;
    const uint32_t* bitmap;  // optional exact membership bitmap (bit L set iff nonzero)
};

// COO position of linear key L, or -1 if X is zero there.
__device__ __forceinline__ int64_t nz_find(const NzTable& t, uint64_t L) {
    const uint64_t want = L + 1;
    uint64_t h = mix64(L) & t.mask;
    for (uint64_t probe = 0; probe <= t.mask; ++probe) {
        const uint64_t k = gld(t.keys + h);
        if (k == want) return (int64_t)gld(t.pos + h);
        if (k == 0) return -1;
        h = (h + 1) & t.mask;
    }
    return -1;
}

// COO position of linear key L, or -1: the bitmap (when present) answers
// "not stored" with one load, so only stored entries walk the hash.
__device__ __forceinline__ int64_t nz_lookup(const NzTable& t, uint64_t L) {
    if (t.bitmap && !((gld(t.bitmap + (L >> 5)) >> (L & 31)) & 1u)) return -1;
    return nz_find(t, L);
}

// Whether X is nonzero at linear key L: one bitmap load when the bitmap
// exists, else the hash probe sequence.
__device__ __forceinline__ bool nz_member(const NzTable& t, uint64_t L) {
    if (t.bitmap) return (gld(t.bitmap + (L >> 5)) >> (L & 31)) & 1u;
    return nz_find(t, L) >= 0;
}

// Rejection candidate j (purpose 2): its indices, and whether X is zero there.
template <int D>
__device__ __forceinline__ bool candidate_accepted(const Dims& dims, const NzTable& tab, uint64_t seed,
                                                   uint64_t pid, uint64_t iter, uint64_t j, uint32_t (&i)[D]) {
    draw_index<D>(seed, pid, j, iter, kPurposeCandidate, dims.n, i);
    return !nz_member(tab, linear_key<D>(i, dims.n));
}

// ---------------------------------------------------------------------------
// Storage types.  bf16 is kept as raw 16-bit words; gathers widen to float.
// ---------------------------------------------------------------------------
struct bf16_t {
    uint16_t bits;
};

template <typename S> struct Compute { using type = S; };
template <> struct Compute<bf16_t> { using type = float; };

template <typename T> __device__ __forceinline__ T load_as(const T* p) { return *p; }
template <typename T>
__device__ __forceinline__ typename Compute<T>::type widen(T v) { return v; }
template <> __device__ __forceinline__ float widen<bf16_t>(bf16_t v) {
    return __uint_as_float((uint32_t)v.bits << 16);
}

// float -> bf16 with round to nearest, ties to even (NaN stays NaN).
__device__ __forceinline__ bf16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return bf16_t{(uint16_t)((u >> 16) | 0x40)};
    u += 0x7FFFu + ((u >> 16) & 1u);
    return bf16_t{(uint16_t)(u >> 16)};
}

// ---------------------------------------------------------------------------
// Losses: g = df/dm and f, with eps where the paper writes log m or x/m.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T loss_g(int loss, T x, T m, T eps) {
    if (loss == GCP_LOSS_GAUSSIAN) return T(2) * (m - x);
    if (loss == GCP_LOSS_BERNOULLI_ODDS) return T(1) / (m + T(1)) - x / (m + eps);
    if (loss == GCP_LOSS_GAMMA) return T(1) / (m + eps) - x / ((m + eps) * (m + eps));
    if (loss == GCP_LOSS_BETA_HALF) return T(1) / sqrt(m + eps) - x / ((m + eps) * sqrt(m + eps));
    return T(1) - x / (m + eps);
}

template <typename T>
__device__ __forceinline__ T loss_f(int loss, T x, T m, T eps) {
    if (loss == GCP_LOSS_GAUSSIAN) return (x - m) * (x - m);
    if (loss == GCP_LOSS_BERNOULLI_ODDS) return log(m + T(1)) - x * log(m + eps);
    if (loss == GCP_LOSS_GAMMA) return x / (m + eps) + log(m + eps);
    if (loss == GCP_LOSS_BETA_HALF) return T(2) * sqrt(m + eps) + T(2) * x / sqrt(m + eps);
    return m - x * log(m + eps);
}

// Stratum weights w[code] and whether the code subtracts g(0, m).
struct Weights {
    double w[5];
};

__device__ __forceinline__ bool stratum_corrected(int code) { return code == GCP_STRATUM_NZ_CORR; }

// ---------------------------------------------------------------------------
// Wave helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

}  // namespace gcp
