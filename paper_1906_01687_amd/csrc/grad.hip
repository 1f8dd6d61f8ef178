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
#include "kernels.hpp"

namespace gcp {

struct ReduceArgs {
    int d;
    int accumulate;
    int64_t P;
    int64_t off[GCP_MAX_D + 1];
    int64_t blk_start[GCP_MAX_D + 1];  // first workgroup of mode k; [d] = grid size
    uint64_t* bump_counter;
    const double* scale;  // device scalar multiplying every gradient element (nullable)
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
// within 0.5 %; 24 and 32 loads in flight (one round of loads for the 206
// partials of the binary step) measured 29.5 and 30.7 us against 29.2.
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
    if (a.scale) g *= *a.scale;
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

void allow_full_lds(const void* kernel) {
    static std::mutex mu;
    static std::unordered_set<const void*> done;
    std::lock_guard<std::mutex> lk(mu);
    if (done.insert(kernel).second)
        (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

std::atomic<int> g_cols_per_lane{0};

// Stride of the item permutation g -> g * stride mod n: with stratified or
// semi-stratified sampling the nonzero items (a draw and two dependent
// gathers each) come first and the zero items (staged by the count kernel, or
// a draw with no data) after, so in order they would fill whole CUs with one
// kind; a stride near n / phi coprime to n deals both kinds evenly over the
// workgroups.  Identity otherwise, or when the products could overflow 64 bits.
static uint64_t item_stride(int64_t n, bool mixed) {
    if (!mixed || n < 3 || n >= ((int64_t)1 << 32)) return 1;
    auto gcd = [](uint64_t x, uint64_t y) {
        while (y) {
            const uint64_t t = x % y;
            x = y;
            y = t;
        }
        return x;
    };
    uint64_t s = (uint64_t)((double)n * 0.6180339887498949);
    if (s < 2) s = 2;
    while (gcd(s, (uint64_t)n) != 1) ++s;
    return s % (uint64_t)n;
}

bool cols_per_lane_fits(int64_t r, int cpl) {
    if (cpl == 1) return r >= 1 && r <= kWave;
    // wider chunks pair with lane groups of at least 8 / cpl lanes (r > 4)
    if (cpl == 2 || cpl == 4) return r > 4 && r <= (int64_t)kWave * cpl;
    return false;
}

int cols_per_lane(int64_t r, int hint, bool device_atomics) {
    if (hint == 0) hint = g_cols_per_lane.load(std::memory_order_relaxed);
    if (hint != 0 && cols_per_lane_fits(r, hint)) return hint;
    // Automatic.  Wider layouts spread the per-sample work (broadcast of the
    // sample, the derivative, the group sum) over more columns, but when r is
    // not a multiple of lps each further column step is a partly filled
    // instruction, and a device atomic costs one operation per row sector per
    // instruction, so a mode on device atomics keeps one column per lane
    // (measured on MI355X: rank 8 with LDS partials 22.6 -> 21.2 us with two
    // columns; rank 32 with LDS partials 156 -> 129 us with four; rank 10 with
    // a device-atomic mode 90 -> 125 us with two).  Ranks above 64 need them.
    if (r > 2 * kWave) return 4;
    if (r > kWave) return 2;
    if (device_atomics || r <= 4) return 1;
    if (r <= 16) return 2;
    return 4;
}

void lds_swizzle_params(int d, int64_t r, int lps, int cpl, int elem_bytes, uint32_t* shift, uint32_t* mask) {
    *shift = 0;
    *mask = 0;
    // In one column step the 64 / lps samples of a wave add into chunk c of
    // their rows; with rows of at most 256 bytes (64 LDS banks) the row's
    // place in a 256-byte window spreads them over only 256 / (r * 8)
    // positions.  Flipping the chunk index by the row bits just above those
    // that fix that place spreads them over 256 / (lps * 8).  Measured on
    // MI355X with this pattern: FP64 adds at r = 8, 16, 32 take about a fifth
    // fewer cycles per instruction; the FP32 compare-and-swap adds gain a few
    // percent, so only FP64 partials are swizzled.  Chunks of at least 32
    // bytes (lps >= 4) keep the 32-byte reads of the partial's flush whole.
    if (elem_bytes != 8 || cpl < 2 || lps < 4 || r != (int64_t)cpl * lps || r * 8 > 256 || d > 3) return;
    auto lg = [](int64_t v) {
        int l = 0;
        while ((int64_t{1} << l) < v) ++l;
        return l;
    };
    const int chunk_bit = lg((int64_t)lps * 8);  // lowest bit of the chunk index
    const int row_bit = lg(r * 8);               // lowest bit of the row index
    const int window_bit = row_bit > 8 ? row_bit : 8;
    *shift = (uint32_t)(window_bit - chunk_bit);
    *mask = (uint32_t)(cpl - 1) << chunk_bit;
}

int lanes_per_sample(int64_t r, int cpl) {
    const int64_t need = (r + cpl - 1) / cpl;
    int l = 1;
    while (l < need) l <<= 1;
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


static GradArgs base_args(const gcp_tensor* X, const gcp_factors* M, const ScatterPlan& pl, double* acc,
                          void* partials) {
    GradArgs a{};
    for (int k = 0; k < X->d; ++k) a.dims.n[k] = X->dims[k];
    a.format = X->format;
    a.r = (int)M->rank;
    a.cpl = cols_per_lane(M->rank, 0, pl.priv_mask != (1u << X->d) - 1u);
    a.lps = lanes_per_sample(M->rank, a.cpl);
    lds_swizzle_params(X->d, M->rank, a.lps, a.cpl, pl.lds_elem, &a.lds_swz_shift, &a.lds_swz_mask);
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
    dispatch_d(X->d, [&](auto dc) { grad_launch<decltype(dc)::value, true>(a, pl, M->dtype, GCP_F32, s, nullptr, nullptr); });
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
            a.rej_status = rs->status;
        }
    }
    a.n_direct_items = (a.n_direct + kWave - 1) / kWave;
    const bool two_kinds = (cfg->sampler == GCP_SAMPLER_STRATIFIED || cfg->sampler == GCP_SAMPLER_SEMI_STRATIFIED) &&
                           cfg->p > 0 && cfg->q > 0;
    a.item_stride = item_stride(a.n_direct_items + a.n_zero_items, two_kinds);
    // with nothing sampled the single workgroup still publishes a zero partial
    dispatch_d(X->d, [&](auto dc) {
        grad_launch<decltype(dc)::value, false>(a, pl, M->dtype, X->vdtype, s, ev_start, ev_stop);
    });
    return check_launch("gcp_sampled_grad");
}

gcp_status launch_reduce(const gcp_factors* M, const ScatterPlan& pl, const double* acc, const void* partials,
                         void* const* G, int accumulate, const AdamParams* adam, uint64_t* bump_counter,
                         hipStream_t s, const double* scale) {
    ReduceArgs a{};
    a.bump_counter = bump_counter;
    a.scale = scale;
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


gcp_status launch_loss_grad(gcp_loss loss, const gcp_tensor* X, const gcp_sampling* cfg, const gcp_factors* M,
                            const uint32_t* idx, const void* xval, const uint8_t* stratum, int64_t S,
                            double eps, void* ytilde, double* loss_sum, hipStream_t s) {
    if (S <= 0) return GCP_OK;
    LossArgs a{};
    a.loss = loss;
    a.r = (int)M->rank;
    a.cpl = cols_per_lane(M->rank, 0);
    a.lps = lanes_per_sample(M->rank, a.cpl);
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
