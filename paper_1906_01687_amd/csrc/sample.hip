// sample.hip -- index draws of the sampled GCP gradient (Kolda & Hong,
// Sec. 4.1-4.3, Alg. 1-3): uniform draws, nonzero picks, semi-stratified
// "zeros", and stratified zeros by rejection against a hash of the nonzeros.
//
// The rejection loop of Alg. 2 keeps drawing until q zeros are accepted.  On
// the GPU the candidates j = 0, 1, 2, ... are examined in tiles of 1024; an
// ordered compaction (per-tile counts, one scan, per-tile ballot ranks) keeps
// exactly the first q accepted in counter order, and a one-workgroup refill
// kernel continues the counter stream on the device in the rare case the
// first batch holds fewer than q zeros.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "device.hpp"

namespace gcp {

// ---------------------------------------------------------------------------
// Nonzero hash build (CAS insert of key+1, linear probing).
// ---------------------------------------------------------------------------
__global__ void fill_u64_kernel(uint64_t* __restrict__ p, int64_t n, uint64_t v) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

template <int D>
__global__ void nz_build_kernel(const uint32_t* __restrict__ coo, int64_t nnz, Dims dims,
                                unsigned long long* __restrict__ keys, uint32_t* __restrict__ pos,
                                uint64_t mask) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t i[D];
#pragma unroll
        for (int k = 0; k < D; ++k) i[k] = coo[e * D + k];
        const uint64_t L = linear_key<D>(i, dims.n);
        const unsigned long long want = L + 1;
        uint64_t h = mix64(L) & mask;
        for (uint64_t probe = 0; probe <= mask; ++probe) {
            const unsigned long long old = atomicCAS(&keys[h], 0ull, want);
            if (old == 0ull || old == want) {
                pos[h] = (uint32_t)e;
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

template <int D>
__global__ void nz_bitmap_kernel(const uint32_t* __restrict__ coo, int64_t nnz, Dims dims, uint32_t* bitmap) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t i[D];
#pragma unroll
        for (int k = 0; k < D; ++k) i[k] = coo[e * D + k];
        const uint64_t L = linear_key<D>(i, dims.n);
        atomicOr(&bitmap[L >> 5], 1u << (L & 31));
    }
}

// ---------------------------------------------------------------------------
// Direct draws: uniform, nonzero picks, semi-stratified zeros.
// ---------------------------------------------------------------------------
struct DirectArgs {
    Dims dims;
    uint64_t seed, pid, iter;
    const uint64_t* iter_ctr;
    int kind;
    int format;
    int64_t count, out_off, nnz;
    const void* values;
    const uint32_t* coo;
    NzTable tab;
    uint32_t* idx;
    void* xval;
    uint8_t* stratum;
    uint8_t nz_code;
};

template <int D, typename VT>
__global__ void sample_direct_kernel(DirectArgs a) {
    const VT* __restrict__ vals = static_cast<const VT*>(a.values);
    VT* __restrict__ xout = static_cast<VT*>(a.xval);
    const uint64_t iter = effective_iteration(a.iter, a.iter_ctr);
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < a.count;
         c += (int64_t)gridDim.x * blockDim.x) {
        uint32_t i[D];
        VT x = VT(0);
        uint8_t code;
        if (a.kind == kKindNonzero) {
            const uint64_t e = draw_nonzero(a.seed, a.pid, (uint64_t)c, iter, (uint64_t)a.nnz);
#pragma unroll
            for (int k = 0; k < D; ++k) i[k] = a.coo[e * D + k];
            x = vals[e];
            code = a.nz_code;
        } else {
            if (a.kind == kKindFull) unravel<D>((uint64_t)c, a.dims.n, i);
            else draw_index<D>(a.seed, a.pid, (uint64_t)c, iter, kPurposeUniform, a.dims.n, i);
            if (a.kind == kKindUniform || a.kind == kKindFull) {
                const uint64_t L = linear_key<D>(i, a.dims.n);
                if (a.format == GCP_DENSE) {
                    x = vals[L];
                } else {
                    const int64_t e = nz_lookup(a.tab, L);
                    x = e >= 0 ? vals[e] : VT(0);
                }
                code = GCP_STRATUM_UNIFORM;
            } else {
                code = GCP_STRATUM_SEMI_ZERO;
            }
        }
        const int64_t o = a.out_off + c;
#pragma unroll
        for (int k = 0; k < D; ++k) a.idx[o * D + k] = i[k];
        xout[o] = x;
        a.stratum[o] = code;
    }
}

// ---------------------------------------------------------------------------
// Rejection pipeline for stratified zeros.  Candidate j belongs to chunk
// j / 64; one wave examines one chunk, so a ballot ranks its accepted
// candidates in counter order.
// ---------------------------------------------------------------------------
struct RejArgs {
    Dims dims;
    uint64_t seed, pid, iter;
    const uint64_t* iter_ctr;
    int64_t ncand;  // candidates in the first batch
    int64_t q;      // zeros wanted
    int64_t p_off;  // output offset of zero 0
    NzTable tab;
    uint32_t* idx;
    void* xval;
    uint8_t* stratum;
    int vdtype;
    uint32_t* chunk_count;
    uint64_t* chunk_prefix;
    uint32_t* group_sum;
    uint32_t* zstage;
    uint32_t* status;
    int64_t nchunks;
};

// Counts the accepted candidates of each 64-candidate chunk, stages their
// indices compacted in counter order (zstage[chunk * 64 + rank][k]) and
// writes the sum of each workgroup's 4 chunks (group_sum).
template <int D>
__global__ __launch_bounds__(kRejThreads) void rej_count_kernel(RejArgs a) {
    __shared__ uint32_t wave_cnt[kRejThreads / kWave];
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t iter = effective_iteration(a.iter, a.iter_ctr);
    uint32_t i[D];
    const bool acc = j < a.ncand && candidate_accepted<D>(a.dims, a.tab, a.seed, a.pid, iter, (uint64_t)j, i);
    const uint64_t bal = __ballot(acc);
    const int64_t chunk = j / kRejChunk;
    const uint32_t cnt = (uint32_t)__popcll(bal);
    if (j == 0) a.status[0] = 0;
    if (a.zstage && acc) {
        const int64_t o = chunk * kRejChunk + __popcll(bal & ((1ull << lane) - 1ull));
#pragma unroll
        for (int k = 0; k < D; ++k) a.zstage[o * D + k] = i[k];
    }
    if (lane == 0) {
        if (chunk < a.nchunks) a.chunk_count[chunk] = cnt;
        wave_cnt[threadIdx.x / kWave] = cnt;
    }
    if (a.group_sum) {
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int w = 0; w < kRejThreads / kWave; ++w) t += wave_cnt[w];
            a.group_sum[blockIdx.x] = t;
        }
    }
}

// Exclusive scan of the chunk counts by one workgroup of 1024 threads;
// chunk_prefix[nchunks] receives the total.
__global__ __launch_bounds__(1024) void rej_scan_kernel(RejArgs a) {
    __shared__ uint64_t part[1024];
    __shared__ uint64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < a.nchunks; base += 1024) {
        const int64_t b = base + tid;
        const uint64_t v = b < a.nchunks ? a.chunk_count[b] : 0;
        part[tid] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan
            const uint64_t add = tid >= o ? part[tid - o] : 0;
            __syncthreads();
            part[tid] += add;
            __syncthreads();
        }
        if (b < a.nchunks) a.chunk_prefix[b] = carry + part[tid] - v;
        __syncthreads();
        if (tid == 1023) carry += part[1023];
        __syncthreads();
    }
    if (tid == 0) {
        a.chunk_prefix[a.nchunks] = carry;
    }
}

template <int D>
__device__ __forceinline__ void write_zero(const RejArgs& a, uint64_t rank, const uint32_t (&i)[D]) {
    const int64_t o = a.p_off + (int64_t)rank;
#pragma unroll
    for (int k = 0; k < D; ++k) a.idx[o * D + k] = i[k];
    if (a.xval) {
        if (a.vdtype == GCP_F64) static_cast<double*>(a.xval)[o] = 0.0;
        else static_cast<float*>(a.xval)[o] = 0.0f;
    }
    if (a.stratum) a.stratum[o] = GCP_STRATUM_ZERO;
}

template <int D>
__global__ __launch_bounds__(kRejThreads) void rej_write_kernel(RejArgs a) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t iter = effective_iteration(a.iter, a.iter_ctr);
    uint32_t i[D];
    const bool acc = j < a.ncand && candidate_accepted<D>(a.dims, a.tab, a.seed, a.pid, iter, (uint64_t)j, i);
    const uint64_t bal = __ballot(acc);
    const int64_t chunk = j / kRejChunk;
    if (chunk >= a.nchunks) return;  // whole wave beyond the batch
    const uint64_t rank = a.chunk_prefix[chunk] + __popcll(bal & ((1ull << lane) - 1ull));
    if (acc && rank < (uint64_t)a.q) write_zero<D>(a, rank, i);
}

// Continues the candidate stream after the first batch until q zeros exist.
// One wave; `filled` is wave-uniform, so all lanes leave the loop together.
template <int D>
__global__ __launch_bounds__(kWave) void rej_refill_kernel(RejArgs a) {
    const int lane = threadIdx.x;
    uint64_t filled = a.chunk_prefix[a.nchunks];
    if (filled >= (uint64_t)a.q) return;
    const uint64_t iter = effective_iteration(a.iter, a.iter_ctr);
    uint64_t base = (uint64_t)a.ncand;
    for (int64_t t = 0; t < kRejRefillTurns && filled < (uint64_t)a.q; ++t) {
        uint32_t i[D];
        const bool acc = candidate_accepted<D>(a.dims, a.tab, a.seed, a.pid, iter, base + lane, i);
        const uint64_t bal = __ballot(acc);
        const uint64_t rank = filled + __popcll(bal & ((1ull << lane) - 1ull));
        if (acc && rank < (uint64_t)a.q) write_zero<D>(a, rank, i);
        filled += __popcll(bal);
        base += kWave;
    }
    if (lane == 0 && filled < (uint64_t)a.q) a.status[0] = 1;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static Dims make_dims(const gcp_tensor* X) {
    Dims d{};
    for (int k = 0; k < X->d; ++k) d.n[k] = X->dims[k];
    return d;
}

static NzTable make_table(const gcp_tensor* X) {
    NzTable t{};
    if (X->nz_table && X->nz_slots > 0) {
        t.keys = static_cast<const uint64_t*>(X->nz_table);
        t.pos = reinterpret_cast<const uint32_t*>(static_cast<const char*>(X->nz_table) + 8 * X->nz_slots);
        t.mask = (uint64_t)X->nz_slots - 1;
    }
    t.bitmap = X->nz_bitmap;
    return t;
}

static int grid_for(int64_t n, int threads, int cap = 8192) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

gcp_status launch_nz_build(const gcp_tensor* X, void* table, int64_t slots, hipStream_t s) {
    auto* keys = static_cast<unsigned long long*>(table);
    auto* pos = reinterpret_cast<uint32_t*>(static_cast<char*>(table) + 8 * slots);
    // keys and positions are cleared with a fill kernel (graph-capture safe)
    fill_u64_kernel<<<grid_for(slots + (slots + 1) / 2, 256), 256, 0, s>>>(
        static_cast<uint64_t*>(table), slots + (slots + 1) / 2, 0ull);
    if (X->nnz > 0) {
        const int g = grid_for(X->nnz, 256);
        const Dims dims = make_dims(X);
        dispatch_d(X->d, [&](auto dc) {
            constexpr int D = decltype(dc)::value;
            hipLaunchKernelGGL(nz_build_kernel<D>, dim3(g), dim3(256), 0, s, X->coo_idx, X->nnz, dims,
                               keys, pos, (uint64_t)slots - 1);
        });
    }
    return check_launch("gcp_nz_index_build");
}

gcp_status launch_nz_bitmap(const gcp_tensor* X, uint32_t* bitmap, size_t bytes, hipStream_t s) {
    const int64_t words = (int64_t)(bytes / 8);  // the size is a whole number of 64-bit words
    fill_u64_kernel<<<grid_for(words, 256), 256, 0, s>>>(reinterpret_cast<uint64_t*>(bitmap), words, 0ull);
    if (X->nnz > 0) {
        const int g = grid_for(X->nnz, 256);
        const Dims dims = make_dims(X);
        dispatch_d(X->d, [&](auto dc) {
            constexpr int D = decltype(dc)::value;
            hipLaunchKernelGGL(nz_bitmap_kernel<D>, dim3(g), dim3(256), 0, s, X->coo_idx, X->nnz, dims, bitmap);
        });
    }
    return check_launch("gcp_nz_bitmap_build");
}

template <int D>
static void direct_launch(const DirectArgs& a, int vdtype, hipStream_t s) {
    const int g = grid_for(a.count, 256);
    if (vdtype == GCP_F64) hipLaunchKernelGGL((sample_direct_kernel<D, double>), dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((sample_direct_kernel<D, float>), dim3(g), dim3(256), 0, s, a);
}

gcp_status launch_sample_direct(const gcp_tensor* X, const gcp_sampling* cfg, int kind, int64_t count,
                                int64_t out_off, uint32_t* idx, void* xval, uint8_t* stratum,
                                hipStream_t s) {
    if (count <= 0) return GCP_OK;
    DirectArgs a{};
    a.dims = make_dims(X);
    a.seed = cfg->seed;
    a.pid = cfg->problem_id;
    a.iter = cfg->iteration;
    a.iter_ctr = cfg->iteration_counter;
    a.kind = kind;
    a.format = X->format;
    a.count = count;
    a.out_off = out_off;
    a.nnz = X->nnz;
    a.values = X->values;
    a.coo = X->coo_idx;
    a.tab = make_table(X);
    a.idx = idx;
    a.xval = xval;
    a.stratum = stratum;
    a.nz_code = cfg->sampler == GCP_SAMPLER_SEMI_STRATIFIED ? GCP_STRATUM_NZ_CORR : GCP_STRATUM_NZ;
    dispatch_d(X->d, [&](auto dc) { direct_launch<decltype(dc)::value>(a, X->vdtype, s); });
    return check_launch("gcp_sample");
}

static RejArgs rej_args(const gcp_tensor* X, const gcp_sampling* cfg, int64_t ncand, const RejScratch& rs) {
    RejArgs a{};
    a.dims = make_dims(X);
    a.seed = cfg->seed;
    a.pid = cfg->problem_id;
    a.iter = cfg->iteration;
    a.iter_ctr = cfg->iteration_counter;
    a.ncand = ncand;
    a.q = cfg->q;
    a.tab = make_table(X);
    a.vdtype = X->vdtype;
    a.chunk_count = rs.chunk_count;
    a.chunk_prefix = rs.chunk_prefix;
    a.group_sum = rs.group_sum;
    a.zstage = rs.zstage;
    a.status = rs.status;
    a.nchunks = rs.nchunks;
    return a;
}

gcp_status launch_rejection_count(const gcp_tensor* X, const gcp_sampling* cfg, int64_t ncand,
                                  const RejScratch& rs, bool scan, hipStream_t s) {
    if (cfg->q <= 0) return GCP_OK;
    const RejArgs a = rej_args(X, cfg, ncand, rs);
    const unsigned blocks = (unsigned)((ncand + kRejThreads - 1) / kRejThreads);
    dispatch_d(X->d, [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        hipLaunchKernelGGL(rej_count_kernel<D>, dim3(blocks), dim3(kRejThreads), 0, s, a);
    });
    if (scan) hipLaunchKernelGGL(rej_scan_kernel, dim3(1), dim3(1024), 0, s, a);
    return check_launch("stratified rejection count");
}

gcp_status launch_rejection_write(const gcp_tensor* X, const gcp_sampling* cfg, int64_t ncand,
                                  const RejScratch& rs, uint32_t* idx_out, int64_t p_off, void* xval,
                                  uint8_t* stratum, hipStream_t s) {
    if (cfg->q <= 0) return GCP_OK;
    RejArgs a = rej_args(X, cfg, ncand, rs);
    a.p_off = p_off;
    a.idx = idx_out;
    a.xval = xval;
    a.stratum = stratum;
    const unsigned blocks = (unsigned)((ncand + kRejThreads - 1) / kRejThreads);
    dispatch_d(X->d, [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        hipLaunchKernelGGL(rej_write_kernel<D>, dim3(blocks), dim3(kRejThreads), 0, s, a);
        hipLaunchKernelGGL(rej_refill_kernel<D>, dim3(1), dim3(kWave), 0, s, a);
    });
    return check_launch("stratified rejection write");
}

__global__ void bump_counter_kernel(uint64_t* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) c[0] += 1;
}

gcp_status launch_bump_counter(uint64_t* counter, hipStream_t s) {
    if (!counter) return GCP_OK;
    hipLaunchKernelGGL(bump_counter_kernel, dim3(1), dim3(64), 0, s, counter);
    return check_launch("iteration counter");
}

}  // namespace gcp
