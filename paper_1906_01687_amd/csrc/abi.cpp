// abi.cpp -- the extern "C" entry points of libgcp: host-side argument
// validation, workspace sizing and carving, and the launch sequence of each
// call.  No device synchronisation and no allocation happen here.
#include <hip/hip_runtime.h>
#include <hip/hip_runtime_api.h>

#include <math.h>

#include <cmath>
#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "gcp.h"

namespace gcp {

static thread_local std::string g_last_error;

static std::string gcp_last_error_str() { return g_last_error; }

gcp_status set_error(gcp_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

void clear_error() { g_last_error.clear(); }

gcp_status check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(GCP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return GCP_OK;
}

static unsigned __int128 omega128(const gcp_tensor* X) {
    unsigned __int128 w = 1;
    for (int k = 0; k < X->d; ++k) w *= (unsigned __int128)(uint64_t)X->dims[k];
    return w;
}

static double omega_d(const gcp_tensor* X) {
    double w = 1.0;
    for (int k = 0; k < X->d; ++k) w *= (double)X->dims[k];
    return w;
}

void stratum_weights(const gcp_tensor* X, const gcp_sampling* cfg, double w[5]) {
    const double omega = omega_d(X);
    const double eta = (double)X->nnz;
    w[GCP_STRATUM_UNIFORM] = cfg->sampler == GCP_SAMPLER_FULL ? 1.0 : (cfg->s > 0 ? omega / (double)cfg->s : 0.0);
    w[GCP_STRATUM_NZ] = cfg->p > 0 ? eta / (double)cfg->p : 0.0;
    w[GCP_STRATUM_ZERO] = cfg->q > 0 ? (omega - eta) / (double)cfg->q : 0.0;
    w[GCP_STRATUM_NZ_CORR] = w[GCP_STRATUM_NZ];
    w[GCP_STRATUM_SEMI_ZERO] = cfg->q > 0 ? omega / (double)cfg->q : 0.0;
    // weighted objective (eq. wgcp): entries a COO tensor does not store weigh
    // w_zero, so the zero strata carry it; stored entries get theirs per sample
    const double wz = zero_weight(X);
    w[GCP_STRATUM_ZERO] *= wz;
    w[GCP_STRATUM_SEMI_ZERO] *= wz;
}

double zero_weight(const gcp_tensor* X) {
    return (X->weights && X->format == GCP_COO) ? X->w_zero : 1.0;
}

double corr_zero_weight(const gcp_tensor* X, const gcp_sampling* cfg) {
    // the g(0, m) part of a corrected nonzero: (eta / p) * w_zero
    double w[5];
    stratum_weights(X, cfg, w);
    return w[GCP_STRATUM_NZ_CORR] * zero_weight(X);
}

int64_t full_count(const gcp_tensor* X) { return (int64_t)omega128(X); }

int64_t rejection_batch(const gcp_tensor* X, const gcp_sampling* cfg) {
    const double omega = omega_d(X);
    const double zeta = omega - (double)X->nnz;
    const double rho = cfg->rho > 0.0 ? cfg->rho : 1.1;
    double n = ceil(rho * (double)cfg->q * omega / zeta);
    if (!(n >= 1.0)) n = 1.0;
    if (n > 4.0e15) n = 4.0e15;
    return (int64_t)n;
}

RejScratch carve_rejection(Carver& c, void* base, int64_t ncand, bool staged, int d) {
    RejScratch r{};
    r.nchunks = (ncand + kRejChunk - 1) / kRejChunk;
    if (r.nchunks < 1) r.nchunks = 1;
    r.ngroups = (ncand + kRejThreads - 1) / kRejThreads;
    if (r.ngroups < 1) r.ngroups = 1;
    r.chunk_count = c.take<uint32_t>(base, (size_t)r.nchunks);
    r.chunk_prefix = c.take<uint64_t>(base, (size_t)r.nchunks + 1);
    if (staged) {
        r.group_sum = c.take<uint32_t>(base, (size_t)r.ngroups);
        r.zstage = c.take<uint32_t>(base, (size_t)r.nchunks * kRejChunk * (size_t)d);
    }
    r.status = c.take<uint32_t>(base, 1);
    return r;
}

int device_cu_count() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
static gcp_status check_tensor(const gcp_tensor* X) {
    if (!X) return set_error(GCP_ERR_INVALID_ARG, "X is NULL");
    if (X->d < 1 || X->d > GCP_MAX_D) return set_error(GCP_ERR_INVALID_ARG, "X->d must be in [1, 8]");
    if (X->format != GCP_DENSE && X->format != GCP_COO)
        return set_error(GCP_ERR_INVALID_ARG, "X->format must be GCP_DENSE or GCP_COO");
    if (X->vdtype != GCP_F32 && X->vdtype != GCP_F64)
        return set_error(GCP_ERR_INVALID_ARG, "X->vdtype must be GCP_F32 or GCP_F64");
    if (X->weights && !std::isfinite(X->w_zero))
        return set_error(GCP_ERR_INVALID_ARG, "X->w_zero must be finite");
    for (int k = 0; k < X->d; ++k)
        if (X->dims[k] < 1 || X->dims[k] > (int64_t)0xFFFFFFFFll)
            return set_error(GCP_ERR_INVALID_ARG, "X->dims[" + std::to_string(k) + "] must be in [1, 2^32 - 1]");
    if (omega128(X) >= ((unsigned __int128)1 << 63))
        return set_error(GCP_ERR_UNSUPPORTED, "the number of tensor entries must be below 2^63");
    if (X->format == GCP_DENSE) {
        if (!X->values) return set_error(GCP_ERR_INVALID_ARG, "dense X->values is NULL");
    } else {
        if (X->nnz < 0 || X->nnz > (int64_t)0xFFFFFFFFll)
            return set_error(GCP_ERR_INVALID_ARG, "X->nnz must be in [0, 2^32 - 1]");
        if ((unsigned __int128)(uint64_t)X->nnz > omega128(X))
            return set_error(GCP_ERR_INVALID_ARG, "X->nnz exceeds the number of entries");
        if (X->nnz > 0 && (!X->coo_idx || !X->values))
            return set_error(GCP_ERR_INVALID_ARG, "COO X needs coo_idx and values");
    }
    return GCP_OK;
}

static gcp_status check_table(const gcp_tensor* X) {
    if (!X->nz_table) return set_error(GCP_ERR_INVALID_ARG, "X->nz_table is NULL (build it with gcp_nz_index_build)");
    if (X->nz_slots < 2 || (X->nz_slots & (X->nz_slots - 1)) || X->nz_slots <= X->nnz)
        return set_error(GCP_ERR_INVALID_ARG, "X->nz_slots must be a power of two above nnz");
    return GCP_OK;
}

static gcp_status check_sampling(const gcp_tensor* X, const gcp_sampling* cfg) {
    if (!cfg) return set_error(GCP_ERR_INVALID_ARG, "cfg is NULL");
    switch (cfg->sampler) {
    case GCP_SAMPLER_FULL:
        // every entry's value is looked up in the nonzero table, also when
        // the tensor stores no entries
        if (X->format == GCP_COO && full_count(X) > 0) {
            if (gcp_status st = check_table(X)) return st;
        }
        break;
    case GCP_SAMPLER_UNIFORM:
        if (cfg->s < 0) return set_error(GCP_ERR_INVALID_ARG, "cfg->s must be >= 0");
        if (X->format == GCP_COO && cfg->s > 0) {
            if (gcp_status st = check_table(X)) return st;
        }
        break;
    case GCP_SAMPLER_STRATIFIED:
    case GCP_SAMPLER_SEMI_STRATIFIED: {
        if (X->format != GCP_COO)
            return set_error(GCP_ERR_INVALID_ARG, "stratified and semi-stratified sampling need a COO tensor");
        if (cfg->p < 0 || cfg->q < 0) return set_error(GCP_ERR_INVALID_ARG, "cfg->p and cfg->q must be >= 0");
        if (cfg->p > 0 && X->nnz == 0) return set_error(GCP_ERR_INVALID_ARG, "p > 0 needs at least one nonzero");
        if (cfg->sampler == GCP_SAMPLER_STRATIFIED && cfg->q > 0) {
            if (!X->nz_bitmap) {
                if (gcp_status st = check_table(X)) return st;
            }
            const double omega = omega_d(X), zeta = omega - (double)X->nnz;
            if (!(zeta > 0.0)) return set_error(GCP_ERR_INVALID_ARG, "stratified zeros requested but X has no zeros");
            if (zeta < omega * (1.0 / 1048576.0))
                return set_error(GCP_ERR_UNSUPPORTED, "rejection needs zeros to be at least 2^-20 of the entries");
            // Drawing q zeros takes a negative-binomial number of candidates:
            // mean q / pi, standard deviation sqrt(q (1 - pi)) / pi, for the
            // zero fraction pi = zeta / omega (Sec. 4.2, App. B).  The first
            // batch (rho times the mean) and the device refill cap must cover
            // the mean plus eight standard deviations.
            const double pi = zeta / omega, q = (double)cfg->q;
            const double need = q / pi + 8.0 * std::sqrt(q * (1.0 - pi)) / pi;
            const double have = (double)rejection_batch(X, cfg) + (double)kRejRefillCandidates;
            if (need > have)
                return set_error(GCP_ERR_UNSUPPORTED,
                                 "stratified rejection: q zeros need about " + std::to_string((int64_t)need) +
                                     " candidates, beyond the first batch plus the refill cap (" +
                                     std::to_string((int64_t)have) + "); raise cfg->rho");
        }
        break;
    }
    default:
        return set_error(GCP_ERR_INVALID_ARG, "cfg->sampler is not a gcp_sampler");
    }
    return GCP_OK;
}

static gcp_status check_factors(const gcp_tensor* X, const gcp_factors* M) {
    if (!M) return set_error(GCP_ERR_INVALID_ARG, "M is NULL");
    if (M->dtype != GCP_F32 && M->dtype != GCP_F64 && M->dtype != GCP_BF16)
        return set_error(GCP_ERR_INVALID_ARG, "M->dtype must be GCP_F32, GCP_F64 or GCP_BF16");
    if (M->rank < 1) return set_error(GCP_ERR_INVALID_ARG, "M->rank must be >= 1");
    if (M->rank > GCP_MAX_RANK) return set_error(GCP_ERR_UNSUPPORTED, "M->rank above 256 is not supported");
    const uint64_t esz = M->dtype == GCP_F64 ? 8 : (M->dtype == GCP_F32 ? 4 : 2);
    for (int k = 0; k < X->d; ++k) {
        if (!M->A[k]) return set_error(GCP_ERR_INVALID_ARG, "M->A[" + std::to_string(k) + "] is NULL");
        // factor rows are gathered through buffer descriptors with 32-bit byte offsets
        if ((uint64_t)X->dims[k] * (uint64_t)M->rank * esz > 0xFFFFFFFFull)
            return set_error(GCP_ERR_UNSUPPORTED, "factor block " + std::to_string(k) + " exceeds 4 GiB");
    }
    return GCP_OK;
}

static gcp_status check_loss(gcp_loss loss) {
    if (loss != GCP_LOSS_GAUSSIAN && loss != GCP_LOSS_BERNOULLI_ODDS && loss != GCP_LOSS_POISSON &&
        loss != GCP_LOSS_GAMMA && loss != GCP_LOSS_BETA_HALF)
        return set_error(GCP_ERR_INVALID_ARG, "loss is not a gcp_loss");
    return GCP_OK;
}

static int64_t sample_count(const gcp_tensor* X, const gcp_sampling* cfg) {
    if (cfg->sampler == GCP_SAMPLER_FULL) return full_count(X);
    return cfg->sampler == GCP_SAMPLER_UNIFORM ? cfg->s : cfg->p + cfg->q;
}

static size_t sample_ws(const gcp_tensor* X, const gcp_sampling* cfg, Carver& c, void* base, RejScratch* rs) {
    if (cfg->sampler == GCP_SAMPLER_STRATIFIED && cfg->q > 0) {
        RejScratch r = carve_rejection(c, base, rejection_batch(X, cfg), false, X->d);
        if (rs) *rs = r;
    }
    return c.bytes();
}

static gcp_status check_adam(gcp_dtype dtype, int64_t P, const void* A, const float* A_master, const void* B,
                             const void* C, const int64_t* state, double alpha, double beta1, double beta2,
                             double eps, gcp_eps_mode eps_mode) {
    if (P < 0) return set_error(GCP_ERR_INVALID_ARG, "P must be >= 0");
    if (dtype != GCP_F32 && dtype != GCP_F64 && dtype != GCP_BF16)
        return set_error(GCP_ERR_INVALID_ARG, "dtype must be GCP_F32, GCP_F64 or GCP_BF16");
    if (!state) return set_error(GCP_ERR_INVALID_ARG, "state is NULL");
    if (P > 0 && (!A || !B || !C)) return set_error(GCP_ERR_INVALID_ARG, "A, B and C must be non-NULL");
    if (dtype == GCP_BF16 && P > 0 && !A_master)
        return set_error(GCP_ERR_INVALID_ARG, "GCP_BF16 needs the float master copy A_master");
    if (eps_mode != GCP_EPS_INSIDE_SQRT && eps_mode != GCP_EPS_OUTSIDE_SQRT)
        return set_error(GCP_ERR_INVALID_ARG, "eps_mode is not a gcp_eps_mode");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return set_error(GCP_ERR_INVALID_ARG, "beta1 and beta2 must be in [0, 1)");
    if (!(eps >= 0.0) || !(alpha >= 0.0)) return set_error(GCP_ERR_INVALID_ARG, "alpha and eps must be >= 0");
    return GCP_OK;
}

static size_t mttkrp_ws(const gcp_tensor* X, const gcp_factors* M, int64_t S, void* base, ScatterPlan* plan,
                        double** acc, void** partials) {
    const ScatterPlan pl = plan_scatter(X, M, (S + 63) / 64);
    Carver c;
    double* a = c.take<double>(base, (size_t)acc_words(pl));
    void* p = c.take<char>(base, scatter_partials_bytes(pl, M->dtype));
    if (plan) *plan = pl;
    if (acc) *acc = a;
    if (partials) *partials = p;
    return c.bytes();
}

struct FusedLayout {
    ScatterPlan plan;
    int64_t ncand;
    double* acc;
    void* partials;
    RejScratch rs;
    bool rejection;
};

static size_t fused_ws(const gcp_tensor* X, const gcp_factors* M, const gcp_sampling* cfg, void* base,
                       FusedLayout* out) {
    FusedLayout f{};
    f.rejection = cfg->sampler == GCP_SAMPLER_STRATIFIED && cfg->q > 0;
    f.ncand = f.rejection ? rejection_batch(X, cfg) : 0;
    f.plan = plan_scatter(X, M, fused_items(X, cfg, f.ncand));
    Carver c;
    f.acc = c.take<double>(base, (size_t)acc_words(f.plan));
    f.partials = c.take<char>(base, scatter_partials_bytes(f.plan, M->dtype));
    if (f.rejection) f.rs = carve_rejection(c, base, f.ncand, true, X->d);
    if (out) *out = f;
    return c.bytes();
}

// Kernel timing session (see gcp_timing_start in gcp.h).
struct Timing {
    std::mutex mu;
    std::vector<hipEvent_t> start, stop;
    size_t used = 0;
    bool armed = false;
};
static Timing g_timing;

// The next event pair of an armed timing session, or none.  Nothing is timed
// on a stream that is being captured into a graph: an event there would not
// give per-replay timings.
static void timing_take(hipStream_t s, hipEvent_t* start, hipEvent_t* stop) {
    *start = *stop = nullptr;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (!g_timing.armed || g_timing.used >= g_timing.start.size()) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return;
    }
    *start = g_timing.start[g_timing.used];
    *stop = g_timing.stop[g_timing.used];
    ++g_timing.used;
}

// The launch sequence shared by gcp_sampled_grad and gcp_sampled_adam_step.
static gcp_status sampled_common(gcp_loss loss, const gcp_tensor* X, const gcp_factors* M, const gcp_sampling* cfg,
                                 double eps, void* const* G, double* loss_sum, void* ws, size_t ws_bytes,
                                 const AdamParams* adam, hipStream_t stream) {
    const size_t need = fused_ws(X, M, cfg, nullptr, nullptr);
    if (!ws || ws_bytes < need) return set_error(GCP_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    FusedLayout f{};
    fused_ws(X, M, cfg, ws, &f);
    const bool scanned = f.rejection && f.rs.ngroups > kMaxGroupsInKernel;
    if (f.rejection) {
        if (gcp_status st = launch_rejection_count(X, cfg, f.ncand, f.rs, scanned, stream)) return st;
    }
    if (gcp_status st = launch_fill_zero(f.acc, acc_words(f.plan), stream)) return st;
    hipEvent_t ev0, ev1;
    timing_take(stream, &ev0, &ev1);
    if (gcp_status st = launch_grad_fused(loss, X, M, cfg, eps, f.plan, f.ncand, f.rejection ? &f.rs : nullptr,
                                          scanned, f.acc, f.partials, loss_sum, adam ? adam->state : nullptr, ev0,
                                          ev1, stream))
        return st;
    return launch_reduce(M, f.plan, f.acc, f.partials, G, 0, adam, cfg->iteration_counter, stream);
}

// Workspace of gcp_sampled_grad_noalloc: one array per device, shared by
// every call on that device.  Host code never uses the array's name as an
// address (in host code it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, once per device, with that device
// current.
static __device__ __align__(256) unsigned char scratch[GCP_NOALLOC_SCRATCH_BYTES];

static gcp_status scratch_address(void** out) {
    static std::mutex mu;
    static void* addr[64] = {nullptr};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return set_error(GCP_ERR_HIP, "gcp_sampled_grad_noalloc: no current HIP device (or more than 64)");
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(GCP_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        }
        addr[dev] = p;
    }
    *out = addr[dev];
    return GCP_OK;
}

// One problem of a batch (gcp_batched_create).
static gcp_status check_problem(const gcp_problem* pr, int32_t b) {
    const std::string at = "problem " + std::to_string(b) + ": ";
    if (gcp_status st = check_loss((gcp_loss)pr->loss)) return set_error(st, at + gcp_last_error_str());
    if (gcp_status st = check_tensor(&pr->X)) return set_error(st, at + gcp_last_error_str());
    if (gcp_status st = check_sampling(&pr->X, &pr->cfg)) return set_error(st, at + gcp_last_error_str());
    if (pr->cfg.sampler == GCP_SAMPLER_STRATIFIED)
        return set_error(GCP_ERR_UNSUPPORTED, at + "batches take UNIFORM or SEMI_STRATIFIED sampling");
    if (gcp_status st = check_factors(&pr->X, &pr->M)) return set_error(st, at + gcp_last_error_str());
    int64_t P = 0;
    for (int k = 0; k < pr->X.d; ++k) P += pr->X.dims[k] * pr->M.rank;
    if (P > 0 && (!pr->A || !pr->B || !pr->C)) return set_error(GCP_ERR_INVALID_ARG, at + "A, B and C must be non-NULL");
    if (pr->M.dtype == GCP_BF16 && !pr->A_master)
        return set_error(GCP_ERR_INVALID_ARG, at + "GCP_BF16 needs the float master copy A_master");
    const size_t esz = pr->M.dtype == GCP_F64 ? 8 : (pr->M.dtype == GCP_F32 ? 4 : 2);
    int64_t off = 0;
    for (int k = 0; k < pr->X.d; ++k) {
        if (pr->M.A[k] != static_cast<const char*>(pr->A) + off * esz)
            return set_error(GCP_ERR_INVALID_ARG, at + "M.A[k] must be the mode-k block of the flat array A");
        off += pr->X.dims[k] * pr->M.rank;
    }
    return GCP_OK;
}

}  // namespace gcp

using namespace gcp;

extern "C" {

const char* gcp_last_error(void) { return g_last_error.c_str(); }

int gcp_abi_version(void) { return GCP_ABI_VERSION; }

int64_t gcp_nz_table_slots(int64_t nnz) {
    int64_t s = 64;
    while (s < 2 * nnz) s <<= 1;
    return s;
}

size_t gcp_nz_table_bytes(int64_t slots) { return slots > 0 ? (size_t)slots * 12u : 0u; }

gcp_status gcp_nz_index_build(const gcp_tensor* X, void* table, int64_t slots, hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_tensor(X)) return st;
    if (X->format != GCP_COO) return set_error(GCP_ERR_INVALID_ARG, "gcp_nz_index_build needs a COO tensor");
    if (!table) return set_error(GCP_ERR_INVALID_ARG, "table is NULL");
    if (slots < 2 || (slots & (slots - 1)) || slots <= X->nnz)
        return set_error(GCP_ERR_INVALID_ARG, "slots must be a power of two above nnz");
    return launch_nz_build(X, table, slots, stream);
}

size_t gcp_nz_bitmap_bytes(const gcp_tensor* X) {
    if (!X || X->format != GCP_COO || X->d < 1 || X->d > GCP_MAX_D) return 0;
    unsigned __int128 w = 1;
    for (int k = 0; k < X->d; ++k) {
        if (X->dims[k] < 1) return 0;
        w *= (unsigned __int128)(uint64_t)X->dims[k];
    }
    if (w >= ((unsigned __int128)1 << 63)) return 0;
    return (size_t)((w + 63) / 64) * 8u;
}

gcp_status gcp_nz_bitmap_build(const gcp_tensor* X, uint32_t* bitmap, size_t bytes, hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_tensor(X)) return st;
    if (X->format != GCP_COO) return set_error(GCP_ERR_INVALID_ARG, "gcp_nz_bitmap_build needs a COO tensor");
    if (!bitmap) return set_error(GCP_ERR_INVALID_ARG, "bitmap is NULL");
    const size_t need = gcp_nz_bitmap_bytes(X);
    if (bytes < need) return set_error(GCP_ERR_INVALID_ARG, "bitmap needs " + std::to_string(need) + " bytes");
    return launch_nz_bitmap(X, bitmap, need, stream);
}

gcp_status gcp_set_cols_per_lane(int32_t cpl) {
    clear_error();
    if (cpl != 0 && cpl != 1 && cpl != 2 && cpl != 4)
        return set_error(GCP_ERR_INVALID_ARG, "cols_per_lane must be 0, 1, 2 or 4");
    g_cols_per_lane.store(cpl, std::memory_order_relaxed);
    return GCP_OK;
}

size_t gcp_sample_workspace_bytes(const gcp_tensor* X, const gcp_sampling* cfg) {
    if (!X || !cfg) return 0;
    Carver c;
    return sample_ws(X, cfg, c, nullptr, nullptr);
}

gcp_status gcp_sample(const gcp_tensor* X, const gcp_sampling* cfg, uint32_t* idx, void* xval, uint8_t* stratum,
                      void* ws, size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_tensor(X)) return st;
    if (gcp_status st = check_sampling(X, cfg)) return st;
    const int64_t S = sample_count(X, cfg);
    if (S == 0) return launch_bump_counter(cfg->iteration_counter, stream);
    if (!idx || !xval || !stratum) return set_error(GCP_ERR_INVALID_ARG, "idx, xval and stratum must be non-NULL");
    Carver c;
    RejScratch rs{};
    const size_t need = sample_ws(X, cfg, c, ws, &rs);
    if (need > 0 && (!ws || ws_bytes < need))
        return set_error(GCP_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    if (cfg->sampler == GCP_SAMPLER_UNIFORM || cfg->sampler == GCP_SAMPLER_FULL) {
        const int kind = cfg->sampler == GCP_SAMPLER_FULL ? kKindFull : kKindUniform;
        if (gcp_status st = launch_sample_direct(X, cfg, kind, S, 0, idx, xval, stratum, stream)) return st;
    } else {
        if (gcp_status st = launch_sample_direct(X, cfg, kKindNonzero, cfg->p, 0, idx, xval, stratum, stream))
            return st;
        if (cfg->sampler == GCP_SAMPLER_SEMI_STRATIFIED) {
            if (gcp_status st = launch_sample_direct(X, cfg, kKindSemiZero, cfg->q, cfg->p, idx, xval, stratum, stream))
                return st;
        } else {
            const int64_t ncand = rejection_batch(X, cfg);
            if (gcp_status st = launch_rejection_count(X, cfg, ncand, rs, true, stream)) return st;
            if (gcp_status st = launch_rejection_write(X, cfg, ncand, rs, idx, cfg->p, xval, stratum, stream))
                return st;
        }
    }
    return launch_bump_counter(cfg->iteration_counter, stream);
}

gcp_status gcp_loss_grad(gcp_loss loss, const gcp_tensor* X, const gcp_sampling* cfg, const gcp_factors* M,
                         const uint32_t* idx, const void* xval, const uint8_t* stratum, int64_t S, double eps,
                         void* ytilde, double* loss_sum, hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_loss(loss)) return st;
    if (gcp_status st = check_tensor(X)) return st;
    if (!cfg) return set_error(GCP_ERR_INVALID_ARG, "cfg is NULL");
    if (gcp_status st = check_factors(X, M)) return st;
    if (S < 0) return set_error(GCP_ERR_INVALID_ARG, "S must be >= 0");
    if (S == 0) return GCP_OK;
    if (!idx || !xval || !stratum || !ytilde)
        return set_error(GCP_ERR_INVALID_ARG, "idx, xval, stratum and ytilde must be non-NULL");
    if (X->weights && X->format == GCP_COO && X->nnz > 0) {
        // the stored samples carry indices only: a nonzero's weight is found
        // through the index table
        if (gcp_status st = check_table(X)) return st;
    }
    return launch_loss_grad(loss, X, cfg, M, idx, xval, stratum, S, eps, ytilde, loss_sum, stream);
}

size_t gcp_mttkrp_workspace_bytes(const gcp_tensor* X, const gcp_factors* M, int64_t S) {
    if (!X || !M || X->d < 1 || X->d > GCP_MAX_D || M->rank < 1 || S < 0) return 0;
    return mttkrp_ws(X, M, S, nullptr, nullptr, nullptr, nullptr);
}

gcp_status gcp_mttkrp_scaled(const gcp_tensor* X, const gcp_factors* M, const uint32_t* idx, const void* ytilde,
                             int64_t S, void* const* G, int accumulate, const double* scale, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_tensor(X)) return st;
    if (gcp_status st = check_factors(X, M)) return st;
    if (S < 0) return set_error(GCP_ERR_INVALID_ARG, "S must be >= 0");
    if (!G) return set_error(GCP_ERR_INVALID_ARG, "G is NULL");
    for (int k = 0; k < X->d; ++k)
        if (!G[k]) return set_error(GCP_ERR_INVALID_ARG, "G[" + std::to_string(k) + "] is NULL");
    if (S > 0 && (!idx || !ytilde)) return set_error(GCP_ERR_INVALID_ARG, "idx and ytilde must be non-NULL");
    const size_t need = gcp_mttkrp_workspace_bytes(X, M, S);
    if (!ws || ws_bytes < need) return set_error(GCP_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    ScatterPlan pl{};
    double* acc = nullptr;
    void* partials = nullptr;
    mttkrp_ws(X, M, S, ws, &pl, &acc, &partials);
    if (gcp_status st = launch_fill_zero(acc, acc_words(pl), stream)) return st;
    if (gcp_status st = launch_grad_list(X, M, idx, ytilde, S, pl, acc, partials, stream)) return st;
    return launch_reduce(M, pl, acc, partials, G, accumulate, nullptr, nullptr, stream, scale);
}

gcp_status gcp_mttkrp(const gcp_tensor* X, const gcp_factors* M, const uint32_t* idx, const void* ytilde, int64_t S,
                      void* const* G, int accumulate, void* ws, size_t ws_bytes, hipStream_t stream) {
    return gcp_mttkrp_scaled(X, M, idx, ytilde, S, G, accumulate, nullptr, ws, ws_bytes, stream);
}

int64_t gcp_rejection_status_offset(const gcp_tensor* X, const gcp_factors* M, const gcp_sampling* cfg) {
    if (!X || !cfg || X->d < 1 || X->d > GCP_MAX_D) return -1;
    if (cfg->sampler != GCP_SAMPLER_STRATIFIED || cfg->q <= 0) return -1;
    char* const base = reinterpret_cast<char*>(size_t(1) << 40);  // carve against a fake base, keep offsets
    if (!M) {
        Carver c;
        RejScratch rs{};
        sample_ws(X, cfg, c, base, &rs);
        return rs.status ? (int64_t)(reinterpret_cast<char*>(rs.status) - base) : -1;
    }
    if (M->rank < 1) return -1;
    FusedLayout f{};
    fused_ws(X, M, cfg, base, &f);
    return f.rs.status ? (int64_t)(reinterpret_cast<char*>(f.rs.status) - base) : -1;
}

size_t gcp_sampled_grad_workspace_bytes(const gcp_tensor* X, const gcp_factors* M, const gcp_sampling* cfg) {
    if (!X || !M || !cfg || X->d < 1 || X->d > GCP_MAX_D || M->rank < 1) return 0;
    return fused_ws(X, M, cfg, nullptr, nullptr);
}

gcp_status gcp_sampled_grad(gcp_loss loss, const gcp_tensor* X, const gcp_factors* M, const gcp_sampling* cfg,
                            double eps, void* const* G, double* loss_sum, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_loss(loss)) return st;
    if (gcp_status st = check_tensor(X)) return st;
    if (gcp_status st = check_sampling(X, cfg)) return st;
    if (gcp_status st = check_factors(X, M)) return st;
    if (!G) return set_error(GCP_ERR_INVALID_ARG, "G is NULL");
    for (int k = 0; k < X->d; ++k)
        if (!G[k]) return set_error(GCP_ERR_INVALID_ARG, "G[" + std::to_string(k) + "] is NULL");
    return sampled_common(loss, X, M, cfg, eps, G, loss_sum, ws, ws_bytes, nullptr, stream);
}

gcp_status gcp_sampled_grad_noalloc(gcp_loss loss, const gcp_tensor* X, const gcp_factors* M,
                                    const gcp_sampling* cfg, double eps, void* const* G, double* loss_sum,
                                    hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_loss(loss)) return st;
    if (gcp_status st = check_tensor(X)) return st;
    if (gcp_status st = check_sampling(X, cfg)) return st;
    if (gcp_status st = check_factors(X, M)) return st;
    if (!G) return set_error(GCP_ERR_INVALID_ARG, "G is NULL");
    for (int k = 0; k < X->d; ++k)
        if (!G[k]) return set_error(GCP_ERR_INVALID_ARG, "G[" + std::to_string(k) + "] is NULL");
    const size_t need = fused_ws(X, M, cfg, nullptr, nullptr);
    if (need > GCP_NOALLOC_SCRATCH_BYTES)
        return set_error(GCP_ERR_WORKSPACE, "gcp_sampled_grad_noalloc: the call needs " + std::to_string(need) +
                                                " bytes of scratch, above the static " +
                                                std::to_string((size_t)GCP_NOALLOC_SCRATCH_BYTES) +
                                                "; use gcp_sampled_grad with a workspace");
    void* ws = nullptr;
    if (gcp_status st = scratch_address(&ws)) return st;
    return sampled_common(loss, X, M, cfg, eps, G, loss_sum, ws, GCP_NOALLOC_SCRATCH_BYTES, nullptr, stream);
}

gcp_status gcp_sampled_adam_step(gcp_loss loss, const gcp_tensor* X, const gcp_factors* M, const gcp_sampling* cfg,
                                 double eps, void* A, float* A_master, void* B, void* C, int64_t* state,
                                 double alpha, double beta1, double beta2, double adam_eps, double lower,
                                 gcp_eps_mode eps_mode, void* const* G, double* loss_sum, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_loss(loss)) return st;
    if (gcp_status st = check_tensor(X)) return st;
    if (gcp_status st = check_sampling(X, cfg)) return st;
    if (gcp_status st = check_factors(X, M)) return st;
    int64_t P = 0;
    for (int k = 0; k < X->d; ++k) P += X->dims[k] * M->rank;
    if (gcp_status st = check_adam((gcp_dtype)M->dtype, P, A, A_master, B, C, state, alpha, beta1, beta2, adam_eps,
                                   eps_mode))
        return st;
    // the gathers must read the very parameters the step updates: A_k = A + offset_k
    const size_t esz = M->dtype == GCP_F64 ? 8 : (M->dtype == GCP_F32 ? 4 : 2);
    int64_t off = 0;
    for (int k = 0; k < X->d; ++k) {
        if (M->A[k] != static_cast<const char*>(A) + off * esz)
            return set_error(GCP_ERR_INVALID_ARG, "M->A[k] must be the mode-k block of the flat parameter array A");
        off += X->dims[k] * M->rank;
    }
    const AdamParams ap{A, A_master, B, C, state, alpha, beta1, beta2, adam_eps, lower, (int)eps_mode};
    return sampled_common(loss, X, M, cfg, eps, G, loss_sum, ws, ws_bytes, &ap, stream);
}

gcp_status gcp_bf16_round(int64_t P, const float* src, void* dst, hipStream_t stream) {
    clear_error();
    if (P < 0) return set_error(GCP_ERR_INVALID_ARG, "P must be >= 0");
    if (P > 0 && (!src || !dst)) return set_error(GCP_ERR_INVALID_ARG, "src and dst must be non-NULL");
    return launch_bf16_round(P, src, dst, stream);
}

gcp_status gcp_adam_step(int64_t P, gcp_dtype dtype, void* A, float* A_master, const void* G, void* B, void* C,
                         int64_t* state, double alpha, double beta1, double beta2, double eps, double lower,
                         gcp_eps_mode eps_mode, hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_adam(dtype, P, A, A_master, B, C, state, alpha, beta1, beta2, eps, eps_mode)) return st;
    if (P > 0 && !G) return set_error(GCP_ERR_INVALID_ARG, "G must be non-NULL");
    return launch_adam(P, dtype, A, A_master, G, B, C, state, alpha, beta1, beta2, eps, lower, eps_mode, stream);
}

gcp_status gcp_batched_create(const gcp_problem* problems, int32_t count, const gcp_batch_tuning* tune,
                              gcp_batch** batch) {
    clear_error();
    return batch_create(problems, count, tune, batch, check_problem);
}

size_t gcp_batched_workspace_bytes(const gcp_batch* batch) { return batch_ws_bytes(batch); }

gcp_status gcp_batched_prepare(gcp_batch* batch, void* ws, size_t ws_bytes, hipStream_t stream) {
    clear_error();
    return batch_prepare(batch, ws, ws_bytes, stream);
}

gcp_status gcp_batched_grad(gcp_batch* batch, uint64_t* iteration_counter, hipStream_t stream) {
    clear_error();
    hipEvent_t ev0, ev1;
    timing_take(stream, &ev0, &ev1);
    return batch_step(batch, nullptr, iteration_counter, ev0, ev1, stream);
}

gcp_status gcp_batched_adam_step(gcp_batch* batch, int64_t* state, uint64_t* iteration_counter, double alpha,
                                 double beta1, double beta2, double adam_eps, gcp_eps_mode eps_mode,
                                 hipStream_t stream) {
    clear_error();
    if (!state) return set_error(GCP_ERR_INVALID_ARG, "state is NULL");
    if (eps_mode != GCP_EPS_INSIDE_SQRT && eps_mode != GCP_EPS_OUTSIDE_SQRT)
        return set_error(GCP_ERR_INVALID_ARG, "eps_mode is not a gcp_eps_mode");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return set_error(GCP_ERR_INVALID_ARG, "beta1 and beta2 must be in [0, 1)");
    if (!(adam_eps >= 0.0) || !(alpha >= 0.0)) return set_error(GCP_ERR_INVALID_ARG, "alpha and eps must be >= 0");
    const AdamParams ap{nullptr, nullptr, nullptr, nullptr, state, alpha, beta1, beta2, adam_eps, 0.0, (int)eps_mode};
    hipEvent_t ev0, ev1;
    timing_take(stream, &ev0, &ev1);
    return batch_step(batch, &ap, iteration_counter, ev0, ev1, stream);
}

gcp_status gcp_batched_plan(const gcp_batch* batch, int64_t* n_blocks, int64_t* n_units, int64_t* block_ptr,
                            int32_t* unit_problem, int64_t* unit_items) {
    clear_error();
    return batch_plan(batch, n_blocks, n_units, block_ptr, unit_problem, unit_items);
}

void gcp_batched_destroy(gcp_batch* batch) { batch_destroy(batch); }

gcp_status gcp_batched_graph_capture(gcp_batch* batch, int32_t steps, int64_t* state, uint64_t* iteration_counter,
                                     double alpha, double beta1, double beta2, double adam_eps,
                                     gcp_eps_mode eps_mode) {
    clear_error();
    if (!state) return set_error(GCP_ERR_INVALID_ARG, "state is NULL");
    if (eps_mode != GCP_EPS_INSIDE_SQRT && eps_mode != GCP_EPS_OUTSIDE_SQRT)
        return set_error(GCP_ERR_INVALID_ARG, "eps_mode is not a gcp_eps_mode");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return set_error(GCP_ERR_INVALID_ARG, "beta1 and beta2 must be in [0, 1)");
    if (!(adam_eps >= 0.0) || !(alpha >= 0.0)) return set_error(GCP_ERR_INVALID_ARG, "alpha and eps must be >= 0");
    const AdamParams ap{nullptr, nullptr, nullptr, nullptr, state, alpha, beta1, beta2, adam_eps, 0.0, (int)eps_mode};
    return batch_graph_capture(batch, steps, &ap, iteration_counter);
}

gcp_status gcp_batched_graph_launch(gcp_batch* batch, hipStream_t stream) {
    clear_error();
    return batch_graph_launch(batch, stream);
}

void gcp_batched_graph_destroy(gcp_batch* batch) { batch_graph_destroy(batch); }

// ---------------------------------------------------------------------------
// GCP-Adam driver (Alg. 4): host control flow over the entry points above.
// ---------------------------------------------------------------------------
namespace {

struct FitLayout {
    void* step_ws;
    size_t step_bytes;
    uint32_t* idx;
    void* xval;
    uint8_t* stratum;
    void* ytilde;
    void* sample_ws;
    size_t sample_bytes;
    double* loss_sum;
    void* A_save;
    float* master_save;
    void* B_save;
    void* C_save;
    int64_t* state_save;
    int64_t S_est, P;
    size_t esz, msz;
};

size_t fit_layout(const gcp_tensor* X, const gcp_factors* M, const gcp_fit_options* opt, void* base,
                  FitLayout* L) {
    FitLayout f{};
    int64_t P = 0;
    for (int k = 0; k < X->d; ++k) P += X->dims[k] * M->rank;
    f.P = P;
    f.esz = M->dtype == GCP_F64 ? 8 : (M->dtype == GCP_F32 ? 4 : 2);
    f.msz = M->dtype == GCP_F64 ? 8 : 4;
    const size_t vsz = X->vdtype == GCP_F64 ? 8 : 4;
    f.S_est = opt->est.sampler == GCP_SAMPLER_FULL ? full_count(X)
              : (opt->est.sampler == GCP_SAMPLER_UNIFORM ? opt->est.s : opt->est.p + opt->est.q);
    gcp_sampling grad = opt->grad;
    grad.iteration_counter = nullptr;
    gcp_sampling est = opt->est;
    est.iteration_counter = nullptr;
    f.step_bytes = gcp_sampled_grad_workspace_bytes(X, M, &grad);
    f.sample_bytes = gcp_sample_workspace_bytes(X, &est);
    Carver c;
    f.step_ws = c.take<char>(base, std::max<size_t>(1, f.step_bytes));
    f.idx = c.take<uint32_t>(base, (size_t)std::max<int64_t>(1, f.S_est) * (size_t)X->d);
    f.xval = c.take<char>(base, (size_t)std::max<int64_t>(1, f.S_est) * vsz);
    f.stratum = c.take<uint8_t>(base, (size_t)std::max<int64_t>(1, f.S_est));
    f.ytilde = c.take<char>(base, (size_t)std::max<int64_t>(1, f.S_est) * f.msz);
    f.sample_ws = c.take<char>(base, std::max<size_t>(1, f.sample_bytes));
    f.loss_sum = c.take<double>(base, 1);
    f.A_save = c.take<char>(base, (size_t)std::max<int64_t>(1, P) * f.esz);
    f.master_save = c.take<float>(base, M->dtype == GCP_BF16 ? (size_t)std::max<int64_t>(1, P) : 1);
    f.B_save = c.take<char>(base, (size_t)std::max<int64_t>(1, P) * f.msz);
    f.C_save = c.take<char>(base, (size_t)std::max<int64_t>(1, P) * f.msz);
    f.state_save = c.take<int64_t>(base, 2);
    if (L) *L = f;
    return c.bytes();
}

gcp_status check_fit(const gcp_tensor* X, const gcp_factors* M, const gcp_fit_options* opt) {
    if (!opt) return set_error(GCP_ERR_INVALID_ARG, "opt is NULL");
    if (opt->tau < 1) return set_error(GCP_ERR_INVALID_ARG, "opt->tau must be >= 1");
    if (opt->kappa < 0) return set_error(GCP_ERR_INVALID_ARG, "opt->kappa must be >= 0");
    if (opt->max_epochs < 0) return set_error(GCP_ERR_INVALID_ARG, "opt->max_epochs must be >= 0");
    if (!(opt->nu > 0.0 && opt->nu <= 1.0)) return set_error(GCP_ERR_INVALID_ARG, "opt->nu must be in (0, 1]");
    if (gcp_status st = check_tensor(X)) return st;
    if (gcp_status st = check_sampling(X, &opt->grad)) return st;
    if (gcp_status st = check_sampling(X, &opt->est)) return st;
    if (gcp_status st = check_factors(X, M)) return st;
    return GCP_OK;
}

gcp_status copy_async(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return GCP_OK;
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return set_error(GCP_ERR_HIP, "device copy failed");
    return GCP_OK;
}

}  // namespace

size_t gcp_adam_fit_workspace_bytes(const gcp_tensor* X, const gcp_factors* M, const gcp_fit_options* opt) {
    clear_error();
    if (check_fit(X, M, opt) != GCP_OK) return 0;
    return fit_layout(X, M, opt, nullptr, nullptr);
}

gcp_status gcp_adam_fit(gcp_loss loss, const gcp_tensor* X, const gcp_factors* M, const gcp_fit_options* opt,
                        double eps, void* A, float* A_master, void* B, void* C, int64_t* state, double* history,
                        int8_t* accepted, int32_t* epochs, double* alpha_out, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
    clear_error();
    if (gcp_status st = check_loss(loss)) return st;
    if (gcp_status st = check_fit(X, M, opt)) return st;
    if (!history || !accepted || !epochs) return set_error(GCP_ERR_INVALID_ARG, "history, accepted and epochs are required");
    FitLayout f{};
    const size_t need = fit_layout(X, M, opt, ws, &f);
    if (!ws || ws_bytes < need)
        return set_error(GCP_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    gcp_sampling grad = opt->grad;
    grad.iteration_counter = nullptr;
    gcp_sampling est = opt->est;
    est.iteration_counter = nullptr;
    // the fixed estimation set
    if (gcp_status st = gcp_sample(X, &est, f.idx, f.xval, f.stratum, f.sample_ws, f.sample_bytes, stream)) return st;
    auto estimate = [&](double* F) -> gcp_status {
        if (gcp_status st = launch_fill_zero(f.loss_sum, 1, stream)) return st;
        if (gcp_status st = gcp_loss_grad(loss, X, &est, M, f.idx, f.xval, f.stratum, f.S_est, eps, f.ytilde,
                                          f.loss_sum, stream))
            return st;
        if (hipMemcpyAsync(F, f.loss_sum, sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return set_error(GCP_ERR_HIP, "reading the loss estimate failed");
        return GCP_OK;
    };
    const size_t pa = (size_t)f.P * f.esz, pm = (size_t)f.P * f.msz;
    auto save = [&](bool restore) -> gcp_status {
        // restore = false: parameters -> copies; true: copies -> parameters
        auto cp = [&](void* live, void* copy, size_t bytes) {
            return restore ? copy_async(live, copy, bytes, stream) : copy_async(copy, live, bytes, stream);
        };
        if (gcp_status st = cp(A, f.A_save, pa)) return st;
        if (M->dtype == GCP_BF16)
            if (gcp_status st = cp(A_master, f.master_save, (size_t)f.P * 4)) return st;
        if (gcp_status st = cp(B, f.B_save, pm)) return st;
        if (gcp_status st = cp(C, f.C_save, pm)) return st;
        return cp(state, f.state_save, 2 * sizeof(int64_t));
    };
    double F = 0.0;
    if (gcp_status st = estimate(&F)) return st;
    history[0] = F;
    accepted[0] = 1;
    double alpha = opt->alpha;
    int32_t bad = 0, epoch = 0;
    uint64_t step = 0;
    while (bad <= opt->kappa && epoch < opt->max_epochs) {
        if (gcp_status st = save(false)) return st;
        const double F_old = F;
        for (int32_t j = 0; j < opt->tau; ++j) {
            grad.iteration = opt->grad.iteration + step++;
            if (gcp_status st = gcp_sampled_adam_step(loss, X, M, &grad, eps, A, A_master, B, C, state, alpha,
                                                      opt->beta1, opt->beta2, opt->adam_eps, opt->lower,
                                                      (gcp_eps_mode)opt->eps_mode, nullptr, nullptr, f.step_ws,
                                                      f.step_bytes, stream))
                return st;
        }
        if (gcp_status st = estimate(&F)) return st;
        ++epoch;
        history[epoch] = F;
        if (F > F_old) {
            // undo the epoch: parameters, moments and step count; smaller steps
            if (gcp_status st = save(true)) return st;
            F = F_old;
            alpha *= opt->nu;
            ++bad;
            accepted[epoch] = 0;
        } else {
            accepted[epoch] = 1;
        }
    }
    if (hipStreamSynchronize(stream) != hipSuccess) return set_error(GCP_ERR_HIP, "hipStreamSynchronize failed");
    *epochs = epoch;
    if (alpha_out) *alpha_out = alpha;
    return GCP_OK;
}

gcp_status gcp_timing_start(int64_t max_launches) {
    clear_error();
    if (max_launches < 1 || max_launches > (1 << 20))
        return set_error(GCP_ERR_INVALID_ARG, "max_launches must be in [1, 2^20]");
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (g_timing.armed) return set_error(GCP_ERR_INVALID_ARG, "a timing session is already running");
    g_timing.start.assign((size_t)max_launches, nullptr);
    g_timing.stop.assign((size_t)max_launches, nullptr);
    for (int64_t e = 0; e < max_launches; ++e) {
        if (hipEventCreate(&g_timing.start[e]) != hipSuccess || hipEventCreate(&g_timing.stop[e]) != hipSuccess) {
            for (auto& ev : g_timing.start) if (ev) (void)hipEventDestroy(ev);
            for (auto& ev : g_timing.stop) if (ev) (void)hipEventDestroy(ev);
            g_timing.start.clear();
            g_timing.stop.clear();
            return set_error(GCP_ERR_HIP, "hipEventCreate failed");
        }
    }
    g_timing.used = 0;
    g_timing.armed = true;
    return GCP_OK;
}

gcp_status gcp_timing_stop(double* total_ms, int64_t* launches) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (!g_timing.armed) return set_error(GCP_ERR_INVALID_ARG, "no timing session is running");
    double sum = 0.0;
    gcp_status st = GCP_OK;
    for (size_t e = 0; e < g_timing.used; ++e) {
        float ms = 0.f;
        if (hipEventSynchronize(g_timing.stop[e]) != hipSuccess ||
            hipEventElapsedTime(&ms, g_timing.start[e], g_timing.stop[e]) != hipSuccess) {
            st = set_error(GCP_ERR_HIP, "reading timing events failed");
            break;
        }
        sum += ms;
    }
    for (auto& ev : g_timing.start) (void)hipEventDestroy(ev);
    for (auto& ev : g_timing.stop) (void)hipEventDestroy(ev);
    if (total_ms) *total_ms = sum;
    if (launches) *launches = (int64_t)g_timing.used;
    g_timing.start.clear();
    g_timing.stop.clear();
    g_timing.used = 0;
    g_timing.armed = false;
    return st;
}

}  // extern "C"
