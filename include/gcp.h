/*
 * gcp.h -- C ABI of libgcp: the sampled gradient of generalized CP (GCP)
 * tensor decomposition on AMD Instinct MI355X (gfx950).
 *
 * Method: Kolda & Hong, "Stochastic Gradients for Large-Scale Tensor
 * Decomposition".  One stochastic gradient draws sample indices (uniform,
 * stratified with rejection, or semi-stratified; Sec. 4.1-4.3, Alg. 1-3),
 * evaluates the CP model at them (eq. Mdef), applies the weighted loss
 * derivative (eq. Y with the per-stratum weights of Sec. 4.1-4.3) and
 * accumulates every mode's gradient as a sparse MTTKRP, G_k = Ytilde_(k) Z_k
 * (eqs. mttkrp, Gks).  The Adam step with projection follows (Alg. 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Indices are 0-based (the paper counts from 1).  A multi-index i =
 *   (i_1..i_d) has the row-major linear key L = ((i_1 n_2 + i_2) n_3 + ...).
 * - Factor matrix A_k is n_k x r, row-major (a row is r contiguous values).
 * - Dense X is row-major (last mode fastest).  COO X is nnz x d uint32 mode
 *   indices, row-major, plus nnz values; no coordinate may appear twice.
 * - Every pointer argument except the descriptor structs themselves is DEVICE
 *   memory owned by the caller.  The library never allocates; each call that
 *   needs scratch space takes a caller-owned workspace whose size is given by
 *   the matching *_workspace_bytes() query.
 * - Every call is asynchronous on the caller's stream and validates its
 *   arguments on the host only (no device synchronisation).  On failure it
 *   returns a non-zero gcp_status, launches nothing, and gcp_last_error()
 *   returns a message for the calling thread.
 * - Random draws: Philox4x64-10 (Salmon et al., SC'11) with key =
 *   (seed, problem_id) and counter = (j, iteration, purpose, block); word k of
 *   sample j's stream is word k mod 4 of block k / 4, and randi(n) =
 *   floor(w * n / 2^64).  Purposes: 0 uniform draws and semi-stratified
 *   "zeros", 1 nonzero picks, 2 rejection candidates.  The same (seed,
 *   problem_id, iteration) always yields the same samples.
 * - Sample order: for stratified and semi-stratified sampling the p nonzero
 *   samples come first (j = 0..p-1), then the q zero samples.  Stratified
 *   zeros are the first q accepted rejection candidates in counter order.
 */
#ifndef GCP_H
#define GCP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCP_ABI_VERSION 1
#define GCP_MAX_D 8        /* modes per tensor */
#define GCP_MAX_RANK 256   /* CP rank r (above 64, the gathers take 2 or 4 columns per lane) */

typedef enum gcp_status {
    GCP_OK = 0,
    GCP_ERR_INVALID_ARG = 1,   /* a null pointer, bad size, or inconsistent argument */
    GCP_ERR_UNSUPPORTED = 2,   /* valid by the method but outside what this build handles */
    GCP_ERR_HIP = 3,           /* a HIP runtime call failed (launch error) */
    GCP_ERR_WORKSPACE = 4      /* workspace smaller than the *_workspace_bytes() query */
} gcp_status;

typedef enum gcp_dtype { GCP_F32 = 0, GCP_F64 = 1, GCP_BF16 = 2 } gcp_dtype;

/* Losses f(x, m) and g = df/dm (paper, Sec. 1, 4.2 and 5.3).  eps is added
 * where the paper divides by m or takes log m or a power of m (u = m + eps):
 *   GAUSSIAN        f = (x - m)^2,                  g = 2 (m - x)
 *   BERNOULLI_ODDS  f = log(m + 1) - x log u,        g = 1/(m + 1) - x/u
 *   POISSON         f = m - x log u,                 g = 1 - x/u
 *   GAMMA           f = x/u + log u,                 g = 1/u - x/u^2
 *   BETA_HALF       f = 2 u^(1/2) + 2 x u^(-1/2),    g = u^(-1/2) - x u^(-3/2)
 * (GAMMA: shape-1 Gamma data, Sec. 1 and the Sec. 5.2 test problems;
 * BETA_HALF: beta-divergence with beta = 1/2 up to terms free of m, Sec. 5.3.) */
typedef enum gcp_loss {
    GCP_LOSS_GAUSSIAN = 0,
    GCP_LOSS_BERNOULLI_ODDS = 1,
    GCP_LOSS_POISSON = 2,
    GCP_LOSS_GAMMA = 3,
    GCP_LOSS_BETA_HALF = 4
} gcp_loss;

/* Samplers: UNIFORM (Sec. 4.1, Alg. 1; s draws with replacement, weight
 * omega/s); STRATIFIED (Sec. 4.2, Alg. 2; p nonzeros with weight eta/p, q zeros
 * by rejection with weight zeta/q); SEMI_STRATIFIED (Sec. 4.3, Alg. 3; p
 * nonzeros with weight eta/p and derivative g(x,m) - g(0,m), q uniform
 * "zeros" with x := 0 and weight omega/q); FULL (every entry once, sample c
 * being entry c in row-major order, weight 1: the exact, non-stochastic
 * gradient and loss of eqs. gcp, Y, Gk; s, p, q unused; a COO tensor needs
 * nz_table).  omega = prod n_k, eta = nnz, zeta = omega - eta. */
typedef enum gcp_sampler {
    GCP_SAMPLER_UNIFORM = 0,
    GCP_SAMPLER_STRATIFIED = 1,
    GCP_SAMPLER_SEMI_STRATIFIED = 2,
    GCP_SAMPLER_FULL = 3
} gcp_sampler;

/* Per-sample stratum codes written by gcp_sample and read by gcp_loss_grad.
 * ytilde = w * g(x, m) except NZ_CORR, where ytilde = w * (g(x,m) - g(0,m)). */
typedef enum gcp_stratum {
    GCP_STRATUM_UNIFORM = 0,    /* w = omega / s  */
    GCP_STRATUM_NZ = 1,         /* w = eta / p    */
    GCP_STRATUM_ZERO = 2,       /* w = zeta / q, x = 0 */
    GCP_STRATUM_NZ_CORR = 3,    /* w = eta / p    */
    GCP_STRATUM_SEMI_ZERO = 4   /* w = omega / q, x := 0 */
} gcp_stratum;

typedef enum gcp_format { GCP_DENSE = 0, GCP_COO = 1 } gcp_format;

/* Alg. 4 writes A <- A - alpha Bhat / sqrt(Chat + eps) (INSIDE, the default);
 * OUTSIDE is the Kingma-Ba form A <- A - alpha Bhat / (sqrt(Chat) + eps). */
typedef enum gcp_eps_mode { GCP_EPS_INSIDE_SQRT = 0, GCP_EPS_OUTSIDE_SQRT = 1 } gcp_eps_mode;

/* The data tensor X (Sec. 3.2: dense storage n^d, coordinate storage (d+1) nnz). */
typedef struct gcp_tensor {
    int32_t d;                   /* number of modes, 1..GCP_MAX_D */
    int32_t format;              /* gcp_format */
    int32_t vdtype;              /* value type: GCP_F32 or GCP_F64 */
    int32_t reserved;            /* set to 0 */
    int64_t dims[GCP_MAX_D];     /* n_1..n_d, each in [1, 2^32 - 1]; prod < 2^63 */
    const void *values;          /* dense: prod(dims) values; COO: nnz values */
    const uint32_t *coo_idx;     /* COO: nnz x d indices; NULL for dense */
    int64_t nnz;                 /* COO: stored nonzeros (eta), < 2^32; dense: 0 */
    const void *nz_table;        /* COO: table from gcp_nz_index_build (needed by
                                    STRATIFIED and by UNIFORM on COO); else NULL */
    int64_t nz_slots;            /* slots of nz_table */
    const uint32_t *nz_bitmap;   /* COO, optional: bit L of the bitmap from
                                    gcp_nz_bitmap_build is set iff X is nonzero at
                                    linear key L.  When given, the rejection test of
                                    STRATIFIED reads it instead of the hash table
                                    (one load instead of a probe sequence). */
    const void *weights;         /* optional entry weights w_i of the weighted
                                    objective sum_i w_i f(x_i, m_i) (eq. wgcp,
                                    Sec. 4.4), type vdtype: dense, one per entry;
                                    COO, one per stored entry.  NULL: all 1. */
    double w_zero;               /* with weights on a COO tensor: the weight of
                                    every entry it does not store (zeros; 0 for
                                    missing data).  Ignored without weights or
                                    for dense tensors. */
} gcp_tensor;

/* The factor matrices A_1..A_d of the CP model (eq. Mdef). */
typedef struct gcp_factors {
    int32_t dtype;               /* storage: GCP_F32, GCP_F64 or GCP_BF16 */
    int32_t reserved;            /* set to 0 */
    int64_t rank;                /* r, 1..GCP_MAX_RANK */
    const void *A[GCP_MAX_D];    /* A[k]: dims[k] x rank, row-major, device; each
                                    block below 4 GiB (else GCP_ERR_UNSUPPORTED) */
} gcp_factors;

/* What one stochastic gradient samples. */
typedef struct gcp_sampling {
    int32_t sampler;             /* gcp_sampler */
    int32_t reserved;            /* set to 0 */
    int64_t s;                   /* UNIFORM: number of samples (> 0) */
    int64_t p;                   /* STRATIFIED / SEMI: nonzero samples (>= 0) */
    int64_t q;                   /* STRATIFIED / SEMI: zero samples (>= 0) */
    uint64_t seed;               /* Philox key word 0 */
    uint64_t problem_id;         /* Philox key word 1 */
    uint64_t iteration;          /* Philox counter word 1: one value per gradient */
    double rho;                  /* STRATIFIED: rejection candidates are drawn in a
                                    first batch of ceil(rho * q * omega / zeta);
                                    rho <= 0 selects 1.1 (Sec. 4.2, App. B).  The
                                    samples never depend on rho. */
    uint64_t *iteration_counter; /* nullable device pointer.  When set, the draws use
                                    iteration + *iteration_counter (read on the
                                    device) and the call adds 1 to
                                    *iteration_counter after its last read, so a
                                    captured HIP graph of the call draws fresh
                                    samples on every replay.  Calls sharing a
                                    counter must not overlap. */
} gcp_sampling;

/* Message describing the last failure on the calling thread ("" if none). */
const char *gcp_last_error(void);
int gcp_abi_version(void);

/* ---------------------------------------------------------------------------
 * Nonzero index (Sec. 4.2: rejection needs a membership test of the sampled
 * index against the list of nonzeros; the paper suggests hash tables).
 * An open-addressing table of the nonzeros' linear keys and their COO
 * positions: 8-byte keys then 4-byte positions, 12 bytes per slot.
 * gcp_nz_table_slots(nnz) returns the power of two >= 2 nnz (at least 64) to
 * use.  gcp_nz_index_build clears and fills `table` (gcp_nz_table_bytes(slots)
 * bytes of device memory) from X's coordinates; X->nz_table is not read.
 * Rebuild whenever X's coordinates change. */
int64_t gcp_nz_table_slots(int64_t nnz);
size_t gcp_nz_table_bytes(int64_t slots);
gcp_status gcp_nz_index_build(const gcp_tensor *X, void *table, int64_t slots,
                              hipStream_t stream);

/* Exact membership bitmap of X's nonzeros: prod(dims) bits (32-bit words).
 * gcp_nz_bitmap_bytes returns its size in bytes (0 if X is not COO);
 * gcp_nz_bitmap_build clears and fills `bitmap` (device memory of at least
 * that size) from X's coordinates. */
size_t gcp_nz_bitmap_bytes(const gcp_tensor *X);
gcp_status gcp_nz_bitmap_build(const gcp_tensor *X, uint32_t *bitmap, size_t bytes,
                               hipStream_t stream);

/* ---------------------------------------------------------------------------
 * gcp_set_cols_per_lane -- process-wide tuning choice of how the gradient
 * kernels lay a sample's r rank columns (eq. Mdef) over a wave: a sample
 * takes the power of two lps >= ceil(r / cpl) lanes and lane j of them the
 * cpl columns j, j + lps, ... (cpl = 1, 2 or 4).  0 (the default) picks by rank: 1 for r <= 4, 2
 * for r <= 16, else 4.  cpl = 1 carries r <= 64, 2 carries 4 < r <= 128, 4
 * carries 4 < r <= 256; a choice that does not fit a call's rank falls back
 * to the automatic one.  Results do not depend on it beyond floating-point
 * summation order.  Returns GCP_ERR_INVALID_ARG for other values. */
gcp_status gcp_set_cols_per_lane(int32_t cpl);

/* ---------------------------------------------------------------------------
 * gcp_sample -- the sampling lines of Alg. 1 (uniform), Alg. 2 (nonzero picks
 * xi = randi(eta) and the rejection loop for zeros) and Alg. 3 (nonzero picks
 * and "zeros" drawn without rejection).
 * Writes S = s (UNIFORM) or p + q samples:
 *   idx[S * d]   uint32 mode indices of each sample
 *   xval[S]      X at the sample (X->vdtype); 0 for the zero strata
 *   stratum[S]   gcp_stratum code of each sample
 * STRATIFIED needs q = 0 or zeta > 0, and X->nz_table or X->nz_bitmap.  UNIFORM on a COO
 * tensor looks values up through X->nz_table.  ws: gcp_sample_workspace_bytes
 * bytes (0 except for STRATIFIED).  The rejection loop is exact: if the first
 * candidate batch holds fewer than q zeros, a device-side loop continues the
 * counter stream until q are found (no host round trip).  That loop examines
 * at most 2^22 further candidates; a configuration whose first batch
 * (cfg->rho times q omega / zeta) plus that cap falls short of q omega / zeta
 * plus eight standard deviations of the candidate count (App. B) is refused
 * with GCP_ERR_UNSUPPORTED, so the cap is reached with probability below
 * 1e-15.  If it is reached, the rejection status word reads 1 (see
 * gcp_rejection_status_offset): gcp_sample leaves the zero slots past the
 * last one drawn unwritten, and the fused calls use the zeros drawn so far. */
size_t gcp_sample_workspace_bytes(const gcp_tensor *X, const gcp_sampling *cfg);
gcp_status gcp_sample(const gcp_tensor *X, const gcp_sampling *cfg,
                      uint32_t *idx, void *xval, uint8_t *stratum,
                      void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * gcp_loss_grad -- model entries and weighted derivatives at given samples
 * (Alg. 1-3: m_i = sum_j prod_k A_k(i_k, j), then ytilde_i += w g(x_i, m_i)).
 * Weights come from the stratum codes, X's dims and nnz, and cfg's s, p, q,
 * times the entry weights of X when it has them (a weighted COO tensor then
 * needs nz_table, through which a sample's stored weight is found).
 *   ytilde[S]   out; F64 when M->dtype is GCP_F64, else F32 (computed in F32)
 *   loss_sum    nullable device double; the call ADDS the weighted loss
 *               estimate sum_i w f(x_i, m_i) (eqs. Fhat, Fhat-strat; for the
 *               NZ_CORR stratum w (f(x,m) - f(0,m))).
 * Duplicate samples are independent entries (their contributions add). */
gcp_status gcp_loss_grad(gcp_loss loss, const gcp_tensor *X, const gcp_sampling *cfg,
                         const gcp_factors *M, const uint32_t *idx, const void *xval,
                         const uint8_t *stratum, int64_t S, double eps,
                         void *ytilde, double *loss_sum, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * gcp_mttkrp -- the sparse MTTKRP of every mode over S samples (eqs. mttkrp,
 * Gks; Alg. 1-3 last loop): G_k(i_k, :) += ytilde_i * prod_{k' != k} A_k'(i_k', :).
 *   G[k]        out, dims[k] x rank row-major; F64 when M->dtype is GCP_F64,
 *               else F32.  Overwritten unless `accumulate` is non-zero.
 * Accumulation: each workgroup sums the modes whose rows fit in its LDS in
 * FP64 (or, for FP32/BF16 factors whose FP64 partial does not fit, in FP32)
 * and publishes one partial (FP32; FP64 for FP64 factors); the partials are
 * summed in FP64 in a fixed order.  Longer modes are summed with FP64 device
 * atomics.
 * The workspace (gcp_mttkrp_workspace_bytes(X, M, S) bytes) holds both. */
size_t gcp_mttkrp_workspace_bytes(const gcp_tensor *X, const gcp_factors *M, int64_t S);
gcp_status gcp_mttkrp(const gcp_tensor *X, const gcp_factors *M, const uint32_t *idx,
                      const void *ytilde, int64_t S, void *const *G, int accumulate,
                      void *ws, size_t ws_bytes, hipStream_t stream);
/* gcp_mttkrp_scaled -- gcp_mttkrp with every G_k scaled by the device scalar
 * *scale (nullable: 1), read on the device when the reduction runs: the
 * adjoint of a sampled loss F(A) (eq. Gks) times an upstream derivative that
 * lives in device memory, with no host round trip.  With accumulate, G_k +=
 * scale * MTTKRP. */
gcp_status gcp_mttkrp_scaled(const gcp_tensor *X, const gcp_factors *M, const uint32_t *idx,
                             const void *ytilde, int64_t S, void *const *G, int accumulate,
                             const double *scale, void *ws, size_t ws_bytes, hipStream_t stream);

/* Byte offset, in the workspace of a STRATIFIED call with q > 0, of the
 * rejection status word (uint32): 0 once the call has drawn all q zeros, 1 if
 * the device refill stopped at its cap (Sec. 4.2, Alg. 2; see gcp_sample).
 * M == NULL: the workspace of gcp_sample; otherwise that of gcp_sampled_grad
 * and gcp_sampled_adam_step with these factors.  -1 when the call has no
 * rejection step.  The word is written on the call's stream; read it after
 * the call completes. */
int64_t gcp_rejection_status_offset(const gcp_tensor *X, const gcp_factors *M, const gcp_sampling *cfg);

/* ---------------------------------------------------------------------------
 * gcp_sampled_grad -- the whole stochastic gradient of Alg. 1 / 2 / 3 in as
 * few launches as possible: draws, model entries, derivatives and the MTTKRP
 * of every mode, without writing the samples out.  Same samples as
 * gcp_sample with the same cfg; G equal to gcp_sample -> gcp_loss_grad ->
 * gcp_mttkrp up to floating-point summation order.  G and loss_sum as in
 * gcp_mttkrp and gcp_loss_grad (G is overwritten). */
size_t gcp_sampled_grad_workspace_bytes(const gcp_tensor *X, const gcp_factors *M,
                                        const gcp_sampling *cfg);
gcp_status gcp_sampled_grad(gcp_loss loss, const gcp_tensor *X, const gcp_factors *M,
                            const gcp_sampling *cfg, double eps, void *const *G,
                            double *loss_sum, void *ws, size_t ws_bytes, hipStream_t stream);

/* gcp_sampled_grad_noalloc -- gcp_sampled_grad for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels, with the workspace taken
 * from a static device array of GCP_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends.  The caller still
 * passes X, M, G and loss_sum.  The call allocates nothing; the first call on
 * a device looks the array up there (hipGetSymbolAddress).  A problem whose
 * gcp_sampled_grad_workspace_bytes exceeds the array is refused with
 * GCP_ERR_WORKSPACE before any launch.  Every call on a device shares that
 * device's array, and each call clears what must start at zero: calls that
 * overlap on one device (two streams) race, so serialise them. */
#define GCP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
gcp_status gcp_sampled_grad_noalloc(gcp_loss loss, const gcp_tensor *X, const gcp_factors *M,
                                    const gcp_sampling *cfg, double eps, void *const *G,
                                    double *loss_sum, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * gcp_sampled_adam_step -- one iteration of Alg. 4's inner loop: the
 * stochastic gradient of gcp_sampled_grad followed by the Adam step of
 * gcp_adam_step on all modes, with the gradient reduction and the update
 * fused into one kernel.  Samples, gradient and update equal
 * gcp_sampled_grad followed by gcp_adam_step up to floating-point order.
 *   A          the flat parameter array updated by the step (dtype M->dtype,
 *              sum_k n_k r values); M->A[k] must point at mode k's block of it
 *              (A + offset_k), so the gradient is taken at the same A.
 *   A_master, B, C, state, alpha, beta1, beta2, adam_eps, lower, eps_mode
 *              as in gcp_adam_step.
 *   G          nullable; when given, G[k] (nullable entries) receive the
 *              gradient as in gcp_sampled_grad.
 *   ws         gcp_sampled_grad_workspace_bytes(X, M, cfg) bytes. */
gcp_status gcp_sampled_adam_step(gcp_loss loss, const gcp_tensor *X, const gcp_factors *M,
                                 const gcp_sampling *cfg, double eps, void *A, float *A_master,
                                 void *B, void *C, int64_t *state, double alpha, double beta1,
                                 double beta2, double adam_eps, double lower,
                                 gcp_eps_mode eps_mode, void *const *G, double *loss_sum,
                                 void *ws, size_t ws_bytes, hipStream_t stream);

/* gcp_bf16_round -- dst[e] = src[e] rounded to bf16 (round to nearest, ties
 * to even), e < P: the BF16 gather copy of FP32 master factors (the storage
 * reading of the BF16 factors; the same rounding gcp_adam_step applies after
 * each update).  dst holds P uint16 bf16 values. */
gcp_status gcp_bf16_round(int64_t P, const float *src, void *dst, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * gcp_adam_step -- one Adam step with projection over P parameters at once
 * (Alg. 4: B <- b1 B + (1-b1) G; C <- b2 C + (1-b2) G^2; Bhat = B/(1-b1^t);
 * Chat = C/(1-b2^t); A <- max(A - alpha Bhat / sqrt(Chat + eps), lower)).
 * All modes' factors are updated together from gradients taken at the same
 * A, so A, G, B, C are flat arrays covering sum_k n_k r parameters.
 *   dtype GCP_F64: A, G, B, C double.  GCP_F32: float.  GCP_BF16: A is the
 *   bf16 copy used for gathers, A_master the float master that is updated
 *   (then rounded to nearest even into A); G, B, C float.
 *   state[2]  device int64: state[0] is t, the number of steps taken so far;
 *             state[1] is internal and must be 0 between calls.  Zero both
 *             before the first step.  The step uses t + 1 (so the first step
 *             divides by 1 - b^1) and leaves state[0] = t + 1, all on device.
 *   lower     projection bound; -INFINITY for none.
 * Calls on one state must not overlap. */
gcp_status gcp_adam_step(int64_t P, gcp_dtype dtype, void *A, float *A_master,
                         const void *G, void *B, void *C, int64_t *state,
                         double alpha, double beta1, double beta2, double eps,
                         double lower, gcp_eps_mode eps_mode, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * gcp_adam_fit -- GCP-Adam (Alg. 4) on one problem.  The loss is first
 * estimated on one fixed sample set (EstObj: the weighted sum of f over the
 * set, eqs. Fhat and Fhat-strat; `est` is drawn once).  Each epoch saves the
 * parameters, moments and step count, takes `tau` fused sampled Adam steps
 * (gcp_sampled_adam_step; the j-th step of the whole fit draws with
 * iteration grad.iteration + j, so steps of an undone epoch are not redrawn)
 * and estimates the loss again.  If the estimate rose, the epoch is undone
 * (parameters, moments and step count restored, the estimate reverts), the
 * learning rate is multiplied by nu and the count of bad epochs grows; the fit
 * stops once that count exceeds kappa, or after max_epochs epochs.
 *   A, A_master, B, C, state  as in gcp_sampled_adam_step (M->A[k] must be the
 *               mode blocks of A); updated in place.
 *   history     host, max_epochs + 1 doubles: [0] the first estimate, [e] the
 *               estimate after epoch e (before any undo).
 *   accepted    host, max_epochs + 1 bytes: 1 if epoch e was kept ([0] = 1).
 *   epochs      host out: the number of epochs run.
 *   alpha_out   host out (nullable): the final learning rate.
 * The workspace holds the fused step's workspace, the estimation samples and
 * the copies for undo (gcp_adam_fit_workspace_bytes).  The call synchronises
 * `stream` once per epoch to read the estimate; it returns when the fit ends. */
typedef struct gcp_fit_options {
    gcp_sampling grad;           /* stochastic-gradient draws (iteration_counter ignored) */
    gcp_sampling est;            /* the fixed estimation sample set */
    double alpha;                /* learning rate (0.01 in the paper) */
    double beta1, beta2, adam_eps;
    double lower;                /* projection bound; -INFINITY for none */
    double nu;                   /* learning-rate factor after a bad epoch (0.1) */
    int32_t eps_mode;            /* gcp_eps_mode */
    int32_t tau;                 /* steps per epoch (1000 in the paper), >= 1 */
    int32_t kappa;               /* bad epochs tolerated (1), >= 0 */
    int32_t max_epochs;          /* hard cap on epochs, >= 0 */
} gcp_fit_options;

size_t gcp_adam_fit_workspace_bytes(const gcp_tensor *X, const gcp_factors *M,
                                    const gcp_fit_options *opt);
gcp_status gcp_adam_fit(gcp_loss loss, const gcp_tensor *X, const gcp_factors *M,
                        const gcp_fit_options *opt, double eps, void *A, float *A_master,
                        void *B, void *C, int64_t *state, double *history, int8_t *accepted,
                        int32_t *epochs, double *alpha_out, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batches of independent problems: one persistent gradient launch and one
 * reduction + Adam launch advance every problem of the batch by one step of
 * Alg. 4's inner loop.  The persistent workgroups share the batch's samples
 * by estimated cost (gcp_batch_schedule), so problems of very different sizes
 * finish together.
 *
 * gcp_problem describes one problem: its data X, factors M (M.A[k] must be
 * the mode-k blocks of the flat array A), sampling cfg (UNIFORM or
 * SEMI_STRATIFIED; STRATIFIED is refused with GCP_ERR_UNSUPPORTED, since its
 * zeros come from a rejection pass whose counts must be scanned before the
 * gradient launch (Alg. 2), a third launch per step, while semi-stratified
 * sampling serves sparse problems in a batch with the same variance (Sec.
 * 5.4, Table 1) and no such pass; cfg.iteration is the problem's base iteration and
 * cfg.iteration_counter is ignored -- the batch call takes one counter for
 * all problems), loss and its eps, the Adam projection bound `lower`, and the
 * flat parameter, moment and (nullable) gradient arrays.  All problems of a
 * batch share d, the factor dtype and the value dtype.  Each problem's
 * samples are exactly those gcp_sample would draw for it alone (its own seed
 * and problem_id), so a batch and per-problem calls agree up to floating-point
 * order.
 *
 * gcp_batched_create plans the batch on the host (no device work) and
 * returns an opaque handle; gcp_batched_workspace_bytes sizes its workspace;
 * gcp_batched_prepare uploads the descriptor tables into the workspace and
 * clears the gradient accumulators (set-up, synchronises the stream);
 * gcp_batched_grad writes every problem's G; gcp_batched_adam_step applies
 * Adam to every problem (state as in gcp_adam_step, one for the batch).  Both
 * step calls are asynchronous, launch two kernels and can be captured in a
 * HIP graph; they leave the accumulators cleared.  Calls on one batch must not
 * overlap.  `tune` (nullable) sets the launch shape; zeros pick defaults. */
typedef struct gcp_problem {
    gcp_tensor X;
    gcp_factors M;
    gcp_sampling cfg;
    int32_t loss;                /* gcp_loss */
    int32_t reserved;            /* set to 0 */
    double eps;                  /* loss eps (1e-10 in the examples) */
    double lower;                /* Adam projection bound; -INFINITY for none */
    void *A;                     /* flat parameters, sum_k n_k r values of M.dtype */
    float *A_master;             /* GCP_BF16 only: float master copy */
    void *B;                     /* Adam moments (FP64 for FP64 factors, else FP32) */
    void *C;
    void *G;                     /* nullable: flat gradient output */
} gcp_problem;

typedef enum gcp_batch_schedule {
    /* every workgroup takes one run of the problem-ordered 64-sample items of
       equal estimated cost: a problem spans few workgroups, so few LDS
       partials are flushed per step */
    GCP_BATCH_CONTIGUOUS = 0,
    /* work units of unit_items items, dealt largest first to the least-loaded
       workgroup (longest-processing-time scheduling) */
    GCP_BATCH_LPT = 1
} gcp_batch_schedule;

typedef struct gcp_batch_tuning {
    int32_t threads;             /* threads per gradient workgroup: 256, 512 or 1024 (0: 1024) */
    int32_t unit_items;          /* GCP_BATCH_LPT: 64-sample items per work unit (0: 64) */
    int32_t schedule;            /* gcp_batch_schedule */
    int32_t cols_per_lane;       /* rank columns each lane gathers and scatters: 1, 2 or 4
                                    (0: by rank, as gcp_set_cols_per_lane); a value that
                                    does not fit a problem's rank falls back to 0 */
} gcp_batch_tuning;

typedef struct gcp_batch gcp_batch;

gcp_status gcp_batched_create(const gcp_problem *problems, int32_t count,
                              const gcp_batch_tuning *tune, gcp_batch **batch);
size_t gcp_batched_workspace_bytes(const gcp_batch *batch);
gcp_status gcp_batched_prepare(gcp_batch *batch, void *ws, size_t ws_bytes, hipStream_t stream);
gcp_status gcp_batched_grad(gcp_batch *batch, uint64_t *iteration_counter, hipStream_t stream);
gcp_status gcp_batched_adam_step(gcp_batch *batch, int64_t *state, uint64_t *iteration_counter,
                                 double alpha, double beta1, double beta2, double adam_eps,
                                 gcp_eps_mode eps_mode, hipStream_t stream);
/* The host plan of a batch (no device work): the number of gradient
 * workgroups and work units; then, for arrays that are non-NULL, the first
 * unit of every workgroup (block_ptr, n_blocks + 1 entries, caller-owned),
 * each unit's problem (n_units entries) and its half-open range of 64-sample
 * items (unit_items, 2 * n_units entries: begin, end).  Call once with NULL
 * arrays to size them. */
gcp_status gcp_batched_plan(const gcp_batch *batch, int64_t *n_blocks, int64_t *n_units,
                            int64_t *block_ptr, int32_t *unit_problem, int64_t *unit_items);
void gcp_batched_destroy(gcp_batch *batch);

/* gcp_batched_graph_capture -- records `steps` consecutive
 * gcp_batched_adam_step calls (Alg. 4's inner loop for every problem of the
 * batch; with iteration_counter, each step draws the next sample sets) into a
 * HIP graph that the batch owns, and instantiates it.  The arguments (state,
 * iteration_counter, alpha, beta1, beta2, adam_eps, eps_mode) are fixed at
 * capture, as in gcp_batched_adam_step.  The steps are recorded on a stream the
 * library creates for the batch, so nothing runs during the capture.
 * gcp_batched_graph_launch replays all `steps` on the caller's stream, allocating
 * nothing.  A new capture replaces the graph; gcp_batched_graph_destroy and
 * gcp_batched_destroy free it.  The batch must be prepared. */
gcp_status gcp_batched_graph_capture(gcp_batch *batch, int32_t steps, int64_t *state,
                                     uint64_t *iteration_counter, double alpha, double beta1,
                                     double beta2, double adam_eps, gcp_eps_mode eps_mode);
gcp_status gcp_batched_graph_launch(gcp_batch *batch, hipStream_t stream);
void gcp_batched_graph_destroy(gcp_batch *batch);

/* ---------------------------------------------------------------------------
 * Kernel timing for measurement harnesses (results never depend on it).
 * gcp_timing_start(n) creates n pairs of HIP events up front (so timing adds
 * no allocation to the calls it measures) and arms them: each following
 * gcp_sampled_grad / gcp_sampled_adam_step / gcp_batched_* step call launches
 * its gradient kernel (model entries, derivatives and MTTKRP scatter) with one
 * pair stamped at the kernel's own start and end, until n pairs are used.  Calls on a stream that is being captured into a graph
 * are not timed.  gcp_timing_stop waits for the recorded events, writes the
 * summed kernel time in milliseconds and the number of timed launches, and
 * destroys the events.  Host-global: one timing session at a time. */
gcp_status gcp_timing_start(int64_t max_launches);
gcp_status gcp_timing_stop(double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* GCP_H */
