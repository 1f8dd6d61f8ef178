/*
 * gcp_oracle.c -- plain FP64 CPU reference for the sampled GCP gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this file:
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header, table or helper with the HIP library.
 *
 * What it follows (Kolda & Hong, "Stochastic Gradients for Large-Scale Tensor
 * Decomposition"):
 *   - the CP model entry m_i = sum_j prod_k A_k(i_k, j)          (eq. Mdef, Alg. 1)
 *   - the elementwise derivative y_i = df/dm (x_i, m_i)           (eq. Y)
 *   - sampled MTTKRP G_k = Ytilde_(k) Z_k                         (eq. Gks)
 *   - uniform sampling with weight omega/s                        (Sec. 4.1, Alg. 1)
 *   - stratified sampling, nonzeros eta/p, zeros by rejection
 *     with weight zeta/q                                          (Sec. 4.2, Alg. 2)
 *   - semi-stratified sampling with the g(0,m) correction         (Sec. 4.3, Alg. 3)
 *   - the Adam update with projection                             (Sec. 5.1, Alg. 4)
 *   - the loss estimates                                          (eqs. Fhat, Fhat-strat)
 *
 * Everything is computed in double precision, one sample after another, in
 * the order the algorithms state.  No blocking, no threads, no fusion.
 *
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
 * (seed, problem_id), counter = (j, iteration, purpose, block).  randi(n) is
 * the high 64 bits of the 128-bit product w*n (0-based).  Purposes: 0 uniform
 * draws and semi-stratified "zeros", 1 nonzero picks, 2 rejection candidates.
 *
 * Functions with no independent pin are marked "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* Test hook: a nonzero value plants one deliberate mistake, so the pin tests
 * can show that each pin catches it.  0 = correct oracle. */
static int g_mutation = 0;
void orc_set_mutation(int m) { g_mutation = m; }
int orc_get_mutation(void) { return g_mutation; }

enum { ORC_GAUSSIAN = 0, ORC_BERNOULLI_ODDS = 1, ORC_POISSON = 2, ORC_GAMMA = 3, ORC_BETA_HALF = 4 };
enum { ORC_UNIFORM = 0, ORC_STRATIFIED = 1, ORC_SEMI = 2 };
/* sample stratum codes (one per sample) */
enum { ORC_S_UNIFORM = 0, ORC_S_NZ = 1, ORC_S_ZERO = 2, ORC_S_NZ_CORR = 3, ORC_S_SEMI_ZERO = 4 };

/* ------------------------------------------------------------------------ */
/* Philox4x64-10, from its published definition.                            */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t k0 = key[0], k1 = key[1];
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* randi(n), 0-based: floor(w * n / 2^64). */
uint64_t orc_randi(uint64_t w, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)w * n) >> 64);
}

/* Word k (k = 0.. ) of the random stream of sample j for a purpose. */
static uint64_t draw_word(uint64_t seed, uint64_t pid, uint64_t j, uint64_t iter,
                          uint64_t purpose, int k)
{
    uint64_t key[2] = {seed, pid};
    uint64_t ctr[4] = {j, iter, purpose, (uint64_t)(k / 4)};
    uint64_t out[4];
    orc_philox4x64_10(key, ctr, out);
    return out[k % 4];
}

/* ------------------------------------------------------------------------ */
/* Loss functions f(x, m) and derivatives g = df/dm.                          */
/* Gaussian (x-m)^2; Bernoulli-odds log(m+1) - x log(m+eps); Poisson          */
/* m - x log(m+eps).  eps sits only where the paper writes log m or x/m.      */
/* ------------------------------------------------------------------------ */
double orc_loss_f(int loss, double x, double m, double eps)
{
    switch (loss) {
    case ORC_GAUSSIAN:       return (x - m) * (x - m);
    case ORC_BERNOULLI_ODDS: return log(m + 1.0) - x * log(m + eps);
    case ORC_POISSON:        return m - x * log(m + eps);
    /* Gamma with shape 1 (Sec. 1): x/m + log m */
    case ORC_GAMMA:          return x / (m + eps) + log(m + eps);
    /* beta-divergence with beta = 1/2 (Sec. 5.3): 2 m^(1/2) + 2 x m^(-1/2) */
    case ORC_BETA_HALF:      return 2.0 * sqrt(m + eps) + 2.0 * x / sqrt(m + eps);
    }
    return NAN;
}

double orc_loss_g(int loss, double x, double m, double eps)
{
    switch (loss) {
    case ORC_GAUSSIAN:
        if (g_mutation == 1) return 2.0 * (x - m);          /* planted: sign flip */
        return 2.0 * (m - x);
    case ORC_BERNOULLI_ODDS: return 1.0 / (m + 1.0) - x / (m + eps);
    case ORC_POISSON:        return 1.0 - x / (m + eps);
    case ORC_GAMMA:          return 1.0 / (m + eps) - x / ((m + eps) * (m + eps));
    case ORC_BETA_HALF:      return 1.0 / sqrt(m + eps) - x / ((m + eps) * sqrt(m + eps));
    }
    return NAN;
}

/* ------------------------------------------------------------------------ */
/* Index helpers.                                                            */
/* ------------------------------------------------------------------------ */
static uint64_t linear_key(int d, const int64_t *dims, const int64_t *i)
{
    uint64_t L = 0;
    for (int k = 0; k < d; ++k) L = L * (uint64_t)dims[k] + (uint64_t)i[k];
    return L;
}

typedef struct { uint64_t key; int64_t pos; } keypos;

static int cmp_keypos(const void *a, const void *b)
{
    uint64_t x = ((const keypos *)a)->key, y = ((const keypos *)b)->key;
    return (x > y) - (x < y);
}

/* Sorted list of the nonzeros' linear keys (the paper's presorted list). */
static keypos *sorted_nonzeros(int d, const int64_t *dims, int64_t nnz, const int64_t *coo_idx)
{
    keypos *kp = (keypos *)malloc(sizeof(keypos) * (size_t)(nnz > 0 ? nnz : 1));
    for (int64_t e = 0; e < nnz; ++e) {
        kp[e].key = linear_key(d, dims, coo_idx + e * d);
        kp[e].pos = e;
    }
    qsort(kp, (size_t)nnz, sizeof(keypos), cmp_keypos);
    return kp;
}

/* Position of key in the nonzero list, or -1 if x at that index is zero. */
static int64_t find_nonzero(const keypos *kp, int64_t nnz, uint64_t key)
{
    int64_t lo = 0, hi = nnz - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (kp[mid].key == key) return kp[mid].pos;
        if (kp[mid].key < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Sampling (Alg. 1 index line; Alg. 2 nonzero and rejection loops; Alg. 3).  */
/*                                                                           */
/* Output, sample c = 0..S-1 (S = s for uniform, p + q otherwise):           */
/*   idx[c*d + k]  0-based mode indices                                      */
/*   xval[c]       the data value at that index (0 for zero-stratum samples)  */
/*   stratum[c]    one of the ORC_S_* codes                                  */
/*   cand[c]       the counter j the sample came from                        */
/* Nonzero-stratum samples come first (j = 0..p-1), then the zero stratum.    */
/* Stratified zeros: candidates j = 0,1,2,... are drawn like uniform indices; */
/* a candidate that hits a nonzero is rejected; the first q accepted are the  */
/* sample.  Returns the number of candidates examined (stratified) or the    */
/* number of samples, or -1 on bad arguments.                                */
/* ------------------------------------------------------------------------ */
int64_t orc_sample(int sampler, int d, const int64_t *dims,
                   const double *dense,
                   int64_t nnz, const int64_t *coo_idx, const double *coo_val,
                   int64_t s, int64_t p, int64_t q,
                   uint64_t seed, uint64_t pid, uint64_t iter,
                   int64_t *idx, double *xval, int32_t *stratum, int64_t *cand)
{
    if (d < 1 || d > 8) return -1;
    uint64_t omega = 1;
    for (int k = 0; k < d; ++k) omega *= (uint64_t)dims[k];
    keypos *kp = NULL;
    if (!dense) kp = sorted_nonzeros(d, dims, nnz, coo_idx);
    int64_t i[8];
    int64_t ret = -1;

    if (sampler == ORC_UNIFORM) {
        for (int64_t c = 0; c < s; ++c) {
            for (int k = 0; k < d; ++k)
                i[k] = (int64_t)orc_randi(draw_word(seed, pid, (uint64_t)c, iter, 0, k), (uint64_t)dims[k]);
            uint64_t L = linear_key(d, dims, i);
            double x;
            if (dense) x = dense[L];
            else {
                int64_t e = find_nonzero(kp, nnz, L);
                x = (e >= 0) ? coo_val[e] : 0.0;
            }
            memcpy(idx + c * d, i, sizeof(int64_t) * d);
            xval[c] = x; stratum[c] = ORC_S_UNIFORM; cand[c] = c;
        }
        ret = s;
    } else if (sampler == ORC_STRATIFIED || sampler == ORC_SEMI) {
        if (dense || nnz <= 0) goto done;
        /* nonzeros: xi = randi(eta), i = index of the xi-th nonzero */
        for (int64_t c = 0; c < p; ++c) {
            int64_t e = (int64_t)orc_randi(draw_word(seed, pid, (uint64_t)c, iter, 1, 0), (uint64_t)nnz);
            memcpy(idx + c * d, coo_idx + e * d, sizeof(int64_t) * d);
            xval[c] = coo_val[e];
            stratum[c] = (sampler == ORC_SEMI) ? ORC_S_NZ_CORR : ORC_S_NZ;
            cand[c] = c;
        }
        if (sampler == ORC_STRATIFIED) {
            if ((uint64_t)nnz >= omega && q > 0) goto done;      /* no zeros to draw */
            int64_t c = 0;
            uint64_t j = 0;
            while (c < q) {
                for (int k = 0; k < d; ++k)
                    i[k] = (int64_t)orc_randi(draw_word(seed, pid, j, iter, 2, k), (uint64_t)dims[k]);
                int64_t e = find_nonzero(kp, nnz, linear_key(d, dims, i));
                int reject = (e >= 0);
                if (g_mutation == 2) reject = 0;                 /* planted: no rejection */
                if (!reject) {
                    int64_t o = p + c;
                    memcpy(idx + o * d, i, sizeof(int64_t) * d);
                    xval[o] = 0.0; stratum[o] = ORC_S_ZERO; cand[o] = (int64_t)j;
                    ++c;
                }
                ++j;
            }
            ret = (int64_t)j;
        } else {
            /* semi-stratified "zeros": uniform over all indices, no rejection, x := 0 */
            for (int64_t c = 0; c < q; ++c) {
                for (int k = 0; k < d; ++k)
                    i[k] = (int64_t)orc_randi(draw_word(seed, pid, (uint64_t)c, iter, 0, k), (uint64_t)dims[k]);
                int64_t o = p + c;
                memcpy(idx + o * d, i, sizeof(int64_t) * d);
                xval[o] = 0.0; stratum[o] = ORC_S_SEMI_ZERO; cand[o] = c;
            }
            ret = p + q;
        }
    }
done:
    free(kp);
    return ret;
}

/* Entry weights of the weighted objective sum_i w_i f(x_i, m_i) (eq. wgcp,
 * Sec. 4.4) at each sample: a stored entry's own weight (dense: wdense[L];
 * COO: coo_w of the stored entry), w_zero for an entry a COO tensor does not
 * store.  Zero samples (stratified) are such entries; the "zeros" of
 * semi-stratified sampling stand for every entry at x = 0 in the correction
 * scheme, so they take w_zero as well.  Returns 0, or -1 on bad arguments. */
int orc_entry_weights(int d, const int64_t *dims, const double *wdense, int64_t nnz, const int64_t *coo_idx,
                      const double *coo_w, double w_zero, int64_t S, const int64_t *idx, const int32_t *stratum,
                      double *wout)
{
    if (d < 1 || d > 8) return -1;
    keypos *kp = NULL;
    if (!wdense) kp = sorted_nonzeros(d, dims, nnz, coo_idx);
    for (int64_t c = 0; c < S; ++c) {
        const int64_t *i = idx + c * d;
        if (stratum[c] == ORC_S_ZERO || stratum[c] == ORC_S_SEMI_ZERO) {
            wout[c] = w_zero;
        } else if (wdense) {
            wout[c] = wdense[linear_key(d, dims, i)];
        } else {
            int64_t e = find_nonzero(kp, nnz, linear_key(d, dims, i));
            wout[c] = (e >= 0) ? coo_w[e] : w_zero;
        }
    }
    free(kp);
    return 0;
}

/* Per-stratum weights (Sec. 4.1-4.3).  ytilde = w * (g(x,m) - corr * g(0,m)). */
static double stratum_weight(int st, double omega, double eta, int64_t s, int64_t p, int64_t q)
{
    switch (st) {
    case ORC_S_UNIFORM:   return omega / (double)s;
    case ORC_S_NZ:        return eta / (double)p;
    case ORC_S_ZERO:      return (omega - eta) / (double)q;
    case ORC_S_NZ_CORR:   return eta / (double)p;
    case ORC_S_SEMI_ZERO: return (g_mutation == 3) ? (omega - eta) / (double)q  /* planted: rejection weight */
                                                    : omega / (double)q;
    }
    return NAN;
}

/* Model entry m_i = sum_j prod_k A_k(i_k, j) (eq. Mdef). */
static double model_entry(int d, int64_t r, const double *const *A, const int64_t *i)
{
    double m = 0.0;
    for (int64_t j = 0; j < r; ++j) {
        double prod = 1.0;
        for (int k = 0; k < d; ++k) prod *= A[k][i[k] * r + j];
        m += prod;
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Sampled gradient (Alg. 1-3 loop bodies, then the d sparse MTTKRPs).       */
/* G[k] (dims[k] x r, row-major) is overwritten.  Each sample adds           */
/*   G_k(i_k, :) += ytilde * prod_{k' != k} A_k'(i_k', :).                   */
/* ytilde_out (nullable) receives ytilde per sample; the return value is the */
/* weighted loss estimate (eq. Fhat / Fhat-strat; the semi-stratified form   */
/* sum_nz (eta/p)[f(x,m) - f(0,m)] + sum_zero (omega/q) f(0,m) is the same   */
/* correction argument applied to f -- parity unpinned as a paper formula,   */
/* pinned here only by its expectation).                                     */
/* ------------------------------------------------------------------------ */
double orc_grad_weighted(int loss, int d, const int64_t *dims, int64_t r, const double *const *A,
                         int64_t S, const int64_t *idx, const double *xval, const int32_t *stratum,
                         const double *wgt, double w_zero, int64_t nnz, int64_t s, int64_t p, int64_t q,
                         double eps, double *ytilde_out, double *const *G);

double orc_grad(int loss, int d, const int64_t *dims, int64_t r, const double *const *A,
                int64_t S, const int64_t *idx, const double *xval, const int32_t *stratum,
                int64_t nnz, int64_t s, int64_t p, int64_t q, double eps,
                double *ytilde_out, double *const *G)
{
    return orc_grad_weighted(loss, d, dims, r, A, S, idx, xval, stratum, NULL, 1.0, nnz, s, p, q, eps,
                             ytilde_out, G);
}

/* The same with entry weights (eq. wgcp: ytilde_i = s_i w_i g(x_i, m_i) for
 * the sampling weight s_i; a corrected nonzero gives s_i (w_i g(x,m) - w_zero
 * g(0,m)), so that with the semi-stratified "zeros" (weight w_zero) the
 * estimate stays unbiased for sum_i w_i f(x_i, m_i)).  wgt NULL: all 1. */
double orc_grad_weighted(int loss, int d, const int64_t *dims, int64_t r, const double *const *A,
                         int64_t S, const int64_t *idx, const double *xval, const int32_t *stratum,
                         const double *wgt, double w_zero, int64_t nnz, int64_t s, int64_t p, int64_t q,
                         double eps, double *ytilde_out, double *const *G)
{
    double omega = 1.0;
    for (int k = 0; k < d; ++k) omega *= (double)dims[k];
    double eta = (double)nnz;
    for (int k = 0; k < d; ++k) memset(G[k], 0, sizeof(double) * (size_t)(dims[k] * r));
    double F = 0.0;
    for (int64_t c = 0; c < S; ++c) {
        const int64_t *i = idx + c * d;
        double x = xval[c];
        int st = stratum[c];
        double m = model_entry(d, r, A, i);
        double w = stratum_weight(st, omega, eta, s, p, q);
        double we = wgt ? wgt[c] : 1.0;
        double wz = wgt ? ((g_mutation == 7) ? we : w_zero) : 1.0;   /* 7 planted: own weight in the correction */
        double y, f;
        if (st == ORC_S_NZ_CORR) {
            y = (g_mutation == 4) ? w * we * orc_loss_g(loss, x, m, eps)      /* planted: no correction */
                                  : w * (we * orc_loss_g(loss, x, m, eps) - wz * orc_loss_g(loss, 0.0, m, eps));
            f = w * (we * orc_loss_f(loss, x, m, eps) - wz * orc_loss_f(loss, 0.0, m, eps));
        } else {
            y = w * we * orc_loss_g(loss, x, m, eps);
            /* 8 planted: a zero sample's loss term weighted omega/q instead of zeta/q */
            double wf = (g_mutation == 8 && st == ORC_S_ZERO) ? omega / (double)q : w;
            f = wf * we * orc_loss_f(loss, x, m, eps);
        }
        if (ytilde_out) ytilde_out[c] = y;
        F += f;
        for (int k = 0; k < d; ++k) {
            int kk = (g_mutation == 5 && d > 1) ? (k + 1) % d : k;     /* planted: wrong factor left out */
            for (int64_t j = 0; j < r; ++j) {
                double z = 1.0;
                for (int k2 = 0; k2 < d; ++k2)
                    if (k2 != kk) z *= A[k2][i[k2] * r + j];
                G[k][i[k] * r + j] += y * z;
            }
        }
    }
    return F;
}

/* ------------------------------------------------------------------------ */
/* Full (non-sampled) gradient by enumeration of every index, weight 1:      */
/* G_k = Y_(k) Z_k with y_i = g(x_i, m_i) (eqs. Y, Gk).  Tiny tensors only.  */
/* Returns F(X, M) = sum_i f(x_i, m_i) (eq. gcp).                            */
/* ------------------------------------------------------------------------ */
double orc_full_grad(int loss, int d, const int64_t *dims, int64_t r, const double *const *A,
                     const double *dense, double eps, double *const *G)
{
    int64_t omega = 1;
    for (int k = 0; k < d; ++k) omega *= dims[k];
    for (int k = 0; k < d; ++k) memset(G[k], 0, sizeof(double) * (size_t)(dims[k] * r));
    int64_t i[8];
    double F = 0.0;
    for (int64_t L = 0; L < omega; ++L) {
        int64_t rem = L;
        for (int k = d - 1; k >= 0; --k) { i[k] = rem % dims[k]; rem /= dims[k]; }
        double m = model_entry(d, r, A, i);
        double x = dense[L];
        double y = orc_loss_g(loss, x, m, eps);
        F += orc_loss_f(loss, x, m, eps);
        for (int k = 0; k < d; ++k)
            for (int64_t j = 0; j < r; ++j) {
                double z = 1.0;
                for (int k2 = 0; k2 < d; ++k2)
                    if (k2 != k) z *= A[k2][i[k2] * r + j];
                G[k][i[k] * r + j] += y * z;
            }
    }
    return F;
}

/* ------------------------------------------------------------------------ */
/* One Adam step with projection (Alg. 4 inner loop) over P parameters.      */
/* t is the step number after the increment (t >= 1): the first step uses   */
/* 1 - beta^1 in the bias corrections.  eps_mode 0: eps inside the square    */
/* root as Alg. 4 writes it; 1: outside (sqrt(Chat) + eps).                  */
/* ------------------------------------------------------------------------ */
void orc_adam(int64_t P, double *A, const double *G, double *B, double *C, int64_t t,
              double alpha, double beta1, double beta2, double eps, double lower, int eps_mode)
{
    double bc1 = 1.0 - pow(beta1, (double)t);
    double bc2 = 1.0 - pow(beta2, (double)t);
    for (int64_t e = 0; e < P; ++e) {
        double g = G[e];
        B[e] = beta1 * B[e] + (1.0 - beta1) * g;
        C[e] = beta2 * C[e] + (1.0 - beta2) * g * g;
        double bhat = B[e] / bc1;
        double chat = C[e] / bc2;
        double den = (eps_mode == 0) ? sqrt(chat + eps) : sqrt(chat) + eps;
        if (g_mutation == 6) den = sqrt(chat) + eps;               /* planted: eps outside */
        double a = A[e] - alpha * bhat / den;
        A[e] = (a < lower) ? lower : a;
    }
}
