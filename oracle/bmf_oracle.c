/*
 * bmf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU oracle for the BPMF Gibbs sweep used on every data
 * subset of posterior propagation (Qin et al., "Distributed Bayesian Matrix
 * Factorization with Limited Communication", arXiv:1703.00734).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header or table with the GPU library; the two agree only on
 * the published definitions below (model, Philox4x32-10, Box-Muller,
 * Marsaglia-Tsang, Bartlett) and on the counter layout of the random stream.
 *
 * Model (Sec. 2.1, eq. BMF_likelihood, BMF_likelihood_normal, prior_X, prior_W):
 *   y_nd ~ N(x_n^T w_d, 1/tau) on the observed set, x_n ~ N_K(mu_X, Lambda_X^-1),
 *   w_d ~ N_K(mu_W, Lambda_W^-1).  The row conditional is the conjugate Gaussian
 *   N(A^-1 h, A^-1) with A = P + tau sum_d w_d w_d^T, h = P m + tau sum_d r_nd w_d.
 * Hyperparameters: Normal-Wishart draws of the BPMF Gibbs sampler of
 *   Salakhutdinov & Mnih (2008b), with the centred scatter matrix of the
 *   Sec. 5.1 footnote; tau either fixed (Sec. 5.1) or Gamma-sampled.
 * Moment matching (Sec. 4.1, "Moment matching approximation"): per-row Gaussian
 *   from the sample mean and covariance of the kept Gibbs samples.
 *
 * Random stream (shared definition, independent code on each side):
 *   key = (seed mod 2^32, seed >> 32); counter = (c0, c1, c2, c3) with
 *   c0 = entity id, c1 = sweep index (0xFFFFFFFF at initialisation),
 *   c2 = (block id << 8) | purpose, c3 = draw group / rejection attempt.
 *   u(x) = ((x >> 9) + 0.5) * 2^-23 (exact in FP32 and FP64); normals by
 *   Box-Muller on (u0,u1), (u2,u3).
 *
 * Every function is single-purpose and written for checking by eye, in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, "Parallel random      */
/* numbers: as easy as 1, 2, 3").  Ten rounds of the 4x32 S-box; the key is  */
/* bumped by the Weyl constants between rounds.                              */
/* ------------------------------------------------------------------------- */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void orc_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

/* n counters (n x 4, row-major) -> n outputs (n x 4) under one seed. */
void orc_philox_batch(int64_t n, const uint32_t *ctr, uint64_t seed, uint32_t *out)
{
    uint32_t key[2];
    orc_key(seed, key);
    for (int64_t i = 0; i < n; ++i)
        orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* 23-bit uniform on the open interval (0,1): (m + 0.5) 2^-23 with m < 2^23
 * has at most 24 significant bits, so it is exact in FP32 and in FP64. */
double orc_u23(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* n standard normals z[0..n) for counter (c0, c1, c2, g), g = 0, 1, ...:
 * group g yields z[4g..4g+3] by two Box-Muller transforms. */
void orc_normals(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, int32_t n, double *z)
{
    uint32_t key[2];
    orc_key(seed, key);
    const double two_pi = 6.283185307179586476925286766559;
    for (int32_t g = 0; 4 * g < n; ++g) {
        uint32_t ctr[4] = {c0, c1, c2, (uint32_t)g};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        double r1 = sqrt(-2.0 * log(orc_u23(o[0])));
        double t1 = two_pi * orc_u23(o[1]);
        double r2 = sqrt(-2.0 * log(orc_u23(o[2])));
        double t2 = two_pi * orc_u23(o[3]);
        double v[4] = {r1 * cos(t1), r1 * sin(t1), r2 * cos(t2), r2 * sin(t2)};
        for (int q = 0; q < 4 && 4 * g + q < n; ++q)
            z[4 * g + q] = v[q];
    }
}

/* Gamma(shape, 1) by Marsaglia & Tsang (2000), "A simple method for generating
 * gamma variables".  Attempt k uses counter (c0, c1, c2, k): the normal from
 * Box-Muller on (u0, u1), the acceptance uniform from u2.  For shape < 1 the
 * boost Gamma(a) = Gamma(a+1) * U^(1/a) is used with U = u(first word) of
 * counter (c0, c1, c2, 0xFFFFFFFF), an attempt index never reached.  A draw that rejects ORC_GAMMA_MAX_ATTEMPTS times
 * (probability far below 1e-60) returns the value d. */
#define ORC_GAMMA_MAX_ATTEMPTS 64
double orc_gamma(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, double shape)
{
    uint32_t key[2];
    orc_key(seed, key);
    double boost = 1.0;
    double a = shape;
    if (a < 1.0) {
        uint32_t ctr[4] = {c0, c1, c2, 0xFFFFFFFFu};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        boost = pow(orc_u23(o[0]), 1.0 / a);
        a = a + 1.0;
    }
    const double d = a - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    const double two_pi = 6.283185307179586476925286766559;
    for (uint32_t k = 0; k < ORC_GAMMA_MAX_ATTEMPTS; ++k) {
        uint32_t ctr[4] = {c0, c1, c2, k};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        double z = sqrt(-2.0 * log(orc_u23(o[0]))) * cos(two_pi * orc_u23(o[1]));
        double v = 1.0 + c * z;
        if (v <= 0.0)
            continue;
        v = v * v * v;
        double u = orc_u23(o[2]);
        if (log(u) < 0.5 * z * z + d - d * v + d * log(v))
            return d * v * boost;
    }
    return d * boost;
}

/* ------------------------------------------------------------------------- */
/* Dense FP64 linear algebra on row-major K x K matrices.                    */
/* ------------------------------------------------------------------------- */

/* Cholesky-Banachiewicz: L lower with L L^T = A.  Returns 0, or -1 when a
 * pivot is not positive (A not positive definite). */
static int orc_chol(int K, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)K * K);
    for (int i = 0; i < K; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * K + j];
            for (int p = 0; p < j; ++p)
                s -= L[i * K + p] * L[j * K + p];
            if (i == j) {
                if (!(s > 0.0))
                    return -1;
                L[i * K + i] = sqrt(s);
            } else {
                L[i * K + j] = s / L[j * K + j];
            }
        }
    }
    return 0;
}

/* Solve L y = b (forward substitution). */
static void orc_solve_lower(int K, const double *L, const double *b, double *y)
{
    for (int i = 0; i < K; ++i) {
        double s = b[i];
        for (int p = 0; p < i; ++p)
            s -= L[i * K + p] * y[p];
        y[i] = s / L[i * K + i];
    }
}

/* Solve L^T x = b (back substitution with the transpose of L). */
static void orc_solve_lower_T(int K, const double *L, const double *b, double *x)
{
    for (int i = K - 1; i >= 0; --i) {
        double s = b[i];
        for (int p = i + 1; p < K; ++p)
            s -= L[p * K + i] * x[p];
        x[i] = s / L[i * K + i];
    }
}

/* Inverse of an SPD matrix from its Cholesky factor: A^-1 = L^-T L^-1. */
static void orc_inverse_from_chol(int K, const double *L, double *Ainv)
{
    double *e = (double *)calloc((size_t)K, sizeof(double));
    double *y = (double *)calloc((size_t)K, sizeof(double));
    double *x = (double *)calloc((size_t)K, sizeof(double));
    for (int c = 0; c < K; ++c) {
        memset(e, 0, sizeof(double) * K);
        e[c] = 1.0;
        orc_solve_lower(K, L, e, y);
        orc_solve_lower_T(K, L, y, x);
        for (int r = 0; r < K; ++r)
            Ainv[r * K + c] = x[r];
    }
    free(e); free(y); free(x);
}

/* Public wrappers so tests can pin the factorisation against a library. */
int orc_cholesky(int32_t K, const double *A, double *L) { return orc_chol(K, A, L); }

/* ------------------------------------------------------------------------- */
/* Model steps.                                                              */
/* ------------------------------------------------------------------------- */

/* Sequential FP64 mean of the observed values, left to right in COO order. */
double orc_seq_mean(int64_t n, const float *val)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += (double)val[i];
    return n > 0 ? s / (double)n : 0.0;
}

/* Initial factors of one side of a block: x_n = K^(-1/4) z_n with z_n from
 * counter (n, 0xFFFFFFFF, c2, g). */
void orc_init_side(int64_t R, int32_t K, uint64_t seed, uint32_t c2, double *out)
{
    const double s = pow((double)K, -0.25);
    for (int64_t n = 0; n < R; ++n) {
        orc_normals(seed, (uint32_t)n, 0xFFFFFFFFu, c2, K, out + n * K);
        for (int k = 0; k < K; ++k)
            out[n * K + k] *= s;
    }
}

/* One Gibbs update of every entity of one side of one block (rows: CSR over
 * the block's rows with the column factors as `other`; columns: CSC with the
 * row factors).  For entity n:
 *     A = P_n + tau * sum_{d in Omega_n} w_d w_d^T
 *     h = P_n m_n + tau * sum_{d in Omega_n} r_nd w_d
 *     L = chol(A);  mu = L^-T (L^-1 h);  x_n = mu + L^-T z,  z ~ N(0, I_K)
 * where z comes from counter (n, t, c2, g).  With per_row = 0, P (K x K) and
 * m (K) are the shared Gaussian prior of the side; with per_row = 1, P is
 * R x K x K and m is R x K (propagated per-row priors, eq. stage2a-stage3).
 * Returns the number of entities whose A failed the Cholesky (then x_n is left
 * unchanged); 0 in every valid run. */
/* The conditional system of one entity: with G = sum_{d in Omega_n} w_d w_d^T
 * and s = sum_{d in Omega_n} r_nd w_d (entries ptr[n] .. ptr[n+1] of idx/val),
 *     A = P_n + tau G,   h = P_n m_n + tau s.
 * With per-column noise precisions (the tau_d variant of Sec. 2.1) the row
 * update weights each entry by its column's tau_d: wt (indexed like `other`,
 * or NULL for 1) gives G = sum tau_d w_d w_d^T and s = sum tau_d r_nd w_d,
 * with tau = 1.  G and hs are scratch (K x K and K). */
static void orc_cond_system(int32_t K, int64_t e0, int64_t e1, const int32_t *idx, const double *val,
                            const double *other, const double *wt, const double *Pn, const double *mn,
                            double tau, double *G, double *hs, double *A, double *h)
{
    memset(G, 0, sizeof(double) * (size_t)K * K);
    memset(hs, 0, sizeof(double) * (size_t)K);
    for (int64_t e = e0; e < e1; ++e) {
        const double *w = other + (int64_t)idx[e] * K;
        const double r = val[e];
        const double we = wt ? wt[idx[e]] : 1.0;
        for (int a = 0; a < K; ++a) {
            for (int b = 0; b < K; ++b)
                G[a * K + b] += we * w[a] * w[b];
            hs[a] += we * r * w[a];
        }
    }
    for (int a = 0; a < K; ++a) {
        double pm = 0.0;
        for (int b = 0; b < K; ++b) {
            A[a * K + b] = Pn[a * K + b] + tau * G[a * K + b];
            pm += Pn[a * K + b] * mn[b];
        }
        h[a] = pm + tau * hs[a];
    }
}

/* The conditional precision A_n of every entity of one side (R x K x K), as
 * the update below forms it (for the positive-definiteness pin). */
void orc_cond_precision(int64_t R, int32_t K, const int64_t *ptr, const int32_t *idx,
                        const double *val, const double *other, int32_t per_row,
                        const double *P, const double *m, double tau, double *A)
{
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        double *G = (double *)malloc(sizeof(double) * (size_t)K * K);
        double *hs = (double *)malloc(sizeof(double) * (size_t)K);
        double *h = (double *)malloc(sizeof(double) * (size_t)K);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (int64_t n = 0; n < R; ++n) {
            const double *Pn = per_row ? P + n * K * K : P;
            const double *mn = per_row ? m + n * K : m;
            orc_cond_system(K, ptr[n], ptr[n + 1], idx, val, other, NULL, Pn, mn, tau, G, hs,
                            A + n * (int64_t)K * K, h);
        }
        free(G); free(hs); free(h);
    }
}

/* orc_update_side with per-column noise precisions (the tau_d variant of
 * Sec. 2.1): wt (per entity of the other side, the row update's entry weights
 * tau_d) and taus (per entity of this side, the column update's tau_d); either
 * NULL for the scalar tau. */
int64_t orc_update_side_w(int64_t R, int32_t K, const int64_t *ptr, const int32_t *idx,
                          const double *val, const double *other, const double *wt, const double *taus,
                          int32_t per_row, const double *P, const double *m, double tau, uint64_t seed,
                          uint32_t t, uint32_t c2, double *out, int32_t nthreads);

int64_t orc_update_side(int64_t R, int32_t K, const int64_t *ptr, const int32_t *idx,
                        const double *val, const double *other, int32_t per_row,
                        const double *P, const double *m, double tau, uint64_t seed,
                        uint32_t t, uint32_t c2, double *out, int32_t nthreads)
{
    return orc_update_side_w(R, K, ptr, idx, val, other, NULL, NULL, per_row, P, m, tau, seed, t, c2, out,
                             nthreads);
}

int64_t orc_update_side_w(int64_t R, int32_t K, const int64_t *ptr, const int32_t *idx,
                          const double *val, const double *other, const double *wt, const double *taus,
                          int32_t per_row, const double *P, const double *m, double tau, uint64_t seed,
                          uint32_t t, uint32_t c2, double *out, int32_t nthreads)
{
    int64_t failures = 0;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(+ : failures)
#endif
    {
        double *G = (double *)malloc(sizeof(double) * (size_t)K * K);
        double *A = (double *)malloc(sizeof(double) * (size_t)K * K);
        double *L = (double *)malloc(sizeof(double) * (size_t)K * K);
        double *hs = (double *)malloc(sizeof(double) * (size_t)K);
        double *h = (double *)malloc(sizeof(double) * (size_t)K);
        double *y = (double *)malloc(sizeof(double) * (size_t)K);
        double *mu = (double *)malloc(sizeof(double) * (size_t)K);
        double *z = (double *)malloc(sizeof(double) * (size_t)K);
        double *v = (double *)malloc(sizeof(double) * (size_t)K);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (int64_t n = 0; n < R; ++n) {
            const double *Pn = per_row ? P + n * K * K : P;
            const double *mn = per_row ? m + n * K : m;
            orc_cond_system(K, ptr[n], ptr[n + 1], idx, val, other, wt, Pn, mn, taus ? taus[n] : tau, G, hs,
                            A, h);
            if (orc_chol(K, A, L) != 0) {
                failures += 1;
                continue;
            }
            orc_solve_lower(K, L, h, y);
            orc_solve_lower_T(K, L, y, mu);
            orc_normals(seed, (uint32_t)n, t, c2, K, z);
            orc_solve_lower_T(K, L, z, v);
            for (int a = 0; a < K; ++a)
                out[n * K + a] = mu[a] + v[a];
        }
        free(G); free(A); free(L); free(hs); free(h); free(y); free(mu); free(z); free(v);
    }
    return failures;
}

/* Sum of squared residuals over a block's observed entries (CSR walk in row
 * order): SSE = sum (r_nd - x_n^T w_d)^2. */
double orc_sse(int64_t R, int32_t K, const int64_t *ptr, const int32_t *idx, const double *val,
               const double *X, const double *W)
{
    double sse = 0.0;
    for (int64_t n = 0; n < R; ++n) {
        for (int64_t e = ptr[n]; e < ptr[n + 1]; ++e) {
            double pred = 0.0;
            for (int k = 0; k < K; ++k)
                pred += X[n * K + k] * W[(int64_t)idx[e] * K + k];
            const double res = val[e] - pred;
            sse += res * res;
        }
    }
    return sse;
}

/* Noise precision draw: tau ~ Gamma(shape a0 + M/2, rate b0 + SSE/2), the
 * Gamma attempts on counter (0, t, c2, k). */
double orc_tau_draw(double sse, int64_t M, double a0, double b0, uint64_t seed, uint32_t t,
                    uint32_t c2)
{
    const double shape = a0 + 0.5 * (double)M;
    const double rate = b0 + 0.5 * sse;
    return orc_gamma(seed, 0u, t, c2, shape) / rate;
}

/* Per-column noise precisions (the tau_d variant of Sec. 2.1): for column d
 * of a block with M_d entries and residual SSE_d, tau_d ~ Gamma(shape
 * a0 + M_d/2, rate b0 + SSE_d/2), the attempts on counter (d, t, c2, k).
 * C columns; sse and cnt per column. */
void orc_tau_cols(int64_t C, const double *sse, const int64_t *cnt, double a0, double b0, uint64_t seed,
                  uint32_t t, uint32_t c2, double *tau)
{
    for (int64_t d = 0; d < C; ++d) {
        const double shape = a0 + 0.5 * (double)cnt[d];
        const double rate = b0 + 0.5 * sse[d];
        tau[d] = orc_gamma(seed, (uint32_t)d, t, c2, shape) / rate;
    }
}

/* Normal-Wishart hyperparameter draw for one side of one block, given its Nb
 * factor rows X (Nb x K).  With x_bar = mean of the rows and the centred
 * scatter S_bar = (1/Nb) sum (x - x_bar)(x - x_bar)^T (Sec. 5.1 footnote):
 *     beta* = beta0 + Nb,  nu* = nu0 + Nb,  mu* = (beta0 mu0 + Nb x_bar)/beta*
 *     W*^-1 = W0^-1 + Nb S_bar + (beta0 Nb / beta*) (mu0 - x_bar)(mu0 - x_bar)^T
 *     Lambda ~ Wishart(W*, nu*)   (E[Lambda] = nu* W*),
 *     mu ~ N(mu*, (beta* Lambda)^-1).
 * The Wishart draw is Bartlett's decomposition: with R R^T = W*^-1 and
 * T = R^-T (so T T^T = W*), A lower triangular with A_kk^2 ~ chi2(nu* - k + 1)
 * (k = 1..K, from Gamma on counter (k, t, c2, attempt)) and A_kl ~ N(0,1) for
 * k > l (normals stream on counter (0, t, c2, g), strict lower triangle in
 * row-major order), Lambda = T A A^T T^T.  Then C = chol(Lambda) and
 * mu = mu* + beta*^(-1/2) C^-T z with z from counter (K + 1, t, c2, g).
 * Returns 0, or -1 if a factorisation fails. */
int orc_nw_draw(int64_t Nb, int32_t K, const double *X, const double *mu0, double beta0,
                double nu0, const double *W0inv, uint64_t seed, uint32_t t, uint32_t c2,
                double *Lam, double *mu)
{
    const size_t KK = (size_t)K * K;
    double *xbar = (double *)calloc((size_t)K, sizeof(double));
    double *S = (double *)calloc(KK, sizeof(double));
    double *Winv = (double *)calloc(KK, sizeof(double));
    double *Rf = (double *)calloc(KK, sizeof(double));
    double *T = (double *)calloc(KK, sizeof(double));
    double *Ab = (double *)calloc(KK, sizeof(double));
    double *TA = (double *)calloc(KK, sizeof(double));
    double *C = (double *)calloc(KK, sizeof(double));
    double *mus = (double *)calloc((size_t)K, sizeof(double));
    double *z = (double *)calloc((size_t)K + 4, sizeof(double));
    double *v = (double *)calloc((size_t)K, sizeof(double));
    double *col = (double *)calloc((size_t)K, sizeof(double));
    double *e = (double *)calloc((size_t)K, sizeof(double));
    int status = 0;

    /* sample mean and centred scatter (N * S_bar) */
    for (int64_t n = 0; n < Nb; ++n)
        for (int k = 0; k < K; ++k)
            xbar[k] += X[n * K + k];
    for (int k = 0; k < K; ++k)
        xbar[k] /= (double)Nb;
    for (int64_t n = 0; n < Nb; ++n)
        for (int a = 0; a < K; ++a)
            for (int b = 0; b < K; ++b)
                S[a * K + b] += (X[n * K + a] - xbar[a]) * (X[n * K + b] - xbar[b]);

    const double N = (double)Nb;
    const double beta_s = beta0 + N;
    const double nu_s = nu0 + N;
    for (int k = 0; k < K; ++k)
        mus[k] = (beta0 * mu0[k] + N * xbar[k]) / beta_s;
    const double coef = beta0 * N / beta_s;
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b)
            Winv[a * K + b] = W0inv[a * K + b] + S[a * K + b] +
                              coef * (mu0[a] - xbar[a]) * (mu0[b] - xbar[b]);

    /* T = R^-T where R R^T = W*^-1: column c of R^-T solves R^T x = e_c. */
    if (orc_chol(K, Winv, Rf) != 0) {
        status = -1;
        goto done;
    }
    for (int c = 0; c < K; ++c) {
        memset(e, 0, sizeof(double) * K);
        e[c] = 1.0;
        orc_solve_lower_T(K, Rf, e, col);
        for (int r = 0; r < K; ++r)
            T[r * K + c] = col[r];
    }

    /* Bartlett factor A. */
    for (int k = 1; k <= K; ++k) {
        const double chi2 = 2.0 * orc_gamma(seed, (uint32_t)k, t, c2, 0.5 * (nu_s - k + 1.0));
        Ab[(k - 1) * K + (k - 1)] = sqrt(chi2);
    }
    {
        const int noff = K * (K - 1) / 2;
        double *zoff = (double *)calloc((size_t)noff + 4, sizeof(double));
        if (noff > 0)
            orc_normals(seed, 0u, t, c2, noff, zoff);
        int q = 0;
        for (int a = 1; a < K; ++a)
            for (int b = 0; b < a; ++b)
                Ab[a * K + b] = zoff[q++];
        free(zoff);
    }

    /* Lambda = (T A)(T A)^T */
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            double s = 0.0;
            for (int p = 0; p < K; ++p)
                s += T[a * K + p] * Ab[p * K + b];
            TA[a * K + b] = s;
        }
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            double s = 0.0;
            for (int p = 0; p < K; ++p)
                s += TA[a * K + p] * TA[b * K + p];
            Lam[a * K + b] = s;
        }

    /* mu = mu* + beta*^(-1/2) C^-T z */
    if (orc_chol(K, Lam, C) != 0) {
        status = -1;
        goto done;
    }
    orc_normals(seed, (uint32_t)(K + 1), t, c2, K, z);
    orc_solve_lower_T(K, C, z, v);
    for (int k = 0; k < K; ++k)
        mu[k] = mus[k] + v[k] / sqrt(beta_s);

done:
    free(xbar); free(S); free(Winv); free(Rf); free(T); free(Ab); free(TA); free(C);
    free(mus); free(z); free(v); free(col); free(e);
    return status;
}

/* Moment matching of one side of one block from S kept samples
 * (samples is S x R x K): per row, mu_hat = sample mean,
 * Sigma_hat = sum (x - mu_hat)(x - mu_hat)^T / (S - 1) (two passes), and
 * Lambda_hat = Sigma_hat^-1 through its Cholesky factor.  When S <= K or the
 * factorisation fails, Sigma_hat += delta I with
 * delta = 1e-6 tr(Sigma_hat)/K + 1e-300 before inverting.  Needs S >= 2.
 * Returns the number of rows that took the ridge. */
int64_t orc_mm(int64_t R, int32_t K, int32_t S, const double *samples, double *mu,
               double *Lam)
{
    int64_t ridged = 0;
    const size_t KK = (size_t)K * K;
    double *Sig = (double *)malloc(sizeof(double) * KK);
    double *L = (double *)malloc(sizeof(double) * KK);
    for (int64_t n = 0; n < R; ++n) {
        double *mn = mu + n * K;
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int q = 0; q < S; ++q)
                s += samples[((int64_t)q * R + n) * K + k];
            mn[k] = s / (double)S;
        }
        memset(Sig, 0, sizeof(double) * KK);
        for (int q = 0; q < S; ++q) {
            const double *x = samples + ((int64_t)q * R + n) * K;
            for (int a = 0; a < K; ++a)
                for (int b = 0; b < K; ++b)
                    Sig[a * K + b] += (x[a] - mn[a]) * (x[b] - mn[b]);
        }
        for (size_t p = 0; p < KK; ++p)
            Sig[p] /= (double)(S - 1);
        int need_ridge = (S <= K) || (orc_chol(K, Sig, L) != 0);
        if (need_ridge) {
            double tr = 0.0;
            for (int k = 0; k < K; ++k)
                tr += Sig[k * K + k];
            const double delta = 1e-6 * tr / (double)K + 1e-300;
            for (int k = 0; k < K; ++k)
                Sig[k * K + k] += delta;
            orc_chol(K, Sig, L);
            ridged += 1;
        }
        orc_inverse_from_chol(K, L, Lam + n * KK);
    }
    free(Sig); free(L);
    return ridged;
}

/* ------------------------------------------------------------------------- */
/* Clustering of the kept samples for the dominant-mode (PP-DM) and mixture  */
/* (PP-GMM) approximations (Sec. 4.1; Sec. 5.1, which clusters each          */
/* parameter's samples with the nonparametric lambda-means algorithm).  The  */
/* iteration is the hard-clustering one of DP-means (Kulis and Jordan, 2012): */
/* in sample order, each sample joins the nearest centre unless that centre  */
/* is farther than lambda, in which case it opens a new cluster on itself;   */
/* then every centre moves to the mean of its members.  Readings (the paper  */
/* gives no lambda or stopping rule): one initial cluster at the mean of all */
/* samples; lambda^2 = c^2 sum_t |x_(t+1) - x_t|^2 / (2 (S - 1)), the mean   */
/* squared step between successive kept samples over two, times the square  */
/* of a scale c; at most cmax clusters (a sample that would open one more    */
/* joins its nearest); clusters left without members are dropped, the others */
/* keep their order; the iteration stops when the assignment repeats or      */
/* after maxit rounds.  Distances and sums run in index order, unfused.      */
/* ------------------------------------------------------------------------- */

/* Squared distance of two K-vectors, components in order. */
static double orc_dist2(int K, const double *a, const double *b)
{
    double s = 0.0;
    for (int k = 0; k < K; ++k) {
        const double d = a[k] - b[k];
        s = s + d * d;
    }
    return s;
}

/* One entity: xs[q] points at sample q (K values).  Writes labels[q] and
 * returns the number of clusters. */
static int orc_lmeans_one(int K, int S, const double *const *xs, double lam_scale, int cmax,
                          int maxit, int32_t *labels, double *cent, int32_t *cnt, int32_t *prev)
{
    /* lambda from the successive steps */
    double steps = 0.0;
    for (int q = 0; q + 1 < S; ++q)
        steps = steps + orc_dist2(K, xs[q + 1], xs[q]);
    const double lam2 = S > 1 ? lam_scale * lam_scale * steps / (2.0 * (double)(S - 1)) : 0.0;
    /* one cluster at the mean */
    int C = 1;
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int q = 0; q < S; ++q)
            s = s + xs[q][k];
        cent[k] = s / (double)S;
    }
    for (int q = 0; q < S; ++q)
        prev[q] = -1;
    for (int it = 0; it < maxit; ++it) {
        /* assignment, in sample order */
        for (int q = 0; q < S; ++q) {
            int best = 0;
            double dbest = orc_dist2(K, xs[q], cent);
            for (int c = 1; c < C; ++c) {
                const double d = orc_dist2(K, xs[q], cent + (size_t)c * K);
                if (d < dbest) {
                    dbest = d;
                    best = c;
                }
            }
            if (dbest > lam2 && C < cmax) {
                memcpy(cent + (size_t)C * K, xs[q], sizeof(double) * K);
                best = C++;
            }
            labels[q] = best;
        }
        /* centres: member means (sums in sample order); drop empty clusters */
        for (int c = 0; c < C; ++c) {
            cnt[c] = 0;
            for (int k = 0; k < K; ++k)
                cent[(size_t)c * K + k] = 0.0;
        }
        for (int q = 0; q < S; ++q) {
            double *m = cent + (size_t)labels[q] * K;
            for (int k = 0; k < K; ++k)
                m[k] = m[k] + xs[q][k];
            cnt[labels[q]] += 1;
        }
        int Cn = 0;
        for (int c = 0; c < C; ++c) {
            if (cnt[c] == 0)
                continue;
            for (int k = 0; k < K; ++k)
                cent[(size_t)Cn * K + k] = cent[(size_t)c * K + k] / (double)cnt[c];
            cnt[Cn] = cnt[c];
            for (int q = 0; q < S; ++q)
                if (labels[q] == c)
                    labels[q] = Cn;
            ++Cn;
        }
        C = Cn;
        int same = 1;
        for (int q = 0; q < S; ++q) {
            same &= labels[q] == prev[q];
            prev[q] = labels[q];
        }
        if (same)
            break;
    }
    return C;
}

/* Labels (R x S, row n = entity n) and cluster counts of every entity of one
 * side of one block; samples are S x R x K as for orc_mm.  Returns the total
 * number of clusters. */
int64_t orc_lmeans(int64_t R, int32_t K, int32_t S, const double *samples, double lam_scale, int32_t cmax,
                   int32_t maxit, int32_t *labels, int32_t *nclust)
{
    int64_t total = 0;
    const double **xs = (const double **)malloc(sizeof(double *) * (size_t)S);
    double *cent = (double *)malloc(sizeof(double) * (size_t)cmax * K);
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)cmax);
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)S);
    for (int64_t n = 0; n < R; ++n) {
        for (int q = 0; q < S; ++q)
            xs[q] = samples + ((int64_t)q * R + n) * K;
        nclust[n] = orc_lmeans_one(K, S, xs, lam_scale, cmax, maxit, labels + n * S, cent, cnt, prev);
        total += nclust[n];
    }
    free(xs); free(cent); free(cnt); free(prev);
    return total;
}

/* Moment matching (as orc_mm) of the samples q of entity n with
 * labels[n * S + q] == which[n] (which[n] < 0: every sample), in sample
 * order; at least two must be selected.  count[n] = selected samples, logdet[n]
 * = log det Lambda_hat.  Returns the number of rows that took the ridge
 * (selected count <= K, or the factorisation failed). */
int64_t orc_mm_sel(int64_t R, int32_t K, int32_t S, const double *samples, const int32_t *labels,
                   const int32_t *which, double *mu, double *Lam, double *logdet, int32_t *count)
{
    int64_t ridged = 0;
    const size_t KK = (size_t)K * K;
    double *Sig = (double *)malloc(sizeof(double) * KK);
    double *L = (double *)malloc(sizeof(double) * KK);
    for (int64_t n = 0; n < R; ++n) {
        double *mn = mu + n * K;
        int m = 0;
        for (int q = 0; q < S; ++q)
            m += which[n] < 0 || labels[n * S + q] == which[n];
        count[n] = m;
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int q = 0; q < S; ++q)
                if (which[n] < 0 || labels[n * S + q] == which[n])
                    s += samples[((int64_t)q * R + n) * K + k];
            mn[k] = s / (double)m;
        }
        memset(Sig, 0, sizeof(double) * KK);
        for (int q = 0; q < S; ++q) {
            if (!(which[n] < 0 || labels[n * S + q] == which[n]))
                continue;
            const double *x = samples + ((int64_t)q * R + n) * K;
            for (int a = 0; a < K; ++a)
                for (int b = 0; b < K; ++b)
                    Sig[a * K + b] += (x[a] - mn[a]) * (x[b] - mn[b]);
        }
        for (size_t p = 0; p < KK; ++p)
            Sig[p] /= (double)(m - 1);
        int need_ridge = (m <= K) || (orc_chol(K, Sig, L) != 0);
        if (need_ridge) {
            double tr = 0.0;
            for (int k = 0; k < K; ++k)
                tr += Sig[k * K + k];
            const double delta = 1e-6 * tr / (double)K + 1e-300;
            for (int k = 0; k < K; ++k)
                Sig[k * K + k] += delta;
            orc_chol(K, Sig, L);
            ridged += 1;
        }
        double ld = 0.0;
        for (int k = 0; k < K; ++k)
            ld -= 2.0 * log(L[k * K + k]);
        logdet[n] = ld;
        orc_inverse_from_chol(K, L, Lam + n * KK);
    }
    free(Sig); free(L);
    return ridged;
}
