/*
 * bmf.h -- C ABI of the MI355X (gfx950) library for the BPMF Gibbs sweep run on
 * every data subset of posterior propagation (PP), after Qin, Blomstedt,
 * Leppaaho, Parviainen & Kaski, "Distributed Bayesian Matrix Factorization with
 * Limited Communication" (arXiv:1703.00734).
 *
 * Problem statement (Sec. 2.1, eq. MF, BMF_likelihood, BMF_likelihood_normal,
 * prior_X, prior_W): Y is a partially observed N x D matrix, Y ~ X W^T with
 * X in R^{N x K}, W in R^{D x K}; y_nd ~ N(x_n^T w_d, 1/tau) on the observed
 * set; x_n ~ N_K(mu_X, Lambda_X^-1), w_d ~ N_K(mu_W, Lambda_W^-1) with
 * Normal-Wishart hyperpriors (Sec. 5.1).  Y is split into I x J blocks
 * (Sec. 3, eq. joint_MF_posterior) and processed in the three PP stages of
 * Sec. 3.2 (eq. stage1, stage2a, stage2b, stage3; Algorithm 1) with
 * moment-matched Gaussian priors propagated between stages (Sec. 4.1), then
 * aggregated per row (Sec. 4.2, eq. post_marg_aggregation, Algorithm 2) and
 * used for prediction with posterior means (Sec. 5.2).
 *
 * Conventions for every entry point:
 *   - Every call returns a bmf_status; nothing is thrown across the ABI.  On an
 *     error the context (when there is one) keeps a message readable through
 *     bmf_last_error() until the next call on it.
 *   - Pointers named "host" are host memory, read (or written) only during the
 *     call and owned by the caller.  Device memory is either the caller's
 *     workspace (bmf_config.workspace, e.g. a torch uint8 tensor, which must
 *     outlive the context) or, when that is NULL, allocated by bmf_init and
 *     released by bmf_free.
 *   - All device work is ordered on bmf_config.stream (a hipStream_t; NULL is
 *     the default stream).  A context is not thread-safe.
 *   - Entity ids passed in (COO rows/columns, prediction pairs) are the
 *     caller's original 0-based ids; the library maps them through its own
 *     ordering and partition.
 */
#ifndef BMF_H
#define BMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bmf_ctx bmf_ctx;

typedef enum {
    BMF_OK = 0,
    BMF_EINVAL = 1,       /* bad argument or bad input data */
    BMF_ENOMEM = 2,       /* host or device allocation failed / workspace too small */
    BMF_EDEVICE = 3,      /* a HIP call failed, or no usable gfx950 device */
    BMF_ENOTPD = 4,       /* a precision matrix failed its Cholesky in FP64 */
    BMF_ESTATE = 5,       /* call out of order (e.g. stage 3 before stage 2) */
    BMF_EUNSUPPORTED = 6, /* valid request outside what this build supports (K > 64) */
    BMF_EABORT = 7        /* the progress callback asked to stop (bmf_set_progress) */
} bmf_status;

/* Storage and arithmetic of the row/column conditional updates.
 * Hyperparameter, tau, moment-matching and aggregation arithmetic is FP64 in
 * every mode.  In the FP32 and BF16 modes with K > 16, an entity with at most
 * eight entries under a propagated (moment-matched) prior skips the Cholesky:
 * its prior's factor, computed once per stage in FP64 and stored in FP32, is
 * applied directly (no entries) or updated by rank-one modifications (one to
 * eight), giving the same factor and draw up to rounding.
 *
 * BF16 mode stores the chain state itself (every X and W row) in BF16: each
 * draw is computed in FP32 from BF16 inputs, then rounded to nearest even for
 * the state, so the Normal-Wishart statistics, the tau residuals, the next
 * pass's gathers and bmf_get_state all see the rounded values.  The kept
 * samples (moment matching, prediction) and bmf_get_draw / bmf_get_sample hold
 * the FP32 draw before rounding.  Against the FP64 conditional draw from the
 * same (BF16) inputs and noise, the FP32 draw is within about 1e-5 relative
 * (FP32 arithmetic; measured at most 3e-6 per row at the benchmark sizes) and
 * the stored state is its round-to-nearest-even, within 2^-8 relative per
 * entry on top of that (the BF16 unit roundoff). */
typedef enum {
    BMF_PREC_FP64 = 0,    /* FP64 state, gathers, Gram, Cholesky and solves */
    BMF_PREC_FP32 = 1,    /* FP32 state and gathers, FP32 Gram; FP32 Cholesky with
                             FP64 fallback */
    BMF_PREC_BF16 = 2     /* BF16 state (so BF16 gathers), FP32 accumulation of
                             exact BF16 products (MFMA for K > 16), FP32 Cholesky
                             with FP64 fallback, FP32 kept samples */
} bmf_precision;

/* Row/column ordering before partitioning (Sec. 5.2): the given ids, a random
 * permutation (stable sort on a Philox key per entity), or decreasing number
 * of observations (ties by id). */
typedef enum {
    BMF_ORDER_GIVEN = 0,
    BMF_ORDER_RANDOM = 1,
    BMF_ORDER_DECREASING = 2
} bmf_order;

/* Parametric approximation of each stage's subset posteriors, propagated as
 * the next stages' priors and aggregated by Algorithm 2 (Sec. 4.1; Sec. 5.1):
 *   MM  -- moment matching: per row the mean and inverse covariance of the
 *          kept samples;
 *   DM  -- dominant mode: the kept samples of each row are clustered by
 *          lambda-means and the largest cluster is moment-matched;
 *   GMM -- mixture: the ncomp largest clusters with at least two members, each
 *          moment-matched, weights proportional to their sizes; a row under a
 *          mixture prior takes, every sweep, the component of largest
 *          responsibility pi_c N(x_n | mu_c, Lambda_c^-1) at its current value
 *          as its prior (Sec. 5.1), and aggregation uses the pooled moments
 *          (Sec. 4.2, eq. marginal_mixture).
 * lambda-means is the DP-means iteration: in sample order each sample joins its
 * nearest centre, or opens a new cluster when that centre is farther than
 * lambda (at most 16 clusters); centres move to their members' means; until the
 * assignment repeats (at most 32 rounds), starting from one cluster at the
 * mean.  lambda^2 = lambda_scale^2 times half the mean squared step between
 * successive kept samples of the row.  DM and GMM need K <= 32 and
 * max_kept <= 256. */
typedef enum {
    BMF_APPROX_MM = 0,
    BMF_APPROX_DM = 1,
    BMF_APPROX_GMM = 2
} bmf_approx;

typedef struct {
    /* data: COO training set, host memory, 0-based, no duplicate (row, col).
     * The largest row or column part times the factor row stride in bytes
     * (K rounded up to 16 bytes; K at 32 and 64) must stay below 2^32, since
     * the gather kernels form 32-bit row offsets (BMF_EUNSUPPORTED otherwise). */
    int64_t N, D;                /* matrix shape */
    int32_t K;                   /* rank, 1 <= K <= 64 */
    int64_t nnz;                 /* number of observed training entries */
    const int32_t *row;          /* host, nnz */
    const int32_t *col;          /* host, nnz */
    const float *val;            /* host, nnz, finite */
    /* partition (Sec. 3, Sec. 5.2): I row parts x J column parts of size
     * ceil(N/I) and ceil(D/J); I = J = 1 is plain BPMF */
    int32_t I, J;
    int32_t order;               /* bmf_order */
    /* Normal-Wishart hyperprior shared by X and W: mu0 (K, NULL = 0),
     * beta0 > 0, nu0 > K - 1, scale W0 (K x K row-major SPD, NULL = I) */
    const double *mu0;
    double beta0, nu0;
    const double *W0;
    /* noise precision: sample_tau != 0 draws tau ~ Gamma(shape tau_a0, rate
     * tau_b0) prior each sweep; otherwise tau = tau_fixed (Sec. 5.1) */
    int32_t sample_tau;
    double tau_a0, tau_b0, tau_fixed;
    uint64_t seed;               /* Philox4x32-10 key (low word, high word) */
    /* kept sweeps within a stage: t >= burnin && (t - burnin) % thin == 0;
     * at most max_kept are stored per stage (sizes the sample store) */
    int32_t burnin, thin, max_kept;
    int32_t precision;           /* bmf_precision */
    double pivot_theta;          /* FP32 Cholesky pivot test: a row whose pivot
                                    falls below pivot_theta * its diagonal entry
                                    is redone in FP64 (0 => 2^-10) */
    int32_t batched;             /* 1: all blocks of a stage in one launch per
                                    pass, each sweep replayed from a captured
                                    HIP graph; 0: one launch sequence per block,
                                    launched eagerly */
    int32_t lane_nnz;            /* K <= 16 update kernels: observed entries per
                                    lane when sizing lane groups; 0 = chosen by
                                    the autotuner at each stage begin (batched)
                                    or 32 (per block) */
    void *workspace;             /* device memory owned by the caller, or NULL */
    size_t workspace_bytes;      /* its size; see bmf_workspace_size */
    void *stream;                /* hipStream_t, NULL = default stream */
    int32_t approx;              /* bmf_approx (0 = moment matching) */
    double lambda_scale;         /* lambda-means scale, > 0 (0 => 2) */
    int32_t ncomp;               /* mixture components, 1..4 (0 => 3) */
    /* per-column noise precisions (Sec. 2.1, the tau_d variant of eq.
     * BMF_likelihood_normal): y_nd ~ N(x_n^T w_d, 1/tau_d), one tau_d per
     * column of each block, each with the Gamma(tau_a0, tau_b0) prior (or
     * tau_fixed when tau is not sampled) and drawn every sweep from
     * Gamma(tau_a0 + M_d/2, tau_b0 + SSE_d/2) over its M_d entries.  The row
     * update then weights each entry by its column's tau_d (the library forms
     * sqrt(tau_d) w_d and sqrt(tau_d) r_nd at the start of each sweep), the
     * column update uses its own.  FP32 and FP64 precision only. */
    int32_t tau_per_column;
    /* bmf_init lays out the ordering, partition and per-block CSR/CSC
     * (Sec. 5.2) on the GPU by default: a radix sort of one unique key per
     * entry and order, the same plan as the host planner's; it allocates and
     * frees its own temporary device memory (about 40 bytes per entry) during
     * the call.  plan_on_host != 0 keeps the whole plan on the host
     * (bmf_init_host always does). */
    int32_t plan_on_host;
} bmf_config;

/* Fill *cfg with defaults: K = 10, I = J = 1, beta0 = 2, nu0 = K, tau Gamma(1,1)
 * sampled, tau_fixed = 1, burnin = 0, thin = 1, max_kept = 1, FP32, batched,
 * lane_nnz = 0 (autotuned), pivot_theta = 2^-10, moment matching
 * (lambda_scale = 2, ncomp = 3 for the other approximations).  Data pointers
 * are NULL. */
bmf_status bmf_config_defaults(bmf_config *cfg);

/* Bytes of device workspace bmf_init needs for cfg (host only, touches no
 * device).  Validates cfg like bmf_init. */
bmf_status bmf_workspace_size(const bmf_config *cfg, size_t *bytes);

/* Validate cfg and its data, compute the global mean (centering), the
 * ordering, the I x J partition and every block's CSR and CSC (integer work,
 * exact), and upload them.  *out receives the context. */
bmf_status bmf_init(const bmf_config *cfg, bmf_ctx **out);

/* The host half of bmf_init only: validation, centering, ordering, partition
 * and CSR/CSC, with no device touched.  The context answers the introspection
 * calls bmf_block_info, bmf_global_mean, bmf_get_positions and
 * bmf_get_block_csr; every call that needs the device returns BMF_ESTATE. */
bmf_status bmf_init_host(const bmf_config *cfg, bmf_ctx **out);

/* Run nsweeps Gibbs sweeps (Sec. 5.1; Salakhutdinov & Mnih 2008b) on every
 * block of the active stage.  When no stage is active, stage 1 is begun
 * first (for I = J = 1 that is the whole of plain BPMF).  A sweep: every row
 * given W, every column given the new X, Normal-Wishart draws for each side
 * that is not propagated, then tau when sampled; kept sweeps store a sample. */
bmf_status bmf_gibbs_sweep(bmf_ctx *c, int32_t nsweeps);

/* Begin PP stage `stage` (1, 2 or 3; Sec. 3.2, Algorithm 1) and run nsweeps
 * sweeps on all of its blocks.  Beginning stage s > 1 first moment-matches
 * the kept samples of stage s - 1 (Sec. 4.1) and binds them as per-row
 * Gaussian priors: the X side of block (i, j) is propagated iff j > 0 (from
 * block (i, 0)), the W side iff i > 0 (from block (0, j)); a propagated side
 * takes no Normal-Wishart draw.  Stages must be begun in order (else
 * BMF_ESTATE); a stage with no blocks (stage 3 when I = 1 or J = 1) returns
 * BMF_OK and does nothing.  Moment matching needs at least 2 kept samples and,
 * for a well-conditioned prior, more than K of them: with S <= K the sample
 * covariance is singular, every row is ridged (counted in bmf_get_stats) and
 * the propagated prior is nearly degenerate in the missing directions. */
bmf_status bmf_pp_stage(bmf_ctx *c, int32_t stage, int32_t nsweeps);

/* Predict n entries (row[q], col[q]) (host, original ids) into out (host):
 * out[q] = y_bar + mu*_x^T mu*_w with the per-row aggregated posterior means
 * of Algorithm 2 (for a 1 x 1 partition, the sample means).  Needs at least
 * one kept sample in every block of the last stage, and every stage that has
 * blocks completed (BMF_ESTATE otherwise). */
bmf_status bmf_predict(bmf_ctx *c, int64_t n, const int32_t *row, const int32_t *col,
                       float *out);

/* Allocation-free prediction, for callers that cannot allocate device memory
 * (tight serving loops, code that must not call hipMalloc).  Same arguments,
 * ids and result as bmf_predict (the same kernel arithmetic, bit for bit), but
 * it allocates nothing: the pairs' ids and the outputs are staged through one
 * fixed device array owned by the library (12 MiB per GPU, held until the
 * process ends), and it launches only the prediction itself.  So:
 *   - n <= 1048576 pairs per call (BMF_EINVAL above that: split the request);
 *   - the aggregated means must already be current (bmf_aggregate, or a
 *     bmf_predict, since the last sweep), else BMF_ESTATE;
 *   - every context on one GPU shares that array: calls that overlap in time on
 *     one GPU (from several threads, or on streams not ordered with each other)
 *     race and must be serialised by the caller.
 * Synchronises the context's stream before returning. */
bmf_status bmf_predict_noalloc(bmf_ctx *c, int64_t n, const int32_t *row, const int32_t *col,
                               float *out);

/* Release the context (and the device memory it allocated itself). */
bmf_status bmf_free(bmf_ctx *c);

/* Message of the last failed call on c (never NULL). */
const char *bmf_last_error(const bmf_ctx *c);
const char *bmf_status_string(bmf_status s);

/* ------------------------------------------------------------------------ */
/* Introspection and test hooks (same conventions).  Blocks are numbered     */
/* b = i * J + j.  Dense host arrays are row-major FP64 in local order.      */
/* ------------------------------------------------------------------------ */

/* Shape of block b: rows R, columns C, training entries M, stage 1..3. */
bmf_status bmf_block_info(const bmf_ctx *c, int32_t b, int64_t *R, int64_t *C, int64_t *M,
                          int32_t *stage);

/* Global mean of the training values (the centering constant y_bar). */
bmf_status bmf_global_mean(const bmf_ctx *c, double *ybar);

/* Ordering/partition: pos_row[N], pos_col[D] = position of each original id
 * in the chosen order (block = pos / ceil(N/I), local id = pos % ceil(N/I)). */
bmf_status bmf_get_positions(const bmf_ctx *c, int64_t *pos_row, int64_t *pos_col);

/* Block b's CSR (which = 0: ptr[R+1], idx[M] = local columns, entry[M] = index
 * of the entry in the caller's COO arrays) or CSC (which = 1: ptr[C+1], idx =
 * local rows).  ptr is relative to the block (ptr[0] = 0).  Any output may be
 * NULL. */
bmf_status bmf_get_block_csr(const bmf_ctx *c, int32_t b, int32_t which, int64_t *ptr,
                             int32_t *idx, int64_t *entry);

/* State of block b (which must belong to the active stage): X (R x K),
 * W (C x K), hyper = [Lambda_X (K x K), mu_X (K), Lambda_W (K x K), mu_W (K)],
 * tau.  NULL outputs/inputs are skipped.  set_state converts to the storage
 * precision of the context. */
bmf_status bmf_get_state(bmf_ctx *c, int32_t b, double *X, double *W, double *hyper, double *tau);
bmf_status bmf_set_state(bmf_ctx *c, int32_t b, const double *X, const double *W,
                         const double *hyper, const double *tau);

/* One sub-step of a sweep on block b at sweep index t (the Philox counter):
 * which = 0 rows, 1 columns, 2 Normal-Wishart draw for X, 3 for W, 4 tau. */
bmf_status bmf_step(bmf_ctx *c, int32_t b, int32_t which, int64_t t);

/* The draws of the last bmf_step of kind 0 (side 0) or 1 (side 1) on block b,
 * in the sample precision (FP64, or FP32 in the FP32 and BF16 modes), before
 * they are rounded to the state precision: x (n x K). */
bmf_status bmf_get_draw(bmf_ctx *c, int32_t b, int32_t side, double *x);

/* Moment-matched per-row Gaussian of block b (side 0 = X rows, 1 = W columns)
 * after its stage has been finalised: mu (n x K) and Lambda (n x K x K, full
 * symmetric).  Either output may be NULL. */
bmf_status bmf_get_mm(bmf_ctx *c, int32_t b, int32_t side, double *mu, double *Lam);

/* Cluster label of every kept sample of every row of block b (side 0 = X rows,
 * 1 = W columns) after its stage has been finalised under the dominant-mode or
 * mixture approximation (Sec. 5.1, lambda-means): labels (n x S, host), S the
 * number of samples the stage kept; labels are 0-based in the order the
 * clusters were opened.  BMF_ESTATE under moment matching. */
bmf_status bmf_get_clusters(bmf_ctx *c, int32_t b, int32_t side, int32_t *labels);

/* Component comp (0-based, by decreasing size) of the per-row fit of block b
 * under the dominant-mode (comp 0 only) or mixture approximation: weights pi
 * (n; 0 for a row with fewer components), means mu (n x K), precisions Lambda
 * (n x K x K), log det Lambda (n).  Any output may be NULL. */
bmf_status bmf_get_component(bmf_ctx *c, int32_t b, int32_t side, int32_t comp, double *pi, double *mu,
                             double *Lam, double *logdet);

/* Per-column noise precisions tau_d of block b (C values, host) when
 * bmf_config.tau_per_column is set and b is in the active stage
 * (BMF_ESTATE otherwise). */
bmf_status bmf_get_tau_cols(bmf_ctx *c, int32_t b, double *tau);

/* Aggregated per-row posterior means (after bmf_predict or bmf_aggregate):
 * side 0: mu_x (N x K) in original row ids; side 1: mu_w (D x K). */
bmf_status bmf_aggregate(bmf_ctx *c);
bmf_status bmf_get_aggregate(bmf_ctx *c, int32_t side, double *mu);

/* Counters accumulated since bmf_init: rows redone in FP64 after a failed
 * FP32 pivot test, rows whose FP64 precision failed its Cholesky, rows whose
 * moment-matched covariance needed the ridge, aggregation eigenvalue
 * corrections; and train_sse, the residual sum of squares of the centred
 * training values, sum over observed (r_nd - x_n^T w_d)^2, over every block of
 * the active stage, as evaluated by the last sweep's column pass (the
 * statistic of the tau draw, eq. BMF_likelihood_normal; FP64; 0 before the
 * first sweep of a stage).  Any output may be NULL. */
bmf_status bmf_get_stats(bmf_ctx *c, int64_t *fallback_rows, int64_t *nonpd_rows,
                         int64_t *mm_ridged, int64_t *agg_corrections, double *train_sse);

/* Kept sample `slot` (0 = first kept sweep) of block b of the active stage,
 * side 0 (X rows) or 1 (W columns), in the sample precision (FP64, or the
 * FP32 draw before any BF16 rounding): x (n x K, FP64 host).  BMF_EINVAL when
 * the slot has not been written in this stage. */
bmf_status bmf_get_sample(bmf_ctx *c, int32_t b, int32_t side, int32_t slot, double *x);

/* Progress callback: called on the host before every sweep that
 * bmf_gibbs_sweep or bmf_pp_stage is about to enqueue, with the stage and the
 * sweep index within it.  A non-zero return stops the call with BMF_EABORT
 * before that sweep is enqueued: the context then holds the consistent state
 * after the previous sweep, which bmf_save_state can write and a later
 * bmf_gibbs_sweep continues exactly (every draw is addressed by its Philox
 * counter).  fn = NULL removes the callback. */
typedef int32_t (*bmf_progress_fn)(void *user, int32_t stage, int64_t sweep);
bmf_status bmf_set_progress(bmf_ctx *c, bmf_progress_fn fn, void *user);

/* Checkpoint and resume at stage and sweep granularity (the paper's stages
 * exchange their propagated posteriors through files, Sec. 5.2 footnote).
 * bmf_save_state writes one flat binary file (host path): a header (magic,
 * version, N, D, K, nnz, I, J, order, precision, seed, sampling settings and a
 * 64-bit fingerprint of the training data), the stage bookkeeping (active
 * stage, moment-matched stages, sweeps run, samples kept, the update
 * kernels' lane-group sizing), the counters, and the device arrays that the
 * rest of the chain depends on: every factor row, hyperparameter slot and tau
 * of the active stage's blocks, its kept samples, the moment-matched rows of
 * every finished stage and their prior factors.  bmf_load_state restores them
 * into a context made by bmf_init with the same configuration and data
 * (BMF_EINVAL on a header or fingerprint mismatch or a short file); the
 * chain then continues bit for bit as if it had not been interrupted.  Both
 * synchronise the context's stream. */
bmf_status bmf_save_state(bmf_ctx *c, const char *path);
bmf_status bmf_load_state(bmf_ctx *c, const char *path);

/* Per-kernel timing: when enabled, every launch is bracketed by HIP events on
 * the context's stream (sweeps are then launched eagerly, not from the graph).
 * bmf_kernel_times returns, for up to n kernel classes, their names (static
 * strings), the launch counts and total milliseconds accumulated since the
 * context was created, and the number of classes in *count. */
bmf_status bmf_enable_timing(bmf_ctx *c, int32_t on);
bmf_status bmf_kernel_times(bmf_ctx *c, int32_t n, const char **names, int64_t *launches,
                            double *ms, int32_t *count);

/* Lane-group sizing of the active stage's K <= 16 update kernels: observed
 * entries per lane of the row pass and of the column pass (autotuned or set). */
bmf_status bmf_get_schedule(const bmf_ctx *c, int32_t *lane_nnz_rows, int32_t *lane_nnz_cols);

/* Rows + columns updated per sweep and training entries visited per sweep,
 * summed over the blocks of the active stage. */
bmf_status bmf_stage_work(const bmf_ctx *c, int64_t *row_updates, int64_t *ratings);

#ifdef __cplusplus
}
#endif

#endif /* BMF_H */
