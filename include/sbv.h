/*
 * sbv.h -- C ABI of the MI355X Scaled Block Vecchia (SBV) log-likelihood library
 * (libsbv.so).  Plain pointers and sizes only.
 *
 * The method: the inputs X (n x d) are scaled by anisotropic ranges (Alg. 2),
 * clustered into blocks (k-means, or random anchors, Alg. 3), the blocks are put
 * in a uniformly random order (Alg. 1), and every block conditions on the m points
 * of strictly earlier blocks nearest its centroid (Alg. 4, Sec. 4.2 Eq.
 * (mmsearchingBV)).  The log-likelihood is the sum over blocks of the
 * conditional Gaussian log-densities of Alg. 5 with the Matern kernel of
 * Sec. 4.4 Eq. (scale)/(maternkernel).
 *
 * Conventions shared by every entry point:
 *  - theta of one dataset packs d+2 log-parameters
 *      [log beta_1 .. log beta_d, log sigma^2, log tau^2]
 *    (ranges, process variance, nugget).  The nugget is added on the diagonal
 *    only.  The Matern smoothness is fixed per dataset and passed as two_nu in
 *    {1, 3, 5, 7} (nu = 1/2, 3/2, 5/2, 7/2, closed forms of Eq. (maternkernel)
 *    taken literally in r, i.e. without a sqrt(2 nu) factor).
 *  - Each block term carries -(b_i/2) log(2 pi), so conditioning every block on
 *    all earlier points reproduces the exact log-likelihood of Eq. (1).
 *  - Ownership: the caller owns every buffer it passes; the library copies what
 *    it keeps (a handle owns its device copies).  Host entry points are
 *    synchronous.  *_dev entry points take device pointers and a HIP stream
 *    (passed as void*) and are asynchronous: their buffers must stay valid until
 *    the stream reaches that point.
 *  - Errors: every function returns an sbv_status; on failure outputs are left
 *    untouched unless stated, and sbv_last_error() describes the failure.
 *  - One handle must not be used from two host threads at once.
 */
#ifndef SBV_H
#define SBV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SBV_OK = 0,
  SBV_E_INVAL = 1,  /* bad argument (NaN/inf, sizes, unsupported nu, bad structure) */
  SBV_E_NOMEM = 2,  /* host or device allocation failed                             */
  SBV_E_DEVICE = 3, /* HIP error or no device                                       */
  SBV_E_NOTPD = 4,  /* a block is not positive definite even in FP64                */
  SBV_E_NOCONV = 5  /* sbv_fit reached its evaluation limit                          */
} sbv_status;

enum { SBV_FP64 = 0, SBV_FP32 = 1 };
enum { SBV_KMEANS = 0, SBV_RAC = 1 };
enum { SBV_NELDER_MEAD = 0, SBV_LBFGS = 1 };

/* Opaque handle: one dataset with its block structure, resident on the device. */
typedef struct sbv_blocks_s* sbv_blocks;

typedef struct {
  int32_t method;      /* SBV_KMEANS or SBV_RAC (Alg. 3: random anchors, no Lloyd pass) */
  int32_t lloyd_iters; /* k-means passes after the anchor assignment (ignored for RAC)   */
  int32_t min_bs;      /* smallest block size (0: no bound)                              */
  int32_t max_bs;      /* largest block size (0: no bound)                               */
  int32_t n_slabs;     /* Alg. 2 slabs along the most relevant scaled dimension (0, 1:   */
                       /* one slab); blocks are clustered within their slab             */
  uint64_t seed;       /* anchors use seed, the block order seed + 1                     */
  double nns_alpha;    /* neighbour search: > 0 filtered with this expansion factor     */
                       /* (Eq. (distancethreashold)), < 0 brute force, 0 automatic      */
} sbv_build_opts;

/*
 * Build the block structure on the device (Alg. 2 scaling by beta_build, Alg. 3
 * anchors + optional k-means, random block order of Alg. 1, block centroids and
 * the exact m nearest points of strictly earlier blocks of Alg. 4: a filtered
 * search whose distance threshold follows Eq. (distancethreashold) with a
 * conservative candidate test and a retry at twice the threshold until the
 * answer is provably exact, or brute force; both give the same sets).  X: host, row-major n x d FP64; y: host, n FP64 (may be
 * NULL: observations set to 0).  n_blocks: requested block count K (<= n); the
 * final count can differ when size bounds split or merge clusters.  m >= 0.
 * On success *out owns device copies of X and y in block order.
 */
sbv_status sbv_build_blocks(const double* X, const double* y, int64_t n, int32_t d,
                            const double* beta_build, int64_t n_blocks, int32_t m,
                            const sbv_build_opts* opts, sbv_blocks* out);

/*
 * Create a handle from an explicit structure (exchange format).  block_ptr
 * (K+1) and block_pts (n) list the blocks in rank order as original point ids;
 * nn_ptr (K+1) and nn_idx (nn_ptr[K]) list each block's conditioning points as
 * original ids.  Every neighbour must belong to a strictly earlier block and
 * every point to exactly one block; otherwise SBV_E_INVAL.  Conditioning and
 * block sizes are limited to m_i + b_i <= sbv_max_joint_size().
 */
sbv_status sbv_blocks_import(const double* X, const double* y, int64_t n, int32_t d, int64_t K,
                             const int64_t* block_ptr, const int64_t* block_pts,
                             const int64_t* nn_ptr, const int64_t* nn_idx, sbv_blocks* out);

/* Sizes of a handle: points, dimension, blocks, total conditioning entries. */
sbv_status sbv_blocks_info(sbv_blocks h, int64_t* n, int32_t* d, int64_t* K, int64_t* nnz_nn);

/* Read the structure back in the exchange format (host arrays sized by info). */
sbv_status sbv_blocks_export(sbv_blocks h, int64_t* block_ptr, int64_t* block_pts,
                             int64_t* nn_ptr, int64_t* nn_idx);

/* Replace the observations (host, n FP64 in original point order). */
sbv_status sbv_blocks_set_y(sbv_blocks h, const double* y);

/* Replace the observations from a device buffer (n FP64, original order). */
sbv_status sbv_blocks_set_y_dev(sbv_blocks h, const double* y_dev, void* stream);

/* Free a handle; NULL-safe. */
void sbv_blocks_free(sbv_blocks h);

/* Largest joint size m_i + b_i a block may have. */
int32_t sbv_max_joint_size(void);

/*
 * SBV log-likelihood of n_sets datasets (Alg. 5 summed over blocks, Alg. 1
 * Step 5 as an on-device FP64 reduction).  theta: host, packed per set
 * (d_j + 2 values each, sets in order); two_nu: host, one per set; prec:
 * SBV_FP64, or SBV_FP32 (FP32 covariance and Cholesky, FP64 log-det and
 * quadratic-form accumulation; blocks with a pivot below threshold are
 * recomputed in FP64).  loglik: host, n_sets values.  If a block is not
 * positive definite in FP64, that set's value is -inf and SBV_E_NOTPD is
 * returned (other sets stay valid).
 */
sbv_status sbv_loglik(const sbv_blocks* sets, int32_t n_sets, const double* theta,
                      const int32_t* two_nu, int32_t prec, double* loglik);

/* Device variant: theta_dev and loglik_dev are device pointers; the work is
 * queued on `stream` (a hipStream_t; NULL = default stream) with no host
 * synchronisation.  Non-positive-definite sets give -inf. */
sbv_status sbv_loglik_dev(const sbv_blocks* sets, int32_t n_sets, const double* theta_dev,
                          const int32_t* two_nu, int32_t prec, double* loglik_dev, void* stream);

/*
 * For callers that cannot allocate device memory (code queued inside a HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * log-likelihood of ONE handle, as sbv_loglik_dev computes it (same kernels,
 * size buckets and reduction with the default kernel choice, so the same value
 * bit for bit unless sbv_autotune changed that choice), queued on `stream` (a hipStream_t; NULL = default stream) with no
 * allocation and no host synchronisation.  theta_dev (d+2 log-parameters) and
 * loglik_dev (1 value, -inf when a block is not positive definite) are device
 * pointers owned by the caller.  The per-block terms, flags, FP32 fallback
 * lists and counters live in a fixed device array inside the library (about
 * 5 MB per device, held until the process ends), so:
 *  - the handle may have at most 262,144 blocks and joint sizes m_i + b_i up
 *    to 272 (larger handles: SBV_E_INVAL, nothing queued);
 *  - calls that overlap on one device (two host threads, or two streams
 *    without ordering between them) share that array and race; order them;
 *  - sbv_blocks_terms does not see the block terms of these calls.
 */
sbv_status sbv_loglik_noalloc_dev(sbv_blocks h, const double* theta_dev, int32_t two_nu, int32_t prec,
                                  double* loglik_dev, void* stream);

/*
 * Log-likelihood and its gradient with respect to the packed log-parameters
 * (structure and nu held fixed), from a hand-written adjoint of the block
 * factorisation.  grad: n_sets packed (d_j + 2) values, same order as theta.
 * A set with a block that is not positive definite in FP64 gets l = -inf and
 * a NaN gradient (host variant: SBV_E_NOTPD naming the set; other sets stay
 * valid).
 */
sbv_status sbv_loglik_grad(const sbv_blocks* sets, int32_t n_sets, const double* theta,
                           const int32_t* two_nu, int32_t prec, double* loglik, double* grad);
sbv_status sbv_loglik_grad_dev(const sbv_blocks* sets, int32_t n_sets, const double* theta_dev,
                               const int32_t* two_nu, int32_t prec, double* loglik_dev,
                               double* grad_dev, void* stream);

/*
 * Vecchia conditional simulation on the handle's structure: blocks are visited
 * in rank order (level by level on the device) and each draws
 *   y_B = Sigma_BJ Sigma_JJ^{-1} y_J + L' xi_B,  L' = chol(Sigma_BB - Sigma_BJ Sigma_JJ^{-1} Sigma_JB),
 * i.e. the conditional mean and covariance of Alg. 5 Step 1 (Sec. 5.5).  With
 * every earlier point in J this is an exact draw from N(0, Sigma).  theta: d+2
 * log-parameters; xi: n standard-normal innovations in original point order
 * (drawn by the caller); y: n outputs in original order (may be NULL).  The
 * simulated observations also replace the handle's observations.
 */
sbv_status sbv_sample(sbv_blocks h, const double* theta, int32_t two_nu, const double* xi, double* y);
sbv_status sbv_sample_dev(sbv_blocks h, const double* theta_dev, int32_t two_nu, const double* xi_dev,
                          double* y_dev, void* stream);

/* ---- prediction (Sec. 5.5 GP Prediction; Sec. 4.2 predictive product) ----
 * New inputs X* are grouped into prediction blocks B*_j; each block takes the
 * m_pred observed points nearest its centroid (in beta_build-scaled space,
 * exact search over every observed point) as NN(B*_j), and
 *   p(y* | y) ~ prod_j p(y_{B*_j} | y_{NN(B*_j)}).
 * For every block, Alg. 5 Step 1 on [NN(B*_j); B*_j] gives the conditional mean
 * mu_new and covariance Sigma_new; the library reports mu_new and the
 * predictive variance diag(Sigma_new) of a new observation (the nugget is on
 * Sigma_new's diagonal).  A prediction structure refers to its observed
 * handle, which must outlive it; predictions use the handle's current
 * observations.  Joint sizes m_pred + |B*_j| are limited to 272.
 */
typedef struct sbv_pred_s* sbv_pred;

/* Build a prediction structure: X* (host, row-major n_pred x d) clustered as
 * sbv_build_blocks does (opts; no conditioning among new points), then the
 * m_pred nearest observed points of each block.  n_blocks <= n_pred. */
sbv_status sbv_pred_build(sbv_blocks h, const double* Xp, int64_t n_pred, const double* beta_build,
                          int64_t n_blocks, int32_t m_pred, const sbv_build_opts* opts, sbv_pred* out);

/* Explicit prediction structure (exchange format): block_ptr (K+1) and
 * block_pts (n_pred) list the blocks as ids of X*; nn_ptr (K+1) and nn_idx
 * list each block's conditioning points as observed ids (original order of the
 * handle's points).  Bad ids, a non-permutation or a joint size above 272:
 * SBV_E_INVAL. */
sbv_status sbv_pred_import(sbv_blocks h, const double* Xp, int64_t n_pred, int64_t K, const int64_t* block_ptr,
                           const int64_t* block_pts, const int64_t* nn_ptr, const int64_t* nn_idx, sbv_pred* out);
sbv_status sbv_pred_info(sbv_pred p, int64_t* n_pred, int64_t* K, int64_t* nnz_nn);
sbv_status sbv_pred_export(sbv_pred p, int64_t* block_ptr, int64_t* block_pts, int64_t* nn_ptr, int64_t* nn_idx);
void sbv_pred_free(sbv_pred p); /* NULL-safe */

/* Predictive means and variances at theta (host, d+2 log-parameters): mean and
 * var are host arrays of n_pred values in the order of X*.  A block that is
 * not positive definite in FP64 gives NaN for its points and SBV_E_NOTPD. */
sbv_status sbv_predict(sbv_pred p, const double* theta, int32_t two_nu, double* mean, double* var);

/* Conditional simulation of predictions (Sec. 5.5): n_draws draws per point
 * from N(mean_j, var_j) with the caller's standard-normal innovations xi_dev
 * (device, n_draws x n_pred, draw-major), summarised on the device as
 * stats_dev (4 n_pred values: sample means, sample variances with divisor
 * n_draws - 1, then the lower and upper ends of the 95 % interval
 * mean -/+ 1.959964 sd).  mean_dev, var_dev: device, n_pred.  Asynchronous on
 * `stream`. */
sbv_status sbv_predict_draws_dev(const double* mean_dev, const double* var_dev, int64_t n_pred, const double* xi_dev,
                                 int32_t n_draws, double* stats_dev, void* stream);

/* Options of the maximum-likelihood driver. */
typedef struct {
  int32_t optimizer;          /* SBV_NELDER_MEAD (values only) or SBV_LBFGS (values + gradients)   */
  int32_t prec;               /* SBV_FP64 or SBV_FP32 evaluations                                  */
  int32_t fp64_polish;        /* with SBV_FP32: continue in FP64 from the FP32 optimum; the FP32    */
                              /* phase then stops at a relative change of max(ftol, 1e-7), and for */
                              /* L-BFGS at its first failed line search (8 trials each)            */
  int32_t max_evals;          /* objective evaluations allowed (-> SBV_E_NOCONV when reached)       */
  double ftol;                /* Nelder-Mead: stop when the simplex spread of -l is <= ftol |l|;   */
                              /* L-BFGS: stop when one iteration changes -l by <= ftol |l|         */
  double gtol;                /* L-BFGS: stop when max |dl/dtheta_k| <= gtol                        */
  int32_t rebuild_rounds;     /* outer rounds that rebuild the structure at the fitted ranges and   */
                              /* refit (0: the structure stays fixed); needs a built handle         */
  int32_t lbfgs_m;            /* L-BFGS memory (0: 10)                                              */
  double init_step;           /* Nelder-Mead initial simplex edge in log-parameter units (0: 0.5)  */
  const char* checkpoint_path;/* optional JSON state file, rewritten every iteration; if it exists */
                              /* at the start the run resumes from it                               */
} sbv_fit_opts;

/* Objective of sbv_minimize: returns f(x) and, when grad != NULL, its gradient.
 * A non-finite return marks x as outside the domain. */
typedef double (*sbv_objective)(const double* x, double* grad, void* ctx);

/*
 * Minimise fn over n variables from x (overwritten with the best point):
 * Nelder-Mead (1965) or L-BFGS (Liu & Nocedal 1989) with a strong-Wolfe line
 * search, per opts (prec/fp64_polish/rebuild_rounds ignored).  Returns
 * SBV_E_NOCONV when max_evals is reached first (x, fbest still written).
 */
sbv_status sbv_minimize(int32_t method, int32_t n, double* x, sbv_objective fn, void* ctx,
                        const sbv_fit_opts* opts, double* fbest, int32_t* n_evals);

/*
 * Maximum-likelihood estimate of theta (the d+2 log-parameters) on one handle,
 * maximising the SBV log-likelihood with the device evaluations: the
 * optimiser loop of Alg. 1 (Steps 4-5 repeated until convergence; Sec. 8 runs
 * it with NLopt).  theta0: host, d+2 finite values (else SBV_E_INVAL).
 * theta_hat receives the optimum, loglik_fp64 a final FP64 evaluation there
 * (always FP64, whatever o->prec), n_evals the objective evaluations used
 * (all rounds), seconds the wall time.  The structure is built at fixed
 * ranges (Sec. 4.4 scales the inputs before clustering); with
 * o->rebuild_rounds = R > 0 the fit is followed by R rounds that rebuild the
 * handle's structure with its own recipe (sbv_build_blocks arguments) at the
 * fitted ranges exp(theta_hat[0:d]) and continue the fit from there, so the
 * handle then holds the last rebuilt structure (handles from
 * sbv_blocks_import: SBV_E_INVAL).  SBV_E_NOCONV: max_evals reached (outputs
 * still written).
 */
sbv_status sbv_fit(sbv_blocks set, const double* theta0, int32_t two_nu, const sbv_fit_opts* o,
                   double* theta_hat, double* loglik_fp64, int32_t* n_evals, double* seconds);

/* ---- learned warm start ------------------------------------------------
 * A fully connected FP32 network in -> hidden (x layers, GELU in its exact
 * erf form) -> out, trained and run on the device by the library's own
 * kernels (tiled GEMM with bias/GELU epilogues, GELU backward, MSE, Adam), that
 * maps summary statistics of a dataset to a starting theta for sbv_fit.
 * Parameters are packed layer by layer as W (outputs x inputs, row-major) then
 * b; initialisation is He-normal from SplitMix64(seed).
 */
typedef struct sbv_mlp_s* sbv_mlp;

sbv_status sbv_mlp_create(int32_t in, int32_t hidden, int32_t layers, int32_t out, uint64_t seed,
                          sbv_mlp* h);
void sbv_mlp_free(sbv_mlp h);
int64_t sbv_mlp_num_params(sbv_mlp h);
sbv_status sbv_mlp_get_params(sbv_mlp h, float* params);
sbv_status sbv_mlp_set_params(sbv_mlp h, const float* params);
/* Mean-squared-error loss of one batch (X: n x in, Y: n x out, host, used as
 * given -- no standardisation) and its gradient (host, num_params floats). */
sbv_status sbv_mlp_loss_grad(sbv_mlp h, const float* X, const float* Y, int32_t n, float* loss, float* grad);
/* Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8) on column-standardised X and Y
 * (statistics kept in the handle) for `epochs` shuffled passes of `batch`
 * rows; final_loss = mean batch loss of the last epoch (standardised units). */
sbv_status sbv_mlp_train(sbv_mlp h, const float* X, const float* Y, int64_t n, int32_t epochs,
                         int32_t batch, float lr, uint64_t seed, float* final_loss);
/* Predictions for n rows of raw features (standardisation applied and undone). */
sbv_status sbv_mlp_predict(sbv_mlp h, const float* X, int64_t n, float* Y);
sbv_status sbv_mlp_save(sbv_mlp h, const char* path);
sbv_status sbv_mlp_load(const char* path, sbv_mlp* h);
/*
 * Summary statistics of a dataset (4 + 5 (d + 2) values, 64 for d = 10) on a
 * subsample of min(n, sub_n) points chosen by SplitMix64(seed): log var(y),
 * log mean 1/2 (y_i - y_nn1(i))^2, and for the 1st, 2nd, 4th, 8th and 16th
 * Euclidean neighbour the least-squares coefficients of the scaled
 * semivariance 1/2 (y_i - y_j)^2 / var(y) on [1, dx_1^2 .. dx_d^2] with the
 * fit's R^2, then d/10 and 1.  X row-major n x d, y n values, both host FP64.
 */
sbv_status sbv_features(const double* X, const double* y, int64_t n, int32_t d, int64_t sub_n, uint64_t seed,
                        double* feat);

/*
 * Batched evaluation of many datasets as one captured launch sequence.  The
 * first call for a (sets, two_nu, prec, with_grad) combination captures every
 * kernel of the evaluation -- all size buckets of all sets, the FP32 fallback
 * pass, the reductions -- into a hipGraph; later calls replay it.  theta_dev
 * (packed per set) is copied into the plan's fixed parameter buffer before the
 * replay and loglik_dev (n_sets) / grad_dev (packed per set, with_grad only)
 * are copied out after it, all on `stream`.
 */
sbv_status sbv_eval_graph_dev(const sbv_blocks* sets, int32_t n_sets, const double* theta_dev,
                              const int32_t* two_nu, int32_t prec, int32_t with_grad, double* loglik_dev,
                              double* grad_dev, void* stream);

/*
 * Autotuner: for every size bucket of the sets' plan, time `reps` launches of
 * each kernel variant able to hold the bucket's joint sizes (tile capacity and
 * wave count), with and without the lookahead schedule (the next diagonal tile
 * factored during the current trailing update), at theta (host, packed per
 * set) and precision prec, and keep the fastest for later evaluations.
 * chosen_tiles (optional, 16 entries) receives the chosen tile capacity per
 * bucket, longest bucket first; chosen_lookahead (optional, 16 entries) 1
 * where the lookahead schedule won, else 0 (always 0 for the large-block
 * bucket, which has a single schedule); chosen_waves (optional, 16 entries)
 * the waves per compute unit of the chosen kernel (waves per workgroup times
 * the workgroups it is built to share a unit with; the 16-wave kernels and the
 * two-workgroups-per-unit kernels exist for FP32 only).  Then whole evaluations with one launch per size bucket are
 * timed against ONE persistent launch for all register-path blocks of all
 * sets (the largest chosen variant, workgroups taking blocks longest first
 * from a device counter); chosen_persistent (optional) receives 1 when the
 * persistent launch won.  The environment variable SBV_PERSISTENT=1 / =0
 * overrides that choice at evaluation time.  Synchronous.
 */
sbv_status sbv_autotune(const sbv_blocks* sets, int32_t n_sets, const int32_t* two_nu, const double* theta,
                        int32_t prec, int32_t reps, int32_t* chosen_tiles, int32_t* chosen_lookahead,
                        int32_t* chosen_waves, int32_t* chosen_persistent);

/*
 * Dense covariance matrix of Eq. (maternkernel) between two point lists, on the
 * device: out_dev[a * nb + b] = sigma^2 rho(r_ab) with r_ab the distance of
 * Sec. 4.4 Eq. (scale), plus tau^2 when same != 0 and a == b (the two lists
 * are the same observations).  Xa_dev (na x d), Xb_dev (nb x d), theta_dev
 * (d + 2 log-parameters) and out_dev (na x nb, row-major) are device buffers;
 * asynchronous on `stream`.  For exact-GP comparisons (Eq. (1), the KL
 * divergence of Eq. (kldivergence)) and data generation at small n.
 */
sbv_status sbv_cov_matrix_dev(const double* Xa_dev, int64_t na, const double* Xb_dev, int64_t nb, int32_t d,
                              const double* theta_dev, int32_t two_nu, int32_t same, double* out_dev, void* stream);

/* Number of blocks recomputed in FP64 by the last SBV_FP32 evaluation of this
 * handle (synchronises the device). */
sbv_status sbv_blocks_fallback_count(sbv_blocks h, int64_t* count);

/* Per-block terms l_i of the last evaluation of this handle, in rank order
 * (host, K values; synchronises the device). */
sbv_status sbv_blocks_terms(sbv_blocks h, double* terms);

/*
 * Measurement hooks (used by the benchmark).  sbv_timing_enable(1) makes every
 * subsequent evaluation bracket each kernel-variant launch with HIP events on
 * the launch stream; sbv_timing_read sums the elapsed milliseconds and launch
 * counts per size bucket for one precision (arrays of length sbv_timing_read's
 * *n_variants, at most 16; synchronises the device).  A size bucket holds the
 * blocks whose smallest fitting kernel variant has that index.
 * sbv_timing_enable(0) discards the records.  sbv_plan_flops reports, per size
 * bucket, the algorithmic FLOP sum_i (nA_i^3/3 + nA_i^2) of one evaluation of
 * these sets (nA_i = m_i + b_i) and the tile capacity (16-row tiles) of the
 * FP64 kernel launched for it, which the autotuner may have raised.
 */
sbv_status sbv_timing_enable(int32_t on);
sbv_status sbv_timing_read(int32_t prec, int32_t* n_variants, double* ms_total, int64_t* launches);
sbv_status sbv_plan_flops(const sbv_blocks* sets, int32_t n_sets, const int32_t* two_nu, double* flops,
                          int32_t* tiles_of_variant, int32_t* n_variants);

/* Message of the last failure on the calling thread (valid until the next call). */
const char* sbv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SBV_H */
