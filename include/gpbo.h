/*
 * gpbo.h -- C ABI of the MI355X Gaussian-process surrogate / expected-
 * improvement engine.
 *
 * What it computes.  The paper's search method (Sec. III-A) trains a surrogate
 * model on the configurations evaluated so far, lets an acquisition function
 * choose the next configuration, evaluates it and retrains; Sec. IV-D names
 * the surrogate -- a Gaussian process whose training cost is cubic in the
 * number N of evaluations -- and runs the independent (or merged) sub-searches
 * of a tuning problem in parallel.  This library is the data-parallel inner
 * step of that loop for one sub-search or a batch of them:
 *
 *   observations (X, y) --gpbo_fit--> model --gpbo_score(X*)--> mu, sigma, EI,
 *                                                               argmax EI
 *
 * The paper does not give the Gaussian-process formulas; the library uses the
 * textbook ones (Rasmussen & Williams 2006, Alg. 2.1 and eqs. 2.25-2.26, 4.9,
 * 4.17) and the closed-form expected improvement for minimisation (Jones,
 * Schonlau & Welch 1998, eq. 15).  A learned prescreen (an MLP ensemble trained
 * on the search's own evaluations) narrows million-point candidate pools
 * before the exact Gaussian process re-scores the survivors.
 *
 * Conventions for every entry point.
 *   - Every call returns a gpbo_status.  Nothing is thrown across the ABI.
 *   - "device" pointers are HIP device memory on the context's device;
 *     "host" pointers are ordinary host memory.  All matrices are row-major.
 *   - The caller owns every buffer it passes.  The library copies what it
 *     keeps (a model holds its own copy of X and its factors), so the caller
 *     may free its inputs as soon as a call returns.
 *   - Work is queued on the context's HIP stream and runs asynchronously,
 *     except where an entry point says it synchronises.
 *   - On a non-OK status the outputs are undefined; gpbo_last_error() gives a
 *     one-line description.
 *   - A context is used by one host thread at a time.
 */
#ifndef GPBO_H
#define GPBO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GPBO_OK = 0,
  GPBO_E_INVALID_ARG = 1,  /* a size, pointer or enum is out of range          */
  GPBO_E_NOT_PD = 2,       /* K(X,X) + noise I is not numerically positive-    */
                           /* definite; the failing pivot is reported          */
  GPBO_E_NONFINITE = 3,    /* X or y holds a NaN or an infinity                */
  GPBO_E_OOM = 4,          /* a device allocation failed                       */
  GPBO_E_HIP = 5,          /* the HIP runtime reported an error (or no device) */
  GPBO_E_UNSUPPORTED = 6   /* a valid request this build does not implement    */
} gpbo_status;

/* Covariance functions, both with one lengthscale per input dimension.
 *   SE:        k(a,b) = sf2 * exp(-r^2 / 2)                       (R&W eq. 4.9)
 *   MATERN52:  k(a,b) = sf2 * (1 + sqrt5 r + 5 r^2 / 3) exp(-sqrt5 r) (eq. 4.17)
 * with r^2 = sum_k ((a_k - b_k) / l_k)^2.                                    */
typedef enum { GPBO_KERNEL_SE = 0, GPBO_KERNEL_MATERN52 = 1 } gpbo_kernel;

/* Arithmetic of the scoring contractions (cross-covariance and the posterior
 * products).  The fit is always float64.
 *   FP64: everything in float64; outputs are double.
 *   FP32: cross-covariance in float32, posterior products on float32 matrix
 *         cores with float32 accumulation; outputs are float.  A model whose
 *         K is ill-conditioned (model statistic [7] above
 *         GPBO_ESCALATE_KINV) is scored with float64 arithmetic instead --
 *         float64 cross-covariance, mean and matrix-core products, same
 *         float inputs and outputs -- so that the posterior mean and
 *         standard deviation stay within 1e-4 (relative) of float64.  The
 *         decision is taken on the device when the fit's statistics have
 *         not been read yet.  The large-n path (gpbo_ctx_set_score_path)
 *         does not escalate.
 *   BF16: cross-covariance computed in float32 and rounded to bfloat16, the
 *         inverse Cholesky factor rounded to bfloat16, products on bfloat16
 *         matrix cores with float32 accumulation; outputs are float.  No
 *         escalation: errors grow with the conditioning of K.              */
typedef enum { GPBO_FP64 = 0, GPBO_FP32 = 1, GPBO_BF16 = 2 } gpbo_precision;

/* Optional device allocator.  alloc returns device memory of at least `bytes`
 * bytes usable on `stream` (NULL on failure); free releases it.  With no
 * allocator the library calls hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} gpbo_allocator;

typedef struct gpbo_ctx_s* gpbo_ctx;
typedef struct gpbo_model_s* gpbo_model;
typedef struct gpbo_mlp_s* gpbo_mlp;

/* One sub-search: the evaluated configurations and the fixed hyperparameters.
 * X: device, n x d float64.  y: device, n float64 (objective to minimise).
 * lengthscale: host, d float64, all > 0.  signal_var > 0, noise_var >= 0 are
 * variances in units of the normalised y.
 * normalize_y: 1 = y is z-scored with its population standard deviation
 *   (a zero spread falls back to 1); 0 = y is only centred.
 * refine_alpha: 0 = alpha = K^-1 ytilde from float64 inverse-factor products
 *   plus one float64 refinement step; 1 = float32 products plus one float64
 *   residual-and-correction step (iterative refinement). */
typedef struct {
  int32_t n;
  int32_t d;
  const double* X;
  const double* y;
  int32_t kernel;
  const double* lengthscale;
  double signal_var;
  double noise_var;
  int32_t normalize_y;
  int32_t refine_alpha;
} gpbo_problem;

/* Scalars of a fitted model, in the order of gpbo_model_stats:
 * [0] mean of y, [1] scale s_y, [2] f_best = min y, [3] log marginal
 * likelihood of the normalised y, [4] log det K, [5] residual norm
 * |ytilde - K alpha| before refinement, [6] the same after refinement,
 * [7] the mean diagonal of signal_var * K^-1, i.e. signal_var trace(K^-1) / n
 * (each (K^-1)_ii is the reciprocal of the leave-one-out predictive variance
 * at x_i; large values mean nearly redundant observations and an
 * ill-conditioned K).  GPBO_FP32 scoring escalates a model to float64
 * arithmetic when [7] exceeds GPBO_ESCALATE_KINV (see gpbo_precision). */
#define GPBO_NSTATS 8
#define GPBO_ESCALATE_KINV 8.0

const char* gpbo_status_string(gpbo_status s);
/* Description of the last failure on ctx (or of the last failed context
 * creation when ctx is NULL).  Valid until the next call on ctx. */
const char* gpbo_last_error(gpbo_ctx ctx);
/* Library version as major*10000 + minor*100 + patch. */
int32_t gpbo_version(void);

/* Create a context on HIP device `device`, queuing work on `stream` (a
 * hipStream_t; NULL = the default stream).  Returns GPBO_E_HIP when there is
 * no usable device.  Launch graphs (the fit's launch sequence, batched
 * scoring, network training) are captured and replayed only on a created
 * stream: the legacy default stream cannot be captured, and there every
 * call launches eagerly (same results).  The environment variable
 * GPBO_NO_GRAPH=1 at creation turns replay off. */
gpbo_status gpbo_ctx_create(int32_t device, void* stream, const gpbo_allocator* alloc,
                            gpbo_ctx* out);
/* Waits for the context's stream, then frees every model and MLP still
 * alive on the context (their handles become invalid) and the context. */
gpbo_status gpbo_ctx_destroy(gpbo_ctx ctx);
/* Replace the stream work is queued on.  Waits first for the work queued
 * on the previous stream (when the two differ). */
gpbo_status gpbo_ctx_set_stream(gpbo_ctx ctx, void* stream);
/* Kernel timing.  While enabled, every launch of a candidate-scoring kernel
 * (the dominant kernel of gpbo_score: the fused kernel, or the triangular
 * product of the large-n path; the persistent kernel of gpbo_score_batched,
 * which then launches eagerly instead of replaying its graph) and of the
 * network forward kernel (gpbo_mlp_forward, gpbo_mlp_prescreen*) is bracketed
 * by HIP events recorded on the context's stream.  gpbo_ctx_timing synchronises the stream, returns the
 * number of timed launches and their summed duration in milliseconds, and
 * resets both.  Either output may be NULL. */
gpbo_status gpbo_ctx_enable_timing(gpbo_ctx ctx, int32_t enable);
gpbo_status gpbo_ctx_timing(gpbo_ctx ctx, int64_t* launches, double* total_ms);
/* Scoring path of gpbo_score (both compute the same quantities):
 *   GPBO_PATH_AUTO  : fused for small n, chunked for large n (float32);
 *   GPBO_PATH_FUSED : one workgroup per candidate tile, cross-covariance in
 *                     LDS, then the matrix-core product;
 *   GPBO_PATH_LARGE : float32 only; per candidate chunk the cross-covariance
 *                     is written to a workspace and contracted with the
 *                     packed inverse factor by a triangular matrix-core
 *                     product (the timed kernel is that product).
 * Returns GPBO_E_INVALID_ARG for an unknown path; gpbo_score returns
 * GPBO_E_UNSUPPORTED when the forced path cannot take the problem. */
typedef enum gpbo_score_path {
  GPBO_PATH_AUTO = 0,
  GPBO_PATH_FUSED = 1,
  GPBO_PATH_LARGE = 2
} gpbo_score_path;
gpbo_status gpbo_ctx_set_score_path(gpbo_ctx ctx, gpbo_score_path path);

/* ---------------------------------------------------------------------- */
/* Fit (training the surrogate, Sec. IV-D: cubic in n).                    */
/* ---------------------------------------------------------------------- */
/* Normalise y, build K = k(X,X) + noise_var I, factor K = L L^T (float64,
 * blocked, on the GPU), form L^-1, solve alpha and the log marginal
 * likelihood.  SYNCHRONISES the stream once, to read the factorisation's
 * status.  On GPBO_E_NOT_PD *bad_pivot (host, may be NULL) receives the
 * 0-based index of the first pivot that is not positive.  *lml (host, may be
 * NULL) receives the log marginal likelihood.  *out receives a model that
 * owns copies of everything it needs; free it with gpbo_model_free. */
gpbo_status gpbo_fit(gpbo_ctx ctx, const gpbo_problem* prob, gpbo_model* out, double* lml,
                     int32_t* bad_pivot);

/* The same fit without the synchronisation: the work is queued on the
 * context's stream and *out receives the model at once, so a Bayesian-
 * optimisation step can queue the fit and the scoring of the next pool back
 * to back and synchronise once.  The factorisation's status is not known
 * yet: gpbo_model_status (which synchronises the stream) returns GPBO_OK,
 * GPBO_E_NOT_PD (with *bad_pivot) or GPBO_E_NONFINITE, and *lml (host, may be
 * NULL).  Scores of a model whose status is not GPBO_OK are undefined.
 * Unlike gpbo_fit, the caller's X and y are read by the queued work: they
 * must stay allocated and unchanged until the stream has run the fit (for
 * instance until gpbo_model_status returns).
 * Returns GPBO_E_INVALID_ARG / GPBO_E_UNSUPPORTED / GPBO_E_OOM as gpbo_fit
 * does for problems rejected before any work is queued. */
gpbo_status gpbo_fit_async(gpbo_ctx ctx, const gpbo_problem* prob, gpbo_model* out);
gpbo_status gpbo_model_status(gpbo_ctx ctx, gpbo_model model, int32_t* bad_pivot, double* lml);
/* gpbo_fit_batched without the synchronisation, in the same way: status[b]
 * (host, B) reports only the checks made before any work is queued; the
 * factorisation status of each model comes from gpbo_model_status (the first
 * such call for a model of the batch reads the statuses of the whole batch
 * with one copy). */
gpbo_status gpbo_fit_batched_async(gpbo_ctx ctx, int32_t B, const gpbo_problem* probs,
                                   gpbo_model* out, int32_t* status);
/* gpbo_model_status of B models: status (host, B) and lml (host, B, may be
 * NULL; NaN where the fit failed).  Returns the first failing status. */
gpbo_status gpbo_model_status_batched(gpbo_ctx ctx, int32_t B, const gpbo_model* models,
                                      int32_t* status, double* lml);

/* Fit B independent sub-searches (Sec. IV-D runs them in parallel).  Problems
 * of different n and d are factored together, largest first.  SYNCHRONISES
 * once.  status (host, B) receives each problem's status; lml (host, B) may be
 * NULL.  Returns GPBO_OK when every problem fitted, else the first failing
 * problem's status (the models of failed problems are NULL).  The models of
 * one call share one device allocation, released with the last of them. */
gpbo_status gpbo_fit_batched(gpbo_ctx ctx, int32_t B, const gpbo_problem* probs,
                             gpbo_model* out, double* lml, int32_t* status);

/* Rank-one update: the re-training step of the optimisation loop (Sec. III-A
 * retrains the surrogate after each evaluation; Sec. IV-D gives every search
 * a budget of evaluations) when the hyperparameters stay fixed.  Adds one
 * evaluated configuration to each of B fitted models: K gains a row and a
 * column k = k(X, x_new), kappa = signal_var + noise_var; L gains the row
 * [l^T, delta] with l = L^-1 k and delta = sqrt(kappa - l^T l), and L^-1 the
 * row [-(L^-T l)^T / delta, 1 / delta] -- O(n^2) per model instead of the
 * O(n^3) refit.  y is normalised again over the n + 1 values, and alpha, the
 * log marginal likelihood and the statistics are recomputed as the fit
 * computes them (with its refinement option).  The result equals a refit on
 * the n + 1 observations up to rounding.
 * models: B distinct models of ctx.  x_new: device, B rows of ldx float64
 * (row b holds model b's d values, ldx >= every d).  y_new: device, B
 * float64.  Both are read by the queued work: keep them allocated and
 * unchanged until the stream has run it.
 * ASYNCHRONOUS like gpbo_fit_batched_async: gpbo_model_status then reports
 * GPBO_E_NOT_PD with bad_pivot = the old n when the new pivot is not
 * positive (a repeated configuration with noise_var = 0, for instance) and
 * GPBO_E_NONFINITE for a non-finite x_new or y_new; such a model stays failed
 * (fit it again), and so does a model whose fit had failed.  The model's n
 * counts the new row either way.  A model whose 64-row padding is full moves
 * to buffers one tile larger (a device allocation and a copy on the device);
 * score operands built earlier are rebuilt by the next scoring call.
 * Returns GPBO_E_INVALID_ARG (NULL, repeated or foreign models, ldx too
 * small, host pointers), GPBO_E_UNSUPPORTED (n would exceed 65536) or
 * GPBO_E_OOM before any work is queued. */
gpbo_status gpbo_append_batched(gpbo_ctx ctx, int32_t B, const gpbo_model* models,
                                const double* x_new, int32_t ldx, const double* y_new);

/* ---------------------------------------------------------------------- */
/* Hyperparameter fitting (the surrogate's training, Sec. IV-D).            */
/* ---------------------------------------------------------------------- */
/* Gradient of the log marginal likelihood of B fitted models with respect to
 * theta = (log l_1 .. log l_d, log signal_var, log noise_var), with the
 * normalised y held fixed:
 *   dLML/dtheta_j = 1/2 tr((alpha alpha^T - K^-1) dK/dtheta_j)
 * (Rasmussen & Williams 2006, eq. 5.9), K^-1 = L^-T L^-1 formed tile by tile
 * in float64 from the model's inverse factor.  grad: device, B x ldg float64
 * (ldg >= every d + 2; zero beyond d + 2; a row of NaN for a model whose fit
 * failed).  lml: device, B float64 (the models' log marginal likelihoods;
 * may be NULL).  Asynchronous. */
gpbo_status gpbo_lml_grad_batched(gpbo_ctx ctx, int32_t B, const gpbo_model* models, int32_t ldg,
                                  double* grad, double* lml);

/* Options of gpbo_fit_hyper_batched. */
typedef struct {
  int32_t starts;   /* starting points per problem (>= 1) */
  int32_t steps;    /* Adam steps per start (>= 0) */
  double lr;        /* Adam step size in log space (beta1 0.9, beta2 0.999, eps 1e-8) */
  double jitter0;   /* first jitter, in units of signal_var (> 0; 1e-8 is usual) */
  int32_t retries;  /* jitter escalations (x10 each) before a start is abandoned */
} gpbo_hyper_opts;

/* Fit the hyperparameters of B problems by maximising the log marginal
 * likelihood from opts->starts starting points each: every start takes
 * opts->steps Adam steps (Kingma & Ba 2015) up gpbo_lml_grad_batched's
 * gradient, clipped to [lo, hi] after each step; all starts of all problems
 * are fitted in one batched call per step.  A fit that is not positive
 * definite is repeated with signal_var * jitter0 * 10^(k-1) added to the
 * noise variance, k = 1 .. retries (the log-noise derivative stays that of
 * the noise variance itself); a start whose retries all fail is abandoned.
 * After the last step each start's LML is evaluated the same way and the
 * largest wins (lowest start index among ties).
 * probs: host, B problems; X and y (device) as for gpbo_fit, kernel,
 *   normalize_y and refine_alpha used, lengthscale / signal_var / noise_var
 *   ignored.
 * theta0: host, B x starts x ldt (start s of problem b at row b*starts+s).
 * lo, hi: host, B x ldt bounds of theta (finite, lo <= hi).  ldt >= d + 2.
 * theta (host, B x ldt), lml (host, B), jitter (host, B, may be NULL): the
 *   winning start's hyperparameters, LML and the jitter its last fit needed.
 * out (host, B, may be NULL): models fitted at the winning hyperparameters
 *   (noise_var + jitter); free them with gpbo_model_free.
 * status (host, B): GPBO_OK, or GPBO_E_NOT_PD when every start was abandoned.
 * SYNCHRONISES once or twice per step.  Returns the first failing status. */
gpbo_status gpbo_fit_hyper_batched(gpbo_ctx ctx, int32_t B, const gpbo_problem* probs,
                                   const gpbo_hyper_opts* opts, const double* theta0,
                                   const double* lo, const double* hi, int32_t ldt, double* theta,
                                   double* lml, double* jitter, gpbo_model* out, int32_t* status);

/* Release a model (NULL is ignored).  Work still queued that uses it may
 * run on: with a context allocator the buffers go back in the order of the
 * stream they were allocated on, without a wait, when every use of the
 * model was queued on that stream.  A model used on another stream first
 * waits for the whole device (that stream may still be reading it); a
 * context moved to another stream since the allocation, or hipFree
 * without an allocator, waits for the context's stream. */
gpbo_status gpbo_model_free(gpbo_model model);
/* Host copy of the GPBO_NSTATS scalars (synchronises). */
gpbo_status gpbo_model_stats(gpbo_model model, double* stats);
gpbo_status gpbo_model_shape(gpbo_model model, int32_t* n, int32_t* d);
/* Device copies of the factors (for checks): L (n x n, lower, float64),
 * L^-1 (n x n, lower, float64) and alpha (n, float64).  Any may be NULL. */
gpbo_status gpbo_model_factors(gpbo_ctx ctx, gpbo_model model, double* L, double* Linv,
                               double* alpha);

/* ---------------------------------------------------------------------- */
/* Scoring (the acquisition step, Sec. III-A).                             */
/* ---------------------------------------------------------------------- */
/* Posterior mean mu, standard deviation sigma (of the latent function, no
 * noise) and expected improvement for minimisation against f_best = min y:
 *   mu = ymean + s_y k*^T alpha
 *   sigma = s_y sqrt(max(signal_var - |L^-1 k*|^2, 0))
 *   EI = (f_best - mu) Phi(z) + sigma phi(z), z = (f_best - mu) / sigma
 *        (EI = max(f_best - mu, 0) when sigma = 0)
 * Xc: device, m x d, double for GPBO_FP64, float otherwise.
 * mu, sigma, ei: device, m each, double for GPBO_FP64, float otherwise; each
 * may be NULL.  argmax (int64) and ei_max (double): the index of the
 * largest EI (lowest index among ties; NaN never wins) and its value; both
 * may be NULL, in which case no reduction runs.  Each may be device memory
 * (written by the queued work: the call is asynchronous) or host memory
 * (the call then SYNCHRONISES the stream and writes it before returning).
 * m = 0 is allowed (argmax = -1, ei_max = -inf).
 * With the environment variable GPBO_DEBUG=1 at context creation the pool
 * is first checked for NaN and infinity (GPBO_E_NONFINITE; this check
 * synchronises the stream). */
gpbo_status gpbo_score(gpbo_ctx ctx, gpbo_model model, int64_t m, const void* Xc,
                       gpbo_precision prec, void* mu, void* sigma, void* ei, int64_t* argmax,
                       double* ei_max);

/* Score B models, each on its own candidate pool, in one persistent launch
 * (the paper runs independent sub-searches in parallel, Sec. IV-D), with
 * the quantities of gpbo_score per problem.
 * m, Xc, mu, sigma, ei: host arrays of B entries (Xc[b], mu[b], sigma[b],
 * ei[b] are device pointers typed as in gpbo_score; any output entry, or a
 * whole output array, may be NULL).  argmax and ei_max: arrays of B entries,
 * device memory (asynchronous) or host memory (the call synchronises), each
 * may be NULL.  With GPBO_FP32, problems above the escalation threshold are
 * scored by a second persistent launch in float64 arithmetic (see
 * gpbo_precision); the split is made on the device.  The launch sequence is
 * captured in a HIP graph on first use of a batch shape (B, precision,
 * tiles, candidate tiles, outputs) and replayed for later calls of that
 * shape, also with other models and pools: the kernels read them from
 * descriptors uploaded by each call.  Up to 8 shapes are kept.  GPBO_DEBUG
 * checks every pool as gpbo_score does. */
gpbo_status gpbo_score_batched(gpbo_ctx ctx, int32_t B, const gpbo_model* models,
                               const int64_t* m, const void* const* Xc, gpbo_precision prec,
                               void* const* mu, void* const* sigma, void* const* ei,
                               int64_t* argmax, double* ei_max);

/* Build, now, the scoring operands of B models for a precision (the scaled
 * observations, the packed inverse factor and scaled alpha), for all of
 * them in one launch pair on the context's stream (the float64 operands a
 * GPBO_FP32 batch may escalate to are still built by the scoring call).  gpbo_score and gpbo_score_batched
 * build what a model lacks on their own; calling this first over all the
 * models a step will score (several batched launches over fresh fits, Sec.
 * IV-D) replaces one preparation per scoring call by one for the step.
 * Operands already built are kept.  Asynchronous; GPBO_E_OOM when the
 * device allocation fails. */
gpbo_status gpbo_score_prepare_batched(gpbo_ctx ctx, int32_t B, const gpbo_model* models,
                                       gpbo_precision prec);

/* Posterior mean and two cheap upper bounds, without the triangular
 * product: the cost is the cross-covariance alone (about 2nd flops and n
 * exponentials per candidate against the n^2 of the variance), so a large
 * pool can be narrowed before exact scoring.  Conditioning the latent
 * function on fewer observations never lowers its posterior variance
 * (R&W Sec. 2.2), and the one noisy observation with the largest covariance
 * leaves sf2 - k_max^2 / (sf2 + noise_var): sigma_ub = s_y sqrt of that is
 * an upper bound of sigma, and, EI growing with sigma, ei_ub =
 * EI(mu, sigma_ub) is an upper bound of EI.
 * Xc: device, m x d float; mu, sigma_ub, ei_ub: device, m float each (any
 * may be NULL).  float32 arithmetic as in the GPBO_FP32 cross-covariance
 * (no escalation).  Asynchronous. */
gpbo_status gpbo_score_bound(gpbo_ctx ctx, gpbo_model model, int64_t m, const float* Xc,
                             float* mu, float* sigma_ub, float* ei_ub);

/* Exact judge of a prescreened subset of a pool (the learned prescreen's
 * re-score and its fallback): of the k1 candidates Xc[idx[i]] (Xc: device,
 * m x d float; idx: device, k1 int64, entries in [0, m)), the k2 with the
 * largest EI upper bound (gpbo_score_bound; every one of them when k2 >= k1)
 * are scored exactly on the GPBO_FP32 path, and the one with the largest EI
 * is returned: *next its index into Xc, *ei_max its EI.  *certified is 1
 * when that EI is not below the k2-th largest bound (the smallest bound
 * scored; every unscored bound is at most that) plus an allowance for
 * float32 rounding (2e-4 s_y sqrt(signal_var)): then no candidate of the
 * subset left unscored can have a larger EI; 0 otherwise (call again with a
 * larger k2 to widen the exact set).  Candidates with equal bounds at the
 * threshold are taken in index order.  next, ei_max, certified: device or
 * host memory (host memory synchronises); ei_max and certified may be NULL.
 * Asynchronous for device outputs. */
gpbo_status gpbo_score_subset(gpbo_ctx ctx, gpbo_model model, int64_t m, const float* Xc,
                              int64_t k1, const int64_t* idx, int64_t k2, int64_t* next,
                              double* ei_max, int32_t* certified);

/* Top k of v (device, m floats) by (value descending, index ascending); idx
 * is a device array of k int64.  NaN entries never rank.  k <= 8192
 * (GPBO_E_UNSUPPORTED above).  Asynchronous. */
gpbo_status gpbo_topk(gpbo_ctx ctx, int64_t m, const float* v, int64_t k, int64_t* idx);
/* The same k entries as gpbo_topk (membership by value descending, index
 * ascending among ties) for any k <= m, as a set: idx (device, k int64) in
 * ascending index order.  Asynchronous. */
gpbo_status gpbo_topk_set(gpbo_ctx ctx, int64_t m, const float* v, int64_t k, int64_t* idx);

/* gpbo_topk that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, results and errors as gpbo_topk; its
 * scratch (radix state, histogram, per-block counts, the k selected keys and
 * indices) is a static device array of GPBO_TOPK_NOALLOC_SCRATCH bytes per
 * GPU, held by the library until the process ends, whose address is resolved
 * when the first context on that GPU is created.  Every call on a GPU shares
 * that GPU's array (the launch sequence re-initialises it, so the contents a
 * previous call left do not matter): calls that can overlap on one GPU --
 * other streams, other contexts, other threads -- race, and the caller must
 * serialise them.  Returns GPBO_E_UNSUPPORTED when the scratch the sizes
 * need exceeds the array (it holds every k <= 8192 at any m < 2^32).
 * Asynchronous. */
#define GPBO_TOPK_NOALLOC_SCRATCH (128 * 1024)
gpbo_status gpbo_topk_noalloc(gpbo_ctx ctx, int64_t m, const float* v, int64_t k, int64_t* idx);

/* The next configuration of each of B searches after a batched scoring call
 * (the acquisition's choice, Sec. III-A): x_next[b, :d_b] = Xc[b][argmax[b],
 * :] widened to float64, zero from column d_b to ldx - 1, where d_b is model
 * b's dimension.  models, m, Xc: as passed to gpbo_score_batched (Xc[b]
 * float64 for GPBO_FP64, float otherwise).  argmax: device, B int64 (as
 * gpbo_score_batched writes it); an index outside [0, m[b]) -- the -1 of an
 * empty pool -- gives a row of NaN.  x_next: device, B x ldx float64,
 * ldx >= every d_b.  Asynchronous: queue it behind the scoring call and copy
 * x_next to the host once, instead of reading B rows one by one. */
gpbo_status gpbo_next_batched(gpbo_ctx ctx, int32_t B, const gpbo_model* models, const int64_t* m,
                              const void* const* Xc, gpbo_precision prec, const int64_t* argmax,
                              int32_t ldx, double* x_next);
/* out[i, :] = Xc[idx[i], :] for i < k (device float arrays, row-major, d
 * columns).  Asynchronous. */
gpbo_status gpbo_gather_rows(gpbo_ctx ctx, int64_t k, const int64_t* idx, int32_t d,
                             const float* Xc, float* out);

/* ---------------------------------------------------------------------- */
/* Interdependence analysis: the set of searches (Sec. IV-B to IV-D).      */
/* Host computations on host arrays; no device work, no context.          */
/* ---------------------------------------------------------------------- */
/* Sensitivity of R routines to P parameters from a one-at-a-time sweep
 * (Sec. IV-B): from a baseline configuration, V variations of each parameter
 * alone; S[r * P + j] = (1/V) sum_i |(base[r] - out[(j * V + i) * R + r]) /
 * base[r]|, the mean relative change of routine r's output (its runtime, or
 * any objective) when parameter j varies.  base: host, R outputs at the
 * baseline; out: host, P x V x R outputs at the variations; S: host, R x P.
 * GPBO_E_INVALID_ARG for a zero or non-finite baseline output. */
gpbo_status gpbo_sensitivity(int32_t P, int32_t R, int32_t V, const double* base,
                             const double* out, double* S);
/* The set of searches from the sensitivities (Sec. IV-C, IV-D).  owner[j]
 * (host, P) is the routine parameter j belongs to.  The influence of j on
 * routine r is S[r][j] relative to r's most sensitive own parameter; an
 * influence of at least `cutoff` (e.g. 0.25) on another routine links the two
 * routines, and linked routines are tuned in one merged search.  A search of
 * more than max_dims parameters (the paper uses 10) keeps the most
 * influential ones (largest influence on any routine of the search, lower
 * index among ties); the others are fixed at their defaults.  Outputs
 * (host): routine_search (R) the search of each routine, numbered in order
 * of each search's lowest routine; param_search (P) the search of each
 * parameter or -1 when the cap dropped it; *n_searches. */
gpbo_status gpbo_plan_searches(int32_t P, int32_t R, const double* S, const int32_t* owner,
                               double cutoff, int32_t max_dims, int32_t* routine_search,
                               int32_t* param_search, int32_t* n_searches);

/* ---------------------------------------------------------------------- */
/* Learned prescreen: an ensemble of MLPs d_in -> H -> H -> 1 (GELU),        */
/* bfloat16 weights and activations on the matrix cores with float32         */
/* accumulation, float32 master weights and Adam state.                      */
/* ---------------------------------------------------------------------- */
/* Parameter layout of one member (P = H*d_in + H + H*H + H + H + 1 floats):
 *   W1 (H x d_in), b1 (H), W2 (H x H), b2 (H), w3 (H), b3 (1).
 * init: device, members x P float32 initial master weights. */
gpbo_status gpbo_mlp_create(gpbo_ctx ctx, int32_t members, int32_t d_in, int32_t hidden,
                            const float* init, gpbo_mlp* out);
/* Release a network (NULL is ignored).  Waits for the whole device first:
 * its buffers may be in use on any stream the context has queued on. */
gpbo_status gpbo_mlp_free(gpbo_mlp mlp);
/* Number of parameters of one member. */
int64_t gpbo_mlp_nparams(int32_t d_in, int32_t hidden);
/* Device copy of the float32 master weights (members x P). */
gpbo_status gpbo_mlp_params(gpbo_ctx ctx, gpbo_mlp mlp, float* out);
/* Mean-squared-error loss (1/n) sum (out_i - y_i)^2 of every member on
 * (X: device n x d_in float, y: device n float) and its gradient with
 * respect to the master weights.  grad: device members x P float; loss:
 * device members float. */
gpbo_status gpbo_mlp_grads(gpbo_ctx ctx, gpbo_mlp mlp, int32_t n, const float* X,
                           const float* y, float* grad, float* loss);
/* `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning
 * rate lr) on every member.  loss_hist: device steps x members float (the
 * loss before each step), may be NULL.  The step sequence is captured in a
 * HIP graph and replayed.  Asynchronous. */
gpbo_status gpbo_mlp_train(gpbo_ctx ctx, gpbo_mlp mlp, int32_t n, const float* X,
                           const float* y, int32_t steps, double lr, float* loss_hist);
/* `steps` Adam steps as gpbo_mlp_train, on the observations of a fitted
 * model: inputs its X (cast to float32), targets its normalised y (the
 * fit's z-score, or centring with normalize_y = 0), so that the network
 * learns the same targets as the Gaussian process; its outputs are then in
 * the model's normalised units.  The model's n must be a multiple of 64 and
 * its d equal to d_in.  Queued behind the model's fit on the context's
 * stream (an asynchronous fit needs no status call first).  Asynchronous. */
gpbo_status gpbo_mlp_train_model(gpbo_ctx ctx, gpbo_mlp mlp, gpbo_model model, int32_t steps,
                                 double lr, float* loss_hist);
/* Grid of the network's pass over a pool (gpbo_mlp_forward,
 * gpbo_mlp_prescreen*): 0 (the default) launches one workgroup per 64-sample
 * tile and member, filling every compute unit; k > 0 launches k workgroups
 * per compute unit, each looping over tiles, so that part of every compute
 * unit stays free for work queued on other streams -- the Gaussian-process
 * fit of the same optimisation step, which the prescreen's judge needs next.
 * Results do not depend on it.  Returns GPBO_E_INVALID_ARG for k < 0. */
gpbo_status gpbo_mlp_set_occupancy(gpbo_ctx ctx, gpbo_mlp mlp, int32_t workgroups_per_cu);
/* Member outputs on m candidates: out is device members x m float. */
gpbo_status gpbo_mlp_forward(gpbo_ctx ctx, gpbo_mlp mlp, int64_t m, const float* Xc,
                             float* out);
/* The selection half of a prescreen, on member outputs already computed
 * (gpbo_mlp_forward), so that a step can queue the network's pass, then the
 * Gaussian-process fit, then the selection: outs is device E x m float
 * (member-major); rule GPBO_SELECT_EI scores the ensemble EI against f_best
 * = arg, GPBO_SELECT_LCB the negated lower confidence bound with kappa =
 * arg >= 0; then the k best indices as gpbo_mlp_prescreen returns them.
 * score_out (device m float) may be NULL.  Uses the context's scratch
 * (allocated or grown on first need).  Asynchronous. */
#define GPBO_SELECT_EI 0
#define GPBO_SELECT_LCB 1
gpbo_status gpbo_ens_select(gpbo_ctx ctx, int32_t E, int64_t m, const float* outs, int32_t rule,
                            double arg, int64_t k, int64_t* topk_idx, float* score_out);
/* Prescreen: ensemble mean and population standard deviation over members,
 * EI against f_best (in the network's output units, evaluated in float64 and
 * rounded to float), then the indices of the k largest EI (device int64): for
 * k <= 8192 sorted by descending EI, ascending index among ties; for larger k
 * (up to m) the same set in ascending index order (see gpbo_topk_set).
 * ei_out (device m float) may be NULL.  Asynchronous.  Called on the
 * network's own context, the pass keeps its workspace (member outputs,
 * scores, selection scratch) between calls and allocates only when a larger
 * pool comes; such calls must stay in that context's stream order. */
gpbo_status gpbo_mlp_prescreen(gpbo_ctx ctx, gpbo_mlp mlp, int64_t m, const float* Xc,
                               double f_best, int64_t k, int64_t* topk_idx, float* ei_out);
/* Prescreen by the ensemble's lower confidence bound: score = -(mean - kappa
 * sd) (mean and population standard deviation over the members, in the
 * network's output units; larger is better for minimisation), then the
 * indices of the k largest scores (device int64; ordered as in
 * gpbo_mlp_prescreen).  kappa >= 0; kappa = 0 ranks by the predicted mean.
 * score_out (device m float) may be NULL.  Asynchronous. */
gpbo_status gpbo_mlp_prescreen_lcb(gpbo_ctx ctx, gpbo_mlp mlp, int64_t m, const float* Xc,
                                   double kappa, int64_t k, int64_t* topk_idx, float* score_out);

#ifdef __cplusplus
}
#endif

#endif /* GPBO_H */
