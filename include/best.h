/*
 * best.h - C ABI of the MI355X (gfx950) batched emulator posterior sampler.
 *
 * The library evaluates a dense tanh-MLP log-likelihood emulator and its gradient for
 * thousands of chains at once and fuses it with the MH, MALA, HMC and AIES updates of
 * "Posterior sampling in the Age of Emulators" (Sec. 2 and Sec. 3).  The target is
 * declarative (struct best_problem):
 *
 *   log pi(x) = gauss_coef * G(phi(x)) + part(x) + offset        inside [lower, upper]
 *             = -inf                                              outside (hard box)
 *   G(y)      = -1/2 (y - m)^T P (y - m)
 *   phi(x)    = x, except phi_v = x_v + beta((x_u - center)^2 - kappa) (twisted pair)
 *   part(x)   = mlp_coef * MLP((x - in_center) * in_invscale)     plain_mode 0
 *               the same inside [train_lo, train_hi], plain(x) outside plain_mode 1
 *               plain(x) everywhere                                 plain_mode 2
 *   MLP       h_0 = t, h_l = tanh(W_l h_{l-1} + b_l), out = w_out . h_L + b_out
 *   plain(x)  chi^2 log-likelihood of a spectrum of damped cosines (struct best_plain_model)
 *
 * Every sampler except AIES runs in the whitened space of Sec. 2.2 / Algorithm 1:
 * x = mu + L z with log pi_z(z) = log pi(mu + L z) + sum_i log L_ii, so HMC has the
 * identity mass matrix.  The whitening (mu, L) is set by best_adapt (Sec. 3.2).
 *
 * Conventions for every call:
 *   - Return value: BEST_OK (0) or a BEST_E* code; no exception crosses the ABI and the
 *     library never aborts.  best_last_error(ctx) returns the message of the last failure
 *     on that context (valid until the next call on it).
 *   - Arrays of chain quantities are structure-of-arrays: element (i, c) of a [d][n]
 *     array lives at index i * n + c (chain index fastest).
 *   - Device pointers unless a flag says host.  The caller owns every pointer it passes;
 *     the library copies what it keeps (the problem at best_init).
 *   - Work is enqueued on the context's stream (best_config.stream, a hipStream_t, NULL
 *     for the default stream).  Calls that return statistics synchronise that stream.
 *   - One context is one stream and is not re-entrant; distinct contexts are independent.
 *   - Precision (best_config.precision) applies to the hidden-layer GEMMs only; the
 *     whitening, energies and Metropolis log-ratios are always computed in FP64.
 */
#ifndef BEST_H
#define BEST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define BEST_OK 0
#define BEST_EINVAL 1  /* an argument is invalid (NULL, size, shape, option) */
#define BEST_ENOMEM 2  /* a device or host allocation failed */
#define BEST_EHIP 3    /* a HIP runtime call or kernel launch failed */
#define BEST_ENOTPD 4  /* covariance not positive definite even after jitter */
#define BEST_ESTATE 5  /* call not valid in the current state (e.g. AIES with odd n) */

/* ---- precision of the hidden-layer GEMMs ---- */
#define BEST_FP64 0 /* FP64 MFMA (v_mfma_f64_16x16x4) */
#define BEST_FP32 1 /* FP32 MFMA (v_mfma_f32_16x16x4) */
#define BEST_FP16 2 /* FP16 MFMA with FP32 accumulation */
#define BEST_BF16 3 /* BF16 MFMA with FP32 accumulation */

/* ---- samplers (Sec. 2) ---- */
#define BEST_MH 0   /* random-walk Metropolis-Hastings in whitened space */
#define BEST_MALA 1 /* Metropolis-adjusted Langevin, Sec. 2.1 */
#define BEST_HMC 2  /* Hamiltonian Monte Carlo, leapfrog, identity mass (Sec. 2.1-2.2) */
#define BEST_AIES 3 /* affine-invariant ensemble sampler, stretch move (Sec. 2.3) */
#define BEST_NUTS 4 /* No-U-Turn sampler, Hoffman & Gelman's efficient slice version,
                       identity mass in whitened space (named among the samplers, Sec. 2.1) */
#define BEST_NUTS_MAX_DEPTH 12
#define BEST_DE 5   /* differential-evolution move of the ensemble sampler (Sec. 2.3):
                       y = x_i + gamma (x_j - x_k), gamma = (1 + eta) 2.38 / sqrt(2 d),
                       eta ~ N(0, de_sigma^2), two half-ensembles as for AIES */

/* ---- walker initialisation (Sec. 3.2) ---- */
#define BEST_INIT_UNIFORM 0    /* uniform in the prior box */
#define BEST_INIT_REPLICATED 1 /* every chain at init_point */
#define BEST_INIT_GAUSSIAN 2   /* init_point + init_scale * L0 xi, xi ~ N(0, I) */
#define BEST_INIT_HYPERSPHERE 3 /* the hypersphere-based perturbation of Sec. 3.2:
                                   init_point + init_scale * L0 r u with u = xi / |xi| uniform
                                   on the unit sphere and r = U^(1/d), i.e. uniform in the
                                   ellipsoid of whitened radius init_scale, whose spread does
                                   not grow with d as a Gaussian's norm (sqrt d) does */

/* ---- flags for best_logL_grad / best_get_state / best_set_state ---- */
#define BEST_HOST_PTRS 1u /* the array arguments are host pointers */
#define BEST_AOS 2u       /* best_logL_grad: x and grad are point-major [n][d] (element
                             (c, i) at c * d + i) instead of structure-of-arrays */

typedef struct best_ctx best_ctx;
typedef struct best_trainer best_trainer;

/* Plain forward model (the synthetic stand-in for an expensive likelihood pipeline):
 *   t = (x - center) * invscale
 *   S_j = sum_m exp(a_m . t) exp(-gamma0_m exp(g_m . t) xgrid_j)
 *               cos(2 pi k_m xgrid_j + pi tanh(p_m . t))
 *   plain(x) = -1/2 sum_j (S_j - data_j)^2 inv_sigma2_j
 * a, g, p are [n_terms][d] row-major; k, gamma0 are [n_terms]; the rest [n_bins] / [d]. */
typedef struct {
  int32_t n_bins, n_terms;
  const double *xgrid, *data, *inv_sigma2;
  const double *a, *g, *p;
  const double *k, *gamma0;
  const double *center, *invscale;
} best_plain_model;

/* The target (see the top of this file).  All pointers are host pointers; the problem is
 * deep-copied by best_init.  mlp_params is the flat vector
 *   [W1 (H x d), b1 (H), W2 (H x H), b2, ..., W_L (H x H), b_L, w_out (H), b_out]
 * of length best_mlp_nparams(d, width, n_hidden).  width must be a multiple of 128 and at
 * most 2048; 1 <= d <= 32; 1 <= n_hidden <= 16. */
typedef struct {
  int32_t d;
  const double *lower, *upper;
  double gauss_coef;
  const double *gauss_mean; /* [d] */
  const double *gauss_prec; /* [d*d] row-major, symmetric */
  int32_t twist_u, twist_v; /* twist_u < 0: no twist */
  double twist_beta, twist_center, twist_kappa;
  int32_t width, n_hidden;
  const double *mlp_params;
  const double *in_center, *in_invscale; /* [d] */
  double mlp_coef, offset;
  int32_t plain_mode; /* 0, 1 or 2 (see top) */
  const double *train_lo, *train_hi; /* [d], plain_mode 1 only */
  const best_plain_model *plain;     /* plain_mode 1 or 2 */
  int32_t box_penalty;  /* 0: hard box (log pi = -inf outside); 1: smooth penalty (Sec. 3.1)
                           - sum_i [exp(r_i/w) - 1 - r_i/w] outside, r_i = distance outside
                           the box in box widths, zero value and slope at the faces */
  double penalty_width; /* w of the penalty (> 0, e.g. 0.01); ignored for the hard box */
} best_problem;

typedef struct {
  int64_t n_chains;          /* >= 1 (AIES needs an even count) */
  int32_t precision;         /* BEST_FP64 / FP32 / FP16 / BF16 */
  uint64_t seed;             /* Philox key */
  int32_t init;              /* BEST_INIT_* */
  const double *init_point;  /* [d] host, NULL = box centre */
  double init_scale;         /* BEST_INIT_GAUSSIAN / HYPERSPHERE scale (whitened units) */
  void *stream;              /* hipStream_t or NULL */
  int32_t chains_per_block;  /* 0 = automatic, else 16, 32 or 64 */
} best_config;

/* Per-call sampler options. */
typedef struct {
  double eps;             /* MALA / HMC step size (whitened units); <= 0: use the
                             context's current step size (dual-averaging result) */
  double mh_scale;        /* MH proposal scale in whitened units (e.g. 2.4/sqrt(d)) */
  double stretch_a;       /* AIES stretch parameter a > 1 (2 in the paper) */
  int32_t n_leapfrog;     /* HMC leapfrog steps per trajectory (>= 1) */
  int32_t thin;           /* record every thin-th step (>= 1) */
  float *record;          /* device [record_capacity][d][n_chains] x-space samples or NULL */
  int64_t record_capacity;
  int32_t adapt_eps;      /* 1: dual-averaging update of the step size after every step */
  double target_accept;   /* dual-averaging target (e.g. 0.57 MALA, 0.8 HMC / NUTS) */
  int32_t max_depth;      /* NUTS maximum tree depth, 1 .. BEST_NUTS_MAX_DEPTH: at most
                             2^max_depth - 1 evaluations per transition */
  double de_sigma;        /* DE: standard deviation of eta (>= 0; the paper's sigma_gamma) */
} best_step_params;

typedef struct {
  int64_t accepted;        /* accepted transitions summed over chains and steps */
  int64_t evals;           /* emulator evaluations (logL or logL+grad); NUTS: the leaves of
                              every chain's trajectory (the idle slots of chains that
                              stopped before others in their tile are not counted) */
  int64_t n_nonfinite;     /* proposals whose log pi was NaN (rejected) */
  int64_t n_oob;           /* proposals outside the prior box (rejected with the hard box) */
  int64_t n_recorded;      /* record slots written */
  double sum_accept_prob;  /* sum of min(1, alpha); NUTS: of the per-transition mean over
                              leaves of min(1, exp(H0 - H)) */
  double ms;               /* wall time of the call's kernels (hipEvents) */
  double eps;              /* current step size after the call */
  double eps_bar;          /* dual-averaging averaged step size */
} best_step_stats;

typedef struct {
  const float *samples;  /* device [n_samples][d][n_chains] window, NULL = current x */
  int64_t n_samples;
  int32_t update_mean;   /* 1: mu <- ensemble mean, 0: keep mu */
  int32_t reset_da;      /* 1: restart dual averaging from the current step size */
  int32_t finalize_da;   /* 1: step size <- dual-averaging average */
  double target_accept;  /* for reset_da */
} best_adapt_params;

typedef struct {
  double jitter;  /* lambda * mean(diag Sigma) added to the diagonal (0 if none) */
  double logdet;  /* sum_i log L_ii of the new whitening */
  double eps;     /* step size after the call */
} best_adapt_info;

/* ---- lifetime ---- */

/* Validate and copy the problem, allocate device state, initialise the walkers
 * (uniform / replicated / Gaussian; Sec. 3.2), set the initial whitening mu = box centre,
 * L = diag(0.1 (upper - lower)) (Sec. 4: a diagonal covariance scaled to the box), and
 * evaluate log pi and its gradient at the start.  *out is NULL on failure. */
int best_init(best_ctx **out, const best_problem *p, const best_config *c);
void best_destroy(best_ctx *h); /* NULL is a no-op; frees every library buffer */
const char *best_strerror(int code);
const char *best_last_error(const best_ctx *h);
int64_t best_mlp_nparams(int32_t d, int32_t width, int32_t n_hidden);

/* ---- the hot path ---- */

/* Batch evaluation of log pi(x) and grad_x log pi(x) at n points x: the emulator evaluated
 * for many walkers at once, whose cost stays flat in the batch size up to the device's
 * width (Sec. 2.3 and Fig. 1), with the gradient the samplers of Sec. 2.1 need.  x and grad
 * are [d][n] (structure-of-arrays), or [n][d] with BEST_AOS (converted on the device through
 * a library scratch of 2 d n + n doubles, allocated by the first such call or a larger n).
 * grad may be NULL (logL only).  Device pointers, or host pointers with BEST_HOST_PTRS (then
 * the call synchronises).  The prior box applies: -inf outside (the gradient returned there
 * is that of the unbounded expression), or the smooth penalty with box_penalty = 1. */
int best_logL_grad(best_ctx *h, const double *x, int64_t n, double *logL, double *grad,
                   uint32_t flags);

/* Advance every chain n_steps transitions of `sampler` (BEST_MH / MALA / HMC / AIES /
 * NUTS / DE).  AIES and DE need an even number of walkers (DE at least 4): BEST_ESTATE.  Randomness: Philox4x32-10 keyed by the seed, counter = (chain, global step,
 * stream << 24 | substep, block); the global step counter advances by n_steps.
 * out (may be NULL) receives the call's statistics; the call synchronises the stream.
 * MALA, HMC and NUTS need a gradient precision other than BEST_FP64 (BEST_ESTATE).  The
 * first NUTS call (or one with a deeper max_depth) allocates the trajectory buffers,
 * (8 + 4 max_depth) d + 2 max_depth + 1 doubles per chain; BEST_ENOMEM if that fails. */
int best_step(best_ctx *h, int32_t sampler, int64_t n_steps, const best_step_params *p,
              best_step_stats *out);

/* Covariance adaptation (Sec. 3.2): FP64 mean and covariance of the window (or of the
 * current ensemble), symmetrised, Cholesky with jitter escalation (lambda = 1e-10 ...
 * 1e-2 of the mean diagonal), new whitening (mu, L); every chain is re-whitened.  On
 * BEST_ENOTPD the previous whitening is kept.  Also resets / finalises dual averaging. */
int best_adapt(best_ctx *h, const best_adapt_params *p, best_adapt_info *out);

/* Gradient of sum_c w_c log pi(x_c) with respect to the MLP parameters theta (the flat
 * vector of best_problem.mlp_params): the weight gradients that training and
 * differentiation through the emulator need (the paper relies on automatic differentiation
 * of the emulator, Sec. 1 and Sec. 2.1).  Reverse mode through the context's network at
 * its precision: delta_L = u_c w_out (1 - h_L^2), delta_{l-1} = (W_l^T delta_l)(1 - h_{l-1}^2)
 * with u_c = mlp_coef w_c, then dW_l = sum_c delta_l h_{l-1}^T, db_l = sum_c delta_l,
 * dw_out = sum_c u_c h_L, db_out = sum_c u_c (FP32 matrix cores, FP64 results).  A point
 * whose log pi does not use the MLP (outside the training box with plain_mode 1) adds
 * nothing; plain_mode 2 gives zeros.  The prior box is ignored (the gradient of the
 * unbounded expression, as for best_logL_grad).  x: device [d][n]; upstream: device [n]
 * FP64, NULL for all ones; grad_params: device FP64 [best_mlp_nparams].  Asynchronous on
 * the context's stream.  The first call (or a larger n) allocates 2 nh width + d + 1 floats
 * per point, n rounded up to 16 (BEST_ENOMEM).  FP64 contexts: BEST_ESTATE. */
int best_logL_param_grad(best_ctx *h, const double *x, int64_t n, const double *upstream,
                         double *grad_params);

/* ---- state, whitening, diagnostics ---- */
/* Checkpoint / resume.  get: x [d][n], logL [n], grad [d][n] (any may be NULL).  set: x,
 * and either both logL and grad (restored as given, so a resumed run continues bit-for-bit
 * with the same step counter) or neither (re-evaluated). */
int best_get_state(best_ctx *h, double *x, double *logL, double *grad, uint32_t flags);
int best_set_state(best_ctx *h, const double *x, const double *logL, const double *grad,
                   uint32_t flags);
int best_get_whitening(best_ctx *h, double *mu, double *L);       /* host, [d], [d*d] */
int best_set_whitening(best_ctx *h, const double *mu, const double *L);
uint64_t best_get_step_counter(const best_ctx *h);
int best_set_step_counter(best_ctx *h, uint64_t step);
int best_set_step_size(best_ctx *h, double eps);
/* Re-initialise every walker (Sec. 3.2 initialisation strategies, used by the burn-in loop
 * that re-centres the ensemble on its best-fit point): BEST_INIT_UNIFORM in the prior box,
 * BEST_INIT_REPLICATED at point, BEST_INIT_GAUSSIAN point + scale L xi and
 * BEST_INIT_HYPERSPHERE point + scale L r u (as for best_config.init) with the CURRENT
 * whitening factor L (xi, u, r from Philox stream 4 at the current step counter, which is
 * not advanced).  point: host [d] inside the box (ignored for uniform).  log pi and its
 * gradient are re-evaluated; the whitening and step size are kept.  Gaussian and
 * hypersphere draws may fall outside the box (log pi = -inf there with the hard box). */
int best_reinit(best_ctx *h, int32_t init, const double *point, double scale);
/* Per-dimension step multipliers m (host [d], each finite and > 0; NULL removes them) for
 * the whitened-space MALA and MH transitions (Sec. 4.3: larger steps for chosen
 * dimensions): dimension i uses eps m_i in MALA's drift, noise and proposal density, and
 * mh_scale m_i in MH.  HMC and NUTS ignore them.  Kept until replaced. */
int best_set_step_multipliers(best_ctx *h, const double *m);
/* Replace the MLP weights (flat host vector, same layout as best_problem.mlp_params). */
int best_set_mlp(best_ctx *h, const double *params, double mlp_coef, double offset);

/* Multi-chain effective sample size of a record ([T][d][n_chains] device floats) per
 * parameter: rho_t = 1 - (W - mean_m gamma_{m,t}) / var+, Geyer initial monotone
 * sequence, tau = max(-1 + 2 sum P_k, 1 / log10(M T)), ESS = M T / tau (Geyer 1992;
 * Vehtari et al. 2021; the throughput metric reported with the samplers, not the paper's).
 * Autocovariances are summed directly on the device in FP64.  T >= 4.
 * ess_out: host [d].  flags_out: host [d] or NULL, per parameter one of
 *   BEST_ESS_OK          the pair sums turned non-positive inside the window;
 *   BEST_ESS_UNTRUNCATED every pair sum the window holds is positive: the window is
 *                        shorter than the autocorrelation, tau is a lower bound and the
 *                        ESS an upper bound;
 *   BEST_ESS_FROZEN      the within-chain variance W is 0 (every chain constant over the
 *                        window, e.g. nothing accepted): no estimate exists, ESS = 0. */
#define BEST_ESS_OK 0
#define BEST_ESS_UNTRUNCATED 1
#define BEST_ESS_FROZEN 2
int best_ess(best_ctx *h, const float *record, int64_t T, double *ess_out, int32_t *flags_out);
/* best_ess for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same estimate, bit for bit,
 * with no hipMalloc / hipFree.  Its device scratch is one fixed array per GPU
 * (4 * 2^20 doubles = 32 MiB, held by each GPU the library runs on until the process ends),
 * so d * ceil(n_chains / 64) * 64 must be at most 2^20 (BEST_EINVAL otherwise, with the
 * sizes in best_last_error).  The context's device must be current (BEST_ESTATE).  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU (several threads,
 * or contexts on different streams) race and must be serialised by the caller.  Host-side
 * working arrays of the Geyer sums are ordinary host memory.  Synchronises the stream. */
int best_ess_noalloc(best_ctx *h, const float *record, int64_t T, double *ess_out,
                     int32_t *flags_out);

/* ---- convergence metrics (Sec. 4.1) ----
 * Samples are device records [T][d][n_chains] (floats, chain fastest), as best_step writes
 * them; d is the context's.  Results are host scalars / arrays; each call allocates its
 * device scratch, synchronises the stream and frees it. */

/* Gelman-Rubin type statistic of Sec. 4.1: B = covariance of the chain means (unbiased),
 * W = mean of the chain covariances (unbiased); with D = diag(sqrt(B_ii)),
 * R - 1 = max |eigenvalue| of (D^-1 W D^-1)^-1 (D^-1 B D^-1), written to *rminus1.
 * T >= 2, n_chains >= 2.  BEST_EINVAL if some B_ii is 0 (identical chain means),
 * BEST_ENOTPD if the normalised W is not positive definite. */
int best_rhat(best_ctx *h, const float *samples, int64_t T, int64_t n_chains, double *rminus1);

/* Credible limits and the credible metric of Sec. 4.1.  lo / hi (host [d], may be NULL):
 * equal-tailed limits of every parameter at level alpha, the sample quantiles at
 * (1 - alpha)/2 and 1 - (1 - alpha)/2 of the T n_chains draws (rule: h = (n - 1) p,
 * k = floor(h), v_k + (h - k)(v_{k+1} - v_k) over the sorted values v).  With mu and L
 * (host [d] and [d*d] row-major lower triangle, positive diagonal) the draws are whitened
 * first, z = L^-1 (x - mu).  With ref_lo / ref_hi (host [d], the reference limits in the
 * same coordinates) *metric = max_i (|hi_i - ref_hi_i| + |lo_i - ref_lo_i|) /
 * (ref_hi_i - ref_lo_i).  At most 2^31 - 1 draws. */
int best_credible(best_ctx *h, const float *samples, int64_t T, int64_t n_chains, double alpha,
                  const double *mu, const double *L, const double *ref_lo,
                  const double *ref_hi, double *lo, double *hi, double *metric);

/* Sliced Wasserstein distance of Sec. 4.1 between sample sets a ([Ta][d][chains_a]) and b
 * ([Tb][d][chains_b]): the mean over n_proj fixed unit directions w_k of the 1-d
 * Wasserstein-1 distance between the projected draws, integral |F_a - F_b| over the merged
 * sorted projections.  w_k = xi / |xi| with xi the d normals of Philox (key proj_seed,
 * counter (k, 0, stream 6, 0)), so equal seeds give the same directions in every call.
 * Optional whitening (mu, L) as for best_credible.  At most 2^31 - 1 draws in total. */
int best_sliced_wasserstein(best_ctx *h, const float *a, int64_t Ta, int64_t chains_a,
                            const float *b, int64_t Tb, int64_t chains_b, int32_t n_proj,
                            uint64_t proj_seed, const double *mu, const double *L, double *out);

/* ---- learned emulator (training on plain-model pairs) ---- */

/* A trainer owns an FP64 master copy of the MLP parameters and Adam moments on the device.
 * Training minimises mean_c (MLP(t_c) - y_c)^2 with Adam (b1 0.9, b2 0.999, eps 1e-8).
 * width: a multiple of 128 in [128, 2048]; precision FP32, FP16 or BF16. */
int best_trainer_create(best_trainer **out, int32_t d, int32_t width, int32_t n_hidden,
                        const double *init_params, int32_t precision, void *stream);
void best_trainer_destroy(best_trainer *t);
/* One epoch over perm ([n] device int32): batch i = perm[iB .. (i+1)B), ragged tail dropped.
 * t_in: device [n][d] normalised inputs (FP32), y: device [n] standardised targets (FP32).
 * The learning rate follows lr1 + (lr0 - lr1)(1 + cos(pi s / total_steps)) / 2 at Adam
 * step s (counted from step0).  mean_loss (host, may be NULL) receives the epoch mean of
 * the minibatch losses (synchronises). */
int best_train_epoch(best_trainer *t, const float *t_in, const float *y, int64_t n,
                     const int32_t *perm, int32_t batch, double lr0, double lr1,
                     int64_t step0, int64_t total_steps, double *mean_loss);
/* Gradient of the minibatch loss at the current parameters (no update); grad: host
 * [nparams] FP64; loss: host. */
int best_train_grad(best_trainer *t, const float *t_in, const float *y, int64_t batch,
                    double *grad, double *loss);
int best_trainer_get_params(best_trainer *t, double *out); /* host [nparams] */
const char *best_trainer_last_error(const best_trainer *t);

/* Standardise n training targets: out[i] = (y[i] - mean) / std with the population std.
 * y: device FP64 [n]; out: device FP32 [n]; mean_std: host [2] receives (mean, std).  The
 * emulator then predicts log L = mean + std * MLP.  n >= 2; synchronises `stream`. */
int best_standardise(const double *y, int64_t n, float *out, double *mean_std, void *stream);

/* Normalised training inputs of the emulator: t[c][i] = (x[i][c] - center[i]) * invscale[i]
 * (the same map best_problem.in_center / in_invscale apply before the MLP).  x: device FP64
 * [d][n] (the library's structure-of-arrays layout); t: device FP32 [n][d] (the layout of
 * best_train_epoch's t_in); center, invscale: host [d], finite.  Synchronises `stream`. */
int best_normalise_inputs(const double *x, int64_t n, int32_t d, const double *center,
                          const double *invscale, float *t, void *stream);

/* Importance weights of emulator samples under the plain likelihood:
 * w_i = exp(lp_i - le_i) / sum_j exp(lp_j - le_j), evaluated with the maximum subtracted;
 * kish (host) = (sum w)^2 / sum w^2.  lp, le, w: device FP64 [n]; synchronises `stream`. */
int best_importance_weights(const double *logl_plain, const double *logl_emu, int64_t n,
                            double *w, double *kish, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BEST_H */
