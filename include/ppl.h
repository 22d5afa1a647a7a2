/*
 * ppl.h -- C ABI of the MI355X (gfx950) particle-inference library libppl.so.
 *
 * The library runs the data-parallel hot path of particle-based inference over
 * hand-written generative models: many independent executions (particles)
 * draw latents at the model's `sample` sites and add to a log-weight at its
 * `factor` sites (paper Sec. 3.4, figure "sample-factor-observe-impl");
 * importance sampling normalises the log-weights over the executions (Sec.
 * 3.6.2); sequential Monte Carlo -- the particle-based method the paper names
 * as future work (Sec. 6) -- suspends every particle at each `factor`,
 * computes a log-sum-exp normaliser and the effective sample size (ESS), and
 * resamples systematically before resuming.  A suspended particle is a resume
 * point (the index of the next factor) plus fixed-size state in device memory,
 * in place of the paper's delimited continuations (Sec. 1.2, 4.3); every model
 * has a static maximum state size (Sec. 4.2.4).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are DEVICE pointers; everything else is host memory.
 *     The caller owns every buffer (inputs, outputs and the workspace); the
 *     library never allocates, frees or retains caller memory.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream)
 *     and is asynchronous unless a result struct asks for host scalars.
 *   - Return value: PPL_OK (0) or a negative PPL_E_* code.  Host-detectable
 *     errors (arguments, model id, workspace size, no gfx950 device) are
 *     reported before anything is launched.  Nothing throws across the ABI.
 *     ppl_last_error() gives a text for the last failing call on the thread.
 *   - Layouts are structure-of-arrays: a per-particle field f of particle i
 *     lives at [f * n_particles + i].
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by `seed`;
 *     counter = (particle or slot index, block index, step, instance << 8 | tag)
 *     with tags 0 = prior, 1 = proposal, 2 = resampling, 4 = simulated
 *     training pairs, 5 = network initialisation.  Results depend only on
 *     (seed, inputs), never on the launch configuration.
 */
#ifndef PPL_H
#define PPL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status -- */
enum {
    PPL_OK = 0,
    PPL_E_ARG = -1,          /* invalid argument (null pointer, bad size, bad hyper-parameter) */
    PPL_E_MODEL = -2,        /* unknown model id, or model not supported by this entry point   */
    PPL_E_DEVICE = -3,       /* no HIP device, or the current device is not gfx950            */
    PPL_E_HIP = -4,          /* a HIP runtime call failed (text in ppl_last_error)            */
    PPL_E_WORKSPACE = -5,    /* workspace missing or smaller than ppl_workspace_size()        */
    PPL_E_NONFINITE = -6,    /* a log-weight was NaN (device-detected)                        */
    PPL_E_ZERO_WEIGHT = -7,  /* every weight was zero: log Z-hat = -inf (device-detected)      */
    PPL_E_UNSUPPORTED = -8   /* valid request outside what the library implements            */
};

/* Short description of a status code (static storage). */
const char *ppl_status_string(int status);
/* Detail text of the last failing call on the calling thread ("" if none). */
const char *ppl_last_error(void);
/* Library ABI version (major * 100 + minor). */
int ppl_version(void);

/* ------------------------------------------------------------- models -- */
enum {
    /* Polynomial fit, the paper's running example (Sec. 1.1, figure "ppl-example2"):
     * n ~ UniformDiscrete{n_lo..n_hi}; c_j ~ Normal(0, sd) for j < n;
     * factor(-sum_d (y_d - sum_j c_j x_d^j)^2 / 2).  FP64 throughout.
     * data: x[D], y[D] float64; hyper = {sd, n_lo, n_hi} (default {10, 2, 5}, n_hi <= 5).
     * latents [6][N] float64: n, c_0..c_4 (c_j for j >= n are drawn but unused). */
    PPL_MODEL_POLY = 1,
    /* Bayesian linear regression: w_k ~ Normal(0, prior_sd), k < d;
     * observe(Normal(x_d . w, noise_sd), y_d) for every row (Sec. 3.4: observe
     * is factor of the log-density).  Likelihood in FP32, normaliser in FP64.
     * data: x = X row-major [D][d] float32, y[D] float32, dim = d in {4, 8, 12, 16};
     * hyper = {prior_sd, noise_sd} (default {1, 0.5}).  latents [d][N] float32. */
    PPL_MODEL_BLR = 2,
    /* Linear-Gaussian state space: x_0 = m0 + p0_sd z, x_t = a x_{t-1} + q_sd eps_t;
     * observe(Normal(x_t, r_sd), y_t), one factor per step.  FP32 state.
     * data: y[T] float32, x = NULL; hyper = {a, q_sd, r_sd, m0, p0_sd}
     * (default {0.9, 1, 0.5, 0, 0}).  latents [1][N] float32 (final x). */
    PPL_MODEL_LGSSM = 3,
    /* Gaussian mixture with K known components (1 <= K <= 8):
     * pi ~ Dirichlet(1_K), mu_k ~ Normal(0, mu_sd); one factor per datum,
     * log sum_k pi_k Normal(y_d; mu_k, comp_sd).  FP32 state.
     * data: y[D] float32, dim = K; hyper = {mu_sd, comp_sd} (default {5, 1}).
     * latents [2K][N] float32: log pi_0..log pi_{K-1}, mu_0..mu_{K-1}. */
    PPL_MODEL_GMM = 4,
    /* The BLR model of PPL_MODEL_BLR (same data, hyper-parameters, latents,
     * draws, proposals and summaries), with the likelihood evaluated from
     * sufficient statistics: A = X^T X, b = X^T y, c = y^T y are formed once
     * per call in FP64 (O(D d^2)), then each particle's residual sum of
     * squares is c - 2 w.b + w^T A w in FP64 (O(d^2) instead of O(D d)).
     * Importance sampling only. */
    PPL_MODEL_BLR_STATS = 5,
    /* Hidden Markov model with K discrete states over T steps (1 <= K <= 8,
     * 1 <= T <= 40): z_0 ~ Categorical(pi0), z_t ~ Categorical(A[z_{t-1}]),
     * observe(Normal(mu[z_t], sigma), y_t).  Every sample site has finite
     * support, so exact inference by enumeration applies (ppl_enumerate).
     * FP64 throughout.  data: y[T] float64, x = NULL, dim = K, dtype PPL_F64;
     * hyper = {K, sigma, pi0[K], A[K][K] (row = previous state), mu[K]}
     * (n_hyper = 2 + 2K + K^2, required; probabilities >= 0 and finite,
     * sigma > 0). */
    PPL_MODEL_HMM = 6
};

enum { PPL_F32 = 1, PPL_F64 = 2 };

/* Observed data of one model instance.  x / y are DEVICE pointers (read-only,
 * caller-owned); hyper is a HOST array (NULL or n_hyper == 0: model defaults). */
typedef struct ppl_data {
    const void *x;
    const void *y;
    int64_t n_data;          /* D (rows / points) or T (steps) */
    int32_t dim;             /* BLR: d; GMM: K; otherwise 0 */
    int32_t dtype;           /* PPL_F64 for POLY, PPL_F32 otherwise */
    const double *hyper;
    int32_t n_hyper;
} ppl_data;

/* Outputs.  Every pointer may be NULL (not produced).
 * d_scalars (DEVICE, 8 doubles, written asynchronously):
 *   [0] log Z-hat   [1] ESS (FP64)   [2] number of resamplings   [3] status (0 or PPL_E_*)
 *   [4] max log-weight   [5] s1 = sum exp(lw - max)   [6] s2 = sum exp(2(lw - max))   [7] N
 * Host scalars log_evidence / ess / n_resample / status are filled only when
 * sync_host != 0 (the call then blocks on the stream and also returns
 * PPL_E_NONFINITE / PPL_E_ZERO_WEIGHT when the device flagged them). */
typedef struct ppl_result {
    double log_evidence;
    double ess;
    int64_t n_resample;
    int32_t status;
    int32_t sync_host;
    double *d_scalars;        /* [8] */
    void *d_latents;          /* SoA [n_latent][N], model dtype (see the model list) */
    void *d_log_weights;      /* [N] final unnormalised log-weights: float64 for importance
                               * sampling (the FP64 sum the normaliser uses), float32 for SMC */
    double *d_summaries;      /* model posterior summaries (see ppl_importance) */
    /* SMC traces (ppl_smc only): */
    double *d_ess_trace;      /* [T]: ESS after factor t, before resampling */
    uint8_t *d_resampled;     /* [T]: 1 if resampled after factor t */
    int32_t *d_ancestors;     /* [max_events][N]: ancestor vector of each resampling event */
    int64_t max_events;       /* rows available in d_ancestors and d_event_lw */
    float *d_event_lw;        /* [max_events][N]: the log-weights each resampling event resampled from
                               * (FP32, as the event saw them); needs max_events > 0 */
    double *d_logz_trace;     /* [T]: the normaliser increment LSE(lw) - log N added to log Z-hat after
                               * factor t (at each resampling and after the last factor), 0 elsewhere;
                               * entries after a failing factor are not written */
    double *d_move_log_alpha; /* [max_events][move_steps][N]: log acceptance ratio of each
                               * resample-move step (ppl_smc_ex with move_steps > 0) */
} ppl_result;

/* Proposal for importance sampling (NULL or kind PPL_Q_PRIOR: the prior,
 * i.e. likelihood weighting).  Latents are drawn from the proposal stream
 * (tag 1) and each log-weight is log p + log L - log q.
 * PPL_Q_GAUSS_FULL (BLR): d_params = float32 [d] mean followed by [d][d]
 *   row-major lower-triangular Cholesky factor L (positive diagonal);
 *   w = mean + L z with z ~ N(0, I); dim = d.
 * PPL_Q_POLY_MIX (POLY with degrees 2..5): d_params = float64 [332]:
 *   lognl[4] (log-probabilities of n = 2..5), logmix[8] (log mixture weights),
 *   mean[4][8][5], lsd[4][8][5] (log-scales), indexed [n - 2][component][j];
 *   block 0 word 0 picks n and word 1 the component by inverse CDF, blocks 1, 2
 *   give eight normals (single-precision-stream Box-Muller), c_j = mean +
 *   exp(lsd) z_j for j < n; q(n, c) = P(n) sum_m w_m prod_j N(c_j; mean, e^lsd).
 *   dim = 5.
 * PPL_Q_GMM_MIX (GMM, K components): d_params = float64 [8 + 16 (2K - 1)]:
 *   logmix[8], mean[8][2K-1], lsd[8][2K-1] over the ordered unconstrained
 *   latents u = (mu_(1), log(mu_(k) - mu_(k-1)) for k = 2..K,
 *   log pi_(k) - log pi_(K) for k = 1..K-1); block 0 word 0 picks the
 *   component, blocks 1..4 give sixteen normals.  log p(u) includes log (K-1)!
 *   (Dirichlet(1)), log K! (the orderings) and the Jacobians of the gap and
 *   softmax maps.  dim = 2K - 1.
 * These two are what ppl_proposal_infer decodes from the network output. */
enum { PPL_Q_PRIOR = 0, PPL_Q_GAUSS_FULL = 1, PPL_Q_POLY_MIX = 2, PPL_Q_GMM_MIX = 3 };
typedef struct ppl_proposal {
    int32_t kind;
    int32_t dim;
    const void *d_params;
} ppl_proposal;

enum { PPL_ALGO_IS = 0, PPL_ALGO_SMC = 1, PPL_ALGO_LSE = 2, PPL_ALGO_RESAMPLE = 3, PPL_ALGO_MCMC = 4, PPL_ALGO_ENUM = 5 };

/* Bytes of device workspace an entry point needs for (model, data, N).
 * The workspace is a caller-owned device buffer, at least 256-byte aligned,
 * whose contents need not be initialised and may be reused between calls on
 * one stream. */
int ppl_workspace_size(int model, const ppl_data *data, int64_t n_particles, int algo,
                       size_t *bytes);

/* Importance sampling (paper Sec. 3.6.2): run the model n_particles times,
 * each execution's sample/factor calls give it a log-weight; the FP64
 * log-sum-exp normaliser gives log Z-hat = LSE(lw) - log N and
 * ESS = (sum w)^2 / sum w^2.
 * model: PPL_MODEL_POLY, PPL_MODEL_BLR, PPL_MODEL_BLR_STATS or PPL_MODEL_GMM.
 * n_particles in [1, 2^31).
 * GMM importance sampling draws its latents and evaluates the prior and
 * proposal densities in FP64; the likelihood is FP32 per datum (hardware exp
 * and log, as in the SMC), summed in FP32 within blocks of 16 data and in
 * FP64 across blocks.  Its latents are float64 [2K][N] (log pi_k, mu_k) and
 * its prior draws are those of the SMC initial particles.
 * d_summaries (FP64):
 *   POLY: [0..3] P(n = 2..5 | y); [4 + 5(n-2) + j] E[c_j | n, y] (0 where that
 *         degree has no mass); [24 + j] E[c_j 1{j < n} | y]        -> 29 values
 *   BLR, BLR_STATS: [0..d-1] E[w | y]                                -> d values
 *   GMM:  [k] E[mu_(k) | y], the k-th smallest mean, k < K           -> 8 values */
int ppl_importance(int model, const ppl_data *data, int64_t n_particles, uint64_t seed,
                   const ppl_proposal *q, void *d_ws, size_t ws_bytes, void *stream,
                   ppl_result *out);

/* ppl_importance without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, outputs and errors as
 * ppl_importance; the workspace is a fixed library-owned device array of
 * PPL_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends).  Requests
 * whose ppl_workspace_size(..., PPL_ALGO_IS) exceeds it fail with
 * PPL_E_UNSUPPORTED before anything is launched: about 10^8 particles for
 * BLR with d = 16.  Calls no allocating routine.  Every call on one GPU uses
 * the same array, so calls that overlap on a GPU (other streams or threads)
 * race; serialise them. */
enum { PPL_NOALLOC_SCRATCH_BYTES = 16 << 20 };
int ppl_importance_noalloc(int model, const ppl_data *data, int64_t n_particles, uint64_t seed,
                           const ppl_proposal *q, void *stream, ppl_result *out);

/* FP64 normaliser of a device log-weight vector d_lw[n] (dtype PPL_F32 or
 * PPL_F64), the normalisation step of importance sampling (paper Sec. 3.6.2:
 * the weights of the executions are normalised over all of them):
 * d_out[5] = {max, s1, s2, LSE = max + log s1, ESS = s1^2 / s2}.
 * -inf entries carry zero weight; all -inf gives LSE = -inf and ESS = 0;
 * a NaN entry makes every output NaN. */
int ppl_lse_ess(const void *d_lw, int dtype, int64_t n, double *d_out, void *d_ws,
                size_t ws_bytes, void *stream);

/* Systematic resampling with integer-quantised weights, the resampling step
 * of particle-based inference (paper Sec. 6, named there as future work);
 * association-free, so the result does not depend on the reduction order:
 *   q_i = floor(exp(lw_i - max) * 2^k), k = 62 - ceil(log2 n);  Q = inclusive
 *   prefix sum, S = Q_{n-1};  R = 64-bit word from Philox block
 *   (0, 0, step, inst << 8 | 2);  U = floor(R S / 2^64);
 *   d_anc[j] = min{a : n Q_a > j S + U}, j < n.
 * NaN entries carry zero weight; if every weight is zero, every d_anc[j] = -1. */
int ppl_resample(const void *d_lw, int dtype, int64_t n, uint64_t seed, uint32_t step,
                 uint32_t inst, int32_t *d_anc, void *d_ws, size_t ws_bytes, void *stream);

/* Systematic resampling followed by the gather of the particle state, the
 * resampling step between factors of particle-based inference (paper Sec. 6,
 * future work).  Ancestors follow ppl_resample's rule with the same Philox
 * block, so d_anc (optional, may be NULL) equals ppl_resample's output; then
 *   d_state_out[f * n + j] = d_state_in[f * n + d_anc[j]],  f < n_fields, j < n
 * for structure-of-arrays state of 32-bit words (FP32 or int32 fields), laid
 * out [n_fields][n].  Both state buffers are caller-owned device memory of
 * n_fields * n * 4 bytes and must not overlap (PPL_E_ARG).  Workspace: the
 * PPL_ALGO_RESAMPLE size.  If every weight is zero, every d_anc[j] = -1 and
 * every output word is a quiet NaN (0x7fc00000). */
int ppl_resample_gather(const void *d_lw, int dtype, int64_t n, uint64_t seed, uint32_t step,
                        uint32_t inst, int32_t n_fields, const void *d_state_in,
                        void *d_state_out, int32_t *d_anc, void *d_ws, size_t ws_bytes,
                        void *stream);

/* Raw stream: d_out[4 i + r] = word r of Philox4x32-10 block
 * (i, c1, c2, c3) under key seed, for i < n.  Every random choice a sample
 * site makes (paper Sec. 3.4) is drawn from these words. */
int ppl_philox(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
               uint32_t *d_out, void *stream);

/* Sequential Monte Carlo over the model's factors (paper Sec. 6 future work;
 * sample/factor semantics of Sec. 3.4).  Bootstrap proposal; after factor t
 * (t < T - 1) the particles are resampled with ppl_resample's rule when
 * ESS < ess_frac * N, and the epoch's normaliser LSE(lw) - log N is added to
 * log Z-hat in FP64; the final epoch's normaliser is added after the last
 * factor.  model: PPL_MODEL_LGSSM or PPL_MODEL_GMM.  ess_frac in [0, 1].
 * One workgroup per CU holds up to 4096 particles, so N is limited by the
 * device (2^20 on 256 CUs; PPL_E_UNSUPPORTED beyond).  Checking aid: with the
 * environment variable PPL_SMC_POLL_ALL=1 every read of another workgroup's
 * tagged resampling words takes the polling path; the results do not change. */
int ppl_smc(int model, const ppl_data *data, int64_t n_particles, uint64_t seed,
            double ess_frac, void *d_ws, size_t ws_bytes, void *stream, ppl_result *out);

/* Options of ppl_smc_ex. */
typedef struct ppl_smc_options {
    double ess_frac;          /* resample when ESS < ess_frac N; in [0, 1] */
    int32_t move_steps;       /* resample-move: Metropolis-Hastings steps per particle after each
                               * resampling (0: none); PPL_MODEL_GMM only; 0..64 */
    int32_t reserved;
    double move_scale;        /* random-walk scale factor lambda (0: 2.38 / sqrt(2K - 1)) */
    int64_t t_begin;          /* first factor of this call: 0, or > 0 to resume from d_checkpoint */
    int64_t t_end;            /* factor to stop before (0: T); < T stores the run's state in d_checkpoint */
    void *d_checkpoint;       /* DEVICE buffer of ppl_smc_checkpoint_bytes() (caller-owned), needed when
                               * t_begin > 0 or t_end < T */
} ppl_smc_options;

/* Bytes of an SMC checkpoint: a 256-byte header (next factor, N, state fields,
 * log Z so far, resamplings, last merged maximum, status) and per particle its
 * state fields, log-weight and the log-weight's compensation term. */
int ppl_smc_checkpoint_bytes(int model, const ppl_data *data, int64_t n_particles, size_t *bytes);

/* ppl_smc with options; resample-move for the mixture model.  After each
 * resampling at factor s every particle takes move_steps Metropolis-Hastings
 * steps (the acceptance rule of the paper's MH method, Sec. 3.6.3) whose
 * target is the posterior given y_0..y_s, so particles that resampling made
 * identical spread out again (particle inference, Sec. 6).  The log-weights
 * stay 0 (the moves keep the equally weighted population's target).
 *   coordinates u = (log pi_k - log pi_K for k < K, mu_k for k <= K); prior
 *     density Dirichlet(1) x Normal(0, mu_sd)^K, with the softmax Jacobian;
 *   proposal u' = u + h z, z standard normal, h fixed by s:
 *     h_mu = lambda / sqrt(1 / mu_sd^2 + (s + 1) / (K comp_sd^2)),
 *     h_b  = lambda / sqrt(3 / pi^2 + (s + 1) / (2K));
 *   accept when log v < log alpha = [l(u') + log p(u')] - [l(u) + log p(u)]
 *     in FP64, l the log-likelihood of y_0..y_s (FP32 factors summed in FP32
 *     within blocks of 16 data and in FP64 across blocks);
 *   words: move m of slot j uses Philox blocks (j, 8m + b, s, inst << 8 | 7),
 *     b < 4 for sixteen normals (the first 2K - 1 used), word 0 of block
 *     8m + 4 for the uniform v.
 * Each move costs O(s K) per particle.  d_move_log_alpha (with max_events)
 * records log alpha per event, step and particle.
 * Stop and resume: a call runs factors t_begin .. t_end - 1.  With t_end < T
 * it stores the run's state in d_checkpoint and reports the log Z-hat
 * accumulated so far (the increments of the resamplings up to t_end - 1) with
 * ESS 0; a later call with t_begin = that t_end (same model, data, N, seed and
 * options) continues from it, and the pieces together give the same bits as
 * one call over all T factors (every random word is a function of the factor
 * index; the checkpoint holds the FP32 log-weights with their compensation
 * terms and the FP64 log Z-hat exactly).  A checkpoint whose header does not
 * match (next factor, N, state fields) makes the status PPL_E_ARG on the
 * device.  Traces and event records are written for the factors and events
 * of each call (event rows continue the checkpoint's count). */
int ppl_smc_ex(int model, const ppl_data *data, int64_t n_particles, uint64_t seed, const ppl_smc_options *opt,
               void *d_ws, size_t ws_bytes, void *stream, ppl_result *out);

/* ------------------------------------------- Metropolis-Hastings -- */
/* Outputs of ppl_mcmc (any pointer may be NULL).
 * d_scalars (DEVICE, 4 doubles): {acceptance rate, samples kept (chains x
 *   iterations after the burn-in), chains, status}. */
typedef struct ppl_mcmc_result {
    double accept_rate;       /* host copy of d_scalars[0] (sync_host only) */
    int32_t sync_host;
    int32_t reserved;
    double *d_scalars;        /* [4] */
    double *d_state;          /* [6][n_chains] final n and c_0..c_4 (slots j >= n hold 0) */
    int64_t *d_accepts;       /* [n_chains] accepted proposals per chain */
    double *d_summaries;      /* [29], the layout of ppl_importance's POLY summaries, from every chain's
                               * states after the burn-in */
    int8_t *d_n_trace;        /* [n_iters][n_chains] n after each iteration */
    double *d_log_alpha;      /* [n_iters][n_chains] log acceptance ratio of each proposal */
} ppl_mcmc_result;

/* Lightweight Metropolis-Hastings (paper Sec. 3.6.3): n_chains independent
 * chains of n_iters iterations, one chain per GPU lane.  A chain's trace is
 * the set of sites its execution reached; an iteration picks one uniformly,
 * resamples it from its prior and re-executes the model, keeping the values
 * of sites both executions reach, drawing sites only the new one reaches
 * fresh from their prior and dropping the others; accepted when
 * log v < log L(x') - log L(x) + log |trace(x)| - log |trace(x')|.
 * model: PPL_MODEL_POLY (trace n, c_0..c_{n-1}; data and hyper-parameters as
 * for importance sampling).  Words of iteration t of chain c (tag 8): block
 * (c, 3t, 0) word 0 the site (0 is n, j + 1 is c_j), word 1 the proposed n,
 * word 2 the uniform v; blocks (c, 3t + 1, 0) and (c, 3t + 2, 0) one
 * double-precision Box-Muller pair each (z_0 for a resampled coefficient,
 * z_1.. for fresh ones).  Chain c starts from the prior draw of importance
 * sampling's execution c.  FP64 throughout.  n_chains in [1, 2^31),
 * n_iters >= 0, 0 <= burn_in <= n_iters.  Workspace: PPL_ALGO_MCMC bytes
 * for n_chains (ppl_workspace_size with n_particles = n_chains). */
int ppl_mcmc(int model, const ppl_data *data, int64_t n_chains, int64_t n_iters, int64_t burn_in, uint64_t seed,
             void *d_ws, size_t ws_bytes, void *stream, ppl_mcmc_result *out);

/* ------------------------------------------------------ enumeration -- */
/* Outputs of ppl_enumerate (any device pointer may be NULL). */
typedef struct ppl_enum_result {
    double log_evidence;      /* host copies of d_scalars[0], [2], [3] (sync_host only) */
    double map_log_joint;
    int32_t status;
    int32_t sync_host;
    double *d_scalars;        /* [4]: log Z, number of paths K^T, log joint of the most probable
                               * path, status (0, PPL_E_ZERO_WEIGHT or PPL_E_NONFINITE) */
    double *d_marginals;      /* [T][K]: P(z_t = k | y) */
    int32_t *d_map;           /* [T]: the most probable path (the lowest path index among equal
                               * log joints; index = sum_t z_t K^(T-1-t)) */
} ppl_enum_result;

/* Exact inference by enumeration (paper Sec. 3.6.1): every execution of the
 * model, i.e. every path z in {0..K-1}^T, weighted by the product of its
 * sample probabilities and its factors; Z = sum_z exp(lw(z)).  Every path is
 * evaluated (no dynamic programming over the chain structure).  Sums are FP64
 * relative to the largest log-weight; a NaN log-weight makes the status
 * PPL_E_NONFINITE and log Z NaN; all weights zero: PPL_E_ZERO_WEIGHT and
 * log Z = -inf.  model: PPL_MODEL_HMM; K^T <= 2^50.  Workspace:
 * ppl_workspace_size(PPL_MODEL_HMM, data, 1, PPL_ALGO_ENUM).  With sync_host
 * the call blocks on the stream and returns the device status. */
int ppl_enumerate(int model, const ppl_data *data, void *d_ws, size_t ws_bytes, void *stream, ppl_enum_result *out);

/* ------------------------------------------------------ batched SMC -- */
/* One model instance of a batched run.  The caller passes the same table
 * twice: a HOST copy (validated and used for scheduling) and a DEVICE copy
 * with identical bytes (read by the kernel).  Instance i uses Philox
 * instance id i (counter word 3 = i << 8 | tag), so its result equals a
 * ppl_smc-style run of that instance alone with instance id i. */
typedef struct ppl_instance {
    const float *y;           /* DEVICE observations [n_data] */
    int64_t n_data;           /* D_i (factors) */
    int64_t n_particles;      /* N_i */
    int32_t dim;              /* GMM: K_i in 1..8 */
    int32_t flags;            /* 0 or PPL_INST_NO_RECORD */
    double hyper[2];          /* GMM: {mu_sd, comp_sd}; 0 = default {5, 1} */
    int32_t move_steps;       /* resample-move steps per particle after each resampling (0..64; see ppl_smc_ex) */
    int32_t reserved;
    double move_scale;        /* random-walk scale factor (0: 2.38 / sqrt(2K - 1)) */
} ppl_instance;

/* The instance's resampling events are not recorded: it has no rows in
 * d_ancestors / d_event_lw of ppl_batch_result (see there). */
enum { PPL_INST_NO_RECORD = 1 };

/* Launch configuration of the batched engine (0 fields = default/derived).
 * particles_per_lane P in {1,2,4,8}; wgs_per_instance W = 512-thread
 * workgroups that hold one instance (W * 512 * P >= max N_i, W <= 64);
 * spec_block = largest number of factors advanced between synchronisations
 * (1..256).  For every valid choice the outputs are the same bits: log-weights,
 * latents, ancestors, decisions, normaliser increments, log Z-hat and final
 * ESS (the normaliser sums weights as exact 128-bit fixed-point integers).
 * Only the trigger ESS values (d_ess_trace) follow the launch shape in their
 * last bits, through the order of their FP32 / FP64 partial sums; a decision
 * whose ESS lies within that rounding of ess_frac N may therefore differ. */
typedef struct ppl_tune {
    int32_t particles_per_lane;
    int32_t wgs_per_instance;
    int32_t spec_block;
    int32_t reserved;
} ppl_tune;

/* Outputs of a batched run (any pointer may be NULL):
 *   d_out [n_inst][4] FP64: log Z-hat, final ESS, resamplings, status;
 *   d_log_weights [sum N_i] float32, instance i at offset P_i = sum_{k<i} N_k;
 *   d_latents [16 * sum N_i] float32, instance i at 16 P_i as [2 K_i][N_i]
 *             (log pi_k then mu_k);
 *   d_ess_trace / d_resampled / d_logz_trace [sum D_i], instance i at offset
 *             sum_{k<i} D_k (d_logz_trace as in ppl_result);
 *   d_ancestors [max_events * sum' N_i] int32 and d_event_lw [max_events *
 *             sum' N_i] float32, where sum' runs over the recorded instances
 *             (flags without PPL_INST_NO_RECORD): recorded instance i at
 *             max_events * R_i, R_i = sum' over recorded k < i of N_k, as
 *             [max_events][N_i]: the ancestor vectors of its first max_events
 *             resampling events and the log-weights they resampled from;
 *   d_move_log_alpha [max_events * sum' M_i N_i] FP64: recorded instance i
 *             with M_i = move_steps > 0 at max_events * sum' over recorded
 *             k < i of M_k N_k, as [max_events][M_i][N_i]: the log acceptance
 *             ratios of its resample-move steps;
 *   d_counters [4] int64, work summed over the instances: particle-factors
 *             evaluated in speculative blocks (first passes, including
 *             factors past a trigger), particle-factors recomputed after a
 *             rollback, speculative blocks (team merges), resampling events.
 *             The algorithmic count is sum N_i D_i. */
typedef struct ppl_batch_result {
    double *d_out;
    float *d_log_weights;
    float *d_latents;
    double *d_ess_trace;
    uint8_t *d_resampled;
    int32_t *d_ancestors;
    int64_t max_events;
    float *d_event_lw;
    double *d_logz_trace;
    double *d_move_log_alpha;
    int64_t *d_counters;
} ppl_batch_result;

/* Workspace bytes for a batched run with configuration `tune` (NULL: enough
 * for every configuration the autotuner tries). */
int ppl_smc_batched_workspace_size(int model, int32_t n_inst, const ppl_instance *h_inst, const ppl_tune *tune,
                                   size_t *bytes);

/* Batched SMC over n_inst independent mixture-model instances in one
 * persistent cooperative launch (same per-instance algorithm and outputs as
 * ppl_smc: particle inference with a resampling step at the factors, paper
 * Sec. 6; the factor of Sec. 3.4 is one datum's mixture density).  tune NULL: the autotuner's cached choice for this batch shape,
 * else the defaults.  model: PPL_MODEL_GMM.  n_inst in 1..1024. */
int ppl_smc_batched(int model, int32_t n_inst, const ppl_instance *h_inst, const ppl_instance *d_inst,
                    uint64_t seed, double ess_frac, const ppl_tune *tune, void *d_ws, size_t ws_bytes,
                    void *stream, ppl_batch_result *out);

/* Autotuner for ppl_smc_batched (a launch-shape search with no counterpart
 * in the paper): times each candidate configuration once on this batch
 * (after a warm-up run, synchronising the stream): P in {1, 2, 4, 8} with speculative
 * blocks of 16..256 factors, each with the smallest team W that holds the
 * largest instance and with 2 W.  Returns the fastest in *best and caches it
 * for batches of the same shape (instance count, particle and data totals,
 * largest instance), in the process and in the PPL_TUNE_CACHE file (see
 * ppl_smc_tune_lookup).  Writes the outputs like ppl_smc_batched. */
int ppl_smc_autotune(int model, int32_t n_inst, const ppl_instance *h_inst, const ppl_instance *d_inst,
                     uint64_t seed, double ess_frac, void *d_ws, size_t ws_bytes, void *stream,
                     ppl_batch_result *out, ppl_tune *best);

/* The configuration a call with tune == NULL would use for this batch shape
 * (instance count, particle and data totals, largest instance): the
 * autotuner's result cached in this process, or a line of the persisted
 * cache.  PPL_E_UNSUPPORTED if there is none (the call would use the
 * defaults).  Persisted cache: when the environment variable PPL_TUNE_CACHE
 * names a file, ppl_smc_autotune appends each result to it (keyed by the
 * device architecture and compute-unit count and the batch shape), and
 * lookups merge that file's lines for the current device into the process
 * cache the first time they see it.  An unreadable file counts as empty. */
int ppl_smc_tune_lookup(int model, int32_t n_inst, const ppl_instance *h_inst, ppl_tune *out);
/* Forgets the process cache (the next lookup re-reads PPL_TUNE_CACHE). */
void ppl_smc_tune_cache_clear(void);

/* --------------------------------------------------- learned proposal -- */
/* A small network maps 64 summary statistics of a dataset to a Gaussian-
 * mixture proposal over the model's latents (PPL_Q_POLY_MIX / PPL_Q_GMM_MIX):
 * an MLP 64 -> 256 -> 256 -> 256 with ReLU after the first two layers, BF16
 * matrix-core products accumulating in FP32.  It is trained on (latent, data)
 * pairs simulated from the model's own prior by minimising -log q(latent | data)
 * with Adam, then used as the importance-sampling proposal (Sec. 3.6.2 with a
 * proposal other than the prior).  The prior proposal stays available through
 * ppl_importance.
 *
 * Summaries (FP64, then BF16 at the network input):
 *   POLY (42 used): mean x^j y / 10 (j = 0..7); mean x^k (k = 1..14);
 *     mean y^2 / 100; least-squares coefficients for n = 2..5 / 10;
 *     log(1 + (RSS_n - RSS_5) / 2) / 10 for n = 2..5 (residual sums of squares
 *     of the least-squares fits: the log-likelihood gaps); log D / 10.
 *   GMM (53 used): order statistics y_(floor((q + 1/2) D / 16)) / 10 (q < 16);
 *     counts on the unit bins of [-16, 16), ends clamped, / D; mean / 10;
 *     sd / 10; skewness; excess kurtosis / 10; log D / 10.
 * Output head (network outputs o[256]):
 *   POLY: o[0:4] degree logits; o[4:12] mixture logits; for degree n a block
 *     at 12 + 8 (n - 2)(n + 1): 8n means (10 o) then 8n log-scales
 *     (5 tanh(o / 5)), component-major.
 *   GMM: o[0:8] mixture logits; 8(2K-1) means (5 o); 8(2K-1) log-scales. */

/* Bytes of one parameter block (device, caller-owned, 256-byte aligned): FP32
 * master weights and biases, Adam first and second moments, BF16 copies of
 * the weights in [out][in] and [in][out] layouts, the Adam step count, then
 * the two BF16 layouts again in the order the fused training pass loads them
 * (all copies written by ppl_proposal_init and every Adam step). */
size_t ppl_proposal_weights_bytes(void);

/* Glorot-uniform initialisation: element e of W_l[out][in] (l = 0, 1, 2) is
 * (2u - 1) sqrt(6 / (in + out)) in FP32, u from word e mod 4 of Philox block
 * (e div 4, l, 0, tag 5); zero biases, moments and step count. */
int ppl_proposal_init(void *d_weights, uint64_t seed, void *stream);

/* Training configuration.  hyper (HOST) are the simulation hyper-parameters:
 * POLY {sd, n_lo, n_hi, noise_sd} (default {10, 2, 5, 1}; 2 <= n_lo <= n_hi <= 5);
 * GMM {mu_sd, comp_sd} (default {5, 1}).  Adam fields 0 take the defaults
 * lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8.  lr_decay_steps > 0 decays the
 * learning rate along a half cosine from lr (at step count 0) to
 * lr * lr_final_frac (at step count lr_decay_steps and after); the step count
 * is the parameter block's, so the schedule continues across calls. */
typedef struct ppl_train_config {
    int64_t n_pairs;         /* simulated pairs in this call, a multiple of batch */
    int32_t batch;           /* pairs per Adam step: a multiple of 64 in [64, 65536] */
    int32_t dim;             /* GMM: K in 1..8; POLY: 0 */
    int64_t n_data;          /* points per simulated dataset: POLY >= 1, GMM 1..4096 */
    double lr, beta1, beta2, eps;
    const double *hyper;
    int32_t n_hyper;
    int32_t use_graph;       /* nonzero: capture one step (it also simulates the next batch)
                                as a HIP graph, replayed for every step but the last */
    int64_t lr_decay_steps;  /* 0: constant learning rate */
    double lr_final_frac;    /* in [0, 1] */
} ppl_train_config;

int ppl_proposal_train_workspace_size(int model, const ppl_train_config *cfg, size_t *bytes);

/* n_pairs / batch Adam steps.  Step t (the block's step count, which
 * persists across calls) simulates pairs i < batch from Philox tag 4 with
 * counter (i, block, t, 4); the loss is the batch mean of -log q(latent_i |
 * summaries_i).  d_loss_trace (optional, FP64 [n_pairs / batch]) receives each
 * step's mean loss.  model: PPL_MODEL_POLY or PPL_MODEL_GMM. */
int ppl_proposal_train(int model, const ppl_train_config *cfg, uint64_t seed, void *d_weights,
                       double *d_loss_trace, void *d_ws, size_t ws_bytes, void *stream);

/* One batch of step `step` at the current weights, without updating them (a
 * checking aid; the workspace is that of ppl_proposal_train).  Outputs
 * (any may be NULL):
 *   d_grad [148224] FP32: gradient of the batch-mean loss, parameter order
 *     W1[256][64], b1[256], W2[256][256], b2, W3[256][256], b3;
 *   d_loss [1] FP64: the batch-mean loss;
 *   d_summaries [batch][64] FP64; d_latents [batch][16] FP64 (POLY: n, c_0..c_4;
 *     GMM: u_0..u_{2K-2}); d_outputs [256][batch] FP32 network outputs. */
int ppl_proposal_gradient(int model, const ppl_train_config *cfg, uint64_t seed, uint32_t step,
                          const void *d_weights, float *d_grad, double *d_loss, double *d_summaries,
                          double *d_latents, float *d_outputs, void *d_ws, size_t ws_bytes, void *stream);

int ppl_proposal_infer_workspace_size(int model, const ppl_data *data, int64_t n_particles, size_t *bytes);

/* Amortised inference: summaries of the observed data, one forward pass,
 * decode to PPL_Q_POLY_MIX / PPL_Q_GMM_MIX parameters, then importance
 * sampling with that proposal (outputs as ppl_importance).  widen >= 1
 * multiplies every component's scales (log-scales + log widen; 1 = as
 * trained), a tempering of the proposal for data unlike the training pairs.
 * d_q_params (optional) receives the decoded parameters, d_data_summaries
 * (optional) the 64 FP64 summaries.  POLY needs the degree range 2..5; GMM
 * needs D <= 8192. */
int ppl_proposal_infer(int model, const ppl_data *data, const void *d_weights, int64_t n_particles,
                       uint64_t seed, double widen, double *d_q_params, double *d_data_summaries,
                       void *d_ws, size_t ws_bytes, void *stream, ppl_result *out);

/* Adaptive tempering: runs ppl_proposal_infer with n_pilot particles (Philox
 * key `seed`) for each of the n_cand widen values in cand (HOST), and returns
 * in *best the one whose pilot ESS is largest (ties: the earlier candidate),
 * with the pilot ESS values in ess_out[n_cand] (HOST).  Needs no reference
 * value.  Blocks on the stream; the workspace is that of ppl_proposal_infer
 * for n_pilot particles.  n_cand in 1..16. */
int ppl_proposal_pick_widen(int model, const ppl_data *data, const void *d_weights, int64_t n_pilot,
                            uint64_t seed, const double *cand, int32_t n_cand, double *best, double *ess_out,
                            void *d_ws, size_t ws_bytes, void *stream);

/* Kernel timing (a measurement aid).  ppl_timing_enable(1) clears the
 * accumulators and makes the launchers bracket their dominant kernels
 * (blr_is_kernel, poly_is_kernel, smc kernels) with HIP events recorded on
 * the launch stream; ppl_timing_enable(0) stops recording.
 * ppl_timing_query waits for the recorded events of `kernel` and returns the
 * summed elapsed milliseconds and the number of timed launches. */
int ppl_timing_enable(int on);
int ppl_timing_query(const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* PPL_H */
