/*
 * pf.h — C ABI of the MI355X (gfx950) bootstrap particle filter.
 *
 * The filter is Alg. 2 (Particle-Filter) of Murray, "Bayesian state-space
 * modelling on high-performance hardware using LibBi" (Sec. 3.1.2): particles
 * are propagated through the state-space model's transition, weighted by the
 * observation density, the marginal likelihood estimate is accumulated as the
 * product over time of the mean weight, and particles are resampled with
 * replacement in proportion to their weights.  The paper states the filter
 * over an interval t_{r:s} so that callers (marginal Metropolis-Hastings,
 * Alg. 3; SMC over parameters, Alg. 4) can run it piecewise; pf_step and
 * pf_resample are that unit for one observation interval.  Resampling is
 * systematic (one of the collective resamplers named in Sec. 3.3).
 *
 * Conventions (all entry points):
 *  - Device memory is owned by the caller: pf_workspace_bytes() says how
 *    much, pf_init() carves it.  The library allocates no device memory.
 *    Host arrays referenced by pf_config are copied during pf_init(); the
 *    caller may free them when it returns.
 *  - Every call is asynchronous on the HIP stream given to pf_init() (NULL =
 *    the null stream), except pf_loglik(), pf_get_*() and pf_timing_get(),
 *    which synchronise that stream.
 *  - Status codes: PF_OK; PF_E_INVAL for an argument rejected on the host
 *    before any HIP call; PF_E_DEVICE for a HIP runtime error; PF_E_STATE for
 *    a call out of order (pf_step twice without pf_resample, a step past T,
 *    any call on a destroyed handle); PF_E_NUMERIC from pf_loglik() when some
 *    filter met a time at which no weight was positive and finite (that
 *    filter's log-likelihood is then -infinity, and the flag is sticky until
 *    pf_reset).  pf_last_error() returns a message for the last failing call
 *    on the calling thread.
 *  - A handle is not thread safe; distinct handles are independent.
 *  - No call falls back to the CPU: without a gfx950 device every call that
 *    needs one returns PF_E_DEVICE.
 *
 * Particle state as the host sees it (pf_get_state, pf_set_state) is
 * structure-of-arrays: component i of particle k of filter b is at
 * x[i * N_total + offset_b + k], with offset_b the sum of the particle counts
 * of filters before b.  The device layout inside the workspace is the
 * library's own (the plain layout keeps 64-particle tiles with each tile's
 * components contiguous; the batched layout one row per component).
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pf_status {
  PF_OK = 0,
  PF_E_INVAL = 1,
  PF_E_DEVICE = 2,
  PF_E_STATE = 3,
  PF_E_NUMERIC = 4
} pf_status;

/* State-space models (Sec. 2.1).
 * PF_MODEL_WK: windkessel pressure, d = 1; exact step of the two-element
 *   windkessel ODE with the flow held constant over a substep (eq.
 *   2-windkessel), plus Gaussian noise on the pressure; observation of the
 *   three-element aortal pressure P_p + Z F (eq. 3-windkessel) with Gaussian
 *   noise.  theta = (a, c, Z, sigma_p, m0, s0): a = exp(-h/(RC)),
 *   c = R(1-a), initial P_p ~ N(m0, s0^2).  Requires cfg.q.
 * PF_MODEL_L96: Lorenz '96 (eq. lorenz96-sde), d in {4, 8, 16, 32, 40};
 *   classic RK4 substeps of length h on the drift, then the increment
 *   sigma dW with dW ~ N(0, h) per component; initial x ~ N(0, I);
 *   observation of components obs_idx with Gaussian noise.
 *   theta = (F, sigma).
 * PF_MODEL_L96_STAGE: the paper's form of the stochastic Lorenz '96 (Sec.
 *   2.1.2: the SDE read as an ODE whose forcing includes sigma dW/dt): per
 *   substep the forcing of component i is F + sigma sqrt(h) z_i / h, held
 *   over the step and integrated by the same classic RK4; no increment is
 *   added after the step.  Same theta, normals and observation model. */
enum { PF_MODEL_WK = 1, PF_MODEL_L96 = 2, PF_MODEL_L96_STAGE = 3 };

/* Arithmetic of the hot path.
 * PF_FP64: everything in FP64.
 * PF_FP32_MIXED: particle state, propagation and the observation residuals
 *   in FP32 (the log-weight is summed in FP64 from the FP32 state); the
 *   max-shifted sums, the weight prefix scan, the likelihood increment, its
 *   running sum and the ESS in FP64.  The state is rounded to FP32 after
 *   every substep.
 * PF_FP32_ACCURATE: the particle state is stored in FP32 and the model's
 *   slopes (the Lorenz '96 drift at the RK4 stages, the windkessel
 *   increment) and the normals are evaluated in FP32, as in PF_FP32_MIXED;
 *   within an observation interval the state and each substep's increment
 *   are carried in FP64, and the log-weight is taken from that state before
 *   it is rounded for storage.  The collective is as in PF_FP32_MIXED. */
enum { PF_FP64 = 0, PF_FP32_MIXED = 1, PF_FP32_ACCURATE = 2 };

/* Kernel organisation.
 * PF_LAYOUT_PLAIN: each filter is stepped by its own kernels (ancestors from
 *   the last resampling's marks, gather, propagate + weight; block combine,
 *   weight scan and stratum marks); any particle count up to 2^31 - 1.
 * PF_LAYOUT_BATCHED: all filters are stepped together: one flat propagate +
 *   weight kernel over every filter's particles, then one workgroup per
 *   filter for the collective part (likelihood, scan, ancestors; the gather
 *   is fused into the next propagation), filters split into groups stepped
 *   concurrently; every filter's particle count must be
 *   <= PF_BATCHED_MAX_PARTICLES. */
enum { PF_LAYOUT_PLAIN = 0, PF_LAYOUT_BATCHED = 1 };
#define PF_BATCHED_MAX_PARTICLES 8192

typedef struct pf_config {
  int32_t model;              /* PF_MODEL_* */
  int32_t precision;          /* PF_FP64, PF_FP32_MIXED or PF_FP32_ACCURATE */
  int32_t layout;             /* PF_LAYOUT_* */
  int32_t d;                  /* state dimension */
  int32_t K;                  /* substeps per observation interval, >= 1 */
  int32_t T;                  /* number of observation times, >= 1 */
  double h;                   /* substep length, > 0 */
  int32_t n_obs;              /* observed components per time, >= 1 */
  const int32_t* obs_idx;     /* host [n_obs], each in [0, d) */
  double obs_sd;              /* observation noise sd, > 0 */
  const double* obs;          /* host [T][n_obs], finite */
  const double* q;            /* host [T*K + 1] windkessel flow F(n h); NULL for L96 */
  int32_t B;                  /* number of filters, >= 1 */
  int32_t n_theta;            /* 6 for WK, 2 for L96 */
  const int64_t* n_particles; /* host [B], each >= 1 */
  const double* theta;        /* host [B][n_theta] */
  uint64_t seed;              /* key of the counter-based generator */
} pf_config;

typedef struct pf_handle pf_handle;

/* Device bytes pf_init() needs for cfg, or 0 if cfg is invalid (the reason
 * is then in pf_last_error()). */
size_t pf_workspace_bytes(const pf_config* cfg);

/* Validate cfg, carve d_workspace (device memory of ws_bytes >= the size
 * query, 256-byte aligned), copy cfg's host arrays to it and draw the initial
 * particles x(t0) ~ p(X0 | theta) with uniform weights (Alg. 2,
 * initialisation).  Sets t = 0 and every log-likelihood to 0.  hip_stream is
 * a hipStream_t or NULL.  On PF_OK *out receives a new handle. */
pf_status pf_init(const pf_config* cfg, void* d_workspace, size_t ws_bytes, void* hip_stream,
                  pf_handle** out);

/* One observation interval for every filter (Alg. 2, propagation and
 * weighting, time t -> t+1): K substeps of the transition from the current
 * equally weighted particles, log-weights log p(y(t+1) | x), then in FP64
 * M = max lw, S = sum exp(lw - M), ell = M + ln S - ln N (the log of the
 * time-(t+1) factor of the likelihood estimate), loglik += ell and
 * ESS = S^2 / sum exp(2(lw - M)).  Requires t < T and the previous interval
 * resampled. */
pf_status pf_step(pf_handle* h);

/* Systematic resampling of every filter after pf_step (Sec. 3.3): one
 * uniform u from the generator, strata (u + k)/N, ancestor
 * a_k = min{ j : N W_j > (u + k) S } with W the FP64 prefix sum of
 * exp(lw - M); the resampled set x_k = x_{a_k} is what the next pf_step
 * propagates (it gathers through the ancestors as it loads the state, so
 * the set is written out only for pf_get_state).  Ancestors are sorted. */
pf_status pf_resample(pf_handle* h);

/* Synchronise the stream and copy out per-filter results: loglik_out[B]
 * (running marginal log-likelihood), ess_out[B] (ESS of the last step; may be
 * NULL), *t_out (observations processed; may be NULL).  Returns
 * PF_E_NUMERIC if any filter is flagged (its loglik is -infinity). */
pf_status pf_loglik(pf_handle* h, double* loglik_out, double* ess_out, int32_t* t_out);

/* Per-step traces, synchronous: ell_out[B][T] and ess_out[B][T] (entries
 * after the current t are 0).  Either pointer may be NULL. */
pf_status pf_get_trace(pf_handle* h, double* ell_out, double* ess_out);

/* Wait for the work the handle has issued, then release the handle and its
 * HIP graph objects, streams and events (not the workspace).  The handle is
 * gone even when the wait reports an error. */
pf_status pf_destroy(pf_handle* h);

/* Run n_steps observation intervals (pf_step + pf_resample each) by replaying
 * HIP graphs captured on the first call (and again after a change of tuning
 * or resampler).  Each graph is captured on one stream and holds kernel
 * launches only: graphs of 1, 2, 4, ... 128 intervals (up to 8 for the plain
 * layout with more than four filters), of every filter (plain layout) or of
 * one filter group (batched layout, launched on the group's own stream
 * between a fork from and a join into the handle's stream); a run replays
 * the longest that fit first (200 = 128 + 64 + 8).  A batched handle set to
 * eager replay (pf_set_replay, or pf_autotune when it measured eager
 * launches faster on this host) issues the same kernels as eager launches
 * instead.  Same results as the eager calls either way. */
pf_status pf_graph_run(pf_handle* h, int32_t n_steps);

/* Replace every filter's parameters (host [B][n_theta]) and re-initialise
 * (t = 0, loglik = 0, fresh x(t0)) with generator iteration field
 * `iteration` (< 2^20), so that successive restarts draw independent
 * particles — the unit marginal Metropolis-Hastings needs (Alg. 3).
 * pf_reset keeps theta. */
pf_status pf_set_theta(pf_handle* h, const double* theta, uint32_t iteration);
pf_status pf_reset(pf_handle* h, uint32_t iteration);

/* ---- the windkessel Kalman filter ---------------------------------------- */
/* Exact marginal likelihood of every filter's parameters under the
 * windkessel model by the Kalman filter (Sec. 3.1.1, Alg. 1 with one state
 * and one observation, where each Cholesky factor is a square root), one
 * lane per filter, FP64: from N(m0, s0^2), per substep m <- a m + c q_{n-1},
 * V <- a^2 V + sigma_p^2; per observation v = y - (m + Z q), S = V + obs_sd^2,
 * ell = -(ln(2 pi S) + v^2/S)/2, then m += (V/S) v, V <- (1 - V/S) V.
 * loglik_out [B] and, if not NULL, ell_out [B][T] are host arrays; the
 * handle's particles are untouched.  Synchronous. */
pf_status pf_kalman(pf_handle* h, double* loglik_out, double* ell_out);

/* Marginal Metropolis-Hastings on the windkessel's circuit parameters
 * (R, C, Z, sigma^2) driven by the Kalman filter's exact likelihood
 * (Sec. 3.2.1, eq. mh, Alg. 3 with Alg. 1 as the likelihood; the priors and
 * proposals of Sec. 2.1.1's parameter and proposal blocks, Gamma and
 * Inverse-Gamma read as (shape, scale)).  The model parameters follow from
 * (R, C, Z, sigma^2) with the handle's substep h: a = exp(-h/(R C)),
 * c = R (1 - a) (eq. 2-windkessel), pressure noise sd c sigma (the noise is
 * on the flow), P_p(t_0) ~ N(m0, s0^2).  Prior: R, C, Z ~ Gamma(shape_k,
 * scale_k), sigma^2 ~ Inv-Gamma(ig_shape, ig_scale).  Proposal: R, C, Z each
 * a Gaussian step of sd step_sd[k] truncated to positive values (sd 0: the
 * parameter stays), sigma^2' ~ Inv-Gamma(ig_prop_shape, ig_prop_factor
 * sigma^2) (factor 0: it stays); the acceptance ratio carries both
 * proposals' density ratios. */
typedef struct pf_wk_mh {
  double prior_shape[3];  /* Gamma prior shapes of R, C, Z, > 0 */
  double prior_scale[3];  /* Gamma prior scales of R, C, Z, > 0 */
  double ig_shape;        /* Inverse-Gamma prior of sigma^2: shape > 0 */
  double ig_scale;        /* and scale > 0 */
  double step_sd[3];      /* truncated-Gaussian proposal sd of R, C, Z, >= 0 */
  double ig_prop_shape;   /* shape of the sigma^2 proposal, > 0 when moved */
  double ig_prop_factor;  /* its scale is ig_prop_factor sigma^2; >= 0 */
  double m0, s0;          /* initial pressure mean and sd (s0 >= 0) */
} pf_wk_mh;

/* B independent chains, one per filter slot of the windkessel handle h (its
 * flow series, observations, observation sd and h; its particles are
 * untouched), all iterations of a chain in one lane of one kernel on the
 * handle's stream (asynchronous).  The random numbers are inputs, device
 * arrays (FP64, 8-byte aligned, not overlapping the outputs):
 *   theta0 [B][4]       initial (R, C, Z, sigma^2), each > 0;
 *   prop   [iters][B][4] u_R, u_C, u_Z uniforms in (0, 1) and g, a
 *                       Gamma(ig_prop_shape, 1) variate;
 *   alpha  [iters][B]   uniforms in (0, 1].
 * Iteration i: for each moved k of R, C, Z with sd s, p0 = Phi(-x_k/s) and
 * y_k = x_k + s z, z = Phi^{-1}(p0 + u (1 - p0)) if u <= 1/2, else
 * -Phi^{-1}((1 - u)(1 - p0)) (one truncated draw by inversion, evaluated on
 * the tail that keeps it accurate); sigma^2' = factor sigma^2 / g.  A
 * proposal with a component that is not positive and finite is rejected
 * without a likelihood; otherwise it is accepted iff ln alpha <= (l' - l) +
 * ((ln p(theta') - ln p(theta)) + ln q(theta | theta') - ln q(theta' |
 * theta)).  Outputs, device arrays: theta_trace [iters][B][4] and ll_trace
 * [iters][B] (the chain after each iteration), accepts [B], and, if not
 * NULL, ll0 [B] (the initial states' log-likelihoods).  Inputs outside the
 * stated ranges are not reported; they never fault, and their results are
 * not specified. */
pf_status pf_kalman_pmmh(pf_handle* h, const pf_wk_mh* spec, int32_t iters,
                         const double* d_theta0, const double* d_prop, const double* d_alpha,
                         double* d_theta_trace, double* d_ll_trace, int32_t* d_accepts,
                         double* d_ll0);

/* ---- resampling variants ------------------------------------------------ */
/* Which resampler the filters use and when (Sec. 3.3 names multinomial,
 * systematic and stratified resampling and resamplers that avoid the
 * collective over the weights).  Takes effect from the next interval;
 * synchronous (rebuilds captured graphs).
 *   PF_RESAMPLE_SYSTEMATIC (default): one uniform u per filter and time,
 *     a_k = min{j : N W_j > (u + k) S}.
 *   PF_RESAMPLE_STRATIFIED: one uniform u_k per stratum (word k mod 4 of the
 *     generator at (k div 4, t, tag 3 | block 1 | iteration, b)),
 *     a_k = min{j : N W_j > (u_k + k) S}; sorted like systematic.
 *   PF_RESAMPLE_METROPOLIS: output k starts at particle k and takes `steps`
 *     Metropolis moves (<= PF_METROPOLIS_MAX_STEPS): proposal j' =
 *     floor(w N 2^-32), accepted iff ln u <= lw_j' - lw_j (ln by the same
 *     atanh series as the normals), move s using words 2r, 2r+1,
 *     r = (s-1) mod 2, of the generator at (k, t, tag 3 | block
 *     2 + (s-1) div 2 | iteration, b).  No scan or counts; unsorted; tends
 *     to multinomial resampling as steps grows.
 *   PF_RESAMPLE_REJECTION: needs the largest log-weight M but no scan:
 *     output k tries candidates j, k first, then floor(w N 2^-32) for fresh
 *     words w, accepting the first with ln u <= lw_j - M (the same ln);
 *     attempts 2p and 2p+1 use words (0, 1) and (2, 3) of the generator at
 *     (k, t + (p div 256) 2^20, tag 11 | block p mod 256 | iteration, b)
 *     (needs T < 2^20).  Each output is k with probability w_k/w_max +
 *     (1 - w_k/w_max) W_k, else j with (1 - w_k/w_max) W_j: unbiased
 *     offspring counts.  The expected number of attempts per output is
 *     N w_max / sum w (up to N for a collapsed filter); after 2^21 attempts
 *     the output keeps k.  Unsorted.
 *   PF_RESAMPLE_MULTINOMIAL (Alg. 2's own): independent uniforms u_k (word
 *     k mod 4 of the generator at (k div 4, t, tag 10 | iteration, b)),
 *     a_k = min{j : W_j > u_k S} by binary search of the cumulative weights;
 *     unsorted.
 * ess_frac: resample only when ESS < ess_frac N (+inf: every time).  A time
 * that does not resample keeps its log-weights (the next interval adds to
 * them), its likelihood factor is ln sum exp(carried + new) - ln sum
 * exp(carried) (ln N after a resampling), and its ancestors are the
 * identity.  pf_resample_u needs the default; pf_smc2 and pf_backtrace need
 * ess_frac = +inf. */
#define PF_RESAMPLE_SYSTEMATIC 0
#define PF_RESAMPLE_STRATIFIED 1
#define PF_RESAMPLE_METROPOLIS 2
#define PF_RESAMPLE_MULTINOMIAL 3
#define PF_RESAMPLE_REJECTION 4
#define PF_METROPOLIS_MAX_STEPS 508
pf_status pf_set_resampler(pf_handle* h, int32_t scheme, int32_t steps, double ess_frac);

/* ---- ancestry storage and the state sample ------------------------------- */
/* The bootstrap filter's single state sample x'(t_{0:s}) (Alg. 2, last lines;
 * Sec. 3.1.2): one particle drawn from the final weights and traced back
 * through its ancestors.  A caller-owned device history of
 * pf_history_bytes(cfg) bytes (256-byte aligned) holds every time's
 * propagated particles [T+1][d][N_total] (state precision; slot 0 the
 * initial particles) and ancestors [T][N_total] (slot t-1: those drawn from
 * the time-t weights), plus the backtrace's output.  pf_history_attach
 * (at t = 0, after pf_init or pf_reset; NULL detaches) records slot 0 and
 * makes every later interval, eager or graph-replayed, and every
 * re-initialisation record its slot (batched layout: the stepping kernels
 * also store their particles and ancestors there; plain layout: a copy
 * kernel per filter and interval).  pf_backtrace (after a resampled interval, at the
 * handle's time s) draws, per filter b, the final particle as the time-s
 * systematic ancestor at slot floor(w N_b 2^-32), w the first word of the
 * generator at counter (0, s, tag 9 | iteration, b) (a uniform slot makes
 * that ancestor one draw from the final weights), walks j <- a^j(t_i) for
 * i = s..1 (identity at i = 1), and writes the path to host path_out
 * [B][s+1][d] (FP64) and, if not NULL, the particle indices to idx_out
 * [B][s+1].  pf_set_state does not touch the history; pf_smc2 refuses
 * handles with a history.  Synchronous. */
size_t pf_history_bytes(const pf_config* cfg);
pf_status pf_history_attach(pf_handle* h, void* d_history, size_t bytes);
pf_status pf_backtrace(pf_handle* h, double* path_out, int32_t* idx_out);

/* ---- parameter inference drivers ---------------------------------------- */
/* Marginal Metropolis-Hastings chains (Sec. 3.2.1, eq. mh, Alg. 3) on the
 * Lorenz '96 forcing F with sigma fixed, one chain per filter of the handle
 * (all chains' filters are stepped together each iteration; the batched
 * layout is the intended one).  The chain state is theta = log F; proposal
 * theta' = theta + step_sd z; prior F ~ U(f_lo, f_hi), whose density in log F
 * carries the Jacobian F; a move is accepted iff F' lies in [f_lo, f_hi] and
 * ln(alpha) <= (ll' - ll) + (theta' - theta) (ties accept, as in Alg. 3).
 * Iteration i (0-based) runs its filters with generator iteration field
 * i + 1; the initial estimate uses 0.  The chain layer's random numbers are
 * inputs (host): log_f0[B], z[iters][B], alpha[iters][B] in (0, 1).  Outputs
 * (host): log_f_trace[iters][B], ll_trace[iters][B], accepts[B].
 * Synchronous; leaves the handle holding the last proposal's run. */
pf_status pf_pmmh(pf_handle* h, int32_t iters, const double* log_f0, const double* z,
                  const double* alpha, double step_sd, double f_lo, double f_hi, double sigma,
                  double* log_f_trace, double* ll_trace, int32_t* accepts);

/* SMC over the parameters with a particle filter attached to every
 * theta-particle (Sec. 3.2.2, Alg. 4; SMC^2 when the attached filter is the
 * bootstrap filter of Alg. 2).  Theta-particle j owns filter slot j of the
 * batched handle h; `proposal` is a second batched handle made from the same
 * configuration (model, sizes, particle counts, observations, seed,
 * precision) on the same stream, whose filters run the rejuvenation
 * proposals.  h is re-initialised with theta0 and generator iteration field
 * 0.  Per time i = 1..T_run, in the algorithm's order:
 *   1. theta-ancestors by systematic resampling (as for the particles; the
 *      algorithm writes multinomial) of the theta-weights v(t_{i-1}), the
 *      last likelihood increments, with uniform u[i-1]; at i = 1 the weights
 *      are uniform and the ancestors the identity;
 *   2. every slot takes its ancestor's parameters, likelihood and equally
 *      weighted particles; with unequal particle counts destination particle
 *      k takes source particle floor((k + w 2^-32) n_src / n_dst), w =
 *      w_copy[i-1][j] (systematic selection on equal weights);
 *   3. one marginal Metropolis-Hastings move per theta-particle (Alg. 3, eq.
 *      mh): theta' = theta + step_sd z[i-1][j] (parameters with step_sd 0
 *      stay), uniform prior on [lo, hi] for the moved parameters; outside it
 *      the move is rejected; inside, the proposal handle's filter j runs
 *      theta' over t_{0:i-1} with iteration field i, giving l' and x', and
 *      the move is accepted iff log_alpha[i-1][j] <= l' - l (ties accept),
 *      when theta, l and the filter become the proposal's;
 *   4. every filter of h advances over t_{i-1:i}; its increment ell_i^j is
 *      the new theta-log-weight and l^j += ell_i^j.
 * The evidence estimate is the sum over i of ln(sum_j exp v^j(t_i)) - ln B.
 * theta and z use the cfg.theta layout ([B][n_theta], raw: L96 (F, sigma),
 * windkessel (a, c, Z, sigma_p, m0, s0)); step_sd, lo, hi hold n_theta
 * (<= 8) entries.  B <= 8192, T_run <= cfg.T, particle counts <= 8192.
 * d_ws: caller-owned device memory of ws_bytes >= pf_smc2_workspace_bytes(),
 * 256-byte aligned.  Host inputs are copied at the call; outputs are host
 * arrays (the traces may be NULL).  The random numbers of this layer are
 * inputs.  Synchronous.  PF_E_NUMERIC if some time had no positive
 * theta-weight (the evidence is then -inf). */
typedef struct pf_smc2_in {
  int32_t T_run;
  const double* theta0;     /* [B][n_theta] initial theta-particles */
  const double* z;          /* [T_run][B][n_theta] proposal normals */
  const double* log_alpha;  /* [T_run][B] logs of the acceptance uniforms */
  const double* u;          /* [T_run] theta-resampling uniforms in [0, 1) */
  const uint32_t* w_copy;   /* [T_run][B] whole-filter copy offsets */
  double step_sd[8];
  double lo[8];
  double hi[8];
  int32_t filter;           /* PF_FILTER_PARTICLE, or PF_FILTER_KALMAN (windkessel) */
} pf_smc2_in;
typedef struct pf_smc2_out {
  double* theta;            /* [B][n_theta] final theta-particles */
  double* logw;             /* [B] final theta-log-weights (ell_T) */
  double* loglik;           /* [B] likelihood estimates l^j */
  int32_t* accepts;         /* [B] accepted moves */
  double* ess;              /* [T_run] theta-ESS after each time */
  double* log_evidence;     /* [1] */
  int32_t* anc_trace;       /* [T_run][B] theta-ancestors, or NULL */
  int32_t* acc_trace;       /* [T_run][B] accept flags, or NULL */
  double* logw_trace;       /* [T_run][B] theta-log-weights, or NULL */
  double* theta_trace;      /* [T_run][B][n_theta] theta-particles, or NULL */
} pf_smc2_out;
/* With filter = PF_FILTER_KALMAN (windkessel model; Alg. 4 with the Kalman
 * filter of Sec. 3.1.1 as Filter) each theta-particle carries an exact
 * Kalman filter (m, V) instead of particles: step 2 copies (m, V), step 3's
 * proposal filter is a Kalman filter from (m0', s0'^2) over t_{0:i-1}, step
 * 4 advances it, and the increments are exact; `proposal` is ignored (may be
 * NULL), any layout is accepted, and the handle's particle filters are
 * re-initialised afterwards. */
#define PF_FILTER_PARTICLE 0
#define PF_FILTER_KALMAN 1
size_t pf_smc2_workspace_bytes(const pf_config* cfg, int32_t T_run);
pf_status pf_smc2(pf_handle* h, pf_handle* proposal, void* d_ws, size_t ws_bytes,
                  const pf_smc2_in* in, pf_smc2_out* out);

/* Autotuner for the batched layout: for each candidate workgroup size of the
 * per-filter collective kernel (256, 512, 1024 lanes) and each number of
 * filter groups (1, 2, 4; groups are balanced by particle count and stepped
 * concurrently on their own streams, so one group's collective overlaps
 * another's propagation), re-initialises the filters and times `steps`
 * intervals (at most T - 1, after one untimed interval) of this handle's own
 * workload on eager launches — no graph is captured or destroyed per
 * candidate — and keeps the fastest pair.  It then captures the chosen
 * tuning's graphs once, times their replay over the same intervals, sets
 * the replay mode of pf_graph_run to whichever of the two was faster
 * (pf_get_tuning reports it), and re-initialises the filters (t = 0).  On
 * an error while trying the candidates the handle is put back on its
 * previous tuning; on any error it is re-initialised.
 * ms_out[9] (may be NULL) receives the mean interval time in ms of candidate
 * (groups index g, size index s) at [3g + s] (-1 when groups > B);
 * *threads_out and *groups_out (may be NULL) the choice.  Plain layout:
 * nothing to tune (both outputs 0). */
pf_status pf_autotune(pf_handle* h, int32_t steps, int32_t* threads_out, int32_t* groups_out,
                      double* ms_out);

/* Set the batched layout's tuning directly: collective_threads in
 * {256, 512, 1024}, groups in [1, 8] (capped at B).  Takes effect from the
 * next interval; the plain layout ignores it.  A different tuning waits for
 * the work already issued, drops the captured graphs (rebuilt by the next
 * pf_graph_run) and goes back to graph replay; the tuning the handle has
 * already changes nothing. */
pf_status pf_set_tuning(pf_handle* h, int32_t collective_threads, int32_t groups);

/* How pf_graph_run issues a batched handle's intervals: eager = 1, as eager
 * launches (the host issues them at the device's pace); eager = 0, by graph
 * replay (the default).  The plain layout always replays graphs.
 * PF_E_INVAL for another value. */
pf_status pf_set_replay(pf_handle* h, int32_t eager);

/* The batched layout's tuning and replay mode (host outputs, each may be
 * NULL): collective width, filter groups, and 1 for eager replay; zeros for
 * the plain layout. */
pf_status pf_get_tuning(pf_handle* h, int32_t* collective_threads, int32_t* groups,
                        int32_t* eager_replay);

/* ---- inspection and teacher forcing (synchronous; same kernels) -------- */
/* Current particle set, FP64 host [d][N_total]: after pf_resample (or init)
 * the equally weighted set; after pf_step the propagated, weighted set. */
pf_status pf_get_state(pf_handle* h, double* x_out);
/* Overwrite the current equally weighted set (only between intervals);
 * values are rounded to the path's precision. */
pf_status pf_set_state(pf_handle* h, const double* x_in);
/* Log-weights of the last pf_step, FP64 host [N_total]. */
pf_status pf_get_logweights(pf_handle* h, double* lw_out);
/* Ancestors of the last pf_resample, host [N_total], indices local to each
 * filter. */
pf_status pf_get_ancestors(pf_handle* h, int32_t* a_out);
/* pf_resample with caller-given uniforms u[B] in [0, 1) instead of the
 * generator's (brute-force checks of the resampler). */
pf_status pf_resample_u(pf_handle* h, const double* u);

/* ---- checkpoint and resume ---------------------------------------------- */
/* Resume from a checkpoint.  The filter is defined over an interval so that
 * it can be restarted from its own output (Sec. 3.1.2; SMC over parameters
 * re-enters it interval by interval, Alg. 4).  Puts every filter at t
 * observations processed (0 <= t <= T) with the equally weighted set x_in
 * (FP64 host [d][N_total], as pf_get_state returns it after pf_resample;
 * values are rounded to the path's precision) and the running
 * log-likelihoods loglik[B] (-infinity sets the filter's numeric flag; NaN
 * or +infinity is PF_E_INVAL).  The generator is positional: its counters
 * name the filter, particle, substep and the handle's iteration field, not a
 * place in a sequence.  So a handle with the same configuration, seed and
 * iteration (pf_reset) goes on exactly as the run the checkpoint came from:
 * T intervals in one run, and T/2 intervals, pf_get_state and pf_loglik,
 * then pf_restore and T/2 more on a fresh handle, give the same bits.  Equal
 * weights are assumed: after an interval in which an ESS-triggered
 * resampler kept its weights, those weights are not restored.  Trace rows
 * from t on are cleared.  PF_E_STATE between pf_step and pf_resample and on
 * a handle with a history attached.  Synchronous. */
pf_status pf_restore(pf_handle* h, int32_t t, const double* x_in, const double* loglik);

/* ---- stateless systematic resampler ------------------------------------ */
/* The resampling collective of one filter on its own (Alg. 2's likelihood
 * and ancestor lines with the systematic resampling of Sec. 3.3), for a
 * caller that propagates and weights particles itself.  Input: d_lw, n FP64
 * log-weights in device memory (a NaN counts as weight 0), and the uniform
 * u in [0, 1).  In FP64: M = max lw, S = sum exp(lw - M),
 * ell = M + ln S - ln n, ESS = S^2 / sum exp(2(lw - M)), and the ancestors
 * a_k = min{ j : n W_j > (u + k) S }, k = 0..n-1, with W the prefix sum of
 * exp(lw - M) (sorted; rounding overflow goes to the last positive weight)
 * — the same kernels and bits as pf_resample_u on the plain layout.
 * Outputs, device memory: d_anc[n] (int32), d_stats[2] = (ell, ESS); with
 * no positive finite weight ell = -infinity, ESS = 0 and the ancestors are
 * the identity.  Scratch: d_workspace, at least
 * pf_systematic_workspace_bytes(n) bytes (about 4.2 n), 256-byte aligned,
 * owned by the caller and reused freely between calls.  Asynchronous on
 * hip_stream (NULL = the null stream); every operation is a kernel launch,
 * so the call may be captured into a HIP graph.  Arguments are checked on
 * the host (PF_E_INVAL: NULL pointer, n outside [1, 2^31 - 1], u outside
 * [0, 1), workspace too small or misaligned) before any HIP call.  Calls on
 * one workspace must not overlap. */
size_t pf_systematic_workspace_bytes(int64_t n);
pf_status pf_systematic(const double* d_lw, int64_t n, double u, int32_t* d_anc, double* d_stats,
                        void* d_workspace, size_t ws_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * pf_systematic with the same inputs, outputs and results, but with no
 * workspace argument.  Its scratch is a static device array sized for
 * PF_SYSTEMATIC_NOALLOC_MAX_N weights (about 4.3 MB), one copy per GPU the
 * library runs on, held until the process ends; the call allocates nothing
 * (no hipMalloc, no allocating library routine).  n above the maximum is
 * rejected with PF_E_INVAL.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (on different streams, or from different
 * threads without ordering) race and must not be issued; calls in stream
 * order are safe.  The first call on a device looks up the array's device
 * address (hipGetSymbolAddress) and keeps it. */
#define PF_SYSTEMATIC_NOALLOC_MAX_N (1 << 20)
pf_status pf_systematic_noalloc(const double* d_lw, int64_t n, double u, int32_t* d_anc,
                                double* d_stats, void* hip_stream);

/* ---- synthetic data ----------------------------------------------------- */
/* Simulate the model from theta (host [n_theta]) with generator key
 * data_seed, in FP64 on the device (the same transition and observation
 * arithmetic as the filter, with the particle index fixed to 0).  d_out is a
 * caller-owned device buffer of out_doubles >= pf_simulate_doubles(cfg)
 * doubles; it receives the truth x(t_0..t_T) as [T+1][d] followed by the
 * observations as [T][n_obs]; the rest is scratch.  cfg.obs, cfg.B,
 * cfg.n_particles and cfg.theta are ignored.  Synchronous. */
size_t pf_simulate_doubles(const pf_config* cfg);
pf_status pf_simulate(const pf_config* cfg, const double* theta, uint64_t data_seed,
                      double* d_out, size_t out_doubles, void* hip_stream);

/* ---- measurement -------------------------------------------------------- */
typedef struct pf_timing {
  double propagate_ms;   /* propagate + weight kernels */
  double combine_ms;     /* block-combine kernels (likelihood increment, offsets) */
  double scan_ms;        /* weight scan + stratum count kernels */
  double gather_ms;      /* plain layout: ancestor kernels of the resamplers
                            without marks (and of an attached history) */
  double batched_ms;     /* batched layout: the collective kernels */
  int64_t propagate_launches, combine_launches, scan_launches, gather_launches,
      batched_launches;
} pf_timing;
/* When on, eager pf_step/pf_resample bracket each kernel with HIP events on
 * the handle's stream; pf_timing_get() synchronises and sums them.  Turning
 * it on or off waits for the issued work and clears the sums. */
pf_status pf_timing_enable(pf_handle* h, int32_t on);
pf_status pf_timing_get(pf_handle* h, pf_timing* out);

/* Message for the last failing call on this thread ("" if none). */
const char* pf_last_error(void);
/* Library version string. */
const char* pf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
