/*
 * Plain CPU oracle for the bootstrap particle filter — TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product (the HIP library and its Python
 * binding) never calls it, and it shares no code with the product.
 *
 * Everything is FP64, single threaded, sequential and unblocked, following
 * the paper's statement of the methods:
 *   - bootstrap particle filter: Sec. 3.1.2, Alg. 2 (Particle-Filter);
 *   - Kalman filter likelihood: Sec. 3.1.1, Alg. 1 (scalar case);
 *   - marginal Metropolis-Hastings: Sec. 3.2.1, eq. (mh), Alg. 3;
 *   - SMC over parameters with attached particle or Kalman filters (SMC^2):
 *     Sec. 3.2.2, Alg. 4;
 *   - models: Sec. 2.1.1 eqs. (2-windkessel), (3-windkessel) and Sec. 2.1.2
 *     eq. (lorenz96-sde) with classic fixed-step RK4, the noise added after
 *     the step or, in the paper's form, inside the stages.
 *
 * Readings where the paper is silent are stated beside each function.
 * Particle state is structure-of-arrays: x[i*N + j] is component i of
 * particle j.
 */
#ifndef PF_ORACLE_H
#define PF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MODEL_WK = 1, ORC_MODEL_L96 = 2, ORC_MODEL_L96_STAGE = 3 };
enum { ORC_TAG_INIT = 1, ORC_TAG_NOISE = 2, ORC_TAG_RESAMPLE = 3, ORC_TAG_DATA = 4,
       ORC_TAG_OBS = 8, ORC_TAG_PATH = 9, ORC_TAG_MULTI = 10,
       ORC_TAG_REJECT = 11 };
#define ORC_REJECT_MAX_ATTEMPTS (1 << 21)
enum { ORC_OK = 0, ORC_NUMERIC = 4 };

typedef struct orc_problem {
  int32_t model;          /* ORC_MODEL_WK or ORC_MODEL_L96 */
  int32_t d;              /* state dimension */
  int32_t K;              /* substeps per observation interval */
  int32_t T;              /* number of observations */
  double h;               /* substep length */
  int32_t n_obs;          /* observed components per time */
  const int32_t* obs_idx; /* [n_obs] */
  double obs_sd;          /* observation noise sd */
  const double* obs;      /* [T][n_obs] (may be NULL for simulation) */
  const double* q;        /* windkessel flow series [T*K+1], NULL for L96 */
  uint64_t seed;          /* Philox key */
} orc_problem;

/* counter-based generator */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t w);
double orc_ln(double x);
void orc_sincos2pi(double u, double* s, double* c);
void orc_normals4(uint64_t seed, uint32_t tag, uint32_t blk, uint32_t iter, uint32_t j,
                  uint32_t n, uint32_t b, double z[4]);
void orc_normals_bulk(uint64_t seed, uint32_t tag, uint32_t iter, uint32_t b, uint32_t n,
                      int64_t count, double* z /* [count][4] for j = 0..count-1, blk 0 */);

/* models */
void orc_l96_drift(int32_t d, const double* x, double F, double* out);

/* filter pieces (step level) */
void orc_init(const orc_problem* P, const double* theta, int64_t N, uint32_t b, uint32_t iter,
              double* x);
void orc_propagate(const orc_problem* P, const double* theta, int64_t N, uint32_t b,
                   uint32_t iter, int32_t t, const double* x_in, double* x_out);
void orc_init_idx(const orc_problem* P, const double* theta, int64_t n, const int64_t* idx,
                  uint32_t b, uint32_t iter, double* x);
void orc_propagate_idx(const orc_problem* P, const double* theta, int64_t n, const int64_t* idx,
                       uint32_t b, uint32_t iter, int32_t t, const double* x_in, double* x_out);
void orc_weight(const orc_problem* P, const double* theta, int64_t N, int32_t t,
                const double* x, double* lw);
double orc_resample_u(uint64_t seed, int32_t t, uint32_t b, uint32_t iter);
int32_t orc_reduce_resample(int64_t N, const double* lw, double u, double* ell, double* ess,
                            int32_t* a);
void orc_gather(int32_t d, int64_t N, const double* x, const int32_t* a, double* x_out);

/* whole filter over t = 1..T; traces are optional (NULL) */
int32_t orc_pf_run(const orc_problem* P, const double* theta, int64_t N, uint32_t b,
                   uint32_t iter, int32_t T_run, double* ell, double* ess, double* loglik,
                   int32_t* anc_trace, double* lw_trace, double* x_final,
                   const double* u_override);

/* exact Kalman filter on the windkessel (scalar linear-Gaussian) */
double orc_kf_wk(const orc_problem* P, const double* theta, double* ell);

/* synthetic truth and observations */
void orc_simulate(const orc_problem* P, const double* theta, uint64_t data_seed,
                  double* x_traj /* [T+1][d] */, double* obs /* [T][n_obs] */);

/* marginal Metropolis-Hastings chains on Lorenz '96 log F */
int32_t orc_pmmh(const orc_problem* P, int64_t N, int32_t chain0, int32_t n_chains,
                 int32_t n_chains_total, int32_t iters, const double* log_f0,
                 const double* z, const double* alpha, double step_sd, double f_lo,
                 double f_hi, double sigma, double* log_f_trace /* [iters][n_chains] */,
                 double* ll_trace /* [iters][n_chains] */, int32_t* accepts /* [n_chains] */);

/* resampling variants and ESS-triggered resampling */
double orc_strat_u(uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int64_t k);
void orc_stratified_ancestors(int64_t N, const double* W, double S, int64_t jstar,
                              uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int32_t* a);
void orc_metropolis_ancestors(int64_t N, const double* lw, int32_t steps, uint64_t seed,
                              int32_t t, uint32_t b, uint32_t iter, int32_t* a);
void orc_reject_pair(uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int64_t k, int64_t r,
                     int64_t N, int64_t* j, double* u);
void orc_rejection_ancestors(int64_t N, const double* lw, uint64_t seed, int32_t t, uint32_t b,
                             uint32_t iter, int32_t* a);
double orc_multi_u(uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int64_t k);
void orc_multinomial_ancestors(int64_t N, const double* W, double S, int64_t jstar,
                               uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int32_t* a);
int32_t orc_pf_run_ex(const orc_problem* P, const double* theta, int64_t N, uint32_t b,
                      uint32_t iter, int32_t T_run, int32_t resampler, int32_t steps,
                      double ess_frac, double* ell, double* ess, double* loglik,
                      int32_t* anc_trace, double* lw_trace, int32_t* res_trace,
                      double* x_final);

/* the single state sample of Alg. 2 (ancestry traced back) */
int64_t orc_path_slot(uint64_t seed, int32_t s, uint32_t b, uint32_t iter, int64_t N);
int32_t orc_pf_path(const orc_problem* P, const double* theta, int64_t N, uint32_t b,
                    uint32_t iter, int32_t T_run, double* loglik, double* path, int64_t* idx);

/* windkessel Kalman filter, one interval; SMC with attached Kalman filters */
double orc_kf_wk_interval(const orc_problem* P, const double* theta, int32_t t, double* m,
                          double* V);
int32_t orc_smc2_kalman(const orc_problem* P, int32_t B, int32_t n_theta, const double* theta0,
                        int32_t T_run, const double* step_sd, const double* lo,
                        const double* hi, const double* z, const double* log_alpha,
                        const double* u_theta, double* theta_out, double* logw_out,
                        double* loglik_out, int32_t* accepts, double* ess_theta,
                        double* log_evidence, int32_t* anc_trace, int32_t* acc_trace,
                        double* logw_trace, double* mV_out);

/* whole-filter copy index (systematic selection on equal weights) */
int64_t orc_copy_index(int64_t k, int64_t n_src, int64_t n_dst, uint32_t w);

/* SMC over parameters with attached particle filters (SMC^2, Alg. 4) */
int32_t orc_smc2(const orc_problem* P, int32_t B, const int64_t* n_particles, int32_t n_theta,
                 const double* theta0, int32_t T_run, const double* step_sd, const double* lo,
                 const double* hi, const double* z, const double* log_alpha,
                 const double* u_theta, const uint32_t* w_copy, double* theta_out,
                 double* logw_out, double* loglik_out, int32_t* accepts, double* ess_theta,
                 double* log_evidence, int32_t* anc_trace, int32_t* acc_trace,
                 double* logw_trace, double* theta_trace, double* x_final);

/* Marginal Metropolis-Hastings on the windkessel parameters (R, C, Z,
 * sigma^2) with the Kalman filter's exact likelihood (Alg. 3 on Alg. 1);
 * priors and proposals of Sec. 2.1.1's parameter and proposal blocks. */
typedef struct orc_wk_mh {
  double prior_shape[3];  /* Gamma prior shapes of R, C, Z */
  double prior_scale[3];  /* Gamma prior scales of R, C, Z */
  double ig_shape;        /* Inverse-Gamma prior of sigma^2: shape */
  double ig_scale;        /* and scale */
  double step_sd[3];      /* truncated Gaussian proposal sd of R, C, Z (0: fixed) */
  double ig_prop_shape;   /* sigma^2' ~ Inv-Gamma(ig_prop_shape, ig_prop_factor sigma^2) */
  double ig_prop_factor;  /* (0: sigma^2 fixed) */
  double m0, s0;          /* P_p(t_0) ~ N(m0, s0^2) */
} orc_wk_mh;
double orc_ndtri(double p);
void orc_wk_theta(const orc_problem* P, const orc_wk_mh* H, const double* rczs, double* theta);
double orc_wk_log_prior(const orc_wk_mh* H, const double* rczs);
int32_t orc_kf_pmmh(const orc_problem* P, const orc_wk_mh* H, int32_t n_chains, int32_t iters,
                    const double* theta0, const double* prop, const double* alpha,
                    double* theta_trace, double* ll_trace, int32_t* accepts);

#ifdef __cplusplus
}
#endif
#endif
