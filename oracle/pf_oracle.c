/*
 * Plain CPU oracle for the bootstrap particle filter — TEST INFRASTRUCTURE.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  FP64, single threaded, sequential.  Build with contraction off
 * (-ffp-contract=off) so every expression below is evaluated as written.
 *
 * Functions whose only pin is agreement with a definition given here (not
 * by the paper) say so in their comment.
 */
#include "pf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  The paper's library has a pseudorandom number
 * generator but does not name it (Sec. 4); this counter-based generator is
 * our reading, chosen so that every draw is a pure function of its position.
 * One round: the two 32x32->64 products M0*c0 and M1*c2 are split into
 * high/low words and mixed with c1, c3 and the round key; the key is bumped
 * by the Weyl constants between rounds.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform on (0,1): the centre of the w-th of 2^32 equal cells (exact). */
double orc_u01(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* Natural log of a positive normal double, from IEEE +,-,*,/ only:
 * x = f*2^e with f in [sqrt(1/2), sqrt(2)), ln f = 2 atanh(s), s=(f-1)/(f+1),
 * atanh summed as its odd power series through s^21 (|s| <= 0.1716, so the
 * first dropped term is below 2^-56 relative).  Written out, rather than
 * taken from libm, so that the normal transform is one fixed function of the
 * generator's words (a reading; the paper fixes no transform).  Pinned
 * against libm log in the tests. */
double orc_ln(double x) {
  uint64_t bits;
  memcpy(&bits, &x, sizeof bits);
  int e = (int)((bits >> 52) & 0x7ff) - 1022;
  bits = (bits & 0x000fffffffffffffULL) | 0x3fe0000000000000ULL; /* f in [0.5, 1) */
  double f;
  memcpy(&f, &bits, sizeof f);
  if (f < 0x1.6a09e667f3bcdp-1) { /* sqrt(1/2) */
    f = f + f;
    e = e - 1;
  }
  double s = (f - 1.0) / (f + 1.0);
  double s2 = s * s;
  double p = 1.0 / 21.0;
  p = p * s2 + 1.0 / 19.0;
  p = p * s2 + 1.0 / 17.0;
  p = p * s2 + 1.0 / 15.0;
  p = p * s2 + 1.0 / 13.0;
  p = p * s2 + 1.0 / 11.0;
  p = p * s2 + 1.0 / 9.0;
  p = p * s2 + 1.0 / 7.0;
  p = p * s2 + 1.0 / 5.0;
  p = p * s2 + 1.0 / 3.0;
  p = p * s2 + 1.0;
  double lnf = (2.0 * s) * p;
  double de = (double)e;
  /* ln 2 split so that de * LN2_HI is exact for |e| < 2^11 */
  return de * 0x1.62e42feep-1 + (de * 0x1.a39ef35793c76p-33 + lnf);
}

/* sin(2 pi u) and cos(2 pi u) for u in [0, 1): reduce to the nearest quarter
 * turn k (exact on the dyadic u), then Taylor series of sin and cos on
 * |phi| <= pi/4 through phi^19 and phi^18.  Same reading as orc_ln. */
void orc_sincos2pi(double u, double* s_out, double* c_out) {
  double v = 4.0 * u;
  double kf = floor(v + 0.5);
  double f = v - kf;
  int k = ((int)kf) & 3;
  double p = f * 0x1.921fb54442d18p0; /* pi/2 */
  double p2 = p * p;
  double sp = -1.0 / 121645100408832000.0;    /* -1/19! */
  sp = sp * p2 + 1.0 / 355687428096000.0;     /*  1/17! */
  sp = sp * p2 - 1.0 / 1307674368000.0;       /* -1/15! */
  sp = sp * p2 + 1.0 / 6227020800.0;          /*  1/13! */
  sp = sp * p2 - 1.0 / 39916800.0;            /* -1/11! */
  sp = sp * p2 + 1.0 / 362880.0;              /*  1/9!  */
  sp = sp * p2 - 1.0 / 5040.0;                /* -1/7!  */
  sp = sp * p2 + 1.0 / 120.0;                 /*  1/5!  */
  sp = sp * p2 - 1.0 / 6.0;                   /* -1/3!  */
  sp = sp * p2 + 1.0;
  sp = sp * p;
  double cp = -1.0 / 6402373705728000.0;      /* -1/18! */
  cp = cp * p2 + 1.0 / 20922789888000.0;      /*  1/16! */
  cp = cp * p2 - 1.0 / 87178291200.0;         /* -1/14! */
  cp = cp * p2 + 1.0 / 479001600.0;           /*  1/12! */
  cp = cp * p2 - 1.0 / 3628800.0;             /* -1/10! */
  cp = cp * p2 + 1.0 / 40320.0;               /*  1/8!  */
  cp = cp * p2 - 1.0 / 720.0;                 /* -1/6!  */
  cp = cp * p2 + 1.0 / 24.0;                  /*  1/4!  */
  cp = cp * p2 - 1.0 / 2.0;                   /* -1/2!  */
  cp = cp * p2 + 1.0;
  double s, c;
  switch (k) {
    case 0: s = sp; c = cp; break;
    case 1: s = cp; c = -sp; break;
    case 2: s = -sp; c = -cp; break;
    default: s = -cp; c = sp; break;
  }
  *s_out = s;
  *c_out = c;
}

/* Four standard normals from one generator call: Box-Muller on the word
 * pairs (w0, w1) and (w2, w3), radius sqrt(-2 ln u_a), angle 2 pi u_b.
 * Counter layout: (particle j, substep or time n, tag<<28 | blk<<20 | iter,
 * filter b); key = the 64-bit seed split low/high.  Component i of a state
 * uses blk = i/4 and the (i mod 4)-th normal. */
void orc_normals4(uint64_t seed, uint32_t tag, uint32_t blk, uint32_t iter, uint32_t j,
                  uint32_t n, uint32_t b, double z[4]) {
  uint32_t ctr[4] = {j, n, (tag << 28) | (blk << 20) | iter, b};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  for (int p = 0; p < 2; ++p) {
    double ua = orc_u01(w[2 * p]);
    double ub = orc_u01(w[2 * p + 1]);
    double r = sqrt(-2.0 * orc_ln(ua));
    double s, c;
    orc_sincos2pi(ub, &s, &c);
    z[2 * p] = r * c;
    z[2 * p + 1] = r * s;
  }
}

void orc_normals_bulk(uint64_t seed, uint32_t tag, uint32_t iter, uint32_t b, uint32_t n,
                      int64_t count, double* z) {
  for (int64_t j = 0; j < count; ++j) orc_normals4(seed, tag, 0, iter, (uint32_t)j, n, b, z + 4 * j);
}

/* one normal for component i of "particle" j at counter n */
static double normal_at(uint64_t seed, uint32_t tag, uint32_t iter, uint32_t j, uint32_t n,
                        uint32_t b, int i) {
  double z[4];
  orc_normals4(seed, tag, (uint32_t)(i / 4), iter, j, n, b, z);
  return z[i % 4];
}

/* ------------------------------------------------------------------------
 * Models.
 * ---------------------------------------------------------------------- */

/* Initial state x(t0) ~ p(X0 | theta) (Alg. 2, initialisation).
 * Windkessel: P_p(t0) ~ N(m0, s0^2) (Sec. 2.1.1, initial block: mean 90,
 * sd 15).  Lorenz '96: x_i(t0) ~ N(0, 1) (the workload's initial law). */
static void init_one(const orc_problem* P, const double* th, uint64_t seed, uint32_t tag,
                     uint32_t iter, uint32_t j, uint32_t b, double* x /* [d] */) {
  if (P->model == ORC_MODEL_WK) {
    double z = normal_at(seed, tag, iter, j, 0, b, 0);
    x[0] = th[4] + th[5] * z;
  } else {
    for (int i = 0; i < P->d; ++i) x[i] = normal_at(seed, tag, iter, j, 0, b, i);
  }
}

/* Lorenz '96 drift (eq. lorenz96-ode), cyclic indices:
 * f_i = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + F. */
void orc_l96_drift(int32_t d, const double* x, double F, double* out) {
  for (int i = 0; i < d; ++i) {
    int ip1 = (i + 1) % d, im1 = (i + d - 1) % d, im2 = (i + d - 2) % d;
    out[i] = ((x[ip1] - x[im2]) * x[im1] - x[i]) + F;
  }
}

/* The drift with a per-component forcing F_i. */
static void l96_drift_vec(int32_t d, const double* x, const double* F, double* out) {
  for (int i = 0; i < d; ++i) {
    int ip1 = (i + 1) % d, im1 = (i + d - 1) % d, im2 = (i + d - 2) % d;
    out[i] = ((x[ip1] - x[im2]) * x[im1] - x[i]) + F[i];
  }
}

/* One substep n (from t_{n-1} to t_n) of the transition.
 * Windkessel, exact solution of the two-element ODE over a step with the
 * flow held at F(t_{n-1}) (eq. 2-windkessel), plus an additive Gaussian
 * pressure perturbation of sd sigma_p:  p <- (a p + c q_{n-1}) + sigma_p z.
 * Lorenz '96: one classic RK4 step of size h of the drift, then the
 * Wiener increment sigma dW_i with dW_i ~ N(0, h) added after the step
 * (reading of eq. lorenz96-sde; the variance matches the paper's dW). */
static void substep_one(const orc_problem* P, const double* th, uint64_t seed, uint32_t tag,
                        uint32_t iter, uint32_t j, uint32_t b, int32_t n, double* x,
                        double* w /* scratch 6*d */) {
  if (P->model == ORC_MODEL_WK) {
    double z = normal_at(seed, tag, iter, j, (uint32_t)n, b, 0);
    double a = th[0], c = th[1], sp = th[3];
    x[0] = (a * x[0] + c * P->q[n - 1]) + sp * z;
    return;
  }
  int d = P->d;
  double F = th[0];
  double h = P->h, hh = 0.5 * P->h, h6 = P->h / 6.0;
  double sq = th[1] * sqrt(P->h);
  double *k1 = w, *k2 = w + d, *k3 = w + 2 * d, *k4 = w + 3 * d, *xt = w + 4 * d;
  if (P->model == ORC_MODEL_L96_STAGE) {
    /* The paper's form (Sec. 2.1.2): the SDE read as an ODE with the
     * forcing F + sigma dW_i/dt, dW_i = sqrt(h) z_i held over the step, so
     * component i's forcing is F_i = F + (sq z_i) / h; classic RK4 of that
     * ODE, nothing added after the step.  k2..k4 hold F_i meanwhile. */
    double* Fi = w + 5 * d;
    for (int i = 0; i < d; ++i)
      Fi[i] = F + (sq * normal_at(seed, tag, iter, j, (uint32_t)n, b, i)) / h;
    l96_drift_vec(d, x, Fi, k1);
    for (int i = 0; i < d; ++i) xt[i] = x[i] + hh * k1[i];
    l96_drift_vec(d, xt, Fi, k2);
    for (int i = 0; i < d; ++i) xt[i] = x[i] + hh * k2[i];
    l96_drift_vec(d, xt, Fi, k3);
    for (int i = 0; i < d; ++i) xt[i] = x[i] + h * k3[i];
    l96_drift_vec(d, xt, Fi, k4);
    for (int i = 0; i < d; ++i) x[i] = x[i] + h6 * ((k1[i] + k4[i]) + 2.0 * (k2[i] + k3[i]));
    return;
  }
  orc_l96_drift(d, x, F, k1);
  for (int i = 0; i < d; ++i) xt[i] = x[i] + hh * k1[i];
  orc_l96_drift(d, xt, F, k2);
  for (int i = 0; i < d; ++i) xt[i] = x[i] + hh * k2[i];
  orc_l96_drift(d, xt, F, k3);
  for (int i = 0; i < d; ++i) xt[i] = x[i] + h * k3[i];
  orc_l96_drift(d, xt, F, k4);
  for (int i = 0; i < d; ++i) {
    double xn = x[i] + h6 * ((k1[i] + k4[i]) + 2.0 * (k2[i] + k3[i]));
    double z = normal_at(seed, tag, iter, j, (uint32_t)n, b, i);
    x[i] = xn + sq * z;
  }
}

/* Observation log-density log p(y(t) | x(t), theta), Gaussian with sd
 * obs_sd on each observed component; the normalising constant is kept so
 * the estimator targets the same likelihood as the Kalman filter.
 * Windkessel (eq. 3-windkessel): mean P_p + Z F(t).  Lorenz '96: mean x_i. */
static double logdens_one(const orc_problem* P, const double* th, int32_t t, const double* x,
                          const double* y) {
  double inv_sd = 1.0 / P->obs_sd;
  double cst = -(double)P->n_obs * (log(P->obs_sd) + 0.5 * 1.8378770664093454836);
  double acc = 0.0;
  for (int o = 0; o < P->n_obs; ++o) {
    double mu;
    if (P->model == ORC_MODEL_WK)
      mu = x[0] + th[2] * P->q[(int64_t)t * P->K];
    else
      mu = x[P->obs_idx[o]];
    double e = (y[o] - mu) * inv_sd;
    acc = acc + e * e;
  }
  return -0.5 * acc + cst;
}

/* ------------------------------------------------------------------------
 * Filter pieces.
 * ---------------------------------------------------------------------- */

void orc_init(const orc_problem* P, const double* theta, int64_t N, uint32_t b, uint32_t iter,
              double* x) {
  double* xj = (double*)malloc(sizeof(double) * (size_t)P->d);
  for (int64_t j = 0; j < N; ++j) {
    init_one(P, theta, P->seed, ORC_TAG_INIT, iter, (uint32_t)j, b, xj);
    for (int i = 0; i < P->d; ++i) x[(int64_t)i * N + j] = xj[i];
  }
  free(xj);
}

/* Propagate each particle from t-1 to t: K substeps n = (t-1)K+1 .. tK
 * (Alg. 2, propagation). */
void orc_propagate(const orc_problem* P, const double* theta, int64_t N, uint32_t b,
                   uint32_t iter, int32_t t, const double* x_in, double* x_out) {
  int d = P->d;
  double* xj = (double*)malloc(sizeof(double) * (size_t)d);
  double* w = (double*)malloc(sizeof(double) * 6 * (size_t)d);
  for (int64_t j = 0; j < N; ++j) {
    for (int i = 0; i < d; ++i) xj[i] = x_in[(int64_t)i * N + j];
    for (int s = 1; s <= P->K; ++s)
      substep_one(P, theta, P->seed, ORC_TAG_NOISE, iter, (uint32_t)j, b,
                  (t - 1) * P->K + s, xj, w);
    for (int i = 0; i < d; ++i) x_out[(int64_t)i * N + j] = xj[i];
  }
  free(w);
  free(xj);
}

/* The same two steps for a subset of particles: column c of x holds
 * particle idx[c] of a filter, so it draws that particle's numbers.  Lets
 * the tests check single outputs of runs too large for the whole oracle. */
void orc_init_idx(const orc_problem* P, const double* theta, int64_t n, const int64_t* idx,
                  uint32_t b, uint32_t iter, double* x) {
  double* xj = (double*)malloc(sizeof(double) * (size_t)P->d);
  for (int64_t c = 0; c < n; ++c) {
    init_one(P, theta, P->seed, ORC_TAG_INIT, iter, (uint32_t)idx[c], b, xj);
    for (int i = 0; i < P->d; ++i) x[(int64_t)i * n + c] = xj[i];
  }
  free(xj);
}

void orc_propagate_idx(const orc_problem* P, const double* theta, int64_t n, const int64_t* idx,
                       uint32_t b, uint32_t iter, int32_t t, const double* x_in, double* x_out) {
  int d = P->d;
  double* xj = (double*)malloc(sizeof(double) * (size_t)d);
  double* w = (double*)malloc(sizeof(double) * 6 * (size_t)d);
  for (int64_t c = 0; c < n; ++c) {
    for (int i = 0; i < d; ++i) xj[i] = x_in[(int64_t)i * n + c];
    for (int s = 1; s <= P->K; ++s)
      substep_one(P, theta, P->seed, ORC_TAG_NOISE, iter, (uint32_t)idx[c], b,
                  (t - 1) * P->K + s, xj, w);
    for (int i = 0; i < d; ++i) x_out[(int64_t)i * n + c] = xj[i];
  }
  free(w);
  free(xj);
}

/* Log-weights lw_j = log p(y(t) | x_j(t), theta) (Alg. 2, weighting). */
void orc_weight(const orc_problem* P, const double* theta, int64_t N, int32_t t,
                const double* x, double* lw) {
  double* xj = (double*)malloc(sizeof(double) * (size_t)P->d);
  for (int64_t j = 0; j < N; ++j) {
    for (int i = 0; i < P->d; ++i) xj[i] = x[(int64_t)i * N + j];
    lw[j] = logdens_one(P, theta, t, xj, P->obs + (int64_t)(t - 1) * P->n_obs);
  }
  free(xj);
}

/* The single uniform of systematic resampling at time t for filter b. */
double orc_resample_u(uint64_t seed, int32_t t, uint32_t b, uint32_t iter) {
  uint32_t ctr[4] = {0u, (uint32_t)t, ((uint32_t)ORC_TAG_RESAMPLE << 28) | iter, b};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  return orc_u01(w[0]);
}

/* Likelihood increment, ESS and systematic resampling of one weight vector.
 *   M   = max_j lw_j (NaN log-weights count as zero weight)
 *   w_j = exp(lw_j - M),  W_j = sum_{i<=j} w_i (left to right),  S = W_{N-1}
 *   ell = M + ln S - ln N    (log of the time-t factor of the likelihood
 *                             estimate, Alg. 2 "marginal likelihood" line)
 *   ESS = S^2 / sum_j w_j^2
 * Systematic resampling (Sec. 3.3 names it among the collective resamplers;
 * Kitagawa 1996): one uniform u, strata (u+k)/N, k = 0..N-1, and
 *   a_k = min { j : N W_j > (u + k) S }
 * i.e. stratum k falls in particle j's half-open cell [W_{j-1}, W_j); a
 * particle of zero weight has an empty cell.  If rounding leaves no such j,
 * a_k is the last particle of positive weight.  Returns ORC_NUMERIC (and
 * ell = -inf, identity ancestors) when no weight is positive and finite. */
int32_t orc_reduce_resample(int64_t N, const double* lw, double u, double* ell, double* ess,
                            int32_t* a) {
  double M = -INFINITY;
  for (int64_t j = 0; j < N; ++j)
    if (lw[j] > M) M = lw[j];
  if (!(M > -INFINITY) || !(M < INFINITY)) {
    *ell = -INFINITY;
    *ess = 0.0;
    for (int64_t k = 0; k < N; ++k) a[k] = (int32_t)k;
    return ORC_NUMERIC;
  }
  double* W = (double*)malloc(sizeof(double) * (size_t)N);
  double acc = 0.0, acc2 = 0.0;
  int64_t jstar = -1;
  for (int64_t j = 0; j < N; ++j) {
    double w = (lw[j] == lw[j]) ? exp(lw[j] - M) : 0.0;
    acc = acc + w;
    acc2 = acc2 + w * w;
    W[j] = acc;
    if (w > 0.0) jstar = j;
  }
  double S = acc;
  *ell = (M + log(S)) - log((double)N);
  *ess = (S * S) / acc2;
  double Nd = (double)N;
  int64_t j = 0;
  for (int64_t k = 0; k < N; ++k) {
    double thr = (u + (double)k) * S;
    while (j < N && !(Nd * W[j] > thr)) ++j;
    a[k] = (int32_t)(j < N ? j : jstar);
  }
  free(W);
  return ORC_OK;
}

/* x'_k = x_{a_k}: offspring take their ancestor's state. */
void orc_gather(int32_t d, int64_t N, const double* x, const int32_t* a, double* x_out) {
  for (int i = 0; i < d; ++i)
    for (int64_t k = 0; k < N; ++k) x_out[(int64_t)i * N + k] = x[(int64_t)i * N + a[k]];
}

/* Alg. 2 over t = 1..T_run from a fresh initialisation.  Order within each
 * time: propagate, weight, accumulate the likelihood factor, resample and
 * gather (the paper draws ancestors at the top of the next iteration; the
 * draw at t = 1 from uniform initial weights is skipped as it changes
 * nothing in law — a reading).  The marginal log-likelihood is the running
 * sum of ell_t. */
int32_t orc_pf_run(const orc_problem* P, const double* theta, int64_t N, uint32_t b,
                   uint32_t iter, int32_t T_run, double* ell, double* ess, double* loglik,
                   int32_t* anc_trace, double* lw_trace, double* x_final,
                   const double* u_override) {
  int d = P->d;
  double* x = (double*)malloc(sizeof(double) * (size_t)d * (size_t)N);
  double* xp = (double*)malloc(sizeof(double) * (size_t)d * (size_t)N);
  double* lw = (double*)malloc(sizeof(double) * (size_t)N);
  int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int32_t status = ORC_OK;
  double ll = 0.0;
  orc_init(P, theta, N, b, iter, x);
  for (int32_t t = 1; t <= T_run; ++t) {
    orc_propagate(P, theta, N, b, iter, t, x, xp);
    orc_weight(P, theta, N, t, xp, lw);
    if (lw_trace) memcpy(lw_trace + (int64_t)(t - 1) * N, lw, sizeof(double) * (size_t)N);
    double u = u_override ? u_override[t - 1] : orc_resample_u(P->seed, t, b, iter);
    double e, s;
    int32_t st = orc_reduce_resample(N, lw, u, &e, &s, a);
    if (st != ORC_OK) status = st;
    ll = ll + e;
    ell[t - 1] = e;
    ess[t - 1] = s;
    if (anc_trace) memcpy(anc_trace + (int64_t)(t - 1) * N, a, sizeof(int32_t) * (size_t)N);
    orc_gather(d, N, xp, a, x);
  }
  *loglik = (status == ORC_OK) ? ll : -INFINITY;
  if (x_final) memcpy(x_final, x, sizeof(double) * (size_t)d * (size_t)N);
  free(a);
  free(lw);
  free(xp);
  free(x);
  return status;
}

/* Exact marginal likelihood of the windkessel by the Kalman filter (Alg. 1
 * with N_x = N_y = 1, where every Cholesky factor is a square root): per
 * substep, mean m <- a m + c q_{n-1} and variance V <- a^2 V + sigma_p^2;
 * at each observation, innovation v = y - (m + Z q), innovation variance
 * S = V + obs_sd^2, ell = -(ln(2 pi S) + v^2 / S)/2, then condition. */
double orc_kf_wk(const orc_problem* P, const double* theta, double* ell) {
  double a = theta[0], c = theta[1], Z = theta[2], sp = theta[3];
  double m = theta[4], V = theta[5] * theta[5];
  double R = P->obs_sd * P->obs_sd;
  double ll = 0.0;
  for (int32_t t = 1; t <= P->T; ++t) {
    for (int s = 1; s <= P->K; ++s) {
      int64_t n = (int64_t)(t - 1) * P->K + s;
      m = a * m + c * P->q[n - 1];
      V = a * a * V + sp * sp;
    }
    double qn = P->q[(int64_t)t * P->K];
    double v = P->obs[t - 1] - (m + Z * qn);
    double S = V + R;
    double e = -0.5 * (log(2.0 * 3.14159265358979323846 * S) + v * v / S);
    double Kg = V / S;
    m = m + Kg * v;
    V = (1.0 - Kg) * V;
    ell[t - 1] = e;
    ll += e;
  }
  return ll;
}

/* Synthetic truth and observations from the same model with the data seed:
 * initial state and state noise under tag DATA (particle 0, filter 0),
 * observation noise under tag OBS at counter n = t, blk = o/4. */
void orc_simulate(const orc_problem* P, const double* theta, uint64_t data_seed,
                  double* x_traj, double* obs) {
  int d = P->d;
  double* x = (double*)malloc(sizeof(double) * (size_t)d);
  double* w = (double*)malloc(sizeof(double) * 6 * (size_t)d);
  init_one(P, theta, data_seed, ORC_TAG_DATA, 0, 0, 0, x);
  memcpy(x_traj, x, sizeof(double) * (size_t)d);
  for (int32_t t = 1; t <= P->T; ++t) {
    for (int s = 1; s <= P->K; ++s)
      substep_one(P, theta, data_seed, ORC_TAG_DATA, 0, 0, 0, (t - 1) * P->K + s, x, w);
    memcpy(x_traj + (int64_t)t * d, x, sizeof(double) * (size_t)d);
    for (int o = 0; o < P->n_obs; ++o) {
      double mu = (P->model == ORC_MODEL_WK) ? x[0] + theta[2] * P->q[(int64_t)t * P->K]
                                             : x[P->obs_idx[o]];
      double z = normal_at(data_seed, ORC_TAG_OBS, 0, 0, (uint32_t)t, 0, o);
      obs[(int64_t)(t - 1) * P->n_obs + o] = mu + P->obs_sd * z;
    }
  }
  free(w);
  free(x);
}

/* Marginal Metropolis-Hastings (Alg. 3, eq. mh) on theta = log F of the
 * Lorenz '96 model with sigma fixed, one chain per filter index b.
 * Proposal: symmetric Gaussian random walk theta' = theta + step_sd z.
 * Prior: F ~ U(f_lo, f_hi); in log F coordinates its density carries the
 * Jacobian F, so the acceptance ratio is
 *     l' F' 1[f_lo <= F' <= f_hi] / (l F),
 * and a move is accepted iff ln(alpha) <= (ll' - ll) + (theta' - theta)
 * (ties accept, as in Alg. 3).  Iteration i (1-based) runs its filter with
 * generator iteration field i; the initial filter uses 0.  The random
 * numbers of this layer (z, alpha, the initial theta) are inputs. */
int32_t orc_pmmh(const orc_problem* P, int64_t N, int32_t chain0, int32_t n_chains,
                 int32_t n_chains_total, int32_t iters, const double* log_f0,
                 const double* z, const double* alpha, double step_sd, double f_lo,
                 double f_hi, double sigma, double* log_f_trace, double* ll_trace,
                 int32_t* accepts) {
  double* ell = (double*)malloc(sizeof(double) * (size_t)P->T);
  double* ess = (double*)malloc(sizeof(double) * (size_t)P->T);
  for (int32_t cc = 0; cc < n_chains; ++cc) {
    int32_t c = chain0 + cc;
    double th = log_f0[c];
    double theta[2] = {exp(th), sigma};
    double ll;
    orc_pf_run(P, theta, N, (uint32_t)c, 0, P->T, ell, ess, &ll, NULL, NULL, NULL, NULL);
    int32_t acc = 0;
    for (int32_t i = 0; i < iters; ++i) {
      double thp = th + step_sd * z[(int64_t)i * n_chains_total + c];
      double Fp = exp(thp);
      if (Fp >= f_lo && Fp <= f_hi) {
        double thetap[2] = {Fp, sigma};
        double llp;
        orc_pf_run(P, thetap, N, (uint32_t)c, (uint32_t)(i + 1), P->T, ell, ess, &llp, NULL,
                   NULL, NULL, NULL);
        double lhs = log(alpha[(int64_t)i * n_chains_total + c]);
        if (lhs <= (llp - ll) + (thp - th)) {
          th = thp;
          ll = llp;
          ++acc;
        }
      }
      log_f_trace[(int64_t)i * n_chains + cc] = th;
      ll_trace[(int64_t)i * n_chains + cc] = ll;
    }
    accepts[cc] = acc;
  }
  free(ess);
  free(ell);
  return ORC_OK;
}

/* Whole-filter copy used when a theta-particle takes another's filter (the
 * attached state sample travels with the theta-particle, Sec. 3.2.2).  The
 * source's N_s equally weighted particles are re-represented by the
 * destination's N_d particles with systematic selection on equal weights:
 * destination particle k takes source particle floor((k + u) N_s / N_d),
 * u = w 2^-32 for a 32-bit word w.  Evaluated exactly in integers as
 * ((k 2^32 + w) N_s) div (N_d 2^32), which fits 64 bits for N <= 2^13.  For
 * N_s = N_d this is the identity. */
int64_t orc_copy_index(int64_t k, int64_t n_src, int64_t n_dst, uint32_t w) {
  uint64_t num = (((uint64_t)k << 32) | (uint64_t)w) * (uint64_t)n_src;
  return (int64_t)(num / ((uint64_t)n_dst << 32));
}

/* SMC over the parameters with a particle filter attached to every
 * theta-particle: Sec. 3.2.2, Alg. 4 (SMC^2 when the attached filter is the
 * bootstrap particle filter of Alg. 2).  Per observation time i = 1..T_run,
 * in the algorithm's order:
 *   1. theta-ancestors from the theta-weights v(t_{i-1}) (systematic, as for
 *      the state particles; the algorithm writes multinomial — a reading);
 *      at i = 1 the weights are uniform and the draw is the identity;
 *   2. each theta-particle takes its ancestor's parameters, likelihood and
 *      filter (orc_copy_index for unequal particle counts);
 *   3. rejuvenation by one marginal Metropolis-Hastings step (Alg. 3, eq.
 *      mh): a Gaussian random walk theta' = theta + step_sd z on the
 *      parameters with step_sd > 0, a uniform prior box [lo, hi] on those
 *      parameters; outside the box the move is rejected without a filter
 *      run; inside, a fresh filter for theta' over t_{0:i-1} (generator
 *      iteration field i, filter index j) gives l' and x'; the move is
 *      accepted iff log_alpha <= l' - l (symmetric proposal and flat prior
 *      cancel; ties accept), and then theta, l and the filter become the
 *      proposal's;
 *   4. the attached filter advances over t_{i-1:i} (iteration field 0,
 *      filter index j): its likelihood increment ell_i^j is the new
 *      theta-log-weight v^j(t_i) and l^j += ell_i^j.
 * After each time the theta-weights' ESS is recorded and the evidence
 * estimate accumulates ln(sum_j exp v^j(t_i)) - ln B (the theta-weights are
 * uniform after every resampling) — the evidence is not in the paper; a
 * reading.  The random numbers of this layer are inputs: z [T_run][B][n_theta],
 * log_alpha [T_run][B], u_theta [T_run] (entry i-1 for time i's
 * theta-resampling), w_copy [T_run][B].  Filter j's particles are stored as
 * one structure-of-arrays block; x_final is [d][sum N] with filter j at
 * columns off_j..off_j+N_j-1.  Returns ORC_NUMERIC (and evidence -inf) if
 * every theta-weight of some time is zero. */
int32_t orc_smc2(const orc_problem* P, int32_t B, const int64_t* n_particles, int32_t n_theta,
                 const double* theta0, int32_t T_run, const double* step_sd, const double* lo,
                 const double* hi, const double* z, const double* log_alpha,
                 const double* u_theta, const uint32_t* w_copy, double* theta_out,
                 double* logw_out, double* loglik_out, int32_t* accepts, double* ess_theta,
                 double* log_evidence, int32_t* anc_trace, int32_t* acc_trace,
                 double* logw_trace, double* theta_trace, double* x_final) {
  const int d = P->d;
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)B + 1));
  int64_t nmax = 1;
  off[0] = 0;
  for (int32_t j = 0; j < B; ++j) {
    off[j + 1] = off[j] + n_particles[j];
    if (n_particles[j] > nmax) nmax = n_particles[j];
  }
  const int64_t ntot = off[B];
  double* th = (double*)malloc(sizeof(double) * (size_t)B * n_theta);
  double* th_new = (double*)malloc(sizeof(double) * (size_t)B * n_theta);
  double* thp = (double*)malloc(sizeof(double) * (size_t)n_theta);
  double* x = (double*)malloc(sizeof(double) * (size_t)d * (size_t)ntot);
  double* x_new = (double*)malloc(sizeof(double) * (size_t)d * (size_t)ntot);
  double* xp = (double*)malloc(sizeof(double) * (size_t)d * (size_t)nmax);
  double* xprop = (double*)malloc(sizeof(double) * (size_t)d * (size_t)nmax);
  double* lw = (double*)malloc(sizeof(double) * (size_t)nmax);
  int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)nmax);
  double* scratch = (double*)malloc(sizeof(double) * ((size_t)T_run + 1) * 2);
  double* l = (double*)malloc(sizeof(double) * (size_t)B);
  double* l_new = (double*)malloc(sizeof(double) * (size_t)B);
  double* v = (double*)malloc(sizeof(double) * (size_t)B);
  int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)B);
  int32_t status = ORC_OK;
  double evidence = 0.0;

  memcpy(th, theta0, sizeof(double) * (size_t)B * n_theta);
  for (int32_t j = 0; j < B; ++j) {
    orc_init(P, th + (size_t)j * n_theta, n_particles[j], (uint32_t)j, 0, x + d * off[j]);
    l[j] = 0.0;
    v[j] = 0.0;
    a[j] = j;
    accepts[j] = 0;
  }
  for (int32_t i = 1; i <= T_run && status == ORC_OK; ++i) {
    /* 2. take the ancestors' parameters, likelihoods and filters */
    for (int32_t j = 0; j < B; ++j) {
      const int32_t s = a[j];
      const int64_t ns = n_particles[s], nd = n_particles[j];
      memcpy(th_new + (size_t)j * n_theta, th + (size_t)s * n_theta, sizeof(double) * n_theta);
      l_new[j] = l[s];
      const uint32_t w = w_copy[(int64_t)(i - 1) * B + j];
      for (int64_t k = 0; k < nd; ++k) {
        const int64_t p = orc_copy_index(k, ns, nd, w);
        for (int c = 0; c < d; ++c) x_new[d * off[j] + c * nd + k] = x[d * off[s] + c * ns + p];
      }
      if (anc_trace) anc_trace[(int64_t)(i - 1) * B + j] = s;
    }
    /* 3. rejuvenate: one marginal Metropolis-Hastings step per theta-particle */
    for (int32_t j = 0; j < B; ++j) {
      const int64_t nd = n_particles[j];
      int inside = 1;
      for (int32_t p = 0; p < n_theta; ++p) {
        const double cur = th_new[(size_t)j * n_theta + p];
        if (step_sd[p] != 0.0) {
          const double step = step_sd[p] * z[((int64_t)(i - 1) * B + j) * n_theta + p];
          thp[p] = cur + step;
          if (!(thp[p] >= lo[p] && thp[p] <= hi[p])) inside = 0;
        } else {
          thp[p] = cur;
        }
      }
      int32_t acc = 0;
      if (inside) {
        double lp;
        orc_pf_run(P, thp, nd, (uint32_t)j, (uint32_t)i, i - 1, scratch, scratch + T_run + 1,
                   &lp, NULL, NULL, xprop, NULL);
        if (log_alpha[(int64_t)(i - 1) * B + j] <= lp - l_new[j]) {
          memcpy(th_new + (size_t)j * n_theta, thp, sizeof(double) * n_theta);
          l_new[j] = lp;
          memcpy(x_new + d * off[j], xprop, sizeof(double) * (size_t)d * (size_t)nd);
          acc = 1;
          accepts[j] += 1;
        }
      }
      if (acc_trace) acc_trace[(int64_t)(i - 1) * B + j] = acc;
    }
    /* 4. advance every attached filter over t_{i-1:i} */
    for (int32_t j = 0; j < B; ++j) {
      const int64_t nd = n_particles[j];
      const double* tj = th_new + (size_t)j * n_theta;
      orc_propagate(P, tj, nd, (uint32_t)j, 0, i, x_new + d * off[j], xp);
      orc_weight(P, tj, nd, i, xp, lw);
      double e, s;
      orc_reduce_resample(nd, lw, orc_resample_u(P->seed, i, (uint32_t)j, 0), &e, &s, anc);
      orc_gather(d, nd, xp, anc, x + d * off[j]);
      v[j] = e;
      l[j] = l_new[j] + e;
      if (logw_trace) logw_trace[(int64_t)(i - 1) * B + j] = e;
    }
    memcpy(th, th_new, sizeof(double) * (size_t)B * n_theta);
    if (theta_trace)
      memcpy(theta_trace + (int64_t)(i - 1) * B * n_theta, th,
             sizeof(double) * (size_t)B * n_theta);
    /* theta-weights: ESS, evidence factor and the next time's ancestors */
    double e, s;
    const double u = (i < T_run) ? u_theta[i] : 0.5;
    status = orc_reduce_resample(B, v, u, &e, &s, a);
    evidence = evidence + e;
    ess_theta[i - 1] = s;
  }
  *log_evidence = (status == ORC_OK) ? evidence : -INFINITY;
  memcpy(theta_out, th, sizeof(double) * (size_t)B * n_theta);
  for (int32_t j = 0; j < B; ++j) {
    logw_out[j] = v[j];
    loglik_out[j] = l[j];
    if (x_final)
      for (int c = 0; c < d; ++c)
        memcpy(x_final + (int64_t)c * ntot + off[j], x + d * off[j] + c * n_particles[j],
               sizeof(double) * (size_t)n_particles[j]);
  }
  free(a);
  free(v);
  free(l_new);
  free(l);
  free(scratch);
  free(anc);
  free(lw);
  free(xprop);
  free(xp);
  free(x_new);
  free(x);
  free(thp);
  free(th_new);
  free(th);
  free(off);
  return status;
}

/* Index of the final particle of the state sample (Alg. 2, last lines:
 * j ~ Multinomial(w(t_s))).  The time-s systematic ancestors a_k
 * (k = 0..N-1) invert the cumulative weights at (u + k)/N; with k drawn
 * uniformly on 0..N-1, independent of u, that point is uniform on [0, 1), so
 * a_k is one draw from w(t_s).  k = floor(w N 2^-32) for the first word w of
 * the generator at counter (0, s, tag PATH | iteration, b), exact in
 * integers. */
int64_t orc_path_slot(uint64_t seed, int32_t s, uint32_t b, uint32_t iter, int64_t N) {
  uint32_t ctr[4] = {0u, (uint32_t)s, ((uint32_t)ORC_TAG_PATH << 28) | iter, b};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  return (int64_t)(((uint64_t)w[0] * (uint64_t)N) >> 32);
}

/* Alg. 2 over t = 1..T_run, keeping every time's propagated (weighted)
 * particles x(t_i) and ancestors, then the single state sample: the final
 * particle j is the time-T_run ancestor at orc_path_slot, and for
 * i = T_run..1, j <- a^j(t_i), the ancestor that particle j of time t_i was
 * propagated from (the time-(i-1) systematic ancestors; identity at i = 1,
 * whose t_0 draw is skipped), x'(t_{i-1}) = x^j(t_{i-1}).  path [T_run+1][d],
 * idx [T_run+1] (particle indices per time).  Returns the filter status. */
int32_t orc_pf_path(const orc_problem* P, const double* theta, int64_t N, uint32_t b,
                    uint32_t iter, int32_t T_run, double* loglik, double* path, int64_t* idx) {
  const int d = P->d;
  const size_t xs = (size_t)d * (size_t)N;
  double* xh = (double*)malloc(sizeof(double) * xs * ((size_t)T_run + 1));
  int32_t* ah = (int32_t*)malloc(sizeof(int32_t) * (size_t)N * ((size_t)T_run + 1));
  double* x = (double*)malloc(sizeof(double) * xs);
  double* lw = (double*)malloc(sizeof(double) * (size_t)N);
  int32_t status = ORC_OK;
  double ll = 0.0;
  orc_init(P, theta, N, b, iter, xh);  /* time t_0 */
  memcpy(x, xh, sizeof(double) * xs);
  for (int32_t t = 1; t <= T_run; ++t) {
    double* xt = xh + (size_t)t * xs;
    orc_propagate(P, theta, N, b, iter, t, x, xt);
    orc_weight(P, theta, N, t, xt, lw);
    double e, s;
    int32_t st = orc_reduce_resample(N, lw, orc_resample_u(P->seed, t, b, iter), &e, &s,
                                     ah + (size_t)t * N);
    if (st != ORC_OK) status = st;
    ll = ll + e;
    orc_gather(d, N, xt, ah + (size_t)t * N, x);
  }
  *loglik = (status == ORC_OK) ? ll : -INFINITY;
  /* the single state sample, traced back through the ancestry */
  const int64_t k = orc_path_slot(P->seed, T_run, b, iter, N);
  int64_t j = (T_run >= 1) ? ah[(size_t)T_run * N + k] : k;
  idx[T_run] = j;
  for (int32_t i = T_run; i >= 1; --i) {
    if (i >= 2) j = ah[(size_t)(i - 1) * N + j];
    idx[i - 1] = j;
  }
  for (int32_t i = 0; i <= T_run; ++i)
    for (int c = 0; c < d; ++c)
      path[(size_t)i * d + c] = xh[(size_t)i * xs + (size_t)c * N + idx[i]];
  free(lw);
  free(x);
  free(ah);
  free(xh);
  return status;
}

/* ------------------------------------------------------------------------
 * Resampling variants (Sec. 3.3 names multinomial, systematic and
 * stratified resampling and points to resamplers that avoid the collective
 * over the weights) and resampling triggered by the ESS.
 * ------------------------------------------------------------------------ */

/* Stratified offsets: u_k for stratum k is the uniform of word k mod 4 of the
 * generator at counter (k div 4, t, tag RESAMPLE | block 1 | iteration, b). */
double orc_strat_u(uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int64_t k) {
  uint32_t ctr[4] = {(uint32_t)(k >> 2), (uint32_t)t,
                     ((uint32_t)ORC_TAG_RESAMPLE << 28) | (1u << 20) | iter, b};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  return orc_u01(w[k & 3]);
}

/* The pair (j', u) of Metropolis step s (1-based) for output k: words 2r and
 * 2r+1, r = (s-1) mod 2, of the generator at counter (k, t, tag RESAMPLE |
 * block 2 + (s-1) div 2 | iteration, b); j' = floor(w N 2^-32), u the
 * uniform of the second word. */
static void metro_pair(uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int64_t k,
                       int32_t s, int64_t N, int64_t* jp, double* u) {
  const uint32_t blk = 2u + (uint32_t)((s - 1) >> 1);
  uint32_t ctr[4] = {(uint32_t)k, (uint32_t)t,
                     ((uint32_t)ORC_TAG_RESAMPLE << 28) | (blk << 20) | iter, b};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  const int r = (s - 1) & 1;
  *jp = (int64_t)(((uint64_t)w[2 * r] * (uint64_t)N) >> 32);
  *u = orc_u01(w[2 * r + 1]);
}

/* M, the scan W of exp(lw - M) (NaN log-weights weigh 0), S = W_{N-1},
 * S2 and the last positive index; returns 0 if no weight is positive. */
static int weights_scan(int64_t N, const double* lw, double* M_out, double* W, double* S_out,
                        double* S2_out, int64_t* jstar_out) {
  double M = -INFINITY;
  for (int64_t j = 0; j < N; ++j)
    if (lw[j] > M) M = lw[j];
  if (!(M > -INFINITY) || !(M < INFINITY)) return 0;
  double acc = 0.0, acc2 = 0.0;
  int64_t jstar = -1;
  for (int64_t j = 0; j < N; ++j) {
    double w = (lw[j] == lw[j]) ? exp(lw[j] - M) : 0.0;
    acc = acc + w;
    acc2 = acc2 + w * w;
    W[j] = acc;
    if (w > 0.0) jstar = j;
  }
  *M_out = M;
  *S_out = acc;
  *S2_out = acc2;
  *jstar_out = jstar;
  return 1;
}

/* Stratified resampling: a_k = min{ j : N W_j > (u_k + k) S } with the
 * per-stratum offsets of orc_strat_u; rounding overflow goes to the last
 * positive weight, as for systematic resampling. */
void orc_stratified_ancestors(int64_t N, const double* W, double S, int64_t jstar,
                              uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int32_t* a) {
  const double Nd = (double)N;
  int64_t j = 0;
  for (int64_t k = 0; k < N; ++k) {
    const double thr = (orc_strat_u(seed, t, b, iter, k) + (double)k) * S;
    while (j < N && !(Nd * W[j] > thr)) ++j;
    a[k] = (int32_t)(j < N ? j : jstar);
  }
}

/* Metropolis resampling (a resampler without the collective): output k
 * starts at particle k and takes `steps` Metropolis moves with uniform
 * proposals j', accepted iff ln u <= lw_j' - lw_j (own ln, so both sides
 * decide alike; a NaN log-weight counts as -inf).  Unsorted; tends to
 * multinomial resampling as steps grows. */
void orc_metropolis_ancestors(int64_t N, const double* lw, int32_t steps, uint64_t seed,
                              int32_t t, uint32_t b, uint32_t iter, int32_t* a) {
  for (int64_t k = 0; k < N; ++k) {
    int64_t j = k;
    double lj = (lw[j] == lw[j]) ? lw[j] : -INFINITY;
    for (int32_t s = 1; s <= steps; ++s) {
      int64_t jp;
      double u;
      metro_pair(seed, t, b, iter, k, s, N, &jp, &u);
      const double lp = (lw[jp] == lw[jp]) ? lw[jp] : -INFINITY;
      if (orc_ln(u) <= lp - lj) {
        j = jp;
        lj = lp;
      }
    }
    a[k] = (int32_t)j;
  }
}

/* The candidate j and uniform u of attempt r (0-based) of output k of the
 * rejection resampler: attempts 2p and 2p+1 take words (0, 1) and (2, 3)
 * of the generator at counter (k, t + (p div 256) 2^20, tag REJECT | block
 * p mod 256 | iteration, b) (t < 2^20); the candidate is floor(w N 2^-32)
 * of the first word, except at r = 0, where it is k itself; u is the
 * uniform of the second word. */
void orc_reject_pair(uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int64_t k, int64_t r,
                     int64_t N, int64_t* j, double* u) {
  const uint64_t p = (uint64_t)r >> 1;
  uint32_t ctr[4] = {(uint32_t)k, (uint32_t)t + (uint32_t)((p >> 8) << 20),
                     ((uint32_t)ORC_TAG_REJECT << 28) | ((uint32_t)(p & 255) << 20) | iter, b};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  const int h = (int)(r & 1);
  *j = (r == 0) ? k : (int64_t)(((uint64_t)w[2 * h] * (uint64_t)N) >> 32);
  *u = orc_u01(w[2 * h + 1]);
}

/* Rejection resampling (a resampler that needs the maximum weight but no
 * scan; of the family Sec. 3.3 cites as avoiding the collective): output k
 * tries candidates j (k first, then uniform draws over 0..N-1) until one is
 * accepted, attempt r accepting iff ln u_r <= lw_j - M with M the largest
 * log-weight (own ln, so both sides decide alike; a NaN log-weight counts
 * as -inf).  Every attempt after the first is an independent draw from
 * the normalised weights conditioned on acceptance, so a_k = k with
 * probability w_k/w_max + (1 - w_k/w_max) W_k and a_k = j != k with
 * probability (1 - w_k/w_max) W_j: each output's offspring expectations
 * are N W_j.  After ORC_REJECT_MAX_ATTEMPTS attempts without acceptance
 * (probability at most (1 - 1/N)^(2^21)) the output keeps k.  Unsorted. */
void orc_rejection_ancestors(int64_t N, const double* lw, uint64_t seed, int32_t t, uint32_t b,
                             uint32_t iter, int32_t* a) {
  double M = -INFINITY;
  for (int64_t j = 0; j < N; ++j)
    if (lw[j] > M) M = lw[j];
  for (int64_t k = 0; k < N; ++k) {
    int64_t out = k;
    for (int64_t r = 0; r < ORC_REJECT_MAX_ATTEMPTS; ++r) {
      int64_t j;
      double u;
      orc_reject_pair(seed, t, b, iter, k, r, N, &j, &u);
      const double lj = (lw[j] == lw[j]) ? lw[j] : -INFINITY;
      if (orc_ln(u) <= lj - M) {
        out = j;
        break;
      }
    }
    a[k] = (int32_t)out;
  }
}

/* Multinomial resampling, as Alg. 2 writes it: N independent uniforms,
 * u_k = the uniform of word k mod 4 of the generator at (k div 4, t, tag
 * MULTI | iteration, b), and a_k = min{ j : W_j > u_k S } (the inverse of
 * the cumulative weights; rounding overflow to the last positive weight).
 * Unsorted. */
double orc_multi_u(uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int64_t k) {
  uint32_t ctr[4] = {(uint32_t)(k >> 2), (uint32_t)t, ((uint32_t)ORC_TAG_MULTI << 28) | iter, b};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  return orc_u01(w[k & 3]);
}

void orc_multinomial_ancestors(int64_t N, const double* W, double S, int64_t jstar,
                               uint64_t seed, int32_t t, uint32_t b, uint32_t iter, int32_t* a) {
  for (int64_t k = 0; k < N; ++k) {
    const double thr = orc_multi_u(seed, t, b, iter, k) * S;
    int64_t j = 0;
    while (j < N && !(W[j] > thr)) ++j;
    a[k] = (int32_t)(j < N ? j : jstar);
  }
}

/* Alg. 2 with a choice of resampler (0 systematic, 1 stratified, 2
 * Metropolis with `steps` moves, 3 multinomial, 4 rejection) and resampling only when ESS < ess_frac N
 * (ess_frac = +inf: every time).  Without resampling the log-weights carry
 * over: the time-t weights are carry + lw_t, the likelihood factor is
 * ln sum exp(carry + lw_t) - ln sum exp(carry) (ln N after a resampling),
 * and the ancestors are the identity.  lw_trace holds the carried
 * log-weights; res_trace (optional) 1 where the time resampled. */
int32_t orc_pf_run_ex(const orc_problem* P, const double* theta, int64_t N, uint32_t b,
                      uint32_t iter, int32_t T_run, int32_t resampler, int32_t steps,
                      double ess_frac, double* ell, double* ess, double* loglik,
                      int32_t* anc_trace, double* lw_trace, int32_t* res_trace,
                      double* x_final) {
  const int d = P->d;
  double* x = (double*)malloc(sizeof(double) * (size_t)d * (size_t)N);
  double* xp = (double*)malloc(sizeof(double) * (size_t)d * (size_t)N);
  double* lw = (double*)malloc(sizeof(double) * (size_t)N);
  double* carry = (double*)malloc(sizeof(double) * (size_t)N);
  double* W = (double*)malloc(sizeof(double) * (size_t)N);
  int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int32_t status = ORC_OK;
  double ll = 0.0, L_prev = log((double)N);
  orc_init(P, theta, N, b, iter, x);
  for (int64_t j = 0; j < N; ++j) carry[j] = 0.0;
  for (int32_t t = 1; t <= T_run; ++t) {
    orc_propagate(P, theta, N, b, iter, t, x, xp);
    orc_weight(P, theta, N, t, xp, lw);
    for (int64_t j = 0; j < N; ++j) lw[j] = carry[j] + lw[j];
    if (lw_trace) memcpy(lw_trace + (int64_t)(t - 1) * N, lw, sizeof(double) * (size_t)N);
    double M, S, S2;
    int64_t jstar;
    int resample = 1;
    if (!weights_scan(N, lw, &M, W, &S, &S2, &jstar)) {
      /* no positive weight: identity ancestors and uniform weights after it */
      status = ORC_NUMERIC;
      ell[t - 1] = -INFINITY;
      ess[t - 1] = 0.0;
      for (int64_t k = 0; k < N; ++k) a[k] = (int32_t)k;
      L_prev = log((double)N);
    } else {
      const double L = M + log(S);
      ell[t - 1] = L - L_prev;
      ess[t - 1] = (S * S) / S2;
      resample = ess[t - 1] < ess_frac * (double)N;
      if (!resample) {
        for (int64_t k = 0; k < N; ++k) a[k] = (int32_t)k;
        L_prev = L;
      } else {
        L_prev = log((double)N);
        if (resampler == 1) {
          orc_stratified_ancestors(N, W, S, jstar, P->seed, t, b, iter, a);
        } else if (resampler == 2) {
          orc_metropolis_ancestors(N, lw, steps, P->seed, t, b, iter, a);
        } else if (resampler == 3) {
          orc_multinomial_ancestors(N, W, S, jstar, P->seed, t, b, iter, a);
        } else if (resampler == 4) {
          orc_rejection_ancestors(N, lw, P->seed, t, b, iter, a);
        } else {
          const double u = orc_resample_u(P->seed, t, b, iter), Nd = (double)N;
          int64_t j = 0;
          for (int64_t k = 0; k < N; ++k) {
            const double thr = (u + (double)k) * S;
            while (j < N && !(Nd * W[j] > thr)) ++j;
            a[k] = (int32_t)(j < N ? j : jstar);
          }
        }
      }
    }
    ll = ll + ell[t - 1];
    if (res_trace) res_trace[t - 1] = resample;
    if (anc_trace) memcpy(anc_trace + (int64_t)(t - 1) * N, a, sizeof(int32_t) * (size_t)N);
    orc_gather(d, N, xp, a, x);
    for (int64_t j = 0; j < N; ++j) carry[j] = resample ? 0.0 : lw[j];
  }
  *loglik = (status == ORC_OK) ? ll : -INFINITY;
  if (x_final) memcpy(x_final, x, sizeof(double) * (size_t)d * (size_t)N);
  free(a);
  free(W);
  free(carry);
  free(lw);
  free(xp);
  free(x);
  return status;
}

/* One observation interval of the windkessel Kalman filter (the step of
 * orc_kf_wk for time t): K predictions m <- a m + c q_{n-1},
 * V <- a^2 V + sigma_p^2, then the correction with y_t; returns ell_t and
 * updates (m, V). */
double orc_kf_wk_interval(const orc_problem* P, const double* theta, int32_t t, double* m,
                          double* V) {
  double a = theta[0], c = theta[1], Z = theta[2], sp = theta[3];
  double R = P->obs_sd * P->obs_sd;
  double mm = *m, VV = *V;
  for (int s = 1; s <= P->K; ++s) {
    int64_t n = (int64_t)(t - 1) * P->K + s;
    mm = a * mm + c * P->q[n - 1];
    VV = a * a * VV + sp * sp;
  }
  double qn = P->q[(int64_t)t * P->K];
  double v = P->obs[t - 1] - (mm + Z * qn);
  double S = VV + R;
  double e = -0.5 * (log(2.0 * 3.14159265358979323846 * S) + v * v / S);
  double Kg = VV / S;
  *m = mm + Kg * v;
  *V = (1.0 - Kg) * VV;
  return e;
}

/* SMC over the parameters with a Kalman filter attached to every
 * theta-particle (Sec. 3.2.2, Alg. 4 with the Kalman filter of Alg. 1 as
 * Filter; windkessel model): the same order and inputs as orc_smc2, the
 * attached filter's state being (m, V) instead of particles; the
 * theta-particles' proposal filters run t_{0:i-1} from (m0, s0^2), and every
 * increment is exact, so the evidence estimate's only noise is the
 * parameter layer's. */
int32_t orc_smc2_kalman(const orc_problem* P, int32_t B, int32_t n_theta, const double* theta0,
                        int32_t T_run, const double* step_sd, const double* lo,
                        const double* hi, const double* z, const double* log_alpha,
                        const double* u_theta, double* theta_out, double* logw_out,
                        double* loglik_out, int32_t* accepts, double* ess_theta,
                        double* log_evidence, int32_t* anc_trace, int32_t* acc_trace,
                        double* logw_trace, double* mV_out /* [B][2] */) {
  double* th = (double*)malloc(sizeof(double) * (size_t)B * n_theta);
  double* th_new = (double*)malloc(sizeof(double) * (size_t)B * n_theta);
  double* thp = (double*)malloc(sizeof(double) * (size_t)n_theta);
  double* mV = (double*)malloc(sizeof(double) * 2 * (size_t)B);
  double* mV_new = (double*)malloc(sizeof(double) * 2 * (size_t)B);
  double* l = (double*)malloc(sizeof(double) * (size_t)B);
  double* l_new = (double*)malloc(sizeof(double) * (size_t)B);
  double* v = (double*)malloc(sizeof(double) * (size_t)B);
  int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)B);
  int32_t status = ORC_OK;
  double evidence = 0.0;
  memcpy(th, theta0, sizeof(double) * (size_t)B * n_theta);
  for (int32_t j = 0; j < B; ++j) {
    mV[2 * j] = th[(size_t)j * n_theta + 4];
    mV[2 * j + 1] = th[(size_t)j * n_theta + 5] * th[(size_t)j * n_theta + 5];
    l[j] = 0.0;
    v[j] = 0.0;
    a[j] = j;
    accepts[j] = 0;
  }
  for (int32_t i = 1; i <= T_run && status == ORC_OK; ++i) {
    for (int32_t j = 0; j < B; ++j) {
      const int32_t s = a[j];
      memcpy(th_new + (size_t)j * n_theta, th + (size_t)s * n_theta, sizeof(double) * n_theta);
      l_new[j] = l[s];
      mV_new[2 * j] = mV[2 * s];
      mV_new[2 * j + 1] = mV[2 * s + 1];
      if (anc_trace) anc_trace[(int64_t)(i - 1) * B + j] = s;
    }
    for (int32_t j = 0; j < B; ++j) {
      int inside = 1;
      for (int32_t p = 0; p < n_theta; ++p) {
        const double cur = th_new[(size_t)j * n_theta + p];
        if (step_sd[p] != 0.0) {
          const double step = step_sd[p] * z[((int64_t)(i - 1) * B + j) * n_theta + p];
          thp[p] = cur + step;
          if (!(thp[p] >= lo[p] && thp[p] <= hi[p])) inside = 0;
        } else {
          thp[p] = cur;
        }
      }
      int32_t acc = 0;
      if (inside) {
        double m = thp[4], V = thp[5] * thp[5], lp = 0.0;
        for (int32_t t = 1; t <= i - 1; ++t) lp = lp + orc_kf_wk_interval(P, thp, t, &m, &V);
        if (log_alpha[(int64_t)(i - 1) * B + j] <= lp - l_new[j]) {
          memcpy(th_new + (size_t)j * n_theta, thp, sizeof(double) * n_theta);
          l_new[j] = lp;
          mV_new[2 * j] = m;
          mV_new[2 * j + 1] = V;
          acc = 1;
          accepts[j] += 1;
        }
      }
      if (acc_trace) acc_trace[(int64_t)(i - 1) * B + j] = acc;
    }
    for (int32_t j = 0; j < B; ++j) {
      double m = mV_new[2 * j], V = mV_new[2 * j + 1];
      const double e = orc_kf_wk_interval(P, th_new + (size_t)j * n_theta, i, &m, &V);
      mV[2 * j] = m;
      mV[2 * j + 1] = V;
      v[j] = e;
      l[j] = l_new[j] + e;
      if (logw_trace) logw_trace[(int64_t)(i - 1) * B + j] = e;
    }
    memcpy(th, th_new, sizeof(double) * (size_t)B * n_theta);
    double e, s;
    const double u = (i < T_run) ? u_theta[i] : 0.5;
    status = orc_reduce_resample(B, v, u, &e, &s, a);
    evidence = evidence + e;
    ess_theta[i - 1] = s;
  }
  *log_evidence = (status == ORC_OK) ? evidence : -INFINITY;
  memcpy(theta_out, th, sizeof(double) * (size_t)B * n_theta);
  for (int32_t j = 0; j < B; ++j) {
    logw_out[j] = v[j];
    loglik_out[j] = l[j];
    if (mV_out) {
      mV_out[2 * j] = mV[2 * j];
      mV_out[2 * j + 1] = mV[2 * j + 1];
    }
  }
  free(a);
  free(v);
  free(l_new);
  free(l);
  free(mV_new);
  free(mV);
  free(thp);
  free(th_new);
  free(th);
  return status;
}

/* ---- marginal Metropolis-Hastings on the windkessel with the Kalman filter
 * (Sec. 3.2.1, eq. mh, Alg. 3, with the exact likelihood of Alg. 1) ---- */

/* Standard normal distribution function from the complementary error
 * function: Phi(x) = erfc(-x / sqrt 2) / 2 (accurate in both tails). */
static double orc_ncdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* Phi^{-1}(p) for p in (0, 1).  Above 1/2 by symmetry, -Phi^{-1}(1 - p)
 * (1 - p is exact there).  At or below 1/2, Newton's method on
 * ln Phi(z) = ln p from z = 0 (the log form is nearly quadratic in the lower
 * tail, so it converges fast there), kept inside a bracket [lo, hi] that
 * every evaluation narrows; a Newton step that leaves the bracket is replaced
 * by its midpoint.  Stops when the iterate no longer moves. */
double orc_ndtri(double p) {
  if (p > 0.5) return -orc_ndtri(1.0 - p);
  const double inv_sqrt_2pi = 0.39894228040143267794;
  const double lp = log(p);
  double lo = -40.0, hi = 0.0, z = 0.0;
  for (int it = 0; it < 400; ++it) {
    double P = orc_ncdf(z);
    double f = log(P) - lp;
    if (f == 0.0) break;
    if (f < 0.0) lo = z; else hi = z;
    double zn = z - f * P / (inv_sqrt_2pi * exp(-0.5 * z * z));
    if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
    if (zn == z || zn == lo || zn == hi) break;
    z = zn;
  }
  return z;
}

/* The windkessel's model parameters from (R, C, Z, sigma^2), Sec. 2.1.1:
 * a = exp(-h / (R C)), c = R (1 - a) (eq. 2-windkessel), the flow noise of
 * variance sigma^2 scaled by c into the pressure, sd c sigma; the initial
 * state N(m0, s0^2). */
void orc_wk_theta(const orc_problem* P, const orc_wk_mh* H, const double* rczs, double* theta) {
  double a = exp(-P->h / (rczs[0] * rczs[1]));
  double c = rczs[0] * (1.0 - a);
  theta[0] = a;
  theta[1] = c;
  theta[2] = rczs[2];
  theta[3] = c * sqrt(rczs[3]);
  theta[4] = H->m0;
  theta[5] = H->s0;
}

/* ln p(R, C, Z, sigma^2) up to a constant: Gamma(k, s) densities
 * x^{k-1} e^{-x/s} on R, C, Z and the Inverse-Gamma(alpha, beta) density
 * x^{-alpha-1} e^{-beta/x} on sigma^2 (shape and scale parameters). */
double orc_wk_log_prior(const orc_wk_mh* H, const double* x) {
  double lp = 0.0;
  for (int k = 0; k < 3; ++k)
    lp += (H->prior_shape[k] - 1.0) * log(x[k]) - x[k] / H->prior_scale[k];
  lp += -(H->ig_shape + 1.0) * log(x[3]) - H->ig_scale / x[3];
  return lp;
}

/* n_chains independent chains over (R, C, Z, sigma^2).  The random numbers
 * are inputs: prop[i][c][0..2] uniforms in (0, 1) that draw the truncated
 * Gaussian proposals of R, C and Z by inversion, prop[i][c][3] a
 * Gamma(ig_prop_shape, 1) variate g, alpha[i][c] in (0, 1].  Iteration i:
 *   1. proposal: for R, C, Z with sd s > 0, y = x + s z with z drawn from
 *      N(0, 1) truncated to z > -x/s: with p0 = Phi(-x/s),
 *      z = Phi^{-1}(p0 + u (1 - p0)) if u <= 1/2, else
 *      z = -Phi^{-1}((1 - u)(1 - p0)) (the same value, from the upper tail);
 *      sigma^2' = f sigma^2 / g, an Inverse-Gamma(shape, f sigma^2) draw;
 *   2. a proposal with a non-positive or non-finite component lies outside
 *      the prior's support: rejected without a likelihood;
 *   3. otherwise l' is the Kalman filter's log-likelihood at theta', and the
 *      move is accepted iff ln alpha <= (l' - l) + ((ln p(theta') -
 *      ln p(theta)) + ln q(theta | theta') - ln q(theta' | theta)), where the
 *      proposal term is the sum over moved components of
 *      ln Phi(x/s) - ln Phi(y/s) (the truncated Gaussians' normalisers) and
 *      (2 shape + 1) ln r - f (r - 1/r), r = sigma^2'/sigma^2 (the
 *      Inverse-Gamma proposal's density ratio).
 * Outputs: theta_trace[i][c][4], ll_trace[i][c] (the chain after iteration
 * i), accepts[c]. */
int32_t orc_kf_pmmh(const orc_problem* P, const orc_wk_mh* H, int32_t n_chains, int32_t iters,
                    const double* theta0, const double* prop, const double* alpha,
                    double* theta_trace, double* ll_trace, int32_t* accepts) {
  double* ell = (double*)malloc(sizeof(double) * (size_t)(P->T > 0 ? P->T : 1));
  for (int32_t c = 0; c < n_chains; ++c) {
    double x[4], y[4], th[6];
    for (int k = 0; k < 4; ++k) x[k] = theta0[(int64_t)c * 4 + k];
    orc_wk_theta(P, H, x, th);
    double ll = orc_kf_wk(P, th, ell);
    double lp = orc_wk_log_prior(H, x);
    int32_t acc = 0;
    for (int32_t i = 0; i < iters; ++i) {
      const double* u = prop + ((int64_t)i * n_chains + c) * 4;
      double lq = 0.0;
      int inside = 1;
      for (int k = 0; k < 3; ++k) {
        double s = H->step_sd[k];
        if (s > 0.0) {
          double p0 = orc_ncdf(-x[k] / s);
          double z = (u[k] <= 0.5) ? orc_ndtri(p0 + u[k] * (1.0 - p0))
                                   : -orc_ndtri((1.0 - u[k]) * (1.0 - p0));
          y[k] = x[k] + s * z;
          if (!(y[k] > 0.0) || !isfinite(y[k])) {
            inside = 0;
          } else {
            lq += log(orc_ncdf(x[k] / s)) - log(orc_ncdf(y[k] / s));
          }
        } else {
          y[k] = x[k];
        }
      }
      if (H->ig_prop_factor > 0.0) {
        y[3] = H->ig_prop_factor * x[3] / u[3];
        if (!(y[3] > 0.0) || !isfinite(y[3])) {
          inside = 0;
        } else {
          double r = y[3] / x[3];
          lq += (2.0 * H->ig_prop_shape + 1.0) * log(r) - H->ig_prop_factor * (r - 1.0 / r);
        }
      } else {
        y[3] = x[3];
      }
      if (inside) {
        orc_wk_theta(P, H, y, th);
        double llp = orc_kf_wk(P, th, ell);
        double lpp = orc_wk_log_prior(H, y);
        double lhs = log(alpha[(int64_t)i * n_chains + c]);
        if (lhs <= (llp - ll) + ((lpp - lp) + lq)) {
          for (int k = 0; k < 4; ++k) x[k] = y[k];
          ll = llp;
          lp = lpp;
          ++acc;
        }
      }
      for (int k = 0; k < 4; ++k) theta_trace[((int64_t)i * n_chains + c) * 4 + k] = x[k];
      ll_trace[(int64_t)i * n_chains + c] = ll;
    }
    accepts[c] = acc;
  }
  free(ell);
  return ORC_OK;
}
