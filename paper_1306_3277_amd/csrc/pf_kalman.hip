// The windkessel model's Kalman filter (Sec. 3.1.1, Alg. 1 reduced to one
// dimension: every Cholesky factor is a square root), batched over filters,
// one lane per filter, in FP64:
//   k_kf_run          whole runs over t = 1..T (the exact likelihood)
//   k_kf_proposal     SMC over the parameters with attached Kalman filters:
//                     each proposal's filter over t_{0:i-1}
//   k_kf_advance      every attached filter over t_{i-1:i}
//   k_smc2_accept_kf  the Metropolis-Hastings decision with those filters
//   k_kf_pmmh         marginal Metropolis-Hastings chains on (R, C, Z,
//                     sigma^2) with the exact likelihood, a chain per lane
#include <math.h>

#include "pf_kalman.hpp"

namespace pfk {

// One interval: K predictions m <- a m + c q_{n-1}, V <- a^2 V + sigma_p^2,
// then the correction with y_t; returns ell_t.
__device__ __forceinline__ double kf_interval(const double* th, const KfArgs& A, int t, double& m,
                                              double& V) {
  const double a = th[0], c = th[1], Z = th[2], sp = th[3];
  for (int s = 1; s <= A.K; ++s) {
    const int64_t n = (int64_t)(t - 1) * A.K + s;
    m = a * m + c * A.q[n - 1];
    V = a * a * V + sp * sp;
  }
  const double qn = A.q[(int64_t)t * A.K];
  const double v = A.obs[t - 1] - (m + Z * qn);
  const double S = V + A.R;
  const double e = -0.5 * (log(2.0 * 3.14159265358979323846 * S) + v * v / S);
  const double Kg = V / S;
  m = m + Kg * v;
  V = (1.0 - Kg) * V;
  return e;
}

__global__ void k_kf_run(KfArgs A, const double* __restrict__ theta, double* __restrict__ ll,
                         double* __restrict__ ell) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= A.B) return;
  const double* th = theta + (int64_t)b * 8;
  double m = th[4], V = th[5] * th[5], tot = 0.0;
  for (int t = 1; t <= A.T; ++t) {
    const double e = kf_interval(th, A, t, m, V);
    ell[(int64_t)b * A.T + t - 1] = e;
    tot = tot + e;
  }
  ll[b] = tot;
}

// Proposal filters: from (m0', s0'^2) over t = 1..i-1 for the proposals
// inside the prior box.
__global__ void k_kf_proposal(KfArgs A, Smc2Args S, const double* __restrict__ prop_dev,
                              double* __restrict__ prop_l, double* __restrict__ prop_mV, int i) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S.B || !S.inside[j]) return;
  const double* th = prop_dev + (int64_t)j * 8;
  double m = th[4], V = th[5] * th[5], lp = 0.0;
  for (int t = 1; t <= i - 1; ++t) lp = lp + kf_interval(th, A, t, m, V);
  prop_l[j] = lp;
  prop_mV[2 * j] = m;
  prop_mV[2 * j + 1] = V;
}

// Accept iff inside and log_alpha <= l' - l (ties accept); an accepted slot
// takes theta', its derived form, l' and the proposal's filter state.
__global__ void k_smc2_accept_kf(Smc2Args S, const double* __restrict__ log_alpha_row,
                                 const double* __restrict__ prop_dev,
                                 const double* __restrict__ prop_l,
                                 const double* __restrict__ prop_mV, int32_t* acc_tr_row) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S.B) return;
  const int acc = S.inside[j] && (log_alpha_row[j] <= prop_l[j] - S.fs[j].loglik);
  S.accepted[j] = acc;
  if (acc_tr_row) acc_tr_row[j] = acc;
  if (!acc) return;
  S.accepts[j] += 1;
  for (int p = 0; p < S.n_theta; ++p)
    S.raw[(int64_t)j * S.n_theta + p] = S.prop_raw[(int64_t)j * S.n_theta + p];
  for (int p = 0; p < 8; ++p) S.theta_dev[(int64_t)j * 8 + p] = prop_dev[(int64_t)j * 8 + p];
  S.fs[j].loglik = prop_l[j];
  S.fs[j].status = 0;
  S.mV[2 * j] = prop_mV[2 * j];
  S.mV[2 * j + 1] = prop_mV[2 * j + 1];
}

// Every attached filter over t_{i-1:i}: the increment is the new
// theta-log-weight and adds to the likelihood.
__global__ void k_kf_advance(KfArgs A, Smc2Args S, int i) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S.B) return;
  double m = S.mV[2 * j], V = S.mV[2 * j + 1];
  const double e = kf_interval(S.theta_dev + (int64_t)j * 8, A, i, m, V);
  S.mV[2 * j] = m;
  S.mV[2 * j + 1] = V;
  S.fs[j].loglik = S.fs[j].loglik + e;
  S.fs[j].t = i;
  S.ell_tr_w[(int64_t)j * S.T + i - 1] = e;
}

__global__ void k_kf_init(Smc2Args S) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S.B) return;
  const double* th = S.theta_dev + (int64_t)j * 8;
  S.mV[2 * j] = th[4];
  S.mV[2 * j + 1] = th[5] * th[5];
}

// ---------------------------------------------------------------- chains on (R, C, Z, sigma^2)

// Phi(x) from the complementary error function (accurate in both tails).
__device__ __forceinline__ double ncdf(double x) { return 0.5 * erfc(-x * 0.70710678118654752440); }

// Model parameters from (R, C, Z, sigma^2) (Sec. 2.1.1): a = exp(-h/(R C)),
// c = R (1 - a), pressure noise sd c sigma, initial N(m0, s0^2); th[8] as
// the filters hold them.
__device__ __forceinline__ void wk_params(const pf_wk_mh& H, double h, const double* x,
                                          double* th) {
  const double a = exp(-h / (x[0] * x[1]));
  const double c = x[0] * (1.0 - a);
  th[0] = a;
  th[1] = c;
  th[2] = x[2];
  th[3] = c * sqrt(x[3]);
  th[4] = H.m0;
  th[5] = H.s0;
}

// ln p(R, C, Z, sigma^2) up to a constant: Gamma densities x^{k-1} e^{-x/s}
// and the Inverse-Gamma density x^{-alpha-1} e^{-beta/x}.
__device__ __forceinline__ double wk_log_prior(const pf_wk_mh& H, const double* x) {
  double lp = 0.0;
  for (int k = 0; k < 3; ++k) lp += (H.prior_shape[k] - 1.0) * log(x[k]) - x[k] / H.prior_scale[k];
  lp += -(H.ig_shape + 1.0) * log(x[3]) - H.ig_scale / x[3];
  return lp;
}

__device__ __forceinline__ double kf_loglik(const KfArgs& A, const double* th) {
  double m = th[4], V = th[5] * th[5], tot = 0.0;
  for (int t = 1; t <= A.T; ++t) tot = tot + kf_interval(th, A, t, m, V);
  return tot;
}

// One chain per lane through every iteration (Alg. 3): truncated-Gaussian
// proposals of R, C, Z by inversion on the accurate tail, the
// Inverse-Gamma proposal of sigma^2 from the given Gamma variate, support
// check, exact likelihood, prior and proposal density ratios, acceptance.
__global__ void __launch_bounds__(64) k_kf_pmmh(KfArgs A, pf_wk_mh H, double h, int32_t iters,
                                                const double* __restrict__ theta0,
                                                const double* __restrict__ prop,
                                                const double* __restrict__ alpha,
                                                double* __restrict__ theta_trace,
                                                double* __restrict__ ll_trace,
                                                int32_t* __restrict__ accepts,
                                                double* __restrict__ ll0) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= A.B) return;
  double x[4], y[4], th[8];
  for (int k = 0; k < 4; ++k) x[k] = theta0[(int64_t)c * 4 + k];
  wk_params(H, h, x, th);
  double ll = kf_loglik(A, th);
  double lp = wk_log_prior(H, x);
  if (ll0) ll0[c] = ll;
  int32_t acc = 0;
  for (int32_t i = 0; i < iters; ++i) {
    const int64_t row = (int64_t)i * A.B + c;
    const double* u = prop + row * 4;
    double lq = 0.0;
    bool inside = true;
    for (int k = 0; k < 3; ++k) {
      const double s = H.step_sd[k];
      if (s > 0.0) {
        const double p0 = ncdf(-x[k] / s);
        const double z = (u[k] <= 0.5) ? normcdfinv(p0 + u[k] * (1.0 - p0))
                                        : -normcdfinv((1.0 - u[k]) * (1.0 - p0));
        y[k] = x[k] + s * z;
        if (!(y[k] > 0.0) || !isfinite(y[k]))
          inside = false;
        else
          lq += log(ncdf(x[k] / s)) - log(ncdf(y[k] / s));
      } else {
        y[k] = x[k];
      }
    }
    if (H.ig_prop_factor > 0.0) {
      y[3] = H.ig_prop_factor * x[3] / u[3];
      if (!(y[3] > 0.0) || !isfinite(y[3])) {
        inside = false;
      } else {
        const double r = y[3] / x[3];
        lq += (2.0 * H.ig_prop_shape + 1.0) * log(r) - H.ig_prop_factor * (r - 1.0 / r);
      }
    } else {
      y[3] = x[3];
    }
    if (inside) {
      wk_params(H, h, y, th);
      const double llp = kf_loglik(A, th);
      const double lpp = wk_log_prior(H, y);
      if (log(alpha[row]) <= (llp - ll) + ((lpp - lp) + lq)) {
        for (int k = 0; k < 4; ++k) x[k] = y[k];
        ll = llp;
        lp = lpp;
        ++acc;
      }
    }
    for (int k = 0; k < 4; ++k) theta_trace[row * 4 + k] = x[k];
    ll_trace[row] = ll;
  }
  accepts[c] = acc;
}

// ---------------------------------------------------------------- launchers

static inline unsigned kf_blocks(int n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_kf_run(const KfArgs& A, const double* theta, double* ll, double* ell,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_kf_run, kf_blocks(A.B), 256, 0, s, A, theta, ll, ell);
  return hipGetLastError();
}

hipError_t launch_kf_init(const Smc2Args& S, hipStream_t s) {
  hipLaunchKernelGGL(k_kf_init, kf_blocks(S.B), 256, 0, s, S);
  return hipGetLastError();
}

hipError_t launch_kf_proposal(const KfArgs& A, const Smc2Args& S, const double* prop_dev,
                              double* prop_l, double* prop_mV, int i, hipStream_t s) {
  hipLaunchKernelGGL(k_kf_proposal, kf_blocks(S.B), 256, 0, s, A, S, prop_dev, prop_l, prop_mV,
                     i);
  return hipGetLastError();
}

hipError_t launch_smc2_accept_kf(const Smc2Args& S, const double* log_alpha_row,
                                 const double* prop_dev, const double* prop_l,
                                 const double* prop_mV, int32_t* acc_tr_row, hipStream_t s) {
  hipLaunchKernelGGL(k_smc2_accept_kf, kf_blocks(S.B), 256, 0, s, S, log_alpha_row, prop_dev,
                     prop_l, prop_mV, acc_tr_row);
  return hipGetLastError();
}

hipError_t launch_kf_pmmh(const KfArgs& A, const pf_wk_mh& H, double h, int32_t iters,
                          const double* theta0, const double* prop, const double* alpha,
                          double* theta_trace, double* ll_trace, int32_t* accepts, double* ll0,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_kf_pmmh, (unsigned)((A.B + 63) / 64), 64, 0, s, A, H, h, iters, theta0,
                     prop, alpha, theta_trace, ll_trace, accepts, ll0);
  return hipGetLastError();
}

hipError_t launch_kf_advance(const KfArgs& A, const Smc2Args& S, int i, hipStream_t s) {
  hipLaunchKernelGGL(k_kf_advance, kf_blocks(S.B), 256, 0, s, A, S, i);
  return hipGetLastError();
}

}  // namespace pfk
