// The windkessel model's Kalman filter (Sec. 3.1.1, Alg. 1 reduced to one
// dimension: every Cholesky factor is a square root), batched over filters,
// one lane per filter, in FP64:
//   k_kf_run          whole runs over t = 1..T (the exact likelihood)
//   k_kf_proposal     SMC over the parameters with attached Kalman filters:
//                     each proposal's filter over t_{0:i-1}
//   k_kf_advance      every attached filter over t_{i-1:i}
//   k_smc2_accept_kf  the Metropolis-Hastings decision with those filters
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

hipError_t launch_kf_advance(const KfArgs& A, const Smc2Args& S, int i, hipStream_t s) {
  hipLaunchKernelGGL(k_kf_advance, kf_blocks(S.B), 256, 0, s, A, S, i);
  return hipGetLastError();
}

}  // namespace pfk
