// SMC over the parameters with a particle filter attached to every
// theta-particle (Sec. 3.2.2, Alg. 4; SMC^2 when the filter is Alg. 2), on
// top of the batched layout: theta-particle j owns filter slot j.
//
//   k_theta_resample    one workgroup: theta-weights v_j = ell_j of the last
//                       interval, their max, FP64 sums and scan, ESS, the
//                       evidence factor, systematic theta-ancestors by binary
//                       search of the scan, and the move of parameters,
//                       likelihood and status to the new slots.
//   k_filter_copy_*     whole-filter copies into the slots whose ancestor is
//                       another slot (systematic selection when the particle
//                       counts differ), via the spare state buffer.
//   k_smc2_propose      random-walk proposals inside the prior box, written
//                       as the proposal handle's derived parameters.
//   k_smc2_accept       Metropolis-Hastings decision per theta-particle
//                       (Alg. 3, eq. mh) after the proposal filters ran.
//   k_accept_copy       accepted slots take the proposal filter's particles.
#include <math.h>

#include "pf_device.hpp"
#include "pf_smc2.hpp"

namespace pfk {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ double block_max_1024(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_sum_1024(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += red[i];
  __syncthreads();
  return r;
}

// Whole-filter copy index: destination particle k of n_dst takes source
// particle floor((k + w 2^-32) n_src / n_dst) (systematic selection on equal
// weights), exact in 64-bit integers for counts up to 2^13.
__device__ __forceinline__ int64_t copy_index(int64_t k, int64_t n_src, int64_t n_dst,
                                              uint32_t w) {
  const uint64_t num = (((uint64_t)k << 32) | (uint64_t)w) * (uint64_t)n_src;
  return (int64_t)(num / ((uint64_t)n_dst << 32));
}

// ---------------------------------------------------------------- theta layer

// One workgroup of SMC2_NT lanes.  v_j = ell_tr[j*T + col].  Writes the
// theta-ESS and adds ln(sum exp v) - ln B to *evid.  With draw != 0 also
// draws a[k] = min{j : B W_j > (u + k) S} (W the inclusive scan of
// exp(v - max)), falling back to the last positive weight, and moves the
// parameters (raw and derived), likelihood and status of slot a[k] to slot
// k.  If no theta-weight is positive the ancestors are the identity and
// *numeric is set.
__global__ __launch_bounds__(SMC2_NT) void k_theta_resample(Smc2Args S, int32_t col, double u,
                                                            int32_t draw, int32_t* anc_tr_row,
                                                            double* ess_out) {
  __shared__ double W[SMC2_MAXB];
  __shared__ double red[SMC2_NT / 64];
  __shared__ int ired[SMC2_NT / 64];
  const int B = S.B;
  const int tid = threadIdx.x;
  // this lane's contiguous range of theta-particles
  const int per = (B + SMC2_NT - 1) / SMC2_NT;
  const int j0 = tid * per, j1 = min(B, j0 + per);
  double m = -INFINITY;
  for (int j = j0; j < j1; ++j) {
    const double v = S.ell_tr[(int64_t)j * S.T + col];
    if (v > m) m = v;
  }
  const double M = block_max_1024(m, red);
  const bool numeric = !(M > -INFINITY) || !(M < INFINITY);
  double acc = 0.0, acc2 = 0.0;
  int jstar = -1;
  if (!numeric) {
    for (int j = j0; j < j1; ++j) {
      const double w = exp_nonpos(S.ell_tr[(int64_t)j * S.T + col] - M);
      acc = acc + w;
      acc2 = acc2 + w * w;
      W[j] = acc;  // local inclusive scan, offset below
      if (w > 0.0) jstar = j;
    }
  }
  // exclusive scan of the lanes' sums (sequential over the wave sums)
  double x = acc;
  const int lane = tid & 63, wv = tid >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) red[wv] = x;
  int js = jstar;
  for (int o = 32; o > 0; o >>= 1) js = max(js, __shfl_xor(js, o));
  if (lane == 0) ired[wv] = js;
  __syncthreads();
  double base = 0.0;
  for (int i = 0; i < wv; ++i) base += red[i];
  double total = 0.0;
  int jst = -1;
  for (int i = 0; i < SMC2_NT / 64; ++i) {
    total += red[i];
    jst = max(jst, ired[i]);
  }
  const double excl = base + x - acc;
  if (!numeric)
    for (int j = j0; j < j1; ++j) W[j] += excl;
  __syncthreads();  // every lane has read red before it is reused
  const double S2 = block_sum_1024(acc2, red);  // its barriers also order the W writes
  if (tid == 0) {
    *S.numeric = *S.numeric | (numeric ? 1 : 0);
    if (numeric) {
      *ess_out = 0.0;
      *S.evid = -INFINITY;
    } else {
      *ess_out = (total * total) / S2;
      *S.evid = *S.evid + ((M + log(total)) - log((double)B));
    }
  }
  if (!draw) return;
  // ancestors by binary search of the scan
  const double Bd = (double)B;
  for (int k = tid; k < B; k += SMC2_NT) {
    int a = k;
    if (!numeric) {
      const double thr = (u + (double)k) * total;
      int lo = 0, hi = B;  // first j with B W_j > thr, or B
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (Bd * W[mid] > thr) hi = mid;
        else lo = mid + 1;
      }
      a = lo < B ? lo : jst;
    }
    S.a[k] = a;
    if (anc_tr_row) anc_tr_row[k] = a;
  }
  // snapshot the slots' parameters, likelihoods and status, then move them
  for (int j = tid; j < B; j += SMC2_NT) {
    for (int p = 0; p < 8; ++p) S.snap_dev[(int64_t)j * 8 + p] = S.theta_dev[(int64_t)j * 8 + p];
    for (int p = 0; p < S.n_theta; ++p)
      S.snap_raw[(int64_t)j * S.n_theta + p] = S.raw[(int64_t)j * S.n_theta + p];
    S.snap_ll[j] = S.fs[j].loglik;
    S.snap_st[j] = S.fs[j].status;
    if (S.mV) {
      S.snap_mV[2 * j] = S.mV[2 * j];
      S.snap_mV[2 * j + 1] = S.mV[2 * j + 1];
    }
  }
  __syncthreads();
  for (int j = tid; j < B; j += SMC2_NT) {
    const int s = S.a[j];
    for (int p = 0; p < 8; ++p) S.theta_dev[(int64_t)j * 8 + p] = S.snap_dev[(int64_t)s * 8 + p];
    for (int p = 0; p < S.n_theta; ++p)
      S.raw[(int64_t)j * S.n_theta + p] = S.snap_raw[(int64_t)s * S.n_theta + p];
    S.fs[j].loglik = S.snap_ll[s];
    S.fs[j].status = S.snap_st[s];
    if (S.mV) {
      S.mV[2 * j] = S.snap_mV[2 * s];
      S.mV[2 * j + 1] = S.snap_mV[2 * s + 1];
    }
  }
}

// Pass 1 of the whole-filter copies: slot f whose theta-ancestor s differs
// takes s's equally weighted particles, i.e. the propagated states at s's
// pending ancestors, written to the spare buffer.
template <typename Real>
__global__ __launch_bounds__(BATCH_NT) void k_filter_copy_gather(const Real* __restrict__ xcur,
                                                                 Real* __restrict__ xspare,
                                                                 const int32_t* __restrict__ anc,
                                                                 BatchArgs A, Smc2Args S,
                                                                 const uint32_t* __restrict__ w) {
  const int f = A.chunk_f[blockIdx.x];
  const int s = S.a[f];
  if (s == f) return;
  const int64_t off = A.off[f], n = A.off[f + 1] - off;
  const int64_t k = (int64_t)A.chunk_k[blockIdx.x] + threadIdx.x;
  if (k >= n) return;
  const int64_t soff = A.off[s], sn = A.off[s + 1] - soff;
  const int64_t p = copy_index(k, sn, n, w[f]);
  const int64_t src = soff + anc[soff + p];
  for (int i = 0; i < A.d; ++i) xspare[(int64_t)i * A.ld + off + k] = xcur[(int64_t)i * A.ld + src];
}

// Pass 2: the copied particles become the slot's equally weighted set.
template <typename Real>
__global__ __launch_bounds__(BATCH_NT) void k_filter_copy_commit(Real* __restrict__ xcur,
                                                                 const Real* __restrict__ xspare,
                                                                 int32_t* __restrict__ anc,
                                                                 BatchArgs A, Smc2Args S) {
  const int f = A.chunk_f[blockIdx.x];
  if (S.a[f] == f) return;
  const int64_t off = A.off[f], n = A.off[f + 1] - off;
  const int64_t k = (int64_t)A.chunk_k[blockIdx.x] + threadIdx.x;
  if (k >= n) return;
  for (int i = 0; i < A.d; ++i) xcur[(int64_t)i * A.ld + off + k] = xspare[(int64_t)i * A.ld + off + k];
  anc[off + k] = (int32_t)k;
}

// theta' = theta + step_sd z on the moved parameters (two roundings, no
// contraction); inside[j] = every moved parameter within [lo, hi].  The
// proposal handle's derived parameters get theta' (or theta when outside:
// that slot's proposal run is then unused).
__global__ void k_smc2_propose(Smc2Args S, const double* __restrict__ z_row,
                               double* __restrict__ prop_dev) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S.B) return;
  const int nt = S.n_theta;
  double th[8];
  int inside = 1;
  for (int p = 0; p < nt; ++p) {
    const double cur = S.raw[(int64_t)j * nt + p];
    if (S.step_sd[p] != 0.0) {
      const double step = __dmul_rn(S.step_sd[p], z_row[(int64_t)j * nt + p]);
      th[p] = __dadd_rn(cur, step);
      if (!(th[p] >= S.lo[p] && th[p] <= S.hi[p])) inside = 0;
    } else {
      th[p] = cur;
    }
  }
  for (int p = 0; p < nt; ++p) S.prop_raw[(int64_t)j * nt + p] = th[p];
  S.inside[j] = inside;
  double* o = prop_dev + (int64_t)j * 8;
  if (!inside) {
    for (int p = 0; p < 8; ++p) o[p] = S.theta_dev[(int64_t)j * 8 + p];
  } else if (S.model == 1) {
    for (int p = 0; p < 6; ++p) o[p] = th[p];
    o[6] = 0.0;
    o[7] = 0.0;
  } else {
    o[0] = th[0];
    o[1] = __dmul_rn(th[1], S.sqrt_h);
    for (int p = 2; p < 8; ++p) o[p] = 0.0;
  }
}

// Accept iff inside and log_alpha <= l' - l (ties accept).  An accepted slot
// takes theta', its derived form, l' and the proposal filter's status.
__global__ void k_smc2_accept(Smc2Args S, const double* __restrict__ log_alpha_row,
                              const double* __restrict__ prop_dev,
                              const FilterState* __restrict__ pfs, int32_t* acc_tr_row) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S.B) return;
  const double lp = pfs[j].status ? -INFINITY : pfs[j].loglik;
  const int acc = S.inside[j] && (log_alpha_row[j] <= lp - S.fs[j].loglik);
  S.accepted[j] = acc;
  if (acc_tr_row) acc_tr_row[j] = acc;
  if (!acc) return;
  S.accepts[j] += 1;
  for (int p = 0; p < S.n_theta; ++p)
    S.raw[(int64_t)j * S.n_theta + p] = S.prop_raw[(int64_t)j * S.n_theta + p];
  for (int p = 0; p < 8; ++p) S.theta_dev[(int64_t)j * 8 + p] = prop_dev[(int64_t)j * 8 + p];
  S.fs[j].loglik = pfs[j].loglik;
  S.fs[j].status = pfs[j].status;
}

// Accepted slots take the proposal filter's equally weighted particles.
template <typename Real>
__global__ __launch_bounds__(BATCH_NT) void k_accept_copy(Real* __restrict__ xcur,
                                                          int32_t* __restrict__ anc,
                                                          const Real* __restrict__ pxcur,
                                                          const int32_t* __restrict__ panc,
                                                          BatchArgs A, Smc2Args S) {
  const int f = A.chunk_f[blockIdx.x];
  if (!S.accepted[f]) return;
  const int64_t off = A.off[f], n = A.off[f + 1] - off;
  const int64_t k = (int64_t)A.chunk_k[blockIdx.x] + threadIdx.x;
  if (k >= n) return;
  const int64_t src = off + panc[off + k];
  for (int i = 0; i < A.d; ++i) xcur[(int64_t)i * A.ld + off + k] = pxcur[(int64_t)i * A.ld + src];
  anc[off + k] = (int32_t)k;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_theta_resample(const Smc2Args& S, int32_t col, double u, int32_t draw,
                                 int32_t* anc_tr_row, double* ess_out, hipStream_t s) {
  if (S.B < 1 || S.B > SMC2_MAXB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_theta_resample, 1, SMC2_NT, 0, s, S, col, u, draw, anc_tr_row, ess_out);
  return hipGetLastError();
}

hipError_t launch_filter_copy(int prec, void* xcur, void* xspare, int32_t* anc, const BatchArgs& A,
                              const Smc2Args& S, const uint32_t* w, hipStream_t s) {
  const unsigned g = (unsigned)A.n_chunks;
  if (g == 0) return hipSuccess;
  if (prec == 0) {
    hipLaunchKernelGGL(k_filter_copy_gather<double>, g, BATCH_NT, 0, s, (const double*)xcur,
                       (double*)xspare, (const int32_t*)anc, A, S, w);
    hipLaunchKernelGGL(k_filter_copy_commit<double>, g, BATCH_NT, 0, s, (double*)xcur,
                       (const double*)xspare, anc, A, S);
  } else {
    hipLaunchKernelGGL(k_filter_copy_gather<float>, g, BATCH_NT, 0, s, (const float*)xcur,
                       (float*)xspare, (const int32_t*)anc, A, S, w);
    hipLaunchKernelGGL(k_filter_copy_commit<float>, g, BATCH_NT, 0, s, (float*)xcur,
                       (const float*)xspare, anc, A, S);
  }
  return hipGetLastError();
}

hipError_t launch_smc2_propose(const Smc2Args& S, const double* z_row, double* prop_dev,
                               hipStream_t s) {
  const unsigned g = (unsigned)((S.B + 255) / 256);
  hipLaunchKernelGGL(k_smc2_propose, g, 256, 0, s, S, z_row, prop_dev);
  return hipGetLastError();
}

hipError_t launch_smc2_accept(const Smc2Args& S, const double* log_alpha_row,
                              const double* prop_dev, const FilterState* pfs, int32_t* acc_tr_row,
                              hipStream_t s) {
  const unsigned g = (unsigned)((S.B + 255) / 256);
  hipLaunchKernelGGL(k_smc2_accept, g, 256, 0, s, S, log_alpha_row, prop_dev, pfs, acc_tr_row);
  return hipGetLastError();
}

hipError_t launch_accept_copy(int prec, void* xcur, int32_t* anc, const void* pxcur,
                              const int32_t* panc, const BatchArgs& A, const Smc2Args& S,
                              hipStream_t s) {
  const unsigned g = (unsigned)A.n_chunks;
  if (g == 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(k_accept_copy<double>, g, BATCH_NT, 0, s, (double*)xcur, anc,
                       (const double*)pxcur, panc, A, S);
  else
    hipLaunchKernelGGL(k_accept_copy<float>, g, BATCH_NT, 0, s, (float*)xcur, anc,
                       (const float*)pxcur, panc, A, S);
  return hipGetLastError();
}

}  // namespace pfk
