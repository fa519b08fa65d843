// Plain-layout kernels of the gfx950 bootstrap particle filter (Alg. 2):
//   K1 propagate + weight   one particle per lane, K substeps in registers,
//                           log-weight, per-block (max, sum, sum of squares)
//   K2 combine              (filters of more than FUSE_NB blocks) one
//                           workgroup: global max, FP64 block offsets,
//                           likelihood increment, ESS, resampling uniform
//   K3 combine + scan +     (smaller filters combine the block partials in
//      marks                every K3 block instead of K2) FP64 block scan
//                           of exp(lw - M); for each particle the number of
//                           strata its cumulative weight covers, and a mark
//                           (its index) on the first stratum it owns
//   K4 tile gather          per tile of 1024 outputs, a running maximum over
//                           the marks names every output's ancestor (the
//                           work per lane does not depend on the weights),
//                           then the ancestors' states are copied
// plus initialisation and the synthetic-data simulator.  pf_step runs K1
// (K2) K3, pf_resample K4.  The state is kept in 64-particle tiles (pidx).
#include <math.h>

#include "pf_device.hpp"
#include "pf_internal.hpp"

namespace pfk {

__device__ __forceinline__ Key key_of(const KeyArg& k) { return Key{k.lo, k.hi}; }

// ---------------------------------------------------------------- init
template <int MODEL, int D, typename Real>
__global__ __launch_bounds__(K1_NT) void k_init(Real* __restrict__ x, PlainArgs A) {
  const int64_t j = (int64_t)blockIdx.x * K1_NT + threadIdx.x;
  if (j >= A.N) return;
  const Key key = key_of(A.key);
  const uint32_t iter = A.fs->iter;
  const int64_t col = A.off + j;
  if (MODEL == 1) {
    double z0, z1;
    const uint4 w = draw(key, TAG_INIT, 0, iter, (uint32_t)j, 0, A.b);
    bm_pair_f64(w.x, w.y, z0, z1);
    x[col] = (Real)(A.theta[4] + A.theta[5] * z0);
  } else {
#pragma unroll
    for (int blk = 0; blk < D / 4; ++blk) {
      double z[4];
      normals4_f64(draw(key, TAG_INIT, blk, iter, (uint32_t)j, 0, A.b), z);
#pragma unroll
      for (int m = 0; m < 4; ++m) x[pidx(col, 4 * blk + m, D)] = (Real)z[m];
    }
  }
}

__global__ void k_reset(FilterState* fs, double* ell, double* ess, int B, int T, uint32_t iter) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)B * T) {
    ell[i] = 0.0;
    ess[i] = 0.0;
  }
  if (i < B) {
    FilterState f;
    f.loglik = 0.0;
    f.M = 0.0;
    f.S = 0.0;
    f.u = 0.0;
    f.ell = 0.0;
    f.ess = 0.0;
    f.t = 0;
    f.status = 0;
    f.iter = iter;
    f.pad = 0;
    f.lprev = 0.0;
    f.carry = 0;
    f.tk = 0;
    f.cn1 = 0;
    f.amode = AMODE_IDENTITY;
    fs[i] = f;
  }
}

// ---------------------------------------------------------------- combine
// The collective over the block partials (max, sum, sum of squares of the
// 256-particle K1 blocks).  Offsets of the blocks' cumulative weights: K1
// block i owns [off_i, off_{i+1}), off_nb = S.  They are summed
// sequentially within each lane's chunk of partials and scanned across the
// lanes; an exact running maximum then makes them non-decreasing whatever
// the rounding, so the cumulative weights built on them are monotone.
//
// Two forms.  A filter of at most FUSE_NB blocks has every K3 block combine
// all of its partials itself (the same order, the same code, so every block
// obtains the same bits with no extra launch and no communication between
// blocks); the partials are read coalesced and their scaled totals staged
// in LDS.  A larger filter has one K2 workgroup combine them once and store
// the offsets, before K3.
struct Combined {
  double M, S, S2, lo, hi;
};

template <int NT, int MAXNB>
__device__ __forceinline__ Combined combine_block_lds(const double* __restrict__ P, int nb,
                                                      int k1b, int span) {
  constexpr int NW = NT / WAVE;
  __shared__ double sT[MAXNB + MAXNB / 16];  // T_i at i + i/16 (padded against bank conflicts)
  __shared__ double xm[NW], xs[NW], xs2[NW], xv[NW], xo[2];
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  // exchange 1: the global maximum (coalesced reads)
  double m = -INFINITY;
  for (int i = threadIdx.x; i < nb; i += NT) m = fmax(m, P[3 * i]);
  m = wave_max(m);
  if (lane == 0) xm[wv] = m;
  __syncthreads();
  double M = xm[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) M = fmax(M, xm[w]);
  const bool finite = (M > -INFINITY) && (M < INFINITY);
  // block totals T_i = s_i exp(m_i - M) to LDS; sum of squares per lane
  double loc2 = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) {
    const double mb = P[3 * i];
    double T = 0.0;
    if (finite && mb > -INFINITY) {
      const double sc = exp_nonpos(mb - M);
      T = P[3 * i + 1] * sc;
      loc2 += P[3 * i + 2] * (sc * sc);
    }
    sT[i + (i >> 4)] = T;
  }
  __syncthreads();
  // each lane's contiguous chunk, summed sequentially
  const int chunk = (nb + NT - 1) / NT;
  const int i0 = min(nb, (int)threadIdx.x * chunk), i1 = min(nb, i0 + chunk);
  double loc = 0.0;
  for (int i = i0; i < i1; ++i) loc += sT[i + (i >> 4)];
  // exchange 2: scan of the lanes' sums, total of squares
  const double incl = wave_incl_scan(loc, lane);
  const double s2w = wave_sum(loc2);
  if (lane == WAVE - 1) xs[wv] = incl;
  if (lane == 0) xs2[wv] = s2w;
  __syncthreads();
  double pre = incl - loc, S = 0.0, S2 = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < wv) pre += xs[w];
    S += xs[w];
    S2 += xs2[w];
  }
  // this lane's last offset; an exact running maximum over earlier lanes
  // makes the offsets non-decreasing whatever the rounding of the scan
  double last = -INFINITY;
  {
    double run = pre;
    for (int i = i0; i < i1; ++i) {
      last = run;
      run += sT[i + (i >> 4)];
    }
  }
  const double vin = wave_incl_max_scan(last, lane);
  const double vup = wave_prev(vin, -INFINITY);
  if (lane == WAVE - 1) xv[wv] = vin;
  __syncthreads();  // exchange 3
  double vw = -INFINITY, vall = -INFINITY;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < wv) vw = fmax(vw, xv[w]);
    vall = fmax(vall, xv[w]);
  }
  const double vprev = (lane == 0) ? vw : fmax(vup, vw);
  const double Sf = fmax(S, vall);
  // the two offsets this block needs, from the lanes that own them
  const int k1e = k1b + span;
  {
    double run = pre;
    for (int i = i0; i < i1; ++i) {
      if (i == k1b) xo[0] = fmax(run, vprev);
      if (i == k1e) xo[1] = fmax(run, vprev);
      run += sT[i + (i >> 4)];
    }
  }
  if (threadIdx.x == 0 && k1e >= nb) xo[1] = Sf;
  __syncthreads();
  Combined c;
  c.M = finite ? M : -INFINITY;
  c.S = Sf;
  c.S2 = S2;
  c.lo = xo[0];
  c.hi = xo[1];
  return c;
}

// K2 (filters of more than FUSE_NB blocks): one workgroup combines the
// partials, stores the offsets, and does the filter's bookkeeping
// (likelihood increment, ESS, trigger, resampling uniform, traces,
// interval counter).
__global__ __launch_bounds__(K2_NT) void k_combine(const double* __restrict__ part,
                                                   double* __restrict__ boff, PlainArgs A) {
  constexpr int NW = K2_NT / WAVE;
  constexpr int KC = 8;  // block terms cached per lane (nb <= 8192 stays in registers)
  __shared__ double xm[NW], xs[NW], xs2[NW], xv[NW];
  const int nb = A.nblk;
  const double* P = part + 3 * A.boff0;
  double* bo = boff + A.boff0 + A.b;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const int chunk = (nb + K2_NT - 1) / K2_NT;
  const int i0 = min(nb, (int)threadIdx.x * chunk), i1 = min(nb, i0 + chunk);
  // the filter's scalars and the resampling uniform, fetched and drawn while
  // the partials load
  FilterState* fst = A.fs;
  const int t = fst->tk;  // the interval K1 just propagated
  const double loglik0 = fst->loglik;
  const double lprev0 = fst->lprev;
  const int carry0 = fst->carry;
  double u = 0.0;
  if (threadIdx.x == 0)
    u = A.mode == 2 ? fst->u
                    : u01_f64(draw(key_of(A.key), TAG_RESAMPLE, 0, fst->iter, 0, (uint32_t)t, A.b).x);
  // the lane's first KC partials, loaded together (indices past its chunk
  // reread the last block and are masked below)
  double pm[KC], ps[KC], p2[KC];
#pragma unroll
  for (int e = 0; e < KC; ++e) {
    const int i = min(i0 + e, nb - 1);
    pm[e] = P[3 * i];
    ps[e] = P[3 * i + 1];
    p2[e] = P[3 * i + 2];
  }
  // exchange 1: the global maximum
  double m = -INFINITY;
#pragma unroll
  for (int e = 0; e < KC; ++e)
    if (i0 + e < i1) m = fmax(m, pm[e]);
  for (int i = i0 + KC; i < i1; ++i) m = fmax(m, P[3 * i]);
  m = wave_max(m);
  if (lane == 0) xm[wv] = m;
  __syncthreads();
  double M = xm[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) M = fmax(M, xm[w]);
  const bool finite = (M > -INFINITY) && (M < INFINITY);
  // block totals T_i = s_i exp(m_i - M), summed sequentially within the lane;
  // the first KC of a lane's terms stay in registers (unrolled, fixed
  // indices), any further ones are recomputed
  auto term = [&](int i, double& T2) -> double {
    const double mb = P[3 * i];
    T2 = 0.0;
    if (!(finite && mb > -INFINITY)) return 0.0;
    const double sc = exp_nonpos(mb - M);
    T2 = P[3 * i + 2] * (sc * sc);
    return P[3 * i + 1] * sc;
  };
  double Tc[KC];
  double loc = 0.0, loc2 = 0.0;
#pragma unroll
  for (int e = 0; e < KC; ++e) {
    double T = 0.0, T2 = 0.0;
    if (i0 + e < i1 && finite && pm[e] > -INFINITY) {
      const double sc = exp_nonpos(pm[e] - M);
      T2 = p2[e] * (sc * sc);
      T = ps[e] * sc;
    }
    Tc[e] = T;
    loc += T;
    loc2 += T2;
  }
  for (int i = i0 + KC; i < i1; ++i) {
    double T2;
    loc += term(i, T2);
    loc2 += T2;
  }
  // exchange 2: scan of the lanes' sums, total of squares
  const double incl = wave_incl_scan(loc, lane);
  const double s2w = wave_sum(loc2);
  if (lane == WAVE - 1) xs[wv] = incl;
  if (lane == 0) xs2[wv] = s2w;
  __syncthreads();
  double pre = incl - loc, S = 0.0, S2 = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < wv) pre += xs[w];
    S += xs[w];
    S2 += xs2[w];
  }
  // this lane's last offset; an exact running maximum over earlier lanes
  // makes the offsets non-decreasing whatever the rounding of the scan
  double last = -INFINITY;
  {
    double run = pre;
#pragma unroll
    for (int e = 0; e < KC; ++e)
      if (i0 + e < i1) {
        last = run;
        run += Tc[e];
      }
    for (int i = i0 + KC; i < i1; ++i) {
      double T2;
      last = run;
      run += term(i, T2);
    }
  }
  const double vin = wave_incl_max_scan(last, lane);
  const double vup = wave_prev(vin, -INFINITY);
  if (lane == WAVE - 1) xv[wv] = vin;
  __syncthreads();  // exchange 3
  double vw = -INFINITY, vall = -INFINITY;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w < wv) vw = fmax(vw, xv[w]);
    vall = fmax(vall, xv[w]);
  }
  const double vprev = (lane == 0) ? vw : fmax(vup, vw);
  {
    double run = pre;
#pragma unroll
    for (int e = 0; e < KC; ++e)
      if (i0 + e < i1) {
        bo[i0 + e] = fmax(run, vprev);
        run += Tc[e];
      }
    for (int i = i0 + KC; i < i1; ++i) {
      double T2;
      bo[i] = fmax(run, vprev);
      run += term(i, T2);
    }
  }
  const double Sf = fmax(S, vall);
  if (threadIdx.x == 0) {
    bo[nb] = Sf;
    FilterState* f = fst;
    double ell, ess;
    // the factor's normaliser: ln N after a resampling, else the carried
    // weights' ln sum exp
    const double lprev = carry0 ? lprev0 : log((double)A.N);
    int carry = 0;
    if (finite && Sf > 0.0) {
      const double L = M + log(Sf);
      ell = L - lprev;
      ess = (Sf * Sf) / S2;
      carry = !(ess < A.rs.ess_frac * (double)A.N);  // resample when ESS < ess_frac N
      f->lprev = L;
    } else {
      ell = -INFINITY;
      ess = 0.0;
      f->status = 4;
    }
    f->carry = carry;
    f->loglik = loglik0 + ell;
    f->M = finite ? M : -INFINITY;
    f->S = Sf;
    f->ell = ell;
    f->ess = ess;
    f->u = u;
    A.ell_tr[t - 1] = ell;
    A.ess_tr[t - 1] = ess;
    f->t = t;
  }
}


// ---------------------------------------------------------------- K1
// Observation log-density of one particle, in FP64 from the (FP32 or FP64)
// state: the residuals are formed after widening the state, so an FP32 path
// adds no rounding of its own here (a log-weight stored in FP32 would carry
// ~2^-24 |lw|, above the per-step accuracy once |lw| reaches the hundreds).
// Components are visited in increasing index, the order of the sorted
// observation list.
template <int D, typename Real>
__device__ __forceinline__ double l96_logdens(const Real (&x)[D], const double* yrow,
                                              const int32_t* obs_pos, double inv_sd,
                                              double cst) {
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const int o = obs_pos[i];
    if (o >= 0) {
      const double e = (yrow[o] - (double)x[i]) * inv_sd;
      acc = acc + e * e;
    }
  }
  return -0.5 * acc + cst;
}

// The particle output j continues in this interval (plain layout, every
// thread of a K1 block calls it: it has a barrier): the identity, the
// ancestor array, or, after a systematic or stratified collective, the
// running maximum of the marks over the block's tile (one tile of K4_TILE =
// K1_NT outputs per block) started from the tile's owner, as the tile
// gather forms it; those marks are cleared for the next collective and the
// ancestors written out.  Outputs past the filter's strata (rounding) go to
// the last particle of positive weight.
__device__ __forceinline__ int64_t plain_ancestor(int64_t j, int32_t* __restrict__ marks_all,
                                                  const int32_t* __restrict__ owner_all,
                                                  const int32_t* __restrict__ jc_all,
                                                  int32_t* __restrict__ anc,
                                                  const PlainArgs& A, int32_t* wtop,
                                                  int32_t* s_js) {
  const int32_t amode = A.fs->amode;
  const int64_t N = A.N;
  if (amode == AMODE_IDENTITY) return j;
  if (amode == AMODE_ARRAY) return j < N ? (int64_t)anc[A.off + j] : j;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const int64_t k0 = (int64_t)blockIdx.x * K1_NT;
  const int64_t cn1 = A.fs->cn1;
  if (threadIdx.x < WAVE) {
    int found = -1;
    if (k0 + K1_NT > cn1 && cn1 < N) {
      const int nb3 = (int)((N + K3_SPAN - 1) / K3_SPAN);
      for (int base = nb3 - 1; base >= 0 && found < 0; base -= WAVE) {
        const int i = base - (int)threadIdx.x;
        found = wave_max_i(i >= 0 ? jc_all[A.own0 + i] : -1);
      }
    }
    if (threadIdx.x == 0) *s_js = found;
  }
  int32_t* marks = marks_all + A.off;
  int32_t run = k0 < cn1 ? owner_all[A.own0 + blockIdx.x] : -1;
  if (j < N) {
    run = max(run, marks[j]);
    marks[j] = -1;
  }
  const int32_t incl = wave_incl_max_scan_i(run, lane);
  if (lane == WAVE - 1) wtop[wv] = incl;
  __syncthreads();
  int32_t excl = -1;
#pragma unroll
  for (int w = 0; w < K1_NT / WAVE; ++w)
    if (w < wv) excl = max(excl, wtop[w]);
  if (j >= N) return j;
  int32_t a = j < cn1 ? max(excl, incl) : *s_js;
  if (a < 0 || a >= N) {  // never expected; flagged, and kept in bounds
    atomicOr(&A.fs->pad, 1);
    a = 0;
  }
  anc[A.off + j] = a;
  return a;
}

template <int MODEL, int D, typename Real, bool ACC = false>
__global__ __launch_bounds__(K1_NT) void k_propagate_weight(Real* __restrict__ xa,
                                                            Real* __restrict__ xb,
                                                            double* __restrict__ lw,
                                                            double* __restrict__ part,
                                                            int32_t* __restrict__ marks,
                                                            const int32_t* __restrict__ owner,
                                                            const int32_t* __restrict__ jc,
                                                            int32_t* __restrict__ anc,
                                                            PlainArgs A) {
  __shared__ double red[K1_NT / WAVE];
  __shared__ int32_t wtop[K1_NT / WAVE];
  __shared__ int32_t s_js;
  const int64_t j = (int64_t)blockIdx.x * K1_NT + threadIdx.x;
  const int t = A.fs->t + 1;
  const uint32_t iter = A.fs->iter;
  const Key key = key_of(A.key);
  // interval t gathers buffer (t - 1) % 2 and writes buffer t % 2
  const Real* __restrict__ xcur = ((t - 1) & 1) ? xb : xa;
  Real* __restrict__ xprop = (t & 1) ? xb : xa;
  const int64_t src = A.off + plain_ancestor(j, marks, owner, jc, anc, A, wtop, &s_js);
  double l = -INFINITY;
  if (j < A.N) {
    const int64_t col = A.off + j;
    const double* yrow = A.obs + (int64_t)(t - 1) * A.n_obs;
    const int n0 = (t - 1) * A.K;
    if constexpr (MODEL == 1) {
      if constexpr (sizeof(Real) == 8) {
        double p = xcur[src];
        for (int s = 1; s <= A.K; ++s) {
          const uint4 w = draw(key, TAG_NOISE, 0, iter, (uint32_t)j, (uint32_t)(n0 + s), A.b);
          double z0, z1;
          bm_pair_f64(w.x, w.y, z0, z1);
          p = wk_substep_f64(p, A.theta, A.q[n0 + s - 1], z0);
        }
        xprop[col] = p;
        const double e = (yrow[0] - (p + A.theta[2] * A.q[(int64_t)t * A.K])) * A.inv_sd;
        l = -0.5 * (e * e) + A.lw_cst;
      } else {
        float p = xcur[src];
        double pa = p;  // the accurate form carries the pressure in FP64
        const float a = (float)(A.theta[0] - 1.0), c = (float)A.theta[1], sp = (float)A.theta[3];
        for (int s = 1; s <= A.K; ++s) {
          const uint4 w = draw(key, TAG_NOISE, 0, iter, (uint32_t)j, (uint32_t)(n0 + s), A.b);
          float z0, z1;
          bm_pair_f32(w.x, w.y, z0, z1);
          if constexpr (ACC) {
            pa = pa + (double)wk_increment_f32((float)pa, a, c, sp, (float)A.q[n0 + s - 1], z0);
          } else {
            p = wk_substep_f32(p, a, c, sp, (float)A.q[n0 + s - 1], z0);
          }
        }
        if constexpr (ACC) p = (float)pa;
        else pa = p;
        xprop[col] = p;
        const double e = (yrow[0] - (pa + A.theta[2] * A.q[(int64_t)t * A.K])) * A.inv_sd;
        l = -0.5 * (e * e) + A.lw_cst;
      }
    } else {
      Real x[D];
#pragma unroll
      for (int i = 0; i < D; ++i) x[i] = xcur[pidx(src, i, D)];
      if constexpr (sizeof(Real) == 8) {
        const double F = A.theta[0], sq = A.theta[1];
        ModelConsts mc{A.h, A.hh, A.h6, A.inv_sd, A.lw_cst};
        for (int s = 1; s <= A.K; ++s) {
          if constexpr (MODEL == 3)
            l96_substep_stage_f64<D>(x, F, sq, mc, key, TAG_NOISE, iter, (uint32_t)j,
                                     (uint32_t)(n0 + s), A.b);
          else
            l96_substep_f64<D>(x, F, sq, mc, key, TAG_NOISE, iter, (uint32_t)j,
                               (uint32_t)(n0 + s), A.b);
        }
      } else if constexpr (ACC) {
        double xa[D];
#pragma unroll
        for (int i = 0; i < D; ++i) xa[i] = (double)x[i];
        const L96F32A c = l96_f32a_consts(A.theta[0], A.theta[1], A.h);
        for (int s = 1; s <= A.K; ++s) {
          if constexpr (MODEL == 3)
            l96_substep_stage_f32acc<D>(xa, c, key, TAG_NOISE, iter, (uint32_t)j,
                                        (uint32_t)(n0 + s), A.b);
          else
            l96_substep_f32acc<D>(xa, c, key, TAG_NOISE, iter, (uint32_t)j, (uint32_t)(n0 + s),
                                  A.b);
        }
#pragma unroll
        for (int i = 0; i < D; ++i) xprop[pidx(col, i, D)] = (Real)xa[i];
        // the log-weight from the state before it is rounded for storage
        l = l96_logdens<D, double>(xa, yrow, A.obs_pos, A.inv_sd, A.lw_cst);
      } else {
        const L96F32 c = l96_f32_consts(A.theta[0], A.theta[1], A.h);
        for (int s = 1; s <= A.K; ++s) {
          if constexpr (MODEL == 3)
            l96_substep_stage_f32<D>(x, c, key, TAG_NOISE, iter, (uint32_t)j, (uint32_t)(n0 + s),
                                     A.b);
          else
            l96_substep_f32<D>(x, c, key, TAG_NOISE, iter, (uint32_t)j, (uint32_t)(n0 + s), A.b);
        }
      }
      if constexpr (!ACC || sizeof(Real) == 8) {
#pragma unroll
        for (int i = 0; i < D; ++i) xprop[pidx(col, i, D)] = x[i];
        l = l96_logdens<D, Real>(x, yrow, A.obs_pos, A.inv_sd, A.lw_cst);
      }
    }
    // weights kept from a step that did not resample carry over
    if (A.fs->carry) l = lw[col] + l;
    lw[col] = l;
  }
  // a NaN log-weight counts as zero weight
  const double lc = (l == l) ? l : -INFINITY;
  const double m = block_max<K1_NT>(lc, red);
  const double e = (m > -INFINITY && m < INFINITY) ? exp_nonpos(lc - m) : 0.0;
  const double s1 = block_sum<K1_NT>(e, red);
  const double s2 = block_sum<K1_NT>(e * e, red);
  if (threadIdx.x == 0) {
    double* p = part + 3 * (A.boff0 + blockIdx.x);
    p[0] = m;
    p[1] = s1;
    p[2] = s2;
    // the interval K3 processes (it must not read the counter it advances)
    if (blockIdx.x == 0) A.fs->tk = t;
  }
}

// Block partials (max, sum, sum of squares of exp(lw - max)) of caller-given
// FP64 log-weights, the reduction K1 ends with; block 0 publishes the
// interval index as K1 does.
__global__ __launch_bounds__(K1_NT) void k_lw_partials(const double* __restrict__ lw,
                                                       double* __restrict__ part, PlainArgs A) {
  __shared__ double red[K1_NT / WAVE];
  const int64_t j = (int64_t)blockIdx.x * K1_NT + threadIdx.x;
  const double l = j < A.N ? lw[A.off + j] : -INFINITY;
  const double lc = (l == l) ? l : -INFINITY;  // a NaN log-weight counts as zero weight
  const double m = block_max<K1_NT>(lc, red);
  const double e = (m > -INFINITY && m < INFINITY) ? exp_nonpos(lc - m) : 0.0;
  const double s1 = block_sum<K1_NT>(e, red);
  const double s2 = block_sum<K1_NT>(e * e, red);
  if (threadIdx.x == 0) {
    double* p = part + 3 * (A.boff0 + blockIdx.x);
    p[0] = m;
    p[1] = s1;
    p[2] = s2;
    if (blockIdx.x == 0) A.fs->tk = A.fs->t + 1;
  }
}

__global__ void k_set_u(FilterState* fs, double u) {
  if (threadIdx.x == 0 && blockIdx.x == 0) fs->u = u;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- K3
// W_j = boff[blk] + (block-local inclusive scan of exp(lw - M)), made
// non-decreasing by an exact running maximum and capped by boff[blk+1]; then
// c_j = #{k : (u + k) S < N W_j}, the number of strata owned by particles
// 0..j, so particle j owns strata [c_{j-1}, c_j).  Each particle that owns
// any marks the first of them with its index (one store per particle, no
// loop over its offspring); the owner of every K4 tile's first stratum is
// stored by the particle whose strata cover it, so K4 can name every
// stratum's owner from its tile's marks alone.  At a block edge the strata
// between the block's last count and g = count(boff[blk+1]) belong to the
// next block's first particle; the block's last lane records them, because
// only it knows that count.  Strata past the last particle's count (rounding
// overflow) go to the last particle of positive weight (jstar).
template <bool FUSED>
__global__ __launch_bounds__(K3_NT) void k_scan_mark(const double* __restrict__ lw,
                                                     const double* __restrict__ part,
                                                     const double* __restrict__ boff,
                                                     int32_t* __restrict__ marks_all,
                                                     int32_t* __restrict__ owner_all,
                                                     int32_t* __restrict__ jc_all,
                                                     PlainArgs A) {
  constexpr int NW = K3_NT / WAVE;
  __shared__ double xsum[NW], xvmax[NW];
  __shared__ int64_t xcnt[NW];
  __shared__ int xcand[NW];
  const int64_t N = A.N;
  const int64_t jb = (int64_t)blockIdx.x * K3_SPAN;
  const int64_t j0 = jb + (int64_t)threadIdx.x * K3_PER;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  // the lane's K3_PER consecutive log-weights, loaded first so that they
  // arrive while the partials are combined (past the end they reread the
  // last weight)
  double lv[K3_PER];
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) lv[e] = lw[A.off + min(j0 + e, N - 1)];
  FilterState* fst = A.fs;
  const int32_t t_now = fst->tk;  // the interval K1 just propagated
  const uint32_t it_now = fst->iter;
  const Key key = key_of(A.key);
  const int k1b = (int)blockIdx.x * (K3_SPAN / K1_NT);  // first K1 block of this block
  double M, S, u, lo_off, hi_off;
  bool pos, carry;
  if constexpr (FUSED) {
    // mode 0 draws the resampling uniform (while the partials load); modes 1
    // and 2 take the uniform already in the filter's scalars (1 redraws only
    // the ancestors, 2 also does the bookkeeping)
    u = A.mode == 0 ? u01_f64(draw(key, TAG_RESAMPLE, 0, it_now, 0, (uint32_t)t_now, A.b).x)
                    : fst->u;
    const Combined cb =
        combine_block_lds<K3_NT, FUSE_NB>(part + 3 * A.boff0, A.nblk, k1b, K3_SPAN / K1_NT);
    M = cb.M;
    S = cb.S;
    lo_off = cb.lo;
    hi_off = cb.hi;
    pos = (M > -INFINITY) && (M < INFINITY) && (S > 0.0);
    const double ess = pos ? (S * S) / cb.S2 : 0.0;
    // resample when ESS < ess_frac N
    carry = pos && !(ess < A.rs.ess_frac * (double)N);
    if (A.mode != 1 && blockIdx.x == 0 && threadIdx.x == 0) {
      // the filter's bookkeeping: likelihood increment (the normaliser is
      // ln N after a resampling, else the carried weights' ln sum exp), ESS,
      // trigger, uniform, traces, and the interval counter
      const double lprev = fst->carry ? fst->lprev : log((double)N);
      double ell;
      if (pos) {
        const double L = M + log(S);
        ell = L - lprev;
        fst->lprev = L;
      } else {
        ell = -INFINITY;
        fst->status = 4;
      }
      fst->carry = carry;
      fst->loglik = fst->loglik + ell;
      fst->M = M;
      fst->S = S;
      fst->ell = ell;
      fst->ess = ess;
      fst->u = u;
      A.ell_tr[t_now - 1] = ell;
      A.ess_tr[t_now - 1] = ess;
      fst->t = t_now;
    }
  } else {
    // K2 has combined the partials and done the bookkeeping
    M = fst->M;
    S = fst->S;
    u = fst->u;
    pos = (M > -INFINITY) && (M < INFINITY) && (S > 0.0);
    carry = fst->carry;
    const double* bo = boff + A.boff0 + A.b;
    lo_off = bo[k1b];
    hi_off = bo[min(k1b + K3_SPAN / K1_NT, A.nblk)];
  }
  // no cumulative weights needed
  if (A.rs.scheme == RS_METROPOLIS || A.rs.scheme == RS_REJECTION) return;
  // a step that keeps its weights (ESS above the trigger) or has none
  // positive gives every particle one offspring: itself
  const bool finite = pos && !carry;
  const double invS = 1.0 / S;
  const bool strat = A.rs.scheme == RS_STRATIFIED;
  auto count = [&](double W) -> int64_t {
    return strat ? stratum_count_strat(W, S, invS, (int32_t)N, key, t_now, A.b, it_now)
                 : stratum_count(W, S, invS, u, (int32_t)N);
  };
  // in-lane sequential prefix of K3_PER consecutive weights, and the lane's
  // last particle of positive weight (for the rare case where rounding
  // leaves the final strata without an owner)
  double w[K3_PER], loc[K3_PER];
  double run = 0.0;
  int cand = -1;
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) {
    const int64_t j = j0 + e;
    double we = 0.0;
    if (j < N && finite) {
      const double l = lv[e];
      we = (l == l) ? exp_nonpos(l - M) : 0.0;
    }
    w[e] = we;
    if (we > 0.0) cand = (int)j;
    run += we;
    loc[e] = run;
  }
  // exchange 1: the lanes' sums scanned across the block (and the block's
  // candidate, which only lane 0 needs)
  const double incl = wave_incl_scan(run, lane);
  const int cw = wave_max_i(cand);
  if (lane == WAVE - 1) xsum[wv] = incl;
  if (lane == 0) xcand[wv] = cw;
  __syncthreads();
  double pre = incl - run;
#pragma unroll
  for (int q = 0; q < NW; ++q)
    if (q < wv) pre += xsum[q];
  double V[K3_PER];
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) V[e] = lo_off + (pre + loc[e]);
  // exchange 2: an exact running maximum over earlier lanes keeps W
  // non-decreasing across lanes whatever the rounding of the tree scan;
  // capped by the next offset
  const double vin = wave_incl_max_scan(V[K3_PER - 1], lane);
  const double vup = wave_prev(vin, -INFINITY);
  if (lane == WAVE - 1) xvmax[wv] = vin;
  __syncthreads();
  double vw = -INFINITY;
#pragma unroll
  for (int q = 0; q < NW; ++q)
    if (q < wv) vw = fmax(vw, xvmax[q]);
  const double vprev = lane > 0 ? fmax(vup, vw) : (wv > 0 ? vw : lo_off);
  int64_t c[K3_PER];
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) {
    const int64_t j = j0 + e;
    const double W = fmin(fmax(V[e], vprev), hi_off);
    c[e] = (j < N) ? (finite ? count(W) : j + 1) : 0;
    if (A.rs.scheme == RS_MULTINOMIAL && j < N) A.wcum[j] = W;
  }
  // the strata counts at this block's edges (the same function of the same
  // offset values as the neighbouring blocks compute)
  const int64_t g_lo = finite ? count(lo_off) : jb;
  const int64_t jnext = jb + K3_SPAN;
  const int64_t g_hi = (jnext < N) ? (finite ? count(hi_off) : jnext) : N;
  // exchange 3: each lane's first particle continues from the previous
  // lane's last count
  const int64_t cup = wave_prev_i64(c[K3_PER - 1], 0);
  if (lane == WAVE - 1) xcnt[wv] = c[K3_PER - 1];
  __syncthreads();
  int64_t cprev = lane > 0 ? cup : (wv > 0 ? xcnt[wv - 1] : g_lo);
  // strata [rlo, rhi) owned by particle rj: one range per particle, plus,
  // for the block's last particle, the strata below the next block's first
  // count, which belong to the next block's first particle
  int64_t rj[K3_PER + 1], rlo[K3_PER + 1], rhi[K3_PER + 1];
#pragma unroll
  for (int e = 0; e <= K3_PER; ++e) {
    rj[e] = 0;
    rlo[e] = 0;
    rhi[e] = 0;  // empty
  }
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) {
    const int64_t j = j0 + e;
    if (j < N) {
      rj[e] = j;
      rlo[e] = cprev;
      rhi[e] = c[e];
      if (j == N - 1) {
        fst->cn1 = (int32_t)c[e];
      } else if (j == jnext - 1) {
        rj[K3_PER] = j + 1;
        rlo[K3_PER] = c[e];
        rhi[K3_PER] = g_hi;
      }
    }
    cprev = c[e];
  }
  if (A.rs.scheme != RS_MULTINOMIAL) {
    int32_t* marks = marks_all + A.off;
    int32_t* owner = owner_all + A.own0;
    if (threadIdx.x == 0) fst->amode = AMODE_MARKS;  // the next propagation reads them
#pragma unroll
    for (int e = 0; e <= K3_PER; ++e)
      if (rlo[e] < rhi[e]) marks[rlo[e]] = (int32_t)rj[e];
    // Tile q's first stratum q K4_TILE lies in at most one range.  A range
    // covering at most two tile starts is stored by its lane; a longer one
    // (a particle owning many strata) by the whole wave, strided over the
    // lanes, so no lane loops over hundreds of tiles.
#pragma unroll
    for (int e = 0; e <= K3_PER; ++e) {
      const int64_t first = (rlo[e] + K4_TILE - 1) / K4_TILE;
      const int64_t last = rhi[e] > rlo[e] ? (rhi[e] - 1) / K4_TILE : first - 1;
      const bool big = last - first + 1 > 2;
      if (!big)
        for (int64_t q = first; q <= last; ++q) owner[q] = (int32_t)rj[e];
      uint64_t mask = __ballot(big);
      while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const long long bj = __shfl((long long)rj[e], src, WAVE);
        const long long bq0 = __shfl((long long)first, src, WAVE);
        const long long bq1 = __shfl((long long)last, src, WAVE);
        for (long long q = bq0 + lane; q <= bq1; q += WAVE) owner[q] = (int32_t)bj;
      }
    }
  }
  if (threadIdx.x == 0) {
    int cb = xcand[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) cb = max(cb, xcand[q]);
    jc_all[A.own0 + blockIdx.x] = cb;
  }
}

// ---------------------------------------------------------------- K4
// The resampled set, on demand (the stepping path never runs this: the next
// propagation gathers through the pending ancestors itself).  One block per
// tile of K4_TILE outputs: with marks pending, a running maximum over the
// tile's marks (which it clears), started from the owner of the tile's
// first stratum, names each output's ancestor (outputs past the strata take
// the last particle of positive weight); with the identity or the ancestor
// array pending, those.  The ancestors are written out, and with buffers
// given, buffer t % 2 (t = fs->t) is gathered through them into buffer
// (t + 1) % 2.
template <int D, typename Real>
__global__ __launch_bounds__(K4_NT) void k_tile_gather(int32_t* __restrict__ marks_all,
                                                       const int32_t* __restrict__ owner_all,
                                                       const int32_t* __restrict__ jc_all,
                                                       Real* __restrict__ xa,
                                                       Real* __restrict__ xb,
                                                       int32_t* __restrict__ anc,
                                                       PlainArgs A) {
  static_assert(K4_PER == 1 && K4_NT == K1_NT, "one output per lane, one tile per block");
  __shared__ int32_t wtop[K4_NT / WAVE];
  __shared__ int32_t s_js;
  const int64_t k = (int64_t)blockIdx.x * K4_TILE + threadIdx.x;
  const int64_t a = plain_ancestor(k, marks_all, owner_all, jc_all, anc, A, wtop, &s_js);
  if (k >= A.N) return;
  anc[A.off + k] = (int32_t)a;
  if (xa == nullptr) return;
  const int t = A.fs->t;
  const Real* __restrict__ xprop = (t & 1) ? xb : xa;
  Real* __restrict__ xout = (t & 1) ? xa : xb;
  const int64_t src = A.off + a, dst = A.off + k;
  if constexpr (D > 0) {
#pragma unroll
    for (int i = 0; i < D; ++i) xout[pidx(dst, i, D)] = xprop[pidx(src, i, D)];
  } else {
    for (int i = 0; i < A.d; ++i) xout[pidx(dst, i, A.d)] = xprop[pidx(src, i, A.d)];
  }
}

__global__ void k_set_amode(FilterState* fs, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) fs[i].amode = v;
}

// ---------------------------------------------------------------- Metropolis resampling
// A resampler without the collective over the weights: output k starts at
// particle k and takes A.rs.steps Metropolis moves with uniform proposals,
// reading the FP64 log-weights directly (a NaN counts as -inf).  A step that
// keeps its weights, or has none positive, gives the identity.
__global__ __launch_bounds__(K1_NT) void k_metropolis(const double* __restrict__ lw,
                                                      int32_t* __restrict__ anc, PlainArgs A) {
  const int64_t k = (int64_t)blockIdx.x * K1_NT + threadIdx.x;
  if (k >= A.N) return;
  const FilterState* f = A.fs;
  const bool draw_rs = (f->M > -INFINITY) && (f->M < INFINITY) && (f->S > 0.0) && !f->carry;
  const double* l = lw + A.off;
  const int32_t N = (int32_t)A.N;
  int32_t j = (int32_t)k;
  if (draw_rs) {
    const Key key = key_of(A.key);
    const int32_t t = f->t;
    const uint32_t it = f->iter;
    double lj = l[j];
    lj = (lj == lj) ? lj : -INFINITY;
    for (int s = 1; s <= A.rs.steps; s += 2) {
      const uint4 w = metro_draw(key, t, A.b, it, (int32_t)k, s);
      int32_t jp = metro_index(w.x, N);
      double lp = l[jp];
      lp = (lp == lp) ? lp : -INFINITY;
      if (ln_f64(u01_f64(w.y)) <= lp - lj) {
        j = jp;
        lj = lp;
      }
      if (s + 1 <= A.rs.steps) {
        jp = metro_index(w.z, N);
        lp = l[jp];
        lp = (lp == lp) ? lp : -INFINITY;
        if (ln_f64(u01_f64(w.w)) <= lp - lj) {
          j = jp;
          lj = lp;
        }
      }
    }
  }
  anc[A.off + k] = j;
  if (k == 0) A.fs->amode = AMODE_ARRAY;
}

// ---------------------------------------------------------------- rejection resampling
// Needs the largest log-weight (from the step's reduction) but no scan:
// output k tries candidates, k first, then uniform draws, until one passes
// ln u <= lw_j - M.  A step that keeps its weights, or has none positive,
// gives the identity.
__global__ __launch_bounds__(K1_NT) void k_rejection(const double* __restrict__ lw,
                                                     int32_t* __restrict__ anc, PlainArgs A) {
  const int64_t k = (int64_t)blockIdx.x * K1_NT + threadIdx.x;
  if (k >= A.N) return;
  const FilterState* f = A.fs;
  const double M = f->M;
  const bool draw_rs = (M > -INFINITY) && (M < INFINITY) && (f->S > 0.0) && !f->carry;
  const double* l = lw + A.off;
  int32_t j = (int32_t)k;
  if (draw_rs)
    j = reject_ancestor(key_of(A.key), f->t, A.b, f->iter, (int32_t)k, (int32_t)A.N, M,
                        [&](int32_t i) { return l[i]; });
  anc[A.off + k] = j;
  if (k == 0) A.fs->amode = AMODE_ARRAY;
}

// Multinomial resampling, as Alg. 2 writes it: output k takes
// a_k = min{j : W_j > u_k S} for an independent uniform u_k, by binary
// search of the cumulative weights K3 left (exactly non-decreasing);
// rounding overflow goes to the last positive weight (found by K3).  A step that keeps its weights, or has none positive, gives
// the identity.
__global__ __launch_bounds__(K1_NT) void k_multinomial(const double* __restrict__ wcum,
                                                       const int32_t* __restrict__ jc_all,
                                                       int32_t* __restrict__ anc, PlainArgs A) {
  const int64_t k = (int64_t)blockIdx.x * K1_NT + threadIdx.x;
  if (k >= A.N) return;
  const FilterState* f = A.fs;
  const double S = f->S;
  const bool draw_rs = (f->M > -INFINITY) && (f->M < INFINITY) && (S > 0.0) && !f->carry;
  int64_t a = k;
  if (draw_rs) {
    const double thr = multi_u(key_of(A.key), f->t, A.b, f->iter, (int32_t)k) * S;
    int64_t lo = 0, hi = A.N;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (wcum[mid] > thr) hi = mid;
      else lo = mid + 1;
    }
    if (lo < A.N) {
      a = lo;
    } else {
      int32_t js = -1;
      for (int i = (int)((A.N + K3_SPAN - 1) / K3_SPAN) - 1; i >= 0 && js < 0; --i)
        js = jc_all[A.own0 + i];
      a = js >= 0 ? js : 0;
    }
  }
  anc[A.off + k] = (int32_t)a;
  if (k == 0) A.fs->amode = AMODE_ARRAY;
}

// ---------------------------------------------------------------- simulator
template <int MODEL, int D>
__global__ void k_simulate(double* __restrict__ out, PlainArgs A, double obs_sd) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const Key key = key_of(A.key);
  double x[D];
  if (MODEL == 1) {
    double z0, z1;
    const uint4 w = draw(key, TAG_DATA, 0, 0, 0, 0, 0);
    bm_pair_f64(w.x, w.y, z0, z1);
    x[0] = A.theta[4] + A.theta[5] * z0;
  } else {
    for (int blk = 0; blk < D / 4; ++blk) {
      double z[4];
      normals4_f64(draw(key, TAG_DATA, blk, 0, 0, 0, 0), z);
      for (int m = 0; m < 4; ++m) x[4 * blk + m] = z[m];
    }
  }
  for (int i = 0; i < D; ++i) out[i] = x[i];
  double* obs = out + (int64_t)(A.T + 1) * D;
  ModelConsts mc{A.h, A.hh, A.h6, A.inv_sd, A.lw_cst};
  for (int t = 1; t <= A.T; ++t) {
    for (int s = 1; s <= A.K; ++s) {
      const int n = (t - 1) * A.K + s;
      if (MODEL == 1) {
        double z0, z1;
        const uint4 w = draw(key, TAG_DATA, 0, 0, 0, (uint32_t)n, 0);
        bm_pair_f64(w.x, w.y, z0, z1);
        x[0] = wk_substep_f64(x[0], A.theta, A.q[n - 1], z0);
      } else {
        if constexpr (MODEL == 3)
          l96_substep_stage_f64<D>(x, A.theta[0], A.theta[1], mc, key, TAG_DATA, 0, 0,
                                   (uint32_t)n, 0);
        else
          l96_substep_f64<D>(x, A.theta[0], A.theta[1], mc, key, TAG_DATA, 0, 0, (uint32_t)n, 0);
      }
    }
    for (int i = 0; i < D; ++i) out[(int64_t)t * D + i] = x[i];
    for (int o = 0; o < A.n_obs; ++o) {
      double z[4];
      normals4_f64(draw(key, TAG_OBS, (uint32_t)(o / 4), 0, 0, (uint32_t)t, 0), z);
      const double mu = (MODEL == 1) ? x[0] + A.theta[2] * A.q[(int64_t)t * A.K]
                                     : x[A.obs_idx[o]];
      obs[(int64_t)(t - 1) * A.n_obs + o] = mu + obs_sd * z[o % 4];
    }
  }
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblocks(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

#define PF_L96_DIMS(X) X(4) X(8) X(16) X(32) X(40)

hipError_t launch_init(int model, int d, int prec, void* x, const PlainArgs& a, hipStream_t s) {
  const unsigned g = nblocks(a.N, K1_NT);
  if (model == 1) {
    if (prec == 0)
      hipLaunchKernelGGL((k_init<1, 1, double>), g, K1_NT, 0, s, (double*)x, a);
    else
      hipLaunchKernelGGL((k_init<1, 1, float>), g, K1_NT, 0, s, (float*)x, a);
    return hipGetLastError();
  }
  switch (d) {
#define X(DD)                                                                          \
  case DD:                                                                             \
    if (prec == 0)                                                                     \
      hipLaunchKernelGGL((k_init<2, DD, double>), g, K1_NT, 0, s, (double*)x, a);      \
    else                                                                               \
      hipLaunchKernelGGL((k_init<2, DD, float>), g, K1_NT, 0, s, (float*)x, a);        \
    break;
    PF_L96_DIMS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reset(FilterState* fs, double* ell, double* ess, int B, int T, uint32_t iter,
                        hipStream_t s) {
  const int64_t n = (int64_t)B * T > B ? (int64_t)B * T : B;
  hipLaunchKernelGGL(k_reset, nblocks(n, 256), 256, 0, s, fs, ell, ess, B, T, iter);
  return hipGetLastError();
}

hipError_t launch_propagate(int model, int d, int prec, void* xa, void* xb, void* lw,
                            double* part, int32_t* marks, const int32_t* owner,
                            const int32_t* jc, int32_t* anc, const PlainArgs& a, hipStream_t s) {
  const unsigned g = (unsigned)a.nblk;
  if (model == 1) {
    if (prec == 0)
      hipLaunchKernelGGL((k_propagate_weight<1, 1, double>), g, K1_NT, 0, s,
                         (double*)xa, (double*)xb, (double*)lw, part, marks, owner, jc, anc, a);
    else if (prec == 1)
      hipLaunchKernelGGL((k_propagate_weight<1, 1, float>), g, K1_NT, 0, s,
                         (float*)xa, (float*)xb, (double*)lw, part, marks, owner, jc, anc, a);
    else
      hipLaunchKernelGGL((k_propagate_weight<1, 1, float, true>), g, K1_NT, 0, s,
                         (float*)xa, (float*)xb, (double*)lw, part, marks, owner, jc, anc, a);
    return hipGetLastError();
  }
  switch (d * 4 + model) {
#define X(DD)                                                                             \
  case DD * 4 + 2:                                                                        \
    if (prec == 0)                                                                        \
      hipLaunchKernelGGL((k_propagate_weight<2, DD, double>), g, K1_NT, 0, s,             \
                         (double*)xa, (double*)xb, (double*)lw, part, marks, owner, jc, anc, a);      \
    else if (prec == 1)                                                                   \
      hipLaunchKernelGGL((k_propagate_weight<2, DD, float>), g, K1_NT, 0, s,              \
                         (float*)xa, (float*)xb, (double*)lw, part, marks, owner, jc, anc, a);        \
    else                                                                                  \
      hipLaunchKernelGGL((k_propagate_weight<2, DD, float, true>), g, K1_NT, 0, s,        \
                         (float*)xa, (float*)xb, (double*)lw, part, marks, owner, jc, anc, a);        \
    break;                                                                                \
  case DD * 4 + 3:                                                                        \
    if (prec == 0)                                                                        \
      hipLaunchKernelGGL((k_propagate_weight<3, DD, double>), g, K1_NT, 0, s,             \
                         (double*)xa, (double*)xb, (double*)lw, part, marks, owner, jc, anc, a);      \
    else if (prec == 1)                                                                   \
      hipLaunchKernelGGL((k_propagate_weight<3, DD, float>), g, K1_NT, 0, s,              \
                         (float*)xa, (float*)xb, (double*)lw, part, marks, owner, jc, anc, a);        \
    else                                                                                  \
      hipLaunchKernelGGL((k_propagate_weight<3, DD, float, true>), g, K1_NT, 0, s,        \
                         (float*)xa, (float*)xb, (double*)lw, part, marks, owner, jc, anc, a);        \
    break;
    PF_L96_DIMS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_set_u(FilterState* fs, double u, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u, 1, 64, 0, s, fs, u);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, nblocks(n, 256), 256, 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_lw_partials(const double* lw, double* part, const PlainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_lw_partials, nblocks(a.N, K1_NT), K1_NT, 0, s, lw, part, a);
  return hipGetLastError();
}

hipError_t launch_tile_anc(int32_t* marks, const int32_t* owner, const int32_t* jc, int32_t* anc,
                           const PlainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_tile_gather<0, float>), nblocks(a.N, K4_TILE), K4_NT, 0, s, marks, owner,
                     jc, (float*)nullptr, (float*)nullptr, anc, a);
  return hipGetLastError();
}

hipError_t launch_set_amode(FilterState* fs, int n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_amode, (unsigned)((n + 255) / 256), 256, 0, s, fs, n, v);
  return hipGetLastError();
}

hipError_t launch_combine(const double* part, double* boff, const PlainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, 1, K2_NT, 0, s, part, boff, a);
  return hipGetLastError();
}

hipError_t launch_scan_mark(const double* lw, const double* part, const double* boff,
                            int32_t* marks, int32_t* owner, int32_t* jc, const PlainArgs& a,
                            hipStream_t s) {
  const unsigned g = nblocks(a.N, K3_SPAN);
  if (a.nblk <= FUSE_NB)
    hipLaunchKernelGGL(k_scan_mark<true>, g, K3_NT, 0, s, lw, part, boff, marks, owner, jc, a);
  else
    hipLaunchKernelGGL(k_scan_mark<false>, g, K3_NT, 0, s, lw, part, boff, marks, owner, jc, a);
  return hipGetLastError();
}

hipError_t launch_tile_gather(int model, int d, int prec, int32_t* marks, const int32_t* owner,
                              const int32_t* jc, void* xa, void* xb, int32_t* anc,
                              const PlainArgs& a, hipStream_t s) {
  const unsigned g = nblocks(a.N, K4_TILE);
  const int dd = model == 1 ? 1 : d;
  switch (dd) {
#define X(DD)                                                                               \
  case DD:                                                                                  \
    if (prec == 0)                                                                          \
      hipLaunchKernelGGL((k_tile_gather<DD, double>), g, K4_NT, 0, s, marks, owner, jc,      \
                         (double*)xa, (double*)xb, anc, a);                                 \
    else                                                                                    \
      hipLaunchKernelGGL((k_tile_gather<DD, float>), g, K4_NT, 0, s, marks, owner, jc,       \
                         (float*)xa, (float*)xb, anc, a);                                   \
    break;
    X(1) PF_L96_DIMS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_metropolis_anc(const double* lw, int32_t* anc, const PlainArgs& a,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_metropolis, nblocks(a.N, K1_NT), K1_NT, 0, s, lw, anc, a);
  return hipGetLastError();
}

hipError_t launch_rejection_anc(const double* lw, int32_t* anc, const PlainArgs& a,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_rejection, nblocks(a.N, K1_NT), K1_NT, 0, s, lw, anc, a);
  return hipGetLastError();
}

hipError_t launch_multinomial_anc(const double* wcum, const int32_t* jc, int32_t* anc,
                                  const PlainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_multinomial, nblocks(a.N, K1_NT), K1_NT, 0, s, wcum, jc, anc, a);
  return hipGetLastError();
}

hipError_t launch_simulate(int model, int d, double* out, const PlainArgs& a, double obs_sd,
                           hipStream_t s) {
  if (model == 1) {
    hipLaunchKernelGGL((k_simulate<1, 1>), 1, 64, 0, s, out, a, obs_sd);
    return hipGetLastError();
  }
  switch (d * 4 + model) {
#define X(DD)                                                                      \
  case DD * 4 + 2:                                                                 \
    hipLaunchKernelGGL((k_simulate<2, DD>), 1, 64, 0, s, out, a, obs_sd);          \
    break;                                                                         \
  case DD * 4 + 3:                                                                 \
    hipLaunchKernelGGL((k_simulate<3, DD>), 1, 64, 0, s, out, a, obs_sd);          \
    break;
    PF_L96_DIMS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pfk
