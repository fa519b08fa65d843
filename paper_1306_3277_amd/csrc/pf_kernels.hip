// Plain-layout kernels of the gfx950 bootstrap particle filter (Alg. 2):
//   K1 propagate + weight   one particle per lane, K substeps in registers,
//                           log-weight, per-block (max, sum, sum of squares)
//   K2 combine              one workgroup: global max, FP64 block offsets,
//                           likelihood increment, ESS, resampling uniform
//   K3 scan + counts        FP64 block scan of exp(lw - M); for each particle
//                           the number of strata its cumulative weight covers
//   K4 merge-path gather    outputs and particles merged along equal-length
//                           diagonals, so work per lane is independent of the
//                           weights; ancestors staged in LDS, then coalesced
//                           gather of the state rows
// plus initialisation and the synthetic-data simulator.
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
      for (int m = 0; m < 4; ++m) x[(int64_t)(4 * blk + m) * A.ld + col] = (Real)z[m];
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
    f.pad2 = 0;
    fs[i] = f;
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

template <int MODEL, int D, typename Real>
__global__ __launch_bounds__(K1_NT) void k_propagate_weight(const Real* __restrict__ xcur,
                                                            Real* __restrict__ xprop,
                                                            double* __restrict__ lw,
                                                            double* __restrict__ part,
                                                            PlainArgs A) {
  __shared__ double red[K1_NT / WAVE];
  const int64_t j = (int64_t)blockIdx.x * K1_NT + threadIdx.x;
  const int t = A.fs->t + 1;
  const uint32_t iter = A.fs->iter;
  const Key key = key_of(A.key);
  double l = -INFINITY;
  if (j < A.N) {
    const int64_t col = A.off + j;
    const double* yrow = A.obs + (int64_t)(t - 1) * A.n_obs;
    const int n0 = (t - 1) * A.K;
    if constexpr (MODEL == 1) {
      if constexpr (sizeof(Real) == 8) {
        double p = xcur[col];
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
        float p = xcur[col];
        const float a = (float)(A.theta[0] - 1.0), c = (float)A.theta[1], sp = (float)A.theta[3];
        for (int s = 1; s <= A.K; ++s) {
          const uint4 w = draw(key, TAG_NOISE, 0, iter, (uint32_t)j, (uint32_t)(n0 + s), A.b);
          float z0, z1;
          bm_pair_f32(w.x, w.y, z0, z1);
          p = wk_substep_f32(p, a, c, sp, (float)A.q[n0 + s - 1], z0);
        }
        xprop[col] = p;
        const double e =
            (yrow[0] - ((double)p + A.theta[2] * A.q[(int64_t)t * A.K])) * A.inv_sd;
        l = -0.5 * (e * e) + A.lw_cst;
      }
    } else {
      Real x[D];
#pragma unroll
      for (int i = 0; i < D; ++i) x[i] = xcur[(int64_t)i * A.ld + col];
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
#pragma unroll
      for (int i = 0; i < D; ++i) xprop[(int64_t)i * A.ld + col] = x[i];
      l = l96_logdens<D, Real>(x, yrow, A.obs_pos, A.inv_sd, A.lw_cst);
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
  }
}

// ---------------------------------------------------------------- K2
// Offsets of the blocks' cumulative weights.  Block i of a filter owns
// boff[i] .. boff[i+1]; boff[nb] is the total S.  The offsets are summed
// sequentially within each thread's chunk and scanned across chunks; a
// running maximum (exact) then makes them non-decreasing whatever the
// rounding, so the cumulative weights built on them in K3 are monotone and
// the stratum counts can be merged.
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
  const int t = fst->t + 1;
  const double loglik0 = fst->loglik;
  const double lprev0 = fst->lprev;
  const int carry0 = fst->carry;
  double u = 0.0;
  if (threadIdx.x == 0)
    u = u01_f64(draw(key_of(A.key), TAG_RESAMPLE, 0, fst->iter, 0, (uint32_t)t, A.b).x);
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
  const double vup = __shfl_up(vin, 1, WAVE);
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

__global__ void k_set_u(FilterState* fs, double u) {
  if (threadIdx.x == 0 && blockIdx.x == 0) fs->u = u;
}

// ---------------------------------------------------------------- K3
// W_j = boff[blk] + (block-local inclusive scan of exp(lw - M)), made
// non-decreasing by an exact running maximum and capped by boff[blk+1]; then
// count_j = #{k : (u + k) S < N W_j}, the number of strata owned by particles
// 0..j.  Systematic resampling is then the merge of the counts with the
// outputs k = 0..N-1 (K4): at state (j, k), particle j is consumed when
// c_j <= k, otherwise output k gets ancestor j.  Particle j's states are
// (j, k) for k in [c_{j-1}, c_j], i.e. the path diagonals j + c_{j-1} ..
// j + c_j; every lane emits the merge-path state on each K4 block boundary
// (a multiple of K4_DB) that falls in its range, so K4 needs no search.  At a
// block edge the states (j, k), k < g = count(boff[blk]), of the block's
// first particle are emitted by the previous block's last lane, which
// computes the same g from the same boff value.
__device__ __forceinline__ void emit_bounds(int32_t* __restrict__ bstate, int64_t j, int64_t d_lo,
                                            int64_t d_hi) {
  if (d_hi < d_lo) return;
  int64_t D = ((d_lo + K4_DB - 1) / K4_DB) * K4_DB;
  for (; D <= d_hi; D += K4_DB) bstate[D / K4_DB] = (int32_t)j;
}

__global__ __launch_bounds__(K3_NT) void k_scan_count(const double* __restrict__ lw,
                                                      const double* __restrict__ boff,
                                                      int32_t* __restrict__ counts,
                                                      int32_t* __restrict__ bstate_all,
                                                      int32_t* __restrict__ bjs_all,
                                                      PlainArgs A) {
  __shared__ double red[K3_NT / WAVE];
  __shared__ int64_t wlast[K3_NT / WAVE];
  __shared__ int redi[K3_NT / WAVE];
  const int64_t N = A.N;
  const int64_t jb = (int64_t)blockIdx.x * K3_SPAN;
  const int64_t j0 = jb + (int64_t)threadIdx.x * K3_PER;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const FilterState* f = A.fs;
  const double M = f->M, S = f->S, u = f->u;
  // a step that keeps its weights (ESS above the trigger) or has none
  // positive gives every particle one offspring: itself
  const bool finite = (M > -INFINITY) && (M < INFINITY) && (S > 0.0) && !f->carry;
  const double invS = 1.0 / S;
  const bool strat = A.rs.scheme == RS_STRATIFIED;
  const Key key = key_of(A.key);
  const int32_t t_now = f->t;
  const uint32_t it_now = f->iter;
  auto count = [&](double W) -> int64_t {
    return strat ? stratum_count_strat(W, S, invS, (int32_t)N, key, t_now, A.b, it_now)
                 : stratum_count(W, S, invS, u, (int32_t)N);
  };
  const double* bo = boff + A.boff0 + A.b;
  const int k1b = (int)blockIdx.x * (K3_SPAN / K1_NT);  // first K1 block of this block
  const double lo_off = bo[k1b];
  const double hi_off = bo[min(k1b + K3_SPAN / K1_NT, A.nblk)];
  // in-lane sequential prefix of K3_PER consecutive weights
  double w[K3_PER], loc[K3_PER], lv[K3_PER];
  double run = 0.0;
  // loads issued together (past the end they reread the last weight)
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) lv[e] = lw[A.off + min(j0 + e, N - 1)];
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) {
    const int64_t j = j0 + e;
    double we = 0.0;
    if (j < N && finite) {
      const double l = lv[e];
      we = (l == l) ? exp_nonpos(l - M) : 0.0;
    }
    w[e] = we;
    run += we;
    loc[e] = run;
  }
  double tot;
  const double pre = block_incl_scan<K3_NT>(run, red, tot) - run;
  double V[K3_PER];
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) V[e] = lo_off + (pre + loc[e]);
  // exact running maximum over earlier lanes keeps W non-decreasing across
  // lanes whatever the rounding of the tree scan; capped by the next offset
  const double vmax = block_incl_max_scan<K3_NT>(V[K3_PER - 1], red);
  double vprev = __shfl_up(vmax, 1, WAVE);
  __shared__ double wmax[K3_NT / WAVE];
  if (lane == WAVE - 1) wmax[wv] = vmax;
  __syncthreads();
  if (lane == 0) vprev = wv > 0 ? wmax[wv - 1] : lo_off;
  int64_t c[K3_PER];
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) {
    const int64_t j = j0 + e;
    const double W = fmin(fmax(V[e], vprev), hi_off);
    c[e] = (j < N) ? (finite ? count(W) : j + 1) : 0;
    if (A.rs.scheme == RS_MULTINOMIAL && j < N) A.wcum[j] = W;
    if (j < N) counts[A.off + j] = (int32_t)c[e];
  }
  // merge-path states on the K4 block boundaries (see above)
  const int64_t g_lo = finite ? count(lo_off) : jb;
  const int64_t jnext = jb + K3_SPAN;
  const int64_t g_hi = (jnext < N) ? (finite ? count(hi_off) : jnext) : N;
  int64_t cprev = __shfl_up(c[K3_PER - 1], 1, WAVE);
  if (lane == WAVE - 1) wlast[wv] = c[K3_PER - 1];
  __syncthreads();
  if (lane == 0) cprev = wv > 0 ? wlast[wv - 1] : g_lo;
  int32_t* bstate = bstate_all + A.bst0;
  // this lane's diagonal ranges: one per particle, plus (for the filter's or
  // the block's last particle) the overflow outputs and end state, or the
  // next block's first particle below its edge count
  int64_t rj[K3_PER + 1], rlo[K3_PER + 1], rhi[K3_PER + 1];
#pragma unroll
  for (int e = 0; e <= K3_PER; ++e) {
    rj[e] = 0;
    rlo[e] = 1;
    rhi[e] = 0;  // empty
  }
#pragma unroll
  for (int e = 0; e < K3_PER; ++e) {
    const int64_t j = j0 + e;
    if (j < N) {
      rj[e] = j;
      rlo[e] = j + cprev;
      rhi[e] = j + c[e];
      if (j == N - 1) {
        rj[K3_PER] = N;
        rlo[K3_PER] = N + c[e];
        rhi[K3_PER] = 2 * N;
      } else if (j == jnext - 1) {
        rj[K3_PER] = j + 1;
        rlo[K3_PER] = j + 1 + c[e];
        rhi[K3_PER] = j + g_hi;
      }
    }
    cprev = c[e];
  }
  // A range crossing at most two block boundaries is emitted by its lane; a
  // longer one (a particle owning many strata) by the whole wave, strided
  // over the lanes, so no lane loops over hundreds of boundaries.
#pragma unroll
  for (int e = 0; e <= K3_PER; ++e) {
    const int64_t first = (rlo[e] + K4_DB - 1) / K4_DB;
    const int64_t nb = (rhi[e] < rlo[e]) ? 0 : rhi[e] / K4_DB - first + 1;
    const bool big = nb > 2;
    if (!big)
      for (int64_t q = first; q < first + nb; ++q) bstate[q] = (int32_t)rj[e];
    uint64_t mask = __ballot(big);
    while (mask) {
      const int src = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      const long long bj = __shfl((long long)rj[e], src, WAVE);
      const long long bq0 = __shfl((long long)first, src, WAVE);
      const long long bq1 = __shfl((long long)(rhi[e] / K4_DB), src, WAVE);
      for (long long q = bq0 + lane; q <= bq1; q += WAVE) bstate[q] = (int32_t)bj;
    }
  }
  // last particle of positive weight in this block, for the rare case where
  // rounding leaves the final strata without an owner
  int cand = -1;
#pragma unroll
  for (int e = 0; e < K3_PER; ++e)
    if (j0 + e < N && w[e] > 0.0) cand = (int)(j0 + e);
  cand = block_max_i<K3_NT>(cand, redi);
  if (threadIdx.x == 0) bjs_all[A.bj0 + blockIdx.x] = cand;
}

// ---------------------------------------------------------------- K4
// Block b walks diagonals [b K4_DB, (b+1) K4_DB) of the merge path from the
// state K3 recorded, with the block's slice of counts staged in LDS and
// K4_L path steps per lane; the ancestors land in LDS and the state rows
// are then gathered with coalesced stores (all D components of an output in
// flight at once).
template <int D, typename Real>
__global__ __launch_bounds__(K4_NT) void k_merge_gather(const int32_t* __restrict__ counts,
                                                        const int32_t* __restrict__ bstate_all,
                                                        const int32_t* __restrict__ bjs_all,
                                                        const Real* __restrict__ xprop,
                                                        Real* __restrict__ xcur,
                                                        int32_t* __restrict__ anc,
                                                        PlainArgs A) {
  __shared__ int32_t sc[K4_DB + 1];
  __shared__ int32_t sa[K4_DB];
  __shared__ int32_t s_jstar;
  const int64_t N = A.N;
  const int32_t* c = counts + A.off;
  const int32_t* bstate = bstate_all + A.bst0;
  const int64_t d0 = (int64_t)blockIdx.x * K4_DB;
  const int64_t d1 = min(d0 + K4_DB, 2 * N);
  const int64_t j0 = bstate[blockIdx.x];
  const int64_t j1 = (d1 == 2 * N) ? N : (int64_t)bstate[blockIdx.x + 1];
  const int64_t k0 = d0 - j0, k1 = d1 - j1;
  bool bad = !(j0 >= 0 && j0 <= j1 && j1 <= N && k0 >= 0 && k0 <= k1 && k1 <= N);
  for (int i = threadIdx.x; i < K4_DB; i += K4_NT) sa[i] = -1;
  if (!bad)
    for (int64_t i = threadIdx.x; i <= j1 - j0 && j0 + i < N; i += K4_NT) sc[i] = c[j0 + i];
  if (threadIdx.x < WAVE) {
    // only a block that reaches past the last particle can need the last
    // particle of positive weight; find it from the per-block candidates
    int found = -1;
    if (!bad && j1 == N) {
      const int nb3 = (int)((N + K3_SPAN - 1) / K3_SPAN);
      for (int base = nb3 - 1; base >= 0 && found < 0; base -= WAVE) {
        const int i = base - (int)threadIdx.x;
        found = wave_max_i(i >= 0 ? bjs_all[A.bj0 + i] : -1);
      }
    }
    if (threadIdx.x == 0) s_jstar = found;
  }
  __syncthreads();
  const int32_t jstar = s_jstar;
  const int64_t dt = d0 + (int64_t)threadIdx.x * K4_L;
  if (!bad && dt < d1) {
    // first state of this lane: largest j in [lo, hi] with c_{j-1} <= dt - j
    int64_t lo = max(j0, dt - k1), hi = min(j1, dt - k0);
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)sc[mid - j0] <= dt - 1 - mid)
        lo = mid + 1;
      else
        hi = mid;
    }
    int64_t jj = lo, k = dt - lo;
    for (int s = 0; s < K4_L && jj + k < d1; ++s) {
      if (jj < N && (k >= N || (int64_t)sc[jj - j0] <= k)) {
        ++jj;
      } else {
        if (k >= k0 && k < k1) sa[k - k0] = (int32_t)(jj < N ? jj : jstar);
        ++k;
      }
    }
  }
  __syncthreads();
  if (!bad) {
    for (int64_t k = k0 + threadIdx.x; k < k1; k += K4_NT) {
      int32_t aj = sa[k - k0];
      if (aj < 0 || aj >= N) {  // never expected; flagged, and kept in bounds
        bad = true;
        aj = 0;
      }
      anc[A.off + k] = aj;
      const Real* src = xprop + A.off + aj;
      Real* dst = xcur + A.off + k;
      if constexpr (D > 0) {
        Real v[D];
#pragma unroll
        for (int i = 0; i < D; ++i) v[i] = src[(int64_t)i * A.ld];
#pragma unroll
        for (int i = 0; i < D; ++i) dst[(int64_t)i * A.ld] = v[i];
      } else {
        for (int i = 0; i < A.d; ++i) dst[(int64_t)i * A.ld] = src[(int64_t)i * A.ld];
      }
    }
  }
  if (bad) atomicOr(&A.fs->pad, 1);
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
}

// Multinomial resampling, as Alg. 2 writes it: output k takes
// a_k = min{j : W_j > u_k S} for an independent uniform u_k, by binary
// search of the cumulative weights K3 left (exactly non-decreasing);
// rounding overflow goes to the last positive weight (from K3's per-block
// candidates).  A step that keeps its weights, or has none positive, gives
// the identity.
__global__ __launch_bounds__(K1_NT) void k_multinomial(const double* __restrict__ wcum,
                                                       const int32_t* __restrict__ bjs_all,
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
      const int nb3 = (int)((A.N + K3_SPAN - 1) / K3_SPAN);
      for (int i = 0; i < nb3; ++i) js = max(js, bjs_all[A.bj0 + i]);
      a = js >= 0 ? js : 0;
    }
  }
  anc[A.off + k] = (int32_t)a;
}

// x_cur[k] = x_prop[a_k] for unsorted ancestors.
template <typename Real>
__global__ __launch_bounds__(K1_NT) void k_anc_gather(const Real* __restrict__ xprop,
                                                      Real* __restrict__ xcur,
                                                      const int32_t* __restrict__ anc,
                                                      PlainArgs A) {
  const int64_t k = (int64_t)blockIdx.x * K1_NT + threadIdx.x;
  if (k >= A.N) return;
  const int64_t src = A.off + anc[A.off + k];
  for (int i = 0; i < A.d; ++i) xcur[(int64_t)i * A.ld + A.off + k] = xprop[(int64_t)i * A.ld + src];
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

hipError_t launch_propagate(int model, int d, int prec, const void* xcur, void* xprop, void* lw,
                            double* part, const PlainArgs& a, hipStream_t s) {
  const unsigned g = (unsigned)a.nblk;
  if (model == 1) {
    if (prec == 0)
      hipLaunchKernelGGL((k_propagate_weight<1, 1, double>), g, K1_NT, 0, s,
                         (const double*)xcur, (double*)xprop, (double*)lw, part, a);
    else
      hipLaunchKernelGGL((k_propagate_weight<1, 1, float>), g, K1_NT, 0, s,
                         (const float*)xcur, (float*)xprop, (double*)lw, part, a);
    return hipGetLastError();
  }
  switch (d * 4 + model) {
#define X(DD)                                                                             \
  case DD * 4 + 2:                                                                        \
    if (prec == 0)                                                                        \
      hipLaunchKernelGGL((k_propagate_weight<2, DD, double>), g, K1_NT, 0, s,             \
                         (const double*)xcur, (double*)xprop, (double*)lw, part, a);      \
    else                                                                                  \
      hipLaunchKernelGGL((k_propagate_weight<2, DD, float>), g, K1_NT, 0, s,              \
                         (const float*)xcur, (float*)xprop, (double*)lw, part, a);        \
    break;                                                                                \
  case DD * 4 + 3:                                                                        \
    if (prec == 0)                                                                        \
      hipLaunchKernelGGL((k_propagate_weight<3, DD, double>), g, K1_NT, 0, s,             \
                         (const double*)xcur, (double*)xprop, (double*)lw, part, a);      \
    else                                                                                  \
      hipLaunchKernelGGL((k_propagate_weight<3, DD, float>), g, K1_NT, 0, s,              \
                         (const float*)xcur, (float*)xprop, (double*)lw, part, a);        \
    break;
    PF_L96_DIMS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_combine(const double* part, double* boff, const PlainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, 1, K2_NT, 0, s, part, boff, a);
  return hipGetLastError();
}

hipError_t launch_set_u(FilterState* fs, double u, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u, 1, 64, 0, s, fs, u);
  return hipGetLastError();
}

hipError_t launch_scan_count(int prec, const void* lw, const double* boff, int32_t* counts,
                             int32_t* bstate, int32_t* bjs, const PlainArgs& a, hipStream_t s) {
  (void)prec;
  hipLaunchKernelGGL(k_scan_count, nblocks(a.N, K3_SPAN), K3_NT, 0, s, (const double*)lw, boff,
                     counts, bstate, bjs, a);
  return hipGetLastError();
}

hipError_t launch_merge_gather(int model, int d, int prec, const int32_t* counts,
                               const int32_t* bstate, const int32_t* bjs, const void* xprop,
                               void* xcur, int32_t* anc, const PlainArgs& a, hipStream_t s) {
  const unsigned g = nblocks(2 * a.N, K4_DB);
  const int dd = model == 1 ? 1 : d;
  switch (dd) {
#define X(DD)                                                                              \
  case DD:                                                                                 \
    if (prec == 0)                                                                         \
      hipLaunchKernelGGL((k_merge_gather<DD, double>), g, K4_NT, 0, s, counts, bstate, bjs, \
                         (const double*)xprop, (double*)xcur, anc, a);                     \
    else                                                                                   \
      hipLaunchKernelGGL((k_merge_gather<DD, float>), g, K4_NT, 0, s, counts, bstate, bjs,  \
                         (const float*)xprop, (float*)xcur, anc, a);                       \
    break;
    X(1) PF_L96_DIMS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_metropolis_gather(int prec, const double* lw, const void* xprop, void* xcur,
                                   int32_t* anc, const PlainArgs& a, hipStream_t s) {
  const unsigned g = nblocks(a.N, K1_NT);
  hipLaunchKernelGGL(k_metropolis, g, K1_NT, 0, s, lw, anc, a);
  if (prec == 0)
    hipLaunchKernelGGL(k_anc_gather<double>, g, K1_NT, 0, s, (const double*)xprop,
                       (double*)xcur, (const int32_t*)anc, a);
  else
    hipLaunchKernelGGL(k_anc_gather<float>, g, K1_NT, 0, s, (const float*)xprop, (float*)xcur,
                       (const int32_t*)anc, a);
  return hipGetLastError();
}

hipError_t launch_multinomial_gather(int prec, const double* wcum, const int32_t* bjs,
                                     const void* xprop, void* xcur, int32_t* anc,
                                     const PlainArgs& a, hipStream_t s) {
  const unsigned g = nblocks(a.N, K1_NT);
  hipLaunchKernelGGL(k_multinomial, g, K1_NT, 0, s, wcum, bjs, anc, a);
  if (prec == 0)
    hipLaunchKernelGGL(k_anc_gather<double>, g, K1_NT, 0, s, (const double*)xprop,
                       (double*)xcur, (const int32_t*)anc, a);
  else
    hipLaunchKernelGGL(k_anc_gather<float>, g, K1_NT, 0, s, (const float*)xprop, (float*)xcur,
                       (const int32_t*)anc, a);
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
