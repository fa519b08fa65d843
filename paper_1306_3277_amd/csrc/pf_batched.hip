// Batched layout: many filters with uneven particle counts (parameter
// particles of SMC over parameters, Alg. 4, or parallel marginal
// Metropolis-Hastings chains, Alg. 3), stepped together.
//
//   K5a  propagate + weight over a flat grid of 256-particle chunks of all
//        filters; each particle loads its ancestor's state (the gather of
//        the previous resampling is fused into this load), so the state is
//        read and written once per interval.
//   K5b  one workgroup per filter, largest filters dispatched first: the
//        filter's FP64 weights are staged in LDS (at most 8192); block max,
//        sums, scan and stratum counts run in registers and LDS, the
//        ancestors come from marks and a running maximum, and they go to
//        global memory for the next K5a.
// Both kernels read the filter's step counter from device memory and pick
// the state buffers by its parity, so one captured graph replays every step.
#include <math.h>

#include "pf_device.hpp"
#include "pf_internal.hpp"

namespace pfk {

__device__ __forceinline__ Key bkey(const KeyArg& k) { return Key{k.lo, k.hi}; }

// ---------------------------------------------------------------- init
template <int MODEL, int D, typename Real>
__global__ __launch_bounds__(BATCH_NT) void k_batch_init(Real* __restrict__ x,
                                                         int32_t* __restrict__ anc,
                                                         BatchArgs A) {
  const int f = A.chunk_f[A.chunk0 + blockIdx.x];
  const int64_t off = A.off[f];
  const int64_t N = A.off[f + 1] - off;
  const int64_t k = (int64_t)A.chunk_k[A.chunk0 + blockIdx.x] + threadIdx.x;
  if (k >= N) return;
  const Key key = bkey(A.key);
  const uint32_t iter = A.fs[f].iter;
  const double* th = A.theta + (size_t)f * 8;
  anc[off + k] = (int32_t)k;
  if (MODEL == 1) {
    double z0, z1;
    const uint4 w = draw(key, TAG_INIT, 0, iter, (uint32_t)k, 0, (uint32_t)f);
    bm_pair_f64(w.x, w.y, z0, z1);
    x[off + k] = (Real)(th[4] + th[5] * z0);
  } else {
#pragma unroll
    for (int blk = 0; blk < D / 4; ++blk) {
      double z[4];
      normals4_f64(draw(key, TAG_INIT, blk, iter, (uint32_t)k, 0, (uint32_t)f), z);
#pragma unroll
      for (int m = 0; m < 4; ++m) x[(int64_t)(4 * blk + m) * A.ld + off + k] = (Real)z[m];
    }
  }
}

// ---------------------------------------------------------------- K5a
template <int D, typename Real>
__device__ __forceinline__ double batch_logdens(const Real (&x)[D], const double* yrow,
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

template <int MODEL, int D, typename Real, bool HIST, bool ACC>
__global__ __launch_bounds__(BATCH_NT) void k_batch_propagate(Real* __restrict__ xa,
                                                              Real* __restrict__ xb,
                                                              double* __restrict__ lw,
                                                              const int32_t* __restrict__ anc,
                                                              BatchArgs A) {
  const int f = A.chunk_f[A.chunk0 + blockIdx.x];
  const int64_t off = A.off[f];
  const int64_t N = A.off[f + 1] - off;
  const int64_t k = (int64_t)A.chunk_k[A.chunk0 + blockIdx.x] + threadIdx.x;
  if (k >= N) return;
  const int t = A.fs[f].t + 1;
  const uint32_t iter = A.fs[f].iter;
  // state written by step s lives in buffer s % 2
  const Real* xp = ((t - 1) & 1) ? xb : xa;
  Real* xn = (t & 1) ? xb : xa;
  const Key key = bkey(A.key);
  const double* th = A.theta + (size_t)f * 8;
  const double* yrow = A.obs + (int64_t)(t - 1) * A.n_obs;
  const int n0 = (t - 1) * A.K;
  const int64_t src = off + anc[off + k];
  const int64_t dst = off + k;
  double l;
  if constexpr (MODEL == 1) {
    if constexpr (sizeof(Real) == 8) {
      double p = xp[src];
      for (int s = 1; s <= A.K; ++s) {
        const uint4 w = draw(key, TAG_NOISE, 0, iter, (uint32_t)k, (uint32_t)(n0 + s), (uint32_t)f);
        double z0, z1;
        bm_pair_f64(w.x, w.y, z0, z1);
        p = wk_substep_f64(p, th, A.q[n0 + s - 1], z0);
      }
      xn[dst] = p;
      if constexpr (HIST) ((Real*)A.hx)[(int64_t)t * A.ld + dst] = p;
      const double e = (yrow[0] - (p + th[2] * A.q[(int64_t)t * A.K])) * A.inv_sd;
      l = -0.5 * (e * e) + A.lw_cst;
    } else {
      float p = xp[src];
      double pa = p;  // the accurate form carries the pressure in FP64
      const float a = (float)(th[0] - 1.0), c = (float)th[1], sp = (float)th[3];
      for (int s = 1; s <= A.K; ++s) {
        const uint4 w = draw(key, TAG_NOISE, 0, iter, (uint32_t)k, (uint32_t)(n0 + s), (uint32_t)f);
        float z0, z1;
        bm_pair_f32(w.x, w.y, z0, z1);
        if constexpr (ACC)
          pa = pa + (double)wk_increment_f32((float)pa, a, c, sp, (float)A.q[n0 + s - 1], z0);
        else
          p = wk_substep_f32(p, a, c, sp, (float)A.q[n0 + s - 1], z0);
      }
      if constexpr (ACC) p = (float)pa;
      else pa = p;
      xn[dst] = p;
      if constexpr (HIST) ((Real*)A.hx)[(int64_t)t * A.ld + dst] = p;
      const double e = (yrow[0] - (pa + th[2] * A.q[(int64_t)t * A.K])) * A.inv_sd;
      l = -0.5 * (e * e) + A.lw_cst;
    }
  } else {
    Real x[D];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = xp[(int64_t)i * A.ld + src];
    if constexpr (sizeof(Real) == 8) {
      ModelConsts mc{A.h, A.hh, A.h6, A.inv_sd, A.lw_cst};
      for (int s = 1; s <= A.K; ++s) {
        if constexpr (MODEL == 3)
          l96_substep_stage_f64<D>(x, th[0], th[1], mc, key, TAG_NOISE, iter, (uint32_t)k,
                                   (uint32_t)(n0 + s), (uint32_t)f);
        else
          l96_substep_f64<D>(x, th[0], th[1], mc, key, TAG_NOISE, iter, (uint32_t)k,
                             (uint32_t)(n0 + s), (uint32_t)f);
      }
    } else if constexpr (ACC) {
      double xa[D];
#pragma unroll
      for (int i = 0; i < D; ++i) xa[i] = (double)x[i];
      const L96F32A c = l96_f32a_consts(th[0], th[1], A.h);
      for (int s = 1; s <= A.K; ++s) {
        if constexpr (MODEL == 3)
          l96_substep_stage_f32acc<D>(xa, c, key, TAG_NOISE, iter, (uint32_t)k,
                                      (uint32_t)(n0 + s), (uint32_t)f);
        else
          l96_substep_f32acc<D>(xa, c, key, TAG_NOISE, iter, (uint32_t)k, (uint32_t)(n0 + s),
                                (uint32_t)f);
      }
#pragma unroll
      for (int i = 0; i < D; ++i) x[i] = (Real)xa[i];
      // the log-weight from the state before it is rounded for storage
      l = batch_logdens<D, double>(xa, yrow, A.obs_pos, A.inv_sd, A.lw_cst);
    } else {
      const L96F32 c = l96_f32_consts(th[0], th[1], A.h);
      for (int s = 1; s <= A.K; ++s) {
        if constexpr (MODEL == 3)
          l96_substep_stage_f32<D>(x, c, key, TAG_NOISE, iter, (uint32_t)k, (uint32_t)(n0 + s),
                                   (uint32_t)f);
        else
          l96_substep_f32<D>(x, c, key, TAG_NOISE, iter, (uint32_t)k, (uint32_t)(n0 + s),
                             (uint32_t)f);
      }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) xn[(int64_t)i * A.ld + dst] = x[i];
    if constexpr (HIST) {  // the history's slot t, written from the same registers
      Real* xh = (Real*)A.hx + (int64_t)t * D * A.ld;
#pragma unroll
      for (int i = 0; i < D; ++i) xh[(int64_t)i * A.ld + dst] = x[i];
    }
    if constexpr (!ACC || sizeof(Real) == 8) l = batch_logdens<D, Real>(x, yrow, A.obs_pos, A.inv_sd, A.lw_cst);
  }
  // weights kept from a step that did not resample carry over
  if (A.fs[f].carry) l = lw[dst] + l;
  lw[dst] = l;
}

// ---------------------------------------------------------------- K5b
// One workgroup per filter.  Lane t owns the P = ceil(N/NT) consecutive
// particles [tP, tP + P).  The log-weights are read from global memory with
// coalesced loads into an LDS stage (element i at slot i ^ ((i >> 4) & 15),
// so both the coalesced writes and the lanes' reads of their own 16-element
// runs are free of bank conflicts) and read back per lane.  Their weights are
// summed sequentially in the lane (an exact monotone prefix), the lanes'
// totals are scanned across the block (held non-decreasing by a running
// maximum within each wave), and each particle's cumulative weight is
// bounded by the totals before and after its lane's run, so the sequence
// never decreases at lane edges.  The stratum counts stay in registers; the
// ancestors reuse the stage (or, for a stage of at most 32 KB, have an
// array of their own): each particle with offspring marks the first
// stratum it owns, and a running
// maximum over the strata (by 64-stratum rows in each wave, then across the
// waves) gives every stratum its owner, so the work does not depend on how
// the offspring are spread (no per-particle loop that one heavy particle
// could lengthen, no search); each row of owners is stored as it stands.
// The resampling uniform is drawn while the loads are in flight, off the
// critical path.  At most 66 KB of LDS per workgroup.
__device__ __forceinline__ int stage_slot(int i) { return i ^ ((i >> 4) & 15); }

// The ancestors in LDS (the stage, once its weights are read): one padding
// word after every 16, so that lanes reading or writing their own runs of
// P consecutive entries hit distinct banks (8,704 words for 8192 entries).
__device__ __forceinline__ int anc_slot(int i) { return i + (i >> 4); }

// A lane's weights e^{lw - M} over its run [i0, i1) of P <= CNT particles,
// their in-lane prefix sums, sum of squares and last positive index.  The
// body is straight-line over CNT slots (weights past the run are 0 and add
// nothing), so the exponentials interleave; P is the same for every lane,
// so the choice of CNT (the smallest power of two >= P) is a uniform branch.
template <int CNT, int MAXP>
__device__ __forceinline__ void lane_weights(const double* stage, int N, double M, bool finite,
                                             int P, int i0, int i1, double (&loc)[MAXP],
                                             double& run, double& run2, int& cand) {
  if constexpr (CNT > 1) {
    if (P <= CNT / 2) {
      lane_weights<CNT / 2, MAXP>(stage, N, M, finite, P, i0, i1, loc, run, run2, cand);
      return;
    }
  }
  double lv[CNT];
#pragma unroll
  for (int e = 0; e < CNT; ++e) lv[e] = stage[stage_slot(min(i0 + e, N - 1))];
#pragma unroll
  for (int e = 0; e < CNT; ++e) {
    const double we = exp_nonpos(lv[e] - M);  // exp(-inf) = 0
    const double w = (finite && e < P && i0 + e < i1) ? we : 0.0;
    cand = (w > 0.0) ? i0 + e : cand;
    run += w;
    run2 += w * w;
    loc[e] = run;
  }
}

// MAXP bounds the particles per lane: the launcher picks the smallest of
// BATCH_MAXN / NT, half and a quarter of it that covers the group's largest
// filter, so the unrolled per-lane phases do no work for absent particles.
template <int NT, int RS, int MAXP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT >= 512 ? 4 : 2, 8))) void k_batch_resample(const double* __restrict__ lw,
                                                       int32_t* __restrict__ anc,
                                                       BatchArgs A) {
  static_assert(MAXP >= 1 && NT * MAXP <= BATCH_MAXN, "stage size");
  constexpr int NW = NT / WAVE;
  // The ancestor slots (one padding word after every 16) have an array of
  // their own when it fits beside a stage of at most 32 KB (filters of up
  // to 4,096 particles at 512 lanes); then they are cleared at the start,
  // two barriers before any mark.  A larger stage is reused for them once
  // its weights are read, and one barrier orders their clearing before the
  // marks.
  constexpr bool SEP = NT * MAXP <= 4096 && (RS == RS_SYSTEMATIC || RS == RS_STRATIFIED);
  constexpr int NAL = SEP ? NT * MAXP + NT * MAXP / 16 : 1;
  __shared__ double stage[NT * MAXP];
  __shared__ int32_t al_own[NAL];
  __shared__ double xa[NW], xs[NW], xb[NW];
  __shared__ int xi[NW];
  __shared__ double bc;
  int32_t* al = SEP ? al_own : reinterpret_cast<int32_t*>(stage);
  const FilterSlot slot = A.order[A.order0 + blockIdx.x];
  const int f = slot.f;
  const int64_t off = slot.off;
  const int N = slot.n;
  FilterState* fs = A.fs + f;
  // the filter's scalars, fetched with the weights so that no later phase
  // waits on a global load
  const double loglik0 = fs->loglik;
  const double lprev0 = fs->lprev;
  const int carry0 = fs->carry;
  const uint32_t iter = fs->iter;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  const bool resample_only = A.mode != 0;
  const int t = resample_only ? fs->t : fs->t + 1;
  // the history's ancestor slot t-1 of this filter, if one is attached
  int32_t* const ha = A.ha ? A.ha + (int64_t)(t - 1) * A.ld + off : nullptr;
  if constexpr (SEP)
    for (int k = (int)threadIdx.x; k < N; k += NT) al[anc_slot(k)] = -1;
  // (1) coalesced load to the stage and the maximum; the loads are issued
  // together (indices past the filter read its last element and are
  // dropped), so their latencies overlap
  double m = -INFINITY;
  {
    double v[MAXP];
#pragma unroll
    for (int r = 0; r < MAXP; ++r) v[r] = lw[off + min((int)threadIdx.x + r * NT, N - 1)];
    // the resampling uniform, drawn while the loads are in flight and
    // published with the first exchange
    if (threadIdx.x == 0)
      bc = resample_only ? A.u_override[f]
                         : u01_f64(draw(bkey(A.key), TAG_RESAMPLE, 0, iter, 0, (uint32_t)t,
                                        (uint32_t)f).x);
#pragma unroll
    for (int r = 0; r < MAXP; ++r) {
      const int i = (int)threadIdx.x + r * NT;
      if (i < N) {
        const double x = (v[r] == v[r]) ? v[r] : -INFINITY;  // NaN counts as zero weight
        stage[stage_slot(i)] = x;
        m = fmax(m, x);
      }
    }
  }
  m = wave_max(m);
  if (lane == 0) xa[wv] = m;
  __syncthreads();  // 1
  double u = bc;
  double M = xa[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) M = fmax(M, xa[w]);
  const bool finite = (M > -INFINITY) && (M < INFINITY);
  // (2) this lane's run: weights, in-lane prefix, square sum, last positive
  const int P = (N + NT - 1) / NT;
  const int i0 = min(N, (int)threadIdx.x * P), i1 = min(N, i0 + P);
  double loc[MAXP];
  double run = 0.0, run2 = 0.0;
  int cand = -1;
  lane_weights<MAXP, MAXP>(stage, N, M, finite, P, i0, i1, loc, run, run2, cand);
  // one exchange: scan of the lanes' sums, total of squares, last positive
  // The scan's partial sums are rounded along different trees, so one
  // lane's may fall an ulp below the lane before: a running maximum makes
  // them non-decreasing, held past the filter's last particle (lanes with no
  // particles take -inf there), so that a wave's total is its last
  // particle's.
  const double incl = wave_incl_scan(run);
  const double inclm = wave_incl_max_scan((i1 > i0) ? incl : -INFINITY);
  const double s2w = wave_sum(run2);
  const int cw = wave_max_i(cand);
  // (the lane sums go to their own array, so no barrier separates them from
  // the maxima read above; the stage is reused only after this exchange)
  if (lane == WAVE - 1) xs[wv] = (inclm > -INFINITY) ? inclm : 0.0;
  if (lane == 0) {
    xb[wv] = s2w;
    xi[wv] = cw;
  }
  __syncthreads();  // 3
  // S: the waves' totals added in order; base: the same sum over the waves
  // before this one (the same operations, so the same bits)
  double base = 0.0, S = 0.0, S2 = 0.0;
  int jstar = -1;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w == wv) base = S;
    S += xs[w];
    S2 += xb[w];
    jstar = max(jstar, xi[w]);
  }
  // the ancestor slots in the stage start empty once its weights are read
  // (the Metropolis, rejection and multinomial forms still use the stage)
  if constexpr (!SEP && (RS == RS_SYSTEMATIC || RS == RS_STRATIFIED)) {
    for (int k = (int)threadIdx.x; k < N; k += NT) al[anc_slot(k)] = -1;
    __syncthreads();  // 4
  }
  // The cumulative weights: lane l's last particle has V_l = base + its
  // running total; before its first particle stands V_{l-1}, which the lane
  // before computes from the same two values (at a wave's first lane it is
  // base, the previous wave's last V); the particles between take
  // min(V_{l-1} + in-lane prefix, V_l).  Each value lies in [V_{l-1}, V_l]
  // (the prefixes are non-negative), so the sequence never decreases across
  // lanes and waves, and the filter's last particle has exactly S.
  // (the lane move runs in every lane, outside the select: a lane whose
  // source lane is switched off would read nothing)
  const double inprev = wave_prev(inclm, 0.0);
  const double vprev = (lane == 0) ? base : base + inprev;
  const double vlast = base + inclm;
  auto cum = [&](int e) -> double {
    return (i0 + e == i1 - 1) ? vlast : fmin(vprev + loc[e], vlast);
  };
  // every lane holds the same S and S2, so every lane takes the trigger's
  // decision itself (resample when ESS < ess_frac N); a step that keeps its
  // weights, or has none positive, gives every particle one offspring:
  // itself
  const bool ok = finite && S > 0.0;
  const double ess = ok ? (S * S) / S2 : 0.0;
  const int carry = (!resample_only && ok) ? !(ess < A.rs.ess_frac * (double)N) : 0;
  const bool draw_rs = finite && !carry;
  // the filter's bookkeeping, by one lane once nothing waits on it
  auto finish = [&]() {
    if (threadIdx.x != 0 || resample_only) return;
    double ell;
    // the factor's normaliser: ln N after a resampling, else the carried
    // weights' ln sum exp
    const double lprev = carry0 ? lprev0 : log((double)N);
    if (ok) {
      const double L = M + log(S);
      ell = L - lprev;
      fs->lprev = L;
    } else {
      ell = -INFINITY;
      fs->status = 4;
    }
    fs->carry = carry;
    fs->loglik = loglik0 + ell;
    fs->M = finite ? M : -INFINITY;
    fs->S = S;
    fs->ell = ell;
    fs->ess = ess;
    A.ell_tr[(size_t)f * A.T + t - 1] = ell;
    A.ess_tr[(size_t)f * A.T + t - 1] = ess;
    fs->u = u;
    fs->t = t;
  };
  const double invS = 1.0 / S;
  if constexpr (RS == RS_METROPOLIS) {
    // Metropolis resampling from the staged log-weights, no counts or merge:
    // output k starts at particle k and takes A.rs.steps moves
    const Key key = bkey(A.key);
    const uint32_t it = iter;
#pragma unroll 1
    for (int k = (int)threadIdx.x; k < N; k += NT) {
      int j = k;
      if (draw_rs) {
        double lj = stage[stage_slot(j)];
        for (int s1 = 1; s1 <= A.rs.steps; s1 += 2) {
          const uint4 w = metro_draw(key, t, (uint32_t)f, it, k, s1);
          int jp = metro_index(w.x, N);
          double lp = stage[stage_slot(jp)];
          if (ln_f64(u01_f64(w.y)) <= lp - lj) {
            j = jp;
            lj = lp;
          }
          if (s1 + 1 <= A.rs.steps) {
            jp = metro_index(w.z, N);
            lp = stage[stage_slot(jp)];
            if (ln_f64(u01_f64(w.w)) <= lp - lj) {
              j = jp;
              lj = lp;
            }
          }
        }
      }
      anc[off + k] = j;
      if (ha) ha[k] = j;
    }
    finish();
    return;
  }
  if constexpr (RS == RS_REJECTION) {
    // rejection resampling draws its ancestors in k_batch_reject, one lane
    // per output over the whole group (a collapsed filter's outputs take
    // about N attempts each, too many for one workgroup); here only the
    // filter's bookkeeping
    finish();
    return;
  }
  if constexpr (RS == RS_MULTINOMIAL) {
    // multinomial resampling as Alg. 2 writes it: the cumulative weights go
    // to LDS (exactly non-decreasing), then output k takes the first W_j
    // above u_k S by binary search
#pragma unroll
    for (int e = 0; e < MAXP; ++e) {
      const int i = i0 + e;
      if (e < P && i < i1) stage[i] = cum(e);
    }
    __syncthreads();  // 6
    const Key key = bkey(A.key);
    const uint32_t it = iter;
#pragma unroll 1
    for (int k = (int)threadIdx.x; k < N; k += NT) {
      int a = k;
      if (draw_rs) {
        const double thr = multi_u(key, t, (uint32_t)f, it, k) * S;
        int lo = 0, hi = N;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (stage[mid] > thr) hi = mid;
          else lo = mid + 1;
        }
        a = lo < N ? lo : (jstar >= 0 && jstar < N ? jstar : 0);
      }
      anc[off + k] = a;
      if (ha) ha[k] = a;
    }
    finish();
    return;
  }
  // (3) stratum counts of this lane's particles, in registers.  Particle i
  // owns strata [c_{i-1}, c_i).  The count before the lane's first particle
  // is the one the lane before computed for its last, at the same V_{l-1}.
  auto count_at = [&](double W, int i) -> int32_t {
    if (!draw_rs) return i + 1;
    if constexpr (RS == RS_STRATIFIED)
      return stratum_count_strat(W, S, invS, N, bkey(A.key), t, (uint32_t)f, iter);
    else
      return stratum_count(W, S, invS, u, N);
  };
  int32_t cnt[MAXP];
#pragma unroll
  for (int e = 0; e < MAXP; ++e) {
    const int i = i0 + e;
    cnt[e] = (e < P && i < i1) ? count_at(cum(e), i) : 0;
  }
  // (4) ancestors: each particle with offspring marks the first stratum it
  // owns, and a running maximum over the strata then gives each its owner
  // (the runs are in particle order), so every lane does the same work
  // however the offspring fall.
  {
    int cprev = (i0 > 0 && i0 < N) ? count_at(vprev, i0 - 1) : 0;
#pragma unroll
    for (int e = 0; e < MAXP; ++e) {
      const int i = i0 + e;
      if (e < P && i < i1) {
        if (cnt[e] > cprev) al[anc_slot(cprev)] = i;
        cprev = cnt[e];
      }
    }
  }
  __syncthreads();  // 7
  // (5) owners: wave wv takes the strata [wv seg, (wv + 1) seg) in rows of
  // 64, with a running maximum of the marks along each row, carried from
  // row to row and then across the waves; each row is stored as it stands,
  // 64 consecutive ancestors per wave
  const int seg = ((N + NW - 1) / NW + WAVE - 1) & ~(WAVE - 1);  // <= 64 MAXP
  const int sbase = wv * seg;
  int mk[MAXP];
  int rowmax = -1;
#pragma unroll
  for (int r = 0; r < MAXP; ++r) {
    const int k = sbase + r * WAVE + lane;
    const int v = (r * WAVE < seg && k < N) ? al[anc_slot(k)] : -1;
    mk[r] = max(wave_incl_max_scan_rows(v), rowmax);
    rowmax = __builtin_amdgcn_readlane(mk[r], WAVE - 1);
  }
  if (lane == 0) xi[wv] = rowmax;
  __syncthreads();  // 8
  int before = -1;
#pragma unroll
  for (int w = 0; w < NW; ++w)
    if (w < wv) before = max(before, xi[w]);
  // strata past the last count (never expected: the last particle's
  // cumulative weight is S) go to the last positive particle
  const int ctot = count_at(S, N - 1);
  bool bad = false;
  auto owner = [&](int r, int k) -> int32_t {
    int32_t aj = k < ctot ? max(before, mk[r]) : jstar;
    if (aj < 0 || aj >= N) {  // never expected; flagged, kept in bounds
      aj = 0;
      bad = true;
    }
    return aj;
  };
  if (ha) {
#pragma unroll
    for (int r = 0; r < MAXP; ++r) {
      const int k = sbase + r * WAVE + lane;
      if (r * WAVE < seg && k < N) {
        const int32_t aj = owner(r, k);
        anc[off + k] = aj;
        ha[k] = aj;
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < MAXP; ++r) {
      const int k = sbase + r * WAVE + lane;
      if (r * WAVE < seg && k < N) anc[off + k] = owner(r, k);
    }
  }
  if (bad) atomicOr(&fs->pad, 1);
  finish();
}

// Rejection resampling (RS_REJECTION), after the collective's bookkeeping:
// one lane per output over the group's chunks, reading the filter's
// log-weights and largest log-weight M from memory.  A step that keeps its
// weights, or has none positive, gives the identity.
__global__ __launch_bounds__(BATCH_NT) void k_batch_reject(const double* __restrict__ lw,
                                                           int32_t* __restrict__ anc,
                                                           BatchArgs A) {
  const int f = A.chunk_f[A.chunk0 + blockIdx.x];
  const int64_t off = A.off[f];
  const int N = (int)(A.off[f + 1] - off);
  const int k = A.chunk_k[A.chunk0 + blockIdx.x] + (int)threadIdx.x;
  if (k >= N) return;
  const FilterState* fs = A.fs + f;
  const double M = fs->M;
  const int t = fs->t;
  const bool draw_rs = (M > -INFINITY) && (M < INFINITY) && (fs->S > 0.0) && !fs->carry;
  int j = k;
  if (draw_rs) {
    const double* l = lw + off;
    j = reject_ancestor(bkey(A.key), t, (uint32_t)f, fs->iter, k, N, M,
                        [&](int32_t i) { return l[i]; });
  }
  anc[off + k] = j;
  if (A.ha) A.ha[(int64_t)(t - 1) * A.ld + off + k] = j;
}

// x_out = x_prop[ancestors]: materialises the equally weighted set for
// inspection (the stepping kernels never need it).
template <typename Real>
__global__ __launch_bounds__(BATCH_NT) void k_batch_gather(const Real* __restrict__ xprop,
                                                           const int32_t* __restrict__ anc,
                                                           Real* __restrict__ xout,
                                                           BatchArgs A) {
  const int f = A.chunk_f[A.chunk0 + blockIdx.x];
  const int64_t off = A.off[f];
  const int64_t N = A.off[f + 1] - off;
  const int64_t k = (int64_t)A.chunk_k[A.chunk0 + blockIdx.x] + threadIdx.x;
  if (k >= N) return;
  const int64_t src = off + anc[off + k];
  for (int i = 0; i < A.d; ++i) xout[(int64_t)i * A.ld + off + k] = xprop[(int64_t)i * A.ld + src];
}

// ---------------------------------------------------------------- launchers
#define PF_L96_DIMS_B(X) X(4) X(8) X(16) X(32) X(40)

hipError_t launch_batched_init(int model, int d, int prec, void* x, int32_t* anc,
                               const BatchArgs& a, hipStream_t s) {
  const unsigned g = (unsigned)a.n_chunks;
  if (model == 1) {
    if (prec == 0)
      hipLaunchKernelGGL((k_batch_init<1, 1, double>), g, BATCH_NT, 0, s, (double*)x, anc, a);
    else
      hipLaunchKernelGGL((k_batch_init<1, 1, float>), g, BATCH_NT, 0, s, (float*)x, anc, a);
    return hipGetLastError();
  }
  switch (d) {
#define X(DD)                                                                              \
  case DD:                                                                                 \
    if (prec == 0)                                                                         \
      hipLaunchKernelGGL((k_batch_init<2, DD, double>), g, BATCH_NT, 0, s, (double*)x,     \
                         anc, a);                                                          \
    else                                                                                   \
      hipLaunchKernelGGL((k_batch_init<2, DD, float>), g, BATCH_NT, 0, s, (float*)x, anc,  \
                         a);                                                               \
    break;
    PF_L96_DIMS_B(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// K5a with or without the history stores (a separate instantiation, so the
// kernel without a history carries no trace of them); ACC selects the
// accurate FP32 form
template <int MODEL, int D, typename Real, bool ACC = false>
void launch_k5a(unsigned g, hipStream_t s, void* xa, void* xb, double* lw, const int32_t* anc,
                const BatchArgs& a) {
  if (a.hx)
    hipLaunchKernelGGL((k_batch_propagate<MODEL, D, Real, true, ACC>), g, BATCH_NT, 0, s,
                       (Real*)xa, (Real*)xb, lw, anc, a);
  else
    hipLaunchKernelGGL((k_batch_propagate<MODEL, D, Real, false, ACC>), g, BATCH_NT, 0, s,
                       (Real*)xa, (Real*)xb, lw, anc, a);
}

hipError_t launch_batched_propagate(int model, int d, int prec, void* xa, void* xb, double* lw,
                                    const int32_t* anc, const BatchArgs& a, int nchunks,
                                    hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  const unsigned g = (unsigned)nchunks;
  if (model == 1) {
    if (prec == 0)
      launch_k5a<1, 1, double>(g, s, xa, xb, lw, anc, a);
    else if (prec == 1)
      launch_k5a<1, 1, float>(g, s, xa, xb, lw, anc, a);
    else
      launch_k5a<1, 1, float, true>(g, s, xa, xb, lw, anc, a);
    return hipGetLastError();
  }
  switch (d * 4 + model) {
#define X(DD)                                                  \
  case DD * 4 + 2:                                             \
    if (prec == 0)                                             \
      launch_k5a<2, DD, double>(g, s, xa, xb, lw, anc, a);     \
    else if (prec == 1)                                        \
      launch_k5a<2, DD, float>(g, s, xa, xb, lw, anc, a);      \
    else                                                       \
      launch_k5a<2, DD, float, true>(g, s, xa, xb, lw, anc, a); \
    break;                                                     \
  case DD * 4 + 3:                                             \
    if (prec == 0)                                             \
      launch_k5a<3, DD, double>(g, s, xa, xb, lw, anc, a);     \
    else if (prec == 1)                                        \
      launch_k5a<3, DD, float>(g, s, xa, xb, lw, anc, a);      \
    else                                                       \
      launch_k5a<3, DD, float, true>(g, s, xa, xb, lw, anc, a); \
    break;
    PF_L96_DIMS_B(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batched_resample(int nt, const double* lw, int32_t* anc, const BatchArgs& a,
                                   int nfilters, int max_n, int nchunks, hipStream_t s) {
  if (nfilters <= 0) return hipSuccess;
  if (max_n < 1 || max_n > BATCH_MAXN) return hipErrorInvalidValue;
  const unsigned g = (unsigned)nfilters;
  // the fraction of the full per-lane bound the group's largest filter needs
  const int full = BATCH_MAXN / nt;
  const int need = (max_n + nt - 1) / nt;
  const int q = need * 4 <= full ? 4 : need * 2 <= full ? 2 : 1;
#define PF_K5B(NTV, RSV, MP) \
  hipLaunchKernelGGL((k_batch_resample<NTV, RSV, MP>), g, NTV, 0, s, lw, anc, a)
#define PF_K5B_Q(NTV, RSV)                                  \
  switch (q) {                                              \
    case 4: PF_K5B(NTV, RSV, BATCH_MAXN / NTV / 4); break;  \
    case 2: PF_K5B(NTV, RSV, BATCH_MAXN / NTV / 2); break;  \
    default: PF_K5B(NTV, RSV, BATCH_MAXN / NTV); break;     \
  }
#define PF_K5B_RS(NTV)                                         \
  switch (a.rs.scheme) {                                       \
    case RS_SYSTEMATIC: PF_K5B_Q(NTV, RS_SYSTEMATIC); break;   \
    case RS_STRATIFIED: PF_K5B_Q(NTV, RS_STRATIFIED); break;   \
    case RS_METROPOLIS: PF_K5B_Q(NTV, RS_METROPOLIS); break;   \
    case RS_MULTINOMIAL: PF_K5B_Q(NTV, RS_MULTINOMIAL); break; \
    case RS_REJECTION: PF_K5B_Q(NTV, RS_REJECTION); break;     \
    default: return hipErrorInvalidValue;                      \
  }
  switch (nt) {
    case 256:
      PF_K5B_RS(256);
      break;
    case 512:
      PF_K5B_RS(512);
      break;
    case 1024:
      PF_K5B_RS(1024);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef PF_K5B_RS
#undef PF_K5B_Q
#undef PF_K5B
  if (a.rs.scheme == RS_REJECTION && nchunks > 0)
    hipLaunchKernelGGL(k_batch_reject, (unsigned)nchunks, BATCH_NT, 0, s, lw, anc, a);
  return hipGetLastError();
}

hipError_t launch_batched_gather(int prec, const void* xprop, const int32_t* anc, void* xout,
                                 const BatchArgs& a, hipStream_t s) {
  const unsigned g = (unsigned)a.n_chunks;
  if (prec == 0)
    hipLaunchKernelGGL((k_batch_gather<double>), g, BATCH_NT, 0, s, (const double*)xprop, anc,
                       (double*)xout, a);
  else
    hipLaunchKernelGGL((k_batch_gather<float>), g, BATCH_NT, 0, s, (const float*)xprop, anc,
                       (float*)xout, a);
  return hipGetLastError();
}

}  // namespace pfk
