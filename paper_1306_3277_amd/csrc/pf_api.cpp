// Host runtime of the gfx950 particle filter: validates configurations,
// carves the caller's workspace, launches the kernels, captures and replays
// HIP graphs, and implements the inspection and timing calls of pf.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pf.h"
#include "pf_internal.hpp"
#include "pf_kalman.hpp"
#include "pf_path.hpp"
#include "pf_smc2.hpp"
#include "pf_systematic.hpp"

using pfk::FilterState;
using pfk::PlainArgs;
using pfk::BatchArgs;

namespace {

// the last failing call's message on this thread (a fixed buffer: reporting
// an error allocates nothing)
thread_local char g_err[512];

pf_status fail(pf_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

void err_clear() { g_err[0] = 0; }

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(PF_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

bool l96_dim_ok(int d) { return d == 4 || d == 8 || d == 16 || d == 32 || d == 40; }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
  int64_t n_total = 0;
  std::vector<int64_t> off;     // [B+1]
  std::vector<int64_t> boff0;   // [B] first block slot
  std::vector<int32_t> nblk;    // [B]
  std::vector<int64_t> own0;    // [B] first output-tile owner slot
  int64_t own_total = 0;
  int64_t nblk_total = 0;
  // byte offsets into the workspace
  size_t x_cur, x_tmp, lw, marks, anc, part, boff, owner, jc, fs, ell, ess, theta, obs, obs_pos,
      obs_idx, q, b_off, b_order, b_chunk_f, b_chunk_k, b_u, kf_ll, kf_ell, wcum, total;
  int32_t n_chunks = 0;
};

pf_status validate(const pf_config* c) {
  if (!c) return fail(PF_E_INVAL, "cfg is NULL");
  if (c->model != PF_MODEL_WK && c->model != PF_MODEL_L96 && c->model != PF_MODEL_L96_STAGE)
    return fail(PF_E_INVAL, "model %d unknown", c->model);
  if (c->precision != PF_FP64 && c->precision != PF_FP32_MIXED &&
      c->precision != PF_FP32_ACCURATE)
    return fail(PF_E_INVAL, "precision %d unknown", c->precision);
  if (c->layout != PF_LAYOUT_PLAIN && c->layout != PF_LAYOUT_BATCHED)
    return fail(PF_E_INVAL, "layout %d unknown", c->layout);
  if (c->model == PF_MODEL_WK) {
    if (c->d != 1) return fail(PF_E_INVAL, "windkessel needs d = 1 (got %d)", c->d);
    if (c->n_obs != 1) return fail(PF_E_INVAL, "windkessel needs n_obs = 1");
    if (c->n_theta != 6) return fail(PF_E_INVAL, "windkessel needs n_theta = 6");
  } else {
    if (!l96_dim_ok(c->d))
      return fail(PF_E_INVAL, "Lorenz '96 d must be one of 4, 8, 16, 32, 40 (got %d)", c->d);
    if (c->n_theta != 2) return fail(PF_E_INVAL, "Lorenz '96 needs n_theta = 2");
  }
  if (c->K < 1) return fail(PF_E_INVAL, "K must be >= 1");
  if (c->T < 1) return fail(PF_E_INVAL, "T must be >= 1");
  if ((int64_t)c->T * c->K >= (1LL << 31)) return fail(PF_E_INVAL, "T*K too large");
  if (!(c->h > 0.0) || !std::isfinite(c->h)) return fail(PF_E_INVAL, "h must be positive");
  if (c->n_obs < 1 || c->n_obs > c->d) return fail(PF_E_INVAL, "n_obs out of range");
  if (!c->obs_idx) return fail(PF_E_INVAL, "obs_idx is NULL");
  for (int o = 0; o < c->n_obs; ++o) {
    if (c->obs_idx[o] < 0 || c->obs_idx[o] >= c->d)
      return fail(PF_E_INVAL, "obs_idx[%d] = %d out of range", o, c->obs_idx[o]);
    if (o > 0 && c->obs_idx[o] <= c->obs_idx[o - 1])
      return fail(PF_E_INVAL, "obs_idx must be strictly increasing");
  }
  if (!(c->obs_sd > 0.0) || !std::isfinite(c->obs_sd))
    return fail(PF_E_INVAL, "obs_sd must be positive");
  if (!c->obs) return fail(PF_E_INVAL, "obs is NULL");
  for (int64_t i = 0; i < (int64_t)c->T * c->n_obs; ++i)
    if (!std::isfinite(c->obs[i])) return fail(PF_E_INVAL, "obs[%lld] is not finite", (long long)i);
  if (c->model == PF_MODEL_WK) {
    if (!c->q) return fail(PF_E_INVAL, "windkessel needs the flow series q");
    for (int64_t i = 0; i <= (int64_t)c->T * c->K; ++i)
      if (!std::isfinite(c->q[i])) return fail(PF_E_INVAL, "q[%lld] is not finite", (long long)i);
  }
  if (c->B < 1) return fail(PF_E_INVAL, "B must be >= 1");
  if (!c->n_particles || !c->theta) return fail(PF_E_INVAL, "n_particles or theta is NULL");
  int64_t tot = 0;
  for (int b = 0; b < c->B; ++b) {
    const int64_t n = c->n_particles[b];
    if (n < 1) return fail(PF_E_INVAL, "n_particles[%d] = %lld must be >= 1", b, (long long)n);
    if (n > 2147483647LL) return fail(PF_E_INVAL, "n_particles[%d] too large", b);
    if (c->layout == PF_LAYOUT_BATCHED && n > PF_BATCHED_MAX_PARTICLES)
      return fail(PF_E_INVAL, "batched layout needs n_particles <= %d (filter %d has %lld)",
                  PF_BATCHED_MAX_PARTICLES, b, (long long)n);
    tot += n;
    for (int i = 0; i < c->n_theta; ++i)
      if (!std::isfinite(c->theta[(int64_t)b * c->n_theta + i]))
        return fail(PF_E_INVAL, "theta[%d][%d] is not finite", b, i);
  }
  if (tot > 2147483647LL) return fail(PF_E_INVAL, "total particles exceed 2^31 - 1");
  if (c->model == PF_MODEL_WK) {
    for (int b = 0; b < c->B; ++b)
      if (c->theta[(int64_t)b * 6 + 3] < 0 || c->theta[(int64_t)b * 6 + 5] < 0)
        return fail(PF_E_INVAL, "windkessel sds must be >= 0");
  } else {
    for (int b = 0; b < c->B; ++b)
      if (c->theta[(int64_t)b * 2 + 1] < 0) return fail(PF_E_INVAL, "sigma must be >= 0");
  }
  return PF_OK;
}

Layout make_layout(const pf_config* c) {
  Layout L;
  const size_t sx = c->precision == PF_FP64 ? 8 : 4;
  L.off.assign(c->B + 1, 0);
  L.boff0.assign(c->B, 0);
  L.nblk.assign(c->B, 0);
  L.own0.assign(c->B, 0);
  for (int b = 0; b < c->B; ++b) {
    L.own0[b] = L.own_total;
    L.own_total += (c->n_particles[b] + pfk::K4_TILE - 1) / pfk::K4_TILE;
    L.off[b + 1] = L.off[b] + c->n_particles[b];
    L.nblk[b] = (int32_t)((c->n_particles[b] + pfk::K1_NT - 1) / pfk::K1_NT);
    L.boff0[b] = L.nblk_total;
    L.nblk_total += L.nblk[b];
  }
  L.n_total = L.off[c->B];
  {
    int64_t nc = 0;
    for (int b = 0; b < c->B; ++b) nc += (c->n_particles[b] + pfk::BATCH_NT - 1) / pfk::BATCH_NT;
    L.n_chunks = (int32_t)nc;
  }
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at = p;
    p = align256(p + bytes);
    return at;
  };
  const int64_t N = L.n_total;
  // the plain layout's state is kept in whole 64-particle tiles
  L.x_cur = take(sx * (size_t)pfk::plain_state_values(N, c->d));
  L.x_tmp = take(sx * (size_t)pfk::plain_state_values(N, c->d));
  L.lw = take(8 * N);  // log-weights are FP64 in both precisions
  L.marks = take(4 * N);  // -1 between resamplings
  L.anc = take(4 * N);
  L.part = take(24 * L.nblk_total);
  L.boff = take(8 * (L.nblk_total + c->B));  // nblk + 1 offsets per filter
  L.owner = take(4 * (size_t)(L.own_total > 0 ? L.own_total : 1));  // per output tile
  L.jc = take(4 * (size_t)(L.own_total > 0 ? L.own_total : 1));     // per scan block
  L.fs = take(sizeof(FilterState) * c->B);
  L.ell = take(8 * (size_t)c->B * c->T);
  L.ess = take(8 * (size_t)c->B * c->T);
  L.theta = take(8 * 8 * (size_t)c->B);
  L.obs = take(8 * (size_t)c->T * c->n_obs);
  L.obs_pos = take(4 * (size_t)c->d);
  L.obs_idx = take(4 * (size_t)c->n_obs);
  L.q = take(c->model == PF_MODEL_WK ? 8 * ((size_t)c->T * c->K + 1) : 8);
  L.b_off = take(8 * (size_t)(c->B + 1));
  L.b_order = take(sizeof(pfk::FilterSlot) * (size_t)c->B);
  L.b_chunk_f = take(4 * (size_t)(L.n_chunks > 0 ? L.n_chunks : 1));
  L.b_chunk_k = take(4 * (size_t)(L.n_chunks > 0 ? L.n_chunks : 1));
  L.b_u = take(8 * (size_t)c->B);
  L.kf_ll = take(8 * (size_t)c->B);
  L.kf_ell = take(8 * (size_t)c->B * c->T);
  L.wcum = take(c->layout == PF_LAYOUT_PLAIN ? 8 * (size_t)L.n_total : 8);
  L.total = p;
  return L;
}

// derived parameters: WK as given; L96 (F, sigma*sqrt(h))
void derive_theta(const pf_config* c, const double* theta_in, std::vector<double>& out) {
  out.assign((size_t)c->B * 8, 0.0);
  for (int b = 0; b < c->B; ++b) {
    const double* t = theta_in + (size_t)b * c->n_theta;
    double* o = out.data() + (size_t)b * 8;
    if (c->model == PF_MODEL_WK) {
      for (int i = 0; i < 6; ++i) o[i] = t[i];
    } else {
      o[0] = t[0];
      o[1] = t[1] * std::sqrt(c->h);
    }
  }
}

}  // namespace

struct pf_handle {
  pf_config cfg{};           // host pointers cleared after init
  Layout L;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  int phase = 0;             // 0: equally weighted (ready to step), 1: weighted
  int32_t t = 0;
  uint32_t iter = 0;
  bool resampled_once = false;
  bool stepped_once = false;
  std::vector<int64_t> np;
  std::vector<double> theta_host;  // [B][n_theta]
  // batched layout tuning: workgroup size of the per-filter collective, and
  // the number of filter groups stepped concurrently on their own streams
  int batch_nt = 256;
  int groups = 1;
  std::vector<int32_t> grp_chunk0, grp_nchunks, grp_order0, grp_nfilt, grp_maxn;
  // with G > 1 groups, group g's kernels run on side[g]; ev_a[0] forks the
  // side streams from the caller's, ev_b[g] joins group g back.  These
  // events are only ever recorded and waited on outside stream capture.
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev_a, ev_b;
  // timing
  bool timing = false;
  struct Ev {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<Ev> events;
  // graphs, each captured on one stream: gexecs[g * gnv + v] holds 2^v
  // intervals, v < gnv (plain layout: g = 0, every filter; batched layout:
  // filter group g)
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> gexecs;
  int gnv = 0;
  // batched layout: pf_graph_run issues its intervals as eager launches
  // (the autotuner found them faster than the graph replay on this host)
  bool eager_replay = false;
  hipStream_t cap_stream = nullptr;
  // attached history (ancestry storage), or null
  char* hist = nullptr;
  // resampling variant and ESS trigger (default: systematic, every time)
  pfk::ResampleArgs rs{pfk::RS_SYSTEMATIC, 0, INFINITY};
  bool alive = true;

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

namespace {

PlainArgs plain_args(const pf_handle* H, int b) {
  const pf_config& c = H->cfg;
  PlainArgs a{};
  a.N = H->np[b];
  a.ld = H->L.n_total;
  a.off = H->L.off[b];
  a.boff0 = H->L.boff0[b];
  a.own0 = H->L.own0[b];
  a.nblk = H->L.nblk[b];
  a.K = c.K;
  a.T = c.T;
  a.d = c.d;
  a.n_obs = c.n_obs;
  a.b = (uint32_t)b;
  a.key.lo = (uint32_t)(c.seed & 0xffffffffu);
  a.key.hi = (uint32_t)(c.seed >> 32);
  a.h = c.h;
  a.hh = 0.5 * c.h;
  a.h6 = c.h / 6.0;
  a.inv_sd = 1.0 / c.obs_sd;
  a.lw_cst = -(double)c.n_obs * (std::log(c.obs_sd) + 0.5 * 1.8378770664093454836);
  a.theta = H->at<double>(H->L.theta) + (size_t)b * 8;
  a.obs = H->at<double>(H->L.obs);
  a.obs_pos = H->at<int32_t>(H->L.obs_pos);
  a.obs_idx = H->at<int32_t>(H->L.obs_idx);
  a.q = c.model == PF_MODEL_WK ? H->at<double>(H->L.q) : nullptr;
  a.fs = H->at<FilterState>(H->L.fs) + b;
  a.ell_tr = H->at<double>(H->L.ell) + (size_t)b * c.T;
  a.ess_tr = H->at<double>(H->L.ess) + (size_t)b * c.T;
  a.rs = H->rs;
  a.wcum = H->at<double>(H->L.wcum) + (c.layout == PF_LAYOUT_PLAIN ? H->L.off[b] : 0);
  return a;
}

BatchArgs batch_args(const pf_handle* H) {
  const pf_config& c = H->cfg;
  BatchArgs a{};
  a.B = c.B;
  a.K = c.K;
  a.T = c.T;
  a.d = c.d;
  a.n_obs = c.n_obs;
  a.key.lo = (uint32_t)(c.seed & 0xffffffffu);
  a.key.hi = (uint32_t)(c.seed >> 32);
  a.ld = H->L.n_total;
  a.n_chunks = H->L.n_chunks;
  a.h = c.h;
  a.hh = 0.5 * c.h;
  a.h6 = c.h / 6.0;
  a.inv_sd = 1.0 / c.obs_sd;
  a.lw_cst = -(double)c.n_obs * (std::log(c.obs_sd) + 0.5 * 1.8378770664093454836);
  a.theta = H->at<double>(H->L.theta);
  a.obs = H->at<double>(H->L.obs);
  a.obs_pos = H->at<int32_t>(H->L.obs_pos);
  a.q = c.model == PF_MODEL_WK ? H->at<double>(H->L.q) : nullptr;
  a.off = H->at<int64_t>(H->L.b_off);
  a.order = H->at<pfk::FilterSlot>(H->L.b_order);
  a.chunk_f = H->at<int32_t>(H->L.b_chunk_f);
  a.chunk_k = H->at<int32_t>(H->L.b_chunk_k);
  a.chunk0 = 0;
  a.order0 = 0;
  a.fs = H->at<FilterState>(H->L.fs);
  a.ell_tr = H->at<double>(H->L.ell);
  a.ess_tr = H->at<double>(H->L.ess);
  a.u_override = H->at<double>(H->L.b_u);
  a.mode = 0;
  a.rs = H->rs;
  return a;
}

pf_status ev_begin(pf_handle* H, hipEvent_t* e, hipStream_t s) {
  if (!H->timing) return PF_OK;
  HIP_TRY(hipEventCreate(e));
  HIP_TRY(hipEventRecord(*e, s));
  return PF_OK;
}
pf_status ev_end(pf_handle* H, hipEvent_t a, int kind, hipStream_t s) {
  if (!H->timing) return PF_OK;
  hipEvent_t b;
  HIP_TRY(hipEventCreate(&b));
  HIP_TRY(hipEventRecord(b, s));
  H->events.push_back({a, b, kind});
  return PF_OK;
}

pf_status build_groups(pf_handle* H, int G);
void destroy_streams(pf_handle* H);
void destroy_graphs(pf_handle* H);

pf_status check_handle(pf_handle* H) {
  if (!H) return fail(PF_E_INVAL, "handle is NULL");
  if (!H->alive) return fail(PF_E_STATE, "handle was destroyed");
  return PF_OK;
}

// History buffer: xh [T+1][d][N_total] particles, ah [T][N_total] ancestors,
// then the backtrace's indices [B][T+1] and path [B][T+1][d] (FP64).
struct HistLayout {
  size_t xh, ah, idx, path, total;
};

HistLayout hist_layout(const pf_config* c, int64_t n_total) {
  HistLayout L{};
  const size_t sx = c->precision == PF_FP64 ? 8 : 4;
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at = p;
    p = align256(p + bytes);
    return at;
  };
  L.xh = take(sx * (size_t)(c->T + 1) * c->d * (size_t)n_total);
  L.ah = take(4 * (size_t)c->T * (size_t)n_total);
  L.idx = take(4 * (size_t)c->B * (c->T + 1));
  L.path = take(8 * (size_t)c->B * (c->T + 1) * c->d);
  L.total = p;
  return L;
}

pfk::HistArgs hist_args(const pf_handle* H) {
  const HistLayout L = hist_layout(&H->cfg, H->L.n_total);
  pfk::HistArgs a{};
  a.xh = H->hist + L.xh;
  a.ah = (int32_t*)(H->hist + L.ah);
  a.ld = H->L.n_total;
  a.d = H->cfg.d;
  a.T = H->cfg.T;
  return a;
}

// Copy the current slot (the filters' step counters) into the history: the
// particles of every filter (the buffer of the step's parity) and, past
// t_0, the ancestors (the plain layout records past t_0 from
// enqueue_resample, once its ancestors are written out).
pf_status record_all(pf_handle* H, hipStream_t s) {
  if (!H->hist) return PF_OK;
  const pf_config& c = H->cfg;
  const pfk::HistArgs ha = hist_args(H);
  if (c.layout == PF_LAYOUT_PLAIN) {
    for (int b = 0; b < c.B; ++b)
      HIP_TRY(pfk::launch_record_plain(c.precision, H->ws + H->L.x_cur, H->ws + H->L.x_tmp,
                                       H->at<int32_t>(H->L.anc), ha, H->L.off[b], H->np[b],
                                       H->at<FilterState>(H->L.fs) + b, s));
  } else {
    BatchArgs a = batch_args(H);
    HIP_TRY(pfk::launch_record_batched(c.precision, H->ws + H->L.x_cur, H->ws + H->L.x_tmp,
                                       H->at<int32_t>(H->L.anc), ha, a, H->L.n_chunks, s));
  }
  return PF_OK;
}

// init kernels for every filter (fresh x(t0), scalars and traces cleared)
pf_status do_init(pf_handle* H, hipStream_t s) {
  const pf_config& c = H->cfg;
  HIP_TRY(pfk::launch_reset(H->at<FilterState>(H->L.fs), H->at<double>(H->L.ell),
                            H->at<double>(H->L.ess), c.B, c.T, H->iter, s));
  if (c.layout == PF_LAYOUT_PLAIN) {
    // marks a previous run left pending are cleared (the pending ancestors
    // are now the identity)
    HIP_TRY(pfk::launch_fill_i32(H->at<int32_t>(H->L.marks), H->L.n_total, -1, s));
    for (int b = 0; b < c.B; ++b) {
      PlainArgs a = plain_args(H, b);
      HIP_TRY(pfk::launch_init(c.model, c.d, c.precision, H->ws + H->L.x_cur, a, s));
    }
  } else {
    BatchArgs a = batch_args(H);
    HIP_TRY(pfk::launch_batched_init(c.model, c.d, c.precision, H->ws + H->L.x_cur,
                                     H->at<int32_t>(H->L.anc), a, s));
  }
  pf_status st = record_all(H, s);
  if (st) return st;
  H->t = 0;
  H->phase = 0;
  return PF_OK;
}

// Graph lengths: 1, 2, 4, ... intervals up to 2^(n - 1), so that a run of
// any length replays in a few graph launches per stream (each launch costs
// the device several microseconds, and a PMMH or headline pass is T = 200
// intervals).  Up to 128 intervals when an interval is a few kernels (one
// filter, or one filter group), up to 8 when it is a launch per filter of
// many (the plain layout with B > 4), to keep captures small.
int graph_ladder(const pf_handle* H) {
  return (H->cfg.layout == PF_LAYOUT_PLAIN && H->cfg.B > 4) ? 4 : 8;
}

// An attached history's slots, for the stepping kernels that record into
// it (the propagation writes the particles, the collective the ancestors).
void set_history(const pf_handle* H, BatchArgs& a) {
  if (!H->hist) return;
  const pfk::HistArgs h = hist_args(H);
  a.hx = h.xh;
  a.ha = h.ah;
}

// Propagation (K5a) of filter group g on stream s.
pf_status enqueue_group_propagate(pf_handle* H, int g, hipStream_t s) {
  const pf_config& c = H->cfg;
  BatchArgs a = batch_args(H);
  a.chunk0 = H->grp_chunk0[g];
  a.order0 = H->grp_order0[g];
  set_history(H, a);
  hipEvent_t e0{};
  pf_status st = ev_begin(H, &e0, s);
  if (st) return st;
  HIP_TRY(pfk::launch_batched_propagate(c.model, c.d, c.precision, H->ws + H->L.x_cur,
                                        H->ws + H->L.x_tmp, H->at<double>(H->L.lw),
                                        H->at<int32_t>(H->L.anc), a, H->grp_nchunks[g], s));
  return ev_end(H, e0, 0, s);
}

// Collective (K5b: likelihood, ESS, resampling) of filter group g on stream s.
pf_status enqueue_group_collective(pf_handle* H, int g, hipStream_t s) {
  BatchArgs a = batch_args(H);
  a.chunk0 = H->grp_chunk0[g];
  a.order0 = H->grp_order0[g];
  set_history(H, a);
  hipEvent_t e0{};
  pf_status st = ev_begin(H, &e0, s);
  if (st) return st;
  HIP_TRY(pfk::launch_batched_resample(H->batch_nt, H->at<double>(H->L.lw),
                                       H->at<int32_t>(H->L.anc), a, H->grp_nfilt[g],
                                       H->grp_maxn[g], H->grp_nchunks[g], s));
  return ev_end(H, e0, 4, s);
}

// n intervals of filter group g, back to back on stream s (one stream, no
// events: this is what a group's graph holds).
pf_status enqueue_group(pf_handle* H, int g, hipStream_t s, int n) {
  pf_status st;
  for (int i = 0; i < n; ++i)
    if ((st = enqueue_group_propagate(H, g, s)) || (st = enqueue_group_collective(H, g, s)))
      return st;
  return PF_OK;
}

// Fork the filter groups' streams from s (they start after everything
// issued on s so far) and join them back into s.  Never used inside a
// capture.
pf_status fork_groups(pf_handle* H, hipStream_t s) {
  HIP_TRY(hipEventRecord(H->ev_a[0], s));
  for (int g = 0; g < H->groups; ++g) HIP_TRY(hipStreamWaitEvent(H->side[g], H->ev_a[0], 0));
  return PF_OK;
}
pf_status join_groups(pf_handle* H, hipStream_t s) {
  for (int g = 0; g < H->groups; ++g) {
    HIP_TRY(hipEventRecord(H->ev_b[g], H->side[g]));
    HIP_TRY(hipStreamWaitEvent(s, H->ev_b[g], 0));
  }
  return PF_OK;
}

// n intervals of the batched layout issued eagerly from stream s.  With one
// group both kernels go on s.  With G groups (filters dealt so that every
// group holds about the same number of particles) group g's intervals run
// back to back on side[g]: the groups start together after everything
// issued on s so far, drift against each other, and one group's collective
// overlaps another's propagation; s waits for every group at the end.  The
// launches are issued interval by interval across the groups, so no group
// waits for the host to issue another group's whole run.
pf_status enqueue_batched(pf_handle* H, hipStream_t s, int n) {
  pf_status st;
  const int G = H->groups;
  if (G == 1) return enqueue_group(H, 0, s, n);
  if ((st = fork_groups(H, s))) return st;
  for (int i = 0; i < n; ++i)
    for (int g = 0; g < G; ++g)
      if ((st = enqueue_group(H, g, H->side[g], 1))) return st;
  return join_groups(H, s);
}

pf_status enqueue_step(pf_handle* H, hipStream_t s) {
  const pf_config& c = H->cfg;
  if (c.layout == PF_LAYOUT_BATCHED) return enqueue_batched(H, s, 1);
  for (int b = 0; b < c.B; ++b) {
    PlainArgs a = plain_args(H, b);
    hipEvent_t e0{};
    pf_status st = ev_begin(H, &e0, s);
    if (st) return st;
    HIP_TRY(pfk::launch_propagate(c.model, c.d, c.precision, H->ws + H->L.x_cur,
                                  H->ws + H->L.x_tmp, H->ws + H->L.lw,
                                  H->at<double>(H->L.part), H->at<int32_t>(H->L.marks),
                                  H->at<int32_t>(H->L.owner), H->at<int32_t>(H->L.jc),
                                  H->at<int32_t>(H->L.anc), a, s));
    if ((st = ev_end(H, e0, 0, s))) return st;
    // the collective: likelihood increment, ESS, trigger, and (unless
    // Metropolis) the cumulative weights' marks or, for multinomial, the
    // cumulative weights themselves; a large filter's partials are combined
    // once first
    if (a.nblk > pfk::FUSE_NB) {
      if ((st = ev_begin(H, &e0, s))) return st;
      HIP_TRY(pfk::launch_combine(H->at<double>(H->L.part), H->at<double>(H->L.boff), a, s));
      if ((st = ev_end(H, e0, 1, s))) return st;
    }
    if ((st = ev_begin(H, &e0, s))) return st;
    a.mode = 0;
    HIP_TRY(pfk::launch_scan_mark(H->at<double>(H->L.lw), H->at<double>(H->L.part),
                                  H->at<double>(H->L.boff), H->at<int32_t>(H->L.marks),
                                  H->at<int32_t>(H->L.owner), H->at<int32_t>(H->L.jc), a, s));
    if ((st = ev_end(H, e0, 2, s))) return st;
  }
  return PF_OK;
}

// Plain layout, filter b: the pending ancestors written out to the ancestor
// array (from the marks when those are pending), which then become the
// pending form.
pf_status plain_anc_out(pf_handle* H, int b, hipStream_t s) {
  PlainArgs a = plain_args(H, b);
  HIP_TRY(pfk::launch_tile_anc(H->at<int32_t>(H->L.marks), H->at<int32_t>(H->L.owner),
                               H->at<int32_t>(H->L.jc), H->at<int32_t>(H->L.anc), a, s));
  HIP_TRY(pfk::launch_set_amode(a.fs, 1, pfk::AMODE_ARRAY, s));
  return PF_OK;
}

pf_status enqueue_resample(pf_handle* H, hipStream_t s, const double* u) {
  const pf_config& c = H->cfg;
  if (c.layout == PF_LAYOUT_BATCHED) {
    // the ancestors were drawn with the step; the gather happens in the next
    // step's state load.  Given uniforms redraw them without touching the
    // likelihood.
    if (!u) return PF_OK;
    HIP_TRY(hipMemcpyAsync(H->ws + H->L.b_u, u, 8 * (size_t)c.B, hipMemcpyHostToDevice, s));
    BatchArgs a = batch_args(H);
    a.mode = 1;
    const int32_t max_n = (int32_t)*std::max_element(H->np.begin(), H->np.end());
    HIP_TRY(pfk::launch_batched_resample(H->batch_nt, H->at<double>(H->L.lw),
                                         H->at<int32_t>(H->L.anc), a, c.B, max_n,
                                         H->L.n_chunks, s));
    pf_status st = record_all(H, s);  // the redrawn ancestors
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(s));  // u is a host array
    return PF_OK;
  }
  for (int b = 0; b < c.B; ++b) {
    PlainArgs a = plain_args(H, b);
    hipEvent_t e0{};
    pf_status st;
    if (u) {
      // redraw the marks (or cumulative weights) from the given uniform; the
      // step's marks are cleared first
      HIP_TRY(pfk::launch_set_u(a.fs, u[b], s));
      if (H->rs.scheme != pfk::RS_METROPOLIS && H->rs.scheme != pfk::RS_REJECTION) {
        HIP_TRY(pfk::launch_fill_i32(H->at<int32_t>(H->L.marks) + a.off, a.N, -1, s));
        a.mode = 1;
        HIP_TRY(pfk::launch_scan_mark(H->at<double>(H->L.lw), H->at<double>(H->L.part),
                                      H->at<double>(H->L.boff), H->at<int32_t>(H->L.marks),
                                      H->at<int32_t>(H->L.owner), H->at<int32_t>(H->L.jc), a,
                                      s));
      }
    }
    // The systematic and stratified ancestors stay as the collective's marks,
    // which the next propagation reads (it gathers through them); the other
    // resamplers write the ancestor array.  No state is copied here.
    if (H->rs.scheme == pfk::RS_METROPOLIS || H->rs.scheme == pfk::RS_REJECTION ||
        H->rs.scheme == pfk::RS_MULTINOMIAL) {
      if ((st = ev_begin(H, &e0, s))) return st;
      if (H->rs.scheme == pfk::RS_METROPOLIS)  // no scan, counts or merge
        HIP_TRY(pfk::launch_metropolis_anc(H->at<double>(H->L.lw), H->at<int32_t>(H->L.anc), a,
                                           s));
      else if (H->rs.scheme == pfk::RS_REJECTION)  // the step's maximum, no scan
        HIP_TRY(pfk::launch_rejection_anc(H->at<double>(H->L.lw), H->at<int32_t>(H->L.anc), a,
                                          s));
      else  // search of the step's cumulative weights
        HIP_TRY(pfk::launch_multinomial_anc(a.wcum, H->at<int32_t>(H->L.jc),
                                            H->at<int32_t>(H->L.anc), a, s));
      if ((st = ev_end(H, e0, 3, s))) return st;
    } else if (H->hist) {
      // the history keeps the ancestors: written out from the marks
      if ((st = plain_anc_out(H, b, s))) return st;
    }
    if (H->hist)
      HIP_TRY(pfk::launch_record_plain(c.precision, H->ws + H->L.x_cur, H->ws + H->L.x_tmp,
                                       H->at<int32_t>(H->L.anc), hist_args(H), a.off, a.N, a.fs,
                                       s));
  }
  return PF_OK;
}

pf_status upload_theta(pf_handle* H, const double* theta) {
  std::vector<double> th;
  derive_theta(&H->cfg, theta, th);
  HIP_TRY(hipMemcpyAsync(H->ws + H->L.theta, th.data(), th.size() * 8, hipMemcpyHostToDevice,
                         H->stream));
  HIP_TRY(hipStreamSynchronize(H->stream));
  H->theta_host.assign(theta, theta + (size_t)H->cfg.B * H->cfg.n_theta);
  return PF_OK;
}

pf_status require_device() {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(PF_E_DEVICE, "device %d is %s; this library is built for gfx950", dev,
                prop.gcnArchName);
  return PF_OK;
}

// Filters largest first (longest-processing-time order), dealt to G groups
// by always giving the next filter to the group with the fewest particles;
// each group's filters and 256-particle chunks are contiguous in the device
// tables, so a launch covers one group with a base offset.
pf_status build_groups(pf_handle* H, int G) {
  const pf_config& c = H->cfg;
  if (G < 1) G = 1;
  if (G > c.B) G = c.B;
  std::vector<int32_t> order(c.B);
  for (int b = 0; b < c.B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return H->np[x] > H->np[y]; });
  std::vector<std::vector<int32_t>> members(G);
  std::vector<int64_t> load(G, 0);
  for (int32_t b : order) {
    int gbest = 0;
    for (int g = 1; g < G; ++g)
      if (load[g] < load[gbest]) gbest = g;
    members[gbest].push_back(b);
    load[gbest] += H->np[b];
  }
  std::vector<pfk::FilterSlot> ord;
  std::vector<int32_t> chf, chk;
  H->grp_chunk0.assign(G, 0);
  H->grp_nchunks.assign(G, 0);
  H->grp_order0.assign(G, 0);
  H->grp_nfilt.assign(G, 0);
  H->grp_maxn.assign(G, 1);
  // Collective slots: the first one-per-CU slots take the largest filters,
  // and the slots beyond them (which share a CU with those) take the rest
  // smallest first, so the largest filters share their CU with the smallest.
  const int cu_slots = 256;
  for (int g = 0; g < G; ++g) {
    H->grp_order0[g] = (int32_t)ord.size();
    H->grp_chunk0[g] = (int32_t)chf.size();
    const std::vector<int32_t>& mg = members[g];  // largest first
    const int m = (int)mg.size();
    for (int i = 0; i < m; ++i) {
      const int32_t b = i < cu_slots ? mg[i] : mg[m - 1 - (i - cu_slots)];
      ord.push_back({b, (int32_t)H->L.off[b], (int32_t)H->np[b], 0});
    }
    for (int32_t b : mg) {
      for (int64_t k = 0; k < H->np[b]; k += pfk::BATCH_NT) {
        chf.push_back(b);
        chk.push_back((int32_t)k);
      }
    }
    H->grp_nfilt[g] = (int32_t)ord.size() - H->grp_order0[g];
    if (m > 0) H->grp_maxn[g] = (int32_t)H->np[mg[0]];  // members are largest first
    H->grp_nchunks[g] = (int32_t)chf.size() - H->grp_chunk0[g];
  }
  HIP_TRY(hipMemcpyAsync(H->ws + H->L.b_order, ord.data(), sizeof(pfk::FilterSlot) * ord.size(),
                         hipMemcpyHostToDevice, H->stream));
  HIP_TRY(hipMemcpyAsync(H->ws + H->L.b_chunk_f, chf.data(), 4 * chf.size(),
                         hipMemcpyHostToDevice, H->stream));
  HIP_TRY(hipMemcpyAsync(H->ws + H->L.b_chunk_k, chk.data(), 4 * chk.size(),
                         hipMemcpyHostToDevice, H->stream));
  HIP_TRY(hipStreamSynchronize(H->stream));
  // a stream and two events per group (default priority); graphs captured
  // for another group count are rebuilt
  while (G > 1 && (int)H->side.size() < G) {
    hipStream_t st;
    HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    H->side.push_back(st);
    hipEvent_t ea, eb;
    HIP_TRY(hipEventCreateWithFlags(&ea, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&eb, hipEventDisableTiming));
    H->ev_a.push_back(ea);
    H->ev_b.push_back(eb);
  }
  if (G != H->groups) destroy_graphs(H);
  H->groups = G;
  return PF_OK;
}

void destroy_graphs(pf_handle* H) {
  for (auto g : H->gexecs) (void)hipGraphExecDestroy(g);
  for (auto g : H->graphs) (void)hipGraphDestroy(g);
  H->gexecs.clear();
  H->graphs.clear();
  H->gnv = 0;
}

// Waits for everything the handle has issued: its stream, the stream graph
// replays go on, and the group streams.  Graphs, streams and events are only
// destroyed after this, so none is destroyed while work that uses it is in
// flight.
pf_status drain(pf_handle* H) {
  HIP_TRY(hipStreamSynchronize(H->stream));
  if (H->cap_stream) HIP_TRY(hipStreamSynchronize(H->cap_stream));
  for (auto s : H->side) HIP_TRY(hipStreamSynchronize(s));
  return PF_OK;
}

void destroy_streams(pf_handle* H) {
  destroy_graphs(H);
  for (auto s : H->side) (void)hipStreamDestroy(s);
  for (auto e : H->ev_a) (void)hipEventDestroy(e);
  for (auto e : H->ev_b) (void)hipEventDestroy(e);
  if (H->cap_stream) (void)hipStreamDestroy(H->cap_stream);
  H->side.clear();
  H->ev_a.clear();
  H->ev_b.clear();
  H->cap_stream = nullptr;
}

// The stream graph replays go on: the caller's, or a blocking stream of our
// own when the caller uses the null stream (which cannot be captured).
pf_status launch_stream(pf_handle* H, hipStream_t* out) {
  if (H->stream) {
    *out = H->stream;
    return PF_OK;
  }
  if (!H->cap_stream) HIP_TRY(hipStreamCreate(&H->cap_stream));
  *out = H->cap_stream;
  return PF_OK;
}

// Captures the graphs pf_graph_run replays.  Every capture is on one
// stream and holds kernel launches only (no event, copy or memset), so a
// graph never refers to an event or another stream: 2^v intervals for each
// step v of the ladder, of every filter (plain layout) or of each filter
// group (batched layout).  The groups' graphs are launched on their own
// streams between an eager fork and join.
pf_status ensure_graphs(pf_handle* H) {
  if (!H->gexecs.empty()) return PF_OK;
  hipStream_t cs;
  pf_status st = launch_stream(H, &cs);
  if (st) return st;
  const bool tm = H->timing;
  H->timing = false;
  const bool batched = H->cfg.layout == PF_LAYOUT_BATCHED;
  const int ng = batched ? H->groups : 1;
  const int nv = graph_ladder(H);
  for (int g = 0; g < ng && !st; ++g) {
    for (int v = 0; v < nv && !st; ++v) {
      HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      if (batched) {
        st = enqueue_group(H, g, cs, 1 << v);
      } else {
        for (int i = 0; i < (1 << v) && !st; ++i) {
          st = enqueue_step(H, cs);
          if (!st) st = enqueue_resample(H, cs, nullptr);
        }
      }
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(cs, &graph);
      if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        break;
      }
      if (e != hipSuccess) {
        st = fail(PF_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        break;
      }
      H->graphs.push_back(graph);
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        st = fail(PF_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        break;
      }
      H->gexecs.push_back(ex);
    }
  }
  H->timing = tm;
  if (st) destroy_graphs(H);
  else H->gnv = nv;
  return st;
}

}  // namespace

// ---------------------------------------------------------------- stateless systematic resampler
namespace pfk {

pf_status set_error(pf_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { err_clear(); }

int systematic_check(const double* lw, int64_t n, double u, const int32_t* anc,
                     const double* stats) {
  if (!lw || !anc || !stats) return fail(PF_E_INVAL, "NULL device pointer");
  if (n < 1 || n > (int64_t)0x7fffffff)
    return fail(PF_E_INVAL, "n = %lld must be in [1, 2^31 - 1]", (long long)n);
  if (!(u >= 0.0 && u < 1.0)) return fail(PF_E_INVAL, "u = %g must be in [0, 1)", u);
  return PF_OK;
}

int systematic_enqueue(const double* lw, int64_t n, double u, int32_t* anc, double* stats,
                       char* ws, hipStream_t s) {
  const SysLayout L = sys_layout(n);
  FilterState* fs = (FilterState*)(ws + L.fs);
  PlainArgs a{};
  a.N = n;
  a.ld = n;
  a.nblk = (int32_t)((n + K1_NT - 1) / K1_NT);
  a.T = 1;
  a.fs = fs;
  a.ell_tr = stats;
  a.ess_tr = stats + 1;
  a.rs.scheme = RS_SYSTEMATIC;
  a.rs.steps = 0;
  a.rs.ess_frac = INFINITY;
  a.mode = 2;  // bookkeeping with the given uniform
  int32_t* marks = (int32_t*)(ws + L.marks);
  // every launch is a kernel (no memset, no host copy), so a caller may
  // capture the sequence in a graph
  HIP_TRY(launch_reset(fs, stats, stats + 1, 1, 1, 0u, s));
  HIP_TRY(launch_set_u(fs, u, s));
  HIP_TRY(launch_fill_i32(marks, n, -1, s));
  HIP_TRY(launch_lw_partials(lw, (double*)(ws + L.part), a, s));
  if (a.nblk > FUSE_NB) HIP_TRY(launch_combine((double*)(ws + L.part), (double*)(ws + L.boff), a, s));
  HIP_TRY(launch_scan_mark(lw, (double*)(ws + L.part), (double*)(ws + L.boff), marks,
                           (int32_t*)(ws + L.owner), (int32_t*)(ws + L.jc), a, s));
  HIP_TRY(launch_tile_anc(marks, (int32_t*)(ws + L.owner), (int32_t*)(ws + L.jc), anc, a, s));
  return PF_OK;
}

}  // namespace pfk

extern "C" {

const char* pf_last_error(void) { return g_err; }
const char* pf_version(void) { return "pfmi-gfx950 0.1"; }

size_t pf_workspace_bytes(const pf_config* cfg) {
  if (validate(cfg) != PF_OK) return 0;
  return make_layout(cfg).total;
}

size_t pf_systematic_workspace_bytes(int64_t n) {
  if (n < 1 || n > (int64_t)0x7fffffff) {
    fail(PF_E_INVAL, "n = %lld must be in [1, 2^31 - 1]", (long long)n);
    return 0;
  }
  return pfk::sys_layout(n).total;
}

pf_status pf_systematic(const double* d_lw, int64_t n, double u, int32_t* d_anc, double* d_stats,
                        void* d_workspace, size_t ws_bytes, void* hip_stream) {
  err_clear();
  pf_status st = (pf_status)pfk::systematic_check(d_lw, n, u, d_anc, d_stats);
  if (st) return st;
  if (!d_workspace) return fail(PF_E_INVAL, "workspace is NULL");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(PF_E_INVAL, "workspace not 256-byte aligned");
  const size_t need = pfk::sys_layout(n).total;
  if (ws_bytes < need) return fail(PF_E_INVAL, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return (pf_status)pfk::systematic_enqueue(d_lw, n, u, d_anc, d_stats, (char*)d_workspace,
                                            (hipStream_t)hip_stream);
}


pf_status pf_init(const pf_config* cfg, void* d_workspace, size_t ws_bytes, void* hip_stream,
                  pf_handle** out) {
  err_clear();
  if (!out) return fail(PF_E_INVAL, "out is NULL");
  *out = nullptr;
  pf_status st = validate(cfg);
  if (st) return st;
  Layout L = make_layout(cfg);
  if (!d_workspace) return fail(PF_E_INVAL, "workspace is NULL");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(PF_E_INVAL, "workspace not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(PF_E_INVAL, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  if ((st = require_device())) return st;

  pf_handle* H = new pf_handle();
  H->cfg = *cfg;
  H->L = L;
  H->stream = (hipStream_t)hip_stream;
  H->ws = (char*)d_workspace;
  H->np.assign(cfg->n_particles, cfg->n_particles + cfg->B);
  const pf_config& c = *cfg;
  hipStream_t s = H->stream;
  // host arrays -> device
  std::vector<int32_t> pos(c.d, -1);
  for (int o = 0; o < c.n_obs; ++o) pos[c.obs_idx[o]] = o;
  auto cp = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    return hipMemcpyAsync(H->ws + off, src, bytes, hipMemcpyHostToDevice, s);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = cp(L.obs, c.obs, 8 * (size_t)c.T * c.n_obs);
  if (e == hipSuccess) e = cp(L.obs_pos, pos.data(), 4 * (size_t)c.d);
  if (e == hipSuccess) e = cp(L.obs_idx, c.obs_idx, 4 * (size_t)c.n_obs);
  if (e == hipSuccess && c.model == PF_MODEL_WK) e = cp(L.q, c.q, 8 * ((size_t)c.T * c.K + 1));
  if (e == hipSuccess) e = cp(L.b_off, L.off.data(), 8 * (size_t)(c.B + 1));
  // the plain layout's resampling marks start (and are left by every
  // resampling) at -1
  if (e == hipSuccess && c.layout == PF_LAYOUT_PLAIN)
    e = hipMemsetAsync(H->ws + L.marks, 0xff, 4 * (size_t)L.n_total, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete H;
    return fail(PF_E_DEVICE, "copying the configuration failed: %s", hipGetErrorString(e));
  }
  if ((st = upload_theta(H, c.theta)) || (st = build_groups(H, 1))) {
    destroy_streams(H);
    delete H;
    return st;
  }
  H->cfg.obs = nullptr;
  H->cfg.obs_idx = nullptr;
  H->cfg.q = nullptr;
  H->cfg.n_particles = nullptr;
  H->cfg.theta = nullptr;
  if ((st = do_init(H, s))) {
    delete H;
    return st;
  }
  *out = H;
  return PF_OK;
}

pf_status pf_step(pf_handle* H) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (H->phase != 0) return fail(PF_E_STATE, "pf_step called twice without pf_resample");
  if (H->t >= H->cfg.T) return fail(PF_E_STATE, "all %d observations already processed", H->cfg.T);
  if ((st = enqueue_step(H, H->stream))) return st;
  H->t += 1;
  H->phase = 1;
  return PF_OK;
}

pf_status pf_resample(pf_handle* H) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (H->phase != 1) return fail(PF_E_STATE, "pf_resample needs a preceding pf_step");
  if ((st = enqueue_resample(H, H->stream, nullptr))) return st;
  H->phase = 0;
  return PF_OK;
}

pf_status pf_resample_u(pf_handle* H, const double* u) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!u) return fail(PF_E_INVAL, "u is NULL");
  if (H->rs.scheme != pfk::RS_SYSTEMATIC || std::isfinite(H->rs.ess_frac))
    return fail(PF_E_STATE, "pf_resample_u needs systematic resampling at every time");
  for (int b = 0; b < H->cfg.B; ++b)
    if (!(u[b] >= 0.0 && u[b] < 1.0)) return fail(PF_E_INVAL, "u[%d] must lie in [0, 1)", b);
  if (H->phase != 1) return fail(PF_E_STATE, "pf_resample_u needs a preceding pf_step");
  if ((st = enqueue_resample(H, H->stream, u))) return st;
  H->phase = 0;
  return PF_OK;
}

pf_status pf_loglik(pf_handle* H, double* loglik_out, double* ess_out, int32_t* t_out) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!loglik_out) return fail(PF_E_INVAL, "loglik_out is NULL");
  std::vector<FilterState> fs(H->cfg.B);
  HIP_TRY(hipMemcpyAsync(fs.data(), H->ws + H->L.fs, sizeof(FilterState) * fs.size(),
                         hipMemcpyDeviceToHost, H->stream));
  HIP_TRY(hipStreamSynchronize(H->stream));
  bool numeric = false;
  for (int b = 0; b < H->cfg.B; ++b)
    if (fs[b].pad != 0)
      return fail(PF_E_DEVICE, "internal resampling inconsistency flagged on filter %d", b);
  for (int b = 0; b < H->cfg.B; ++b) {
    loglik_out[b] = fs[b].status ? -INFINITY : fs[b].loglik;
    if (ess_out) ess_out[b] = fs[b].ess;
    numeric |= fs[b].status != 0;
  }
  if (t_out) *t_out = H->t;
  if (numeric) return fail(PF_E_NUMERIC, "a filter met a step with no positive finite weight");
  return PF_OK;
}

pf_status pf_get_trace(pf_handle* H, double* ell_out, double* ess_out) {
  pf_status st = check_handle(H);
  if (st) return st;
  const size_t n = (size_t)H->cfg.B * H->cfg.T;
  if (ell_out)
    HIP_TRY(hipMemcpyAsync(ell_out, H->ws + H->L.ell, 8 * n, hipMemcpyDeviceToHost, H->stream));
  if (ess_out)
    HIP_TRY(hipMemcpyAsync(ess_out, H->ws + H->L.ess, 8 * n, hipMemcpyDeviceToHost, H->stream));
  HIP_TRY(hipStreamSynchronize(H->stream));
  return PF_OK;
}

pf_status pf_destroy(pf_handle* H) {
  if (!H) return fail(PF_E_INVAL, "handle is NULL");
  const pf_status st = H->alive ? drain(H) : PF_OK;
  destroy_streams(H);
  for (auto& ev : H->events) {
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  H->alive = false;
  delete H;
  return st;
}

pf_status pf_graph_run(pf_handle* H, int32_t n_steps) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (n_steps < 0) return fail(PF_E_INVAL, "n_steps must be >= 0");
  if (H->phase != 0) return fail(PF_E_STATE, "pf_graph_run needs a resampled particle set");
  if (H->t + n_steps > H->cfg.T)
    return fail(PF_E_STATE, "%d steps from t = %d exceed T = %d", n_steps, H->t, H->cfg.T);
  if (n_steps == 0) return PF_OK;
  hipStream_t ls;
  if ((st = launch_stream(H, &ls))) return st;
  if (H->eager_replay && H->cfg.layout == PF_LAYOUT_BATCHED) {
    if ((st = enqueue_batched(H, ls, n_steps))) return st;
    H->t += n_steps;
    return PF_OK;
  }
  if ((st = ensure_graphs(H))) return st;
  const bool batched = H->cfg.layout == PF_LAYOUT_BATCHED;
  const int G = batched ? H->groups : 1;
  // group g's graphs go on its own stream (the caller's with one group)
  auto gs = [&](int g) { return G == 1 ? ls : H->side[g]; };
  if (G > 1 && (st = fork_groups(H, ls))) return st;
  // the longest graphs first: n = 200 is 128 + 64 + 8
  int left = n_steps;
  for (int v = H->gnv - 1; v >= 0; --v)
    for (; left >= (1 << v); left -= 1 << v)
      for (int g = 0; g < G; ++g) HIP_TRY(hipGraphLaunch(H->gexecs[g * H->gnv + v], gs(g)));
  if (G > 1 && (st = join_groups(H, ls))) return st;
  H->t += n_steps;
  return PF_OK;
}

pf_status pf_set_theta(pf_handle* H, const double* theta, uint32_t iteration) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!theta) return fail(PF_E_INVAL, "theta is NULL");
  if (iteration >= (1u << 20)) return fail(PF_E_INVAL, "iteration must be < 2^20");
  for (int64_t i = 0; i < (int64_t)H->cfg.B * H->cfg.n_theta; ++i)
    if (!std::isfinite(theta[i])) return fail(PF_E_INVAL, "theta[%lld] not finite", (long long)i);
  if ((st = upload_theta(H, theta))) return st;
  H->iter = iteration;
  return do_init(H, H->stream);
}

pf_status pf_reset(pf_handle* H, uint32_t iteration) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (iteration >= (1u << 20)) return fail(PF_E_INVAL, "iteration must be < 2^20");
  H->iter = iteration;
  return do_init(H, H->stream);
}

// Buffer holding the propagated state of step t (both layouts: the step-t
// state lives in buffer t % 2; buffer 0 holds x(t0)).
static size_t state_buf(const pf_handle* H, int32_t t) {
  return (t & 1) ? H->L.x_tmp : H->L.x_cur;
}

pf_status pf_get_state(pf_handle* H, double* x_out) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!x_out) return fail(PF_E_INVAL, "x_out is NULL");
  const size_t n = (size_t)H->cfg.d * H->L.n_total;
  // both layouts keep interval t's propagated particles in buffer t % 2
  size_t src = state_buf(H, H->t);
  if (H->phase == 0) {  // equally weighted set = propagated[ancestors]
    const size_t spare = state_buf(H, H->t + 1);
    if (H->cfg.layout == PF_LAYOUT_BATCHED) {
      BatchArgs a = batch_args(H);
      HIP_TRY(pfk::launch_batched_gather(H->cfg.precision, H->ws + src, H->at<int32_t>(H->L.anc),
                                         H->ws + spare, a, H->stream));
    } else {
      for (int b = 0; b < H->cfg.B; ++b) {
        PlainArgs a = plain_args(H, b);
        HIP_TRY(pfk::launch_tile_gather(H->cfg.model, H->cfg.d, H->cfg.precision,
                                        H->at<int32_t>(H->L.marks), H->at<int32_t>(H->L.owner),
                                        H->at<int32_t>(H->L.jc), H->ws + H->L.x_cur,
                                        H->ws + H->L.x_tmp, H->at<int32_t>(H->L.anc), a,
                                        H->stream));
        HIP_TRY(pfk::launch_set_amode(a.fs, 1, pfk::AMODE_ARRAY, H->stream));
      }
    }
    src = spare;
  }
  const bool plain = H->cfg.layout == PF_LAYOUT_PLAIN;
  const int d = H->cfg.d;
  const int64_t N = H->L.n_total;
  // the plain layout's state is tiled (pidx); the batched layout's is [d][N]
  const size_t nv = plain ? (size_t)pfk::plain_state_values(N, d) : n;
  auto put = [&](auto* v) {
    for (int i = 0; i < d; ++i)
      for (int64_t g = 0; g < N; ++g)
        x_out[(size_t)i * N + g] = (double)v[plain ? pfk::pidx(g, i, d) : (int64_t)i * N + g];
  };
  if (H->cfg.precision == PF_FP64) {
    std::vector<double> tmp(nv);
    HIP_TRY(hipMemcpyAsync(tmp.data(), H->ws + src, 8 * nv, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    put(tmp.data());
  } else {
    std::vector<float> tmp(nv);
    HIP_TRY(hipMemcpyAsync(tmp.data(), H->ws + src, 4 * nv, hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    put(tmp.data());
  }
  return PF_OK;
}

pf_status pf_set_state(pf_handle* H, const double* x_in) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!x_in) return fail(PF_E_INVAL, "x_in is NULL");
  if (H->phase != 0) return fail(PF_E_STATE, "pf_set_state only between intervals");
  const size_t n = (size_t)H->cfg.d * H->L.n_total;
  const bool batched = H->cfg.layout == PF_LAYOUT_BATCHED;
  const size_t dst = state_buf(H, H->t);
  const int d = H->cfg.d;
  const int64_t N = H->L.n_total;
  // the plain layout's state is tiled (pidx); the batched layout's is [d][N]
  const size_t nv = batched ? n : (size_t)pfk::plain_state_values(N, d);
  auto take = [&](auto* v) {
    for (int i = 0; i < d; ++i)
      for (int64_t g = 0; g < N; ++g)
        v[batched ? (int64_t)i * N + g : pfk::pidx(g, i, d)] = x_in[(size_t)i * N + g];
  };
  if (H->cfg.precision == PF_FP64) {
    std::vector<double> tmp(nv, 0.0);
    take(tmp.data());
    HIP_TRY(hipMemcpyAsync(H->ws + dst, tmp.data(), 8 * nv, hipMemcpyHostToDevice, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
  } else {
    std::vector<float> tmp(nv, 0.0f);
    take(tmp.data());
    HIP_TRY(hipMemcpyAsync(H->ws + dst, tmp.data(), 4 * nv, hipMemcpyHostToDevice, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
  }
  if (!batched) {  // the next step reads the given particles as they are
    HIP_TRY(pfk::launch_fill_i32(H->at<int32_t>(H->L.marks), H->L.n_total, -1, H->stream));
    HIP_TRY(pfk::launch_set_amode(H->at<FilterState>(H->L.fs), H->cfg.B, pfk::AMODE_IDENTITY,
                                  H->stream));
  } else {  // the next step reads the given particles as they are
    std::vector<int32_t> ident((size_t)H->L.n_total);
    for (int b = 0; b < H->cfg.B; ++b)
      for (int64_t k = 0; k < H->np[b]; ++k) ident[(size_t)(H->L.off[b] + k)] = (int32_t)k;
    HIP_TRY(hipMemcpyAsync(H->ws + H->L.anc, ident.data(), 4 * ident.size(),
                           hipMemcpyHostToDevice, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
  }
  HIP_TRY(hipStreamSynchronize(H->stream));
  return PF_OK;
}

pf_status pf_restore(pf_handle* H, int32_t t, const double* x_in, const double* loglik) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!x_in || !loglik) return fail(PF_E_INVAL, "x_in and loglik must not be NULL");
  if (H->phase != 0) return fail(PF_E_STATE, "pf_restore only between intervals");
  if (t < 0 || t > H->cfg.T) return fail(PF_E_INVAL, "t = %d outside [0, T = %d]", t, H->cfg.T);
  if (H->hist) return fail(PF_E_STATE, "pf_restore on a handle with a history attached");
  const int B = H->cfg.B;
  for (int b = 0; b < B; ++b)
    if (std::isnan(loglik[b]) || loglik[b] == INFINITY)
      return fail(PF_E_INVAL, "loglik[%d] is NaN or +infinity", b);
  if ((st = drain(H))) return st;
  // every filter at t, equally weighted (no carried weights), with the
  // given running likelihood; -infinity keeps the numeric flag
  std::vector<FilterState> fs((size_t)B);
  HIP_TRY(hipMemcpyAsync(fs.data(), H->ws + H->L.fs, sizeof(FilterState) * fs.size(),
                         hipMemcpyDeviceToHost, H->stream));
  HIP_TRY(hipStreamSynchronize(H->stream));
  for (int b = 0; b < B; ++b) {
    FilterState& f = fs[(size_t)b];
    f.loglik = loglik[b];
    f.status = std::isfinite(loglik[b]) ? 0 : 4;
    f.M = f.S = f.u = f.ell = f.ess = f.lprev = 0.0;
    f.t = t;
    f.tk = t;
    f.carry = 0;
    f.pad = 0;
    f.cn1 = 0;
    f.amode = pfk::AMODE_IDENTITY;
  }
  HIP_TRY(hipMemcpyAsync(H->ws + H->L.fs, fs.data(), sizeof(FilterState) * fs.size(),
                         hipMemcpyHostToDevice, H->stream));
  // trace rows from t on start empty, as after pf_init
  const size_t T = (size_t)H->cfg.T;
  std::vector<double> tr((size_t)B * T);
  for (size_t L : {H->L.ell, H->L.ess}) {
    HIP_TRY(hipMemcpyAsync(tr.data(), H->ws + L, 8 * tr.size(), hipMemcpyDeviceToHost, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
    for (int b = 0; b < B; ++b)
      for (size_t i = (size_t)t; i < T; ++i) tr[(size_t)b * T + i] = 0.0;
    HIP_TRY(hipMemcpyAsync(H->ws + L, tr.data(), 8 * tr.size(), hipMemcpyHostToDevice, H->stream));
    HIP_TRY(hipStreamSynchronize(H->stream));
  }
  // the particles go to the buffer of interval t, read through the identity
  H->t = t;
  return pf_set_state(H, x_in);
}

pf_status pf_get_logweights(pf_handle* H, double* lw_out) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!lw_out) return fail(PF_E_INVAL, "lw_out is NULL");
  if (H->t == 0) return fail(PF_E_STATE, "no step taken yet");
  HIP_TRY(hipMemcpyAsync(lw_out, H->ws + H->L.lw, 8 * (size_t)H->L.n_total,
                         hipMemcpyDeviceToHost, H->stream));
  HIP_TRY(hipStreamSynchronize(H->stream));
  return PF_OK;
}

pf_status pf_get_ancestors(pf_handle* H, int32_t* a_out) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!a_out) return fail(PF_E_INVAL, "a_out is NULL");
  if (H->cfg.layout == PF_LAYOUT_PLAIN && H->phase == 0 && H->t > 0)
    for (int b = 0; b < H->cfg.B; ++b)  // the pending ancestors, written out
      if ((st = plain_anc_out(H, b, H->stream))) return st;
  HIP_TRY(hipMemcpyAsync(a_out, H->ws + H->L.anc, 4 * (size_t)H->L.n_total,
                         hipMemcpyDeviceToHost, H->stream));
  HIP_TRY(hipStreamSynchronize(H->stream));
  return PF_OK;
}

static size_t sim_out_doubles(const pf_config* c) {
  return (size_t)(c->T + 1) * c->d + (size_t)c->T * c->n_obs;
}
static size_t sim_scratch_doubles(const pf_config* c) {
  const size_t nq = c->model == PF_MODEL_WK ? ((size_t)c->T * c->K + 1) : 0;
  return 8 + nq + ((size_t)c->n_obs + 1) / 2;
}

size_t pf_simulate_doubles(const pf_config* cfg) {
  if (!cfg) return 0;
  return sim_out_doubles(cfg) + sim_scratch_doubles(cfg) + 32;
}

pf_status pf_simulate(const pf_config* cfg, const double* theta, uint64_t data_seed,
                      double* d_out, size_t out_doubles, void* hip_stream) {
  err_clear();
  if (!cfg || !theta || !d_out) return fail(PF_E_INVAL, "NULL argument");
  pf_config c = *cfg;
  // the filter-only fields are not needed here
  std::vector<double> dummy_obs((size_t)c.T * c.n_obs, 0.0);
  int64_t one = 1;
  c.obs = dummy_obs.data();
  c.B = 1;
  c.n_particles = &one;
  c.theta = theta;
  c.layout = PF_LAYOUT_PLAIN;
  pf_status st = validate(&c);
  if (st) return st;
  if (out_doubles < pf_simulate_doubles(&c))
    return fail(PF_E_INVAL, "output buffer has %zu doubles, needs %zu", out_doubles,
                pf_simulate_doubles(&c));
  if ((st = require_device())) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<double> th;
  derive_theta(&c, theta, th);
  const size_t nq = c.model == PF_MODEL_WK ? ((size_t)c.T * c.K + 1) : 0;
  // scratch after the outputs, 256-byte aligned
  const size_t base = (sim_out_doubles(&c) + 31) & ~(size_t)31;
  double* dth = d_out + base;
  double* dq = dth + 8;
  int32_t* didx = (int32_t*)(dq + nq);
  HIP_TRY(hipMemcpyAsync(dth, th.data(), 64, hipMemcpyHostToDevice, s));
  if (nq) HIP_TRY(hipMemcpyAsync(dq, c.q, 8 * nq, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(didx, c.obs_idx, 4 * (size_t)c.n_obs, hipMemcpyHostToDevice, s));
  PlainArgs a{};
  a.K = c.K;
  a.T = c.T;
  a.d = c.d;
  a.n_obs = c.n_obs;
  a.key.lo = (uint32_t)(data_seed & 0xffffffffu);
  a.key.hi = (uint32_t)(data_seed >> 32);
  a.h = c.h;
  a.hh = 0.5 * c.h;
  a.h6 = c.h / 6.0;
  a.theta = dth;
  a.q = nq ? dq : nullptr;
  a.obs_idx = didx;
  HIP_TRY(pfk::launch_simulate(c.model, c.d, d_out, a, c.obs_sd, s));
  HIP_TRY(hipStreamSynchronize(s));
  return PF_OK;
}

// Advance every filter through all T intervals from a fresh start, through
// the captured graph.
static pf_status run_full(pf_handle* H) {
  pf_status st = pf_graph_run(H, H->cfg.T - H->t);
  if (st) return st;
  H->phase = 0;
  return PF_OK;
}

pf_status pf_pmmh(pf_handle* H, int32_t iters, const double* log_f0, const double* z,
                  const double* alpha, double step_sd, double f_lo, double f_hi, double sigma,
                  double* log_f_trace, double* ll_trace, int32_t* accepts) {
  pf_status st = check_handle(H);
  if (st) return st;
  const pf_config& c = H->cfg;
  if (c.model != PF_MODEL_L96 && c.model != PF_MODEL_L96_STAGE)
    return fail(PF_E_INVAL, "pf_pmmh needs a Lorenz '96 model");
  if (iters < 0 || iters + 1 >= (1 << 20)) return fail(PF_E_INVAL, "iters out of range");
  if (!log_f0 || (iters > 0 && (!z || !alpha || !log_f_trace || !ll_trace)) || !accepts)
    return fail(PF_E_INVAL, "NULL argument");
  if (!(step_sd >= 0.0) || !(f_lo < f_hi) || !(sigma >= 0.0))
    return fail(PF_E_INVAL, "step_sd, prior bounds or sigma invalid");
  const int B = c.B;
  std::vector<double> th(B), thp(B), ll(B), llp(B), theta(2 * (size_t)B), ess(B);
  for (int b = 0; b < B; ++b) {
    th[b] = log_f0[b];
    theta[2 * b] = std::exp(th[b]);
    theta[2 * b + 1] = sigma;
    accepts[b] = 0;
  }
  // initial estimate with iteration field 0
  if ((st = pf_set_theta(H, theta.data(), 0))) return st;
  if ((st = run_full(H))) return st;
  st = pf_loglik(H, ll.data(), ess.data(), nullptr);
  if (st && st != PF_E_NUMERIC) return st;
  std::vector<char> inside(B);
  for (int32_t i = 0; i < iters; ++i) {
    for (int b = 0; b < B; ++b) {
      thp[b] = th[b] + step_sd * z[(size_t)i * B + b];
      const double Fp = std::exp(thp[b]);
      inside[b] = (Fp >= f_lo && Fp <= f_hi);
      // a proposal outside the prior's support is rejected without a filter
      // estimate; its filter slot reruns the current value meanwhile
      theta[2 * b] = inside[b] ? Fp : std::exp(th[b]);
    }
    if ((st = pf_set_theta(H, theta.data(), (uint32_t)(i + 1)))) return st;
    if ((st = run_full(H))) return st;
    st = pf_loglik(H, llp.data(), ess.data(), nullptr);
    if (st && st != PF_E_NUMERIC) return st;
    for (int b = 0; b < B; ++b) {
      if (inside[b] && std::log(alpha[(size_t)i * B + b]) <= (llp[b] - ll[b]) + (thp[b] - th[b])) {
        th[b] = thp[b];
        ll[b] = llp[b];
        accepts[b] += 1;
      }
      log_f_trace[(size_t)i * B + b] = th[b];
      ll_trace[(size_t)i * B + b] = ll[b];
    }
  }
  err_clear();
  return PF_OK;
}

// Device workspace of pf_smc2: its inputs, the theta-particle state and the
// traces, each 256-byte aligned.
struct Smc2Layout {
  size_t z, la, w, raw, prop_raw, snap_dev, snap_raw, snap_ll, snap_st, a, inside, accepted,
      accepts, evid, numeric, ess, anc_tr, acc_tr, theta_tr, mV, snap_mV, prop_dev, prop_l,
      prop_mV, total;
};

static Smc2Layout smc2_layout(int64_t B, int64_t nth, int64_t T) {
  Smc2Layout L{};
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at = p;
    p = align256(p + (bytes > 0 ? bytes : 1));
    return at;
  };
  L.z = take(8 * (size_t)(T * B * nth));
  L.la = take(8 * (size_t)(T * B));
  L.w = take(4 * (size_t)(T * B));
  L.raw = take(8 * (size_t)(B * nth));
  L.prop_raw = take(8 * (size_t)(B * nth));
  L.snap_dev = take(8 * 8 * (size_t)B);
  L.snap_raw = take(8 * (size_t)(B * nth));
  L.snap_ll = take(8 * (size_t)B);
  L.snap_st = take(4 * (size_t)B);
  L.a = take(4 * (size_t)B);
  L.inside = take(4 * (size_t)B);
  L.accepted = take(4 * (size_t)B);
  L.accepts = take(4 * (size_t)B);
  L.evid = take(8);
  L.numeric = take(4);
  L.ess = take(8 * (size_t)T);
  L.anc_tr = take(4 * (size_t)(T * B));
  L.acc_tr = take(4 * (size_t)(T * B));
  L.theta_tr = take(8 * (size_t)(T * B * nth));
  L.mV = take(16 * (size_t)B);
  L.snap_mV = take(16 * (size_t)B);
  L.prop_dev = take(64 * (size_t)B);
  L.prop_l = take(8 * (size_t)B);
  L.prop_mV = take(16 * (size_t)B);
  L.total = p;
  return L;
}

size_t pf_smc2_workspace_bytes(const pf_config* cfg, int32_t T_run) {
  if (validate(cfg) != PF_OK) return 0;
  if (T_run < 1 || T_run > cfg->T) {
    fail(PF_E_INVAL, "T_run must be in [1, T]");
    return 0;
  }
  return smc2_layout(cfg->B, cfg->n_theta, T_run).total;
}

static bool same_config(const pf_handle* A, const pf_handle* B) {
  const pf_config &a = A->cfg, &b = B->cfg;
  return a.model == b.model && a.precision == b.precision && a.layout == b.layout &&
         a.d == b.d && a.K == b.K && a.T == b.T && a.h == b.h && a.n_obs == b.n_obs &&
         a.obs_sd == b.obs_sd && a.B == b.B && a.n_theta == b.n_theta && a.seed == b.seed &&
         A->np == B->np;
}

pf_status pf_smc2(pf_handle* H, pf_handle* P, void* d_ws, size_t ws_bytes, const pf_smc2_in* in,
                  pf_smc2_out* out) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!in || !out) return fail(PF_E_INVAL, "NULL argument");
  const pf_config& c = H->cfg;
  const bool kalman = in->filter == PF_FILTER_KALMAN;
  if (in->filter != PF_FILTER_PARTICLE && !kalman)
    return fail(PF_E_INVAL, "unknown filter kind %d", in->filter);
  if (kalman) {
    if (c.model != PF_MODEL_WK) return fail(PF_E_INVAL, "Kalman filters need the windkessel model");
  } else {
    if ((st = check_handle(P))) return st;
    if (H == P) return fail(PF_E_INVAL, "the proposal handle must be a second handle");
    if (c.layout != PF_LAYOUT_BATCHED) return fail(PF_E_INVAL, "pf_smc2 needs the batched layout");
    if (!same_config(H, P))
      return fail(PF_E_INVAL, "the proposal handle's configuration differs from the handle's");
    if (H->stream != P->stream) return fail(PF_E_INVAL, "both handles must use the same stream");
    if (H->hist || P->hist)
      return fail(PF_E_STATE, "pf_smc2 does not keep histories: detach them first");
    if (std::isfinite(H->rs.ess_frac) || std::isfinite(P->rs.ess_frac))
      return fail(PF_E_STATE, "pf_smc2 needs resampling at every time (equally weighted filters)");
  }
  if (c.B > pfk::SMC2_MAXB) return fail(PF_E_INVAL, "at most %d theta-particles", pfk::SMC2_MAXB);
  if (c.n_theta > 8) return fail(PF_E_INVAL, "at most 8 parameters");
  const int32_t T = in->T_run;
  if (T < 1 || T > c.T) return fail(PF_E_INVAL, "T_run must be in [1, %d]", c.T);
  if (T >= (1 << 20)) return fail(PF_E_INVAL, "T_run must be < 2^20");
  if (!in->theta0 || !in->z || !in->log_alpha || !in->u || !in->w_copy)
    return fail(PF_E_INVAL, "NULL input array");
  if (!out->theta || !out->logw || !out->loglik || !out->accepts || !out->ess ||
      !out->log_evidence)
    return fail(PF_E_INVAL, "NULL output array");
  const int B = c.B, nth = c.n_theta;
  for (int p = 0; p < nth; ++p)
    if (!(in->step_sd[p] >= 0.0) || !std::isfinite(in->step_sd[p]) ||
        (in->step_sd[p] > 0.0 && !(in->lo[p] <= in->hi[p])))
      return fail(PF_E_INVAL, "step_sd[%d] or its prior box invalid", p);
  for (int32_t i = 0; i < T; ++i)
    if (!(in->u[i] >= 0.0 && in->u[i] < 1.0)) return fail(PF_E_INVAL, "u[%d] not in [0, 1)", i);
  for (int64_t i = 0; i < (int64_t)T * B * nth; ++i)
    if (!std::isfinite(in->z[i])) return fail(PF_E_INVAL, "z[%lld] not finite", (long long)i);
  const Smc2Layout L = smc2_layout(B, nth, T);
  if (!d_ws) return fail(PF_E_INVAL, "workspace is NULL");
  if (((uintptr_t)d_ws & 255) != 0) return fail(PF_E_INVAL, "workspace not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(PF_E_INVAL, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  char* ws = (char*)d_ws;
  hipStream_t s = H->stream;

  // h starts from theta0 with iteration field 0
  if ((st = pf_set_theta(H, in->theta0, 0))) return st;
  HIP_TRY(hipMemcpyAsync(ws + L.z, in->z, 8 * (size_t)T * B * nth, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws + L.la, in->log_alpha, 8 * (size_t)T * B, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws + L.w, in->w_copy, 4 * (size_t)T * B, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ws + L.raw, in->theta0, 8 * (size_t)B * nth, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(ws + L.accepts, 0, 4 * (size_t)B, s));
  HIP_TRY(hipMemsetAsync(ws + L.evid, 0, 8, s));
  HIP_TRY(hipMemsetAsync(ws + L.numeric, 0, 4, s));
  HIP_TRY(hipMemsetAsync(ws + L.anc_tr, 0, 4 * (size_t)B, s));  // time 1: identity, below
  HIP_TRY(hipStreamSynchronize(s));
  {
    std::vector<int32_t> ident(B);
    for (int j = 0; j < B; ++j) ident[j] = j;
    HIP_TRY(hipMemcpyAsync(ws + L.anc_tr, ident.data(), 4 * (size_t)B, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  // capture both handles' graphs before the loop
  if (!kalman && ((st = ensure_graphs(H)) || (st = ensure_graphs(P)))) return st;

  pfk::Smc2Args S{};
  S.B = B;
  S.T = c.T;
  S.n_theta = nth;
  S.model = c.model;
  S.sqrt_h = std::sqrt(c.h);
  for (int p = 0; p < 8; ++p) {
    S.step_sd[p] = p < nth ? in->step_sd[p] : 0.0;
    S.lo[p] = p < nth ? in->lo[p] : 0.0;
    S.hi[p] = p < nth ? in->hi[p] : 0.0;
  }
  S.ell_tr = H->at<double>(H->L.ell);
  S.fs = H->at<FilterState>(H->L.fs);
  S.theta_dev = H->at<double>(H->L.theta);
  S.raw = (double*)(ws + L.raw);
  S.prop_raw = (double*)(ws + L.prop_raw);
  S.snap_dev = (double*)(ws + L.snap_dev);
  S.snap_raw = (double*)(ws + L.snap_raw);
  S.snap_ll = (double*)(ws + L.snap_ll);
  S.snap_st = (int32_t*)(ws + L.snap_st);
  S.a = (int32_t*)(ws + L.a);
  S.inside = (int32_t*)(ws + L.inside);
  S.accepted = (int32_t*)(ws + L.accepted);
  S.accepts = (int32_t*)(ws + L.accepts);
  S.evid = (double*)(ws + L.evid);
  S.numeric = (int32_t*)(ws + L.numeric);
  S.mV = kalman ? (double*)(ws + L.mV) : nullptr;
  S.snap_mV = kalman ? (double*)(ws + L.snap_mV) : nullptr;
  S.ell_tr_w = H->at<double>(H->L.ell);
  const BatchArgs A = batch_args(H);
  double* ess_d = (double*)(ws + L.ess);
  int32_t* anc_tr = (int32_t*)(ws + L.anc_tr);
  int32_t* acc_tr = (int32_t*)(ws + L.acc_tr);
  const double* z_d = (const double*)(ws + L.z);
  const double* la_d = (const double*)(ws + L.la);
  const uint32_t* w_d = (const uint32_t*)(ws + L.w);
  if (kalman) {
    pfk::KfArgs K{};
    K.B = B;
    K.K = c.K;
    K.T = c.T;
    K.R = c.obs_sd * c.obs_sd;
    K.q = H->at<double>(H->L.q);
    K.obs = H->at<double>(H->L.obs);
    double* prop_dev_k = (double*)(ws + L.prop_dev);
    double* prop_l = (double*)(ws + L.prop_l);
    double* prop_mV = (double*)(ws + L.prop_mV);
    HIP_TRY(pfk::launch_kf_init(S, s));
    for (int32_t i = 1; i <= T; ++i) {
      if (i >= 2)
        HIP_TRY(pfk::launch_theta_resample(S, i - 2, in->u[i - 1], 1,
                                           anc_tr + (size_t)(i - 1) * B, ess_d + (i - 2), s));
      HIP_TRY(pfk::launch_smc2_propose(S, z_d + (size_t)(i - 1) * B * nth, prop_dev_k, s));
      HIP_TRY(pfk::launch_kf_proposal(K, S, prop_dev_k, prop_l, prop_mV, i, s));
      HIP_TRY(pfk::launch_smc2_accept_kf(S, la_d + (size_t)(i - 1) * B, prop_dev_k, prop_l,
                                         prop_mV, acc_tr + (size_t)(i - 1) * B, s));
      HIP_TRY(pfk::launch_kf_advance(K, S, i, s));
      HIP_TRY(hipMemcpyAsync(ws + L.theta_tr + 8 * (size_t)(i - 1) * B * nth, ws + L.raw,
                             8 * (size_t)B * nth, hipMemcpyDeviceToDevice, s));
    }
  }
  double* prop_dev = kalman ? nullptr : P->at<double>(P->L.theta);

  for (int32_t i = 1; i <= T && !kalman; ++i) {
    const size_t cur = state_buf(H, i - 1), spare = state_buf(H, i);
    if (i >= 2) {
      // 1-2. theta-ancestors from v(t_{i-1}), the slots' moves and filter copies
      HIP_TRY(pfk::launch_theta_resample(S, i - 2, in->u[i - 1], 1, anc_tr + (size_t)(i - 1) * B,
                                         ess_d + (i - 2), s));
      HIP_TRY(pfk::launch_filter_copy(c.precision, H->ws + cur, H->ws + spare,
                                      H->at<int32_t>(H->L.anc), A, S, w_d + (size_t)(i - 1) * B,
                                      s));
    }
    // 3. rejuvenation: proposals, their filters over t_{0:i-1}, the decisions
    HIP_TRY(pfk::launch_smc2_propose(S, z_d + (size_t)(i - 1) * B * nth, prop_dev, s));
    P->iter = (uint32_t)i;
    if ((st = do_init(P, s))) return st;
    if (i > 1 && (st = pf_graph_run(P, i - 1))) return st;
    HIP_TRY(pfk::launch_smc2_accept(S, la_d + (size_t)(i - 1) * B, prop_dev,
                                    P->at<FilterState>(P->L.fs), acc_tr + (size_t)(i - 1) * B,
                                    s));
    HIP_TRY(pfk::launch_accept_copy(c.precision, H->ws + cur, H->at<int32_t>(H->L.anc),
                                    P->ws + state_buf(P, i - 1), P->at<int32_t>(P->L.anc), A, S,
                                    s));
    // 4. every attached filter advances one interval
    if ((st = pf_graph_run(H, 1))) return st;
    HIP_TRY(hipMemcpyAsync(ws + L.theta_tr + 8 * (size_t)(i - 1) * B * nth, ws + L.raw,
                           8 * (size_t)B * nth, hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(pfk::launch_theta_resample(S, T - 1, 0.5, 0, nullptr, ess_d + (T - 1), s));

  // outputs
  std::vector<double> ell((size_t)B * c.T);
  std::vector<FilterState> fs(B);
  int32_t numeric = 0;
  HIP_TRY(hipMemcpyAsync(out->theta, ws + L.raw, 8 * (size_t)B * nth, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(ell.data(), H->ws + H->L.ell, 8 * ell.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(fs.data(), H->ws + H->L.fs, sizeof(FilterState) * (size_t)B,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(out->accepts, ws + L.accepts, 4 * (size_t)B, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(out->ess, ws + L.ess, 8 * (size_t)T, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(out->log_evidence, ws + L.evid, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&numeric, ws + L.numeric, 4, hipMemcpyDeviceToHost, s));
  if (out->anc_trace)
    HIP_TRY(hipMemcpyAsync(out->anc_trace, ws + L.anc_tr, 4 * (size_t)T * B,
                           hipMemcpyDeviceToHost, s));
  if (out->acc_trace)
    HIP_TRY(hipMemcpyAsync(out->acc_trace, ws + L.acc_tr, 4 * (size_t)T * B,
                           hipMemcpyDeviceToHost, s));
  if (out->theta_trace)
    HIP_TRY(hipMemcpyAsync(out->theta_trace, ws + L.theta_tr, 8 * (size_t)T * B * nth,
                           hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int j = 0; j < B; ++j) {
    out->logw[j] = ell[(size_t)j * c.T + (T - 1)];
    out->loglik[j] = fs[j].status ? -INFINITY : fs[j].loglik;
    if (out->logw_trace)
      for (int32_t i = 0; i < T; ++i) out->logw_trace[(size_t)i * B + j] = ell[(size_t)j * c.T + i];
  }
  if (kalman) {
    // the handle's particle filters did not move: start them afresh
    if ((st = pf_reset(H, 0))) return st;
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (numeric) return fail(PF_E_NUMERIC, "some time had no positive theta-weight");
  err_clear();
  return PF_OK;
}

pf_status pf_kalman(pf_handle* H, double* loglik_out, double* ell_out) {
  pf_status st = check_handle(H);
  if (st) return st;
  const pf_config& c = H->cfg;
  if (c.model != PF_MODEL_WK) return fail(PF_E_INVAL, "pf_kalman needs the windkessel model");
  if (!loglik_out) return fail(PF_E_INVAL, "loglik_out is NULL");
  pfk::KfArgs K{};
  K.B = c.B;
  K.K = c.K;
  K.T = c.T;
  K.R = c.obs_sd * c.obs_sd;
  K.q = H->at<double>(H->L.q);
  K.obs = H->at<double>(H->L.obs);
  HIP_TRY(pfk::launch_kf_run(K, H->at<double>(H->L.theta), H->at<double>(H->L.kf_ll),
                             H->at<double>(H->L.kf_ell), H->stream));
  HIP_TRY(hipMemcpyAsync(loglik_out, H->ws + H->L.kf_ll, 8 * (size_t)c.B, hipMemcpyDeviceToHost,
                         H->stream));
  if (ell_out)
    HIP_TRY(hipMemcpyAsync(ell_out, H->ws + H->L.kf_ell, 8 * (size_t)c.B * c.T,
                           hipMemcpyDeviceToHost, H->stream));
  HIP_TRY(hipStreamSynchronize(H->stream));
  return PF_OK;
}

pf_status pf_kalman_pmmh(pf_handle* H, const pf_wk_mh* spec, int32_t iters,
                         const double* d_theta0, const double* d_prop, const double* d_alpha,
                         double* d_theta_trace, double* d_ll_trace, int32_t* d_accepts,
                         double* d_ll0) {
  pf_status st = check_handle(H);
  if (st) return st;
  const pf_config& c = H->cfg;
  if (c.model != PF_MODEL_WK) return fail(PF_E_INVAL, "pf_kalman_pmmh needs the windkessel model");
  if (!spec) return fail(PF_E_INVAL, "spec is NULL");
  auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
  auto nonneg = [](double v) { return std::isfinite(v) && v >= 0.0; };
  for (int k = 0; k < 3; ++k)
    if (!pos(spec->prior_shape[k]) || !pos(spec->prior_scale[k]) || !nonneg(spec->step_sd[k]))
      return fail(PF_E_INVAL, "prior shape/scale of parameter %d must be > 0, step sd >= 0", k);
  if (!pos(spec->ig_shape) || !pos(spec->ig_scale))
    return fail(PF_E_INVAL, "Inverse-Gamma prior shape and scale must be > 0");
  if (!nonneg(spec->ig_prop_factor) || (spec->ig_prop_factor > 0.0 && !pos(spec->ig_prop_shape)))
    return fail(PF_E_INVAL, "sigma^2 proposal factor must be >= 0 and its shape > 0");
  if (!std::isfinite(spec->m0) || !nonneg(spec->s0))
    return fail(PF_E_INVAL, "m0 must be finite and s0 >= 0");
  if (iters < 0) return fail(PF_E_INVAL, "iters < 0");
  if (!d_theta0 || !d_accepts) return fail(PF_E_INVAL, "NULL argument");
  if (iters > 0 && (!d_prop || !d_alpha || !d_theta_trace || !d_ll_trace))
    return fail(PF_E_INVAL, "NULL argument");
  const void* ptrs[] = {d_theta0, d_prop, d_alpha, d_theta_trace, d_ll_trace, d_ll0};
  for (const void* p : ptrs)
    if (((uintptr_t)p & 7) != 0) return fail(PF_E_INVAL, "arrays must be 8-byte aligned");
  if (((uintptr_t)d_accepts & 3) != 0) return fail(PF_E_INVAL, "accepts must be 4-byte aligned");
  pfk::KfArgs K{};
  K.B = c.B;
  K.K = c.K;
  K.T = c.T;
  K.R = c.obs_sd * c.obs_sd;
  K.q = H->at<double>(H->L.q);
  K.obs = H->at<double>(H->L.obs);
  HIP_TRY(pfk::launch_kf_pmmh(K, *spec, c.h, iters, d_theta0, d_prop, d_alpha, d_theta_trace,
                              d_ll_trace, d_accepts, d_ll0, H->stream));
  err_clear();
  return PF_OK;
}

size_t pf_history_bytes(const pf_config* cfg) {
  if (validate(cfg) != PF_OK) return 0;
  return hist_layout(cfg, make_layout(cfg).n_total).total;
}

pf_status pf_history_attach(pf_handle* H, void* d_hist, size_t bytes) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (d_hist) {
    if (H->t != 0 || H->phase != 0)
      return fail(PF_E_STATE, "attach a history at t = 0 (after pf_init or pf_reset)");
    if (((uintptr_t)d_hist & 255) != 0) return fail(PF_E_INVAL, "history not 256-byte aligned");
    const size_t need = hist_layout(&H->cfg, H->L.n_total).total;
    if (bytes < need) return fail(PF_E_INVAL, "history has %zu bytes, needs %zu", bytes, need);
  }
  if ((st = drain(H))) return st;
  destroy_graphs(H);  // recaptured with (or without) the recording kernels
  H->hist = (char*)d_hist;
  if (d_hist && (st = record_all(H, H->stream))) return st;
  HIP_TRY(hipStreamSynchronize(H->stream));
  return PF_OK;
}

pf_status pf_backtrace(pf_handle* H, double* path_out, int32_t* idx_out) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!H->hist) return fail(PF_E_STATE, "no history attached");
  if (!path_out) return fail(PF_E_INVAL, "path_out is NULL");
  if (H->phase != 0) return fail(PF_E_STATE, "pf_backtrace needs a resampled particle set");
  if (std::isfinite(H->rs.ess_frac))
    return fail(PF_E_STATE, "pf_backtrace needs resampling at every time");
  const pf_config& c = H->cfg;
  const HistLayout L = hist_layout(&c, H->L.n_total);
  const int32_t t = H->t;
  pfk::KeyArg key;
  key.lo = (uint32_t)(c.seed & 0xffffffffu);
  key.hi = (uint32_t)(c.seed >> 32);
  HIP_TRY(pfk::launch_backtrace(c.precision, hist_args(H), c.B, H->at<int64_t>(H->L.b_off),
                                H->at<FilterState>(H->L.fs), key, (int32_t*)(H->hist + L.idx),
                                (double*)(H->hist + L.path), H->stream));
  std::vector<double> path((size_t)c.B * (c.T + 1) * c.d);
  std::vector<int32_t> idx((size_t)c.B * (c.T + 1));
  HIP_TRY(hipMemcpyAsync(path.data(), H->hist + L.path, 8 * path.size(), hipMemcpyDeviceToHost,
                         H->stream));
  HIP_TRY(hipMemcpyAsync(idx.data(), H->hist + L.idx, 4 * idx.size(), hipMemcpyDeviceToHost,
                         H->stream));
  HIP_TRY(hipStreamSynchronize(H->stream));
  for (int b = 0; b < c.B; ++b) {
    std::memcpy(path_out + (size_t)b * (t + 1) * c.d, path.data() + (size_t)b * (c.T + 1) * c.d,
                8 * (size_t)(t + 1) * c.d);
    if (idx_out)
      std::memcpy(idx_out + (size_t)b * (t + 1), idx.data() + (size_t)b * (c.T + 1),
                  4 * (size_t)(t + 1));
  }
  return PF_OK;
}

pf_status pf_set_resampler(pf_handle* H, int32_t scheme, int32_t steps, double ess_frac) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (scheme != PF_RESAMPLE_SYSTEMATIC && scheme != PF_RESAMPLE_STRATIFIED &&
      scheme != PF_RESAMPLE_METROPOLIS && scheme != PF_RESAMPLE_MULTINOMIAL &&
      scheme != PF_RESAMPLE_REJECTION)
    return fail(PF_E_INVAL, "unknown resampler %d", scheme);
  if (scheme == PF_RESAMPLE_REJECTION && H->cfg.T >= (1 << 20))
    return fail(PF_E_INVAL, "rejection resampling needs T < 2^20 (its generator counters)");
  if (steps < 0 || steps > PF_METROPOLIS_MAX_STEPS)
    return fail(PF_E_INVAL, "steps must be in [0, %d]", PF_METROPOLIS_MAX_STEPS);
  if (!(ess_frac >= 0.0)) return fail(PF_E_INVAL, "ess_frac must be >= 0 (or +inf)");
  if ((st = drain(H))) return st;
  destroy_graphs(H);
  H->rs.scheme = scheme;
  H->rs.steps = steps;
  H->rs.ess_frac = ess_frac;
  return PF_OK;
}

pf_status pf_set_tuning(pf_handle* H, int32_t collective_threads, int32_t groups) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (collective_threads != 256 && collective_threads != 512 && collective_threads != 1024)
    return fail(PF_E_INVAL, "collective_threads must be 256, 512 or 1024");
  if (groups < 1 || groups > 8) return fail(PF_E_INVAL, "groups must be in [1, 8]");
  if (H->cfg.layout != PF_LAYOUT_BATCHED) return PF_OK;  // nothing to tune
  // the tuning the handle has already: nothing changes (its graphs and the
  // replay choice stay)
  if (collective_threads == H->batch_nt && std::min(groups, H->cfg.B) == H->groups) return PF_OK;
  if ((st = drain(H))) return st;
  destroy_graphs(H);
  H->eager_replay = false;  // graph replay until a tuner run compares the two
  H->batch_nt = collective_threads;
  if (groups != H->groups) return build_groups(H, groups);
  return PF_OK;
}

pf_status pf_set_replay(pf_handle* H, int32_t eager) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (eager != 0 && eager != 1) return fail(PF_E_INVAL, "eager must be 0 or 1");
  if (H->cfg.layout != PF_LAYOUT_BATCHED) return PF_OK;  // the plain layout always replays graphs
  H->eager_replay = eager == 1;
  return PF_OK;
}

pf_status pf_get_tuning(pf_handle* H, int32_t* collective_threads, int32_t* groups,
                        int32_t* eager_replay) {
  pf_status st = check_handle(H);
  if (st) return st;
  const bool batched = H->cfg.layout == PF_LAYOUT_BATCHED;
  if (collective_threads) *collective_threads = batched ? H->batch_nt : 0;
  if (groups) *groups = batched ? H->groups : 0;
  if (eager_replay) *eager_replay = (batched && H->eager_replay) ? 1 : 0;
  return PF_OK;
}

namespace {
// Mean interval time (ms) of n intervals replayed from the handle's graphs
// after a fresh initialisation and one untimed graph interval (t + 1 + n
// must not exceed T).
pf_status time_graph_replay(pf_handle* H, int n, double* ms_out) {
  pf_status st = do_init(H, H->stream);
  if (st) return st;
  H->eager_replay = false;
  if ((st = pf_graph_run(H, 1))) return st;  // captures the graphs
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  hipStream_t ls = nullptr;
  if (he == hipSuccess) st = launch_stream(H, &ls);
  if (he == hipSuccess && !st) he = hipEventRecord(e0, ls);
  if (he == hipSuccess && !st) st = pf_graph_run(H, n);
  if (he == hipSuccess && !st) he = hipEventRecord(e1, ls);
  if (he == hipSuccess && !st) he = hipEventSynchronize(e1);
  float ms = 0.f;
  if (he == hipSuccess && !st) he = hipEventElapsedTime(&ms, e0, e1);
  if (!st && he != hipSuccess) st = fail(PF_E_DEVICE, "graph timing failed: %s", hipGetErrorString(he));
  // the events go only after the replays they bracket have finished
  const pf_status st_drain = drain(H);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!st) st = st_drain;
  *ms_out = ms / n;
  return st;
}
}  // namespace

pf_status pf_autotune(pf_handle* H, int32_t steps, int32_t* threads_out, int32_t* groups_out,
                      double* ms_out) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (steps < 1) return fail(PF_E_INVAL, "steps must be >= 1");
  if (H->cfg.layout != PF_LAYOUT_BATCHED) {
    if (threads_out) *threads_out = 0;
    if (groups_out) *groups_out = 0;
    return pf_reset(H, H->iter);
  }
  const int cand_nt[3] = {256, 512, 1024};
  const int cand_g[3] = {1, 2, 4};
  const int nt0 = H->batch_nt, g0 = H->groups;
  double best = 1e300;
  int best_nt = nt0, best_g = g0;
  // Candidates are timed on eager launches, so no graph is captured,
  // instantiated or destroyed per candidate: the captured graphs of the
  // chosen tuning are built once, by the next pf_graph_run.  Each candidate
  // starts from a fresh initialisation, runs one untimed interval, then n
  // timed ones (the groups fork once and join once, as in a graph replay).
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) st = fail(PF_E_DEVICE, "hipEventCreate failed: %s", hipGetErrorString(he));
  const int n = steps < H->cfg.T - 1 ? steps : H->cfg.T - 1;
  const bool tm = H->timing;  // no per-kernel timing events for the candidates
  H->timing = false;
  for (int gi = 0; gi < 3 && !st && he == hipSuccess; ++gi) {
    for (int ci = 0; ci < 3 && !st && he == hipSuccess; ++ci) {
      const int idx = gi * 3 + ci;
      if (ms_out) ms_out[idx] = -1.0;
      if (cand_g[gi] > H->cfg.B) continue;
      if ((st = pf_set_tuning(H, cand_nt[ci], cand_g[gi]))) break;
      if ((st = do_init(H, H->stream))) break;
      if ((st = enqueue_batched(H, H->stream, 1))) break;  // untimed
      if (n < 1) continue;
      if ((he = hipEventRecord(e0, H->stream)) != hipSuccess) break;
      if ((st = enqueue_batched(H, H->stream, n))) break;
      if ((he = hipEventRecord(e1, H->stream)) != hipSuccess) break;
      if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
      float ms = 0.f;
      if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      const double per = ms / n;
      if (ms_out) ms_out[idx] = per;
      if (per < best) {
        best = per;
        best_nt = cand_nt[ci];
        best_g = cand_g[gi];
      }
    }
  }
  H->timing = tm;
  if (!st && he != hipSuccess) st = fail(PF_E_DEVICE, "timing failed: %s", hipGetErrorString(he));
  // every exit waits for the candidates' work before the events go
  const pf_status st_drain = drain(H);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!st) st = st_drain;
  if (st) {
    // keep the error message of the failure; best effort back to the
    // tuning the handle had, re-initialised
    char msg[sizeof g_err];
    std::memcpy(msg, g_err, sizeof msg);
    (void)pf_set_tuning(H, nt0, g0);
    (void)pf_reset(H, H->iter);
    std::memcpy(g_err, msg, sizeof msg);
    return st;
  }
  if ((st = pf_set_tuning(H, best_nt, best_g))) return st;
  if (threads_out) *threads_out = best_nt;
  if (groups_out) *groups_out = best_g;
  // the chosen tuning replayed from its graphs (captured once, here) over
  // the same horizon, against its eager time: pf_graph_run then takes the
  // faster (the eager launches win where the host issues them faster than
  // the device runs them)
  if (n >= 1 && best < 1e300) {
    double graph_ms = 0.0;
    if ((st = time_graph_replay(H, n, &graph_ms))) {
      char msg[sizeof g_err];  // keep the failure's message; re-initialise
      std::memcpy(msg, g_err, sizeof msg);
      (void)pf_reset(H, H->iter);
      std::memcpy(g_err, msg, sizeof msg);
      return st;
    }
    H->eager_replay = best < graph_ms;
  }
  return pf_reset(H, H->iter);
}

pf_status pf_timing_enable(pf_handle* H, int32_t on) {
  pf_status st = check_handle(H);
  if (st) return st;
  if ((st = drain(H))) return st;
  for (auto& ev : H->events) {
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  H->events.clear();
  H->timing = on != 0;
  return PF_OK;
}

pf_status pf_timing_get(pf_handle* H, pf_timing* out) {
  pf_status st = check_handle(H);
  if (st) return st;
  if (!out) return fail(PF_E_INVAL, "out is NULL");
  std::memset(out, 0, sizeof *out);
  HIP_TRY(hipStreamSynchronize(H->stream));
  for (auto& ev : H->events) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
    switch (ev.kind) {
      case 0: out->propagate_ms += ms; out->propagate_launches++; break;
      case 1: out->combine_ms += ms; out->combine_launches++; break;
      case 2: out->scan_ms += ms; out->scan_launches++; break;
      case 3: out->gather_ms += ms; out->gather_launches++; break;
      default: out->batched_ms += ms; out->batched_launches++; break;
    }
  }
  return PF_OK;
}

}  // extern "C"
