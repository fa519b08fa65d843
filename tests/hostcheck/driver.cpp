// Call sequences of the library's tests and benchmark legs, run over the CPU
// stand-in runtime (fake_hip.cpp) and stub kernel launchers, so that the host
// layer's handle logic runs under AddressSanitizer and the stand-in's
// stream-capture checks.  Kernels do nothing here: only the host logic and
// the order of runtime calls are exercised, never a result.
//   driver <scenario>   scenario in autotune, groups, bench, plain, errors,
//                       pmmh, smc2, kalman
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sys/mman.h>
#include <random>
#include <string>
#include <vector>

#include "pf.h"

#define OK(x)                                                                          \
  do {                                                                                 \
    pf_status s_ = (x);                                                                \
    if (s_ != PF_OK) {                                                                 \
      printf("FAIL %s -> %d: %s\n", #x, (int)s_, pf_last_error());                     \
      exit(1);                                                                         \
    }                                                                                  \
  } while (0)
#define EXPECT(x, code)                                                                \
  do {                                                                                 \
    pf_status s_ = (x);                                                                \
    if (s_ != (code)) {                                                                \
      printf("FAIL %s -> %d, expected %d: %s\n", #x, (int)s_, (int)(code), pf_last_error()); \
      exit(1);                                                                         \
    }                                                                                  \
  } while (0)

struct Prob {
  pf_config c{};
  std::vector<int32_t> idx;
  std::vector<double> obs, theta, q;
  std::vector<int64_t> np;
};

// Lorenz '96, d = 8, all observed; particle counts from {256, ..., 8192}
static Prob l96(int B, int T, int prec, int layout, int seed) {
  Prob p;
  std::mt19937_64 r(seed);
  const int64_t counts[6] = {256, 512, 1024, 2048, 4096, 8192};
  for (int b = 0; b < B; ++b) {
    p.np.push_back(counts[r() % 6]);
    p.theta.push_back(6.0 + 4.0 * (double)(r() % 1000) / 1000.0);
    p.theta.push_back(0.05 + 0.25 * (double)(r() % 1000) / 1000.0);
  }
  for (int i = 0; i < 8; ++i) p.idx.push_back(i);
  p.obs.assign((size_t)T * 8, 0.5);
  pf_config& c = p.c;
  c.model = PF_MODEL_L96;
  c.precision = prec;
  c.layout = layout;
  c.d = 8;
  c.K = 8;
  c.T = T;
  c.h = 0.05;
  c.n_obs = 8;
  c.obs_idx = p.idx.data();
  c.obs_sd = 0.5;
  c.obs = p.obs.data();
  c.B = B;
  c.n_theta = 2;
  c.n_particles = p.np.data();
  c.theta = p.theta.data();
  c.seed = 0;
  return p;
}

// windkessel, d = 1, K = 10
static Prob wk(int B, int T, int layout) {
  Prob p;
  const double a = std::exp(-0.01 / 1.5);
  for (int b = 0; b < B; ++b) {
    p.np.push_back(256 + 64 * b);
    const double th[6] = {a, 1.0 - a, 0.03, 0.5, 90.0 + b, 15.0};
    p.theta.insert(p.theta.end(), th, th + 6);
  }
  p.idx.push_back(0);
  p.obs.assign(T, 95.0);
  p.q.assign((size_t)T * 10 + 1, 100.0);
  pf_config& c = p.c;
  c.model = PF_MODEL_WK;
  c.precision = PF_FP64;
  c.layout = layout;
  c.d = 1;
  c.K = 10;
  c.T = T;
  c.h = 0.01;
  c.n_obs = 1;
  c.obs_idx = p.idx.data();
  c.obs_sd = 1.0;
  c.obs = p.obs.data();
  c.q = p.q.data();
  c.B = B;
  c.n_theta = 6;
  c.n_particles = p.np.data();
  c.theta = p.theta.data();
  return p;
}

struct Dev {  // "device" memory of the stand-in runtime: zero pages mapped on
              // demand, so the 8.8 GiB history costs nothing until written
  std::vector<std::pair<void*, size_t>> blocks;
  void* get(size_t n) {
    const size_t len = n > 0 ? n : 1;
    void* m = mmap(nullptr, len, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (m == MAP_FAILED) exit(1);
    blocks.push_back({m, len});
    return m;
  }
  ~Dev() {
    for (auto& b : blocks) munmap(b.first, b.second);
  }
};

static pf_handle* open_(Prob& p, Dev& dev, void* stream) {
  const size_t n = pf_workspace_bytes(&p.c);
  if (!n) {
    printf("FAIL workspace size 0: %s\n", pf_last_error());
    exit(1);
  }
  pf_handle* h = nullptr;
  OK(pf_init(&p.c, dev.get(n), n, stream, &h));
  return h;
}

static void advance(pf_handle* h, int n) {
  for (int i = 0; i < n; ++i) {
    OK(pf_step(h));
    OK(pf_resample(h));
  }
}

static void autotune() {
  Dev dev;
  Prob p = l96(40, 6, PF_FP64, PF_LAYOUT_BATCHED, 9);
  pf_handle* h = open_(p, dev, nullptr);
  advance(h, 6);
  std::vector<double> ell(40 * 6), ess(40 * 6);
  OK(pf_get_trace(h, ell.data(), ess.data()));
  int32_t th = 0, gr = 0;
  double ms[9];
  OK(pf_autotune(h, 3, &th, &gr, ms));
  advance(h, 6);
  // three passes in a row (as the benchmark runs them), each followed by
  // graph replays of the chosen tuning
  for (int pass = 0; pass < 3; ++pass) {
    OK(pf_autotune(h, 5, &th, &gr, ms));
    OK(pf_graph_run(h, 2));
    int32_t t2 = 0, g2 = 0, eg = 0;
    OK(pf_get_tuning(h, &t2, &g2, &eg));
    OK(pf_set_replay(h, 1 - eg));  // the other replay mode
    OK(pf_graph_run(h, 3));
    OK(pf_set_tuning(h, 256, 4));
    OK(pf_reset(h, 0));
    OK(pf_graph_run(h, 5));
  }
  EXPECT(pf_set_replay(h, 3), PF_E_INVAL);
  OK(pf_destroy(h));
}

static void groups() {
  const int G[6] = {1, 3, 3, 2, 4, 1};
  const bool graph[6] = {false, false, true, true, true, true};
  for (int k = 0; k < 6; ++k) {
    Dev dev;
    Prob p = l96(23, 13, PF_FP64, PF_LAYOUT_BATCHED, 12);
    pf_handle* h = open_(p, dev, nullptr);
    OK(pf_set_tuning(h, 512, G[k]));
    if (graph[k]) {
      OK(pf_graph_run(h, 2));
      advance(h, 1);
      OK(pf_graph_run(h, 10));
    } else {
      advance(h, 13);
    }
    std::vector<double> x(8 * (size_t)[&] { int64_t s = 0; for (auto v : p.np) s += v; return s; }());
    OK(pf_get_state(h, x.data()));
    OK(pf_destroy(h));
  }
}

static void bench() {
  hipStream_t s;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) exit(1);
  Dev dev;
  Prob p = l96(512, 200, PF_FP32_MIXED, PF_LAYOUT_BATCHED, 2);
  pf_handle* h = open_(p, dev, s);
  int32_t th = 0, gr = 0;
  double ms[9];
  OK(pf_autotune(h, 16, &th, &gr, ms));
  OK(pf_graph_run(h, 200));
  OK(pf_reset(h, 0));
  OK(pf_graph_run(h, 200));
  OK(pf_set_tuning(h, th, 1));
  OK(pf_reset(h, 0));
  OK(pf_timing_enable(h, 1));
  advance(h, 200);
  pf_timing tm;
  OK(pf_timing_get(h, &tm));
  OK(pf_timing_enable(h, 0));
  OK(pf_set_tuning(h, th, gr));
  OK(pf_reset(h, 0));
  OK(pf_graph_run(h, 200));
  // resampling variants and the ESS trigger on the same handle
  for (int sch = 0; sch < 4; ++sch) {
    OK(pf_set_resampler(h, sch, sch == PF_RESAMPLE_METROPOLIS ? 8 : 0, INFINITY));
    OK(pf_reset(h, 0));
    OK(pf_graph_run(h, 20));
  }
  OK(pf_set_resampler(h, PF_RESAMPLE_SYSTEMATIC, 0, 0.5));
  OK(pf_reset(h, 0));
  OK(pf_graph_run(h, 20));
  OK(pf_set_resampler(h, PF_RESAMPLE_SYSTEMATIC, 0, INFINITY));
  // history on the batched handle
  const size_t hb = pf_history_bytes(&p.c);
  OK(pf_reset(h, 0));
  OK(pf_history_attach(h, dev.get(hb), hb));
  OK(pf_graph_run(h, 30));
  std::vector<double> path((size_t)512 * 31 * 8);
  OK(pf_backtrace(h, path.data(), nullptr));
  OK(pf_history_attach(h, nullptr, 0));
  OK(pf_destroy(h));
  // a second batched handle (FP64) on the same stream, autotuned and replayed
  Prob q = l96(512, 200, PF_FP64, PF_LAYOUT_BATCHED, 2);
  pf_handle* h2 = open_(q, dev, s);
  OK(pf_autotune(h2, 4, &th, &gr, ms));
  OK(pf_reset(h2, 0));
  OK(pf_graph_run(h2, 200));
  OK(pf_destroy(h2));
  if (hipStreamDestroy(s) != hipSuccess) exit(1);
}

static void plain() {
  Dev dev;
  Prob p = l96(3, 16, PF_FP64, PF_LAYOUT_PLAIN, 4);
  int64_t n = 0;
  for (auto v : p.np) n += v;
  pf_handle* h = open_(p, dev, nullptr);
  const size_t hb = pf_history_bytes(&p.c);
  OK(pf_history_attach(h, dev.get(hb), hb));
  advance(h, 2);
  OK(pf_graph_run(h, 3));
  std::vector<double> x(8 * (size_t)n), lw(n), path(3 * 6 * 8);
  std::vector<int32_t> a(n), idx(3 * 6);
  OK(pf_backtrace(h, path.data(), idx.data()));
  OK(pf_get_state(h, x.data()));
  const double ll0[3] = {0.0, -1.0, -2.0};
  EXPECT(pf_restore(h, 1, x.data(), ll0), PF_E_STATE);  // a history is attached
  OK(pf_set_state(h, x.data()));
  OK(pf_step(h));
  OK(pf_get_logweights(h, lw.data()));
  const double u[3] = {0.1, 0.5, 0.9};
  OK(pf_resample_u(h, u));
  OK(pf_get_ancestors(h, a.data()));
  for (int sch = 0; sch < 4; ++sch) {
    OK(pf_set_resampler(h, sch, sch == PF_RESAMPLE_METROPOLIS ? 6 : 0, sch == 1 ? 0.5 : INFINITY));
    advance(h, 1);
    OK(pf_graph_run(h, 1));
  }
  double ll[3], ess[3];
  int32_t t = 0;
  OK(pf_loglik(h, ll, ess, &t));
  OK(pf_history_attach(h, nullptr, 0));
  OK(pf_restore(h, 5, x.data(), ll));
  advance(h, 2);
  OK(pf_graph_run(h, 1));
  OK(pf_timing_enable(h, 1));
  OK(pf_reset(h, 1));
  advance(h, 2);
  pf_timing tm;
  OK(pf_timing_get(h, &tm));
  OK(pf_destroy(h));
}

static void errors() {
  Dev dev;
  Prob p = l96(5, 4, PF_FP32_MIXED, PF_LAYOUT_BATCHED, 6);
  pf_handle* h = open_(p, dev, nullptr);
  int64_t n = 0;
  for (auto v : p.np) n += v;
  std::vector<double> x(8 * (size_t)n, 0.25), ll(5, 0.0);
  EXPECT(pf_resample(h), PF_E_STATE);
  OK(pf_step(h));
  EXPECT(pf_step(h), PF_E_STATE);
  EXPECT(pf_restore(h, 0, x.data(), ll.data()), PF_E_STATE);  // between step and resample
  EXPECT(pf_graph_run(h, 1), PF_E_STATE);
  OK(pf_resample(h));
  EXPECT(pf_graph_run(h, 4), PF_E_STATE);
  EXPECT(pf_graph_run(h, -1), PF_E_INVAL);
  EXPECT(pf_set_tuning(h, 300, 2), PF_E_INVAL);
  EXPECT(pf_set_tuning(h, 512, 9), PF_E_INVAL);
  EXPECT(pf_set_resampler(h, 5, 0, INFINITY), PF_E_INVAL);
  EXPECT(pf_restore(h, 7, x.data(), ll.data()), PF_E_INVAL);
  EXPECT(pf_restore(h, 0, nullptr, ll.data()), PF_E_INVAL);
  ll[3] = NAN;
  EXPECT(pf_restore(h, 0, x.data(), ll.data()), PF_E_INVAL);
  ll[3] = -INFINITY;
  OK(pf_restore(h, 2, x.data(), ll.data()));
  OK(pf_graph_run(h, 1));
  OK(pf_restore(h, 1, x.data(), ll.data()));
  OK(pf_graph_run(h, 3));
  EXPECT(pf_step(h), PF_E_STATE);  // t = T
  OK(pf_set_tuning(h, 1024, 8));   // groups capped at B
  OK(pf_reset(h, 2));
  OK(pf_graph_run(h, 4));
  OK(pf_destroy(h));
}

static void pmmh() {
  Dev dev;
  const int B = 16, iters = 5;
  Prob p = l96(B, 20, PF_FP32_MIXED, PF_LAYOUT_BATCHED, 3);
  for (auto& v : p.np) v = 512;
  pf_handle* h = open_(p, dev, nullptr);
  OK(pf_set_tuning(h, 256, 2));
  std::vector<double> lf0(B, std::log(8.0)), z((size_t)iters * B, 0.3), al((size_t)iters * B, 0.5);
  std::vector<double> lft((size_t)iters * B), llt((size_t)iters * B);
  std::vector<int32_t> acc(B);
  OK(pf_pmmh(h, iters, lf0.data(), z.data(), al.data(), 0.05, 6.0, 10.0, 0.1, lft.data(),
             llt.data(), acc.data()));
  OK(pf_destroy(h));
}

static void smc2_run(Prob& p, Dev& dev, bool kalman, int G) {
  const int B = p.c.B, T = p.c.T, nth = p.c.n_theta;
  pf_handle* h = open_(p, dev, nullptr);
  pf_handle* P = kalman ? nullptr : open_(p, dev, nullptr);
  OK(pf_set_tuning(h, 512, G));
  if (P) OK(pf_set_tuning(P, 512, G));
  const size_t wb = pf_smc2_workspace_bytes(&p.c, T);
  std::vector<double> z((size_t)T * B * nth, 0.5), la((size_t)T * B, -0.7), u(T, 0.37);
  std::vector<uint32_t> w((size_t)T * B, 12345u);
  pf_smc2_in in{};
  in.T_run = T;
  in.theta0 = p.theta.data();
  in.z = z.data();
  in.log_alpha = la.data();
  in.u = u.data();
  in.w_copy = w.data();
  for (int i = 0; i < nth; ++i) {
    in.step_sd[i] = 0.0;
    in.lo[i] = -1e300;
    in.hi[i] = 1e300;
  }
  if (kalman) {
    in.step_sd[4] = 1.0;
    in.lo[4] = 60.0;
    in.hi[4] = 120.0;
    in.filter = PF_FILTER_KALMAN;
  } else {
    in.step_sd[0] = 0.1;
    in.lo[0] = 6.0;
    in.hi[0] = 10.0;
    in.filter = PF_FILTER_PARTICLE;
  }
  std::vector<double> th((size_t)B * nth), logw(B), ll(B), ess(T), ev(1), lwt((size_t)T * B),
      tht((size_t)T * B * nth);
  std::vector<int32_t> acc(B), at((size_t)T * B), act((size_t)T * B);
  pf_smc2_out out{th.data(), logw.data(), ll.data(), acc.data(), ess.data(), ev.data(),
                  at.data(), act.data(), lwt.data(), tht.data()};
  // the kernels do not run, so the evidence may come out as "no positive
  // weight"; both outcomes end the host loop normally
  const pf_status st = pf_smc2(h, P, dev.get(wb), wb, &in, &out);
  if (st != PF_OK && st != PF_E_NUMERIC) {
    printf("FAIL pf_smc2 -> %d: %s\n", (int)st, pf_last_error());
    exit(1);
  }
  if (P) OK(pf_destroy(P));
  OK(pf_destroy(h));
}

static void smc2() {
  Dev dev;
  Prob p = l96(24, 9, PF_FP32_MIXED, PF_LAYOUT_BATCHED, 5);
  smc2_run(p, dev, false, 1);
  Prob q = l96(24, 9, PF_FP32_MIXED, PF_LAYOUT_BATCHED, 5);
  smc2_run(q, dev, false, 3);
}

static void kalman() {
  Dev dev;
  Prob p = wk(6, 8, PF_LAYOUT_PLAIN);
  pf_handle* h = open_(p, dev, nullptr);
  std::vector<double> ll(6), ell(6 * 8);
  OK(pf_kalman(h, ll.data(), ell.data()));
  advance(h, 3);
  OK(pf_destroy(h));
  Prob q = wk(6, 8, PF_LAYOUT_BATCHED);
  smc2_run(q, dev, true, 2);
}

int main(int argc, char** argv) {
  const std::string s = argc > 1 ? argv[1] : "";
  if (s == "autotune") autotune();
  else if (s == "groups") groups();
  else if (s == "bench") bench();
  else if (s == "plain") plain();
  else if (s == "errors") errors();
  else if (s == "pmmh") pmmh();
  else if (s == "smc2") smc2();
  else if (s == "kalman") kalman();
  else {
    printf("unknown scenario '%s'\n", s.c_str());
    return 2;
  }
  printf("scenario %s done\n", s.c_str());
  return 0;
}
