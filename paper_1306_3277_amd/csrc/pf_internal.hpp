// Internal types shared by the kernels (pf_kernels.hip, pf_batched.hip) and
// the host runtime (pf_api.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {

// Per-filter scalars kept in device memory.
struct FilterState {
  double loglik;  // running marginal log-likelihood
  double M;       // max log-weight of the last step
  double S;       // sum exp(lw - M) of the last step
  double u;       // uniform of the pending systematic resampling
  double ell;     // last likelihood increment
  double ess;     // last ESS
  int32_t t;      // observation intervals completed
  int32_t status; // 0, or 4 once a step had no positive finite weight (sticky)
  uint32_t iter;  // generator iteration field of the current run
  int32_t pad;    // nonzero if the resampler met an inconsistency (never expected)
  double lprev;   // ln sum exp(carried log-weights) when carry is set
  int32_t carry;  // 1 if the last step kept its weights (ESS above the trigger)
  int32_t tk;     // plain layout: the interval the last propagation processed
  int32_t cn1;    // plain layout: strata owned by the whole filter (count of its last particle)
  int32_t amode;  // plain layout: where the next propagation finds its ancestors
                  // (AMODE_IDENTITY, AMODE_MARKS or AMODE_ARRAY)
};

// Plain layout: the ancestors the next propagation gathers through.  After
// an initialisation or a state set: none (the identity).  After a
// systematic or stratified collective: its marks and tile owners, turned
// into ancestors by the propagation itself (or by the tile-gather kernel
// when the resampled set is asked for).  After the other resamplers, or once
// the marks have been turned into ancestors: the ancestor array.
enum : int32_t { AMODE_IDENTITY = 0, AMODE_MARKS = 1, AMODE_ARRAY = 2 };

// Resampling variants: the ancestors of a resampling time.
enum : int32_t { RS_SYSTEMATIC = 0, RS_STRATIFIED = 1, RS_METROPOLIS = 2, RS_MULTINOMIAL = 3,
                 RS_REJECTION = 4 };

// How a filter resamples: the variant, its Metropolis moves, and the ESS
// trigger (resample when ESS < ess_frac N; +inf: every time).
struct ResampleArgs {
  int32_t scheme;
  int32_t steps;
  double ess_frac;
};

struct KeyArg {
  uint32_t lo, hi;
};

// Plain layout state: particles in tiles of PT = 64 (one wave).  Tile q
// holds components 0..d-1 of particles [64q, 64q + 64) as d rows of 64
// values, so one component of 64 consecutive particles is one contiguous
// segment and each particle's d components lie in one block of 64 d values
// (the gather reads an ancestor's components from one region of memory
// instead of d rows a whole state apart).  g is the particle's index over
// all filters.
constexpr int PT = 64;
__host__ __device__ __forceinline__ int64_t pidx(int64_t g, int i, int d) {
  return ((g >> 6) * (int64_t)d + i) * PT + (g & (PT - 1));
}
// values held by a plain-layout state of n particles (whole tiles)
__host__ __device__ __forceinline__ int64_t plain_state_values(int64_t n, int d) {
  return ((n + PT - 1) / PT) * PT * (int64_t)d;
}

// Arguments of the per-filter (plain layout) kernels.
struct PlainArgs {
  int64_t N;              // particles of this filter
  int64_t ld;             // particles over all filters (N_total)
  int64_t off;            // first particle of this filter
  int64_t boff0;          // first block-partial slot of this filter
  int64_t own0;           // first output-tile owner / scan-block slot of this filter
  int32_t nblk;           // 256-particle blocks of this filter
  int32_t K, T, d, n_obs;
  uint32_t b;
  KeyArg key;
  double h, hh, h6, inv_sd, lw_cst;
  const double* theta;    // device, derived parameters of this filter
  const double* obs;      // device [T][n_obs]
  const int32_t* obs_pos; // device [d]: position in the observation row, or -1
  const int32_t* obs_idx; // device [n_obs]
  const double* q;        // device windkessel flow (or null)
  FilterState* fs;        // this filter's scalars
  double* ell_tr;         // this filter's trace rows [T]
  double* ess_tr;
  ResampleArgs rs;
  double* wcum;           // this filter's cumulative weights [N] (multinomial only)
  int32_t mode;           // K2/K3: 0 step (bookkeeping, uniform drawn); 1 ancestors only
                          // (given uniform); 2 bookkeeping with the given uniform
};

// One filter of a batched collective launch: its index, first particle and
// particle count (fewer than 2^31 particles in all), read with one load.
struct FilterSlot {
  int32_t f, off, n, pad;
};

// Arguments of the batched-layout kernels.
struct BatchArgs {
  int32_t B, K, T, d, n_obs;
  KeyArg key;
  int64_t ld;
  int32_t n_chunks;         // 256-particle propagation chunks over all filters
  double h, hh, h6, inv_sd, lw_cst;
  const double* theta;      // device [B][8] derived parameters
  const double* obs;        // device [T][n_obs]
  const int32_t* obs_pos;   // device [d]
  const double* q;          // device windkessel flow (or null)
  const int64_t* off;       // device [B+1] first particle of each filter
  const FilterSlot* order;  // device [B] filters, largest first within a group
  const int32_t* chunk_f;   // device [n_chunks] filter of each chunk
  const int32_t* chunk_k;   // device [n_chunks] first particle of each chunk
  int32_t chunk0;           // first chunk of the launch (its filter group)
  int32_t order0;           // first filter slot of the launch in `order`
  FilterState* fs;          // device [B]
  double* ell_tr;           // device [B][T]
  double* ess_tr;
  const double* u_override; // device [B] (resample-only mode)
  int32_t mode;             // 0: likelihood + ancestors; 1: ancestors only, given u
  ResampleArgs rs;
  // an attached history (else null): particles [T+1][d][ld] in the state's
  // precision, ancestors [T][ld]; the stepping kernels write slot t
  void* hx;
  int32_t* ha;
};

constexpr int K1_NT = 256;  // particles per propagate / scan block
constexpr int K2_NT = 512;  // combine threads (filters of more than FUSE_NB blocks)
#ifndef PF_FUSE_NB
#define PF_FUSE_NB 1024
#endif
constexpr int FUSE_NB = PF_FUSE_NB;  // up to this many K1 blocks, K3 combines the partials itself
constexpr int K3_NT = 256;  // scan + mark threads
constexpr int K3_PER = 4;   // consecutive particles per scan lane
constexpr int K3_SPAN = K3_NT * K3_PER;  // particles per scan block (4 K1 blocks)
constexpr int K4_NT = 256;  // tile-gather threads
constexpr int K4_PER = 1;   // outputs per tile-gather lane
constexpr int K4_TILE = K4_NT * K4_PER;  // outputs per tile (one owner each)
static_assert(K4_TILE == K1_NT, "a propagation block names the ancestors of one tile");
constexpr int BATCH_NT = 256;
constexpr int BATCH_MAXN = 8192;

// ---- launchers (pf_kernels.hip) ----
hipError_t launch_init(int model, int d, int prec, void* x, const PlainArgs& a, hipStream_t s);
hipError_t launch_reset(FilterState* fs, double* ell, double* ess, int B, int T, uint32_t iter,
                        hipStream_t s);
// Plain-layout state buffers: the interval-t propagated particles live in
// buffer t % 2 (xa holds x(t_0)); the propagation of interval t gathers
// buffer (t - 1) % 2 through the pending ancestors (FilterState::amode).
hipError_t launch_propagate(int model, int d, int prec, void* xa, void* xb, void* lw,
                            double* part, int32_t* marks, const int32_t* owner,
                            const int32_t* jc, int32_t* anc, const PlainArgs& a, hipStream_t s);
hipError_t launch_set_amode(FilterState* fs, int n, int32_t v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_combine(const double* part, double* boff, const PlainArgs& a, hipStream_t s);
hipError_t launch_lw_partials(const double* lw, double* part, const PlainArgs& a, hipStream_t s);
hipError_t launch_tile_anc(int32_t* marks, const int32_t* owner, const int32_t* jc, int32_t* anc,
                           const PlainArgs& a, hipStream_t s);
hipError_t launch_scan_mark(const double* lw, const double* part, const double* boff,
                            int32_t* marks, int32_t* owner, int32_t* jc, const PlainArgs& a,
                            hipStream_t s);
// The resampled set of the interval the filter stands at (t = fs->t):
// buffer t % 2 gathered through the pending ancestors into buffer
// (t + 1) % 2, the ancestors written out (marks cleared).  The pending mode
// becomes AMODE_ARRAY with launch_set_amode afterwards (the kernel's blocks
// all read it).  launch_tile_anc: the ancestors only.
hipError_t launch_tile_gather(int model, int d, int prec, int32_t* marks, const int32_t* owner,
                              const int32_t* jc, void* xa, void* xb, int32_t* anc,
                              const PlainArgs& a, hipStream_t s);
hipError_t launch_set_u(FilterState* fs, double u, hipStream_t s);
// Ancestors of the resamplers without marks; the pending mode becomes
// AMODE_ARRAY.
hipError_t launch_metropolis_anc(const double* lw, int32_t* anc, const PlainArgs& a,
                                 hipStream_t s);
hipError_t launch_rejection_anc(const double* lw, int32_t* anc, const PlainArgs& a,
                                hipStream_t s);
hipError_t launch_multinomial_anc(const double* wcum, const int32_t* jc, int32_t* anc,
                                  const PlainArgs& a, hipStream_t s);
hipError_t launch_simulate(int model, int d, double* out, const PlainArgs& a, double obs_sd,
                           hipStream_t s);
// ---- batched (pf_batched.hip) ----
hipError_t launch_batched_init(int model, int d, int prec, void* x, int32_t* anc,
                               const BatchArgs& a, hipStream_t s);
hipError_t launch_batched_propagate(int model, int d, int prec, void* xa, void* xb, double* lw,
                                    const int32_t* anc, const BatchArgs& a, int nchunks,
                                    hipStream_t s);
// The collective of nfilters filters (the launch's slots in `order`); with
// rejection resampling also the ancestors of the launch's nchunks chunks.
hipError_t launch_batched_resample(int nt, const double* lw, int32_t* anc, const BatchArgs& a,
                                   int nfilters, int max_n, int nchunks, hipStream_t s);
hipError_t launch_batched_gather(int prec, const void* xprop, const int32_t* anc, void* xout,
                                 const BatchArgs& a, hipStream_t s);

}  // namespace pfk
