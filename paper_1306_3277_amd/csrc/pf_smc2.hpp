// SMC over the parameters (Sec. 3.2.2, Alg. 4) on the batched layout:
// kernel arguments and launchers shared by pf_smc2.hip and the C ABI.
#pragma once
#include "pf_internal.hpp"

namespace pfk {

constexpr int SMC2_NT = 1024;    // lanes of the theta-resampling workgroup
constexpr int SMC2_MAXB = 8192;  // theta-particles (the scan lives in LDS)

// Theta-particle j owns filter slot j of a batched handle.
struct Smc2Args {
  int32_t B, T, n_theta, model;
  double sqrt_h;                 // sqrt(h), rounded on the host
  double step_sd[8], lo[8], hi[8];
  const double* ell_tr;          // the handle's [B][T] likelihood increments
  FilterState* fs;               // the handle's filter states
  double* theta_dev;             // the handle's [B][8] derived parameters
  double* raw;                   // [B][n_theta] theta-particles
  double* prop_raw;              // [B][n_theta] proposals
  double* snap_dev;              // [B][8] snapshot during the theta move
  double* snap_raw;              // [B][n_theta]
  double* snap_ll;               // [B]
  int32_t* snap_st;              // [B]
  int32_t* a;                    // [B] theta-ancestors
  int32_t* inside;               // [B] proposal inside the prior box
  int32_t* accepted;             // [B] move accepted this time
  int32_t* accepts;              // [B] accepted moves so far
  double* evid;                  // running evidence estimate
  int32_t* numeric;              // set if some time had no positive theta-weight
  // attached Kalman filters (windkessel): state (m, V) per slot, or null
  double* mV;                    // [B][2]
  double* snap_mV;               // [B][2]
  double* ell_tr_w;              // the handle's [B][T] increments, written
};

hipError_t launch_theta_resample(const Smc2Args& S, int32_t col, double u, int32_t draw,
                                 int32_t* anc_tr_row, double* ess_out, hipStream_t s);
hipError_t launch_filter_copy(int prec, void* xcur, void* xspare, int32_t* anc, const BatchArgs& A,
                              const Smc2Args& S, const uint32_t* w, hipStream_t s);
hipError_t launch_smc2_propose(const Smc2Args& S, const double* z_row, double* prop_dev,
                               hipStream_t s);
hipError_t launch_smc2_accept(const Smc2Args& S, const double* log_alpha_row,
                              const double* prop_dev, const FilterState* pfs, int32_t* acc_tr_row,
                              hipStream_t s);
hipError_t launch_accept_copy(int prec, void* xcur, int32_t* anc, const void* pxcur,
                              const int32_t* panc, const BatchArgs& A, const Smc2Args& S,
                              hipStream_t s);

}  // namespace pfk
