// The windkessel Kalman filter, batched (Sec. 3.1.1, Alg. 1 in one
// dimension): arguments and launchers shared by pf_kalman.hip and the C ABI.
#pragma once
#include "pf.h"
#include "pf_smc2.hpp"

namespace pfk {

struct KfArgs {
  int32_t B, K, T;
  double R;            // observation variance obs_sd^2
  const double* q;     // device flow series [T*K + 1]
  const double* obs;   // device observations [T]
};

hipError_t launch_kf_run(const KfArgs& A, const double* theta, double* ll, double* ell,
                         hipStream_t s);
hipError_t launch_kf_init(const Smc2Args& S, hipStream_t s);
hipError_t launch_kf_proposal(const KfArgs& A, const Smc2Args& S, const double* prop_dev,
                              double* prop_l, double* prop_mV, int i, hipStream_t s);
hipError_t launch_smc2_accept_kf(const Smc2Args& S, const double* log_alpha_row,
                                 const double* prop_dev, const double* prop_l,
                                 const double* prop_mV, int32_t* acc_tr_row, hipStream_t s);
hipError_t launch_kf_pmmh(const KfArgs& A, const pf_wk_mh& H, double h, int32_t iters,
                          const double* theta0, const double* prop, const double* alpha,
                          double* theta_trace, double* ll_trace, int32_t* accepts, double* ll0,
                          hipStream_t s);
hipError_t launch_kf_advance(const KfArgs& A, const Smc2Args& S, int i, hipStream_t s);

}  // namespace pfk
