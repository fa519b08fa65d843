// Ancestry storage and the single state sample (Alg. 2, last lines):
// kernel arguments and launchers shared by pf_path.hip and the C ABI.
#pragma once
#include "pf_internal.hpp"

namespace pfk {

// A caller-owned history: xh [T+1][d][ld] particles (precision of the
// state), ah [T][ld] ancestors (slot t-1 holds those drawn at time t).
struct HistArgs {
  void* xh;
  int32_t* ah;
  int64_t ld;
  int32_t d, T;
};

hipError_t launch_record_plain(int prec, const void* xa, const void* xb, const int32_t* anc,
                               const HistArgs& H, int64_t off, int64_t N, const FilterState* fs,
                               hipStream_t s);
hipError_t launch_record_batched(int prec, const void* xa, const void* xb, const int32_t* anc,
                                 const HistArgs& H, const BatchArgs& A, int nchunks,
                                 hipStream_t s);
hipError_t launch_backtrace(int prec, const HistArgs& H, int B, const int64_t* offs,
                            const FilterState* fs, KeyArg key, int32_t* idx, double* path,
                            hipStream_t s);

}  // namespace pfk
