// The stateless systematic resampler over caller-given log-weights
// (pf_systematic): its scratch layout, shared by the entry point that takes a
// workspace and the one whose scratch is a static device array.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pf.h"
#include "pf_internal.hpp"

namespace pfk {

// the library's error reporting (pf_api.cpp): set_error sets the message
// pf_last_error returns and passes the status through; clear_error empties it
pf_status set_error(pf_status st, const char* fmt, ...);
void clear_error();

// Byte offsets of the scratch regions for n weights, 256-byte aligned:
// block partials (3 doubles per 256 weights), block offsets, per-output
// marks, per-tile owners, per-scan-block candidates, the filter scalars.
struct SysLayout {
  size_t part, boff, marks, owner, jc, fs, total;
};

constexpr size_t sys_align(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr SysLayout sys_layout(int64_t n) {
  const size_t nblk = (size_t)((n + K1_NT - 1) / K1_NT);
  const size_t ntile = (size_t)((n + K4_TILE - 1) / K4_TILE);
  SysLayout L{};
  size_t p = 0;
  L.part = p;
  p = sys_align(p + 24 * nblk);
  L.boff = p;
  p = sys_align(p + 8 * (nblk + 1));
  L.marks = p;
  p = sys_align(p + 4 * (size_t)n);
  L.owner = p;
  p = sys_align(p + 4 * ntile);
  L.jc = p;
  p = sys_align(p + 4 * ntile);
  L.fs = p;
  p = sys_align(p + sizeof(FilterState));
  L.total = p;
  return L;
}

// Validate the arguments (host only, no HIP call); PF_OK or PF_E_INVAL with
// the message set.
int systematic_check(const double* lw, int64_t n, double u, const int32_t* anc,
                     const double* stats);
// Issue the kernels on stream s with the scratch at ws (sys_layout(n).total
// bytes, 256-byte aligned).  Allocates nothing.
int systematic_enqueue(const double* lw, int64_t n, double u, int32_t* anc, double* stats,
                       char* ws, hipStream_t s);

}  // namespace pfk
