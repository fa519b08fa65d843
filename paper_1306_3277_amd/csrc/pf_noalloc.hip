// pf_systematic_noalloc: pf_systematic with its scratch in a static device
// array instead of a caller workspace, for callers that cannot allocate.
// Each GPU the library runs on holds its own copy of the array (sized for
// PF_SYSTEMATIC_NOALLOC_MAX_N weights) until the process ends.  In host code
// the array's name is not a device address: its address on the current
// device comes from hipGetSymbolAddress, taken once per device at the first
// call there and kept; only that address is handed to the kernels.
#include <mutex>

#include "pf_systematic.hpp"

namespace {

constexpr size_t kScratchBytes = pfk::sys_layout(PF_SYSTEMATIC_NOALLOC_MAX_N).total;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];  // scratch's address on each device, once looked up
std::mutex g_mu;

}  // namespace

extern "C" pf_status pf_systematic_noalloc(const double* d_lw, int64_t n, double u,
                                           int32_t* d_anc, double* d_stats, void* hip_stream) {
  pfk::clear_error();
  pf_status st = (pf_status)pfk::systematic_check(d_lw, n, u, d_anc, d_stats);
  if (st) return st;
  if (n > PF_SYSTEMATIC_NOALLOC_MAX_N)
    return pfk::set_error(PF_E_INVAL, "n = %lld exceeds the allocation-free maximum of %d weights",
                (long long)n, PF_SYSTEMATIC_NOALLOC_MAX_N);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return pfk::set_error(PF_E_DEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return pfk::set_error(PF_E_DEVICE, "device %d out of range", dev);
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return pfk::set_error(PF_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                    hipGetErrorString(e));
      g_scratch_ptr[dev] = p;
    }
    base = g_scratch_ptr[dev];
  }
  return (pf_status)pfk::systematic_enqueue(d_lw, n, u, d_anc, d_stats, (char*)base,
                                            (hipStream_t)hip_stream);
}
