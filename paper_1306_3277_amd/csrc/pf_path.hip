// Ancestry storage and the single state sample of the bootstrap filter
// (Alg. 2, last lines): with a history buffer attached, every time's
// propagated (weighted) particles and the ancestors drawn from their weights
// go to per-time slots; the slot index is the filter's step counter read on
// the device, so captured graphs record too.  The copy kernels here record
// the plain layout's intervals and any layout's initial particles (and
// ancestors redrawn from given uniforms); the batched layout's stepping
// kernels store their intervals' slots themselves.  The backtrace draws the
// final particle from the last weights and follows the ancestry back to t_0,
// one workgroup per filter.
#include "pf_device.hpp"
#include "pf_path.hpp"

namespace pfk {

constexpr uint32_t TAG_PATH = 9;  // generator tag of the final draw

// Plain layout, one filter: slot t = fs->t gets the particles of buffer
// t % 2 (the propagated ones after a step, the initial ones at t = 0; read
// from the state's 64-particle tiles) and, for t >= 1, the ancestors drawn
// at time t (written out before this runs).
// The history itself keeps one row of N_total values per component.
template <typename Real>
__global__ __launch_bounds__(256) void k_record_plain(const Real* __restrict__ xa,
                                                      const Real* __restrict__ xb,
                                                      const int32_t* __restrict__ anc,
                                                      HistArgs H, int64_t off, int64_t N,
                                                      const FilterState* __restrict__ fs) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  const int t = fs->t;
  const Real* __restrict__ x = (t & 1) ? xb : xa;  // the interval-t particles
  Real* xh = (Real*)H.xh + (int64_t)t * H.d * H.ld;
  for (int i = 0; i < H.d; ++i) xh[(int64_t)i * H.ld + off + k] = x[pidx(off + k, i, H.d)];
  if (t >= 1) H.ah[(int64_t)(t - 1) * H.ld + off + k] = anc[off + k];
}

// Batched layout, the chunks of one launch: filter f's slot t = fs[f].t gets
// its propagated particles (buffer t % 2) and, for t >= 1, its ancestors.
template <typename Real>
__global__ __launch_bounds__(BATCH_NT) void k_record_batched(const Real* __restrict__ xa,
                                                             const Real* __restrict__ xb,
                                                             const int32_t* __restrict__ anc,
                                                             HistArgs H, BatchArgs A) {
  const int f = A.chunk_f[A.chunk0 + blockIdx.x];
  const int64_t off = A.off[f];
  const int64_t N = A.off[f + 1] - off;
  const int64_t k = (int64_t)A.chunk_k[A.chunk0 + blockIdx.x] + threadIdx.x;
  if (k >= N) return;
  const int t = A.fs[f].t;
  const Real* x = (t & 1) ? xb : xa;
  Real* xh = (Real*)H.xh + (int64_t)t * H.d * H.ld;
  for (int i = 0; i < H.d; ++i) xh[(int64_t)i * H.ld + off + k] = x[(int64_t)i * H.ld + off + k];
  if (t >= 1) H.ah[(int64_t)(t - 1) * H.ld + off + k] = anc[off + k];
}

// One workgroup per filter b at its time s = fs[b].t.  Lane 0 draws the
// final particle: slot k = floor(w N 2^-32) of the time-s systematic
// ancestors (a uniform slot makes the ancestor one draw from the final
// weights), then walks j <- a^j(t_i) for i = s..1 (the time-(i-1)
// ancestors; identity at i = 1).  Then the lanes gather the path
// [s+1][d] in FP64.
template <typename Real>
__global__ __launch_bounds__(64) void k_backtrace(HistArgs H, const int64_t* __restrict__ offs,
                                                  const FilterState* __restrict__ fs, KeyArg key,
                                                  int32_t* __restrict__ idx,
                                                  double* __restrict__ path) {
  const int b = blockIdx.x;
  const int s = fs[b].t;
  const int64_t off = offs[b], N = offs[b + 1] - off;
  int32_t* ib = idx + (int64_t)b * (H.T + 1);
  if (threadIdx.x == 0) {
    const uint4 w = draw(Key{key.lo, key.hi}, TAG_PATH, 0, fs[b].iter, 0, (uint32_t)s,
                         (uint32_t)b);
    const int64_t k = (int64_t)(((uint64_t)w.x * (uint64_t)N) >> 32);
    // indices are clamped to the filter, so a slot that was never recorded
    // cannot send a read outside it
    int64_t j = s >= 1 ? H.ah[(int64_t)(s - 1) * H.ld + off + k] : k;
    j = j < 0 ? 0 : (j >= N ? N - 1 : j);
    ib[s] = (int32_t)j;
    for (int i = s; i >= 1; --i) {
      if (i >= 2) {
        j = H.ah[(int64_t)(i - 2) * H.ld + off + j];
        j = j < 0 ? 0 : (j >= N ? N - 1 : j);
      }
      ib[i - 1] = (int32_t)j;
    }
  }
  __syncthreads();
  const Real* xh = (const Real*)H.xh;
  double* pb = path + (int64_t)b * (H.T + 1) * H.d;
  for (int e = threadIdx.x; e < (s + 1) * H.d; e += 64) {
    const int i = e / H.d, c = e - i * H.d;
    pb[e] = (double)xh[((int64_t)i * H.d + c) * H.ld + off + ib[i]];
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_record_plain(int prec, const void* xa, const void* xb, const int32_t* anc,
                               const HistArgs& H, int64_t off, int64_t N, const FilterState* fs,
                               hipStream_t s) {
  const unsigned g = (unsigned)((N + 255) / 256);
  if (g == 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(k_record_plain<double>, g, 256, 0, s, (const double*)xa,
                       (const double*)xb, anc, H, off, N, fs);
  else
    hipLaunchKernelGGL(k_record_plain<float>, g, 256, 0, s, (const float*)xa, (const float*)xb,
                       anc, H, off, N, fs);
  return hipGetLastError();
}

hipError_t launch_record_batched(int prec, const void* xa, const void* xb, const int32_t* anc,
                                 const HistArgs& H, const BatchArgs& A, int nchunks,
                                 hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  const unsigned g = (unsigned)nchunks;
  if (prec == 0)
    hipLaunchKernelGGL(k_record_batched<double>, g, BATCH_NT, 0, s, (const double*)xa,
                       (const double*)xb, anc, H, A);
  else
    hipLaunchKernelGGL(k_record_batched<float>, g, BATCH_NT, 0, s, (const float*)xa,
                       (const float*)xb, anc, H, A);
  return hipGetLastError();
}

hipError_t launch_backtrace(int prec, const HistArgs& H, int B, const int64_t* offs,
                            const FilterState* fs, KeyArg key, int32_t* idx, double* path,
                            hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (prec == 0)
    hipLaunchKernelGGL(k_backtrace<double>, B, 64, 0, s, H, offs, fs, key, idx, path);
  else
    hipLaunchKernelGGL(k_backtrace<float>, B, 64, 0, s, H, offs, fs, key, idx, path);
  return hipGetLastError();
}

}  // namespace pfk
