// Device-side building blocks of the gfx950 particle filter: the
// counter-based generator, the normal transforms, the two models'
// transitions and observation densities, and wave/block reductions.
//
// Compiled with -ffp-contract=off: every FP64 expression is evaluated as
// written, which makes the FP64 path reproduce the generator's normals and
// the model arithmetic bit for bit.  The FP32 path asks for fused
// multiply-adds explicitly (fmaf).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {

enum : uint32_t { TAG_INIT = 1, TAG_NOISE = 2, TAG_RESAMPLE = 3, TAG_DATA = 4, TAG_OBS = 8,
                  TAG_MULTI = 10, TAG_REJECT = 11 };
constexpr int WAVE = 64;

// ---------------------------------------------------------------- generator
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplies mixed with the round key; the key schedule is uniform across a
// wave, so it lives in scalar registers.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    // From the third round on every operand varies per lane, and the
    // three-input exclusive or takes one instruction (truth table 0x96); in
    // the first two rounds some words are uniform across the wave and the
    // compiler keeps that part on the scalar unit.
    uint32_t n0, n2;
    if (r < 2) {
      n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
      n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    } else {
      n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
      n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    }
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  return make_uint4(c0, c1, c2, c3);
}

// Counter word 2: tag (4 bits) | component block (8 bits) | iteration (20 bits).
__device__ __forceinline__ uint32_t ctr_word2(uint32_t tag, uint32_t blk, uint32_t iter) {
  return (tag << 28) | (blk << 20) | iter;
}

struct Key {
  uint32_t lo, hi;
};

__device__ __forceinline__ uint4 draw(Key key, uint32_t tag, uint32_t blk, uint32_t iter,
                                      uint32_t j, uint32_t n, uint32_t b) {
  return philox(j, n, ctr_word2(tag, blk, iter), b, key.lo, key.hi);
}

// ---------------------------------------------------------------- FP64 normals
// u = (w + 1/2) 2^-32; ln from the atanh series on [sqrt(1/2), sqrt(2));
// sin/cos of 2 pi u by quarter-turn reduction and Taylor series; radius
// sqrt(-2 ln u_a).  IEEE +, -, *, / and sqrt only, so the host and the device
// produce the same bits.
__device__ __forceinline__ double u01_f64(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

__device__ __forceinline__ double ln_f64(double x) {
  uint64_t bits = (uint64_t)__double_as_longlong(x);
  int e = (int)((bits >> 52) & 0x7ff) - 1022;
  double f = __longlong_as_double((long long)((bits & 0x000fffffffffffffULL) | 0x3fe0000000000000ULL));
  if (f < 0x1.6a09e667f3bcdp-1) {
    f = f + f;
    e = e - 1;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double s2 = s * s;
  double p = 1.0 / 21.0;
  p = p * s2 + 1.0 / 19.0;
  p = p * s2 + 1.0 / 17.0;
  p = p * s2 + 1.0 / 15.0;
  p = p * s2 + 1.0 / 13.0;
  p = p * s2 + 1.0 / 11.0;
  p = p * s2 + 1.0 / 9.0;
  p = p * s2 + 1.0 / 7.0;
  p = p * s2 + 1.0 / 5.0;
  p = p * s2 + 1.0 / 3.0;
  p = p * s2 + 1.0;
  const double lnf = (2.0 * s) * p;
  const double de = (double)e;
  return de * 0x1.62e42feep-1 + (de * 0x1.a39ef35793c76p-33 + lnf);
}

__device__ __forceinline__ void sincos2pi_f64(double u, double& s_out, double& c_out) {
  const double v = 4.0 * u;
  const double kf = __builtin_floor(v + 0.5);
  const double f = v - kf;
  const int k = ((int)kf) & 3;
  const double p = f * 0x1.921fb54442d18p0;
  const double p2 = p * p;
  double sp = -1.0 / 121645100408832000.0;
  sp = sp * p2 + 1.0 / 355687428096000.0;
  sp = sp * p2 - 1.0 / 1307674368000.0;
  sp = sp * p2 + 1.0 / 6227020800.0;
  sp = sp * p2 - 1.0 / 39916800.0;
  sp = sp * p2 + 1.0 / 362880.0;
  sp = sp * p2 - 1.0 / 5040.0;
  sp = sp * p2 + 1.0 / 120.0;
  sp = sp * p2 - 1.0 / 6.0;
  sp = sp * p2 + 1.0;
  sp = sp * p;
  double cp = -1.0 / 6402373705728000.0;
  cp = cp * p2 + 1.0 / 20922789888000.0;
  cp = cp * p2 - 1.0 / 87178291200.0;
  cp = cp * p2 + 1.0 / 479001600.0;
  cp = cp * p2 - 1.0 / 3628800.0;
  cp = cp * p2 + 1.0 / 40320.0;
  cp = cp * p2 - 1.0 / 720.0;
  cp = cp * p2 + 1.0 / 24.0;
  cp = cp * p2 - 1.0 / 2.0;
  cp = cp * p2 + 1.0;
  const bool odd = (k & 1) != 0;
  const double s0 = odd ? cp : sp;
  const double c0 = odd ? -sp : cp;
  const bool neg = (k & 2) != 0;
  s_out = neg ? -s0 : s0;
  c_out = neg ? -c0 : c0;
}

__device__ __forceinline__ void bm_pair_f64(uint32_t wa, uint32_t wb, double& z0, double& z1) {
  const double r = __builtin_sqrt(-2.0 * ln_f64(u01_f64(wa)));
  double s, c;
  sincos2pi_f64(u01_f64(wb), s, c);
  z0 = r * c;
  z1 = r * s;
}

__device__ __forceinline__ void normals4_f64(uint4 w, double z[4]) {
  bm_pair_f64(w.x, w.y, z[0], z[1]);
  bm_pair_f64(w.z, w.w, z[2], z[3]);
}

// ---------------------------------------------------------------- FP32 normals
// Uniforms from the whole 32-bit word: float(w) 2^-32 + 2^-33 keeps 24
// significant bits at every magnitude, so the small u that make the tails
// of the normal keep their relative precision (a fixed 23-bit grid would
// lose it there).  u lies in (0, 1]; u = 1 gives a zero radius.  Hardware
// log2 / sqrt / sin / cos; sin and cos take their argument in revolutions,
// so cos(2 pi u) is one instruction.
__device__ __forceinline__ float u01_f32(uint32_t w) {
  return fmaf((float)w, 0x1p-32f, 0x1p-33f);
}

__device__ __forceinline__ void bm_pair_f32(uint32_t wa, uint32_t wb, float& z0, float& z1) {
  const float ua = u01_f32(wa);
  const float ub = u01_f32(wb);
  // -2 ln u = -2 ln(2) log2(u)
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
  z0 = r * __builtin_amdgcn_cosf(ub);
  z1 = r * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ void normals4_f32(uint4 w, float z[4]) {
  bm_pair_f32(w.x, w.y, z[0], z[1]);
  bm_pair_f32(w.z, w.w, z[2], z[3]);
}

// ---------------------------------------------------------------- models
// Per-filter constants, derived on the host in FP64.
struct ModelConsts {
  double h, hh, h6;        // substep, h/2, h/6 (Lorenz '96 RK4)
  double inv_sd, lw_cst;   // 1/obs_sd and -n_obs (ln obs_sd + ln(2 pi)/2)
};

// Windkessel substep n (t_{n-1} -> t_n), exact two-element step with the
// flow held at q_{n-1}, plus pressure noise:  p <- (a p + c q_{n-1}) + sp z.
__device__ __forceinline__ double wk_substep_f64(double p, const double* th, double q_prev,
                                                 double z) {
  return (th[0] * p + th[1] * q_prev) + th[3] * z;
}

// FP32 form: the increment (a - 1) p + c q + sp z is formed first and added
// to the pressure (|p| ~ 90) once (the accurate form adds it to an FP64
// pressure).
__device__ __forceinline__ float wk_increment_f32(float p, float am1, float c, float sp,
                                                  float q_prev, float z) {
  return fmaf(sp, z, fmaf(am1, p, c * q_prev));
}
__device__ __forceinline__ float wk_substep_f32(float p, float am1, float c, float sp,
                                                float q_prev, float z) {
  return p + wk_increment_f32(p, am1, c, sp, q_prev, z);
}

// Lorenz '96 drift, written as the oracle writes it:
//   f_i = ((x_{i+1} - x_{i-2}) x_{i-1} - x_i) + F.
template <int D>
__device__ __forceinline__ void l96_drift_f64(const double (&x)[D], double F, double (&k)[D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
    k[i] = ((x[(i + 1) % D] - x[(i + D - 2) % D]) * x[(i + D - 1) % D] - x[i]) + F;
}

// One RK4 substep of the drift plus the Wiener increment, FP64, with the
// same expression tree as the oracle:
//   x <- (x + h6 ((k1 + k4) + 2 (k2 + k3))) + sq z.
template <int D>
__device__ __forceinline__ void l96_substep_f64(double (&x)[D], double F, double sq,
                                                const ModelConsts& mc, Key key, uint32_t tag,
                                                uint32_t iter, uint32_t j, uint32_t n,
                                                uint32_t b) {
  double k[D], xt[D], s14[D], s23[D];
  l96_drift_f64<D>(x, F, k);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    s14[i] = k[i];
    xt[i] = x[i] + mc.hh * k[i];
  }
  l96_drift_f64<D>(xt, F, k);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    s23[i] = k[i];
    xt[i] = x[i] + mc.hh * k[i];
  }
  l96_drift_f64<D>(xt, F, k);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    s23[i] = s23[i] + k[i];
    xt[i] = x[i] + mc.h * k[i];
  }
  l96_drift_f64<D>(xt, F, k);
#pragma unroll
  for (int i = 0; i < D; ++i) s14[i] = s14[i] + k[i];
#pragma unroll
  for (int blk = 0; blk < D / 4; ++blk) {
    double z[4];
    normals4_f64(draw(key, tag, blk, iter, j, n, b), z);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = 4 * blk + m;
      const double xn = x[i] + mc.h6 * (s14[i] + 2.0 * s23[i]);
      x[i] = xn + sq * z[m];
    }
  }
}

// FP32 Lorenz '96 substep.  With g_i = (x_{i+1} - x_{i-2}) x_{i-1} - x_i the
// drift is g_i + F, and since the RK4 weights sum to h the increment is
//   F h + (h/6) g1 + (h/3) g2 + (h/3) g3 + (h/6) g4 + sq z,
// accumulated from F h with fused multiply-adds and added to the state once
// (|x| ~ 10 with ulp ~ 1e-6: the state is rounded once per substep).  Stage
// inputs are (x + c F) + c g with x + c F formed once per substep for c = h/2
// and once for c = h and kept (4D live registers) when D <= 16; for larger D
// they are x + c (g + F), so only 3D registers stay live and occupancy holds.  The
// Wiener increment sq z is formed as sqrt(-2 ln(2) sq^2 log2 u_a)
// cos(2 pi u_b): the noise scale rides in the radius.
struct L96F32 {
  float F, Fh;      // F and F h
  float hF, hF2;    // (h/2) F and h F
  float h, hh, h3, h6;
  float nc2;        // -2 ln(2) sq^2
};

__device__ __forceinline__ L96F32 l96_f32_consts(double F, double sq, double h) {
  L96F32 c;
  c.F = (float)F;
  c.Fh = (float)(F * h);
  c.hF = (float)(0.5 * h * F);
  c.hF2 = (float)(h * F);
  c.h = (float)h;
  c.hh = (float)(0.5 * h);
  c.h3 = (float)(h / 3.0);
  c.h6 = (float)(h / 6.0);
  c.nc2 = (float)(-1.3862943611198906 * sq * sq);
  return c;
}

// radius sqrt(nc2 log2 u_a) and the angle 2 pi u_b of one Box-Muller pair
__device__ __forceinline__ void noise_pair_f32(uint32_t wa, uint32_t wb, float nc2, float& r,
                                               float& cs, float& sn) {
  r = __builtin_amdgcn_sqrtf(nc2 * __builtin_amdgcn_logf(u01_f32(wa)));
  const float ub = u01_f32(wb);
  cs = __builtin_amdgcn_cosf(ub);
  sn = __builtin_amdgcn_sinf(ub);
}

constexpr bool l96_keep_xc(int D) { return D <= 16; }

// one RK4 stage; xc holds x + c_xt F when kept, else x
template <int D>
__device__ __forceinline__ void l96_stage_f32(float (&xt)[D], const float (&xc)[D],
                                              float (&acc)[D], float Fh, float F, float c_acc,
                                              float c_xt, bool first, bool last) {
  const float old0 = xt[0];
  float pm2 = xt[D - 2], pm1 = xt[D - 1];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const float xi = xt[i];
    const float xp1 = (i == D - 1) ? old0 : xt[i + 1];
    const float g = fmaf(xp1 - pm2, pm1, -xi);
    pm2 = pm1;
    pm1 = xi;
    acc[i] = fmaf(c_acc, g, first ? Fh : acc[i]);
    if (!last) xt[i] = l96_keep_xc(D) ? fmaf(c_xt, g, xc[i]) : fmaf(c_xt, g + F, xc[i]);
  }
}

template <int D>
__device__ __forceinline__ void l96_substep_f32(float (&x)[D], const L96F32& c, Key key,
                                                uint32_t tag, uint32_t iter, uint32_t j,
                                                uint32_t n, uint32_t b) {
  float acc[D], xt[D];
#pragma unroll
  for (int i = 0; i < D; ++i) xt[i] = x[i];
  if constexpr (l96_keep_xc(D)) {
    float xc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xc[i] = x[i] + c.hF;
    l96_stage_f32<D>(xt, xc, acc, c.Fh, 0.0f, c.h6, c.hh, true, false);
    l96_stage_f32<D>(xt, xc, acc, c.Fh, 0.0f, c.h3, c.hh, false, false);
#pragma unroll
    for (int i = 0; i < D; ++i) xc[i] = x[i] + c.hF2;
    l96_stage_f32<D>(xt, xc, acc, c.Fh, 0.0f, c.h3, c.h, false, false);
    l96_stage_f32<D>(xt, xc, acc, c.Fh, 0.0f, c.h6, 0.0f, false, true);
  } else {
    l96_stage_f32<D>(xt, x, acc, c.Fh, c.F, c.h6, c.hh, true, false);
    l96_stage_f32<D>(xt, x, acc, c.Fh, c.F, c.h3, c.hh, false, false);
    l96_stage_f32<D>(xt, x, acc, c.Fh, c.F, c.h3, c.h, false, false);
    l96_stage_f32<D>(xt, x, acc, c.Fh, c.F, c.h6, 0.0f, false, true);
  }
#pragma unroll
  for (int blk = 0; blk < D / 4; ++blk) {
    const uint4 w = draw(key, tag, blk, iter, j, n, b);
    float r0, c0, s0, r1, c1, s1;
    noise_pair_f32(w.x, w.y, c.nc2, r0, c0, s0);
    noise_pair_f32(w.z, w.w, c.nc2, r1, c1, s1);
    const int i = 4 * blk;
    x[i] = x[i] + fmaf(r0, c0, acc[i]);
    x[i + 1] = x[i + 1] + fmaf(r0, s0, acc[i + 1]);
    x[i + 2] = x[i + 2] + fmaf(r1, c1, acc[i + 2]);
    x[i + 3] = x[i + 3] + fmaf(r1, s1, acc[i + 3]);
  }
}

// ---------------------------------------------------------------- FP32 slopes, FP64 accumulation
// The accurate FP32 form.  The slopes are evaluated in FP32 on FP32 stage
// inputs, as in the FP32 form, but within an interval the state and each
// substep's increment are carried in FP64: the stage bases (float)(x + c F)
// are rounded once from the FP64 state, the slopes are summed in FP32 pairs
// s14 = g1 + g4 and s23 = g2 + g3 (their rounding weighs h/6 in the
// increment), and F h + (h/6)(s14 + 2 s23) + sq z is formed and added in
// FP64.  The FP32 form's rounding of the state after every substep and of
// its increment are what move its log-weights by up to about 1e-6 of their
// size; here the state is rounded once, when it is stored, and the
// log-weight is taken from the unrounded state.
struct L96F32A {
  float hh, h, nc2;
  double Fh, hF, hF2, h6;
};

__device__ __forceinline__ L96F32A l96_f32a_consts(double F, double sq, double h) {
  L96F32A c;
  c.hh = (float)(0.5 * h);
  c.h = (float)h;
  c.nc2 = (float)(-1.3862943611198906 * sq * sq);
  c.Fh = F * h;
  c.hF = 0.5 * h * F;
  c.hF2 = h * F;
  c.h6 = h / 6.0;
  return c;
}

// one stage: slopes g of the FP32 stage inputs xt, summed into s (or
// starting it), and the next stage inputs xc + c_xt g
template <int D>
__device__ __forceinline__ void l96_stage_acc(float (&xt)[D], const float (&xc)[D], float (&s)[D],
                                              float c_xt, bool start, bool last) {
  const float old0 = xt[0];
  float pm2 = xt[D - 2], pm1 = xt[D - 1];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const float xi = xt[i];
    const float xp1 = (i == D - 1) ? old0 : xt[i + 1];
    const float g = fmaf(xp1 - pm2, pm1, -xi);
    pm2 = pm1;
    pm1 = xi;
    s[i] = start ? g : s[i] + g;
    if (!last) xt[i] = fmaf(c_xt, g, xc[i]);
  }
}

template <int D>
__device__ __forceinline__ void l96_substep_f32acc(double (&x)[D], const L96F32A& c, Key key,
                                                   uint32_t tag, uint32_t iter, uint32_t j,
                                                   uint32_t n, uint32_t b) {
  float xt[D], xc[D], s14[D], s23[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    xt[i] = (float)x[i];
    xc[i] = (float)(x[i] + c.hF);
  }
  l96_stage_acc<D>(xt, xc, s14, c.hh, true, false);
  l96_stage_acc<D>(xt, xc, s23, c.hh, true, false);
#pragma unroll
  for (int i = 0; i < D; ++i) xc[i] = (float)(x[i] + c.hF2);
  l96_stage_acc<D>(xt, xc, s23, c.h, false, false);
  l96_stage_acc<D>(xt, xc, s14, 0.0f, false, true);
#pragma unroll
  for (int blk = 0; blk < D / 4; ++blk) {
    const uint4 w = draw(key, tag, blk, iter, j, n, b);
    float r0, c0, s0, r1, c1, s1;
    noise_pair_f32(w.x, w.y, c.nc2, r0, c0, s0);
    noise_pair_f32(w.z, w.w, c.nc2, r1, c1, s1);
    const float nz[4] = {r0 * c0, r0 * s0, r1 * c1, r1 * s1};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = 4 * blk + m;
      const double drift =
          __builtin_fma(c.h6, __builtin_fma(2.0, (double)s23[i], (double)s14[i]), c.Fh);
      x[i] = x[i] + (drift + (double)nz[m]);
    }
  }
}

// The same for the paper's form (noise inside the stages): the forcing of
// component i over the substep is F + nz_i / h, so the stage bases are
// (float)(x + (c F + (c/h) nz_i)) and the increment starts from F h + nz_i.
template <int D>
__device__ __forceinline__ void l96_substep_stage_f32acc(double (&x)[D], const L96F32A& c,
                                                         Key key, uint32_t tag, uint32_t iter,
                                                         uint32_t j, uint32_t n, uint32_t b) {
  float nz[D];
#pragma unroll
  for (int blk = 0; blk < D / 4; ++blk) {
    const uint4 w = draw(key, tag, blk, iter, j, n, b);
    float r0, c0, s0, r1, c1, s1;
    noise_pair_f32(w.x, w.y, c.nc2, r0, c0, s0);
    noise_pair_f32(w.z, w.w, c.nc2, r1, c1, s1);
    nz[4 * blk] = r0 * c0;
    nz[4 * blk + 1] = r0 * s0;
    nz[4 * blk + 2] = r1 * c1;
    nz[4 * blk + 3] = r1 * s1;
  }
  float xt[D], xc[D], s14[D], s23[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    xt[i] = (float)x[i];
    xc[i] = (float)(x[i] + (c.hF + 0.5 * (double)nz[i]));
  }
  l96_stage_acc<D>(xt, xc, s14, c.hh, true, false);
  l96_stage_acc<D>(xt, xc, s23, c.hh, true, false);
#pragma unroll
  for (int i = 0; i < D; ++i) xc[i] = (float)(x[i] + (c.hF2 + (double)nz[i]));
  l96_stage_acc<D>(xt, xc, s23, c.h, false, false);
  l96_stage_acc<D>(xt, xc, s14, 0.0f, false, true);
#pragma unroll
  for (int i = 0; i < D; ++i)
    x[i] = x[i] + __builtin_fma(c.h6, __builtin_fma(2.0, (double)s23[i], (double)s14[i]),
                                c.Fh + (double)nz[i]);
}

// ---------------------------------------------------------------- Lorenz '96, noise in the stages
// The paper's form of the stochastic model: the SDE read as an ODE whose
// forcing on component i is F + sigma dW_i / h over the step (dW_i = sqrt(h)
// z_i held for the step), integrated by the same classic RK4.  With
// sq = sigma sqrt(h) the forcing is F_i = F + (sq z_i) / h and nothing is
// added after the step.  FP64, the oracle's expression tree.
template <int D>
__device__ __forceinline__ void l96_drift_vec_f64(const double (&x)[D], const double (&F)[D],
                                                  double (&k)[D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
    k[i] = ((x[(i + 1) % D] - x[(i + D - 2) % D]) * x[(i + D - 1) % D] - x[i]) + F[i];
}

template <int D>
__device__ __forceinline__ void l96_substep_stage_f64(double (&x)[D], double F, double sq,
                                                      const ModelConsts& mc, Key key,
                                                      uint32_t tag, uint32_t iter, uint32_t j,
                                                      uint32_t n, uint32_t b) {
  double Fi[D];
#pragma unroll
  for (int blk = 0; blk < D / 4; ++blk) {
    double z[4];
    normals4_f64(draw(key, tag, blk, iter, j, n, b), z);
#pragma unroll
    for (int m = 0; m < 4; ++m) Fi[4 * blk + m] = F + (sq * z[m]) / mc.h;
  }
  double k[D], xt[D], s14[D], s23[D];
  l96_drift_vec_f64<D>(x, Fi, k);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    s14[i] = k[i];
    xt[i] = x[i] + mc.hh * k[i];
  }
  l96_drift_vec_f64<D>(xt, Fi, k);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    s23[i] = k[i];
    xt[i] = x[i] + mc.hh * k[i];
  }
  l96_drift_vec_f64<D>(xt, Fi, k);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    s23[i] = s23[i] + k[i];
    xt[i] = x[i] + mc.h * k[i];
  }
  l96_drift_vec_f64<D>(xt, Fi, k);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    s14[i] = s14[i] + k[i];
    x[i] = x[i] + mc.h6 * (s14[i] + 2.0 * s23[i]);
  }
}

// FP32 form of the same step: the noise term nz_i = sq z_i is drawn first;
// h F_i = F h + nz_i starts the increment, and the stage inputs are
// (x + c F_i) + c g with c F_i = c F + (c/h) nz_i formed once per substep
// for c = h/2 and c = h.
template <int D>
__device__ __forceinline__ void l96_substep_stage_f32(float (&x)[D], const L96F32& c, Key key,
                                                      uint32_t tag, uint32_t iter, uint32_t j,
                                                      uint32_t n, uint32_t b) {
  float nz[D];
#pragma unroll
  for (int blk = 0; blk < D / 4; ++blk) {
    const uint4 w = draw(key, tag, blk, iter, j, n, b);
    float r0, c0, s0, r1, c1, s1;
    noise_pair_f32(w.x, w.y, c.nc2, r0, c0, s0);
    noise_pair_f32(w.z, w.w, c.nc2, r1, c1, s1);
    nz[4 * blk] = r0 * c0;
    nz[4 * blk + 1] = r0 * s0;
    nz[4 * blk + 2] = r1 * c1;
    nz[4 * blk + 3] = r1 * s1;
  }
  float acc[D], xt[D], xc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    xt[i] = x[i];
    acc[i] = c.Fh + nz[i];
    xc[i] = x[i] + fmaf(0.5f, nz[i], c.hF);
  }
  auto stage = [&](float c_acc, float c_xt, bool last) {
    const float old0 = xt[0];
    float pm2 = xt[D - 2], pm1 = xt[D - 1];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const float xi = xt[i];
      const float xp1 = (i == D - 1) ? old0 : xt[i + 1];
      const float g = fmaf(xp1 - pm2, pm1, -xi);
      pm2 = pm1;
      pm1 = xi;
      acc[i] = fmaf(c_acc, g, acc[i]);
      if (!last) xt[i] = fmaf(c_xt, g, xc[i]);
    }
  };
  stage(c.h6, c.hh, false);
  stage(c.h3, c.hh, false);
#pragma unroll
  for (int i = 0; i < D; ++i) xc[i] = x[i] + (c.hF2 + nz[i]);
  stage(c.h3, c.h, false);
  stage(c.h6, 0.0f, true);
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = x[i] + acc[i];
}

// e^x for x <= 0, x = -inf included (weights exp(lw - max lw)).  Reduction
// x = n ln2 + r with |r| <= ln2/2 (ln2 split in two parts, so r is exact to
// about 2^-60), e^r by its Taylor polynomial to degree 13 (truncation below
// 2^-52 relative) in Horner form, and the scale 2^n.  Underflows to 0 below
// -745.2; a NaN argument gives 0.  Branch-free (the out-of-range case is a
// select), so calls on independent arguments interleave.
__device__ __forceinline__ double exp_nonpos(double xin) {
  const bool ok = xin >= -745.2;  // false for -inf and NaN
  const double x = ok ? xin : 0.0;
  const double n = __builtin_rint(x * 0x1.71547652b82fep+0);
  double r = __builtin_fma(-n, 0x1.62e42fefa39efp-1, x);
  r = __builtin_fma(-n, 0x1.abc9e3b39803fp-56, r);
  double p = 0x1.6124613a86d09p-33;           // 1/13!
  p = __builtin_fma(p, r, 0x1.1eed8eff8d898p-29);  // 1/12!
  p = __builtin_fma(p, r, 0x1.ae64567f544e4p-26);  // 1/11!
  p = __builtin_fma(p, r, 0x1.27e4fb7789f5cp-22);  // 1/10!
  p = __builtin_fma(p, r, 0x1.71de3a556c734p-19);  // 1/9!
  p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-16);  // 1/8!
  p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-13);  // 1/7!
  p = __builtin_fma(p, r, 0x1.6c16c16c16c17p-10);  // 1/6!
  p = __builtin_fma(p, r, 0x1.1111111111111p-7);   // 1/5!
  p = __builtin_fma(p, r, 0x1.5555555555555p-5);   // 1/4!
  p = __builtin_fma(p, r, 0x1.5555555555555p-3);   // 1/3!
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  const double v = __builtin_ldexp(p, (int)n);
  return ok ? v : 0.0;
}

// ---------------------------------------------------------------- reductions
// Wave-wide scans and reductions by DPP lane moves: shifts inside 16-lane
// rows (1, 2, 4, 8), then two row broadcasts (lane 15 of a row into the next
// row, then lane 31 into rows 2 and 3).  They stay in the vector unit,
// where a shuffle goes through an LDS permute.  Every lane of the wave must
// be active (call them outside lane-dependent branches and selects, or a
// lane reads a switched-off neighbour); lanes a move does not reach take
// `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_move_i(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v, double old) {
  const int lo = dpp_move_i<CTRL, ROWS>(__double2loint(v), __double2loint(old));
  const int hi = dpp_move_i<CTRL, ROWS>(__double2hiint(v), __double2hiint(old));
  return __hiloint2double(hi, lo);
}
// inclusive sum over lanes 0..lane
__device__ __forceinline__ double wave_incl_scan(double v, int = 0) {
  v += dpp_move<0x111, 0xf>(v, 0.0);  // row_shr 1
  v += dpp_move<0x112, 0xf>(v, 0.0);  // row_shr 2
  v += dpp_move<0x114, 0xf>(v, 0.0);  // row_shr 4
  v += dpp_move<0x118, 0xf>(v, 0.0);  // row_shr 8
  v += dpp_move<0x142, 0xa>(v, 0.0);  // row_bcast 15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v, 0.0);  // row_bcast 31 into rows 2 and 3
  return v;
}
// inclusive running maximum over lanes 0..lane (exact: max does not round)
__device__ __forceinline__ double wave_incl_max_scan(double v, int = 0) {
  v = fmax(v, dpp_move<0x111, 0xf>(v, -INFINITY));
  v = fmax(v, dpp_move<0x112, 0xf>(v, -INFINITY));
  v = fmax(v, dpp_move<0x114, 0xf>(v, -INFINITY));
  v = fmax(v, dpp_move<0x118, 0xf>(v, -INFINITY));
  v = fmax(v, dpp_move<0x142, 0xa>(v, -INFINITY));
  v = fmax(v, dpp_move<0x143, 0xc>(v, -INFINITY));
  return v;
}
__device__ __forceinline__ int wave_incl_max_scan_rows(int v) {
  constexpr int lo = -2147483647 - 1;
  v = max(v, dpp_move_i<0x111, 0xf>(v, lo));
  v = max(v, dpp_move_i<0x112, 0xf>(v, lo));
  v = max(v, dpp_move_i<0x114, 0xf>(v, lo));
  v = max(v, dpp_move_i<0x118, 0xf>(v, lo));
  v = max(v, dpp_move_i<0x142, 0xa>(v, lo));
  v = max(v, dpp_move_i<0x143, 0xc>(v, lo));
  return v;
}
__device__ __forceinline__ int wave_incl_max_scan_i(int v, int = 0) {
  return wave_incl_max_scan_rows(v);
}
// the value of lane 63, in every lane
__device__ __forceinline__ double last_lane(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), WAVE - 1);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), WAVE - 1);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_max(double v) { return last_lane(wave_incl_max_scan(v)); }
__device__ __forceinline__ double wave_sum(double v) { return last_lane(wave_incl_scan(v)); }
__device__ __forceinline__ int wave_max_i(int v) {
  return __builtin_amdgcn_readlane(wave_incl_max_scan_rows(v), WAVE - 1);
}
// lane - 1's value (wave_shr 1); lane 0 takes `old`
__device__ __forceinline__ double wave_prev(double v, double old) {
  return dpp_move<0x138, 0xf>(v, old);
}
__device__ __forceinline__ int64_t wave_prev_i64(int64_t v, int64_t old) {
  const int lo = dpp_move_i<0x138, 0xf>((int)(uint32_t)v, (int)(uint32_t)old);
  const int hi = dpp_move_i<0x138, 0xf>((int)(v >> 32), (int)(old >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Block-wide reductions for a block of NT threads (NT/64 waves); `red` is
// LDS scratch of NT/64 doubles; ends with a barrier so `red` can be reused.
template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  v = wave_max(v);
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int i = 1; i < NT / WAVE; ++i) r = fmax(r, red[i]);
  __syncthreads();
  return r;
}
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  v = wave_sum(v);
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) r += red[i];
  __syncthreads();
  return r;
}
template <int NT>
__device__ __forceinline__ int block_max_i(int v, int* red) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  v = wave_max_i(v);
  if (lane == 0) red[w] = v;
  __syncthreads();
  int r = red[0];
#pragma unroll
  for (int i = 1; i < NT / WAVE; ++i) r = max(r, red[i]);
  __syncthreads();
  return r;
}
// inclusive block scan; returns the thread's inclusive prefix and the total
template <int NT>
__device__ __forceinline__ double block_incl_scan(double v, double* red, double& total) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  v = wave_incl_scan(v, lane);
  if (lane == WAVE - 1) red[w] = v;
  __syncthreads();
  double pre = 0.0, tot = 0.0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) {
    if (i < w) pre += red[i];
    tot += red[i];
  }
  __syncthreads();
  total = tot;
  return pre + v;
}

// inclusive running maximum across a block (exact)
template <int NT>
__device__ __forceinline__ double block_incl_max_scan(double v, double* red) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  v = wave_incl_max_scan(v, lane);
  if (lane == WAVE - 1) red[w] = v;
  __syncthreads();
  double pre = -INFINITY;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i)
    if (i < w) pre = fmax(pre, red[i]);
  __syncthreads();
  return fmax(pre, v);
}

// Number of strata k in [0, N) with (u + k) S < N W, i.e. the particles up
// to and including this one own strata 0 .. count-1.  The estimate from one
// multiplication by invS = 1/S lies within about N 2^-51 of NW/S - u, and a
// stratum's rounded product comparison can differ from the real one only
// within about N 2^-52 of it; so an estimate farther than N 2^-44 from an
// integer is the exact count.  Otherwise (about N 2^-43 of the time) it is
// checked with the exact product comparison on both sides, and a lane whose
// check fails (the estimate rounded across a stratum edge) steps to the
// exact count, so the result does not depend on how the estimate rounds.
// N < 2^31.
__device__ __forceinline__ int32_t stratum_count(double W, double S, double invS, double u,
                                                 int32_t N) {
  const double Nd = (double)N;
  const double NW = Nd * W;
  const double xv = NW * invS - u;
  // fmax maps a NaN estimate to 0; the exact checks below then decide
  int32_t est = (int32_t)__builtin_ceil(fmin(fmax(xv, 0.0), Nd));
  const double fr = xv - __builtin_floor(xv);  // NaN for a NaN estimate
  const double thr = Nd * 0x1p-44;
  if (fr > thr && fr < 1.0 - thr) return est;
  const bool down = est > 0 && !((u + (double)(est - 1)) * S < NW);
  const bool up = est < N && (u + (double)est) * S < NW;
  if (down) {
    --est;
    while (est > 0 && !((u + (double)(est - 1)) * S < NW)) --est;
  } else if (up) {
    ++est;
    while (est < N && (u + (double)est) * S < NW) ++est;
  }
  return est;
}

// ---------------------------------------------------------------- resampling variants

// Stratified offset of stratum k: the uniform of word k mod 4 of the
// generator at (k div 4, t, tag RESAMPLE | block 1 | iteration, b).
__device__ __forceinline__ double strat_u(Key key, int32_t t, uint32_t b, uint32_t iter,
                                          int32_t k) {
  const uint4 w = draw(key, TAG_RESAMPLE, 1, iter, (uint32_t)k >> 2, (uint32_t)t, b);
  const uint32_t r = k & 3;
  return u01_f64(r == 0 ? w.x : r == 1 ? w.y : r == 2 ? w.z : w.w);
}

// Number of strata k in [0, N) with (u_k + k) S < N W for the stratified
// offsets u_k (k + u_k is non-decreasing in k, so these strata are a
// prefix).  Starts from floor(N W / S) and steps with the exact product
// comparisons, each drawing the offset it needs.
__device__ __forceinline__ int32_t stratum_count_strat(double W, double S, double invS,
                                                       int32_t N, Key key, int32_t t, uint32_t b,
                                                       uint32_t iter) {
  const double Nd = (double)N;
  const double NW = Nd * W;
  int32_t est = (int32_t)__builtin_floor(fmin(fmax(NW * invS, 0.0), Nd));
  if (est < N && (strat_u(key, t, b, iter, est) + (double)est) * S < NW) {
    ++est;
    while (est < N && (strat_u(key, t, b, iter, est) + (double)est) * S < NW) ++est;
  } else {
    while (est > 0 && !((strat_u(key, t, b, iter, est - 1) + (double)(est - 1)) * S < NW)) --est;
  }
  return est;
}

// Proposal j' and uniform u of Metropolis move s (1-based) of output k:
// words 2r and 2r+1, r = (s-1) mod 2, of the generator at (k, t, tag
// RESAMPLE | block 2 + (s-1) div 2 | iteration, b); j' = floor(w N 2^-32).
// Moves s and s+1 (s odd) share one draw.
__device__ __forceinline__ uint4 metro_draw(Key key, int32_t t, uint32_t b, uint32_t iter,
                                            int32_t k, int32_t s) {
  return draw(key, TAG_RESAMPLE, 2u + (uint32_t)((s - 1) >> 1), iter, (uint32_t)k, (uint32_t)t,
              b);
}
// Multinomial uniform of output k: word k mod 4 of the generator at
// (k div 4, t, tag MULTI | iteration, b).
__device__ __forceinline__ double multi_u(Key key, int32_t t, uint32_t b, uint32_t iter,
                                          int32_t k) {
  const uint4 w = draw(key, TAG_MULTI, 0, iter, (uint32_t)k >> 2, (uint32_t)t, b);
  const uint32_t r = k & 3;
  return u01_f64(r == 0 ? w.x : r == 1 ? w.y : r == 2 ? w.z : w.w);
}

__device__ __forceinline__ int32_t metro_index(uint32_t w, int32_t N) {
  return (int32_t)(((uint64_t)w * (uint64_t)N) >> 32);
}

// Rejection resampling: attempts 2p and 2p+1 of output k take words (x, y)
// and (z, w) of the generator at (k, t + (p div 256) 2^20, tag REJECT |
// block p mod 256 | iteration, b) (t < 2^20): a candidate floor(w N 2^-32)
// from the first word of each pair (attempt 0's candidate is k itself) and
// a uniform from the second.  At most REJECT_MAX_ATTEMPTS attempts.
constexpr int64_t REJECT_MAX_ATTEMPTS = int64_t(1) << 21;
__device__ __forceinline__ uint4 reject_draw(Key key, int32_t t, uint32_t b, uint32_t iter,
                                             int32_t k, uint32_t p) {
  return draw(key, TAG_REJECT, p & 255u, iter, (uint32_t)k, (uint32_t)t + ((p >> 8) << 20), b);
}

// Output k's ancestor by rejection: candidates until ln u <= lw_j - M (M
// the largest log-weight); a NaN log-weight counts as -inf.  `lwj(j)` reads
// log-weight j.  After REJECT_MAX_ATTEMPTS attempts the output keeps k.
template <class LW>
__device__ __forceinline__ int32_t reject_ancestor(Key key, int32_t t, uint32_t b, uint32_t iter,
                                                   int32_t k, int32_t N, double M, LW lwj) {
#pragma unroll 1
  for (uint32_t p = 0; p < (uint32_t)(REJECT_MAX_ATTEMPTS >> 1); ++p) {
    const uint4 w = reject_draw(key, t, b, iter, k, p);
    int32_t c = p == 0 ? k : metro_index(w.x, N);
    double lc = lwj(c);
    lc = (lc == lc) ? lc : -INFINITY;
    if (ln_f64(u01_f64(w.y)) <= lc - M) return c;
    c = metro_index(w.z, N);
    lc = lwj(c);
    lc = (lc == lc) ? lc : -INFINITY;
    if (ln_f64(u01_f64(w.w)) <= lc - M) return c;
  }
  return k;
}

}  // namespace pfk
