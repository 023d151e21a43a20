// Device building blocks of the particle kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stats.hpp"
#include "types.hpp"
#include "unit_math.hpp"

namespace mlmc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011).  Counter layout used
// by the particle kernels: (block, sample, tag, stream).  Block, tag and
// stream are wave-uniform and only the sample word varies across lanes, so
// both products of the first round, one of the second and one of the third
// stay on the scalar unit.
// ---------------------------------------------------------------------------
struct Words {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
  // Each round's xors take the key and two words.  While one of the two is
  // wave-uniform, grouping it with the key leaves a single vector xor (the
  // scalar unit forms the rest); once both vary, the three-input xor is one
  // v_bitop3_b32 (truth table 0x96).  The groupings follow which words are
  // uniform in rounds 1-4 when only c1 varies; they are exact for any input.
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), hi1 = (uint32_t)(p1 >> 32);
    const uint32_t y0 = (r == 0) ? (c1 ^ (hi1 ^ k0))
                      : (r < 3)  ? (hi1 ^ (c1 ^ k0))
                                 : xor3(hi1, c1, k0);
    const uint32_t y2 = (r == 2) ? (c3 ^ (hi0 ^ k1))
                      : (r < 4)  ? (hi0 ^ (c3 ^ k1))
                                 : xor3(hi0, c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = y0;
    c2 = y2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words{c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// Uniform (2*(w>>9)+1) * 2^-24 on (0,1), bitwise equal in FP32 and FP64.
// FP32: one v_alignbit builds the float 1 + (w>>9) 2^-23 in [1,2); the
// subtraction of 1 - 2^-24 is exact (the result has 24 significant bits).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float uniform_f32(uint32_t w) {
  const uint32_t bits = __builtin_amdgcn_alignbit(0x7Fu, w, 9u);  // 0x3F800000 | (w >> 9)
  return __uint_as_float(bits) - 0.99999994039535522461f;         // 1 - 2^-24
}

__device__ __forceinline__ double uniform_f64(uint32_t w) {
  return (double)((w >> 8) | 1u) * 0x1p-24;
}

// Box-Muller pair: xi = r cos(2 pi u2), g = r sin(2 pi u2), r = sqrt(-2 ln u1).
// FP32 uses the hardware transcendentals: v_log_f32 is log2, and v_sin_f32 /
// v_cos_f32 take their argument in revolutions, so 2 pi u2 is never formed.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& xi, float& g) {
  const float u1 = uniform_f32(wa);
  const float u2 = uniform_f32(wb);
  const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));
  xi = r * __builtin_amdgcn_cosf(u2);
  g = r * __builtin_amdgcn_sinf(u2);
}

// FP64: the logarithm and sine/cosine of unit_math.hpp (series written for
// these uniforms, within 2 ulp).
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& xi, double& g) {
  const double u1 = uniform_f64(wa);
  const double u2 = uniform_f64(wb);
  const double r = sqrt(-2.0 * log_unit(u1));
  double s, c;
  sincospi_unit(2.0 * u2, s, c);
  xi = r * c;
  g = r * s;
}

template <typename Real>
__device__ __forceinline__ Real fma_r(Real a, Real b, Real c);
template <>
__device__ __forceinline__ float fma_r<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
template <>
__device__ __forceinline__ double fma_r<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }

// ---------------------------------------------------------------------------
// Inverse CDF of the density 1 + cos(2 pi x) on [0,1], in FP64.
// With y = 2 pi (x - 1/2) the CDF equation x + sin(2 pi x)/(2 pi) = u becomes
// Kepler's equation at eccentricity one, y - sin y = c = 2 pi (u - 1/2),
// |c| <= pi.  Solve for |c| by Newton from the cube-root start (6|c|)^(1/3),
// which lies left of the root since y - sin y <= y^3/6; y - sin y is convex
// on [0, pi], so after the first step the iterates decrease monotonically.
// y - sin y is evaluated by its Taylor series for small y (no cancellation).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double y_minus_sin(double y) {
  if (y < 0.5) {
    const double y2 = y * y;
    // y^3/3! - y^5/5! + ... - y^15/15!; truncation below 1e-19 relative
    double t = 1.0 / 1307674368000.0;                 // 1/15!
    t = fma(t, -y2, 1.0 / 6227020800.0);              // 1/13!
    t = fma(t, -y2, 1.0 / 39916800.0);                // 1/11!
    t = fma(t, -y2, 1.0 / 362880.0);                  // 1/9!
    t = fma(t, -y2, 1.0 / 5040.0);                    // 1/7!
    t = fma(t, -y2, 1.0 / 120.0);                     // 1/5!
    t = fma(t, -y2, 1.0 / 6.0);                       // 1/3!
    return t * y2 * y;
  }
  return y - sin(y);
}

__device__ __noinline__ double cosine_icdf(double u) {
  const double two_pi = 6.283185307179586476925;
  const double c = two_pi * (u - 0.5);
  const double ac = fabs(c);
  double y = cbrt(6.0 * ac);
  if (y > 3.141592653589793) y = 3.141592653589793;
  for (int it = 0; it < 8; ++it) {
    const double g = y_minus_sin(y) - ac;
    const double dg = 1.0 - cos(y);
    if (!(dg > 0.0)) break;
    const double step = g / dg;
    y -= step;
    if (fabs(step) <= 1e-17 * y) break;
  }
  y = copysign(y, c);
  return 0.5 + y / two_pi;
}

// ---------------------------------------------------------------------------
// Keeps a value live in a VGPR at this point, so the compiler cannot sink its
// computation into a branch (used to keep the collision select branch-free).
template <typename T>
__device__ __forceinline__ void keep(T& v) {
  asm volatile("" : "+v"(v));
}

// Decision "word < threshold" for thresholds in [0, 2^32].  The common path
// compares against threshold-1 in 32 bits (thresholds >= 1); the wide path
// (a zero threshold somewhere in the item) compares in 64 bits.
template <bool WIDE>
__device__ __forceinline__ bool below(uint32_t w, uint32_t thr_m1, uint64_t thr) {
  if constexpr (WIDE) return (uint64_t)w < thr;
  else return w <= thr_m1;
}

// ---------------------------------------------------------------------------
// Wave-level sums in a fixed xor-butterfly: every lane ends with the same,
// deterministic value (IEEE addition is commutative, and all lanes apply the
// same tree).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 1; m < kLanes; m <<= 1) v += __shfl_xor(v, m, kLanes);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int m = 1; m < kLanes; m <<= 1) v += __shfl_xor(v, m, kLanes);
  return v;
}

}  // namespace mlmc
