// FP64 logarithm and sine/cosine of pi x for the uniforms of the random-number
// stream, and e^{-y} - 1 for the diffusive phases of the KD scheme, written
// from their series.  The library versions carry argument
// handling the particle loops never need (their inputs are the 24-bit
// uniforms (2k+1) 2^-24); these take about a third of the instructions and
// stay within 2 ulp (checked over every possible input on the host, where the
// same IEEE operations give the same values).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace mlmc {

// Natural logarithm of a positive normal double.  With x = 2^e F and F in
// [sqrt(1/2), sqrt(2)): ln x = e ln 2 + 2 atanh(s), s = (F - 1)/(F + 1),
// |s| <= 0.1716, and atanh(s)/s = sum_k s^(2k)/(2k+1) is summed to k = 10 (the
// next term is below 2^-57 of the sum).  F - 1 is exact; ln 2 is split so
// that e ln2_hi is exact for |e| < 2^11.
__host__ __device__ inline double log_unit(double x) {
  constexpr double kSqrtHalf = 0.70710678118654752440;
  constexpr double kLn2Hi = 0.6931471805598903;      // 42 significant bits of ln 2
  constexpr double kLn2Lo = 5.497923018708371e-14;   // ln 2 - kLn2Hi
  int e;
  double f = frexp(x, &e);  // x = f 2^e, f in [1/2, 1)
  if (f < kSqrtHalf) {
    f = f * 2.0;
    e -= 1;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double z = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double ls = fma(2.0 * s * z, p, 2.0 * s);  // 2 atanh(s) = 2s + 2s z p
  const double de = (double)e;
  return fma(de, kLn2Hi, fma(de, kLn2Lo, ls));
}

// sin(pi x) and cos(pi x) for 0 <= x <= 2 with x a multiple of 2^-50 (the
// reduction x - n/2 is then exact).  n = the nearest quarter turn, r = x -
// n/2 in [-1/4, 1/4], and sin(pi r), cos(pi r) by their Taylor series to the
// r^19 and r^18 terms (the next terms are below 2^-60); the quarter turn
// swaps and negates them.  Coefficients: (-1)^k pi^(2k+1)/(2k+1)! and
// (-1)^k pi^(2k)/(2k)!, rounded to double.
__host__ __device__ inline void sincospi_unit(double x, double& s, double& c) {
  const double n = rint(2.0 * x);
  const double r = x - 0.5 * n;
  const double z = r * r;
  double ps = -2.2948428997269873e-08;
  ps = fma(ps, z, 7.952054001475513e-07);
  ps = fma(ps, z, -2.1915353447830217e-05);
  ps = fma(ps, z, 0.00046630280576761255);
  ps = fma(ps, z, -0.0073704309457143504);
  ps = fma(ps, z, 0.08214588661112823);
  ps = fma(ps, z, -0.5992645293207921);
  ps = fma(ps, z, 2.5501640398773455);
  ps = fma(ps, z, -5.16771278004997);
  const double sp = fma(r * z, ps, 3.141592653589793 * r);
  double pc = -1.3878952462213771e-07;
  pc = fma(pc, z, 4.303069587032947e-06);
  pc = fma(pc, z, -0.0001046381049248457);
  pc = fma(pc, z, 0.0019295743094039231);
  pc = fma(pc, z, -0.02580689139001406);
  pc = fma(pc, z, 0.2353306303588932);
  pc = fma(pc, z, -1.3352627688545895);
  pc = fma(pc, z, 4.0587121264167685);
  pc = fma(pc, z, -4.934802200544679);
  const double cp = fma(z, pc, 1.0);
  const int q = (int)n & 3;
  const double s0 = (q & 1) ? cp : sp;
  const double c0 = (q & 1) ? sp : cp;
  s = (q & 2) ? -s0 : s0;
  c = ((q + 1) & 2) ? -c0 : c0;
}

// e^{-y} - 1 for 0 <= y <= 700.  y = k ln 2 + r with k the nearest integer
// to y/ln 2, |r| <= ln(2)/2 (r by a two-part ln 2, exact in its first
// product); expm1(-r) by its Taylor series to the 15th power (the next term
// is below 2^-60 of it), and e^{-y} - 1 = 2^-k expm1(-r) + (2^-k - 1) in one
// rounding (2^-k - 1 is exact).
__host__ __device__ inline double expm1_neg(double y) {
  constexpr double kInvLn2 = 1.4426950408889634;
  constexpr double kLn2Hi = 0.6931471805598903;
  constexpr double kLn2Lo = 5.497923018708371e-14;
  const double k = rint(y * kInvLn2);
  const double x = fma(k, kLn2Lo, fma(k, kLn2Hi, -y));  // -(y - k ln 2)
  double q = 7.647163731819816e-13;                      // 1/15!
  q = fma(q, x, 1.1470745597729725e-11);
  q = fma(q, x, 1.6059043836821613e-10);
  q = fma(q, x, 2.08767569878681e-09);
  q = fma(q, x, 2.505210838544172e-08);
  q = fma(q, x, 2.755731922398589e-07);
  q = fma(q, x, 2.7557319223985893e-06);
  q = fma(q, x, 2.48015873015873e-05);
  q = fma(q, x, 0.0001984126984126984);
  q = fma(q, x, 0.001388888888888889);
  q = fma(q, x, 0.008333333333333333);
  q = fma(q, x, 0.041666666666666664);
  q = fma(q, x, 0.16666666666666666);
  q = fma(q, x, 0.5);
  const double p = fma(x * x, q, x);                     // expm1(x)
  const double scale = ldexp(1.0, -(int)k);
  return fma(scale, p, scale - 1.0);
}

}  // namespace mlmc
