// Host check of log_unit and sincospi_unit (csrc/unit_math.hpp) over every
// uniform of the random-number stream, u = (2k+1) 2^-24, k < 2^23: log_unit(u)
// and sincospi_unit(2u) against long-double references; and of expm1_neg on a
// dense sample of [0, 45].  Prints the largest errors in units of the last
// place of the double result.
#include <math.h>
#include <stdio.h>
#include <stdint.h>

#include "unit_math.hpp"

static long double ulp_of(double v) {
  const double a = fabs(v);
  return (long double)(nextafter(a, INFINITY) - a);
}

int main() {
  long double max_log = 0, max_sin = 0, max_cos = 0, max_log_abs = 0;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (uint32_t k = 0; k < (1u << 23); ++k) {
    const double u = (double)(2u * k + 1u) * 0x1p-24;
    const double l = mlmc::log_unit(u);
    const long double lr = logl((long double)u);
    const long double el = fabsl((long double)l - lr);
    if (el / ulp_of((double)lr) > max_log) max_log = el / ulp_of((double)lr);
    if (el > max_log_abs) max_log_abs = el;
    double s, c;
    mlmc::sincospi_unit(2.0 * u, s, c);
    // reference: the argument reduced exactly (x - n/2, n = 2x rounded), then
    // sinl/cosl of pi r in long double and the quarter turn applied, so that
    // pi's rounding never meets a large argument
    const long double x = 2.0L * (long double)u;
    const long double n = rintl(2.0L * x);
    const long double r = x - 0.5L * n;
    const long double a = sinl(pi * r), b = cosl(pi * r);
    const int q = (int)n & 3;
    const long double sr = q == 0 ? a : (q == 1 ? b : (q == 2 ? -a : -b));
    const long double cr = q == 0 ? b : (q == 1 ? -a : (q == 2 ? -b : a));
    const long double es = fabsl((long double)s - sr) / ulp_of((double)sr);
    const long double ec = fabsl((long double)c - cr) / ulp_of((double)cr);
    if (es > max_sin) max_sin = es;
    if (ec > max_cos) max_cos = ec;
  }
  // e^{-y} - 1 on [0, 45] (the KD scheme's exponents R theta): an even grid of
  // 2^24 points, 1024 points per binade down to 2^-1000, and the ulps around
  // every switch of the reduction's k
  long double max_em = 0;
  auto em_check = [&](double y) {
    const long double r = expm1l(-(long double)y);
    const double e = mlmc::expm1_neg(y);
    const long double err = r == 0 ? (e == 0 ? 0.0L : 1e30L) : fabsl((long double)e - r) / ulp_of((double)r);
    if (err > max_em) max_em = err;
  };
  for (uint32_t i = 0; i <= (1u << 24); ++i) em_check((double)i * (45.0 / 16777216.0));
  for (int j = 1; j <= 1000; ++j)
    for (int i = 0; i < 1024; ++i) em_check(ldexp(1.0 + i / 1024.0, -j));
  for (int k = 0; k < 66; ++k) {
    double lo = (k + 0.5) * 0.69314718055994530942, hi = lo;
    for (int t = 0; t < 64; ++t) {
      lo = nextafter(lo, 0.0);
      hi = nextafter(hi, 100.0);
      if (lo >= 0.0 && lo <= 45.0) em_check(lo);
      if (hi <= 45.0) em_check(hi);
    }
  }
  printf("%.4Lf %.4Lf %.4Lf %.3Le %.4Lf\n", max_log, max_sin, max_cos, max_log_abs, max_em);
  return 0;
}
