// Host check of log_unit and sincospi_unit (csrc/unit_math.hpp) over every
// uniform of the random-number stream, u = (2k+1) 2^-24, k < 2^23: log_unit(u)
// and sincospi_unit(2u) against long-double references.  Prints the largest
// errors in units of the last place of the double result.
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
  printf("%.4Lf %.4Lf %.4Lf %.3Le\n", max_log, max_sin, max_cos, max_log_abs);
  return 0;
}
