// Kinetic-diffusion (KD) scheme on the device: one path or one correlated
// fine/coarse pair per lane, FP64 state.
//
// Homogeneous background in the diffusive scaling: collision rate R =
// 1/eps^2, post-collision velocities N(mu, sigma^2) with mu = 0 and sigma =
// 1/eps.  A KD step (Section 2, Algorithm "KD algorithm") starts on the time
// grid at t with velocity v and a pending collision at c = t + E/R: the path
// flies to c, then moves diffusively to the end of the grid step holding c
// (length theta) with the advection a and diffusion d of eqs. advection and
// diffusion, conditioned on the next velocity.  Once the pending collision
// is at or after T the path flies to T.
//
// Pair (Section 3, Algorithm "Correlated KD algorithm"): the coarse path's
// flight mirrors the fine flight kappa_k (eq. nu-update; eq.
// epsilon-update, which in a homogeneous background puts the coarse
// collision at the fine collision time), and its diffusive phase takes the
// normalised weighted sum (eq. chi-update) of the fine diffusive numbers and
// of the velocity numbers of the fine flights in between, weights alpha_m =
// sigma tau'_m and beta_m (eq. weights-beta) after moving zeta_m =
// (1 - e^{-R theta_m})/R from each diffusive phase to the next flight.  The
// fine path steps until its pending collision lies after the end of the
// coarse grid step; step indices are compared as integers of the fine grid.
//
// Random numbers: Philox block 0 = initial condition (Box-Muller pair of
// words 0, 1: cosine branch -> normal x0, sine branch -> nu_0; word 2 ->
// E_0 = -log u; word 3 -> u of the cosine law), block k+1 = KD step k (pair
// of words 0, 1: nu_{k+1}, chi_k; word 2 -> E_{k+1}).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace mlmc {

// Three functions of y = R theta >= 0 that cancel catastrophically when
// written with exp for small y; below y = 0.05 they are summed from their
// Taylor series (terms up to y^16, Horner form), above from exp/expm1:
//   kd_h(y) = e^{-y} - 1 + y                 (the unconditioned variance shape)
//   kd_f(y) = 2(e^{-y} - 1) + y(e^{-y} + 1)  (first term of eq. diffusion)
//   kd_g(y) = 1 - 2y e^{-y} - e^{-2y}        (second term of eq. diffusion)
constexpr double kKdSeriesY = 0.05;
constexpr int kKdTerms = 16;

// Taylor coefficients of y^m, m <= kKdTerms, of the three functions
struct KdCoefs {
  double h[kKdTerms + 1], f[kKdTerms + 1], g[kKdTerms + 1];
};

constexpr KdCoefs kd_make_coefs() {
  KdCoefs c{};
  double inv_fact = 1.0, pow2 = 1.0;
  for (int m = 0; m <= kKdTerms; ++m) {
    if (m > 0) {
      inv_fact /= (double)m;
      pow2 *= 2.0;
    }
    const double sign_odd = (m % 2) ? 1.0 : -1.0;  // (-1)^(m+1)
    c.h[m] = m >= 2 ? -sign_odd * inv_fact : 0.0;
    c.f[m] = m >= 3 ? sign_odd * (double)(m - 2) * inv_fact : 0.0;
    c.g[m] = m >= 3 ? sign_odd * (pow2 - 2.0 * (double)m) * inv_fact : 0.0;
  }
  return c;
}

// sum_{m=LO}^{kKdTerms} c[m] y^m by Horner's rule
template <int LO>
__device__ __forceinline__ double kd_series(const double (&c)[kKdTerms + 1], double y) {
  double s = c[kKdTerms];
#pragma unroll
  for (int m = kKdTerms - 1; m >= LO; --m) s = s * y + c[m];
  double p = 1.0;
#pragma unroll
  for (int m = 0; m < LO; ++m) p *= y;
  return s * p;
}

// With em = e^{-y} - 1 (expm1: accurate for small y) the exp forms above
// are, exactly,
//   kd_h = em + y,   kd_f = 2 em + y (2 + em),   kd_g = -(em (2 + em) + 2 y (1 + em)),
// so one expm1 per diffusive phase serves eqs. advection and diffusion and
// the aggregation weights.
// Branch condition c.  U: c has the same value in every lane (the
// time-parallel paths walk one path per wavefront on wave-uniform values),
// so the branch is taken on the scalar unit instead of under an exec mask;
// the arithmetic on either side is the same.
template <bool U>
__device__ __forceinline__ bool when(bool c) {
  if constexpr (U) return __builtin_amdgcn_readfirstlane((int)c) != 0;
  else return c;
}

__device__ __forceinline__ double kd_h(double y, double em) {
  constexpr KdCoefs C = kd_make_coefs();
  return y < kKdSeriesY ? kd_series<2>(C.h, y) : em + y;
}

template <bool U = false>
__device__ __forceinline__ double kd_f(double y, double em) {
  constexpr KdCoefs C = kd_make_coefs();
  return when<U>(y < kKdSeriesY) ? kd_series<3>(C.f, y) : 2.0 * em + y * (2.0 + em);
}

template <bool U = false>
__device__ __forceinline__ double kd_g(double y, double em) {
  constexpr KdCoefs C = kd_make_coefs();
  return when<U>(y < kKdSeriesY) ? kd_series<3>(C.g, y) : -(em * (2.0 + em) + 2.0 * y * (1.0 + em));
}

// e^{-y} - 1 for y >= 0 (expm1_neg of unit_math.hpp).  Above y = 45,
// e^{-y} < 3e-20 lies far below half the spacing of doubles next to -1
// (2^-54), so every faithfully rounded expm1 returns exactly -1 there.  A wavefront whose lanes all have y > 45
// skips the library call; the per-lane select keeps each lane's value the
// same whichever way its wavefront goes.
constexpr double kKdExpm1Cut = 45.0;

template <bool U = false>
__device__ __forceinline__ double kd_em(double y) {
  if constexpr (U) {
    return when<U>(y > kKdExpm1Cut) ? -1.0 : expm1_neg(y);
  } else {
    if (__all(y > kKdExpm1Cut)) return -1.0;
    return y > kKdExpm1Cut ? -1.0 : expm1_neg(y);
  }
}

struct KdParams {
  double dtf, dtc, R, sigma, mu, T;
  double inv_r;   // 1/R
  double inv_r2;  // 1/R^2
  double c2;      // 2 sigma^2 / R^2
  uint32_t M, tag, strm, key0, key1;
  uint32_t guard;  // bound on fine KD steps (a step advances at least one grid step)
  double inv_dtf, inv_dtc;  // 1/dtf, 1/dtc
  bool pow2_f, pow2_c;      // dtf (dtc) is a power of two
};

__device__ __forceinline__ bool kd_is_pow2(double x) {
  int e;
  return x > 0.0 && frexp(x, &e) == 0.5;
}

// floor(c / dt) on a grid of step dt.  Where dt is a power of two, c (1/dt)
// is exact and equal to the quotient, and the FP64 division is skipped.
__device__ __forceinline__ double kd_grid_floor(double c, double dt, double inv_dt, bool pow2) {
  if (pow2) return floor(c * inv_dt);
  return floor(c / dt);
}

__device__ __forceinline__ KdParams kd_params(const LevelDesc& d) {
  KdParams k;
  k.dtf = d.h_f;
  k.dtc = d.h_c;
  k.R = d.s_f;
  k.sigma = d.s_c;
  k.mu = d.h_f2;
  k.T = d.agg_ms2;
  k.M = d.M;
  k.tag = d.tag;
  k.strm = d.stream;
  k.key0 = d.key0;
  k.key1 = d.key1;
  k.guard = d.n_steps + 2u;
  k.inv_r = 1.0 / k.R;
  k.inv_r2 = k.inv_r * k.inv_r;
  k.c2 = 2.0 * k.sigma * k.sigma * k.inv_r2;
  k.pow2_f = kd_is_pow2(k.dtf);
  k.pow2_c = kd_is_pow2(k.dtc);
  k.inv_dtf = k.pow2_f ? 1.0 / k.dtf : 0.0;
  k.inv_dtc = k.pow2_c ? 1.0 / k.dtc : 0.0;
  return k;
}

// eq. advection and eq. diffusion: a and d of a diffusive phase of length
// theta that ends with velocity v_next; y = R theta, em = e^{-y} - 1.
__device__ __forceinline__ void kd_coeffs(const KdParams& k, double theta, double y, double em,
                                          double v_next, double& a, double& dd) {
  const double dv = v_next - k.mu;
  a = k.mu * theta + dv * (-em) * k.inv_r;
  const double d2 = k.c2 * kd_f(y, em) + dv * dv * k.inv_r2 * kd_g(y, em);
  dd = sqrt(d2 > 0.0 ? d2 : 0.0);
}

// Numbers of KD step b - 1 from Philox block b.
__device__ __forceinline__ void kd_draws(const KdParams& k, uint32_t smp, uint32_t b,
                                         double& nu_next, double& chi, double& E_next) {
  const Words w = philox4x32_10(b, smp, k.tag, k.strm, k.key0, k.key1);
  box_muller(w.w0, w.w1, nu_next, chi);
  E_next = -log_unit(uniform_f64(w.w2));
}

// Optional record of a pair's coarse numbers, for the consistency harness of
// Section 5.1: row k = (chi~, nu~, E~, fine KD steps aggregated) of coarse KD
// step k.  The simulation kernels use KdNoRecord, which compiles away.
struct KdNoRecord {
  static constexpr bool kOn = false;
  __device__ __forceinline__ void put(double, double, double, uint32_t) {}
};

struct KdRecord {
  static constexpr bool kOn = true;
  double* rows;
  uint32_t cap;
  uint32_t n;
  __device__ __forceinline__ void put(double chi, double nu, double e, uint32_t used) {
    if (n < cap) {
      double* r = rows + 4ull * n;
      r[0] = chi;
      r[1] = nu;
      r[2] = e;
      r[3] = (double)used;
    }
    ++n;
  }
};

// One path (COARSE = false) or a correlated pair of sample smp: final
// positions and KD step counts (collisions before T).
template <bool COARSE, typename Rec>
__device__ __forceinline__ void kd_sample_rec(const LevelDesc& d, uint32_t smp, double& xf_out,
                                              double& xc_out, uint32_t& cf_out, uint32_t& cc_out,
                                              Rec& rec) {
  const KdParams k = kd_params(d);
  // initial condition, shared by both paths
  const Words w0 = philox4x32_10(0u, smp, k.tag, k.strm, k.key0, k.key1);
  double nc, ns;
  box_muller(w0.w0, w0.w1, nc, ns);
  double x0;
  if (d.x0_kind == 0) x0 = d.x0_a;
  else if (d.x0_kind == 1) x0 = d.x0_a + d.x0_b * nc;
  else x0 = cosine_icdf(uniform_f64(w0.w3));
  const double E0 = -log_unit(uniform_f64(w0.w2));

  double xf = x0, vf = k.mu + k.sigma * ns, tf = 0.0, tauf = E0 * k.inv_r;
  double cfine = tf + tauf;
  uint32_t cf = 0, cc = 0, b = 1;

  if constexpr (!COARSE) {
    while (cfine < k.T && cf < k.guard) {
      double nu_next, chi, E_next;
      kd_draws(k, smp, b++, nu_next, chi, E_next);
      const double t_next = (kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0) * k.dtf;
      const double theta = t_next - cfine;
      const double y = k.R * theta;
      const double em = kd_em(y);
      const double v_next = k.mu + k.sigma * nu_next;
      double a, dd;
      kd_coeffs(k, theta, y, em, v_next, a, dd);
      xf = xf + vf * tauf + (a + dd * chi);
      tf = t_next;
      tauf = E_next * k.inv_r;
      cfine = tf + tauf;
      vf = v_next;
      ++cf;
    }
    if (tf < k.T) xf = xf + vf * (k.T - tf);
    xf_out = xf;
    xc_out = 0.0;
    cf_out = cf;
    cc_out = 0u;
  } else {
    double xc = x0, vc = vf, tc = 0.0, ccoarse = cfine;
    double nu_f = ns;  // velocity number of the fine path's pending flight
    // index of the fine grid point that ends the pending flight's step
    // (computed once per flight: the loop test and the next step share it)
    double nf = kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0;
    while ((ccoarse < k.T || cfine < k.T) && cf < k.guard) {
      // end of the coarse grid step holding the coarse collision, as an
      // index of the fine grid
      const double end_c = kd_grid_floor(ccoarse, k.dtc, k.inv_dtc, k.pow2_c) + 1.0;
      const double end_c_fine = end_c * (double)k.M;
      double num = 0.0, den = 0.0, zeta_prev = 0.0;
      bool first = true;
      uint32_t used = 0;
      do {
        if constexpr (Rec::kOn) ++used;
        double nu_next, chi, E_next;
        kd_draws(k, smp, b++, nu_next, chi, E_next);
        const double t_next = nf * k.dtf;
        const double theta = t_next - cfine;
        const double y = k.R * theta;
        const double em = kd_em(y);
        const double v_next = k.mu + k.sigma * nu_next;
        double a, dd;
        kd_coeffs(k, theta, y, em, v_next, a, dd);
        xf = xf + vf * tauf + (a + dd * chi);
        // aggregation weights of this fine phase: zeta = (1 - e^{-y})/R, and
        // beta over theta' = theta - zeta, i.e. R theta' = kd_h(y)
        const double zeta = -em * k.inv_r;
        const double yp = kd_h(y, em);
        const double beta = sqrt(k.c2 * kd_h(yp, yp < kKdSeriesY ? 0.0 : kd_em(yp)));
        if (!first) {
          const double alpha = (tauf + zeta_prev) * k.sigma;
          num += alpha * nu_f;
          den += alpha * alpha;
        }
        num += beta * chi;
        den += beta * beta;
        zeta_prev = zeta;
        first = false;
        tf = t_next;
        tauf = E_next * k.inv_r;
        cfine = tf + tauf;
        nf = kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0;
        vf = v_next;
        nu_f = nu_next;
        ++cf;
      } while (!(nf > end_c_fine) && cf < k.guard);
      if (ccoarse < k.T) {
        const double chi_c = den > 0.0 ? num / sqrt(den) : 0.0;
        const double t_next = end_c * k.dtc;
        const double theta = t_next - ccoarse;
        const double y = k.R * theta;
        const double v_next = k.mu + k.sigma * nu_f;
        double a, dd;
        kd_coeffs(k, theta, y, kd_em(y), v_next, a, dd);
        xc = xc + vc * (ccoarse - tc) + (a + dd * chi_c);
        tc = t_next;
        ccoarse = cfine;
        vc = v_next;
        ++cc;
        // E~ of eq. epsilon-update: what is left of the fine flight's number
        if constexpr (Rec::kOn) rec.put(chi_c, nu_f, k.R * (cfine - tc), used);
      }
    }
    if (tf < k.T) xf = xf + vf * (k.T - tf);
    if (tc < k.T) xc = xc + vc * (k.T - tc);
    xf_out = xf;
    xc_out = xc;
    cf_out = cf;
    cc_out = cc;
  }
}

template <bool COARSE>
__device__ __forceinline__ void kd_sample(const LevelDesc& d, uint32_t smp, double& xf_out,
                                          double& xc_out, uint32_t& cf_out, uint32_t& cc_out) {
  KdNoRecord none;
  kd_sample_rec<COARSE>(d, smp, xf_out, xc_out, cf_out, cc_out, none);
}

// ---------------------------------------------------------------------------
// The KD scheme in the backgrounds of Section 5 (flags kFlagBgB1 / kFlagBgB2;
// a > 0 -- a = 0 is the homogeneous path above with R = b): Maxwellian with
// mu = 0 and sigma = 1, collision rate piecewise linear with a kink at x = 1,
//   B1: R(x) = b (a |x - 1| + 1),   B2: R(x) = b (a max(x - 1, 0) + 1).
// ---------------------------------------------------------------------------
struct KdBackground {
  double a, b;
  bool b1;
};

__device__ __forceinline__ double bg_rate(const KdBackground& g, double x) {
  const double u = x - 1.0;
  return g.b * (g.a * (g.b1 ? fabs(u) : fmax(u, 0.0)) + 1.0);
}

// Flight time of eq. intinv from x with velocity v and exponential number E.
// Along the flight the rate is linear in time on each side of the kink, so
// the root of r0 s + k s^2/2 = E is s = 2E / (r0 + sqrt(r0^2 + 2 k E)) (the
// square root is the rate at the collision); a flight heading for the kink
// first spends I1 = s_k (r0 + b)/2 of E on the way there.
template <bool U = false>
__device__ __forceinline__ double bg_flight(const KdBackground& g, double x, double v, double E) {
  const double u = x - 1.0;
  const double r0 = bg_rate(g, x);
  const double ab = g.a * g.b;
  const bool toward = (u < 0.0 && v > 0.0) || (u > 0.0 && v < 0.0);
  // d/ds R(x + v s) on the piece the flight starts on
  double k1;
  if (g.b1) k1 = (u > 0.0 || (u == 0.0 && v > 0.0)) ? ab * v : -ab * v;
  else k1 = (u > 0.0 || (u == 0.0 && v > 0.0)) ? ab * v : 0.0;
  if (when<U>(toward)) {
    const double sk = -u / v;
    const double i1 = 0.5 * sk * (r0 + g.b);
    if (when<U>(E > i1)) {
      const double e2 = E - i1;
      const double k2 = g.b1 ? ab * fabs(v) : (v > 0.0 ? ab * v : 0.0);
      return sk + 2.0 * e2 / (g.b + sqrt(g.b * g.b + 2.0 * k2 * e2));
    }
  }
  return 2.0 * E / (r0 + sqrt(r0 * r0 + 2.0 * k1 * E));
}

// int_0^t R(x + v s) ds (t < 0: minus the integral over [t, 0]); exact by
// the trapezoid rule on each linear piece.
template <bool U = false>
__device__ __forceinline__ double bg_rate_integral(const KdBackground& g, double x, double v,
                                                   double t) {
  double sign = 1.0;
  if (when<U>(t < 0.0)) {
    x = x + v * t;
    t = -t;
    sign = -1.0;
  }
  const double xe = x + v * t;
  const double u0 = x - 1.0, u1 = xe - 1.0;
  double r;
  if (when<U>(u0 * u1 < 0.0)) {
    const double sk = -u0 / v;
    r = 0.5 * sk * (bg_rate(g, x) + g.b) + 0.5 * (t - sk) * (g.b + bg_rate(g, xe));
  } else {
    r = 0.5 * t * (bg_rate(g, x) + bg_rate(g, xe));
  }
  return sign * r;
}

// 1/R and 2 sigma^2/R^2 of a local rate R.
__device__ __forceinline__ void bg_rate_consts(double R, double sigma, double& inv_r,
                                               double& inv_r2, double& c2) {
  inv_r = 1.0 / R;
  inv_r2 = inv_r * inv_r;
  c2 = 2.0 * sigma * sigma * inv_r2;
}

// eqs. advection and diffusion with the local rate R of the phase (its
// 1/R and 2 sigma^2/R^2 are returned for the aggregation weights).
template <bool U = false>
__device__ __forceinline__ void bg_coeffs(double R, double mu, double sigma, double theta,
                                          double y, double em, double v_next, double& a,
                                          double& dd, double& inv_r, double& c2) {
  double inv_r2;
  bg_rate_consts(R, sigma, inv_r, inv_r2, c2);
  const double dv = v_next - mu;
  a = mu * theta + dv * (-em) * inv_r;
  const double d2 = c2 * kd_f<U>(y, em) + dv * dv * inv_r2 * kd_g<U>(y, em);
  dd = sqrt(d2 > 0.0 ? d2 : 0.0);
}

// One path or one correlated pair in a background (Algorithm "KD algorithm",
// Algorithm "Correlated KD algorithm" with the general eq. epsilon-update).
// A pair's fine path keeps stepping past T while the coarse path still has a
// collision before T (those steps only feed the aggregation); the fine path
// itself ends at the first state whose pending collision is at or after T.
template <bool COARSE, typename Rec>
__device__ __forceinline__ void kd_sample_bg_rec(const LevelDesc& d, uint32_t smp,
                                                 double& xf_out, double& xc_out,
                                                 uint32_t& cf_out, uint32_t& cc_out, Rec& rec) {
  const KdParams k = kd_params(d);
  const KdBackground g{d.rsqrt_m, d.s_f, (d.flags & kFlagBgB1) != 0};
  const uint32_t guard = 2u * d.n_steps + 4u;
  const Words w0 = philox4x32_10(0u, smp, k.tag, k.strm, k.key0, k.key1);
  double nc, ns;
  box_muller(w0.w0, w0.w1, nc, ns);
  double x0;
  if (d.x0_kind == 0) x0 = d.x0_a;
  else if (d.x0_kind == 1) x0 = d.x0_a + d.x0_b * nc;
  else x0 = cosine_icdf(uniform_f64(w0.w3));
  const double E0 = -log_unit(uniform_f64(w0.w2));

  double xf = x0, vf = k.mu + k.sigma * ns, tf = 0.0, Ef = E0;
  double tauf = bg_flight(g, xf, vf, Ef);
  double cfine = tf + tauf;
  uint32_t cf = 0, cc = 0, b = 1, steps = 0;

  if constexpr (!COARSE) {
    while (cfine < k.T && steps < guard) {
      double nu_next, chi, E_next;
      kd_draws(k, smp, b++, nu_next, chi, E_next);
      const double t_next = (kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0) * k.dtf;
      const double theta = t_next - cfine;
      const double rl = bg_rate(g, xf + vf * tauf);   // rate at the collision
      const double y = rl * theta;
      const double v_next = k.mu + k.sigma * nu_next;
      double a, dd, inv_r, c2;
      bg_coeffs(rl, k.mu, k.sigma, theta, y, kd_em(y), v_next, a, dd, inv_r, c2);
      xf = xf + vf * tauf + (a + dd * chi);
      tf = t_next;
      vf = v_next;
      Ef = E_next;
      tauf = bg_flight(g, xf, vf, Ef);
      cfine = tf + tauf;
      ++cf;
      ++steps;
    }
    if (tf < k.T) xf = xf + vf * (k.T - tf);
    xf_out = xf;
    xc_out = 0.0;
    cf_out = cf;
    cc_out = 0u;
  } else {
    double xc = x0, vc = vf, tc = 0.0, tauc = tauf, ccoarse = tc + tauc;
    double nu_f = ns;
    bool fine_done = false;
    double xf_end = 0.0;
    // The algorithm's two nested loops (coarse KD steps; the fine steps of
    // each) as one loop of fine steps, a coarse KD step closing each block:
    // the arithmetic and its order are unchanged, but lanes whose blocks
    // differ in length keep stepping together instead of waiting for the
    // longest block of the wavefront.
    double end_c = 0.0, end_c_fine = 0.0, num = 0.0, den = 0.0, zeta_prev = 0.0;
    bool first = true, in_block = false;
    uint32_t used = 0;
    for (;;) {
      if (!in_block) {  // a coarse KD step begins
        if (!((ccoarse < k.T || cfine < k.T) && steps < guard)) break;
        end_c = kd_grid_floor(ccoarse, k.dtc, k.inv_dtc, k.pow2_c) + 1.0;
        end_c_fine = end_c * (double)k.M;
        num = 0.0;
        den = 0.0;
        zeta_prev = 0.0;
        first = true;
        used = 0;
        in_block = true;
      }
      if constexpr (Rec::kOn) ++used;
      if (cfine >= k.T && !fine_done) {
        xf_end = tf < k.T ? xf + vf * (k.T - tf) : xf;
        fine_done = true;
      }
      double nu_next, chi, E_next;
      kd_draws(k, smp, b++, nu_next, chi, E_next);
      const double t_next = (kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0) * k.dtf;
      const double theta = t_next - cfine;
      const double rm = bg_rate(g, xf + vf * tauf);
      const double y = rm * theta;
      const double em = kd_em(y);
      const double v_next = k.mu + k.sigma * nu_next;
      double a, dd, inv_r, c2;
      bg_coeffs(rm, k.mu, k.sigma, theta, y, em, v_next, a, dd, inv_r, c2);
      xf = xf + vf * tauf + (a + dd * chi);
      // aggregation weights of this phase with its own rate
      const double zeta = -em * inv_r;
      const double yp = kd_h(y, em);
      const double beta = sqrt(c2 * kd_h(yp, yp < kKdSeriesY ? 0.0 : kd_em(yp)));
      if (!first) {
        const double alpha = (tauf + zeta_prev) * k.sigma;
        num += alpha * nu_f;
        den += alpha * alpha;
      }
      num += beta * chi;
      den += beta * beta;
      zeta_prev = zeta;
      first = false;
      if (!fine_done) ++cf;
      tf = t_next;
      vf = v_next;
      nu_f = nu_next;
      Ef = E_next;
      tauf = bg_flight(g, xf, vf, Ef);
      cfine = tf + tauf;
      ++steps;
      // the block ends with the first fine step whose pending collision lies
      // past the coarse grid step
      if (kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0 > end_c_fine || steps >= guard) {
        in_block = false;
        if (ccoarse < k.T) {
          const double chi_c = den > 0.0 ? num / sqrt(den) : 0.0;
          const double t_nc = end_c * k.dtc;
          const double theta_c = t_nc - ccoarse;
          const double rc = bg_rate(g, xc + vc * tauc);
          const double yc = rc * theta_c;
          const double v_nc = k.mu + k.sigma * nu_f;
          double ac, ddc, inv_rc, c2c;
          bg_coeffs(rc, k.mu, k.sigma, theta_c, yc, kd_em(yc), v_nc, ac, ddc, inv_rc, c2c);
          xc = xc + vc * tauc + (ac + ddc * chi_c);
          tc = t_nc;
          vc = v_nc;
          // eq. epsilon-update: the pending fine flight's exponential number
          // less the rate integral along it up to the coarse time
          double ec = Ef - bg_rate_integral(g, xf, vf, tc - tf);
          ec = ec < 0.0 ? 0.0 : ec;
          tauc = bg_flight(g, xc, vc, ec);
          ccoarse = tc + tauc;
          ++cc;
          if constexpr (Rec::kOn) rec.put(chi_c, nu_f, ec, used);
        }
      }
    }
    if (!fine_done) xf_end = tf < k.T ? xf + vf * (k.T - tf) : xf;
    if (tc < k.T) xc = xc + vc * (k.T - tc);
    xf_out = xf_end;
    xc_out = xc;
    cf_out = cf;
    cc_out = cc;
  }
}

template <bool COARSE>
__device__ __forceinline__ void kd_sample_bg(const LevelDesc& d, uint32_t smp, double& xf_out,
                                             double& xc_out, uint32_t& cf_out,
                                             uint32_t& cc_out) {
  KdNoRecord none;
  kd_sample_bg_rec<COARSE>(d, smp, xf_out, xc_out, cf_out, cc_out, none);
}

}  // namespace mlmc
