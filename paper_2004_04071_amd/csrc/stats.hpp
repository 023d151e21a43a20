// Pairwise merge of FP64 sample statistics (Chan, Golub, LeVeque), shared by
// the device reductions and the host API.  Contraction into FMA is switched
// off so that host and device round every operation identically.
#pragma once
#include <hip/hip_runtime.h>

#include "types.hpp"

namespace mlmc {

__host__ __device__ inline Stats stats_empty() {
  Stats s;
  s.n = 0.0;
  s.mean_dq = s.m2_dq = s.mean_qf = s.m2_qf = s.mean_qc = s.m2_qc = s.c_fc = 0.0;
  s.coll_f = s.coll_c = 0ull;
  return s;
}

// out = a (+) b: n = na + nb, d = mean_b - mean_a,
//   mean = mean_a + d nb/n,  M2 = M2a + M2b + d^2 na nb/n,
//   C_fc = Ca + Cb + d_f d_c na nb/n.
__host__ __device__ inline Stats stats_merge(const Stats& a, const Stats& b) {
#pragma clang fp contract(off)
  if (b.n == 0.0) return a;
  if (a.n == 0.0) return b;
  Stats o;
  o.n = a.n + b.n;
  const double f = b.n / o.n;
  const double w = a.n * f;
  const double d_dq = b.mean_dq - a.mean_dq;
  const double d_f = b.mean_qf - a.mean_qf;
  const double d_c = b.mean_qc - a.mean_qc;
  o.mean_dq = a.mean_dq + d_dq * f;
  o.mean_qf = a.mean_qf + d_f * f;
  o.mean_qc = a.mean_qc + d_c * f;
  o.m2_dq = (a.m2_dq + b.m2_dq) + (d_dq * d_dq) * w;
  o.m2_qf = (a.m2_qf + b.m2_qf) + (d_f * d_f) * w;
  o.m2_qc = (a.m2_qc + b.m2_qc) + (d_c * d_c) * w;
  o.c_fc = (a.c_fc + b.c_fc) + (d_f * d_c) * w;
  o.coll_f = a.coll_f + b.coll_f;
  o.coll_c = a.coll_c + b.coll_c;
  return o;
}

}  // namespace mlmc
