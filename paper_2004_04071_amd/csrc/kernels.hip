// Particle and reduction kernels of the MLMC-AP library (gfx950).
//
// One wavefront owns one tile of 64 spl consecutive samples of a work item:
// lane i simulates samples tile*64*spl + 64 j + i, j < spl, P of them at a
// time (P = trajectories in flight per lane, for instruction-level
// parallelism; spl = 4 on levels of fewer than 64 fine steps, else 1).
// Particle state lives in registers for the whole trajectory; the only
// memory traffic is one 80-byte statistics record per tile (plus optional
// dumps and histogram counters).
//
// Per fine step (asymptotic-preserving splitting, fixed dt), from three words
// of the trajectory's Philox word stream (decision, radius, angle):
//   x <- x + h v + s xi;  collide iff decision word < thr  ->  v <- equilibrium draw.
// Positions never feed back into the dynamics, so with FP32 state the
// increments of 16 steps are summed on their own and added to x by a
// compensated (Fast2Sum) update: the position then carries about one rounding
// of its own size instead of two per step.
// Coarse path (levels >= 1), one coarse step per block of M fine steps, built
// from the fine random numbers of that block (Section 3.1 mapping by time of
// action; Section 3.2 aggregation):
//   kick   : eq. chi-update -- normalised weighted sum of the fine kick
//            normals and (aggregated coupling) of the fine velocity normals the
//            coarse path does not take, each weighted by its fine transport uses;
//   collide: the smallest fine decision word of the block is below thr_c2
//            <= thr_f, so a coarse collision reuses a fine one (the uniform
//            analogue of eq. epsilon-update) and P = p_c exactly;
//   v      : the fine velocity drawn last in the block (eq. nu-update).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "device.hpp"
#include "kd.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace mlmc {

// The P trajectories of one lane: state, coarse-block bookkeeping, and the
// word stream.  Each trajectory's random numbers are the words of its Philox
// blocks 0, 1, 2, ... (counter (block, sample, tag, stream)); the initial
// condition takes words 0-1 (0-5 for the cosine law) and every fine step the
// next three: decision word, Box-Muller radius word, Box-Muller angle word.
// Four fine steps therefore use exactly three blocks, and a group of four
// steps always starts with two words left over from the previous block.
template <typename Real, int P, int KIND, bool WIDE>
struct Lane {
  static constexpr bool kCoarse = KIND >= kKindPairTwoPointSum;
  static constexpr bool kMaxwell = KIND == kKindFineMaxwell || KIND == kKindPairMaxwellSum ||
                                   KIND == kKindPairMaxwellAggregate;
  static constexpr bool kAgg = KIND == kKindPairMaxwellAggregate;
  static constexpr bool kCompensate = sizeof(Real) == 4;

  Real h_f, s_f, h_c, s_c, agg_ms2, h_f2, rsqrt_m;
  uint32_t thr_f_m1, thr_c2_m1;
  uint64_t thr_f, thr_c2;
  uint32_t tag, strm, key0, key1, M;

  uint32_t smp[P];
  Real xf[P], vf[P], xc[P], vc[P];
  Real af[P], ef[P], ac[P], ec[P];  // group increments and compensation terms
  uint32_t cf[P], cc[P];
  Real sum_xi[P], num[P], den[P], lnu[P], uses[P], have[P];
  uint32_t wmin[P];
  uint32_t l0[P], l1[P];  // words carried into the next group of four steps
  uint32_t m;             // fine steps taken in the current coarse block

  __device__ __forceinline__ explicit Lane(const LevelDesc& d)
      : h_f((Real)d.h_f), s_f((Real)d.s_f), h_c((Real)d.h_c), s_c((Real)d.s_c),
        agg_ms2((Real)d.agg_ms2), h_f2((Real)d.h_f2), rsqrt_m((Real)d.rsqrt_m),
        thr_f_m1(d.thr_f_m1), thr_c2_m1(d.thr_c2_m1), thr_f(d.thr_f), thr_c2(d.thr_c2),
        tag(d.tag), strm(d.stream), key0(d.key0), key1(d.key1), M(d.M), m(0) {}

  __device__ __forceinline__ Words block(uint32_t b, int p) const {
    return philox4x32_10(b, smp[p], tag, strm, key0, key1);
  }

  // +1 or -1 from the top bit of the angle word (the sign of the sine branch)
  __device__ __forceinline__ static Real sign_of(uint32_t w) {
    return ((int32_t)w < 0) ? Real(-1) : Real(1);
  }

  __device__ __forceinline__ void reset_block() {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      sum_xi[p] = Real(0); num[p] = Real(0); den[p] = Real(0);
      lnu[p] = Real(0); uses[p] = Real(0); have[p] = Real(0);
      wmin[p] = 0xFFFFFFFFu;
    }
  }

  // Initial condition of every trajectory (shared by fine and coarse path);
  // returns the index of the next block.
  __device__ __forceinline__ uint32_t init(const LevelDesc& d) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const Words w = block(0, p);
      Real nc, ns;
      box_muller(w.w0, w.w1, nc, ns);
      Real x0;
      l0[p] = w.w2;
      l1[p] = w.w3;
      if (d.x0_kind == 0) {
        x0 = (Real)d.x0_a;
      } else if (d.x0_kind == 1) {
        x0 = fma_r<Real>((Real)d.x0_b, nc, (Real)d.x0_a);
      } else {
        x0 = (Real)cosine_icdf(uniform_f64(w.w2));
        const Words w1 = block(1, p);  // words 4, 5 unused
        l0[p] = w1.w2;
        l1[p] = w1.w3;
      }
      const Real v0 = kMaxwell ? ns : sign_of(w.w1);
      xf[p] = x0; vf[p] = v0; xc[p] = x0; vc[p] = v0;
      af[p] = Real(0); ef[p] = Real(0); ac[p] = Real(0); ec[p] = Real(0);
      cf[p] = 0u; cc[p] = 0u;
    }
    reset_block();
    m = 0;
    return d.x0_kind == 2 ? 2u : 1u;
  }

  // The arithmetic below is shared with the time-parallel path, which must
  // round exactly as this loop does.

  // Fine move of trajectory p with velocity v and kick normal xi.
  __device__ __forceinline__ void move_f(int p, Real v, Real xi) {
    if constexpr (kCompensate)
      af[p] = fma_r<Real>(s_f, xi, fma_r<Real>(h_f, v, af[p]));
    else
      xf[p] = fma_r<Real>(s_f, xi, fma_r<Real>(h_f, v, xf[p]));
  }

  // Coarse move of trajectory p with velocity v and coarse kick normal.
  __device__ __forceinline__ void move_c(int p, Real v, Real kick) {
    if constexpr (kCompensate)
      ac[p] = fma_r<Real>(s_c, kick, fma_r<Real>(h_c, v, ac[p]));
    else
      xc[p] = fma_r<Real>(s_c, kick, fma_r<Real>(h_c, v, xc[p]));
  }

  // Coarse-block bookkeeping of one fine step (kick normal xi, decision word
  // wd, collision hit with new velocity normal vnew).  num accumulates, per
  // fine move made with an in-block velocity draw, that draw's normal
  // (-> sum_j n_j nu_j); den accumulates 2u+1 at the u-th further use of a
  // draw (-> sum_j n_j^2).
  __device__ __forceinline__ static void book(Real& sxi, Real& nm, Real& dn, Real& ln, Real& us,
                                              Real& hv, uint32_t& wm, Real xi, uint32_t wd,
                                              bool hit, Real vnew) {
    sxi += xi;
    wm = min(wm, wd);
    if constexpr (kAgg) {
      nm += ln;
      dn = fma_r<Real>(hv, fma_r<Real>(Real(2), us, Real(1)), dn);
      us += hv;
      ln = hit ? vnew : ln;
      us = hit ? Real(0) : us;
      hv = hit ? Real(1) : hv;
    }
  }

  // Coarse kick normal of a block; if the coarse path collides (chit), the
  // last in-block draw becomes its velocity and leaves the kick.
  __device__ __forceinline__ Real kick_of(bool chit, Real sxi, Real nm, Real dn, Real ln,
                                          Real us) const {
    if constexpr (kAgg) {
      const Real nn = chit ? fma_r<Real>(-us, ln, nm) : nm;
      const Real dd = chit ? fma_r<Real>(-us, us, dn) : dn;
      return fma_r<Real>(h_f, nn, s_f * sxi) * rsqrt_r(fma_r<Real>(h_f2, dd, agg_ms2));
    } else {
      return sxi * rsqrt_m;
    }
  }

  // One fine step of trajectory p: decision word wd, Box-Muller words (wa, wb).
  __device__ __forceinline__ void step(int p, uint32_t wd, uint32_t wa, uint32_t wb) {
    Real xi, g;
    box_muller(wa, wb, xi, g);
    Real vnew = kMaxwell ? g : sign_of(wb);
    keep(vnew);  // computed unconditionally: the select below stays branch-free
    move_f(p, vf[p], xi);
    const bool hit = below<WIDE>(wd, thr_f_m1, thr_f);
    vf[p] = hit ? vnew : vf[p];
    cf[p] += hit ? 1u : 0u;
    if constexpr (kCoarse)
      book(sum_xi[p], num[p], den[p], lnu[p], uses[p], have[p], wmin[p], xi, wd, hit, vnew);
  }

  // Coarse step of every trajectory at the end of a block of M fine steps.
  __device__ __forceinline__ void coarse() {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      // coarse collision: the smallest fine decision word is below thr_c2
      const bool chit = below<WIDE>(wmin[p], thr_c2_m1, thr_c2);
      move_c(p, vc[p], kick_of(chit, sum_xi[p], num[p], den[p], lnu[p], uses[p]));
      vc[p] = chit ? vf[p] : vc[p];
      cc[p] += chit ? 1u : 0u;
    }
    reset_block();
  }

  // x + a as the pair (t, e + ((x - t) + a)) with t = x + a (Fast2Sum: exact
  // when |x| >= |a|; otherwise wrong by at most a rounding of a).
  __device__ __forceinline__ static void fold(Real& x, Real& e, Real& a) {
    const Real t = x + a;
    e += (x - t) + a;
    x = t;
    a = Real(0);
  }

  __device__ __forceinline__ void fold_all() {
    if constexpr (kCompensate) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        fold(xf[p], ef[p], af[p]);
        if constexpr (kCoarse) fold(xc[p], ec[p], ac[p]);
      }
    }
  }

  // Final positions (after run()).
  __device__ __forceinline__ Real pos_f(int p) const {
    return kCompensate ? xf[p] + ef[p] : xf[p];
  }
  __device__ __forceinline__ Real pos_c(int p) const {
    return kCompensate ? xc[p] + ec[p] : xc[p];
  }

  // After a fine step: the coarse step when a block of M fine steps is
  // complete.  MS = 2 or 4 (M divides 4, so blocks align with groups of four
  // steps and the positions are static); MS = 0: M read at run time.
  template <int MS>
  __device__ __forceinline__ void end_step(int k) {
    if constexpr (kCoarse) {
      if constexpr (MS != 0) {
        if ((k + 1) % MS == 0) coarse();
      } else {
        if (++m == M) {  // wave-uniform
          coarse();
          m = 0;
        }
      }
    }
  }

  // Four fine steps from blocks b, b+1, b+2.
  template <int MS>
  __device__ __forceinline__ void group4(uint32_t b) {
    Words w[P];
    uint32_t t[P];
#pragma unroll
    for (int p = 0; p < P; ++p) w[p] = block(b, p);
#pragma unroll
    for (int p = 0; p < P; ++p) step(p, l0[p], l1[p], w[p].w0);
    end_step<MS>(0);
#pragma unroll
    for (int p = 0; p < P; ++p) step(p, w[p].w1, w[p].w2, w[p].w3);
    end_step<MS>(1);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      w[p] = block(b + 1, p);
      step(p, w[p].w0, w[p].w1, w[p].w2);
      t[p] = w[p].w3;
    }
    end_step<MS>(2);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      w[p] = block(b + 2, p);
      step(p, t[p], w[p].w0, w[p].w1);
      l0[p] = w[p].w2;
      l1[p] = w[p].w3;
    }
    end_step<MS>(3);
  }

  // The first `count` (1..3) steps of a group (coarse positions at run time).
  __device__ __forceinline__ void group_tail(uint32_t b, uint32_t count) {
    Words w[P];
#pragma unroll
    for (int p = 0; p < P; ++p) w[p] = block(b, p);
#pragma unroll
    for (int p = 0; p < P; ++p) step(p, l0[p], l1[p], w[p].w0);
    end_step<0>(0);
    if (count > 1) {
#pragma unroll
      for (int p = 0; p < P; ++p) step(p, w[p].w1, w[p].w2, w[p].w3);
      end_step<0>(1);
    }
    if (count > 2) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        w[p] = block(b + 1, p);
        step(p, w[p].w0, w[p].w1, w[p].w2);
      }
      end_step<0>(2);
    }
  }

  __device__ __forceinline__ void run(const LevelDesc& d) {
    uint32_t b = init(d);
    const uint32_t n_steps = d.n_steps;
    uint32_t n = 0;
    // increments are folded into the positions every 16 steps and at the end
    if (!kCoarse || M == 2) {
#pragma unroll 1
      for (; n + 4 <= n_steps; n += 4, b += 3) {
        group4<2>(b);
        if ((n & 12) == 12) fold_all();
      }
    } else if (M == 4) {
#pragma unroll 1
      for (; n + 4 <= n_steps; n += 4, b += 3) {
        group4<4>(b);
        if ((n & 12) == 12) fold_all();
      }
    } else {
#pragma unroll 1
      for (; n + 4 <= n_steps; n += 4, b += 3) {
        group4<0>(b);
        if ((n & 12) == 12) fold_all();
      }
    }
    // blocks of M in {2, 4} end on group boundaries, so the run-time
    // counter starts the tail at zero
    if (n < n_steps) group_tail(b, n_steps - n);
    fold_all();
  }
};

// Shifted sums of one tile's samples (shift = the values of the tile's first
// sample, held by lane 0) and the tile record they give.  The per-lane loop
// and the time-parallel path build their records with this same code, so
// both give bitwise identical records for the same samples.
struct TileSums {
  double k_dq = 0.0, k_f = 0.0, k_c = 0.0;
  double s1_dq = 0.0, s2_dq = 0.0, s1_f = 0.0, s2_f = 0.0, s1_c = 0.0, s2_c = 0.0, s_fc = 0.0;
  uint32_t cnt = 0;
  unsigned long long col_f = 0, col_c = 0;

  template <bool kCoarse>
  __device__ __forceinline__ void shift(double dq, double qf, double qc) {
    k_dq = __shfl(dq, 0, kLanes);
    if constexpr (kCoarse) {
      k_f = __shfl(qf, 0, kLanes);
      k_c = __shfl(qc, 0, kLanes);
    }
  }

  template <bool kCoarse>
  __device__ __forceinline__ void add(double dq, double qf, double qc, uint32_t cf, uint32_t cc) {
    const double e_dq = dq - k_dq;
    s1_dq += e_dq;
    s2_dq = fma(e_dq, e_dq, s2_dq);
    if constexpr (kCoarse) {
      const double e_f = qf - k_f, e_c = qc - k_c;
      s1_f += e_f; s2_f = fma(e_f, e_f, s2_f);
      s1_c += e_c; s2_c = fma(e_c, e_c, s2_c);
      s_fc = fma(e_f, e_c, s_fc);
    }
    cnt += 1u;
    col_f += cf;
    col_c += cc;
  }

  // Fixed xor-butterfly sums over the wavefront; every lane gets the record.
  template <bool kCoarse>
  __device__ __forceinline__ Stats record() const {
    const double n = (double)wave_sum_u64((unsigned long long)cnt);
    const double t1_dq = wave_sum(s1_dq), t2_dq = wave_sum(s2_dq);
    Stats out;
    out.n = n;
    out.mean_dq = k_dq + t1_dq / n;
    out.m2_dq = fmax(fma(-t1_dq, t1_dq / n, t2_dq), 0.0);
    if constexpr (kCoarse) {
      const double t1_f = wave_sum(s1_f), t2_f = wave_sum(s2_f);
      const double t1_c = wave_sum(s1_c), t2_c = wave_sum(s2_c), t_fc = wave_sum(s_fc);
      out.mean_qf = k_f + t1_f / n;
      out.m2_qf = fmax(fma(-t1_f, t1_f / n, t2_f), 0.0);
      out.mean_qc = k_c + t1_c / n;
      out.m2_qc = fmax(fma(-t1_c, t1_c / n, t2_c), 0.0);
      out.c_fc = fma(-t1_f, t1_c / n, t_fc);
    } else {
      out.mean_qf = out.mean_dq;
      out.m2_qf = out.m2_dq;
      out.mean_qc = 0.0;
      out.m2_qc = 0.0;
      out.c_fc = 0.0;
    }
    out.coll_f = wave_sum_u64(col_f);
    out.coll_c = wave_sum_u64(col_c);
    return out;
  }
};

// Optional per-sample outputs of one valid sample: trajectory and collision
// dumps, histogram counters (fine bin, coarse bin, both in the same bin).
template <typename Real, bool kCoarse>
__device__ __forceinline__ void sample_outputs(const LevelDesc& d, uint64_t local, Real xf, Real xc,
                                               uint32_t cf, uint32_t cc) {
  if (d.traj) {
    Real* t = (Real*)d.traj;
    t[local] = xf;
    t[d.n_samples + local] = kCoarse ? xc : Real(0);
  }
  if (d.coll) {
    d.coll[local] = cf;
    d.coll[d.n_samples + local] = cc;
  }
  if (d.flags & kFlagHist) {
    const int nb = (int)d.nbins;
    const double tf = ((double)xf - d.hist_lo) * d.hist_inv_w;
    const int bf = tf < 0.0 ? -1 : (tf >= (double)nb ? nb : (int)tf);
    unsigned long long* hst = d.hist;
    if (bf < 0) atomicAdd(&hst[3 * nb + 0], 1ull);
    else if (bf >= nb) atomicAdd(&hst[3 * nb + 1], 1ull);
    else atomicAdd(&hst[3 * bf], 1ull);
    if (kCoarse) {
      const double tc = ((double)xc - d.hist_lo) * d.hist_inv_w;
      const int bc = tc < 0.0 ? -1 : (tc >= (double)nb ? nb : (int)tc);
      if (bc < 0) atomicAdd(&hst[3 * nb + 2], 1ull);
      else if (bc >= nb) atomicAdd(&hst[3 * nb + 3], 1ull);
      else {
        atomicAdd(&hst[3 * bc + 1], 1ull);
        if (bc == bf) atomicAdd(&hst[3 * bc + 2], 1ull);
      }
    }
  }
}

template <typename Real, int P, int KIND, bool WIDE>
__device__ __forceinline__ void run_tile_impl(const LevelDesc& d, uint32_t tile,
                                              Stats* __restrict__ partials) {
  using S = Lane<Real, P, KIND, WIDE>;
  constexpr bool kCoarse = S::kCoarse;
  const int lane = threadIdx.x & (kLanes - 1);
  const int rounds = (int)d.spl / P;
  const uint64_t tile_samples = (uint64_t)kLanes * d.spl;
  TileSums acc;

#pragma unroll 1
  for (int r = 0; r < rounds; ++r) {
    S st(d);
    uint64_t local[P];
    bool valid[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int j = r * P + p;
      local[p] = (uint64_t)tile * tile_samples + (uint64_t)(j * kLanes + lane);
      valid[p] = local[p] < d.n_samples;
      st.smp[p] = (uint32_t)(d.sample_begin + local[p]);
    }
    st.run(d);
    // Quantity of interest in FP64 (exact squares of FP32 positions).
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const Real xf = st.pos_f(p), xc = st.pos_c(p);
      const bool qoi_x = (d.flags & kFlagQoiX) != 0;
      const double qf = qoi_x ? (double)xf : (double)xf * (double)xf;
      const double qc = kCoarse ? (qoi_x ? (double)xc : (double)xc * (double)xc) : 0.0;
      const double dq = qf - qc;
      if (r == 0 && p == 0) acc.shift<kCoarse>(dq, qf, qc);  // lane 0, sample 0 always exists
      if (valid[p]) {
        acc.add<kCoarse>(dq, qf, qc, st.cf[p], st.cc[p]);
        if (d.flags & kFlagSampleOutputs)  // one test on the common path
          sample_outputs<Real, kCoarse>(d, local[p], xf, xc, st.cf[p], st.cc[p]);
      }
    }
  }
  const Stats out = acc.record<kCoarse>();
  if (lane == 0) partials[d.tile_base + tile] = out;
}

// One tile of a kinetic-diffusion item: lane i simulates samples
// tile*64*spl + 64 j + i, j < spl, with the same record arithmetic as above.
template <bool kCoarse>
__device__ __forceinline__ void run_kd_tile(const LevelDesc& d, uint32_t tile,
                                            Stats* __restrict__ partials) {
  const int lane = threadIdx.x & (kLanes - 1);
  const uint64_t tile_samples = (uint64_t)kLanes * d.spl;
  TileSums acc;
#pragma unroll 1
  for (uint32_t j = 0; j < d.spl; ++j) {
    const uint64_t local = (uint64_t)tile * tile_samples + (uint64_t)(j * kLanes + lane);
    const bool valid = local < d.n_samples;
    double xf = 0.0, xc = 0.0;
    uint32_t cf = 0, cc = 0;
    if (valid) {
      const uint32_t smp = (uint32_t)(d.sample_begin + local);
      if (d.flags & (kFlagBgB1 | kFlagBgB2)) kd_sample_bg<kCoarse>(d, smp, xf, xc, cf, cc);
      else kd_sample<kCoarse>(d, smp, xf, xc, cf, cc);
    }
    const bool qoi_x = (d.flags & kFlagQoiX) != 0;
    const double qf = qoi_x ? xf : xf * xf;
    const double qc = kCoarse ? (qoi_x ? xc : xc * xc) : 0.0;
    const double dq = qf - qc;
    if (j == 0) acc.shift<kCoarse>(dq, qf, qc);  // lane 0, sample 0 always exists
    if (valid) {
      acc.add<kCoarse>(dq, qf, qc, cf, cc);
      if (d.flags & kFlagSampleOutputs) sample_outputs<double, kCoarse>(d, local, xf, xc, cf, cc);
    }
  }
  const Stats out = acc.record<kCoarse>();
  if (lane == 0) partials[d.tile_base + tile] = out;
}

__device__ __forceinline__ void run_kd_unit(const LevelDesc& d, uint32_t unit,
                                            Stats* __restrict__ partials) {
  if (d.kind == kKindKdPair) run_kd_tile<true>(d, unit, partials);
  else run_kd_tile<false>(d, unit, partials);
}

// ---------------------------------------------------------------------------
// Time-parallel trajectory, for items of few long trajectories (the warm-up
// of the fine levels), where one trajectory per lane would leave most of the
// GPU idle while a few wavefronts walk thousands of steps.  A wavefront
// simulates one sample; in chunk c, lane j owns fine step 64 c + j.  What
// does not depend on the particle state is computed by the lanes in
// parallel: the chunk's Philox blocks (lane i computes block i; the words go
// through LDS), the Box-Muller pairs and collision decisions, the velocity
// each step moves with (the draw of the last colliding step before it: a
// ballot and a shuffle), and for a pair every coarse block's collision, kick
// and velocity.  The position increments are then summed in step order on
// wave-uniform values with the very operations of the per-lane loop
// (including the compensated folds), so both give bitwise identical results.
// Needs n_steps >= 1 and, for a pair, M in {2, 4} (coarse blocks inside a
// chunk).  Writes the sample's final state to d.tp_out; the tile records are
// built from there by the reduction.
// ---------------------------------------------------------------------------
constexpr int kTpBlocks = 49;                 // Philox blocks per 64-step chunk
constexpr int kTpWords = 4 * kTpBlocks;       // 196 words; step j reads words 3j+2..3j+4
constexpr int kTpWavesPerBlock = 4;           // kernels here run <= 256 threads
// A KD window whose guessed collision-time chain holds for fewer steps than
// this walks the chain serially instead.
constexpr uint32_t kTpMinGuessed = 16;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float lane_value(float v, uint32_t j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)j));
}
__device__ __forceinline__ double lane_value(double v, uint32_t j) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, (int)j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), (int)j);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Word exchange area of the time-parallel path (one row per wavefront).
__shared__ uint32_t tp_words[kTpWavesPerBlock][kTpWords];

// Step j of a chunk in the serial order of the per-lane loop: fine move,
// coarse move at the end of a coarse block, compensated fold every 16 steps.
template <int MS, typename S, typename Real>
__device__ __forceinline__ void tp_serial_step(S& st, uint32_t j, Real vpre, Real xi, Real vcpre,
                                               Real kick) {
  st.move_f(0, lane_value(vpre, j), lane_value(xi, j));
  if constexpr (S::kCoarse) {
    if ((j & (uint32_t)(MS - 1)) == (uint32_t)(MS - 1))
      st.move_c(0, lane_value(vcpre, j), lane_value(kick, j));
  }
  if ((j & 15u) == 15u) st.fold_all();
}

template <typename Real, int KIND, bool WIDE, int MS>
__device__ __forceinline__ void run_tp(const LevelDesc& d, uint32_t local) {
  using S = Lane<Real, 1, KIND, WIDE>;
  constexpr bool kCoarse = S::kCoarse;
  uint32_t* wl = tp_words[threadIdx.x / kLanes];
  const uint32_t lane = threadIdx.x & (kLanes - 1);
  const unsigned long long lanes_below = (1ull << lane) - 1ull;

  S st(d);
  st.smp[0] = (uint32_t)(d.sample_begin + local);
  const uint32_t first_block = st.init(d) - 1u;  // block of the two carried words
  const uint32_t n = d.n_steps;
  Real vf = st.vf[0], vc = st.vc[0];
  uint32_t cf = 0, cc = 0;

#pragma unroll 1
  for (uint32_t c0 = 0; c0 < n; c0 += kLanes) {
    // words 2 + 3 (c0 + j) .. 4 + 3 (c0 + j) of the stream, from block
    // first_block + 48 (c0 / 64) on (every chunk starts at word 2 of a block)
    wave_sync();
    if (lane < (uint32_t)kTpBlocks) {
      const Words w = st.block(first_block + (c0 / kLanes) * 48u + lane, 0);
      wl[4 * lane + 0] = w.w0;
      wl[4 * lane + 1] = w.w1;
      wl[4 * lane + 2] = w.w2;
      wl[4 * lane + 3] = w.w3;
    }
    wave_sync();
    const uint32_t wd = wl[3 * lane + 2], wa = wl[3 * lane + 3], wb = wl[3 * lane + 4];
    const bool active = c0 + lane < n;
    Real xi, g;
    box_muller(wa, wb, xi, g);
    Real vnew = S::kMaxwell ? g : S::sign_of(wb);
    const bool hit = active && below<WIDE>(wd, st.thr_f_m1, st.thr_f);
    const unsigned long long mask = __ballot(hit);
    const unsigned long long before = mask & lanes_below;
    const int src = before ? 63 - __clzll((long long)before) : (int)lane;
    const Real v_last = __shfl(vnew, src, kLanes);
    const Real vpre = before ? v_last : vf;     // velocity of this step's move
    const Real vpost = hit ? vnew : vpre;       // velocity after its collision

    Real kick = Real(0), vcpre = Real(0);
    unsigned long long cmask = 0;
    if constexpr (kCoarse) {
      // the coarse block of this lane: steps lb .. lb + MS - 1 of the chunk,
      // its bookkeeping replayed in step order exactly as the per-lane loop
      const int lb = (int)(lane & ~(uint32_t)(MS - 1));
      Real sum_xi = Real(0), num = Real(0), den = Real(0), lnu = Real(0), uses = Real(0),
           have = Real(0);
      uint32_t wmin = 0xFFFFFFFFu;
#pragma unroll
      for (int i = 0; i < MS; ++i) {
        const Real xi_i = __shfl(xi, lb + i, kLanes);
        const uint32_t wd_i = (uint32_t)__shfl((int)wd, lb + i, kLanes);
        const Real vn_i = __shfl(vnew, lb + i, kLanes);
        const bool hit_i = (mask >> (lb + i)) & 1ull;
        S::book(sum_xi, num, den, lnu, uses, have, wmin, xi_i, wd_i, hit_i, vn_i);
      }
      const bool chit = below<WIDE>(wmin, st.thr_c2_m1, st.thr_c2);
      kick = st.kick_of(chit, sum_xi, num, den, lnu, uses);
      const bool last = (lane & (uint32_t)(MS - 1)) == (uint32_t)(MS - 1);
      cmask = __ballot(last && active && chit);
      const unsigned long long cbefore = cmask & lanes_below;
      const int csrc = cbefore ? 63 - __clzll((long long)cbefore) : (int)lane;
      const Real vc_last = __shfl(vpost, csrc, kLanes);
      vcpre = cbefore ? vc_last : vc;
    }

    // position increments in step order (wave-uniform values); a full chunk
    // is unrolled so that the lane reads run ahead of the dependent chain
    const uint32_t cnt = min((uint32_t)kLanes, n - c0);
    if (cnt == (uint32_t)kLanes) {
#pragma unroll
      for (uint32_t j = 0; j < (uint32_t)kLanes; ++j) tp_serial_step<MS>(st, j, vpre, xi, vcpre, kick);
    } else {
#pragma unroll 1
      for (uint32_t j = 0; j < cnt; ++j) tp_serial_step<MS>(st, j, vpre, xi, vcpre, kick);
    }
    cf += (uint32_t)__popcll(mask);
    if (mask) vf = lane_value(vnew, 63u - (uint32_t)__clzll((long long)mask));
    if constexpr (kCoarse) {
      cc += (uint32_t)__popcll(cmask);
      if (cmask) vc = lane_value(vpost, 63u - (uint32_t)__clzll((long long)cmask));
    }
  }
  st.fold_all();
  const Real xf = st.pos_f(0), xc = st.pos_c(0);
  if (lane == 0) {
    TpSample r;
    r.xf = (double)xf;
    r.xc = kCoarse ? (double)xc : 0.0;
    r.cf = cf;
    r.cc = cc;
    d.tp_out[local] = r;
    if (d.flags & kFlagSampleOutputs) sample_outputs<Real, kCoarse>(d, local, xf, xc, cf, cc);
  }
}

// Tile record of a time-parallel item from its samples' final states: the
// same arithmetic as run_tile_impl on a 64-sample tile.
template <bool kCoarse>
__device__ __forceinline__ Stats tp_tile_record(const LevelDesc& d, uint32_t tile) {
  const uint32_t lane = threadIdx.x & (kLanes - 1);
  const uint64_t local = (uint64_t)tile * kLanes + lane;
  const bool valid = local < d.n_samples;
  TpSample r{0.0, 0.0, 0u, 0u};
  if (valid) r = d.tp_out[local];
  const bool qoi_x = (d.flags & kFlagQoiX) != 0;
  const double qf = qoi_x ? r.xf : r.xf * r.xf;
  const double qc = kCoarse ? (qoi_x ? r.xc : r.xc * r.xc) : 0.0;
  const double dq = qf - qc;
  TileSums acc;
  acc.shift<kCoarse>(dq, qf, qc);
  if (valid) acc.add<kCoarse>(dq, qf, qc, r.cf, r.cc);
  return acc.record<kCoarse>();
}

// ---------------------------------------------------------------------------
// Time-parallel KD path or pair in a homogeneous background, for items of few
// long paths (the warm-up of the fine levels).  A wavefront simulates one
// sample, in windows of up to 64 fine KD steps.  With a constant collision
// rate the only serial dependence between KD steps is the chain of collision
// times (c_{k+1} = end of the grid step holding c_k, plus the next flight
// E_{k+1}/R) and, for a pair, the coarse steps that chain delimits; a step's
// position increment, its coefficients of eqs. advection and diffusion and
// its aggregation weights depend only on its diffusive length theta and on
// random numbers.  Per window: (A) lane j draws the numbers of step j; (B)
// the chain is taken across the lanes (each lane guesses where its
// predecessor's step ended and checks the guess; a window whose guesses fail
// early walks the chain serially), lane j keeping theta of step j, and the
// coarse steps follow block by block (where step j ends a coarse step, lane j
// keeps that coarse step's theta and flight increment); (C) every lane
// evaluates its step; (D) the position increments are added in step order on
// wave-uniform values, each coarse block's aggregation sums by the lane where
// the block ends, in step order.  Every
// quantity is computed with the operations of the per-lane loop
// (kd_sample_rec) on the same inputs, and the sums are taken in its order, so
// both forms give bitwise identical paths.
// ---------------------------------------------------------------------------
template <bool COARSE>
__device__ __forceinline__ void run_kd_tp(const LevelDesc& d, uint32_t local) {
  const KdParams k = kd_params(d);
  const uint32_t lane = threadIdx.x & (kLanes - 1);
  const uint32_t smp = (uint32_t)(d.sample_begin + local);
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
  double xc = x0, vc = vf, tc = 0.0, ccoarse = cfine;
  double nu_f = ns;                          // velocity number of the pending flight
  double nf = kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0;    // pair: grid end of the pending flight's step
  double end_c = 0.0, end_c_fine = 0.0, num = 0.0, den = 0.0, zeta_prev = 0.0;
  bool in_inner = false, done = false;

#pragma unroll 1
  while (!done) {
    // (A) the numbers of the window's steps: lane j takes Philox block b + j
    double nu_next, chi, E_next;
    kd_draws(k, smp, b + lane, nu_next, chi, E_next);
    // inputs of the window's first step that come from the step before it
    const double tauf0 = tauf, vf0 = vf, nu_f0 = nu_f, zeta0 = zeta_prev;

    // (B) the collision-time chain and the coarse steps.  Lane j takes step
    // j as if every step of the window ended on the grid point after the one
    // before it (a flight shorter than a grid step, the rule at these rates):
    // it rebuilds the pending collision from that grid point and its
    // predecessor's flight number, then finds its own step's grid end.  The
    // first lane whose grid end differs from the assumed one closes the
    // window: its step is exact, the steps after it started from the wrong
    // grid point and are taken again by the next window.  The coarse steps
    // then go block by block on wave-uniform values, a ballot finding where
    // each block of fine steps ends.  Every value comes from the operations
    // of the per-lane loop on the same inputs.
    double theta = 0.0, theta_c = 0.0, pc = 0.0;
    uint64_t first_m = 0, exit_m = 0, upd_m = 0;
    uint32_t cnt = 0;
    {
      const double n0 = COARSE ? nf : kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0;
      const double E_up = __shfl(E_next, (int)(lane == 0 ? 0u : lane - 1u), kLanes);
      const double n_j = n0 + (double)lane;  // assumed grid end of step j
      const double c_l = lane == 0 ? cfine : (n_j - 1.0) * k.dtf + E_up * k.inv_r;
      const double n_true = kd_grid_floor(c_l, k.dtf, k.inv_dtf, k.pow2_f) + 1.0;
      const double t_next_l = n_true * k.dtf;
      const double th_l = t_next_l - c_l;
      const double cn_l = t_next_l + E_next * k.inv_r;  // pending collision after step j
      const unsigned long long wrong = __ballot(!(n_true == n_j));
      const uint32_t lim = wrong ? (uint32_t)__builtin_ctzll(wrong) + 1u : (uint32_t)kLanes;
      double nn_l = 0.0;
      if (lim < kTpMinGuessed) {
        // flights longer than a grid step are common here (a low collision
        // rate): the window walks the chain step by step instead
#pragma unroll 1
        for (uint32_t j = 0; j < (uint32_t)kLanes; ++j) {
          double th;
          if constexpr (!COARSE) {
            if (!(cfine < k.T && cf < k.guard)) {
              done = true;
              break;
            }
            const double t_next = (kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0) * k.dtf;
            th = t_next - cfine;
            tf = t_next;
            tauf = lane_value(E_next, j) * k.inv_r;
            cfine = tf + tauf;
          } else {
            if (!in_inner) {  // head of the per-lane loop's outer iteration
              if (!((ccoarse < k.T || cfine < k.T) && cf < k.guard)) {
                done = true;
                break;
              }
              end_c = kd_grid_floor(ccoarse, k.dtc, k.inv_dtc, k.pow2_c) + 1.0;
              end_c_fine = end_c * (double)k.M;
              first_m |= 1ull << j;
              in_inner = true;
            }
            const double t_next = nf * k.dtf;
            th = t_next - cfine;
            tf = t_next;
            tauf = lane_value(E_next, j) * k.inv_r;
            cfine = tf + tauf;
            nf = kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0;
          }
          theta = lane == j ? th : theta;
          ++cf;
          ++cnt;
          if constexpr (COARSE) {
            if (!(!(nf > end_c_fine) && cf < k.guard)) {  // the inner loop ends after step j
              in_inner = false;
              exit_m |= 1ull << j;
              if (ccoarse < k.T) {
                const double t_next_c = end_c * k.dtc;
                const double thc = t_next_c - ccoarse;
                const double p_c = vc * (ccoarse - tc);
                theta_c = lane == j ? thc : theta_c;
                pc = lane == j ? p_c : pc;
                tc = t_next_c;
                ccoarse = cfine;
                vc = k.mu + k.sigma * lane_value(nu_next, j);
                ++cc;
                upd_m |= 1ull << j;
              }
            }
          }
        }
      } else if constexpr (!COARSE) {
        const unsigned long long stop = __ballot(!(c_l < k.T && cf + lane < k.guard));
        const uint32_t at = stop ? (uint32_t)__builtin_ctzll(stop) : (uint32_t)kLanes;
        cnt = min(at, lim);
        done = at < lim;
      } else {
        nn_l = kd_grid_floor(cn_l, k.dtf, k.inv_dtf, k.pow2_f) + 1.0;  // nf after step j
        cnt = lim;
        uint32_t j = 0;
#pragma unroll 1
        while (j < lim) {
          if (!in_inner) {  // head of the per-lane loop's outer iteration
            const double c_h = lane_value(c_l, j);
            if (!((ccoarse < k.T || c_h < k.T) && cf + j < k.guard)) {
              done = true;
              cnt = j;
              break;
            }
            end_c = kd_grid_floor(ccoarse, k.dtc, k.inv_dtc, k.pow2_c) + 1.0;
            end_c_fine = end_c * (double)k.M;
            first_m |= 1ull << j;
            in_inner = true;
          }
          // the inner loop ends after the first step x >= j whose next grid
          // end passes the coarse step
          const unsigned long long ends =
              __ballot(lane >= j && lane < lim &&
                       !(!(nn_l > end_c_fine) && cf + lane + 1u < k.guard));
          if (!ends) break;  // the block runs on past the window's exact steps
          const uint32_t x = (uint32_t)__builtin_ctzll(ends);
          in_inner = false;
          exit_m |= 1ull << x;
          if (ccoarse < k.T) {
            const double t_next_c = end_c * k.dtc;
            const double thc = t_next_c - ccoarse;
            const double p_c = vc * (ccoarse - tc);
            theta_c = lane == x ? thc : theta_c;
            pc = lane == x ? p_c : pc;
            tc = t_next_c;
            ccoarse = lane_value(cn_l, x);
            vc = k.mu + k.sigma * lane_value(nu_next, x);
            ++cc;
            upd_m |= 1ull << x;
          }
          j = x + 1u;
        }
      }
      if (lim >= kTpMinGuessed) {
        theta = lane < cnt ? th_l : 0.0;
        if (cnt > 0) {
          const uint32_t last = cnt - 1u;
          tf = lane_value(t_next_l, last);
          tauf = lane_value(E_next, last) * k.inv_r;
          cfine = lane_value(cn_l, last);
          if constexpr (COARSE) nf = lane_value(nn_l, last);
          cf += cnt;
        }
      }
    }
    if (cnt == 0) break;

    // (C) each lane's step: flight and diffusive increments, weights
    const uint32_t up = lane == 0 ? 0u : lane - 1u;
    const double E_up = __shfl(E_next, (int)up, kLanes);
    const double nu_up = __shfl(nu_next, (int)up, kLanes);
    const double tauf_j = lane == 0 ? tauf0 : E_up * k.inv_r;
    const double vf_j = lane == 0 ? vf0 : k.mu + k.sigma * nu_up;
    const double y = k.R * theta;
    const double em = kd_em(y);
    const double v_next = k.mu + k.sigma * nu_next;
    double a, dd;
    kd_coeffs(k, theta, y, em, v_next, a, dd);
    const double p = vf_j * tauf_j;
    const double q = a + dd * chi;
    double A1 = 0.0, A2 = 0.0, B1 = 0.0, B2 = 0.0, ac = 0.0, ddc = 0.0;
    if constexpr (COARSE) {
      const double nu_f_j = lane == 0 ? nu_f0 : nu_up;
      const double zeta = -em * k.inv_r;
      const double yp = kd_h(y, em);
      const double beta = sqrt(k.c2 * kd_h(yp, yp < kKdSeriesY ? 0.0 : kd_em(yp)));
      const double zeta_up = __shfl(zeta, (int)up, kLanes);
      const double alpha = (tauf_j + (lane == 0 ? zeta0 : zeta_up)) * k.sigma;
      A1 = alpha * nu_f_j;
      A2 = alpha * alpha;
      B1 = beta * chi;
      B2 = beta * beta;
      zeta_prev = lane_value(zeta, cnt - 1u);
      // coarse coefficients, kept by the lanes whose step ends a coarse step
      const double yc = k.R * theta_c;
      kd_coeffs(k, theta_c, yc, kd_em(yc), v_next, ac, ddc);
    }

    // (D) the sums in step order.  The position increments form one serial
    // chain (a full window unrolled, so that the lane reads run ahead of
    // it).  The sums of a coarse block are taken by the lane of the block's
    // last step in the window, over the block's steps in order, starting
    // from zero at the block's head or from the sums carried into the window;
    // the lanes where a block ends keep them, and the coarse moves follow the
    // pass, their divisions and square roots taken across the lanes.
    if (cnt == (uint32_t)kLanes) {
#pragma unroll
      for (uint32_t j = 0; j < (uint32_t)kLanes; ++j) xf = xf + lane_value(p, j) + lane_value(q, j);
    } else {
#pragma unroll 1
      for (uint32_t j = 0; j < cnt; ++j) xf = xf + lane_value(p, j) + lane_value(q, j);
    }
    double num_j = 0.0, den_j = 0.0;
    if constexpr (COARSE) {
      const unsigned long long upto = lane == 63u ? ~0ull : (2ull << lane) - 1ull;  // lanes <= this one
      const unsigned long long heads = first_m & upto;
      const bool carried = heads == 0;
      const uint32_t h = carried ? 0u : 63u - (uint32_t)__clzll((long long)heads);
      const uint32_t len = lane < cnt ? lane + 1u - h : 0u;
      uint32_t longest = len;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) longest = max(longest, (uint32_t)__shfl_xor((int)longest, o, kLanes));
      longest = __builtin_amdgcn_readfirstlane(longest);
      double s1 = carried ? num : 0.0, s2 = carried ? den : 0.0;
#pragma unroll 1
      for (uint32_t o = 0; o < longest; ++o) {
        const int j = (int)min(h + o, (uint32_t)kLanes - 1u);
        const double a1 = __shfl(A1, j, kLanes), a2 = __shfl(A2, j, kLanes);
        const double b1 = __shfl(B1, j, kLanes), b2 = __shfl(B2, j, kLanes);
        if (o < len) {
          if (carried || o > 0) {  // every step of the block but its head
            s1 += a1;
            s2 += a2;
          }
          s1 += b1;
          s2 += b2;
        }
      }
      num_j = s1;
      den_j = s2;
      if (cnt > 0) {
        const bool runs_on = !((exit_m >> (cnt - 1u)) & 1ull);
        num = runs_on ? lane_value(s1, cnt - 1u) : 0.0;
        den = runs_on ? lane_value(s2, cnt - 1u) : 0.0;
      }
    }
    if constexpr (COARSE) {
      const double chi_c = den_j > 0.0 ? num_j / sqrt(den_j) : 0.0;
      const double inc = ac + ddc * chi_c;
#pragma unroll 1
      for (uint64_t m = upd_m; m != 0; m &= m - 1ull) {
        const uint32_t j = (uint32_t)__builtin_ctzll(m);
        xc = xc + lane_value(pc, j) + lane_value(inc, j);
      }
    }
    const double nu_last = lane_value(nu_next, cnt - 1u);
    nu_f = nu_last;
    vf = k.mu + k.sigma * nu_last;
    b += cnt;
  }
  if (tf < k.T) xf = xf + vf * (k.T - tf);
  if constexpr (COARSE) {
    if (tc < k.T) xc = xc + vc * (k.T - tc);
  }
  const double xco = COARSE ? xc : 0.0;
  const uint32_t cco = COARSE ? cc : 0u;
  if (lane == 0) {
    TpSample r;
    r.xf = xf;
    r.xc = xco;
    r.cf = cf;
    r.cc = cco;
    d.tp_out[local] = r;
    if (d.flags & kFlagSampleOutputs) sample_outputs<double, COARSE>(d, local, xf, xco, cf, cco);
  }
}

// ---------------------------------------------------------------------------
// Time-parallel KD path or pair in a background of Section 5 (kFlagBgB1 /
// kFlagBgB2), for items of few long paths.  A flight's length depends on
// where it starts and a diffusive phase on the rate at its collision, so the
// fine path's state (position, velocity, pending collision) is a serial
// chain; the rest runs across the lanes.  A wavefront simulates one sample
// in windows of up to 64 fine KD steps:
//   (A) lane j draws the numbers of the window's step j;
//   (B) the fine chain is walked on wave-uniform values; lane j keeps step
//       j's diffusive exponent y = R theta, its local rate and its end state;
//   (C) pair: every lane evaluates the aggregation weights of its step
//       (zeta, beta, alpha of eqs. chi-update and weights-beta);
//   (D) pair: the steps are walked again in order on wave-uniform values:
//       the fine steps that make up each coarse KD step, the weighted sums,
//       and the coarse KD steps themselves (eq. chi-update, the coarse
//       diffusive phase, eq. epsilon-update and the next coarse flight).
// The fine path does not depend on the coarse one, so (B) may run ahead of
// the step where (D) ends the pair; steps that (D) does not take are
// dropped.  Every quantity comes from the operations of the per-lane loop
// (kd_sample_bg_rec) on the same inputs, and sums are taken in its order, so
// the two forms give bitwise identical results.
// ---------------------------------------------------------------------------
template <bool COARSE>
__device__ __forceinline__ void run_kd_bg_tp(const LevelDesc& d, uint32_t local) {
  const KdParams k = kd_params(d);
  const KdBackground g{d.rsqrt_m, d.s_f, (d.flags & kFlagBgB1) != 0};
  const uint32_t guard = 2u * d.n_steps + 4u;
  const uint32_t lane = threadIdx.x & (kLanes - 1);
  const uint32_t smp = (uint32_t)(d.sample_begin + local);
  const Words w0 = philox4x32_10(0u, smp, k.tag, k.strm, k.key0, k.key1);
  double nc, ns;
  box_muller(w0.w0, w0.w1, nc, ns);
  double x0;
  if (d.x0_kind == 0) x0 = d.x0_a;
  else if (d.x0_kind == 1) x0 = d.x0_a + d.x0_b * nc;
  else x0 = cosine_icdf(uniform_f64(w0.w3));
  const double E0 = -log_unit(uniform_f64(w0.w2));

  // fine path (wave-uniform)
  double xf = x0, vf = k.mu + k.sigma * ns, tf = 0.0, Ef = E0;
  double tauf = bg_flight<true>(g, xf, vf, Ef);
  double cfine = tf + tauf;
  uint32_t cf = 0, b = 1, steps = 0;
  // coarse path and the state of the pair loop (wave-uniform)
  double xc = x0, vc = vf, tc = 0.0, tauc = tauf, ccoarse = tc + tauc;
  double nu_f = ns, zeta_last = 0.0, xf_end = 0.0, end_c_fine = 0.0, end_c = 0.0;
  double num = 0.0, den = 0.0;
  uint32_t cc = 0;
  bool fine_done = false, in_inner = false, first = true, done = false;

#pragma unroll 1
  while (!done) {
    if constexpr (COARSE) {
      if (when<true>(!in_inner && !((ccoarse < k.T || cfine < k.T) && steps < guard))) break;
    }
    // (A)
    double nu_next, chi, E_next;
    kd_draws(k, smp, b + lane, nu_next, chi, E_next);
    const double xf0 = xf, vf0 = vf, tf0 = tf, tauf0 = tauf, cfine0 = cfine, nu_f0 = nu_f;

    // (B)
    double y_j = 0.0, r_j = 1.0, x_j = 0.0, t_j = 0.0, tau_j = 0.0, c_j = 0.0;
    uint32_t cnt = 0;
#pragma unroll 1
    for (uint32_t j = 0; j < (uint32_t)kLanes; ++j) {
      if constexpr (!COARSE) {
        if (when<true>(!(cfine < k.T && steps < guard))) {
          done = true;
          break;
        }
      } else {
        if (steps + cnt >= guard) break;
      }
      const double t_next = (kd_grid_floor(cfine, k.dtf, k.inv_dtf, k.pow2_f) + 1.0) * k.dtf;
      const double theta = t_next - cfine;
      const double rm = bg_rate(g, xf + vf * tauf);
      const double y = rm * theta;
      const double v_next = k.mu + k.sigma * lane_value(nu_next, j);
      double a, dd, inv_r, c2;
      bg_coeffs<true>(rm, k.mu, k.sigma, theta, y, kd_em<true>(y), v_next, a, dd, inv_r, c2);
      xf = xf + vf * tauf + (a + dd * lane_value(chi, j));
      tf = t_next;
      vf = v_next;
      Ef = lane_value(E_next, j);
      tauf = bg_flight<true>(g, xf, vf, Ef);
      cfine = tf + tauf;
      ++cnt;
      if constexpr (!COARSE) {
        ++cf;
        ++steps;
      } else {
        const bool mine = lane == j;
        y_j = mine ? y : y_j;
        r_j = mine ? rm : r_j;
        x_j = mine ? xf : x_j;
        t_j = mine ? tf : t_j;
        tau_j = mine ? tauf : tau_j;
        c_j = mine ? cfine : c_j;
      }
    }
    if constexpr (!COARSE) {
      b += cnt;
      continue;
    }
    if (cnt == 0) break;

    // (C)
    const uint32_t up = lane == 0 ? 0u : lane - 1u;
    const double em_j = kd_em(y_j);
    double inv_r, inv_r2, c2;
    bg_rate_consts(r_j, k.sigma, inv_r, inv_r2, c2);
    const double zeta = -em_j * inv_r;
    const double yp = kd_h(y_j, em_j);
    const double beta = sqrt(c2 * kd_h(yp, yp < kKdSeriesY ? 0.0 : kd_em(yp)));
    const double zeta_up = __shfl(zeta, (int)up, kLanes);
    const double tau_up = __shfl(tau_j, (int)up, kLanes);
    const double nu_up = __shfl(nu_next, (int)up, kLanes);
    const double alpha = ((lane == 0 ? tauf0 : tau_up) + (lane == 0 ? zeta_last : zeta_up)) * k.sigma;
    const double A1 = alpha * (lane == 0 ? nu_f0 : nu_up);
    const double A2 = alpha * alpha;
    const double B1 = beta * chi;
    const double B2 = beta * beta;
    const double nfp = kd_grid_floor(c_j, k.dtf, k.inv_dtf, k.pow2_f) + 1.0;

    // (D)
    uint32_t taken = 0;
#pragma unroll 1
    for (uint32_t j = 0; j < cnt; ++j) {
      const double c_pre = j == 0 ? cfine0 : lane_value(c_j, j - 1u);
      if (when<true>(!in_inner)) {  // head of the per-lane loop's outer iteration
        if (when<true>(!((ccoarse < k.T || c_pre < k.T) && steps < guard))) {
          done = true;
          break;
        }
        end_c = kd_grid_floor(ccoarse, k.dtc, k.inv_dtc, k.pow2_c) + 1.0;
        end_c_fine = end_c * (double)k.M;
        num = 0.0;
        den = 0.0;
        first = true;
        in_inner = true;
      }
      if (when<true>(c_pre >= k.T && !fine_done)) {
        const double x_pre = j == 0 ? xf0 : lane_value(x_j, j - 1u);
        const double t_pre = j == 0 ? tf0 : lane_value(t_j, j - 1u);
        const double v_pre = j == 0 ? vf0 : k.mu + k.sigma * lane_value(nu_next, j - 1u);
        xf_end = t_pre < k.T ? x_pre + v_pre * (k.T - t_pre) : x_pre;
        fine_done = true;
      }
      if (when<true>(!first)) {
        num += lane_value(A1, j);
        den += lane_value(A2, j);
      }
      num += lane_value(B1, j);
      den += lane_value(B2, j);
      first = false;
      if (!fine_done) ++cf;
      ++steps;
      ++taken;
      if (when<true>(!(!(lane_value(nfp, j) > end_c_fine) && steps < guard))) {  // the inner loop ends
        in_inner = false;
        if (when<true>(ccoarse < k.T)) {
          const double nu_e = lane_value(nu_next, j);
          const double xf_e = lane_value(x_j, j), tf_e = lane_value(t_j, j);
          const double vf_e = k.mu + k.sigma * nu_e;
          const double chi_c = den > 0.0 ? num / sqrt(den) : 0.0;
          const double t_next = end_c * k.dtc;
          const double theta = t_next - ccoarse;
          const double rc = bg_rate(g, xc + vc * tauc);
          const double y = rc * theta;
          double a, dd, ir, cq;
          bg_coeffs<true>(rc, k.mu, k.sigma, theta, y, kd_em<true>(y), vf_e, a, dd, ir, cq);
          xc = xc + vc * tauc + (a + dd * chi_c);
          tc = t_next;
          vc = vf_e;
          double ec = lane_value(E_next, j) - bg_rate_integral<true>(g, xf_e, vf_e, tc - tf_e);
          ec = ec < 0.0 ? 0.0 : ec;
          tauc = bg_flight<true>(g, xc, vc, ec);
          ccoarse = tc + tauc;
          ++cc;
        }
      }
    }
    if (done) {
      // the fine state is the end state of the last step taken
      if (taken > 0) {
        xf = lane_value(x_j, taken - 1u);
        tf = lane_value(t_j, taken - 1u);
        vf = k.mu + k.sigma * lane_value(nu_next, taken - 1u);
      } else {
        xf = xf0;
        tf = tf0;
        vf = vf0;
      }
    } else {
      nu_f = lane_value(nu_next, cnt - 1u);
      zeta_last = lane_value(zeta, cnt - 1u);
    }
    b += cnt;
  }
  if constexpr (!COARSE) {
    if (tf < k.T) xf = xf + vf * (k.T - tf);
    xf_end = xf;
  } else {
    if (!fine_done) xf_end = tf < k.T ? xf + vf * (k.T - tf) : xf;
    if (tc < k.T) xc = xc + vc * (k.T - tc);
  }
  const double xco = COARSE ? xc : 0.0;
  const uint32_t cco = COARSE ? cc : 0u;
  if (lane == 0) {
    TpSample r;
    r.xf = xf_end;
    r.xc = xco;
    r.cf = cf;
    r.cc = cco;
    d.tp_out[local] = r;
    if (d.flags & kFlagSampleOutputs) sample_outputs<double, COARSE>(d, local, xf_end, xco, cf, cco);
  }
}

// One tile of an item (per-lane loop).
template <typename Real, int P, int KIND>
__device__ __forceinline__ void run_unit(const LevelDesc& d, uint32_t unit,
                                         Stats* __restrict__ partials) {
  const bool wide = (d.flags & kFlagWide) != 0;
  // one trajectory per lane where a tile holds fewer samples per lane than P
  // (the long levels' 64-sample tiles, and the narrowed tiles of small items)
  constexpr int P1 = 1;
  if (d.spl < (uint32_t)P) {
    if (wide) run_tile_impl<Real, P1, KIND, true>(d, unit, partials);
    else run_tile_impl<Real, P1, KIND, false>(d, unit, partials);
  } else {
    if (wide) run_tile_impl<Real, P, KIND, true>(d, unit, partials);
    else run_tile_impl<Real, P, KIND, false>(d, unit, partials);
  }
}

// ---------------------------------------------------------------------------
// Plain launch: one unit per wavefront over one work item.
// ---------------------------------------------------------------------------
template <typename Real, int P, int KIND>
__global__ void __launch_bounds__(256) level_kernel(const LevelDesc* __restrict__ items,
                                                     uint32_t item, Stats* __restrict__ partials) {
  const LevelDesc d = items[item];
  const uint32_t wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kLanes);
  if (wave >= d.n_tiles) return;  // the whole wavefront leaves together
  run_unit<Real, P, KIND>(d, wave, partials);
}

// The same for a kinetic-diffusion item.
__global__ void __launch_bounds__(256) kd_level_kernel(const LevelDesc* __restrict__ items,
                                                        uint32_t item, Stats* __restrict__ partials) {
  const LevelDesc d = items[item];
  const uint32_t wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kLanes);
  if (wave >= d.n_tiles) return;
  run_kd_unit(d, wave, partials);
}

// ---------------------------------------------------------------------------
// Time-parallel items of a work table (their chunks are absent from the
// persistent kernel's chunk space).  Wavefront w of the grid takes
// trajectories w, w + W, ... of the table's time-parallel space.
// ---------------------------------------------------------------------------
template <typename Real, int KIND>
__device__ __forceinline__ void run_tp_kind(const LevelDesc& d, uint32_t local) {
  constexpr bool kCoarse = KIND >= kKindPairTwoPointSum;
  const bool wide = (d.flags & kFlagWide) != 0;
  if constexpr (!kCoarse) {
    if (wide) run_tp<Real, KIND, true, 1>(d, local);
    else run_tp<Real, KIND, false, 1>(d, local);
  } else if (d.M == 2) {
    if (wide) run_tp<Real, KIND, true, 2>(d, local);
    else run_tp<Real, KIND, false, 2>(d, local);
  } else {
    if (wide) run_tp<Real, KIND, true, 4>(d, local);
    else run_tp<Real, KIND, false, 4>(d, local);
  }
}

// Item lookups.  Every index space of a work table (chunks, groups,
// time-parallel trajectories) is the concatenation of the items' ranges, so
// the item of position g is the last one whose base is <= g.  Kernels copy
// the bases of tables of up to kLdsItems items into LDS once per block and
// search there; larger tables are searched in global memory.
constexpr uint32_t kLdsItems = 512;

__device__ __forceinline__ uint32_t last_base_le(const uint32_t* bases, uint32_t n, uint32_t g) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (bases[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Block-wide: bases[i] = field(items[i]) for i < n_items (n_items <= kLdsItems).
template <typename F>
__device__ __forceinline__ void load_bases(uint32_t* bases, const LevelDesc* __restrict__ items,
                                           uint32_t n_items, F field) {
  for (uint32_t i = threadIdx.x; i < n_items; i += blockDim.x) bases[i] = field(items[i]);
  __syncthreads();
}

// Trajectory g of the table's time-parallel space (tp_bases: the items'
// tp_base in LDS, or null to search the table).
template <typename Real>
__device__ __forceinline__ void run_tp_index(const LevelDesc* __restrict__ items, uint32_t n_items,
                                             uint32_t g, const uint32_t* tp_bases) {
  uint32_t lo = 0;
  if (tp_bases) {
    lo = last_base_le(tp_bases, n_items, g);
  } else {
    uint32_t hi = n_items;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (items[mid].tp_base <= g) lo = mid; else hi = mid;
    }
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const LevelDesc d = items[lo];
  const uint32_t local = g - d.tp_base;
  switch (d.kind) {
    case kKindFineTwoPoint: run_tp_kind<Real, kKindFineTwoPoint>(d, local); break;
    case kKindFineMaxwell: run_tp_kind<Real, kKindFineMaxwell>(d, local); break;
    case kKindPairTwoPointSum: run_tp_kind<Real, kKindPairTwoPointSum>(d, local); break;
    case kKindPairMaxwellSum: run_tp_kind<Real, kKindPairMaxwellSum>(d, local); break;
    default: run_tp_kind<Real, kKindPairMaxwellAggregate>(d, local); break;
  }
}

// Trajectory g of the time-parallel space of a KD work table.
__device__ __forceinline__ void run_kd_tp_index(const LevelDesc* __restrict__ items,
                                                uint32_t n_items, uint32_t g,
                                                const uint32_t* tp_bases) {
  uint32_t lo = 0;
  if (tp_bases) {
    lo = last_base_le(tp_bases, n_items, g);
  } else {
    uint32_t hi = n_items;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (items[mid].tp_base <= g) lo = mid; else hi = mid;
    }
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const LevelDesc d = items[lo];
  const uint32_t local = g - d.tp_base;
  const bool bg = (d.flags & (kFlagBgB1 | kFlagBgB2)) != 0;
  if (d.kind == kKindKdPair) {
    if (bg) run_kd_bg_tp<true>(d, local);
    else run_kd_tp<true>(d, local);
  } else {
    if (bg) run_kd_bg_tp<false>(d, local);
    else run_kd_tp<false>(d, local);
  }
}

// The time-parallel items alone (the per-level launch form).
template <typename Real>
__global__ void __launch_bounds__(256) tp_kernel(const LevelDesc* __restrict__ items,
                                                  const WorkHeader* __restrict__ hdr) {
  const uint32_t n_items = hdr->n_items;
  const uint32_t total = hdr->total_tp;
  const uint32_t waves = gridDim.x * (blockDim.x / kLanes);
  const uint32_t first = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kLanes);
  for (uint32_t g = first; g < total; g += waves) run_tp_index<Real>(items, n_items, g, nullptr);
}

// The time-parallel items of a KD table alone (the per-level launch form).
__global__ void __launch_bounds__(256) kd_tp_kernel(const LevelDesc* __restrict__ items,
                                                     const WorkHeader* __restrict__ hdr) {
  const uint32_t n_items = hdr->n_items;
  const uint32_t total = hdr->total_tp;
  const uint32_t waves = gridDim.x * (blockDim.x / kLanes);
  const uint32_t first = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kLanes);
  for (uint32_t g = first; g < total; g += waves) run_kd_tp_index(items, n_items, g, nullptr);
}

// ---------------------------------------------------------------------------
// Persistent launch over a work table; items are ordered most expensive
// first.  The chunk space (runs of tiles of one item) is dealt out as
// kChunkStreams interleaved streams, chunks x, x + 8, x + 16, ... to the
// blocks with blockIdx % 8 == x (the blocks of one XCD under round-robin
// dispatch), each stream with its own work counter on its own cache line:
// the wavefronts that arrive first take the first (longest) chunks.  When one
// round covers the whole table (a small launch such as a warm-up), a
// wavefront takes the chunk of its own index instead and touches no counter.
// The grid must have at least kChunkStreams blocks (every stream needs waves).
// KD = true: the kinetic-diffusion instantiation (FP64; its tables hold KD
// items only and no time-parallel items).
// ---------------------------------------------------------------------------
template <typename Real, int P, bool KD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KD ? 3 : 1)))
persistent_kernel(const LevelDesc* __restrict__ items,
                                                          const WorkHeader* __restrict__ hdr,
                                                          unsigned int* __restrict__ counter,
                                                          Stats* __restrict__ partials) {
  __shared__ uint32_t chunk_bases[kLdsItems];
  __shared__ uint32_t tp_bases[kLdsItems];
  const uint32_t n_items = hdr->n_items;
  const uint32_t total = hdr->total_chunks;
  const int lane = threadIdx.x & (kLanes - 1);
  const uint32_t wpb = blockDim.x / kLanes;
  const uint32_t x = blockIdx.x % kChunkStreams;
  const bool lds = n_items <= kLdsItems;
  if (lds) {
    load_bases(chunk_bases, items, n_items, [](const LevelDesc& d) { return (uint32_t)d.chunk_base; });
    load_bases(tp_bases, items, n_items, [](const LevelDesc& d) { return d.tp_base; });
  }
  const uint32_t stream_waves = wpb * ((gridDim.x - x + kChunkStreams - 1) / kChunkStreams);
  const bool one_round = (uint64_t)x + (uint64_t)kChunkStreams * stream_waves >= total;
  // (wave-uniform; readfirstlane tells the compiler so, which keeps the
  // descriptor of the chunk's item in scalar registers)
  uint32_t k = __builtin_amdgcn_readfirstlane((blockIdx.x / kChunkStreams) * wpb +
                                              threadIdx.x / kLanes);  // static index
  // Time-parallel trajectories first, dealt from the last wavefront down (the
  // chunk streams hand out their first chunks to the first wavefronts).
  const uint32_t total_tp = hdr->total_tp;
  if (total_tp) {
    const uint32_t waves = gridDim.x * wpb;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + threadIdx.x / kLanes);
    for (uint32_t t = waves - 1u - wave; t < total_tp; t += waves) {
      if constexpr (KD) run_kd_tp_index(items, n_items, t, lds ? tp_bases : nullptr);
      else run_tp_index<Real>(items, n_items, t, lds ? tp_bases : nullptr);
    }
  }
  if (!one_round) {
    unsigned int first = 0;
    if (lane == 0) first = atomicAdd(&counter[x * kCounterStride], 1u);
    k = __builtin_amdgcn_readfirstlane(__shfl(first, 0, kLanes));
  }
  for (;;) {
    const uint64_t g64 = (uint64_t)x + (uint64_t)kChunkStreams * k;
    if (g64 >= total) break;
    const uint32_t g = (uint32_t)g64;
    uint32_t lo = 0;
    if (lds) {
      lo = last_base_le(chunk_bases, n_items, g);
    } else {
      uint32_t hi = n_items;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (items[mid].chunk_base <= g) lo = mid; else hi = mid;
      }
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const LevelDesc d = items[lo];  // (time-parallel items hold no chunks)
    const uint32_t c = g - (uint32_t)d.chunk_base;
    const uint32_t t0 = c * d.chunk_tiles;
    const uint32_t t1 = min(t0 + d.chunk_tiles, d.n_tiles);
    if constexpr (KD) {
      for (uint32_t t = t0; t < t1; ++t) run_kd_unit(d, t, partials);
    } else switch (d.kind) {
      case kKindFineTwoPoint:
        for (uint32_t t = t0; t < t1; ++t) run_unit<Real, P, kKindFineTwoPoint>(d, t, partials);
        break;
      case kKindFineMaxwell:
        for (uint32_t t = t0; t < t1; ++t) run_unit<Real, P, kKindFineMaxwell>(d, t, partials);
        break;
      case kKindPairTwoPointSum:
        for (uint32_t t = t0; t < t1; ++t) run_unit<Real, P, kKindPairTwoPointSum>(d, t, partials);
        break;
      case kKindPairMaxwellSum:
        for (uint32_t t = t0; t < t1; ++t) run_unit<Real, P, kKindPairMaxwellSum>(d, t, partials);
        break;
      default:
        for (uint32_t t = t0; t < t1; ++t)
          run_unit<Real, P, kKindPairMaxwellAggregate>(d, t, partials);
        break;
    }
    if (one_round) break;
    unsigned int next = 0;
    if (lane == 0) next = atomicAdd(&counter[x * kCounterStride], 1u);
    k = __builtin_amdgcn_readfirstlane(__shfl(next, 0, kLanes));
  }
}

// ---------------------------------------------------------------------------
// Reductions.  Stage 1: group g of an item merges tiles [256 g, 256 g +
// 256): thread t takes tile 256 g + t, then a fixed LDS tree.  Stage 2 merges an item's group results the same way (thread t merges
// groups [t q, t q + q), q = ceil(n_groups / 256)) and folds the result into
// the item's resident statistics slot.
// ---------------------------------------------------------------------------
// Fixed LDS tree over the block's 256 records; the result is left in sh[0].
// Records from index n_live on are empty, and a merge with an empty record
// returns the other one unchanged, so the levels whose stride is at least
// n_live are skipped (block-uniform) without changing the result.
__device__ __forceinline__ void block_tree(const Stats& acc, Stats* sh, uint32_t n_live) {
  const int t = threadIdx.x;
  sh[t] = acc;
  __syncthreads();
#pragma unroll 1
  for (int stride = kReduceThreads / 2; stride > 0; stride >>= 1) {
    if ((uint32_t)stride >= n_live) continue;
    if (t < stride) sh[t] = stats_merge(sh[t], sh[t + stride]);
    __syncthreads();
  }
}

// Folds an item's final record into its resident statistics slot (and the
// host-mapped mirror).
__device__ __forceinline__ void store_item(const LevelDesc& d, const Stats& rec,
                                           Stats* __restrict__ resident,
                                           Stats* __restrict__ mirror) {
  const uint32_t slot = d.result_slot;
  const Stats r = (d.flags & kFlagAccumulate) ? stats_merge(resident[slot], rec) : rec;
  resident[slot] = r;
  if (mirror) mirror[slot] = r;  // host-mapped copy, read after the stream syncs
}

// Merge of one item's group records into its resident slot (stage 2).
__device__ __forceinline__ void merge_item(const LevelDesc& d, const Stats* __restrict__ groups,
                                           Stats* __restrict__ resident, Stats* __restrict__ mirror,
                                           Stats* sh) {
  const uint64_t gbase = d.group_base;
  const uint32_t n_groups = d.n_groups;
  if (n_groups > 1) {
    Stats acc = stats_empty();
    const uint32_t q = (n_groups + kReduceThreads - 1) / kReduceThreads;
    const uint32_t first = threadIdx.x * q;
    for (uint32_t idx = first; idx < n_groups && idx < first + q; ++idx)
      acc = stats_merge(acc, groups[gbase + idx]);
    block_tree(acc, sh, (n_groups + q - 1) / q);
  } else if (threadIdx.x == 0) {
    // the tree over one record and empties returns that record unchanged
    sh[0] = groups[gbase];
  }
  if (threadIdx.x == 0) store_item(d, sh[0], resident, mirror);
  __syncthreads();
}

// Both stages in one launch: blocks take groups in grid-stride order; each
// item counts its finished groups, and the block that finishes an item's last
// group merges that item at once (release/acquire through device-scope fences
// around the count).  Every item has at least one group.
__global__ void __launch_bounds__(kReduceThreads) reduce_kernel(
    const LevelDesc* __restrict__ items, const WorkHeader* __restrict__ hdr,
    Stats* __restrict__ partials, Stats* __restrict__ groups, unsigned int* __restrict__ item_done,
    Stats* __restrict__ resident, Stats* __restrict__ mirror) {
  __shared__ Stats sh[kReduceThreads];
  __shared__ unsigned int item_complete;
  __shared__ uint32_t group_bases[kLdsItems];
  const uint32_t n_items = hdr->n_items;
  const uint32_t total = hdr->total_groups;
  const bool lds = n_items <= kLdsItems;
  if (lds && blockIdx.x < total)
    load_bases(group_bases, items, n_items, [](const LevelDesc& d) { return (uint32_t)d.group_base; });
  for (uint32_t vb = blockIdx.x; vb < total; vb += gridDim.x) {
    uint32_t lo = 0;
    if (lds) {
      lo = last_base_le(group_bases, n_items, vb);
    } else {
      uint32_t hi = n_items;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (items[mid].group_base <= vb) lo = mid; else hi = mid;
      }
    }
    const LevelDesc d = items[lo];
    const uint64_t tile_base = d.tile_base;
    const uint32_t n_tiles = d.n_tiles;
    const uint32_t g = vb - (uint32_t)d.group_base;
    if (d.flags & kFlagTimeParallel) {
      // tile records of a time-parallel item, from its samples' final states
      const uint32_t t_end = min((g + 1) * (uint32_t)kGroupTiles, n_tiles);
      const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
      for (uint32_t t = g * kGroupTiles + wave; t < t_end; t += kReduceThreads / kLanes) {
        const Stats r = (d.flags & kFlagCoarse) ? tp_tile_record<true>(d, t)
                                                : tp_tile_record<false>(d, t);
        if ((threadIdx.x & (kLanes - 1)) == 0) partials[tile_base + t] = r;
      }
      __syncthreads();
    }
    Stats acc = stats_empty();
    const uint32_t first = g * kGroupTiles + threadIdx.x * kReducePerThread;
    for (int k = 0; k < kReducePerThread; ++k) {
      const uint32_t idx = first + k;
      if (idx < n_tiles) acc = stats_merge(acc, partials[tile_base + idx]);
    }
    block_tree(acc, sh, min((uint32_t)kGroupTiles, n_tiles - g * (uint32_t)kGroupTiles));
    if (d.n_groups == 1) {
      // the item's only group: its record is the item's (what the second
      // stage would merge from the one group record), no count needed
      if (threadIdx.x == 0) store_item(d, sh[0], resident, mirror);
      __syncthreads();
      continue;
    }
    if (threadIdx.x == 0) {
      groups[vb] = sh[0];
      __threadfence();  // the group record is visible before it is counted
      const unsigned int prev = atomicAdd(&item_done[lo], 1u);
      item_complete = (prev + 1u == d.n_groups) ? 1u : 0u;
    }
    __syncthreads();
    if (item_complete) {
      __threadfence();  // the other blocks' group records of this item
      merge_item(d, groups, resident, mirror, sh);
    }
    __syncthreads();
  }
}

// First node of every launch: copies the work table and its header from
// host-mapped pinned memory (written by the host before the launch) into
// device memory and clears the chunk and item counters, so one launch needs no
// copy commands.  At most `cap` descriptors are copied.
__global__ void stage_kernel(const WorkHeader* __restrict__ hdr_src,
                             const LevelDesc* __restrict__ items_src, uint32_t cap,
                             WorkHeader* __restrict__ hdr_dst, LevelDesc* __restrict__ items_dst,
                             unsigned int* __restrict__ counter,
                             unsigned int* __restrict__ item_done) {
  static_assert(sizeof(LevelDesc) % sizeof(uint4) == 0, "descriptor copy granularity");
  const uint32_t n_items = min(hdr_src->n_items, cap);
  const uint64_t words = (uint64_t)n_items * (sizeof(LevelDesc) / sizeof(uint4));
  const uint4* src = reinterpret_cast<const uint4*>(items_src);
  uint4* dst = reinterpret_cast<uint4*>(items_dst);
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_items; i += gridDim.x * blockDim.x)
    item_done[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < kChunkStreams) counter[threadIdx.x * kCounterStride] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    WorkHeader h = *hdr_src;
    h.n_items = n_items;
    *hdr_dst = h;
  }
}

// Device-planned top-up.  Right after a warm-up launch's reduction, one block
// computes eqs. Nopt1/Noptj from the warm-up's resident statistics and builds
// the top-up's work table in place of the warm-up's, so that the top-up's
// particle and reduction kernels follow on the stream without a return to
// the host.  The arithmetic is the host's (plan.hpp); every descriptor field
// is the warm-up's except the sample range, the accumulate flag and the tile
// layout.  The warm-up's statistics and the planned numbers go to `rec`
// (host-mapped) for the host's check.  A table that would not fit the tile or
// group buffers is not built: the header then holds no work and rec->declined
// is set.
constexpr int kPlanThreads = 256;

__global__ void __launch_bounds__(kPlanThreads) plan_kernel(
    PlanArgs a, LevelDesc* __restrict__ items, WorkHeader* __restrict__ hdr,
    const Stats* __restrict__ resident, unsigned int* __restrict__ counter,
    unsigned int* __restrict__ item_done, PlanRecord* __restrict__ rec) {
  constexpr int kMax = MLMC_AP_MAX_LEVELS;
  constexpr int kWords = sizeof(LevelDesc) / sizeof(uint4);
  static_assert(kMax <= kPlanThreads, "one thread per level");
  __shared__ LevelDesc src[kMax];
  __shared__ uint64_t begin[kMax], count[kMax], tile_b[kMax], group_b[kMax], chunk_b[kMax];
  __shared__ ItemLayout lay[kMax];
  __shared__ uint32_t src_of[kMax];
  __shared__ uint32_t n_out;
  __shared__ double var[kMax], root[kMax], S_sh;
  __shared__ uint64_t done[kMax], target[kMax];
  const uint32_t t = threadIdx.x;
  const uint32_t nw = a.n_items < (uint32_t)kMax ? a.n_items : (uint32_t)kMax;
  for (uint32_t i = t; i < nw * kWords; i += blockDim.x)
    reinterpret_cast<uint4*>(src)[i] = reinterpret_cast<const uint4*>(items)[i];
  // thread l: level l's statistics, variance and term of S
  const bool lvl = t < (uint32_t)kMax && ((a.level_mask >> t) & 1u);
  if (t < (uint32_t)kMax) {
    var[t] = 0.0;
    root[t] = 0.0;
    done[t] = 0;
    target[t] = 0;
    if (lvl) {
      const Stats st = resident[a.slot_base + t];
      rec->warmup[t] = st;
      var[t] = level_variance(st);
      root[t] = cost_variance_root(var[t], a.cost[t]);
      done[t] = (uint64_t)st.n;
    }
  }
  __syncthreads();
  if (t == 0) {
    double S = 0.0;  // in level order, as the host sums
    for (int l = 0; l < kMax; ++l)
      if ((a.level_mask >> l) & 1u) S += root[l];
    S_sh = S;
  }
  __syncthreads();
  if (lvl) {
    target[t] = level_target(var[t], a.cost[t], S_sh, a.tol, done[t]);
    rec->target[t] = target[t];
  }
  __syncthreads();
  // thread i: the layout of warm-up item i's top-up (if its level needs one)
  if (t < nw) {
    const uint32_t l = src[t].result_slot - a.slot_base;
    count[t] = (l < (uint32_t)kMax && target[l] > done[l]) ? target[l] - done[l] : 0u;
    begin[t] = l < (uint32_t)kMax ? done[l] : 0u;
    if (count[t]) lay[t] = item_layout(src[t].n_steps, count[t]);
  }
  __syncthreads();
  if (t == 0) {
    // the top-up's items keep the warm-up table's order
    uint64_t tiles = 0, groups = 0, chunks = 0;
    uint32_t n = 0;
    for (uint32_t i = 0; i < nw; ++i) {
      if (!count[i]) continue;
      src_of[n] = i;
      tile_b[n] = tiles;
      group_b[n] = groups;
      chunk_b[n] = chunks;
      tiles += lay[i].n_tiles;
      groups += lay[i].n_groups;
      chunks += lay[i].n_chunks;
      ++n;
    }
    const bool fits = tiles <= a.cap_tiles && groups <= a.cap_groups && chunks < 0xFFFFFFF0ull;
    if (!fits) n = 0;
    n_out = n;
    WorkHeader h;
    h.n_items = n;
    h.total_chunks = n ? (uint32_t)chunks : 0u;
    h.total_groups = n ? (uint32_t)groups : 0u;
    h.total_tp = 0u;
    *hdr = h;
    rec->declined = fits ? 0u : 1u;
    rec->n_items = n;
  }
  __syncthreads();
  const uint32_t n = n_out;
  if (t < n) {
    const uint32_t i = src_of[t];
    LevelDesc d = src[i];
    const ItemLayout o = lay[i];
    d.sample_begin = begin[i];
    d.n_samples = count[i];
    d.flags = (d.flags & ~(uint32_t)kFlagTimeParallel) | kFlagAccumulate;
    d.spl = o.spl;
    d.n_tiles = o.n_tiles;
    d.n_groups = o.n_groups;
    d.chunk_tiles = o.chunk_tiles;
    d.n_chunks = o.n_chunks;
    d.tile_base = tile_b[t];
    d.group_base = group_b[t];
    d.chunk_base = chunk_b[t];
    d.tp_base = 0u;
    d.tp_out = nullptr;
    items[t] = d;
    item_done[t] = 0u;
  }
  if (t < kChunkStreams) counter[t * kCounterStride] = 0u;
}

// First kernel of an allocation-free launch: the work header and the single
// descriptor arrive as kernel arguments (no host-side table, no copy), and the
// reduction's item counter and the histogram counters are cleared.
__global__ void stage_args_kernel(WorkHeader h, LevelDesc d, WorkHeader* __restrict__ hdr_dst,
                                  LevelDesc* __restrict__ item_dst,
                                  unsigned int* __restrict__ item_done,
                                  unsigned long long* __restrict__ hist, uint32_t hist_n) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    *hdr_dst = h;
    *item_dst = d;
    item_done[0] = 0u;
  }
  for (uint32_t i = t; i < hist_n; i += gridDim.x * blockDim.x) hist[i] = 0ull;
}

__global__ void fill_u32_kernel(unsigned int* p, uint64_t n, unsigned int v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long* p, uint64_t n, unsigned long long v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// Validation kernels: the same Philox / uniform / Box-Muller code paths.
// ---------------------------------------------------------------------------
__global__ void words_kernel(uint32_t key0, uint32_t key1, uint32_t strm, uint32_t tag,
                             uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps,
                             uint32_t* __restrict__ out) {
  const uint64_t total = n_samples * n_steps;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t s = i / n_steps;
    const uint32_t n = (uint32_t)(i % n_steps);
    const Words w = philox4x32_10(n, (uint32_t)(sample_begin + s), tag, strm, key0, key1);
    out[4 * i + 0] = w.w0; out[4 * i + 1] = w.w1;
    out[4 * i + 2] = w.w2; out[4 * i + 3] = w.w3;
  }
}

template <typename Real>
__global__ void normals_kernel(uint32_t key0, uint32_t key1, uint32_t strm, uint32_t tag,
                               uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps,
                               Real* __restrict__ out) {
  const uint64_t total = n_samples * n_steps;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t s = i / n_steps;
    const uint32_t n = (uint32_t)(i % n_steps);
    const Words w = philox4x32_10(n, (uint32_t)(sample_begin + s), tag, strm, key0, key1);
    Real xi, g;
    box_muller(w.w1, w.w2, xi, g);
    Real u1, u2;
    if constexpr (sizeof(Real) == 4) { u1 = uniform_f32(w.w1); u2 = uniform_f32(w.w2); }
    else { u1 = uniform_f64(w.w1); u2 = uniform_f64(w.w2); }
    out[4 * i + 0] = u1; out[4 * i + 1] = u2;
    out[4 * i + 2] = xi; out[4 * i + 3] = g;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
template <typename Real, int P>
static hipError_t launch_level_p(int kind, const LevelDesc* items, uint32_t item, uint32_t n_tiles,
                                 int block, Stats* partials, hipStream_t s) {
  const uint32_t waves_per_block = (uint32_t)block / kLanes;
  const dim3 grid((n_tiles + waves_per_block - 1) / waves_per_block);
  switch (kind) {
    case kKindFineTwoPoint:
      hipLaunchKernelGGL((level_kernel<Real, P, kKindFineTwoPoint>), grid, dim3(block), 0, s,
                         items, item, partials);
      break;
    case kKindFineMaxwell:
      hipLaunchKernelGGL((level_kernel<Real, P, kKindFineMaxwell>), grid, dim3(block), 0, s,
                         items, item, partials);
      break;
    case kKindPairTwoPointSum:
      hipLaunchKernelGGL((level_kernel<Real, P, kKindPairTwoPointSum>), grid, dim3(block), 0, s,
                         items, item, partials);
      break;
    case kKindPairMaxwellSum:
      hipLaunchKernelGGL((level_kernel<Real, P, kKindPairMaxwellSum>), grid, dim3(block), 0, s,
                         items, item, partials);
      break;
    default:
      hipLaunchKernelGGL((level_kernel<Real, P, kKindPairMaxwellAggregate>), grid, dim3(block),
                         0, s, items, item, partials);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_level(bool fp64, int ppt, int kind, const LevelDesc* items_dev, uint32_t item,
                        uint32_t n_tiles, int block, Stats* partials, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  if (is_kd_kind(kind)) {
    const uint64_t threads = (uint64_t)n_tiles * kLanes;
    const dim3 grid((unsigned)((threads + block - 1) / block));
    hipLaunchKernelGGL(kd_level_kernel, grid, dim3(block), 0, s, items_dev, item, partials);
    return hipGetLastError();
  }
  if (fp64) {
    if (ppt == 1) return launch_level_p<double, 1>(kind, items_dev, item, n_tiles, block, partials, s);
    if (ppt == 2) return launch_level_p<double, 2>(kind, items_dev, item, n_tiles, block, partials, s);
    return launch_level_p<double, 4>(kind, items_dev, item, n_tiles, block, partials, s);
  }
  if (ppt == 1) return launch_level_p<float, 1>(kind, items_dev, item, n_tiles, block, partials, s);
  if (ppt == 2) return launch_level_p<float, 2>(kind, items_dev, item, n_tiles, block, partials, s);
  return launch_level_p<float, 4>(kind, items_dev, item, n_tiles, block, partials, s);
}

int persistent_blocks_per_cu(bool fp64, int ppt, int block, bool kd) {
  int nb = 0;
  hipError_t e;
#define MLMC_OCC(R, PP, K) \
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persistent_kernel<R, PP, K>, block, 0)
  if (kd) {
    e = MLMC_OCC(double, 1, true);
  } else if (fp64) {
    if (ppt == 1) e = MLMC_OCC(double, 1, false);
    else if (ppt == 2) e = MLMC_OCC(double, 2, false);
    else e = MLMC_OCC(double, 4, false);
  } else {
    if (ppt == 1) e = MLMC_OCC(float, 1, false);
    else if (ppt == 2) e = MLMC_OCC(float, 2, false);
    else e = MLMC_OCC(float, 4, false);
  }
#undef MLMC_OCC
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

hipError_t launch_persistent(bool fp64, int ppt, const LevelDesc* items_dev,
                             const WorkHeader* hdr_dev, unsigned int* counter, Stats* partials,
                             int block, int grid, hipStream_t s, bool kd) {
  const dim3 g(grid), b(block);
#define MLMC_PERSIST(R, PP, K) \
  hipLaunchKernelGGL((persistent_kernel<R, PP, K>), g, b, 0, s, items_dev, hdr_dev, counter, partials)
  if (kd) {
    MLMC_PERSIST(double, 1, true);
  } else if (fp64) {
    if (ppt == 1) MLMC_PERSIST(double, 1, false);
    else if (ppt == 2) MLMC_PERSIST(double, 2, false);
    else MLMC_PERSIST(double, 4, false);
  } else {
    if (ppt == 1) MLMC_PERSIST(float, 1, false);
    else if (ppt == 2) MLMC_PERSIST(float, 2, false);
    else MLMC_PERSIST(float, 4, false);
  }
#undef MLMC_PERSIST
  return hipGetLastError();
}

hipError_t launch_reduce(const LevelDesc* items_dev, const WorkHeader* hdr_dev, Stats* partials,
                         Stats* groups, unsigned int* item_done, Stats* resident, Stats* mirror,
                         int grid, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(grid), dim3(kReduceThreads), 0, s, items_dev, hdr_dev,
                     partials, groups, item_done, resident, mirror);
  return hipGetLastError();
}

hipError_t launch_tp(bool fp64, const LevelDesc* items_dev, const WorkHeader* hdr_dev, int grid,
                     hipStream_t s, bool kd) {
  if (kd)
    hipLaunchKernelGGL(kd_tp_kernel, dim3(grid), dim3(256), 0, s, items_dev, hdr_dev);
  else if (fp64)
    hipLaunchKernelGGL(tp_kernel<double>, dim3(grid), dim3(256), 0, s, items_dev, hdr_dev);
  else
    hipLaunchKernelGGL(tp_kernel<float>, dim3(grid), dim3(256), 0, s, items_dev, hdr_dev);
  return hipGetLastError();
}

hipError_t launch_stage(const WorkHeader* hdr_src, const LevelDesc* items_src, uint32_t cap,
                        WorkHeader* hdr_dst, LevelDesc* items_dst, unsigned int* counter,
                        unsigned int* item_done, hipStream_t s) {
  hipLaunchKernelGGL(stage_kernel, dim3(16), dim3(256), 0, s, hdr_src, items_src, cap, hdr_dst,
                     items_dst, counter, item_done);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, uint64_t n, unsigned int v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256),
                     0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256),
                     0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_words(uint32_t key0, uint32_t key1, uint32_t strm, uint32_t tag,
                        uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps,
                        uint32_t* out, hipStream_t s) {
  const uint64_t total = n_samples * n_steps;
  if (total == 0) return hipSuccess;
  const uint64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(words_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0,
                     s, key0, key1, strm, tag, sample_begin, n_samples, n_steps, out);
  return hipGetLastError();
}

hipError_t launch_normals(bool fp64, uint32_t key0, uint32_t key1, uint32_t strm, uint32_t tag,
                          uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps, void* out,
                          hipStream_t s) {
  const uint64_t total = n_samples * n_steps;
  if (total == 0) return hipSuccess;
  const uint64_t blocks = (total + 255) / 256;
  const dim3 g((unsigned)(blocks < 4096 ? blocks : 4096));
  if (fp64)
    hipLaunchKernelGGL(normals_kernel<double>, g, dim3(256), 0, s, key0, key1, strm, tag,
                       sample_begin, n_samples, n_steps, (double*)out);
  else
    hipLaunchKernelGGL(normals_kernel<float>, g, dim3(256), 0, s, key0, key1, strm, tag,
                       sample_begin, n_samples, n_steps, (float*)out);
  return hipGetLastError();
}

// Consistency harness of Section 5.1: one KD pair per thread, its coarse
// numbers recorded (at most `cap` rows per pair; counts[i] = all of its coarse
// KD steps).
__global__ void __launch_bounds__(256) kd_numbers_kernel(LevelDesc d, uint64_t n, uint32_t cap,
                                                         double* __restrict__ rows,
                                                         uint32_t* __restrict__ counts) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  KdRecord rec{rows + i * (uint64_t)cap * 4ull, cap, 0u};
  double xf, xc;
  uint32_t cf, cc;
  const uint32_t smp = (uint32_t)(d.sample_begin + i);
  if (d.flags & (kFlagBgB1 | kFlagBgB2)) kd_sample_bg_rec<true>(d, smp, xf, xc, cf, cc, rec);
  else kd_sample_rec<true>(d, smp, xf, xc, cf, cc, rec);
  counts[i] = rec.n;
}

hipError_t launch_kd_numbers(const LevelDesc& d, uint64_t n, uint32_t cap, double* rows,
                             uint32_t* counts, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(kd_numbers_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, n,
                     cap, rows, counts);
  return hipGetLastError();
}

hipError_t launch_plan(const PlanArgs& a, LevelDesc* items_dev, WorkHeader* hdr_dev,
                       const Stats* resident, unsigned int* counter, unsigned int* item_done,
                       PlanRecord* rec, hipStream_t s) {
  if (a.n_items > (uint32_t)MLMC_AP_MAX_LEVELS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, a, items_dev, hdr_dev,
                     resident, counter, item_done, rec);
  return hipGetLastError();
}

hipError_t launch_stage_args(const WorkHeader& h, const LevelDesc& d, WorkHeader* hdr_dst,
                             LevelDesc* item_dst, unsigned int* item_done,
                             unsigned long long* hist, uint32_t hist_n, hipStream_t s) {
  hipLaunchKernelGGL(stage_args_kernel, dim3(hist_n > 256 ? 4 : 1), dim3(256), 0, s, h, d,
                     hdr_dst, item_dst, item_done, hist, hist_n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch memory of the allocation-free entry point: a file-scope device
// array, one copy on every GPU the library runs on, held until the process
// ends.  Host code never passes `scratch` itself to a kernel (in host code the
// name stands for a host-side shadow, not a device address): the device
// address is looked up once per device, with that device current, and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchMaxDevices];
}  // namespace

hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace mlmc
