// C ABI of the MLMC-AP library: validation, level constants, device
// workspace, work tables, launches and the MLMC control loop (Section 4.1).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "host.hpp"
#include "stats.hpp"

namespace mlmc {

namespace {
thread_local std::string g_last_error;
constexpr double kTwo32 = 4294967296.0;
}  // namespace

mlmc_ap_status set_error(mlmc_ap_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

// ---------------------------------------------------------------------------
// Level constants: dt_l = dt0 / M^l; h, s, p of the splitting scheme;
// thr = round(p 2^32).
// ---------------------------------------------------------------------------
LevelConst level_const(const mlmc_ap_problem& p, int level) {
  LevelConst c;
  c.dt = p.dt0 / std::pow((double)p.M, (double)level);
  const double denom = p.eps * p.eps + c.dt;
  c.h = c.dt * p.eps / denom;
  c.s = std::sqrt(2.0 * c.dt * c.dt / denom);
  c.p = c.dt / denom;
  c.n_steps = (uint64_t)std::llround(p.T / p.dt0) *
              (uint64_t)std::llround(std::pow((double)p.M, (double)level));
  c.thr = (uint64_t)std::llround(c.p * kTwo32);
  return c;
}

// Coarse collision threshold: the smallest of M independent uniform words is
// below t with probability 1 - (1 - t/2^32)^M; t = 2^32 (1 - (1-p_c)^(1/M))
// makes that the coarse level's p_c = thr_c/2^32.  t <= thr_f because
// (1 - p_f)^M <= 1 - p_c, so a coarse collision implies a fine one.
uint64_t coarse_threshold(uint64_t thr_f, uint64_t thr_c, int M) {
  const double pc = (double)thr_c / kTwo32;
  const double t = kTwo32 * -std::expm1(std::log1p(-pc) / (double)M);
  uint64_t r = (uint64_t)std::llround(t);
  return r > thr_f ? thr_f : r;
}

// Expected KD steps of one path of a level: a KD step runs from a grid point
// to the end of the grid step holding the next collision, which advances
// 1/(1 - e^{-R dt}) steps on average, so n (1 - e^{-R dt}) steps per path.
// In a background of Section 5 the rate is at least b, and b is taken.
static double kd_path_cost(const mlmc_ap_problem& p, int level) {
  const LevelConst c = level_const(p, level);
  const double R = p.background == MLMC_AP_BG_DIFFUSIVE ? 1.0 / (p.eps * p.eps) : p.bg_b;
  return (double)c.n_steps * -std::expm1(-R * c.dt);
}

uint64_t pair_cost(const mlmc_ap_problem& p, int level, int coarse_level) {
  if (p.scheme == MLMC_AP_SCHEME_KD) {
    double c = kd_path_cost(p, level);
    if (coarse_level >= 0) c += kd_path_cost(p, coarse_level);
    return std::max<uint64_t>(1, (uint64_t)std::ceil(c));
  }
  const uint64_t n = level_const(p, level).n_steps;
  return coarse_level >= 0 ? n + level_const(p, coarse_level).n_steps : n;
}

uint64_t sample_cost(const mlmc_ap_problem& p, int level, bool single) {
  return pair_cost(p, level, (single || level == 0) ? -1 : level - 1);
}

uint64_t block_factor(const mlmc_ap_problem& p, int level, int coarse_level) {
  uint64_t b = 1;
  for (int i = coarse_level; i < level; ++i) b *= (uint64_t)p.M;
  return b;
}

mlmc_ap_status validate_problem(const mlmc_ap_problem* p) {
  if (!p) return set_error(MLMC_AP_EINVAL, "problem is NULL");
  if (!(p->eps >= 0.0) || !std::isfinite(p->eps))
    return set_error(MLMC_AP_EINVAL, "eps must be finite and >= 0");
  if (!(p->T > 0.0) || !std::isfinite(p->T)) return set_error(MLMC_AP_EINVAL, "T must be > 0");
  if (!(p->dt0 > 0.0) || !std::isfinite(p->dt0))
    return set_error(MLMC_AP_EINVAL, "dt0 must be > 0");
  if (p->M < 2 || p->M > 64) return set_error(MLMC_AP_EINVAL, "M must be in [2, 64]");
  if (p->L < 0 || p->L >= MLMC_AP_MAX_LEVELS) return set_error(MLMC_AP_EINVAL, "L must be in [0, 30]");
  const double ratio = p->T / p->dt0;
  const double n0 = std::round(ratio);
  if (n0 < 1.0 || std::fabs(ratio - n0) > 1e-9 * n0)
    return set_error(MLMC_AP_EINVAL, "T/dt0 must be a positive integer");
  const double nL = n0 * std::pow((double)p->M, (double)p->L);
  if (nL >= 2147483648.0) return set_error(MLMC_AP_EINVAL, "n_L = (T/dt0) M^L must be < 2^31");
  if (p->x0_kind < MLMC_AP_X0_DELTA || p->x0_kind > MLMC_AP_X0_COSINE)
    return set_error(MLMC_AP_EINVAL, "unknown x0_kind");
  if (p->eq_kind != MLMC_AP_EQ_TWO_POINT && p->eq_kind != MLMC_AP_EQ_MAXWELLIAN)
    return set_error(MLMC_AP_EINVAL, "unknown eq_kind");
  if (!std::isfinite(p->x0_a) || !std::isfinite(p->x0_b) || p->x0_b < 0.0)
    return set_error(MLMC_AP_EINVAL, "x0_a must be finite and x0_b finite and >= 0");
  if (p->coupling != MLMC_AP_COUPLING_KICK_SUM && p->coupling != MLMC_AP_COUPLING_AGGREGATE)
    return set_error(MLMC_AP_EINVAL, "unknown coupling");
  if (p->coupling == MLMC_AP_COUPLING_AGGREGATE && p->eq_kind != MLMC_AP_EQ_MAXWELLIAN)
    return set_error(MLMC_AP_EINVAL,
                     "the aggregated coupling needs the Maxwellian equilibrium (a weighted sum "
                     "of +-1 velocities is not Gaussian)");
  if (p->qoi != MLMC_AP_QOI_X2 && p->qoi != MLMC_AP_QOI_X2_HIST && p->qoi != MLMC_AP_QOI_X)
    return set_error(MLMC_AP_EINVAL, "unknown qoi");
  if (p->qoi == MLMC_AP_QOI_X2_HIST) {
    if (p->nbins < 1 || p->nbins > MLMC_AP_MAX_BINS)
      return set_error(MLMC_AP_EINVAL, "nbins must be in [1, 1024]");
    if (!(p->hist_lo < p->hist_hi) || !std::isfinite(p->hist_lo) || !std::isfinite(p->hist_hi))
      return set_error(MLMC_AP_EINVAL, "histogram range must satisfy hist_lo < hist_hi");
  }
  if (p->fp64_state != 0 && p->fp64_state != 1)
    return set_error(MLMC_AP_EINVAL, "fp64_state must be 0 or 1");
  if (p->scheme != MLMC_AP_SCHEME_SPLITTING && p->scheme != MLMC_AP_SCHEME_KD)
    return set_error(MLMC_AP_EINVAL, "unknown scheme");
  if (p->background != MLMC_AP_BG_DIFFUSIVE && p->background != MLMC_AP_BG_B1 &&
      p->background != MLMC_AP_BG_B2)
    return set_error(MLMC_AP_EINVAL, "unknown background");
  if (p->background != MLMC_AP_BG_DIFFUSIVE) {
    if (p->scheme != MLMC_AP_SCHEME_KD)
      return set_error(MLMC_AP_EINVAL, "the backgrounds B1, B2 are for the KD scheme");
    if (!(p->bg_b > 0.0) || !std::isfinite(p->bg_b) || !(p->bg_a >= 0.0) ||
        !std::isfinite(p->bg_a))
      return set_error(MLMC_AP_EINVAL, "a background needs bg_a >= 0 and bg_b > 0, finite");
  }
  if (p->scheme == MLMC_AP_SCHEME_KD) {
    if (p->background == MLMC_AP_BG_DIFFUSIVE && !(p->eps > 0.0))
      return set_error(MLMC_AP_EINVAL, "the KD scheme needs eps > 0");
    if (p->eq_kind != MLMC_AP_EQ_MAXWELLIAN)
      return set_error(MLMC_AP_EINVAL, "the KD scheme needs the Maxwellian equilibrium");
    if (p->fp64_state != 1)
      return set_error(MLMC_AP_EINVAL, "the KD scheme runs with FP64 state (fp64_state = 1)");
  }
  return MLMC_AP_OK;
}

bool time_parallel_candidate(const ItemSpec& s, int32_t tp_max_samples) {
  const mlmc_ap_problem& p = *s.prob;
  const bool kd = p.scheme == MLMC_AP_SCHEME_KD;
  const int64_t limit = tp_max_samples == 0 ? kTpDefaultMaxSamples : tp_max_samples;
  if (limit <= 0 || s.n_samples == 0 || s.n_samples > (uint64_t)limit) return false;
  const bool coarse = !s.single && s.level >= 1;
  const uint64_t mb = coarse ? block_factor(p, s.level, s.coarse_level >= 0 ? s.coarse_level
                                                                              : s.level - 1)
                             : 1;
  // splitting scheme: coarse blocks inside a 64-step chunk (the KD form
  // carries its coarse steps across windows)
  if (!kd && coarse && mb != 2 && mb != 4) return false;
  return level_const(p, s.level).n_steps >= (int64_t)kLongLevelSteps;
}

static bool in_background(const mlmc_ap_problem& p) {
  return p.scheme == MLMC_AP_SCHEME_KD && p.background != MLMC_AP_BG_DIFFUSIVE && p.bg_a > 0.0;
}

// Time-parallel choice for the KD items of a launch that run in a background
// of Section 5.  There a time-parallel wavefront walks every KD step's state
// itself, so the form trades a shorter chain for far more issue slots.
// Latencies in GPU cycles per KD step as kd_path_cost counts them, measured
// on MI355X (B1, a = 10, b = 1000, level 14 paths and pairs with coarse level
// 13 or 3, 1000 samples, one wavefront per SIMD): per lane, a path alone
// 6800 per step, a pair 10200 per fine step (its aggregation weights) and
// 3900 per coarse step; time-parallel 3400, 4700 and 3600.  A time-parallel
// wavefront keeps its SIMD busy for less than half of that time (0.4 is
// taken), so several of them on one SIMD queue behind each other.  The
// launch takes about the longest of: the longest per-lane item, the longest
// time-parallel item, and the time-parallel issue spread over the SIMDs.
// Items are taken longest first while that estimate falls.
constexpr double kBgLaneFine = 6800.0, kBgLanePairFine = 10200.0, kBgLaneCoarse = 3900.0;
constexpr double kBgTpFine = 3400.0, kBgTpPairFine = 4700.0, kBgTpCoarse = 3600.0;
constexpr double kBgTpBusy = 0.4;

static void choose_background_tp(const std::vector<ItemSpec>& specs, int32_t tp_max_samples,
                                 int n_simd, std::vector<bool>& tp) {
  struct Cand {
    double lane, tp;  // latency estimates, cycles
    size_t i;
    bool ok;          // qualifies for the time-parallel form
  };
  std::vector<Cand> c;
  for (size_t i = 0; i < specs.size(); ++i) {
    const ItemSpec& s = specs[i];
    if (!in_background(*s.prob)) continue;
    const double f = kd_path_cost(*s.prob, s.level);
    const bool pair = !s.single && s.level >= 1;
    const double cc = pair ? kd_path_cost(*s.prob, s.coarse_level >= 0 ? s.coarse_level
                                                                       : s.level - 1)
                           : 0.0;
    const double lane = pair ? kBgLanePairFine * f + kBgLaneCoarse * cc : kBgLaneFine * f;
    const double tpl = pair ? kBgTpPairFine * f + kBgTpCoarse * cc : kBgTpFine * f;
    c.push_back({lane, tpl, i, time_parallel_candidate(s, tp_max_samples)});
  }
  if (c.empty()) return;
  std::stable_sort(c.begin(), c.end(), [](const Cand& a, const Cand& b) { return a.lane > b.lane; });
  // the per-lane latency no choice removes: items that do not qualify
  double floor_lat = 0.0;
  for (const Cand& x : c)
    if (!x.ok) floor_lat = std::max(floor_lat, x.lane);
  std::vector<size_t> order;
  for (size_t j = 0; j < c.size(); ++j)
    if (c[j].ok) order.push_back(j);
  double best = 0.0, tp_lat = 0.0, issue = 0.0;
  size_t best_k = 0;
  for (size_t k = 0; k <= order.size(); ++k) {
    if (k > 0) {
      const Cand& x = c[order[k - 1]];
      tp_lat = std::max(tp_lat, x.tp);
      issue += (double)specs[x.i].n_samples * kBgTpBusy * x.tp / (double)std::max(1, n_simd);
    }
    const double lane = k < order.size() ? c[order[k]].lane : 0.0;
    const double t = std::max(std::max(floor_lat, lane), std::max(tp_lat, issue));
    if (k == 0 || t < best) {
      best = t;
      best_k = k;
    }
  }
  for (size_t k = 0; k < best_k; ++k) tp[c[order[k]].i] = true;
}

std::vector<bool> choose_time_parallel(const std::vector<ItemSpec>& specs,
                                       int32_t tp_max_samples, int n_simd) {
  std::vector<bool> tp(specs.size(), false);
  choose_background_tp(specs, tp_max_samples, n_simd, tp);
  std::vector<std::pair<int64_t, size_t>> cand;  // (fine steps, index)
  for (size_t i = 0; i < specs.size(); ++i)
    if (!in_background(*specs[i].prob) && time_parallel_candidate(specs[i], tp_max_samples))
      cand.push_back({level_const(*specs[i].prob, specs[i].level).n_steps, i});
  if (cand.empty()) return tp;
  std::stable_sort(cand.begin(), cand.end(),
                   [](const auto& a, const auto& b) { return a.first > b.first; });
  // The one-trajectory-per-lane loop needs about (longest n_steps) x 50
  // wavefront instructions of latency however few its samples; the
  // time-parallel path costs about 8 instructions per trajectory step spread
  // over the whole GPU.  Take the longest candidates while their time-parallel
  // work stays below that latency.
  const double budget = (double)cand.front().first * (double)kTpStepsPerLongestStep;
  double used = 0.0;
  for (const auto& c : cand) {
    const double w = (double)specs[c.second].n_samples * (double)c.first;
    if (used + w > budget) break;
    used += w;
    tp[c.second] = true;
  }
  return tp;
}

LevelDesc make_desc(const ItemSpec& s, bool tp) {
  const mlmc_ap_problem& p = *s.prob;
  const bool coarse = !s.single && s.level >= 1;
  const int lc = s.coarse_level >= 0 ? s.coarse_level : s.level - 1;
  const LevelConst F = level_const(p, s.level);
  const LevelConst C = coarse ? level_const(p, lc) : F;
  // fine steps per coarse step (M for adjacent levels)
  const uint64_t mb = coarse ? block_factor(p, s.level, lc) : (uint64_t)p.M;
  const bool maxwell = p.eq_kind == MLMC_AP_EQ_MAXWELLIAN;
  const bool agg = coarse && p.coupling == MLMC_AP_COUPLING_AGGREGATE;
  LevelDesc d;
  std::memset(&d, 0, sizeof(d));
  d.h_f = F.h; d.s_f = F.s;
  d.h_c = coarse ? C.h : 0.0;
  d.s_c = coarse ? C.s : 0.0;
  d.agg_ms2 = (double)mb * F.s * F.s;
  d.h_f2 = F.h * F.h;
  d.rsqrt_m = 1.0 / std::sqrt((double)mb);
  d.x0_a = p.x0_a; d.x0_b = p.x0_b;
  if (p.qoi == MLMC_AP_QOI_X2_HIST) {
    d.hist_lo = p.hist_lo;
    d.hist_inv_w = (double)p.nbins / (p.hist_hi - p.hist_lo);
    d.nbins = (uint32_t)p.nbins;
  }
  d.sample_begin = s.sample_begin;
  d.n_samples = s.n_samples;
  d.hist = s.hist;
  d.traj = s.traj;
  d.coll = s.coll;
  d.thr_f = F.thr;
  d.thr_c2 = coarse ? coarse_threshold(F.thr, C.thr, (int)mb) : 1;
  d.thr_f_m1 = d.thr_f >= 1 ? (uint32_t)(d.thr_f - 1) : 0u;
  d.thr_c2_m1 = d.thr_c2 >= 1 ? (uint32_t)(d.thr_c2 - 1) : 0u;
  d.n_steps = (uint32_t)F.n_steps;
  d.M = (uint32_t)mb;
  d.tag = (uint32_t)s.level + (s.single ? 64u : 0u);
  d.stream = p.stream_id;
  d.key0 = (uint32_t)(p.seed & 0xFFFFFFFFull);
  d.key1 = (uint32_t)(p.seed >> 32);
  d.flags = (coarse ? kFlagCoarse : 0u) | (maxwell ? kFlagMaxwell : 0u) |
            (agg ? kFlagAggregate : 0u) | (s.hist ? kFlagHist : 0u) |
            (s.accumulate ? kFlagAccumulate : 0u) |
            ((s.hist || s.traj || s.coll) ? kFlagSampleOutputs : 0u) |
            (p.qoi == MLMC_AP_QOI_X ? kFlagQoiX : 0u);
  if (d.thr_f == 0 || d.thr_c2 == 0) d.flags |= kFlagWide;
  d.kind = coarse ? (maxwell ? (agg ? kKindPairMaxwellAggregate : kKindPairMaxwellSum)
                             : kKindPairTwoPointSum)
                  : (maxwell ? kKindFineMaxwell : kKindFineTwoPoint);
  d.x0_kind = (uint32_t)p.x0_kind;
  if (p.scheme == MLMC_AP_SCHEME_KD) {
    // the KD kinds read their constants from the coefficient slots
    d.h_f = F.dt;
    d.h_c = coarse ? C.dt : 0.0;
    d.agg_ms2 = p.T;
    d.h_f2 = 0.0;                   // Maxwellian mean mu
    d.rsqrt_m = 0.0;
    if (p.background == MLMC_AP_BG_DIFFUSIVE) {
      d.s_f = 1.0 / (p.eps * p.eps);  // collision rate R
      d.s_c = 1.0 / p.eps;            // Maxwellian standard deviation sigma
    } else {
      // Section 5: sigma = 1 and R(x) from (a, b); a = 0 runs the
      // homogeneous path with R = b
      d.s_f = p.bg_b;
      d.s_c = 1.0;
      d.rsqrt_m = p.bg_a;             // slope parameter a of the background
      if (p.bg_a > 0.0) d.flags |= p.background == MLMC_AP_BG_B1 ? kFlagBgB1 : kFlagBgB2;
    }
    d.thr_f = d.thr_c2 = 0;
    d.thr_f_m1 = d.thr_c2_m1 = 0u;
    d.flags &= ~(kFlagWide | kFlagAggregate);
    d.kind = coarse ? kKindKdPair : kKindKdFine;
  }
  const ItemLayout lay = item_layout(F.n_steps, s.n_samples);
  d.spl = lay.spl;
  d.n_tiles = lay.n_tiles;
  d.n_groups = lay.n_groups;
  d.chunk_tiles = lay.chunk_tiles;
  d.n_chunks = lay.n_chunks;
  if (tp) {  // no persistent-kernel chunks; tp_base and tp_out are set by the caller
    d.flags |= kFlagTimeParallel;
    d.n_chunks = 0;
  }
  d.result_slot = s.result_slot;
  return d;
}

Stats stats_from_api(const mlmc_ap_level_stats& a) {
  Stats s;
  s.n = (double)a.n;
  s.mean_dq = a.mean_dq; s.m2_dq = a.m2_dq;
  s.mean_qf = a.mean_qf; s.m2_qf = a.m2_qf;
  s.mean_qc = a.mean_qc; s.m2_qc = a.m2_qc;
  s.c_fc = a.c_fc;
  s.coll_f = a.coll_f; s.coll_c = a.coll_c;
  return s;
}

mlmc_ap_level_stats stats_to_api(const Stats& s) {
  mlmc_ap_level_stats a;
  a.n = (uint64_t)s.n;
  a.mean_dq = s.mean_dq; a.m2_dq = s.m2_dq;
  a.mean_qf = s.mean_qf; a.m2_qf = s.m2_qf;
  a.mean_qc = s.mean_qc; a.m2_qc = s.m2_qc;
  a.c_fc = s.c_fc;
  a.coll_f = s.coll_f; a.coll_c = s.coll_c;
  return a;
}

// ---------------------------------------------------------------------------
// Workspace.
// ---------------------------------------------------------------------------
template <typename T>
static mlmc_ap_status grow_dev(T*& p, size_t& cap, size_t need) {
  if (need <= cap && p) return MLMC_AP_OK;
  size_t n = std::max(need, cap + cap / 2);
  if (n < 64) n = 64;
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
  if (hipMalloc((void**)&p, n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(MLMC_AP_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes");
  }
  cap = n;
  return MLMC_AP_OK;
}

// Pinned host memory that kernels read and write directly (fine-grained, so
// no GPU cache holds a stale copy between launches); `dp` is its device
// address.
template <typename T>
static mlmc_ap_status grow_pinned(T*& p, T*& dp, size_t cap_old, size_t cap_new) {
  if (p && cap_old >= cap_new) return MLMC_AP_OK;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  dp = nullptr;
  if (hipHostMalloc((void**)&p, cap_new * sizeof(T), hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    return set_error(MLMC_AP_ENOMEM, "hipHostMalloc failed");
  }
  if (hipHostGetDevicePointer((void**)&dp, p, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(p);
    p = nullptr;
    dp = nullptr;
    return set_error(MLMC_AP_EDEVICE, "hipHostGetDevicePointer failed");
  }
  return MLMC_AP_OK;
}

mlmc_ap_status Workspace::ensure(size_t n_items, size_t n_tiles, size_t n_groups,
                                 size_t n_slots, size_t n_hist) {
  const void* before[8] = {items_dev, partials, groups, resident, hist_dev, items_host_dev,
                           resident_host_dev, item_done};
  if (n_items > items_cap || !items_dev || !items_host || !item_done) {
    MLMC_TRY(grow_dev(items_dev, items_cap, n_items));
    MLMC_TRY(grow_pinned(items_host, items_host_dev, 0, items_cap));
    size_t done_cap = 0;
    if (item_done) (void)hipFree(item_done);
    item_done = nullptr;
    MLMC_TRY(grow_dev(item_done, done_cap, items_cap));
  }
  if (!hdr_dev) {
    MLMC_HIP(hipMalloc((void**)&hdr_dev, sizeof(WorkHeader)));
    MLMC_HIP(hipMalloc((void**)&counter_dev, sizeof(unsigned int) * kChunkStreams * kCounterStride));
  }
  if (!hdr_host) MLMC_TRY(grow_pinned(hdr_host, hdr_host_dev, 0, 1));
  MLMC_TRY(grow_dev(partials, partials_cap, std::max<size_t>(n_tiles, 1)));
  MLMC_TRY(grow_dev(groups, groups_cap, std::max<size_t>(n_groups, 1)));
  if (n_slots > resident_cap || !resident || !resident_host) {
    MLMC_TRY(grow_dev(resident, resident_cap, std::max<size_t>(n_slots, 1)));
    MLMC_TRY(grow_pinned(resident_host, resident_host_dev, 0, resident_cap));
  }
  MLMC_TRY(grow_dev(hist_dev, hist_cap, std::max<size_t>(n_hist, 1)));
  const void* after[8] = {items_dev, partials, groups, resident, hist_dev, items_host_dev,
                          resident_host_dev, item_done};
  if (std::memcmp(before, after, sizeof(before)) != 0) drop_graphs();  // recapture
  return MLMC_AP_OK;
}

mlmc_ap_status Workspace::ensure_tp(size_t n_samples) {
  if (n_samples == 0) return MLMC_AP_OK;
  return grow_dev(tp_buf, tp_cap, n_samples);
}

void Workspace::drop_graphs() {
  for (auto& e : graphs) {
    if (e.second.exec) (void)hipGraphExecDestroy(e.second.exec);
    if (e.second.def) (void)hipGraphDestroy(e.second.def);
  }
  graphs.clear();
}

void Workspace::release() {
  drop_graphs();
  if (items_dev) (void)hipFree(items_dev);
  if (items_host) (void)hipHostFree(items_host);
  if (hdr_dev) (void)hipFree(hdr_dev);
  if (hdr_host) (void)hipHostFree(hdr_host);
  if (counter_dev) (void)hipFree(counter_dev);
  if (partials) (void)hipFree(partials);
  if (groups) (void)hipFree(groups);
  if (resident) (void)hipFree(resident);
  if (resident_host) (void)hipHostFree(resident_host);
  if (plan_host) (void)hipHostFree(plan_host);
  plan_host = nullptr;
  plan_host_dev = nullptr;
  if (hist_dev) (void)hipFree(hist_dev);
  if (tp_buf) (void)hipFree(tp_buf);
  tp_buf = nullptr;
  if (item_done) (void)hipFree(item_done);
  item_done = nullptr;
  tp_cap = 0;
  items_dev = nullptr; items_host = nullptr; hdr_dev = nullptr; hdr_host = nullptr;
  counter_dev = nullptr; partials = nullptr; groups = nullptr; resident = nullptr;
  resident_host = nullptr; hist_dev = nullptr;
  items_host_dev = nullptr; hdr_host_dev = nullptr; resident_host_dev = nullptr;
  items_cap = partials_cap = groups_cap = resident_cap = hist_cap = 0;
}

static std::mutex g_ws_mu;
static std::map<int, std::unique_ptr<Workspace>> g_ws;

Workspace::~Workspace() {
  release();
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
}

mlmc_ap_status init_workspace(Workspace& ws) {
  int dev = 0;
  MLMC_HIP(hipGetDevice(&dev));
  ws.device = dev;
  hipDeviceProp_t prop;
  MLMC_HIP(hipGetDeviceProperties(&prop, dev));
  ws.n_cu = prop.multiProcessorCount;
  ws.name = prop.gcnArchName;
  MLMC_HIP(hipStreamCreateWithFlags(&ws.capture_stream, hipStreamNonBlocking));
  for (auto& e : ws.ev) MLMC_HIP(hipEventCreate(&e));
  ws.tuning.block = 256;
  ws.tuning.ppt = 1;  // measured best on every level (one sample in flight per lane)
  ws.tuning.waves_per_simd = 4;
  return MLMC_AP_OK;
}

Workspace* workspace() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    set_error(MLMC_AP_EDEVICE, "no HIP device");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto it = g_ws.find(dev);
  if (it != g_ws.end()) return it->second.get();
  std::unique_ptr<Workspace> ws(new Workspace());
  if (init_workspace(*ws) != MLMC_AP_OK) return nullptr;
  Workspace* raw = ws.get();
  g_ws[dev] = std::move(ws);
  return raw;
}

mlmc_ap_tuning resolve_tuning(const Workspace& ws, const mlmc_ap_tuning* t) {
  mlmc_ap_tuning r = ws.tuning;
  if (t) {
    if (t->block) r.block = t->block;
    if (t->ppt) r.ppt = t->ppt;
    if (t->waves_per_simd) r.waves_per_simd = t->waves_per_simd;
    if (t->tp_max_samples) r.tp_max_samples = t->tp_max_samples;
  }
  return r;
}

int persistent_grid(Workspace& ws, const mlmc_ap_tuning& t, bool fp64, bool kd) {
  const int waves_per_block = t.block / kLanes;
  const int waves = ws.n_cu * 4 * t.waves_per_simd;
  int grid = (waves + waves_per_block - 1) / waves_per_block;
  // no more blocks than fit the GPU at once: a block that waits for a free
  // slot would start its statically assigned work (one-round launches,
  // time-parallel trajectories) only after the others finish
  const int key = (fp64 ? 1 : 0) | (kd ? 2 : 0) | (t.ppt << 2) | (t.block << 5);
  auto it = ws.blocks_per_cu.find(key);
  if (it == ws.blocks_per_cu.end())
    it = ws.blocks_per_cu.emplace(key, persistent_blocks_per_cu(fp64, t.ppt, t.block, kd)).first;
  if (it->second > 0) grid = std::min(grid, ws.n_cu * it->second);
  // every chunk stream needs blocks
  return std::max((int)kChunkStreams, grid);
}

static mlmc_ap_status check_tuning(const mlmc_ap_tuning& t) {
  if (t.block != 64 && t.block != 128 && t.block != 256)
    return set_error(MLMC_AP_EINVAL, "tuning.block must be 64, 128 or 256");
  if (t.ppt != 1 && t.ppt != 2 && t.ppt != 4)
    return set_error(MLMC_AP_EINVAL, "tuning.ppt must be 1, 2 or 4");
  if (t.waves_per_simd < 1 || t.waves_per_simd > 8)
    return set_error(MLMC_AP_EINVAL, "tuning.waves_per_simd must be in [1, 8]");
  return MLMC_AP_OK;
}

static const int kReduceGrid = 1024;

static mlmc_ap_status stage(Workspace& ws, hipStream_t s) {
  MLMC_HIP(launch_stage(ws.hdr_host_dev, ws.items_host_dev, (uint32_t)ws.items_cap, ws.hdr_dev,
                        ws.items_dev, ws.counter_dev, ws.item_done, s));
  return MLMC_AP_OK;
}

static mlmc_ap_status reduce(Workspace& ws, hipStream_t s) {
  MLMC_HIP(launch_reduce(ws.items_dev, ws.hdr_dev, ws.partials, ws.groups, ws.item_done,
                         ws.resident, ws.resident_host_dev, kReduceGrid, s));
  return MLMC_AP_OK;
}

// Grid of the per-level form's time-parallel launch.
static int tp_grid(const Workspace& ws) { return std::max(1, ws.n_cu * 8); }

// The whole launch as three kernels: stage the table, simulate (the
// persistent kernel also runs the time-parallel trajectories), reduce (which
// also writes the host mirror of the resident slots).
static mlmc_ap_status record_device_work(Workspace& ws, bool fp64, bool kd,
                                         const mlmc_ap_tuning& t, hipStream_t s) {
  MLMC_TRY(stage(ws, s));
  MLMC_HIP(launch_persistent(fp64, t.ppt, ws.items_dev, ws.hdr_dev, ws.counter_dev, ws.partials,
                             t.block, persistent_grid(ws, t, fp64, kd), s, kd));
  MLMC_TRY(reduce(ws, s));
  return MLMC_AP_OK;
}

mlmc_ap_status run_table(Workspace& ws, const std::vector<ItemSpec>& specs, size_t n_slots,
                         int mode, const mlmc_ap_tuning& tuning, hipStream_t stream,
                         LaunchTiming* timing, const PlanArgs* plan) {
  MLMC_TRY(check_tuning(tuning));
  if (specs.empty()) return MLMC_AP_OK;
  for (const auto& sp : specs)
    if (sp.n_samples == 0) return set_error(MLMC_AP_EINVAL, "work item without samples");
  std::vector<LevelDesc> d(specs.size());
  const std::vector<bool> tp = choose_time_parallel(specs, tuning.tp_max_samples, 4 * ws.n_cu);
  for (size_t i = 0; i < specs.size(); ++i) d[i] = make_desc(specs[i], tp[i]);
  const bool fp64 = specs[0].prob->fp64_state != 0;
  for (const auto& s : specs)
    if ((s.prob->fp64_state != 0) != fp64)
      return set_error(MLMC_AP_EINVAL, "one launch cannot mix FP32 and FP64 particle state");
  const bool kd = specs[0].prob->scheme == MLMC_AP_SCHEME_KD;
  for (const auto& s : specs)
    if ((s.prob->scheme == MLMC_AP_SCHEME_KD) != kd)
      return set_error(MLMC_AP_EINVAL, "one launch cannot mix particle schemes");
  // most expensive chunks first (persistent kernel load balance)
  std::stable_sort(d.begin(), d.end(), [](const LevelDesc& a, const LevelDesc& b) {
    return a.n_steps > b.n_steps;
  });
  uint64_t tiles = 0, groups = 0, chunks = 0, tp_samples = 0;
  for (auto& x : d) {
    x.tile_base = tiles;
    x.group_base = groups;
    x.chunk_base = chunks;
    tiles += x.n_tiles;
    groups += x.n_groups;
    chunks += x.n_chunks;
    if (x.flags & kFlagTimeParallel) tp_samples += x.n_samples;
  }
  if (chunks >= 0xFFFFFFF0ull || groups >= 0xFFFFFFF0ull || tp_samples >= 0xFFFFFFF0ull)
    return set_error(MLMC_AP_EINVAL, "work table too large for one launch");
  if (plan && ((mode != kModeDirect && mode != kModeTimed) || d.size() > MLMC_AP_MAX_LEVELS))
    return set_error(MLMC_AP_EINVAL, "a device-planned top-up needs a direct launch");
  MLMC_TRY(ws.ensure(d.size(), plan ? std::max<size_t>(tiles, kPlanTiles) : tiles,
                     plan ? std::max<size_t>(groups, kPlanGroups) : groups, n_slots, 0));
  MLMC_TRY(ws.ensure_tp(tp_samples));
  if (plan && !ws.plan_host) MLMC_TRY(grow_pinned(ws.plan_host, ws.plan_host_dev, 0, 1));
  uint64_t tp_off = 0;
  for (auto& x : d) {
    x.tp_base = (uint32_t)tp_off;
    if (x.flags & kFlagTimeParallel) {
      x.tp_out = ws.tp_buf + tp_off;
      tp_off += x.n_samples;
    }
  }
  const bool has_tp = tp_samples > 0;
  std::memcpy(ws.items_host, d.data(), d.size() * sizeof(LevelDesc));
  ws.hdr_host->n_items = (uint32_t)d.size();
  ws.hdr_host->total_chunks = (uint32_t)chunks;
  ws.hdr_host->total_groups = (uint32_t)groups;
  ws.hdr_host->total_tp = (uint32_t)tp_samples;

  MLMC_HIP(hipEventRecord(ws.ev[0], stream));
  bool kernel_timed = false;
  if (mode == kModePerLevel) {
    MLMC_TRY(stage(ws, stream));
    MLMC_HIP(hipEventRecord(ws.ev[1], stream));
    if (has_tp) MLMC_HIP(launch_tp(fp64, ws.items_dev, ws.hdr_dev, tp_grid(ws), stream, kd));
    for (size_t i = 0; i < d.size(); ++i)
      if (!(d[i].flags & kFlagTimeParallel))
        MLMC_HIP(launch_level(fp64, tuning.ppt, d[i].kind, ws.items_dev, (uint32_t)i,
                              d[i].n_tiles, tuning.block, ws.partials, stream));
    MLMC_HIP(hipEventRecord(ws.ev[2], stream));
    MLMC_TRY(reduce(ws, stream));
    kernel_timed = true;
  } else if (mode == kModeTimed || mode == kModeDirect || mode == kModeDirectHost) {
    kernel_timed = mode == kModeTimed;
    MLMC_TRY(stage(ws, stream));
    if (kernel_timed) MLMC_HIP(hipEventRecord(ws.ev[1], stream));
    MLMC_HIP(launch_persistent(fp64, tuning.ppt, ws.items_dev, ws.hdr_dev, ws.counter_dev,
                               ws.partials, tuning.block, persistent_grid(ws, tuning, fp64, kd),
                               stream, kd));
    if (kernel_timed) MLMC_HIP(hipEventRecord(ws.ev[2], stream));
    MLMC_TRY(reduce(ws, stream));
    if (plan) {
      // the first top-up, planned on the device from the warm-up's statistics
      PlanArgs a = *plan;
      a.n_items = (uint32_t)d.size();
      a.cap_tiles = (uint32_t)std::min<size_t>(ws.partials_cap, 0xFFFFFFF0u);
      a.cap_groups = (uint32_t)std::min<size_t>(ws.groups_cap, 0xFFFFFFF0u);
      MLMC_HIP(launch_plan(a, ws.items_dev, ws.hdr_dev, ws.resident, ws.counter_dev,
                           ws.item_done, ws.plan_host_dev, stream));
      if (kernel_timed) MLMC_HIP(hipEventRecord(ws.ev[4], stream));
      MLMC_HIP(launch_persistent(fp64, tuning.ppt, ws.items_dev, ws.hdr_dev, ws.counter_dev,
                                 ws.partials, tuning.block, persistent_grid(ws, tuning, fp64, kd),
                                 stream, kd));
      if (kernel_timed) MLMC_HIP(hipEventRecord(ws.ev[5], stream));
      MLMC_TRY(reduce(ws, stream));
    }
  } else if (mode == kModeGraph) {
    const uint64_t key = ((uint64_t)tuning.block << 48) ^ ((uint64_t)tuning.ppt << 40) ^
                         ((uint64_t)tuning.waves_per_simd << 32) ^ (fp64 ? 1ull : 2ull) ^
                         (kd ? 4ull : 0ull) ^
                         ((uint64_t)(uintptr_t)ws.partials << 3);
    auto it = ws.graphs.find(key);
    if (it == ws.graphs.end()) {
      if (ws.graphs.size() >= 16) ws.drop_graphs();  // bound the cache
      MLMC_HIP(hipStreamBeginCapture(ws.capture_stream, hipStreamCaptureModeRelaxed));
      mlmc_ap_status st = record_device_work(ws, fp64, kd, tuning, ws.capture_stream);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(ws.capture_stream, &g);
      if (st != MLMC_AP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return set_error(MLMC_AP_EDEVICE, "hipStreamEndCapture failed");
      Workspace::Graph entry;
      entry.def = g;
      if (hipGraphInstantiate(&entry.exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        return set_error(MLMC_AP_EDEVICE, "hipGraphInstantiate failed");
      }
      it = ws.graphs.emplace(key, entry).first;
    }
    MLMC_HIP(hipGraphLaunch(it->second.exec, stream));
  } else {
    return set_error(MLMC_AP_EINVAL, "unknown launch mode");
  }
  MLMC_HIP(hipEventRecord(ws.ev[3], stream));
  // Poll the launch's last event instead of a blocking wait: the MLMC loop
  // plans its next launch from these statistics, so the wake-up latency of a
  // blocking wait would sit on the critical path of every iteration.
  hipError_t q;
  while ((q = hipEventQuery(ws.ev[3])) == hipErrorNotReady) {
  }
  if (q != hipSuccess) {
    (void)hipGetLastError();
    return set_error(MLMC_AP_EDEVICE, std::string("launch failed: ") + hipGetErrorString(q));
  }
  if (timing) {
    float ms = 0.f;
    MLMC_HIP(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[3]));
    timing->total_s = ms * 1e-3;
    timing->kernel_s = 0.0;
    if (kernel_timed) {
      MLMC_HIP(hipEventElapsedTime(&ms, ws.ev[1], ws.ev[2]));
      timing->kernel_s = ms * 1e-3;
      if (plan) {
        MLMC_HIP(hipEventElapsedTime(&ms, ws.ev[4], ws.ev[5]));
        timing->kernel_s += ms * 1e-3;
      }
    }
  }
  return MLMC_AP_OK;
}

int launch_mode(int32_t batched) {
  switch (batched) {
    case -1: return kModePerLevel;
    case 0: return kModeDirect;
    case 1: return kModeGraph;
    case 2: return kModeTimed;
    case 3: return kModeDirectHost;
    default: return -1;
  }
}

// ---------------------------------------------------------------------------
// Level selection (Section 4.2, Section 5.2).
// ---------------------------------------------------------------------------
// Heuristic level set (Algorithm "Heuristic level selection approach").  The
// set opens with the coarsest adjacent pair (l-1, l) whose difference varies
// no more than level l itself; past it, a level is taken only when its
// difference variance is under half of that of the level taken before it,
// so every correction taken at least halves the previous one; L closes the
// set (the sets end at L, Section 4.1).  No such pair: L alone.
uint64_t select_levels_heuristic(const double* V, const double* Vdiff, int L) {
  if (L <= 0) return 1ull;
  int first = 1;
  while (first <= L && Vdiff[first] > V[first]) ++first;
  if (first > L) return 1ull << L;
  uint64_t set = 3ull << (first - 1);
  double last = Vdiff[first];
  for (int k = first + 1; k <= L; ++k) {
    if (2.0 * Vdiff[k] < last) {
      set |= 1ull << k;
      last = Vdiff[k];
    }
  }
  return set | (1ull << L);
}

// Warm-up depth of Section 5.3: the level whose step is nearest, in log
// scale, to the mean free time 1/R, within [1, L].
int warmup_depth(const mlmc_ap_problem& p) {
  if (p.L <= 0) return 0;
  const double R = p.background == MLMC_AP_BG_DIFFUSIVE ? 1.0 / (p.eps * p.eps) : p.bg_b;
  const double t = std::log(p.dt0 * R) / std::log((double)p.M);
  if (!(t < (double)p.L)) return p.L;
  return std::max(1, std::min(p.L, (int)std::floor(t + 0.5)));
}

// Section 5.3: measured profile up to tau, the O(dt^3) rate of the
// difference variance beyond it (each level divides it by M^3) and the level
// variance of tau.
void extrapolate_variances(const double* V, const double* Vdiff, int tau, int M, int L,
                           double* V_out, double* Vdiff_out) {
  for (int l = 0; l <= L; ++l) {
    if (l <= tau) {
      V_out[l] = V[l];
      Vdiff_out[l] = Vdiff[l];
    } else {
      V_out[l] = V[tau];
      Vdiff_out[l] = Vdiff[tau] / std::pow((double)M, 3.0 * (double)(l - tau));
    }
  }
}

// best[i]: least cost of a hierarchy ending at level i; a hierarchy is a path
// (first level) -> ... -> i, so the levels are taken in increasing order.
double select_levels_optimal(const double* V, const double* C, const double* Vpair,
                             const double* Cpair, int L, uint64_t* mask) {
  const int n = L + 1;
  std::vector<double> best(n);
  std::vector<int> prev(n, -1);
  for (int i = 0; i < n; ++i) {
    best[i] = std::sqrt(V[i] * C[i]);
    for (int j = 0; j < i; ++j) {
      const double c = best[j] + std::sqrt(Vpair[i * n + j] * Cpair[i * n + j]);
      if (c < best[i]) {
        best[i] = c;
        prev[i] = j;
      }
    }
  }
  uint64_t m = 0;
  for (int i = L; i >= 0; i = prev[i]) m |= 1ull << i;
  *mask = m;
  return best[L];
}

// ---------------------------------------------------------------------------
// MLMC control of one request.
// ---------------------------------------------------------------------------
static double wall_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void McRequest::init(const mlmc_ap_problem& p, double rmse_tol, bool plain_mc, uint64_t warmup,
                     int iters, uint64_t cap) {
  prob = p;
  tol = rmse_tol;
  plain = plain_mc;
  n_warmup = warmup;
  max_iter = iters;
  max_per_tick = cap;
  phase = 0;
  iterations = 0;
  converged = false;
  need_check = false;
  // every level the request may reach (L grows up to L_max)
  done.assign(MLMC_AP_MAX_LEVELS, 0);
  target.assign(MLMC_AP_MAX_LEVELS, 0);
  st.assign(MLMC_AP_MAX_LEVELS, stats_empty());
  coarse_of.assign(MLMC_AP_MAX_LEVELS, -1);
  in_set.assign(MLMC_AP_MAX_LEVELS, 0);
  pilot_done.assign(MLMC_AP_MAX_LEVELS, 0);
  pilot_st.assign(MLMC_AP_MAX_LEVELS, stats_empty());
  selected = false;
  level_select = MLMC_AP_LEVELS_ALL;
  tau = p.L;
  L_max = 0;
  levels_added = 0;
  prof_V.clear();
  prof_Vd.clear();
  for (int l = first_level(); l <= p.L; ++l) {
    target[l] = n_warmup;
    in_set[l] = 1;
    coarse_of[l] = (plain || l == 0) ? -1 : l - 1;
  }
  particle_steps = 0;
  launches = 0;
  gpu_seconds = kernel_seconds = 0.0;
  tols.assign(1, rmse_tol);
  stage = 0;
  stage_iter = 0;
  t_start = wall_now();
  snaps.clear();
}

void McRequest::set_selection(int mode, int lmax) {
  level_select = mode;
  L_max = lmax;
  tau = prob.L;
  if (mode == MLMC_AP_LEVELS_HEURISTIC_TAU && !plain) {
    tau = warmup_depth(prob);
    for (int l = tau + 1; l <= prob.L; ++l) {
      in_set[l] = 0;
      target[l] = 0;
    }
  }
}

void McRequest::set_sequence(const std::vector<double>& seq) {
  tols = seq;
  stage = 0;
  tol = tols[0];
}

bool McRequest::pilots_active() const {
  return level_select == MLMC_AP_LEVELS_OPTIMAL && !plain && !selected && prob.L >= 2;
}

bool McRequest::plan(std::vector<ItemSpec>& items, uint32_t slot_base,
                     unsigned long long* hist_base, size_t hist_stride) {
  if (phase == 2) return false;
  bool any = false;
  if (pilots_active()) {
    for (int i = 0; i + 2 <= prob.L; ++i) {
      if (pilot_done[i] >= n_warmup) continue;
      ItemSpec s;
      s.prob = &prob;
      s.level = prob.L;
      s.single = false;
      s.coarse_level = i;
      s.sample_begin = pilot_done[i];
      s.n_samples = n_warmup - pilot_done[i];
      if (max_per_tick && s.n_samples > max_per_tick) s.n_samples = max_per_tick;
      s.result_slot = slot_base + kPilotSlot + (uint32_t)i;
      s.hist = nullptr;
      s.traj = nullptr;
      s.coll = nullptr;
      s.accumulate = pilot_done[i] > 0;
      items.push_back(s);
      any = true;
    }
  }
  for (int l = first_level(); l <= prob.L; ++l) {
    if (!in_set[l] || done[l] >= target[l]) continue;
    uint64_t n = target[l] - done[l];
    if (max_per_tick && n > max_per_tick) n = max_per_tick;
    ItemSpec s;
    s.prob = &prob;
    s.level = l;
    // the first level of a hierarchy that does not start at 0 runs single
    // trajectories (the plain-MC counter tag, independent of the pairs)
    s.single = plain || (l > 0 && coarse_of[l] < 0);
    s.coarse_level = coarse_of[l];
    s.sample_begin = done[l];
    s.n_samples = n;
    s.result_slot = slot_base + (uint32_t)l;
    s.hist = hist_base ? hist_base + (size_t)l * hist_stride : nullptr;
    s.traj = nullptr;
    s.coll = nullptr;
    s.accumulate = done[l] > 0;  // the slot holds samples [0, done[l])
    items.push_back(s);
    any = true;
  }
  return any;
}

static double sample_var(const Stats& s) { return level_variance(s); }

uint64_t McRequest::item_cost(int l) const {
  if (plain) return sample_cost(prob, l, true);
  return pair_cost(prob, l, coarse_of[l]);
}

bool McRequest::device_plannable(PlanArgs& a) const {
  // the first launch of a one-stage estimate on a fixed level set: after it
  // the host would compute the targets of eqs. Nopt1/Noptj and launch them
  if (phase != 0 || iterations != 0 || tols.size() != 1 || L_max != 0 || max_per_tick != 0)
    return false;
  if (!plain && level_select != MLMC_AP_LEVELS_ALL) return false;
  if (pilots_active()) return false;
  std::memset(&a, 0, sizeof(a));
  a.tol = tol;
  a.slot_base = 0;
  for (int l = first_level(); l <= prob.L; ++l) {
    if (!in_set[l]) continue;
    // every level of the set runs its warm-up in this launch
    if (done[l] != 0 || target[l] != n_warmup) return false;
    a.level_mask |= 1u << l;
    a.cost[l] = item_cost(l);
  }
  return a.level_mask != 0;
}

// After the warm-up of adjacent pairs on levels 0..tau: V_l from the fine
// paths (Q_l), V_{l,l-1} from the differences, kept as the profile of every
// later selection; the new set's pairs that are not the warm-up's adjacent
// pairs start over with a warm-up of their own.
void McRequest::select_levels() {
  const int L = prob.L;
  if (!selected) {
    prof_V.assign(tau + 1, 0.0);
    prof_Vd.assign(tau + 1, 0.0);
    for (int l = 0; l <= tau; ++l) {
      const Stats& s = st[l];
      const double n1 = s.n > 1.0 ? s.n - 1.0 : 1.0;
      prof_V[l] = (l == 0 ? s.m2_dq : s.m2_qf) / n1;
      prof_Vd[l] = s.m2_dq / n1;
    }
  }
  std::vector<double> V(L + 1, 0.0), Vd(L + 1, 0.0);
  extrapolate_variances(prof_V.data(), prof_Vd.data(), std::min(tau, L), prob.M, L, V.data(),
                        Vd.data());
  uint64_t mask;
  if (level_select == MLMC_AP_LEVELS_OPTIMAL && L >= 1) {
    // eq. level_selection over every pair: measured variances where a
    // warm-up or pilot pair exists ((i, i-1) and (L, i)), eq. V_approx from
    // the correlations rho_{L,i} elsewhere
    const int n = L + 1;
    std::vector<double> C(n), rho(n, 1.0), Vp(n * n, 0.0), Cp(n * n, 1.0);
    for (int i = 0; i <= L; ++i) C[i] = (double)pair_cost(prob, i, -1);
    auto corr = [](const Stats& s) {
      const double d = std::sqrt(s.m2_qf * s.m2_qc);
      return d > 0.0 ? s.c_fc / d : 0.0;
    };
    for (int i = 0; i + 2 <= L; ++i) rho[i] = corr(pilot_st[i]);
    rho[L - 1] = corr(st[L]);
    for (int i = 1; i <= L; ++i)
      for (int j = 0; j < i; ++j) {
        double v;
        if (j == i - 1) {
          v = Vd[i];
        } else if (i == L) {
          const Stats& ps = pilot_st[j];
          v = ps.m2_dq / (ps.n > 1.0 ? ps.n - 1.0 : 1.0);
        } else {
          const double r2 = rho[i] * rho[i] + rho[j] * rho[j] - 1.0;
          v = V[i] + V[j] - 2.0 * std::sqrt(std::max(0.0, r2) * V[i] * V[j]);
        }
        Vp[i * n + j] = std::max(0.0, v);
        Cp[i * n + j] = (double)pair_cost(prob, i, j);
      }
    select_levels_optimal(V.data(), C.data(), Vp.data(), Cp.data(), L, &mask);
  } else {
    mask = select_levels_heuristic(V.data(), Vd.data(), L);
  }
  apply_levels(mask);
  selected = true;
}

void McRequest::apply_levels(uint64_t mask) {
  int prev = -1;
  for (int l = 0; l <= prob.L; ++l) {
    if (!((mask >> l) & 1ull)) {
      in_set[l] = 0;
      target[l] = done[l];
      continue;
    }
    if (coarse_of[l] != prev || done[l] == 0) {  // not an item with samples yet
      coarse_of[l] = prev;
      done[l] = 0;
      st[l] = stats_empty();
      target[l] = n_warmup;
    }
    in_set[l] = 1;
    prev = l;
  }
}

double McRequest::bias_estimate(double* se) const {
  const int L = prob.L;
  const int c = coarse_of[L];
  if (plain || !in_set[L] || c < 0 || done[L] == 0) {
    *se = std::numeric_limits<double>::quiet_NaN();
    return std::numeric_limits<double>::quiet_NaN();
  }
  const double f = std::pow((double)prob.M, (double)(L - c)) - 1.0;
  *se = std::sqrt(sample_var(st[L]) / (double)done[L]) / f;
  return std::fabs(st[L].mean_dq) / f;
}

bool McRequest::grow_finest() {
  if (prob.L >= L_max) return false;
  double se;
  const double b = bias_estimate(&se);
  if (!(b > tol / std::sqrt(2.0))) return false;
  const int L = ++prob.L;
  ++levels_added;
  if (level_select == MLMC_AP_LEVELS_HEURISTIC_TAU) {
    select_levels();
  } else {
    coarse_of[L] = L - 1;
    done[L] = 0;
    st[L] = stats_empty();
    target[L] = n_warmup;
    in_set[L] = 1;
  }
  return true;
}

void McRequest::absorb(const Stats* slots) {
  for (int l = first_level(); l <= prob.L; ++l) {
    if (!in_set[l]) continue;
    const uint64_t n_new = (uint64_t)slots[l].n;
    if (n_new > done[l]) {
      particle_steps += (n_new - done[l]) * item_cost(l);
      done[l] = n_new;
    }
    st[l] = slots[l];
  }
  if (pilots_active()) {
    for (int i = 0; i + 2 <= prob.L; ++i) {
      const Stats& ps = slots[kPilotSlot + i];
      const uint64_t n_new = (uint64_t)ps.n;
      if (n_new > pilot_done[i]) {
        particle_steps += (n_new - pilot_done[i]) * pair_cost(prob, prob.L, i);
        pilot_done[i] = n_new;
      }
      pilot_st[i] = ps;
    }
  }
  for (;;) {
    for (int l = first_level(); l <= prob.L; ++l)
      if (in_set[l] && done[l] < target[l]) return;  // the current round is not complete
    if (pilots_active())
      for (int i = 0; i + 2 <= prob.L; ++i)
        if (pilot_done[i] < n_warmup) return;
    if (phase == 0) {
      if (level_select != MLMC_AP_LEVELS_ALL && !plain && !selected) {
        select_levels();
        continue;  // warm-up of the set's new pairs, if any
      }
      phase = 1;
    } else {
      double v = 0.0;
      for (int l = first_level(); l <= prob.L; ++l)
        if (in_set[l]) v += sample_var(st[l]) / (double)done[l];
      const bool met = v <= 0.5 * tol * tol;
      if (met && grow_finest()) {  // eq. bias_constraint not yet met: one more level
        stage_iter = 0;
        continue;
      }
      if (met || stage_iter >= max_iter) {
        converged = met;
        if (stage + 1 >= tols.size()) {
          phase = 2;
          return;
        }
        // the next tolerance of the sequence starts from these samples
        snaps.emplace_back();
        fill_result(&snaps.back());
        snaps.back().seconds = wall_now() - t_start;
        ++stage;
        tol = tols[stage];
        stage_iter = 0;
        converged = false;
      }
    }
    // eqs. Nopt1/Noptj with sample variances and the deterministic costs
    // (the arithmetic of plan.hpp, which the device-planned top-up shares)
    double S = 0.0;
    for (int l = first_level(); l <= prob.L; ++l)
      if (in_set[l]) S += cost_variance_root(sample_var(st[l]), item_cost(l));
    for (int l = first_level(); l <= prob.L; ++l)
      if (in_set[l]) target[l] = level_target(sample_var(st[l]), item_cost(l), S, tol, done[l]);
    ++iterations;
    ++stage_iter;
  }
}

void McRequest::fill_result(mlmc_ap_result* out) const {
  std::memset(out, 0, sizeof(*out));
  out->L = prob.L;
  out->iterations = iterations;
  out->converged = converged ? 1 : 0;
  out->status = MLMC_AP_OK;
  double est = 0.0, var = 0.0;
  for (int l = first_level(); l <= prob.L; ++l) {
    if (!in_set[l]) continue;
    est += st[l].mean_dq;
    if (done[l]) var += sample_var(st[l]) / (double)done[l];
    out->N[l] = done[l];
    out->lv[l] = stats_to_api(st[l]);
    out->level_mask |= 1ull << l;
  }
  out->estimate = est;
  out->var_estimator = var;
  out->particle_steps = particle_steps;
  out->launches = launches;
  out->gpu_seconds = gpu_seconds;
  out->kernel_seconds = kernel_seconds;
  out->bias_estimate = bias_estimate(&out->bias_se);
  out->tau = tau;
  out->levels_added = levels_added;
  out->device_planned = device_planned;
}

}  // namespace mlmc

// ===========================================================================
// C ABI
// ===========================================================================
using namespace mlmc;

namespace {

double now_s() { return wall_now(); }

mlmc_ap_options default_options(const mlmc_ap_options* opt) {
  mlmc_ap_options o;
  std::memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.max_iter <= 0) o.max_iter = 10;
  if (o.n_warmup == 0) o.n_warmup = 1000;
  return o;
}

// Runs requests to completion, each MLMC iteration of all of them in one
// launch (mode 1/2) or with one launch per level (mode 0).
mlmc_ap_status run_requests(Workspace& ws, std::vector<McRequest>& reqs, int mode,
                            const mlmc_ap_tuning& tuning, hipStream_t stream,
                            unsigned long long* hist_dev, size_t hist_stride) {
  // per request: one statistics slot per level, then the pilot pairs' slots
  const size_t kStride = 2 * MLMC_AP_MAX_LEVELS + 2;
  const size_t n_slots = reqs.size() * kStride;
  MLMC_TRY(ws.ensure(1, 1, 1, n_slots, 0));
  // A slot's first launch overwrites it on the device; the host mirror of the
  // slots no launch has written yet reads as empty.
  for (size_t i = 0; i < n_slots; ++i) ws.resident_host[i] = stats_empty();
  for (int guard = 0; guard < 100000; ++guard) {
    std::vector<ItemSpec> items;
    std::vector<size_t> owners;
    for (size_t r = 0; r < reqs.size(); ++r) {
      const size_t before = items.size();
      unsigned long long* hb = hist_dev ? hist_dev + r * (MLMC_AP_MAX_LEVELS * hist_stride) : nullptr;
      reqs[r].plan(items, (uint32_t)(r * kStride), hb, hist_stride);
      if (items.size() > before) owners.push_back(r);
    }
    if (items.empty()) return MLMC_AP_OK;
    // A lone request's warm-up in a direct launch takes its first top-up
    // along: the device plans it from the warm-up's statistics (plan_kernel).
    PlanArgs pa;
    const bool chain = (mode == kModeDirect || mode == kModeTimed) && reqs.size() == 1 &&
                       !hist_dev && reqs[0].device_plannable(pa);
    LaunchTiming t;
    MLMC_TRY(run_table(ws, items, n_slots, mode, tuning, stream, &t, chain ? &pa : nullptr));
    if (chain) {
      // the host's own planning from the warm-up's statistics must give the
      // numbers the device launched
      McRequest& q = reqs[0];
      const PlanRecord& rec = *ws.plan_host;
      std::vector<Stats> warm(kStride, stats_empty());
      for (int l = 0; l <= q.prob.L; ++l)
        if ((pa.level_mask >> l) & 1u) warm[l] = rec.warmup[l];
      q.launches += 1;
      q.gpu_seconds += t.total_s;
      q.kernel_seconds += t.kernel_s;
      q.absorb(warm.data());
      for (int l = 0; l <= q.prob.L; ++l)
        if (((pa.level_mask >> l) & 1u) && q.target[l] != rec.target[l])
          return set_error(MLMC_AP_EDEVICE, "device-planned top-up of level " + std::to_string(l) +
                                                " differs from the host's sample number");
      if (!rec.declined) {
        q.launches += 1;
        q.device_planned += 1;
        q.absorb(ws.resident_host);
      }
      continue;
    }
    for (size_t r : owners) {
      reqs[r].launches += 1;
      reqs[r].gpu_seconds += t.total_s;
      reqs[r].kernel_seconds += t.kernel_s;
      reqs[r].absorb(ws.resident_host + r * kStride);
    }
  }
  return set_error(MLMC_AP_EDEVICE, "MLMC loop did not terminate");
}

}  // namespace

extern "C" {

mlmc_ap_status mlmc_ap_init(void) {
  Workspace* ws = workspace();
  if (!ws) return MLMC_AP_EDEVICE;
  void* scratch = nullptr;  // the allocation-free entry point's array on this device
  MLMC_HIP(scratch_address(&scratch));
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_release(void) {
  Workspace* ws = workspace();
  if (!ws) return MLMC_AP_EDEVICE;
  std::lock_guard<std::mutex> lk(ws->mu);
  ws->release();
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_set_tuning(const mlmc_ap_tuning* tuning_host) {
  if (!tuning_host) return set_error(MLMC_AP_EINVAL, "tuning is NULL");
  Workspace* ws = workspace();
  if (!ws) return MLMC_AP_EDEVICE;
  std::lock_guard<std::mutex> lk(ws->mu);
  const mlmc_ap_tuning t = resolve_tuning(*ws, tuning_host);
  MLMC_TRY(check_tuning(t));
  ws->tuning = t;
  return MLMC_AP_OK;
}

const char* mlmc_ap_status_str(mlmc_ap_status s) {
  switch (s) {
    case MLMC_AP_OK: return "ok";
    case MLMC_AP_EINVAL: return "invalid argument";
    case MLMC_AP_ENOMEM: return "out of memory";
    case MLMC_AP_EDEVICE: return "device error";
    case MLMC_AP_EBUSY: return "request exceeds the memory budget";
    case MLMC_AP_ECANCELLED: return "cancelled";
    case MLMC_AP_ENOTFOUND: return "unknown ticket";
    case MLMC_AP_EAGAIN: return "not finished";
  }
  return "unknown status";
}

const char* mlmc_ap_last_error(void) { return g_last_error.c_str(); }

const char* mlmc_ap_version(void) { return "mlmc_ap 0.1 (gfx950)"; }

mlmc_ap_status mlmc_ap_validate(const mlmc_ap_problem* p) { return validate_problem(p); }

mlmc_ap_status mlmc_ap_level_constants(const mlmc_ap_problem* p, int32_t level,
                                       mlmc_ap_level_info* out) {
  MLMC_TRY(validate_problem(p));
  if (!out) return set_error(MLMC_AP_EINVAL, "out is NULL");
  if (level < 0 || level > p->L) return set_error(MLMC_AP_EINVAL, "level must be in [0, L]");
  std::memset(out, 0, sizeof(*out));
  const LevelConst F = level_const(*p, level);
  out->dt = F.dt; out->h = F.h; out->s = F.s; out->p = F.p;
  out->n_steps = F.n_steps;
  out->thr_f = F.thr;
  if (level >= 1) {
    const LevelConst C = level_const(*p, level - 1);
    out->dt_c = C.dt; out->h_c = C.h; out->s_c = C.s; out->p_c = C.p;
    out->thr_c = C.thr;
    out->thr_c2 = coarse_threshold(F.thr, C.thr, p->M);
  }
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_select_levels_heuristic(const double* V_host, const double* Vdiff_host,
                                               int32_t L, uint64_t* mask_out) {
  if (!V_host || !Vdiff_host || !mask_out) return set_error(MLMC_AP_EINVAL, "NULL argument");
  if (L < 0 || L >= MLMC_AP_MAX_LEVELS) return set_error(MLMC_AP_EINVAL, "L must be in [0, 30]");
  for (int l = 0; l <= L; ++l)
    if (!(V_host[l] >= 0.0) || (l > 0 && !(Vdiff_host[l] >= 0.0)))
      return set_error(MLMC_AP_EINVAL, "variances must be >= 0");
  *mask_out = select_levels_heuristic(V_host, Vdiff_host, L);
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_warmup_depth(const mlmc_ap_problem* p, int32_t* tau_out) {
  if (!tau_out) return set_error(MLMC_AP_EINVAL, "tau_out is NULL");
  MLMC_TRY(validate_problem(p));
  *tau_out = warmup_depth(*p);
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_extrapolate_variances(const double* V_host, const double* Vdiff_host,
                                             int32_t tau, int32_t M, int32_t L,
                                             double* V_out_host, double* Vdiff_out_host) {
  if (!V_host || !Vdiff_host || !V_out_host || !Vdiff_out_host)
    return set_error(MLMC_AP_EINVAL, "NULL argument");
  if (L < 0 || L > MLMC_AP_MAX_LEVELS - 1 || tau < 0 || tau > L || M < 2 || M > 64)
    return set_error(MLMC_AP_EINVAL, "need 0 <= tau <= L <= 30 and 2 <= M <= 64");
  for (int l = 0; l <= tau; ++l)
    if (!(V_host[l] >= 0.0) || (l > 0 && !(Vdiff_host[l] >= 0.0)) || !std::isfinite(V_host[l]))
      return set_error(MLMC_AP_EINVAL, "variances must be finite and >= 0");
  extrapolate_variances(V_host, Vdiff_host, tau, M, L, V_out_host, Vdiff_out_host);
  Vdiff_out_host[0] = 0.0;
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_select_levels_optimal(const double* V_host, const double* C_host,
                                             const double* Vpair_host, const double* Cpair_host,
                                             int32_t L, uint64_t* mask_out, double* cost_out) {
  if (!V_host || !C_host || !Vpair_host || !Cpair_host || !mask_out)
    return set_error(MLMC_AP_EINVAL, "NULL argument");
  if (L < 0 || L >= MLMC_AP_MAX_LEVELS) return set_error(MLMC_AP_EINVAL, "L must be in [0, 30]");
  const int n = L + 1;
  for (int i = 0; i < n; ++i) {
    if (!(V_host[i] >= 0.0) || !(C_host[i] > 0.0))
      return set_error(MLMC_AP_EINVAL, "V must be >= 0 and C > 0");
    for (int j = 0; j < i; ++j)
      if (!(Vpair_host[i * n + j] >= 0.0) || !(Cpair_host[i * n + j] > 0.0))
        return set_error(MLMC_AP_EINVAL, "V must be >= 0 and C > 0");
  }
  const double c = select_levels_optimal(V_host, C_host, Vpair_host, Cpair_host, L, mask_out);
  if (cost_out) *cost_out = c;
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_optimal_samples(const double* V, const double* C, int32_t n, double tol,
                                       uint64_t* N) {
  if (!V || !C || !N || n < 1) return set_error(MLMC_AP_EINVAL, "bad arrays");
  if (!(tol > 0.0)) return set_error(MLMC_AP_EINVAL, "tol must be > 0");
  double S = 0.0;
  for (int i = 0; i < n; ++i) {
    if (!(V[i] >= 0.0) || !(C[i] > 0.0)) return set_error(MLMC_AP_EINVAL, "need V >= 0, C > 0");
    S += std::sqrt(V[i] * C[i]);
  }
  for (int i = 0; i < n; ++i) {
    const double x = std::ceil(2.0 / (tol * tol) * std::sqrt(V[i] / C[i]) * S);
    N[i] = x >= 1.8e19 ? UINT64_MAX : (uint64_t)x;
  }
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_merge_stats(const mlmc_ap_level_stats* a, const mlmc_ap_level_stats* b,
                                   mlmc_ap_level_stats* out) {
  if (!a || !b || !out) return set_error(MLMC_AP_EINVAL, "NULL argument");
  *out = stats_to_api(stats_merge(stats_from_api(*a), stats_from_api(*b)));
  return MLMC_AP_OK;
}

static mlmc_ap_status simulate_common(const mlmc_ap_problem* p, int32_t level, int32_t single,
                                      int32_t coarse_level, uint64_t sample_begin,
                                      uint64_t n_samples, mlmc_ap_level_stats* out_host,
                                      void* traj_dev, uint32_t* coll_dev, uint64_t* hist_host,
                                      void* stream) {
  MLMC_TRY(validate_problem(p));
  if (!out_host) return set_error(MLMC_AP_EINVAL, "out_host is NULL");
  if (level < 0 || level > p->L) return set_error(MLMC_AP_EINVAL, "level must be in [0, L]");
  if (single != 0 && single != 1) return set_error(MLMC_AP_EINVAL, "single must be 0 or 1");
  if (sample_begin > 4294967296ull || n_samples > 4294967296ull - sample_begin)
    return set_error(MLMC_AP_EINVAL, "sample_begin + n_samples must not exceed 2^32");
  const bool hist = p->qoi == MLMC_AP_QOI_X2_HIST;
  if (hist && !hist_host)
    return set_error(MLMC_AP_EINVAL, "hist_host is required with QOI_X2_HIST");
  Workspace* ws = workspace();
  if (!ws) return MLMC_AP_EDEVICE;
  std::lock_guard<std::mutex> lk(ws->mu);
  hipStream_t s = (hipStream_t)stream;
  std::memset(out_host, 0, sizeof(*out_host));
  if (n_samples == 0) {
    if (hist) std::memset(hist_host, 0, sizeof(uint64_t) * (3 * (size_t)p->nbins + 4));
    return MLMC_AP_OK;
  }
  const size_t hist_n = hist ? 3 * (size_t)p->nbins + 4 : 0;
  MLMC_TRY(ws->ensure(1, 1, 1, 1, hist_n));
  if (hist) MLMC_HIP(launch_fill_u64(ws->hist_dev, hist_n, 0ull, s));
  ItemSpec it;
  it.prob = p;
  it.level = level;
  it.single = single != 0;
  it.coarse_level = coarse_level;
  it.sample_begin = sample_begin;
  it.n_samples = n_samples;
  it.result_slot = 0;
  it.hist = hist ? ws->hist_dev : nullptr;
  it.traj = traj_dev;
  it.coll = coll_dev;
  it.accumulate = false;
  const mlmc_ap_tuning t = resolve_tuning(*ws, nullptr);
  MLMC_TRY(run_table(*ws, std::vector<ItemSpec>{it}, 1, kModePerLevel, t, s, nullptr));
  *out_host = stats_to_api(ws->resident_host[0]);
  if (hist) {
    MLMC_HIP(hipMemcpy(hist_host, ws->hist_dev, hist_n * sizeof(uint64_t), hipMemcpyDeviceToHost));
  }
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_simulate_level(const mlmc_ap_problem* p, int32_t level, int32_t single,
                                      uint64_t sample_begin, uint64_t n_samples,
                                      mlmc_ap_level_stats* out_host, void* traj_dev,
                                      uint32_t* coll_dev, uint64_t* hist_host, void* stream) {
  return simulate_common(p, level, single, -1, sample_begin, n_samples, out_host, traj_dev,
                         coll_dev, hist_host, stream);
}

// The allocation-free form of mlmc_ap_simulate_level: the same per-level
// kernels, with every buffer they need (descriptor, tile and group records,
// reduction counter, statistics slot, histogram counters) in the device
// scratch array of kernels.hip instead of the library workspace.  No hipMalloc,
// hipHostMalloc, stream or event is created: the descriptor travels as kernel
// arguments and the results come back by asynchronous copies on `stream`.
// The time-parallel path is not used (it would need per-sample staging);
// results are bitwise those of mlmc_ap_simulate_level either way.
static std::mutex g_scratch_call_mu;
static_assert(kScratchMaxSamples == MLMC_AP_NOALLOC_MAX_SAMPLES, "header limit");
static_assert(kScratchBytes == MLMC_AP_NOALLOC_SCRATCH_BYTES, "header size");
static_assert(kScratchHistCounters == 3 * MLMC_AP_MAX_BINS + 4, "histogram counters");

mlmc_ap_status mlmc_ap_simulate_level_noalloc(const mlmc_ap_problem* p, int32_t level,
                                              int32_t single, uint64_t sample_begin,
                                              uint64_t n_samples, mlmc_ap_level_stats* out_host,
                                              void* traj_dev, uint32_t* coll_dev,
                                              uint64_t* hist_host, void* stream) {
  MLMC_TRY(validate_problem(p));
  if (!out_host) return set_error(MLMC_AP_EINVAL, "out_host is NULL");
  if (level < 0 || level > p->L) return set_error(MLMC_AP_EINVAL, "level must be in [0, L]");
  if (single != 0 && single != 1) return set_error(MLMC_AP_EINVAL, "single must be 0 or 1");
  if (sample_begin > 4294967296ull || n_samples > 4294967296ull - sample_begin)
    return set_error(MLMC_AP_EINVAL, "sample_begin + n_samples must not exceed 2^32");
  if (n_samples > kScratchMaxSamples)
    return set_error(MLMC_AP_EINVAL, "n_samples exceeds MLMC_AP_NOALLOC_MAX_SAMPLES (2^22) of "
                                     "the allocation-free entry point");
  const bool hist = p->qoi == MLMC_AP_QOI_X2_HIST;
  if (hist && !hist_host)
    return set_error(MLMC_AP_EINVAL, "hist_host is required with QOI_X2_HIST");
  const size_t hist_n = hist ? 3 * (size_t)p->nbins + 4 : 0;
  std::memset(out_host, 0, sizeof(*out_host));
  if (n_samples == 0) {
    if (hist) std::memset(hist_host, 0, sizeof(uint64_t) * hist_n);
    return MLMC_AP_OK;
  }
  void* base = nullptr;
  MLMC_HIP(scratch_address(&base));
  unsigned char* b = static_cast<unsigned char*>(base);
  WorkHeader* hdr = reinterpret_cast<WorkHeader*>(b);
  LevelDesc* item = reinterpret_cast<LevelDesc*>(b + 256);
  unsigned int* item_done = reinterpret_cast<unsigned int*>(b + 512);
  Stats* resident = reinterpret_cast<Stats*>(b + 768);
  unsigned long long* hist_dev = reinterpret_cast<unsigned long long*>(b + kScratchHistOffset);
  Stats* groups = reinterpret_cast<Stats*>(b + kScratchGroupsOffset);
  Stats* partials = reinterpret_cast<Stats*>(b + kScratchTilesOffset);

  ItemSpec it;
  it.prob = p;
  it.level = level;
  it.single = single != 0;
  it.coarse_level = -1;
  it.sample_begin = sample_begin;
  it.n_samples = n_samples;
  it.result_slot = 0;
  it.hist = hist ? hist_dev : nullptr;
  it.traj = traj_dev;
  it.coll = coll_dev;
  it.accumulate = false;
  const LevelDesc d = make_desc(it, false);  // tile_base = group_base = 0
  if (d.n_tiles > kScratchMaxTiles || d.n_groups > kScratchMaxGroups)
    return set_error(MLMC_AP_EINVAL, "work item does not fit the scratch array");
  WorkHeader h;
  h.n_items = 1;
  h.total_chunks = d.n_chunks;
  h.total_groups = d.n_groups;
  h.total_tp = 0;
  hipStream_t s = (hipStream_t)stream;
  Stats host_stats;
  // every call on a device shares its scratch array: one call at a time
  std::lock_guard<std::mutex> lk(g_scratch_call_mu);
  MLMC_HIP(launch_stage_args(h, d, hdr, item, item_done, hist_dev, (uint32_t)hist_n, s));
  MLMC_HIP(launch_level(p->fp64_state != 0, 1, d.kind, item, 0, d.n_tiles, 256, partials, s));
  MLMC_HIP(launch_reduce(item, hdr, partials, groups, item_done, resident, nullptr,
                         (int)std::min<uint32_t>(d.n_groups, 1024u), s));
  MLMC_HIP(hipMemcpyAsync(&host_stats, resident, sizeof(Stats), hipMemcpyDeviceToHost, s));
  if (hist)
    MLMC_HIP(hipMemcpyAsync(hist_host, hist_dev, sizeof(uint64_t) * hist_n,
                            hipMemcpyDeviceToHost, s));
  MLMC_HIP(hipStreamSynchronize(s));
  *out_host = stats_to_api(host_stats);
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_simulate_pair(const mlmc_ap_problem* p, int32_t level, int32_t coarse_level,
                                     uint64_t sample_begin, uint64_t n_samples,
                                     mlmc_ap_level_stats* out_host, void* traj_dev,
                                     uint32_t* coll_dev, uint64_t* hist_host, void* stream) {
  if (!p) return set_error(MLMC_AP_EINVAL, "problem is NULL");
  if (level < 1 || coarse_level < 0 || coarse_level >= level)
    return set_error(MLMC_AP_EINVAL, "a pair needs 0 <= coarse_level < level");
  return simulate_common(p, level, 0, coarse_level, sample_begin, n_samples, out_host, traj_dev,
                         coll_dev, hist_host, stream);
}

mlmc_ap_status mlmc_ap_kd_coarse_numbers(const mlmc_ap_problem* p, int32_t level,
                                         int32_t coarse_level, uint64_t sample_begin,
                                         uint64_t n_samples, uint32_t max_rows, double* rows_dev,
                                         uint32_t* counts_dev, void* stream) {
  if (!p) return set_error(MLMC_AP_EINVAL, "problem is NULL");
  // the coarse step may exceed T here (the paper's table runs coarse steps up
  // to 64 fine steps from T/2), so T/dt0 need not be an integer: the rest of
  // the problem is checked with dt0 = T
  mlmc_ap_problem q = *p;
  q.dt0 = q.T;
  q.L = std::max(q.L, level);
  MLMC_TRY(validate_problem(&q));
  if (!(p->dt0 > 0.0) || !std::isfinite(p->dt0))
    return set_error(MLMC_AP_EINVAL, "dt0 must be > 0");
  if (p->scheme != MLMC_AP_SCHEME_KD)
    return set_error(MLMC_AP_EINVAL, "coarse numbers are those of the KD scheme");
  if (level < 1 || level >= MLMC_AP_MAX_LEVELS || coarse_level < 0 || coarse_level >= level)
    return set_error(MLMC_AP_EINVAL, "a pair needs 0 <= coarse_level < level <= 30");
  if (sample_begin > 4294967296ull || n_samples > 4294967296ull - sample_begin)
    return set_error(MLMC_AP_EINVAL, "sample_begin + n_samples must not exceed 2^32");
  if (max_rows < 1) return set_error(MLMC_AP_EINVAL, "max_rows must be >= 1");
  if (n_samples == 0) return MLMC_AP_OK;
  if (!rows_dev || !counts_dev) return set_error(MLMC_AP_EINVAL, "rows_dev / counts_dev is NULL");
  // fine steps up to the end of the last coarse step (which may lie past T):
  // what bounds the pair loops
  const double dtc = p->dt0 / std::pow((double)p->M, (double)coarse_level);
  const double K = std::pow((double)p->M, (double)(level - coarse_level));
  const double steps = std::ceil(p->T / dtc - 1e-9) * K;
  if (steps >= 1073741824.0) return set_error(MLMC_AP_EINVAL, "too many fine steps");
  ItemSpec it;
  it.prob = p;
  it.level = level;
  it.single = false;
  it.coarse_level = coarse_level;
  it.sample_begin = sample_begin;
  it.n_samples = n_samples;
  it.result_slot = 0;
  it.hist = nullptr;
  it.traj = nullptr;
  it.coll = nullptr;
  it.accumulate = false;
  LevelDesc d = make_desc(it, false);
  d.n_steps = (uint32_t)std::max(1.0, steps);  // bounds the KD step loops (2 n + 4)
  hipStream_t s = (hipStream_t)stream;
  MLMC_HIP(launch_kd_numbers(d, n_samples, max_rows, rows_dev, counts_dev, s));
  MLMC_HIP(hipStreamSynchronize(s));
  return MLMC_AP_OK;
}

// stages > 0: one request run through the tolerance sequence
// tols[0] 2^(-r/2), r = 0..stages-1; out receives one result per stage.
static mlmc_ap_status estimate_common(const mlmc_ap_problem* p, const double* tols, int32_t n_req,
                                      bool plain, const mlmc_ap_options* opt,
                                      mlmc_ap_result* out, uint64_t* hist_host, void* stream,
                                      int32_t stages = 0) {
  if (n_req < 1 || !p || !tols || !out) return set_error(MLMC_AP_EINVAL, "bad arguments");
  for (int i = 0; i < n_req; ++i) {
    MLMC_TRY(validate_problem(&p[i]));
    if (!(tols[i] > 0.0) || !std::isfinite(tols[i]))
      return set_error(MLMC_AP_EINVAL, "rmse_tol must be > 0");
    if ((p[i].fp64_state != 0) != (p[0].fp64_state != 0))
      return set_error(MLMC_AP_EINVAL, "a batch cannot mix FP32 and FP64 particle state");
    if (p[i].scheme != p[0].scheme)
      return set_error(MLMC_AP_EINVAL, "a batch cannot mix particle schemes");
  }
  const mlmc_ap_options o = default_options(opt);
  const int mode = launch_mode(o.batched);
  if (mode < 0) return set_error(MLMC_AP_EINVAL, "options.batched must be -1, 0, 1, 2 or 3");
  if (o.level_select < MLMC_AP_LEVELS_ALL || o.level_select > MLMC_AP_LEVELS_HEURISTIC_TAU)
    return set_error(MLMC_AP_EINVAL, "options.level_select must be 0, 1, 2 or 3");
  if (o.level_select != MLMC_AP_LEVELS_ALL && hist_host)
    return set_error(MLMC_AP_EINVAL, "level selection does not support per-level histograms");
  if (o.level_select == MLMC_AP_LEVELS_HEURISTIC_TAU && p[0].scheme != MLMC_AP_SCHEME_KD)
    return set_error(MLMC_AP_EINVAL,
                     "LEVELS_HEURISTIC_TAU needs the KD scheme (its O(dt^3) variance rate)");
  if (o.L_max != 0) {
    if (plain) return set_error(MLMC_AP_EINVAL, "plain Monte Carlo has no adaptive L_max");
    if (hist_host) return set_error(MLMC_AP_EINVAL, "L_max does not support histograms");
    if (o.level_select != MLMC_AP_LEVELS_ALL && o.level_select != MLMC_AP_LEVELS_HEURISTIC_TAU)
      return set_error(MLMC_AP_EINVAL, "L_max needs LEVELS_ALL or LEVELS_HEURISTIC_TAU");
    for (int i = 0; i < n_req; ++i) {
      if (o.L_max <= p[i].L || o.L_max > MLMC_AP_MAX_LEVELS - 1)
        return set_error(MLMC_AP_EINVAL, "options.L_max must be 0 or in (L, 30]");
      mlmc_ap_problem q = p[i];
      q.L = o.L_max;
      MLMC_TRY(validate_problem(&q));
    }
  }
  Workspace* ws = workspace();
  if (!ws) return MLMC_AP_EDEVICE;
  std::lock_guard<std::mutex> lk(ws->mu);
  const mlmc_ap_tuning t = resolve_tuning(*ws, &o.tuning);
  MLMC_TRY(check_tuning(t));
  const double t0 = now_s();
  std::vector<McRequest> reqs(n_req);
  for (int i = 0; i < n_req; ++i) {
    reqs[i].init(p[i], tols[i], plain, o.n_warmup, o.max_iter, 0);
    reqs[i].set_selection(o.level_select, o.L_max);
  }
  if (stages > 0) {
    std::vector<double> seq(stages);
    for (int r = 0; r < stages; ++r) seq[r] = tols[0] / std::sqrt(std::ldexp(1.0, r));
    reqs[0].set_sequence(seq);
  }
  // histogram counters (single request with QOI_X2_HIST)
  size_t hist_stride = 0;
  unsigned long long* hist_dev = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (n_req == 1 && p[0].qoi == MLMC_AP_QOI_X2_HIST && hist_host) {
    hist_stride = 3 * (size_t)p[0].nbins + 4;
    MLMC_TRY(ws->ensure(1, 1, 1, MLMC_AP_MAX_LEVELS, hist_stride * MLMC_AP_MAX_LEVELS));
    MLMC_HIP(launch_fill_u64(ws->hist_dev, hist_stride * MLMC_AP_MAX_LEVELS, 0ull, s));
    hist_dev = ws->hist_dev;
  }
  MLMC_TRY(run_requests(*ws, reqs, mode, t, s, hist_dev, hist_stride));
  const double el = now_s() - t0;
  if (stages > 0) {
    const McRequest& q = reqs[0];
    if (q.snaps.size() + 1 != (size_t)stages)
      return set_error(MLMC_AP_EDEVICE, "tolerance sequence ended early");
    for (int r = 0; r + 1 < stages; ++r) out[r] = q.snaps[r];
    q.fill_result(&out[stages - 1]);
    out[stages - 1].seconds = el;
    return MLMC_AP_OK;
  }
  for (int i = 0; i < n_req; ++i) {
    reqs[i].fill_result(&out[i]);
    out[i].seconds = el;
  }
  if (hist_dev) {
    MLMC_HIP(hipMemcpy(hist_host, hist_dev, sizeof(uint64_t) * hist_stride * (p[0].L + 1),
                       hipMemcpyDeviceToHost));
  }
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_estimate(const mlmc_ap_problem* p, double rmse_tol,
                                const mlmc_ap_options* opt, mlmc_ap_result* out_host,
                                uint64_t* hist_host, void* stream) {
  return estimate_common(p, &rmse_tol, 1, false, opt, out_host, hist_host, stream);
}

mlmc_ap_status mlmc_ap_estimate_sequence(const mlmc_ap_problem* p, double rmse_tol0,
                                         int32_t R, const mlmc_ap_options* opt,
                                         mlmc_ap_result* out_host, void* stream) {
  if (R < 0 || R > 40) return set_error(MLMC_AP_EINVAL, "R must be in [0, 40]");
  return estimate_common(p, &rmse_tol0, 1, false, opt, out_host, nullptr, stream, R + 1);
}

mlmc_ap_status mlmc_ap_plain_mc(const mlmc_ap_problem* p, double rmse_tol,
                                const mlmc_ap_options* opt, mlmc_ap_result* out_host,
                                void* stream) {
  return estimate_common(p, &rmse_tol, 1, true, opt, out_host, nullptr, stream);
}

mlmc_ap_status mlmc_ap_estimate_batch(const mlmc_ap_problem* p, const double* rmse_tol,
                                      int32_t n_req, const mlmc_ap_options* opt,
                                      mlmc_ap_result* out_host, void* stream) {
  return estimate_common(p, rmse_tol, n_req, false, opt, out_host, nullptr, stream);
}

mlmc_ap_status mlmc_ap_philox_words(uint64_t seed, uint32_t stream_id, uint32_t tag,
                                    uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps,
                                    uint32_t* out_dev, void* stream) {
  if (!out_dev && n_samples && n_steps) return set_error(MLMC_AP_EINVAL, "out_dev is NULL");
  if (sample_begin + n_samples > 4294967296ull)
    return set_error(MLMC_AP_EINVAL, "sample indices must stay below 2^32");
  MLMC_HIP(launch_words((uint32_t)seed, (uint32_t)(seed >> 32), stream_id, tag, sample_begin,
                        n_samples, n_steps, out_dev, (hipStream_t)stream));
  MLMC_HIP(hipStreamSynchronize((hipStream_t)stream));
  return MLMC_AP_OK;
}

mlmc_ap_status mlmc_ap_rng_normals(uint64_t seed, uint32_t stream_id, uint32_t tag,
                                   uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps,
                                   int32_t fp64, void* out_dev, void* stream) {
  if (!out_dev && n_samples && n_steps) return set_error(MLMC_AP_EINVAL, "out_dev is NULL");
  if (fp64 != 0 && fp64 != 1) return set_error(MLMC_AP_EINVAL, "fp64 must be 0 or 1");
  if (sample_begin + n_samples > 4294967296ull)
    return set_error(MLMC_AP_EINVAL, "sample indices must stay below 2^32");
  MLMC_HIP(launch_normals(fp64 != 0, (uint32_t)seed, (uint32_t)(seed >> 32), stream_id, tag,
                          sample_begin, n_samples, n_steps, out_dev, (hipStream_t)stream));
  MLMC_HIP(hipStreamSynchronize((hipStream_t)stream));
  return MLMC_AP_OK;
}

}  // extern "C"
