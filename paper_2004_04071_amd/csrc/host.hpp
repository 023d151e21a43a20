// Internal host-side machinery shared by the C ABI entry points (host.cpp)
// and the serving loop (server.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "mlmc_ap.h"
#include "plan.hpp"
#include "types.hpp"

namespace mlmc {

mlmc_ap_status set_error(mlmc_ap_status s, const std::string& msg);

#define MLMC_HIP(expr)                                                                \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::mlmc::set_error(MLMC_AP_EDEVICE,                                      \
                               std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

#define MLMC_TRY(expr)                          \
  do {                                          \
    mlmc_ap_status s_ = (expr);                 \
    if (s_ != MLMC_AP_OK) return s_;            \
  } while (0)

// Host-side constants of one level (FP64).
struct LevelConst {
  double dt, h, s, p;
  uint64_t n_steps;
  uint64_t thr;
};

LevelConst level_const(const mlmc_ap_problem& p, int level);
uint64_t coarse_threshold(uint64_t thr_f, uint64_t thr_c, int M);
mlmc_ap_status validate_problem(const mlmc_ap_problem* p);
// Particle steps of one sample: n_l (+ n_{l-1} for a pair at l >= 1).
uint64_t sample_cost(const mlmc_ap_problem& p, int level, bool single);
// The same for a pair whose coarse path is at level coarse_level (< level).
uint64_t pair_cost(const mlmc_ap_problem& p, int level, int coarse_level);
// Fine steps per coarse step of a pair (level, coarse_level): M^(level - coarse_level).
uint64_t block_factor(const mlmc_ap_problem& p, int level, int coarse_level);
// Level selection (see the C ABI): bit masks of the selected levels.
uint64_t select_levels_heuristic(const double* V, const double* Vdiff, int L);
int warmup_depth(const mlmc_ap_problem& p);
void extrapolate_variances(const double* V, const double* Vdiff, int tau, int M, int L,
                           double* V_out, double* Vdiff_out);
double select_levels_optimal(const double* V, const double* C, const double* Vpair,
                             const double* Cpair, int L, uint64_t* mask);

// One work item request: a sample range of one level of one problem.
struct ItemSpec {
  const mlmc_ap_problem* prob;
  int level;
  bool single;
  int coarse_level = -1;     // coarse path of a pair: this level (< level), or -1 for level - 1
  uint64_t sample_begin, n_samples;
  uint32_t result_slot;
  unsigned long long* hist;  // device histogram counters or null
  void* traj;
  uint32_t* coll;
  bool accumulate = true;    // merge into the result slot (else overwrite it)
};

// Time-parallel path (few long trajectories; see the tuning documentation of
// the C ABI): an item qualifies with at most tp_max_samples samples
// (0 = kTpDefaultMaxSamples) of >= 64 fine steps; of the qualifying items of a
// launch the longest are taken while their trajectory steps stay within
// kTpStepsPerLongestStep times the longest item's step count.  KD items in a
// background of Section 5 are chosen by a latency estimate of their own
// (n_simd: SIMDs of the device).  Results do not depend on the choice.
constexpr int64_t kTpDefaultMaxSamples = 4096;
constexpr int64_t kTpStepsPerLongestStep = 4096;
bool time_parallel_candidate(const ItemSpec& s, int32_t tp_max_samples);
std::vector<bool> choose_time_parallel(const std::vector<ItemSpec>& specs,
                                       int32_t tp_max_samples, int n_simd);
LevelDesc make_desc(const ItemSpec& s, bool tp);

// Device workspace of one device: work table, tile partials, group results,
// resident statistics, histogram counters, pinned staging, captured graph.
struct Workspace {
  int device = -1;
  int n_cu = 0;
  std::string name;
  std::mutex mu;
  hipStream_t capture_stream = nullptr;
  // launch start, particle kernel start/end, launch end; particle kernel
  // start/end of a device-planned top-up
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};

  // *_host: pinned host memory the kernels access directly at *_host_dev
  LevelDesc* items_dev = nullptr;
  LevelDesc* items_host = nullptr;
  LevelDesc* items_host_dev = nullptr;
  size_t items_cap = 0;
  WorkHeader* hdr_dev = nullptr;
  WorkHeader* hdr_host = nullptr;
  WorkHeader* hdr_host_dev = nullptr;
  unsigned int* counter_dev = nullptr;
  Stats* partials = nullptr;
  size_t partials_cap = 0;  // tiles
  Stats* groups = nullptr;
  size_t groups_cap = 0;
  Stats* resident = nullptr;
  Stats* resident_host = nullptr;  // written by the item reduction
  Stats* resident_host_dev = nullptr;
  size_t resident_cap = 0;  // slots
  unsigned long long* hist_dev = nullptr;
  size_t hist_cap = 0;      // counters
  unsigned int* item_done = nullptr;  // reduction: finished groups per item (items_cap)
  TpSample* tp_buf = nullptr;  // final states of time-parallel samples
  size_t tp_cap = 0;
  PlanRecord* plan_host = nullptr;  // device-planned top-up: the plan kernel's record
  PlanRecord* plan_host_dev = nullptr;

  // Captured launches by shape (tuning, precision, time-parallel node); every
  // buffer they name is in the workspace, so any reallocation drops them all.
  struct Graph {
    hipGraph_t def = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::map<uint64_t, Graph> graphs;
  std::map<int, int> blocks_per_cu;  // persistent-kernel occupancy by (precision, ppt, block)
  void drop_graphs();

  mlmc_ap_tuning tuning{};      // current default (autotuned or built-in)
  bool tuned = false;

  ~Workspace();

  mlmc_ap_status ensure(size_t n_items, size_t n_tiles, size_t n_groups, size_t n_slots,
                        size_t n_hist);
  mlmc_ap_status ensure_tp(size_t n_samples);
  void release();
};

Workspace* workspace();  // of the current device (created on first use)
// Sets up a private workspace on the current device (the serving loop owns one).
mlmc_ap_status init_workspace(Workspace& ws);
mlmc_ap_tuning resolve_tuning(const Workspace& ws, const mlmc_ap_tuning* t);
int persistent_grid(Workspace& ws, const mlmc_ap_tuning& t, bool fp64, bool kd);

// Device time measured by one launch of a table.
struct LaunchTiming {
  double total_s = 0.0;   // table upload to statistics read-back
  double kernel_s = 0.0;  // particle kernel(s) only (kModeTimed and kModePerLevel, else 0)
};

// Launch forms of a work table (all give bitwise identical results).
enum LaunchMode : int {
  kModePerLevel = 0,  // one plain launch per item
  kModeGraph = 1,     // stage, persistent, reduce replayed from a captured graph
  kModeTimed = 2,     // the three kernels issued directly, HIP events around the particle kernel
  kModeDirect = 3,    // the three kernels issued directly
  kModeDirectHost = 4,  // as kModeDirect, every launch planned by the host
};
// Maps mlmc_ap_options.batched to a launch mode (-1 if invalid).
int launch_mode(int32_t batched);

// Tiles and reduction groups the buffers keep for a device-planned top-up
// (20 MiB of tile records); a larger top-up is declined and planned by the host.
constexpr size_t kPlanTiles = 1u << 18;
constexpr size_t kPlanGroups = kPlanTiles / kGroupTiles + MLMC_AP_MAX_LEVELS;

// Builds the work table of `items` (assigning tile, group and chunk bases),
// launches it in the given mode and leaves the updated resident statistics
// slots in ws.resident_host (written by the reduction).  With `plan` (direct
// and timed modes, items one per level of one request, all levels of
// plan->level_mask): the table is a warm-up; the device then plans the first
// top-up from its statistics and launches it behind it (plan_kernel), and
// ws.plan_host holds the warm-up's statistics and the planned numbers.
mlmc_ap_status run_table(Workspace& ws, const std::vector<ItemSpec>& items, size_t n_slots,
                         int mode, const mlmc_ap_tuning& tuning, hipStream_t stream,
                         LaunchTiming* timing, const PlanArgs* plan = nullptr);

Stats stats_from_api(const mlmc_ap_level_stats& a);
mlmc_ap_level_stats stats_to_api(const Stats& s);

// MLMC control of one request (Section 4.1): warm-up, then eqs. Nopt1/Noptj
// with sample variances and deterministic costs, topped up until the
// statistical constraint holds (or max_iter top-ups ran).
struct McRequest {
  mlmc_ap_problem prob{};
  double tol = 0.0;
  bool plain = false;          // plain Monte Carlo at level L (single trajectories)
  uint64_t n_warmup = 1000;
  int max_iter = 10;
  uint64_t max_per_tick = 0;   // 0 = unlimited samples per level per launch
  int phase = 0;               // 0 warm-up pending, 1 top-ups, 2 finished
  int iterations = 0;
  bool converged = false;
  bool need_check = false;     // statistics changed since the last constraint check
  std::vector<uint64_t> done, target;
  std::vector<Stats> st;       // host copy of the resident statistics per level
  int level_select = 0;        // MLMC_AP_LEVELS_*
  bool selected = false;       // the level set has been chosen
  int tau = 0;                 // highest warm-up level before the selection
  int L_max = 0;               // level-adaptive finest level up to L_max (0: fixed L)
  int levels_added = 0;
  std::vector<double> prof_V, prof_Vd;  // warm-up profile of levels 0..tau
  std::vector<int> coarse_of;  // coarse level of level l's pair; -1: single level
  std::vector<char> in_set;    // level l is part of the hierarchy
  // Pilot pairs (L, i), i <= L - 2, of the cost-optimal selection: their
  // statistics give the correlations rho_{L,i} (slot slot_base + kPilotSlot + i).
  static constexpr uint32_t kPilotSlot = MLMC_AP_MAX_LEVELS + 1;
  std::vector<uint64_t> pilot_done;
  std::vector<Stats> pilot_st;
  bool pilots_active() const;
  uint64_t particle_steps = 0;
  uint64_t launches = 0;
  int device_planned = 0;      // top-ups the device planned after the warm-up
  double gpu_seconds = 0.0, kernel_seconds = 0.0;
  // Tolerance sequence of the epsilon-adaptive on-line phase (Section 5.3):
  // stage r ends when the statistical constraint holds at tols[r] (or after
  // max_iter top-ups), its result is kept in snaps, and stage r + 1 goes on
  // from the same samples.  A plain estimate is the one-stage sequence.
  std::vector<double> tols;
  size_t stage = 0;
  int stage_iter = 0;
  double t_start = 0.0;        // host clock of the call (for snapshot times)
  std::vector<mlmc_ap_result> snaps;

  void init(const mlmc_ap_problem& p, double rmse_tol, bool plain_mc, uint64_t warmup,
            int iters, uint64_t cap);
  int first_level() const { return plain ? prob.L : 0; }
  // Particle steps of one sample of level l's item.
  uint64_t item_cost(int l) const;
  // Selection mode and adaptive finest level (after init): the warm-up of
  // LEVELS_HEURISTIC_TAU runs levels 0..tau only.
  void set_selection(int mode, int lmax);
  // Chooses the level set after the warm-up (level_select != 0), and again
  // for a grown L (from the kept warm-up profile).
  void select_levels();
  // Makes the set's items those of `mask`: an item whose pair is new starts
  // over with a warm-up; one that stays keeps its samples.
  void apply_levels(uint64_t mask);
  // Bias estimate of eq. bias_constraint from the finest term (NaN without
  // a pair at L); *se its standard error.
  double bias_estimate(double* se) const;
  // Level-adaptive L: after the statistical constraint holds, adds level
  // L + 1 if the bias estimate is above tol/sqrt(2) and L < L_max.
  bool grow_finest();
  // Appends this request's work for the next launch; returns false if it has
  // none (finished).  Slots are slot_base + level.
  bool plan(std::vector<ItemSpec>& items, uint32_t slot_base, unsigned long long* hist_base,
            size_t hist_stride);
  // Takes the statistics of the launch and advances the state machine.
  void absorb(const Stats* resident_slots);
  // The next launch is the warm-up of every level of a one-stage estimate,
  // whose first top-up the device can plan (slots from 0): fills `a`.
  bool device_plannable(PlanArgs& a) const;
  void fill_result(mlmc_ap_result* out) const;
  // Replaces the tolerance by a sequence (before the first launch).
  void set_sequence(const std::vector<double>& seq);
};

}  // namespace mlmc
