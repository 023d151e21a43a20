// Host/device shared layouts of the MLMC-AP library (gfx950).
//
// A work item is one (request, level, sample range).  Its samples are split
// into tiles of consecutive global sample indices -- 64 lanes x spl samples,
// with spl = 4 for levels of fewer than 64 fine steps and spl = 1 above (so
// that one wavefront's serial work per tile stays short on the long levels).
// Every tile is reduced by one wavefront into a Stats record, and the records
// of an item are merged by a fixed tree (groups of 256 tiles, then one group
// result per item).  The tile size is a function of the level and the tree a
// function of the item's sample count, so the statistics are bitwise
// independent of launch shape, tuning, and of other items sharing a launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlmc {

constexpr int kLanes = 64;                       // gfx950 wavefront
constexpr uint32_t kTinyLevelSteps = 4;          // below: 2048-sample tiles
constexpr uint32_t kShortLevelSteps = 16;        // below: 1024-sample tiles; from here on 256
constexpr uint32_t kLongLevelSteps = 64;         // from here on: 64-sample tiles

// Samples per lane of a tile of a level with n_steps fine steps: the tile's
// closing wave reduction is spread over more samples where trajectories are
// short, and long trajectories keep one sample per lane.  An item with fewer
// than kMinWideTiles tiles of that size uses a quarter of it (repeatedly, down
// to one sample per lane).
constexpr uint64_t kMinWideTiles = 1024;
__host__ __device__ inline uint32_t samples_per_lane(uint32_t n_steps) {
  return n_steps >= kLongLevelSteps ? 1u
       : (n_steps >= kShortLevelSteps ? 4u : (n_steps >= kTinyLevelSteps ? 16u : 32u));
}
constexpr int kGroupTiles = 256;                 // tiles per first-stage group
constexpr int kReduceThreads = 256;
constexpr int kReducePerThread = kGroupTiles / kReduceThreads;  // 1
// An item holds at most 2^32 samples (the sample counter word), so at most
// 2^26 tiles and 2^18 groups.
constexpr uint64_t kMaxGroupsPerItem = 1ull << 18;
static_assert((uint64_t)kGroupTiles * kMaxGroupsPerItem * kLanes >= (1ull << 32),
              "an item of 2^32 samples must fit the two-stage reduction");

// Work item flags.
enum : uint32_t {
  kFlagCoarse = 1u << 0,      // level >= 1 pair: coarse path present
  kFlagMaxwell = 1u << 1,     // Maxwellian equilibrium (else two-point +-1)
  kFlagAggregate = 1u << 2,   // aggregated coarse kick (else normalised kick sum)
  kFlagHist = 1u << 3,        // histogram QoI
  kFlagWide = 1u << 4,        // a decision threshold is 0: 64-bit compares
  kFlagAccumulate = 1u << 6,  // merge into the resident statistics (else overwrite)
  kFlagTimeParallel = 1u << 7,  // one trajectory per wavefront, steps across lanes
  kFlagSampleOutputs = 1u << 8, // a dump or a histogram is requested
  kFlagQoiX = 1u << 9,          // Q = x(T) (else x(T)^2)
  kFlagBgB1 = 1u << 10,         // KD in background B1 (a > 0): R(x) = b (a |x - 1| + 1)
  kFlagBgB2 = 1u << 11,         // KD in background B2 (a > 0): R = b left of 1, linear right
};

// Final state of one sample of a time-parallel item.
struct alignas(8) TpSample {
  double xf, xc;
  uint32_t cf, cc;
};

// Trajectory kinds (the compile-time specialisations of the particle loop).
enum : int {
  kKindFineTwoPoint = 0,
  kKindFineMaxwell = 1,
  kKindPairTwoPointSum = 2,
  kKindPairMaxwellSum = 3,
  kKindPairMaxwellAggregate = 4,
  kKindKdFine = 5,   // kinetic-diffusion scheme: one path (FP64 state)
  kKindKdPair = 6,   // kinetic-diffusion scheme: correlated fine/coarse pair
};

// The KD kinds use the coefficient slots of LevelDesc as
//   h_f = fine step dt_l, h_c = coarse step dt_{l-1}, s_f = collision rate R
//   (in a background: its parameter b), s_c = Maxwellian standard deviation
//   sigma, agg_ms2 = end time T, h_f2 = Maxwellian mean mu, rsqrt_m = the
//   background's slope parameter a.
__host__ __device__ inline bool is_kd_kind(int kind) { return kind >= kKindKdFine; }

struct alignas(16) LevelDesc {
  double h_f, s_f, h_c, s_c;    // scheme coefficients, fine and coarse
  double agg_ms2;               // M s_f^2 (aggregated kick normalisation)
  double h_f2;                  // h_f^2
  double rsqrt_m;               // 1/sqrt(M)
  double x0_a, x0_b;            // initial law parameters
  double hist_lo, hist_inv_w;   // histogram origin and 1/bin width
  uint64_t sample_begin;        // first global sample index of the item
  uint64_t n_samples;
  uint64_t tile_base;           // first tile slot in the partial buffer
  uint64_t group_base;          // first group slot in the group buffer
  uint64_t chunk_base;          // persistent kernel: first global chunk index
  unsigned long long* hist;     // item histogram counters (3 nbins + 4), or null
  void* traj;                   // trajectory dump (2 n_samples reals), or null
  uint32_t* coll;               // collision dump (2 n_samples), or null
  uint64_t thr_f, thr_c2;       // decision thresholds in [0, 2^32]
  uint32_t thr_f_m1, thr_c2_m1; // threshold - 1 (used when both are >= 1)
  uint32_t n_steps;             // fine steps
  uint32_t M;                   // refinement factor
  uint32_t tag, stream;         // counter words 2 and 3
  uint32_t key0, key1;          // Philox key (seed)
  uint32_t flags;
  int32_t kind;                 // kKind*
  uint32_t x0_kind;
  uint32_t nbins;
  uint32_t n_tiles;
  uint32_t n_groups;
  uint32_t chunk_tiles;         // persistent kernel: tiles per chunk
  uint32_t n_chunks;
  uint32_t result_slot;         // resident statistics slot
  uint32_t spl;                 // samples per lane of a tile (tile = 64 spl samples)
  uint32_t tp_base;             // first trajectory in the table's time-parallel space
  uint32_t pad;
  TpSample* tp_out;             // time-parallel item: final state of every sample
};

static_assert(sizeof(LevelDesc) == 256, "LevelDesc layout");

// Mergeable statistics of a set of samples (FP64 means and centred sums).
struct alignas(16) Stats {
  double n;
  double mean_dq, m2_dq;
  double mean_qf, m2_qf;
  double mean_qc, m2_qc;
  double c_fc;
  unsigned long long coll_f, coll_c;
};

static_assert(sizeof(Stats) == 80, "Stats layout");

}  // namespace mlmc
