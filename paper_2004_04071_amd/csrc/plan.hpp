// Sample numbers of the MLMC loop and the tile layout of a work item, shared
// by the host's planning and the device-planned top-up (plan_kernel), so that
// both compute them with the same operations in the same order.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mlmc_ap.h"
#include "types.hpp"

namespace mlmc {

// Fine steps per lane a persistent-kernel chunk aims at (load balance versus
// work-counter traffic); chunks never exceed 64 tiles, and on the long levels
// a chunk is a single tile so that the slowest chunks end early.
constexpr uint64_t kChunkLaneSteps = 128;
constexpr uint64_t kMinChunksPerItem = 64;

// Tiles, reduction groups and persistent-kernel chunks of an item of
// n_samples samples of n_steps fine steps.
struct ItemLayout {
  uint32_t spl, n_tiles, n_groups, chunk_tiles, n_chunks;
};

__host__ __device__ inline ItemLayout item_layout(uint64_t n_steps, uint64_t n_samples) {
  ItemLayout o;
  // wide tiles (several samples per lane) only where they still give the
  // item at least one wavefront per SIMD; a few samples of short
  // trajectories are spread over one per lane instead
  o.spl = samples_per_lane((uint32_t)n_steps);
  while (o.spl > 1 && n_samples < kMinWideTiles * (uint64_t)kLanes * o.spl)
    o.spl = o.spl > 4u ? o.spl / 4u : 1u;
  // tiles of 64 spl samples (spl a power of two)
  const uint32_t tile_shift = 6u + (uint32_t)__builtin_ctz(o.spl);
  o.n_tiles = (uint32_t)((n_samples + ((1ull << tile_shift) - 1)) >> tile_shift);
  o.n_groups = (o.n_tiles + kGroupTiles - 1) / kGroupTiles;
  // a chunk is about kChunkLaneSteps lane-steps of work, but an item keeps at
  // least kMinChunksPerItem chunks so that a small one is not serialised
  const uint64_t lane_steps = (uint64_t)o.spl * (n_steps + 1);
  uint32_t ct = lane_steps > kChunkLaneSteps ? 0u
                                             : (uint32_t)kChunkLaneSteps / (uint32_t)lane_steps;
  const uint32_t per_item = o.n_tiles / (uint32_t)kMinChunksPerItem;
  const uint32_t cap = per_item > 1 ? per_item : 1;
  if (ct > cap) ct = cap;
  if (ct < 1) ct = 1;
  if (ct > 64) ct = 64;
  o.chunk_tiles = ct;
  o.n_chunks = (o.n_tiles + o.chunk_tiles - 1) / o.chunk_tiles;
  return o;
}

// Sample variance of a level's correction (0 below two samples).
__host__ __device__ inline double level_variance(const Stats& s) {
  return s.n > 1.0 ? s.m2_dq / (s.n - 1.0) : 0.0;
}

// One term sqrt(V_l C_l) of the sum S of eqs. Nopt1/Noptj.
__host__ __device__ inline double cost_variance_root(double var, uint64_t cost) {
  return sqrt(var * (double)cost);
}

// eqs. Nopt1/Noptj for one level: N_l = ceil(2/tol^2 sqrt(V_l/C_l) S) with
// S = sum_k sqrt(V_k C_k), at most 2^32 - 1 (the sample counter word) and
// never below the samples already taken.
__host__ __device__ inline uint64_t level_target(double var, uint64_t cost, double S, double tol,
                                                 uint64_t done) {
  const double N = ceil(2.0 / (tol * tol) * sqrt(var / (double)cost) * S);
  const uint64_t Ni = N >= 4294967295.0 ? 4294967295ull : (uint64_t)N;
  return Ni > done ? Ni : done;
}

// Device-planned top-up (plan_kernel): the request's levels and the warm-up
// table they ran in, by value.
struct PlanArgs {
  double tol;
  uint64_t cost[MLMC_AP_MAX_LEVELS];   // particle steps per sample of level l's item
  uint32_t level_mask;                 // levels of the hierarchy (bit l)
  uint32_t slot_base;                  // resident slot of level l: slot_base + l
  uint32_t n_items;                    // items of the warm-up table (one per level)
  uint32_t cap_tiles, cap_groups;      // tile and group buffer capacities
};

// What the plan kernel leaves in host-mapped memory for the host's check.
struct PlanRecord {
  Stats warmup[MLMC_AP_MAX_LEVELS];    // the warm-up's statistics of level l
  uint64_t target[MLMC_AP_MAX_LEVELS]; // planned sample numbers of level l
  uint32_t declined;                   // 1: the table would not fit; nothing launched
  uint32_t n_items;                    // items of the top-up table
};

}  // namespace mlmc
