// Launchers of the device kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "types.hpp"

namespace mlmc {

// Header of a device work table (read by the graph-captured kernels, so a
// replay picks up whatever table the host uploaded last).
struct alignas(16) WorkHeader {
  uint32_t n_items;
  uint32_t total_chunks;  // persistent kernel chunks
  uint32_t total_groups;
  uint32_t total_tp;      // trajectories of the time-parallel items
};

// Persistent-kernel work counters: one per chunk stream, each on its own
// 128-byte line (kChunkStreams * kCounterStride unsigned ints).
constexpr uint32_t kChunkStreams = 8;
constexpr uint32_t kCounterStride = 32;

// One plain launch over one item (any kind; KD kinds ignore fp64 and ppt).
hipError_t launch_level(bool fp64, int ppt, int kind, const LevelDesc* items_dev, uint32_t item,
                        uint32_t n_tiles, int block, Stats* partials, hipStream_t s);
// Blocks of `block` threads of the persistent kernel that fit one CU at once
// (0 if the runtime cannot say).
// kd: the kinetic-diffusion instantiation (FP64, one path or pair per lane;
// fp64 and ppt are then ignored).
int persistent_blocks_per_cu(bool fp64, int ppt, int block, bool kd);
hipError_t launch_persistent(bool fp64, int ppt, const LevelDesc* items_dev,
                             const WorkHeader* hdr_dev, unsigned int* counter, Stats* partials,
                             int block, int grid, hipStream_t s, bool kd);
// Tile records -> group records -> resident slots in one launch (the tile
// records of a time-parallel item are first built from its samples);
// item_done holds one counter per item, zeroed by the stage kernel; `mirror`
// (host-mapped pinned memory, or null) receives a copy of every slot written.
hipError_t launch_reduce(const LevelDesc* items_dev, const WorkHeader* hdr_dev, Stats* partials,
                         Stats* groups, unsigned int* item_done, Stats* resident, Stats* mirror,
                         int grid, hipStream_t s);
// Time-parallel items of the table (one wavefront per trajectory, grid-stride);
// kd: the kinetic-diffusion form.
hipError_t launch_tp(bool fp64, const LevelDesc* items_dev, const WorkHeader* hdr_dev, int grid,
                     hipStream_t s, bool kd);
// Work table and header from host-mapped pinned memory to the device; clears
// the persistent kernel's chunk counters and the reduction's item counters.
hipError_t launch_stage(const WorkHeader* hdr_src, const LevelDesc* items_src, uint32_t cap,
                        WorkHeader* hdr_dst, LevelDesc* items_dst, unsigned int* counter,
                        unsigned int* item_done, hipStream_t s);
struct PlanArgs;
struct PlanRecord;
// Device-planned top-up after a warm-up launch (one block): eqs. Nopt1/Noptj
// from the resident statistics, the top-up's table in place of the warm-up's
// (a.n_items <= MLMC_AP_MAX_LEVELS items, one per level), counters cleared;
// the warm-up's statistics and the planned numbers to `rec` (host-mapped).
hipError_t launch_plan(const PlanArgs& a, LevelDesc* items_dev, WorkHeader* hdr_dev,
                       const Stats* resident, unsigned int* counter, unsigned int* item_done,
                       PlanRecord* rec, hipStream_t s);
// Allocation-free launch: header and one descriptor as kernel arguments into
// device memory; clears item_done[0] and hist_n histogram counters.
hipError_t launch_stage_args(const WorkHeader& h, const LevelDesc& d, WorkHeader* hdr_dst,
                             LevelDesc* item_dst, unsigned int* item_done,
                             unsigned long long* hist, uint32_t hist_n, hipStream_t s);

// Scratch of the allocation-free entry point (a file-scope device array in
// kernels.hip): kScratchMaxSamples samples per call at most, laid out as
//   [0, 256)              WorkHeader
//   [256, 512)            LevelDesc
//   [512, 768)            item counter of the reduction
//   [768, 1024)           resident Stats slot
//   [1024, ...)           histogram counters, 3 MLMC_AP_MAX_BINS + 4 (uint64)
//   kScratchGroupsOffset  Stats per reduction group
//   kScratchTilesOffset   Stats per tile (a tile holds at least 64 samples)
constexpr uint64_t kScratchMaxSamples = 1ull << 22;
constexpr uint64_t kScratchMaxTiles = kScratchMaxSamples / 64;
constexpr uint64_t kScratchMaxGroups = kScratchMaxTiles / 256;
constexpr uint64_t kScratchHistCounters = 3 * 1024 + 4;
constexpr uint64_t kScratchHistOffset = 1024;
constexpr uint64_t kScratchGroupsOffset =
    (kScratchHistOffset + kScratchHistCounters * 8 + 255) / 256 * 256;
constexpr uint64_t kScratchTilesOffset =
    (kScratchGroupsOffset + kScratchMaxGroups * sizeof(Stats) + 255) / 256 * 256;
constexpr uint64_t kScratchBytes = kScratchTilesOffset + kScratchMaxTiles * sizeof(Stats);
// Device address of the current device's scratch (looked up on the first call
// on each device, then cached).
hipError_t scratch_address(void** out);

// Consistency harness: coarse numbers of the KD pairs of one item (the
// descriptor as a kernel argument), `cap` rows of 4 doubles per pair.
hipError_t launch_kd_numbers(const LevelDesc& d, uint64_t n, uint32_t cap, double* rows,
                             uint32_t* counts, hipStream_t s);

hipError_t launch_fill_u32(unsigned int* p, uint64_t n, unsigned int v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_words(uint32_t key0, uint32_t key1, uint32_t strm, uint32_t tag,
                        uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps,
                        uint32_t* out, hipStream_t s);
hipError_t launch_normals(bool fp64, uint32_t key0, uint32_t key1, uint32_t strm, uint32_t tag,
                          uint64_t sample_begin, uint64_t n_samples, uint32_t n_steps, void* out,
                          hipStream_t s);

}  // namespace mlmc
