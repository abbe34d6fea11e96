// Device-side model and launch descriptors shared by the sampling kernels
// and the host code that builds and launches them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sp_internal.hpp"

namespace sp {

// Device model: every section lives in the caller's buffer.
struct DevModel {
  const uint4* hot;          // [nb + kHotPad][2]: tm1[4] | (blk, 0, 0, 0), read for every block
  const uint4* cold;         // [nb][4]: meta[4] | lst[0..3] | (lst[4], 0, 0, 0) | 0, read when a block fires
  const uint32_t* entries;   // merged (row << 5 | bit) lists, one per drawn location
  const uint32_t* btab;      // per drawn location, the bounds of its code bits' lists in bentries
  const uint32_t* bentries;  // per location and code bit, its column's rows as byte offsets (row << 3)
  const uint32_t* chans;     // [nch][16]: kind | m << 8, T_1..T_{m-1}, then 0xFFFFFFFF
  const uint64_t* c_mask;    // [ceil(n_meas/64)]
  const uint64_t* dense;     // per variable: a bitmap of its non-zero words (ceil(dense_words/64)), then
                             // its dense_words mask words (dense path only)
  uint32_t nb, n_meas, dense_words, nch;
  uint32_t nb_lazy;          // blocks [0, nb_lazy) are lazy, [nb_lazy, nb) eager (sparse path)
};

// One sampling job: a model, an output and a shot range.
struct LaunchArgs {
  DevModel m;
  uint64_t* out;
  uint64_t ld;
  uint64_t first_shot;
  uint64_t shots;
  uint32_t key0, key1;
  uint32_t n_words, n_groups;
};

// One row tile of a model, as the tiled kernel reads it from device memory
// (16-byte multiple, read with 16-byte scalar loads).
struct alignas(16) TileRec {
  DevModel m;
  uint32_t row0;   // first output row of the tile
  uint32_t pad[1];
};

// One launch over every row tile of a model: `tiles` is the model's tile
// table, each tile gets n_groups groups of the same shot range.
struct TiledArgs {
  const TileRec* tiles;
  uint64_t* out;
  uint64_t ld;
  uint64_t first_shot;
  uint64_t shots;
  uint32_t key0, key1;
  uint32_t n_words, n_groups;
  uint32_t n_tiles;
};

// A job inside a batched launch (device memory; 16-byte multiple so that
// kernels read it with 16-byte scalar loads).  A job over a row-tiled model
// (n_tiles > 1) numbers its groups group * n_tiles + tile: a.m and a.out
// are then replaced per group by the tile's record (a.out points at row 0),
// and a.n_groups counts the groups of one tile.
struct alignas(16) BatchJob {
  LaunchArgs a;
  uint32_t group_base;   // global index of the job's first group
  uint32_t n_tiles;      // 0 or 1: a.m is the model; else the tiles in `tiles`
  const TileRec* tiles;
};

// A unit of hand-out in the persistent schedule: `count` consecutive groups
// of one job, starting at its local group `first`.
struct BatchTask {
  uint32_t job, first, count, pad;
};

// Work counters of a batched launch: `next` hands out groups, `done` counts
// workgroups that found no more work; the last one resets both.
struct BatchCounters {
  uint32_t next;
  uint32_t done;
  uint32_t pad[62];
};

int set_error(int code, const std::string& msg);

// Records a wave queues before it evaluates them (sparse path): one per
// (block, word, lane) with a fired location, 16 bytes of draws and a 4-byte
// tag, stored as five arrays of kQueueCap words (draw 0..3, tag).
constexpr uint32_t kQueueCap = 64;
constexpr uint32_t kQueueRecBytes = 20;

// Hot records past the last block, so that a wave may load the record one
// stride ahead of its last block (at most 16 waves) without a bounds test.
constexpr uint32_t kHotPad = 16;

// LDS bytes of one workgroup: its slabs, then (sparse path) one record
// queue of kQueueCap records per wave.
size_t lds_bytes(uint32_t n_meas, uint32_t words_per_group, uint32_t waves_per_group, int path);

// Kernel launchers (sample.hip).
int launch_sample(const LaunchArgs& a, int path, const sp_launch& L, hipStream_t s);
// All row tiles in one launch; `rows_max` sizes the LDS slabs.
int launch_sample_tiles(const TiledArgs& a, uint32_t rows_max, int path, const sp_launch& L, hipStream_t s);
// Persistent schedule: `grid` workgroups take tasks from ctr until none is left.
int launch_batch_persistent(const BatchJob* jobs, const BatchTask* tasks, uint32_t n_tasks, BatchCounters* ctr,
                            uint32_t n_meas_max, int path, const sp_launch& L, uint32_t grid, hipStream_t s);
// Flat schedule: one workgroup per group, group_job[g] names its job.
int launch_batch_flat(const BatchJob* jobs, const uint32_t* group_job, uint32_t total_groups, uint32_t n_meas_max,
                      int path, const sp_launch& L, hipStream_t s);
// Workgroups of the persistent kernel that fit on the device at once.
int batch_grid(const sp_launch& L, uint32_t n_meas_max, int path, uint32_t* grid);

}  // namespace sp

// A device-resident model.  Its output rows are split into row tiles, one
// unless the rows exceed one LDS slab (or a tile size was asked for): tile t
// is a model of its own over rows [row0[t], row0[t] + tiles[t].n_meas),
// drawing only the locations that reach those rows.  Draws are keyed by
// location, so the tiles agree on every draw they share.
struct sp_dmodel {
  std::vector<sp::DevModel> tiles;
  std::vector<uint32_t> row0;
  const sp::TileRec* d_tiles;   // the tile table in device memory (more than one tile), else null
  uint32_t n_meas;       // rows over all tiles
  uint32_t rows_max;     // rows of the largest tile
  uint32_t nb;           // Philox blocks per shot over all tiles
  int path;
  int device;
  size_t lds_max;
  sp_launch launch;
  sp_dims dims;
};
