// Internal declarations shared by the library's HIP sources (never by the oracle).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "mdrq.h"

namespace mdrq {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;

// Output modes of the kernels.  kStage is internal: the bitmap goes to scratch and
// the per-tile counts are kept, ready for the ordered compaction into identifiers.
enum Mode : uint32_t { kIds = 0, kBitmap = 1, kCount = 2, kStage = 3 };

// One predicate as the kernels see it: column base pointer and closed interval.
struct DevPred {
  const float* col;
  float lo;
  float hi;
};

// Cross-workgroup bookkeeping of one scan launch.  Zero between launches: the last
// workgroup of a launch resets it, so launches on one stream need no memset.
struct ScanState {
  uint64_t total;      // finished workgroups (bits 40..63) and their count (bits 0..39)
  uint64_t count_out;  // exact result size, written at the end of a launch
  uint32_t error;      // nonzero: the launch detected an inconsistency
  uint32_t pad;
};

struct ScanParams {
  uint64_t n_rows;
  uint64_t n_tiles;       // wave tiles of 256 * unroll rows
  uint32_t n_preds;
  uint32_t early_out;     // 1: rows rejected by earlier predicates are not re-read
  uint64_t* bitmap;       // kBitmap / kStage: output words
  uint64_t capacity;      // words the bitmap output holds
  uint64_t seg_tiles;     // tiles per workgroup segment
  uint32_t* tile_counts;  // kStage: qualifying rows per tile
  uint32_t* block_sums;   // kStage: qualifying rows per workgroup segment
  ScanState* state;
  DevPred preds[MDRQ_MAX_DIMS];
};

// Ordered compaction of a staged bitmap into ascending identifiers.
struct CompactParams {
  uint64_t n_tiles;
  uint64_t n_words;
  uint64_t seg_tiles;          // as in the scan that staged the bitmap
  const uint64_t* bitmap;
  const uint32_t* tile_counts;
  const uint32_t* block_sums;
  uint32_t* ids;
  uint64_t capacity;           // identifiers the output holds
  uint64_t* count_out;         // exact result size (written by the last workgroup)
};

// Launch one single-query scan.  `unroll` selects the tile height (float4 loads per
// lane per column: 1, 2, 4 or 8).  Returns a hipError_t.
hipError_t launch_scan(const ScanParams& p, uint32_t mode, int unroll, int grid,
                       hipStream_t stream);
hipError_t launch_compact(const CompactParams& c, int unroll, int grid, hipStream_t stream);
int scan_tile_rows(int unroll);
// Workgroups per CU the scan kernel can keep resident (occupancy).
int scan_blocks_per_cu(uint32_t mode, int unroll);

struct ProbeParams {
  uint64_t n_rows;
  uint32_t n_cols;
  uint32_t pad;
  uint32_t* sink;
  const float* cols[MDRQ_MAX_DIMS];
};
hipError_t launch_probe(const ProbeParams& p, int unroll, int grid, hipStream_t stream);

// Load-time validation: NaN count and per-column min/max (order-preserving keys).
struct ColumnStats {
  uint32_t nan_count;
  uint32_t pad;
  uint32_t min_key[MDRQ_MAX_DIMS];
  uint32_t max_key[MDRQ_MAX_DIMS];
};
hipError_t launch_validate(const float* const* cols_dev, uint32_t n_dims, uint64_t n_rows,
                           ColumnStats* stats, hipStream_t stream);
float key_to_float(uint32_t key);

// Thread-local error reporting.
int fail(int code, const std::string& msg);
int fail_hip(hipError_t e, const char* what);
void clear_error();

struct Device {
  int id = 0;
  int cus = 0;
  size_t lds = 0;
};
const Device& device();

}  // namespace mdrq

// Dataset: columns in HBM plus the workspace of its scans.
struct mdrq_dataset {
  uint64_t n_rows = 0;
  uint32_t n_dims = 0;
  bool owned = true;
  float* base = nullptr;                 // owned allocation (all columns)
  uint64_t stride = 0;                   // owned: floats between columns
  std::vector<const float*> cols;        // device pointer of each column
  std::vector<float> col_min, col_max;

  // Single-query workspace (calls are serialised by `mu`).
  std::mutex mu;
  mdrq::ScanState* state = nullptr;      // device
  uint64_t* stage_bitmap = nullptr;      // device, ceil(n_rows / 64) words
  uint32_t* tile_counts = nullptr;       // device, tiles at the smallest tile height
  uint32_t* block_sums = nullptr;        // device, block_sums_len entries
  uint64_t block_sums_len = 0;
  uint64_t max_tiles = 0;
  mdrq::ScanState* host_state = nullptr; // pinned mirror
  void* staging = nullptr;               // device staging for host-resident outputs
  uint64_t staging_bytes = 0;

  // Profiling.
  bool profiling = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  uint64_t prof_launches = 0;
  double prof_scan_ms = 0.0;
  double prof_total_ms = 0.0;
  int unroll = 8;                        // tile height of single-query scans (x 256 rows)
  int64_t grid = 0;                      // workgroups per launch (0 = blocks_per_cu per CU)
  int blocks_per_cu = 3;                 // default launch width, capped by occupancy
};
