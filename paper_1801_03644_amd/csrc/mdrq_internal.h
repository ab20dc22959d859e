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

enum Mode : uint32_t { kIds = 0, kBitmap = 1, kCount = 2 };

// One predicate as the kernels see it: column base pointer and closed interval.
struct DevPred {
  const float* col;
  float lo;
  float hi;
};

// Cross-workgroup bookkeeping of one scan launch.  Zero between launches: the last
// workgroup of a launch resets it, so launches on one stream need no memset.
struct ScanState {
  uint32_t ticket;     // next tile to hand out
  uint32_t done;       // workgroups finished
  uint64_t total;      // qualifying rows, summed over workgroups
  uint64_t count_out;  // written by the last workgroup: exact result size
  uint32_t error;      // nonzero: a bounded wait gave up (results invalid)
  uint32_t pad;
};

struct ScanParams {
  uint64_t n_rows;
  uint32_t n_tiles;
  uint32_t n_preds;
  uint32_t epoch;       // tag of this launch's tile-status words
  uint32_t early_out;   // 1: rows rejected by earlier predicates are not re-read
  uint32_t* ids;        // kIds: output identifiers
  uint64_t* bitmap;     // kBitmap: output words
  uint64_t capacity;    // ids (kIds) or words (kBitmap) the output holds
  ScanState* state;
  uint64_t* status;     // per-tile status words (decoupled look-back)
  DevPred preds[MDRQ_MAX_DIMS];
};

// Launch one single-query scan.  `unroll` selects the tile height (float4 loads per
// lane per column: 1, 2, 4 or 8).  Returns a hipError_t.
hipError_t launch_scan(const ScanParams& p, uint32_t mode, int unroll, int grid,
                       hipStream_t stream);
int scan_tile_rows(int unroll);
// Workgroups per CU the scan kernel can keep resident (occupancy).
int scan_blocks_per_cu(uint32_t mode, int unroll);

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
  uint64_t* status = nullptr;            // device, max tiles entries
  uint32_t status_len = 0;
  uint32_t epoch = 0;
  mdrq::ScanState* host_state = nullptr; // pinned mirror
  void* staging = nullptr;               // device staging for host-resident outputs
  uint64_t staging_bytes = 0;

  // Profiling.
  bool profiling = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  uint64_t prof_launches = 0;
  double prof_ms = 0.0;
  int unroll = 4;                        // tile height of single-query scans
  int64_t grid = 0;                      // workgroups per launch (0 = resident maximum)
};
