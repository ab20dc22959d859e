// Single-query columnar range scan for gfx950 (CDNA4).
//
// The method is the paper's scan over vertically partitioned data (section 5.5):
// every queried dimension is one float32 array, each array is tested against its
// closed interval [lo, hi] (section 2.1), and the per-dimension results are ANDed
// (section 3.2).  Rows that already failed a predicate are not read again for later
// predicates, which is the early break of the paper's sequential scan (section
// 2.2.4) applied per row inside a tile.
//
// GPU design:
//  * A persistent grid of 256-thread workgroups; each wave scans tiles of U x 256 rows,
//    striding over the tiles statically (no order between tiles is needed).  Each
//    lane holds 4 consecutive rows per 16-byte load, so every wave-wide load reads
//    1 KB of one column, contiguous, and one predicate keeps U KB in flight per wave.
//  * Per row the state is one bit; per lane the bits of its 4*U rows sit in one
//    32-bit mask.  Predicate k+1 only loads the 16-byte groups of a lane that still
//    hold a live row, and a wave stops evaluating as soon as none of its rows is
//    alive (uniform branch).
//  * Output is the result bitmap (bit i of word i/64 <=> row i), assembled from the
//    lanes' 4-bit groups with DPP cross-lane ORs, and/or the count.
//  * Each workgroup scans one contiguous segment of tiles and records its count and
//    the count of each tile.  Ascending identifiers take one more launch over the same
//    segments: a workgroup sums the counts of the segments before its own, scans its
//    tiles' counts in LDS, reads its part of the bitmap back (N/8 bytes in total) and
//    writes every identifier at its final position.  No inter-workgroup waiting.
//  * The exact count: in COUNT and BITMAP modes each workgroup adds its count and a
//    finished mark with one atomic, and the last one publishes the total and resets
//    the word (consecutive launches on a stream need no memset); in IDS mode the
//    compaction's last workgroup publishes it.
#include <cstring>
#include <type_traits>

#include "mdrq_internal.h"

namespace mdrq {
namespace {

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return __popcll(m); }

// Bit e of the result <=> lo <= element e <= hi.
typedef float vf4 __attribute__((ext_vector_type(4)));

// Columns are read once per query and exceed every cache: streaming (non-temporal)
// 16-byte loads keep them from displacing reused data and reach a higher read rate on
// this part (about 7.1 TB/s against 6.3 TB/s for ordinary loads in a plain read test).
__device__ __forceinline__ float4 stream_load4(const float* p) {
  const vf4 v = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint32_t hits4(float4 v, float lo, float hi) {
  return static_cast<uint32_t>(lo <= v.x && v.x <= hi) |
         (static_cast<uint32_t>(lo <= v.y && v.y <= hi) << 1) |
         (static_cast<uint32_t>(lo <= v.z && v.z <= hi) << 2) |
         (static_cast<uint32_t>(lo <= v.w && v.w <= hi) << 3);
}

// OR over each aligned group of 8 lanes (DPP: quad swaps, then half-row mirror).
__device__ __forceinline__ uint32_t or_groups_of_8(uint32_t v) {
  v |= static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0xB1, 0xF, 0xF, false));
  v |= static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x4E, 0xF, 0xF, false));
  v |= static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x141, 0xF, 0xF, false));
  return v;
}

// Wave-wide sum of a per-lane count in [0, 64].
__device__ __forceinline__ uint32_t wave_total64(uint32_t c) {
  uint32_t t = 0;
#pragma unroll
  for (int b = 0; b < 7; ++b) t += popc64(ballot((c >> b) & 1u)) << b;
  return t;
}

// Per-lane live-row mask of a wave tile: 4 bits per 16-byte group, 4*U bits.
template <int U>
using LaneMask = typename std::conditional<(U > 8), uint64_t, uint32_t>::type;

// Live-row mask of one wave tile (bit 4u+e <=> row row0 + 256u + 4*lane + e) after
// all predicates, for a tile lying entirely below n_rows.
template <int U>
__device__ __forceinline__ LaneMask<U> eval_full(const ScanParams& p, const uint32_t* ord, uint64_t row0,
                                                 uint32_t lane) {
  using M = LaneMask<U>;
  M m = static_cast<M>(~M{0}) >> (8 * sizeof(M) - 4 * U);
  const uint32_t k_end = p.n_preds;
  for (uint32_t k = 0; k < k_end; ++k) {
    if (k > 0 && p.early_out && ballot(m != 0) == 0) break;
    const uint32_t kk = ord ? ord[k] : k;
    const float* c = p.preds[kk].col + row0 + 4 * lane;
    const float lo = p.preds[kk].lo;
    const float hi = p.preds[kk].hi;
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool need = !p.early_out || ((m >> (4 * u)) & 0xFu) != 0;
      v[u] = need ? stream_load4(c + 256 * u) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) m &= ~(static_cast<M>(~hits4(v[u], lo, hi) & 0xFu) << (4 * u));
  }
  return m;
}

// Same for the last, partial tile: element-wise loads of rows below n_rows only.
// (Runs once per query: kept as plain loops so it does not raise register pressure.)
template <int U>
__device__ LaneMask<U> eval_tail(const ScanParams& p, const uint32_t* ord, uint64_t row0, uint32_t lane) {
  using M = LaneMask<U>;
  M m = 0;
#pragma unroll 1
  for (int b = 0; b < 4 * U; ++b)
    if (row0 + 256 * (b >> 2) + 4 * lane + (b & 3) < p.n_rows) m |= M{1} << b;
#pragma unroll 1
  for (uint32_t k = 0; k < p.n_preds; ++k) {
    const uint32_t kk = ord ? ord[k] : k;
    const float* c = p.preds[kk].col + row0 + 4 * lane;
    const float lo = p.preds[kk].lo;
    const float hi = p.preds[kk].hi;
#pragma unroll 1
    for (int b = 0; b < 4 * U; ++b) {
      const M bit = M{1} << b;
      if (m & bit) {
        const float x = c[256 * (b >> 2) + (b & 3)];
        if (!(lo <= x && x <= hi)) m &= ~bit;
      }
    }
  }
  return m;
}

// Workgroup b scans the contiguous segment of tiles [B + b*S, B + (b+1)*S) below
// p.n_tiles, B = p.tile_begin, S = p.seg_tiles; its waves take every 4th tile of the
// segment.
template <int MODE, int U>
__global__ void __launch_bounds__(kBlock) scan_kernel(ScanParams p) {
  constexpr uint32_t kTileRows = 256 * U;
  __shared__ uint32_t s_block_total;
  __shared__ uint32_t s_order[MDRQ_MAX_DIMS];  // evaluation order, when one is given
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = threadIdx.x / kWave;
  uint32_t wave_count = 0;  // uniform per wave
  if (threadIdx.x == 0) s_block_total = 0;
  if (p.order)
    for (uint32_t i = threadIdx.x; i < p.n_preds; i += kBlock) s_order[i] = p.order[i];
  const uint32_t* ord = p.order ? s_order : nullptr;
  __syncthreads();

  const uint64_t n_words = (p.n_rows + 63) / 64;
  const uint64_t lim = 2 * (p.capacity < n_words ? p.capacity : n_words);  // dwords
  uint32_t* out32 = reinterpret_cast<uint32_t*>(p.bitmap);
  const uint64_t seg_beg = p.tile_begin + static_cast<uint64_t>(blockIdx.x) * p.seg_tiles;
  const uint64_t seg_end = seg_beg + p.seg_tiles < p.n_tiles ? seg_beg + p.seg_tiles : p.n_tiles;
  for (uint64_t tile = seg_beg + wave; tile < seg_end; tile += kWavesPerBlock) {
    const uint64_t row0 = tile * kTileRows;
    const bool full = row0 + kTileRows <= p.n_rows;
    const LaneMask<U> m = full ? eval_full<U>(p, ord, row0, lane) : eval_tail<U>(p, ord, row0, lane);
    if constexpr (MODE != kCount) {
      // Word w holds rows 64w .. 64w+63; lanes 8g .. 8g+7 hold 32 consecutive rows.
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t nib = static_cast<uint32_t>(m >> (4 * u)) & 0xFu;
        const uint32_t v = or_groups_of_8(nib << (4 * (lane & 7)));
        const uint64_t dw = ((row0 + 256 * u) >> 6) * 2 + (lane >> 3);
        if ((lane & 7) == 0 && dw < lim) out32[dw] = v;
      }
    }
    const uint32_t tc = wave_total64(__popcll(static_cast<uint64_t>(m)));
    if constexpr (MODE == kStage) {
      if (lane == 0) p.tile_counts[tile] = tc;
    }
    wave_count += tc;
  }

  if (lane == 0) atomicAdd(&s_block_total, wave_count);
  __syncthreads();
  if (threadIdx.x == 0) {
    if constexpr (MODE == kStage) {
      // The compaction pass sums the segment counts; no cross-workgroup atomics here.
      p.block_sums[blockIdx.x] = s_block_total;
    } else {
      // One atomic per workgroup: finished workgroups in bits 40..63, count below.
      const uint64_t add = (uint64_t{1} << 40) | s_block_total;
      const uint64_t prev = __hip_atomic_fetch_add(&p.state->total, add, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
      if ((prev >> 40) == gridDim.x - 1) {
        const uint64_t total = (prev & ((uint64_t{1} << 40) - 1)) + s_block_total;
        __hip_atomic_store(p.count_out, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&p.state->total, uint64_t{0}, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// ---------------------------------------------------------------- ordered compaction

constexpr uint32_t kChunkWords = kWave;        // one wave-wide load of bitmap words
constexpr uint32_t kScanTiles = 8 * kBlock;    // tile offsets held in LDS at a time

// Exclusive scan over the workgroup of one value per thread; returns the total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t& excl,
                                                         uint32_t* s_wave) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = threadIdx.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d);
    if (lane >= static_cast<uint32_t>(d)) incl += o;
  }
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) {
    base += static_cast<uint32_t>(w) < wave ? s_wave[w] : 0u;
    total += s_wave[w];
  }
  __syncthreads();
  excl = base + incl - v;
  return total;
}

// Inclusive prefix sum over the wave's lanes by DPP: shifts by 1, 2, 4, 8 within each
// row of 16 lanes, then row 0's and row 2's last lane added to rows 1 and 3, then lane
// 31 to rows 2 and 3 (lanes with no source add 0).
__device__ __forceinline__ uint32_t compact_wave_sum(uint32_t v) {
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xF, 0xF, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xF, 0xF, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xF, 0xF, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xF, 0xF, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xA, 0xF, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xC, 0xF, false));
  return v;
}

constexpr uint32_t kCompactStage = 2048;   // ids per wave staged in LDS

// Workgroup b turns the bitmap of its scan segment into ascending identifiers.  Its
// global offset is the sum of the earlier segments' counts; offsets of its tiles come
// from a scan of their counts in LDS; then each wave takes 64-word chunks (4096 rows):
// one coalesced load and a wave scan of the words' popcounts; a chunk of up to 2048 ids
// is staged in LDS as 16-bit row offsets at their output places and written out in
// consecutive 64-lane runs, a denser one is written word by word with one bit per lane.
// Chunks without a hit are skipped without being read.
template <int U>
__global__ void __launch_bounds__(kBlock) compact_kernel(CompactParams c) {
  constexpr uint32_t kTileRows = 256 * U;
  constexpr uint32_t kTilesPerChunk = kChunkWords * 64 / kTileRows;
  __shared__ uint32_t s_off[kScanTiles + 1];
  __shared__ uint32_t s_wave[kWavesPerBlock];
  __shared__ uint16_t s_stage[kWavesPerBlock][kCompactStage];
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1);
  const uint32_t wave = tid / kWave;

  // Offset of this segment: sum of all earlier workgroups' counts.  The last
  // workgroup also publishes the total.
  uint32_t part = 0;
  for (uint32_t j = tid; j < blockIdx.x; j += kBlock) part += c.block_sums[j];
  uint32_t ignore;
  uint64_t carry = block_exclusive_scan(part, ignore, s_wave);
  if (blockIdx.x == gridDim.x - 1 && tid == 0) c.count_out[0] = carry + c.block_sums[blockIdx.x];

  const uint64_t seg_beg = static_cast<uint64_t>(blockIdx.x) * c.seg_tiles;
  const uint64_t seg_end = seg_beg + c.seg_tiles < c.n_tiles ? seg_beg + c.seg_tiles : c.n_tiles;
  if (c.auto_mode) {
    // Every workgroup sums all segment counts and takes the same decision: the bitmap
    // when it is smaller than the identifiers (or only it fits) and the buffer holds it.
    uint32_t all = 0;
    for (uint32_t j = tid; j < gridDim.x; j += kBlock) all += c.block_sums[j];
    const uint64_t total = block_exclusive_scan(all, ignore, s_wave);
    const uint64_t bitmap_bytes = 8 * c.n_words;
    const bool bitmap = c.buf_bytes >= bitmap_bytes &&
                        (bitmap_bytes < 4 * total || c.buf_bytes < 4 * total);
    if (blockIdx.x == 0 && tid == 0) *c.kind_out = bitmap ? 1u : 0u;
    if (bitmap) {
      uint64_t* dst = reinterpret_cast<uint64_t*>(c.ids);
      const uint64_t w_end = seg_end * (kTileRows / 64) < c.n_words ? seg_end * (kTileRows / 64) : c.n_words;
      for (uint64_t w = seg_beg * (kTileRows / 64) + tid; w < w_end; w += kBlock) dst[w] = c.bitmap[w];
      return;
    }
  }
  for (uint64_t t0 = seg_beg; t0 < seg_end; t0 += kScanTiles) {
    const uint32_t nt = static_cast<uint32_t>(seg_end - t0 < kScanTiles ? seg_end - t0 : kScanTiles);
    // Exclusive offsets of tiles t0 .. t0+nt-1 (and the end) into LDS.
    uint32_t v[8];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t t = tid * 8 + i;
      v[i] = t < nt ? c.tile_counts[t0 + t] : 0u;
      sum += v[i];
    }
    uint32_t excl;
    const uint32_t chunk_total = block_exclusive_scan(sum, excl, s_wave);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t t = tid * 8 + i;
      if (t < nt) s_off[t] = excl;
      excl += v[i];
    }
    if (tid == 0) s_off[nt] = chunk_total;
    __syncthreads();
    // Chunks of 64 words; tile boundaries align with chunk boundaries.
    const uint32_t n_chunks = (nt + kTilesPerChunk - 1) / kTilesPerChunk;
    for (uint32_t ch = wave; ch < n_chunks; ch += kWavesPerBlock) {
      const uint32_t ft = ch * kTilesPerChunk;
      const uint32_t lt = ft + kTilesPerChunk < nt ? ft + kTilesPerChunk : nt;
      const uint32_t beg = s_off[ft];
      if (s_off[lt] == beg) continue;
      const uint64_t off = carry + beg;
      if (off >= c.capacity) continue;
      const uint64_t w0 = (t0 + ft) * (kTileRows / 64);
      const uint64_t w = w0 + lane;
      const uint64_t word = w < c.n_words && w < (t0 + lt) * (kTileRows / 64) ? c.bitmap[w] : 0;
      const uint32_t k = __popcll(word);
      const uint32_t incl = compact_wave_sum(k);
      const uint32_t total = __builtin_amdgcn_readlane(incl, 63);   // ids of the chunk
      uint64_t bits = word;
      if (total <= kCompactStage) {
        // The chunk's rows (16-bit offsets) into the wave's LDS buffer at their output
        // places, then out in consecutive 64-lane runs.
        uint16_t* buf = s_stage[wave];
        uint32_t at = incl - k;
        const uint32_t lane_row = lane * 64;
        while (bits) {
          buf[at++] = static_cast<uint16_t>(lane_row + static_cast<uint32_t>(__builtin_ctzll(bits)));
          bits &= bits - 1;
        }
        const uint32_t row0 = static_cast<uint32_t>(w0 * 64);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t i0 = 0; i0 < total; i0 += 4 * kWave) {
          uint32_t v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t i = i0 + kWave * j + lane;
            v[j] = i < total ? row0 + buf[i] : 0u;
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t i = i0 + kWave * j + lane;
            if (i < total && off + i < c.capacity) c.ids[off + i] = v[j];
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
        // A dense chunk, word by word: lane l takes bit l of the word, whose place is
        // the word's offset plus the set bits below it, so each store is one run of
        // consecutive ids.
        const uint32_t before = incl - k;
        const uint32_t row0 = static_cast<uint32_t>(w0 * 64);
        const uint32_t wlo = static_cast<uint32_t>(word);
        const uint32_t whi = static_cast<uint32_t>(word >> 32);
        for (uint32_t j = 0; j < kChunkWords; ++j) {
          const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(wlo), static_cast<int>(j)));
          const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(whi), static_cast<int>(j)));
          const uint32_t at = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(before), static_cast<int>(j)));
          const uint32_t below = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
          const bool set = (((static_cast<uint64_t>(hi) << 32 | lo) >> lane) & 1u) != 0;
          const uint64_t r = off + at + below;
          if (set && r < c.capacity) c.ids[r] = row0 + 64 * j + lane;
        }
      }
    }
    carry += chunk_total;
    __syncthreads();
  }
}

template <int MODE, int U>
void* kernel_ptr() {
  return reinterpret_cast<void*>(&scan_kernel<MODE, U>);
}

void* pick(uint32_t mode, int unroll) {
#define MDRQ_PICK(U)                                             \
  if (unroll == U) {                                             \
    if (mode == kStage) return kernel_ptr<kStage, U>();          \
    if (mode == kBitmap) return kernel_ptr<kBitmap, U>();        \
    return kernel_ptr<kCount, U>();                              \
  }
  MDRQ_PICK(1)
  MDRQ_PICK(2)
  MDRQ_PICK(4)
  MDRQ_PICK(8)
  MDRQ_PICK(16)
#undef MDRQ_PICK
  return nullptr;
}

// ---------------------------------------------------------------- read-bandwidth probe

// Reads full 256*U-row chunks of every listed column with the scan's load pattern and
// folds them into a checksum; only a checksum equal to a fixed pattern is stored.
template <int U>
__global__ void __launch_bounds__(kBlock) probe_kernel(ProbeParams p) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = threadIdx.x / kWave;
  const uint64_t chunk_rows = 256 * U;
  const uint64_t n_chunks = p.n_rows / chunk_rows;
  uint32_t acc = 0;
  for (uint64_t ch = static_cast<uint64_t>(blockIdx.x) * kWavesPerBlock + wave; ch < n_chunks;
       ch += static_cast<uint64_t>(gridDim.x) * kWavesPerBlock) {
    for (uint32_t k = 0; k < p.n_cols; ++k) {
      const float* c = p.cols[k] + ch * chunk_rows + 4 * lane;
      float4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = stream_load4(c + 256 * u);
#pragma unroll
      for (int u = 0; u < U; ++u)
        acc ^= __float_as_uint(v[u].x) ^ __float_as_uint(v[u].y) ^ __float_as_uint(v[u].z) ^
               __float_as_uint(v[u].w);
    }
  }
  if (acc == 0x9E3779B9u) p.sink[0] = acc;
}

// ---------------------------------------------------------------- early-break read bytes

// The column lines the early break must read for one query: for each predicate in
// evaluation order, the 128-byte lines (32 rows) of its column that hold a row every
// earlier predicate accepted (all lines for the first predicate, or for every predicate
// without early-out).  A measurement of the method's own bytes, not part of answering
// the query: one lane per row, each wave covering two lines, grid-stride over the rows.
__global__ void __launch_bounds__(kBlock) lines_kernel(LinesParams p) {
  __shared__ uint32_t s_order[MDRQ_MAX_DIMS];
  __shared__ unsigned long long s_sum;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = threadIdx.x / kWave;
  if (threadIdx.x == 0) s_sum = 0;
  if (p.order)
    for (uint32_t i = threadIdx.x; i < p.n_preds; i += kBlock) s_order[i] = p.order[i];
  __syncthreads();
  uint64_t lines = 0;  // uniform per wave
  for (uint64_t row0 = (static_cast<uint64_t>(blockIdx.x) * kWavesPerBlock + wave) * kWave;
       row0 < p.n_rows; row0 += static_cast<uint64_t>(gridDim.x) * kBlock) {
    const uint64_t row = row0 + lane;
    bool alive = row < p.n_rows;
    for (uint32_t k = 0; k < p.n_preds; ++k) {
      const uint64_t b = ballot(alive || (!p.early_out && row < p.n_rows));
      if (b == 0) break;
      lines += (static_cast<uint32_t>(b) != 0u) + ((b >> 32) != 0u);
      const uint32_t kk = p.order ? s_order[k] : k;
      if (alive) {
        const float x = p.preds[kk].col[row];
        alive = p.preds[kk].lo <= x && x <= p.preds[kk].hi;
      }
    }
  }
  if (lane == 0) atomicAdd(&s_sum, static_cast<unsigned long long>(lines));
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(p.lines, s_sum);
}

// ---------------------------------------------------------------- load validation

__device__ __forceinline__ uint32_t order_key(float x) {
  const uint32_t b = __float_as_uint(x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

struct ValidateArgs {
  const float* cols[MDRQ_MAX_DIMS];
};

__global__ void __launch_bounds__(kBlock) validate_kernel(ValidateArgs a, uint32_t n_dims,
                                                          uint64_t n_rows, ColumnStats* st) {
  const uint32_t j = blockIdx.y;
  const float* c = a.cols[j];
  uint32_t mn = 0xFFFFFFFFu, mx = 0u, nan = 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kBlock;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n_rows;
       i += stride) {
    const float x = c[i];
    if (x != x) {
      nan = 1;
    } else {
      const uint32_t k = order_key(x);
      mn = k < mn ? k : mn;
      mx = k > mx ? k : mx;
    }
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t omn = __shfl_xor(mn, off), omx = __shfl_xor(mx, off), on = __shfl_xor(nan, off);
    mn = omn < mn ? omn : mn;
    mx = omx > mx ? omx : mx;
    nan |= on;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMin(&st->min_key[j], mn);
    atomicMax(&st->max_key[j], mx);
    if (nan) atomicAdd(&st->nan_count, 1u);
  }
}

}  // namespace

int scan_tile_rows(int unroll) { return 256 * unroll; }

int scan_blocks_per_cu(uint32_t mode, int unroll) {
  void* f = pick(mode, unroll);
  if (!f) return 0;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(f),
                                                   kBlock, 0) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

const void* scan_kernel_fn(uint32_t mode, int unroll) { return pick(mode, unroll); }

const void* compact_kernel_fn(int unroll) {
  switch (unroll) {
    case 1: return reinterpret_cast<const void*>(&compact_kernel<1>);
    case 2: return reinterpret_cast<const void*>(&compact_kernel<2>);
    case 4: return reinterpret_cast<const void*>(&compact_kernel<4>);
    case 8: return reinterpret_cast<const void*>(&compact_kernel<8>);
    case 16: return reinterpret_cast<const void*>(&compact_kernel<16>);
    default: return nullptr;
  }
}

hipError_t launch_scan(const ScanParams& p, uint32_t mode, int unroll, int grid,
                       hipStream_t stream) {
  void* f = pick(mode, unroll);
  if (!f) return hipErrorInvalidValue;
  void* args[] = {const_cast<ScanParams*>(&p)};
  return hipLaunchKernel(reinterpret_cast<const void*>(f), dim3(grid), dim3(kBlock), args, 0,
                         stream);
}

hipError_t launch_compact(const CompactParams& c, int unroll, int grid, hipStream_t stream) {
  if (c.n_tiles == 0) return hipSuccess;
  void* args[] = {const_cast<CompactParams*>(&c)};
  const void* f = nullptr;
  switch (unroll) {
    case 1: f = reinterpret_cast<const void*>(&compact_kernel<1>); break;
    case 2: f = reinterpret_cast<const void*>(&compact_kernel<2>); break;
    case 4: f = reinterpret_cast<const void*>(&compact_kernel<4>); break;
    case 8: f = reinterpret_cast<const void*>(&compact_kernel<8>); break;
    case 16: f = reinterpret_cast<const void*>(&compact_kernel<16>); break;
    default: return hipErrorInvalidValue;
  }
  return hipLaunchKernel(f, dim3(grid), dim3(kBlock), args, 0, stream);
}

hipError_t launch_probe(const ProbeParams& p, int unroll, int grid, hipStream_t stream) {
  void* args[] = {const_cast<ProbeParams*>(&p)};
  const void* f = nullptr;
  switch (unroll) {
    case 1: f = reinterpret_cast<const void*>(&probe_kernel<1>); break;
    case 2: f = reinterpret_cast<const void*>(&probe_kernel<2>); break;
    case 4: f = reinterpret_cast<const void*>(&probe_kernel<4>); break;
    case 8: f = reinterpret_cast<const void*>(&probe_kernel<8>); break;
    case 16: f = reinterpret_cast<const void*>(&probe_kernel<16>); break;
    default: return hipErrorInvalidValue;
  }
  return hipLaunchKernel(f, dim3(grid), dim3(kBlock), args, 0, stream);
}

hipError_t launch_lines(const LinesParams& p, int grid, hipStream_t stream) {
  void* args[] = {const_cast<LinesParams*>(&p)};
  return hipLaunchKernel(reinterpret_cast<const void*>(&lines_kernel), dim3(grid), dim3(kBlock), args, 0,
                         stream);
}

hipError_t launch_validate(const float* const* cols_dev, uint32_t n_dims, uint64_t n_rows,
                           ColumnStats* stats, hipStream_t stream) {
  ValidateArgs a{};
  for (uint32_t j = 0; j < n_dims; ++j) a.cols[j] = cols_dev[j];
  uint64_t blocks = (n_rows + kBlock * 16 - 1) / (kBlock * 16);
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  validate_kernel<<<dim3(static_cast<uint32_t>(blocks), n_dims), kBlock, 0, stream>>>(
      a, n_dims, n_rows, stats);
  return hipGetLastError();
}

float key_to_float(uint32_t key) {
  const uint32_t b = (key & 0x80000000u) ? (key & 0x7FFFFFFFu) : ~key;
  float x;
  std::memcpy(&x, &b, sizeof x);
  return x;
}

}  // namespace mdrq
