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
//  * A persistent grid of 256-thread workgroups takes tiles of rows by atomic ticket.
//    A tile is 4 waves x U x 256 rows; each lane holds 4 consecutive rows per
//    16-byte load, so every wave-wide load reads 1 KB of one column, contiguous.
//  * Per row the state is one bit; per lane the bits of its 4*U rows sit in one
//    32-bit mask.  Predicate k+1 only loads the 16-byte groups of a lane that still
//    hold a live row, and a wave stops evaluating as soon as none of its rows is
//    alive (uniform branch).
//  * Identifiers are ranked inside the tile with wave ballots and mbcnt, staged in
//    LDS in row order, and the tile's global offset comes from a decoupled look-back
//    over per-tile status words (Merrill & Garland 2016).  Tiles are handed out in
//    ascending order by the ticket, so every tile a look-back waits on is owned by a
//    running workgroup, and every wait is bounded.
//  * The last workgroup to finish publishes the exact count and resets the launch
//    state, so consecutive launches on a stream need no memset.
#include <cstring>

#include "mdrq_internal.h"

namespace mdrq {
namespace {

constexpr uint32_t kFlagAgg = 1;
constexpr uint32_t kFlagIncl = 2;
constexpr uint32_t kSpinLimit = 1u << 22;   // polls before a look-back gives up

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return __popcll(m); }

__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint32_t flag, uint32_t v) {
  return (static_cast<uint64_t>(epoch & 0x3FFFFFFFu) << 34) |
         (static_cast<uint64_t>(flag) << 32) | v;
}

// Bit e of the result <=> lo <= element e <= hi.
__device__ __forceinline__ uint32_t hits4(float4 v, float lo, float hi) {
  return static_cast<uint32_t>(lo <= v.x && v.x <= hi) |
         (static_cast<uint32_t>(lo <= v.y && v.y <= hi) << 1) |
         (static_cast<uint32_t>(lo <= v.z && v.z <= hi) << 2) |
         (static_cast<uint32_t>(lo <= v.w && v.w <= hi) << 3);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v += __shfl_xor(v, off);
  return v;
}

// Live-row mask of one wave's rows (bit 4u+e <=> row wrow0 + 256u + 4*lane + e) after
// all predicates, for a tile lying entirely below n_rows.
template <int U>
__device__ __forceinline__ uint32_t eval_full(const ScanParams& p, uint64_t wrow0, uint32_t lane) {
  uint32_t m = static_cast<uint32_t>((uint64_t{1} << (4 * U)) - 1u);
  const uint32_t k_end = p.n_preds;
  for (uint32_t k = 0; k < k_end; ++k) {
    if (k > 0 && p.early_out && ballot(m != 0) == 0) break;
    const float* c = p.preds[k].col + wrow0 + 4 * lane;
    const float lo = p.preds[k].lo;
    const float hi = p.preds[k].hi;
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool need = !p.early_out || ((m >> (4 * u)) & 0xFu) != 0;
      v[u] = need ? *reinterpret_cast<const float4*>(c + 256 * u) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) m &= ~((~hits4(v[u], lo, hi) & 0xFu) << (4 * u));
  }
  return m;
}

// Same for the last, partial tile: element-wise loads of rows below n_rows only.
template <int U>
__device__ uint32_t eval_tail(const ScanParams& p, uint64_t wrow0, uint32_t lane) {
  uint32_t m = 0;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (wrow0 + 256 * u + 4 * lane + e < p.n_rows) m |= 1u << (4 * u + e);
  for (uint32_t k = 0; k < p.n_preds; ++k) {
    const float* c = p.preds[k].col + wrow0 + 4 * lane;
    const float lo = p.preds[k].lo;
    const float hi = p.preds[k].hi;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t bit = 1u << (4 * u + e);
        if (m & bit) {
          const float x = c[256 * u + e];
          if (!(lo <= x && x <= hi)) m &= ~bit;
        }
      }
  }
  return m;
}

__device__ __forceinline__ void read_status(const ScanParams& p, int64_t t, uint32_t& flag,
                                            uint32_t& val) {
  if (t < 0) {
    flag = kFlagIncl;
    val = 0;
    return;
  }
  const uint64_t s = __hip_atomic_load(&p.status[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const bool cur = static_cast<uint32_t>(s >> 34) == (p.epoch & 0x3FFFFFFFu);
  flag = cur ? static_cast<uint32_t>(s >> 32) & 3u : 0u;
  val = static_cast<uint32_t>(s);
}

// Exclusive prefix of tile `tile` over all earlier tiles (run by one whole wave).
__device__ uint32_t look_back(const ScanParams& p, uint32_t tile, uint32_t tile_count,
                              uint32_t lane) {
  if (tile == 0) {
    if (lane == 0)
      __hip_atomic_store(&p.status[0], pack_status(p.epoch, kFlagIncl, tile_count),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0)
    __hip_atomic_store(&p.status[tile], pack_status(p.epoch, kFlagAgg, tile_count),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t excl = 0;
  int64_t base = static_cast<int64_t>(tile) - 1;
  uint32_t spins = 0;
  for (;;) {
    const int64_t t = base - static_cast<int64_t>(lane);
    uint32_t flag, val;
    read_status(p, t, flag, val);
    while (ballot(flag == 0) != 0) {
      if (++spins > kSpinLimit) {
        if (flag == 0) {
          flag = kFlagIncl;
          val = 0;
        }
        if (lane == 0)
          __hip_atomic_store(&p.state->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      if (flag == 0) read_status(p, t, flag, val);
    }
    const uint64_t incl = ballot(flag == kFlagIncl);
    if (incl != 0) {
      const uint32_t j = static_cast<uint32_t>(__builtin_ctzll(incl));
      excl += wave_sum(lane <= j ? val : 0u);
      break;
    }
    excl += wave_sum(val);
    base -= kWave;
  }
  if (lane == 0)
    __hip_atomic_store(&p.status[tile], pack_status(p.epoch, kFlagIncl, excl + tile_count),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// Wave-wide sum of a per-lane count in [0, 32].
__device__ __forceinline__ uint32_t wave_total32(uint32_t c) {
  uint32_t t = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b) t += popc64(ballot((c >> b) & 1u)) << b;
  return t;
}

template <int MODE, int U>
__global__ void __launch_bounds__(kBlock) scan_kernel(ScanParams p) {
  constexpr int kRowsPerWave = 256 * U;
  constexpr int kTile = kWavesPerBlock * kRowsPerWave;
  __shared__ uint32_t s_ids[MODE == kIds ? kTile : 1];
  __shared__ uint32_t s_wcnt[kWavesPerBlock];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_off;
  __shared__ uint32_t s_block_total;

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & (kWave - 1);
  const uint32_t wave = tid / kWave;
  uint64_t wave_count = 0;  // uniform per wave
  const uint64_t n_words = (p.n_rows + 63) / 64;
  if (tid == 0) s_block_total = 0;

  for (;;) {
    if (tid == 0)
      s_tile = __hip_atomic_fetch_add(&p.state->ticket, 1u, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= p.n_tiles) break;
    const uint64_t trow0 = static_cast<uint64_t>(tile) * kTile;
    const uint64_t wrow0 = trow0 + static_cast<uint64_t>(wave) * kRowsPerWave;
    const bool full = trow0 + kTile <= p.n_rows;
    const uint32_t m = full ? eval_full<U>(p, wrow0, lane) : eval_tail<U>(p, wrow0, lane);

    if constexpr (MODE == kIds) {
      // Rank every live row in (wave, u, lane, e) order, i.e. ascending row order.
      uint32_t rank[U];
      uint32_t acc = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t c = __popc((m >> (4 * u)) & 0xFu);
        const uint64_t b0 = ballot(c & 1u), b1 = ballot(c & 2u), b2 = ballot(c & 4u);
        rank[u] = acc + mbcnt(b0) + 2 * mbcnt(b1) + 4 * mbcnt(b2);
        acc += popc64(b0) + 2 * popc64(b1) + 4 * popc64(b2);
      }
      if (lane == 0) s_wcnt[wave] = acc;
      __syncthreads();
      uint32_t wbase = 0, tcount = 0;
#pragma unroll
      for (int w = 0; w < kWavesPerBlock; ++w) {
        wbase += (static_cast<uint32_t>(w) < wave) ? s_wcnt[w] : 0u;
        tcount += s_wcnt[w];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        uint32_t nib = (m >> (4 * u)) & 0xFu;
        uint32_t r = wbase + rank[u];
        const uint32_t row = static_cast<uint32_t>(wrow0 + 256 * u + 4 * lane);
        while (nib) {
          const uint32_t e = __builtin_ctz(nib);
          s_ids[r++] = row + e;
          nib &= nib - 1;
        }
      }
      if (wave == 0) {
        const uint32_t off = look_back(p, tile, tcount, lane);
        if (lane == 0) s_off = off;
      }
      __syncthreads();
      const uint64_t off = s_off;
      for (uint32_t i = tid; i < tcount; i += kBlock) {
        const uint64_t pos = off + i;
        if (pos < p.capacity) p.ids[pos] = s_ids[i];
      }
      if (tid == 0) s_block_total += tcount;
    } else {
      if constexpr (MODE == kBitmap) {
        // Word w holds rows 64w .. 64w+63; lanes 8g .. 8g+7 hold 32 consecutive rows.
        const uint64_t lim = 2 * (p.capacity < n_words ? p.capacity : n_words);
        uint32_t* out32 = reinterpret_cast<uint32_t*>(p.bitmap);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          uint32_t v = ((m >> (4 * u)) & 0xFu) << (4 * (lane & 7));
          v |= __shfl_xor(v, 1);
          v |= __shfl_xor(v, 2);
          v |= __shfl_xor(v, 4);
          const uint64_t dw = ((wrow0 + 256 * u) >> 6) * 2 + (lane >> 3);
          if ((lane & 7) == 0 && dw < lim) out32[dw] = v;
        }
      }
      wave_count += wave_total32(__popc(m));
    }
    __syncthreads();
  }

  if constexpr (MODE != kIds) {
    if (lane == 0) atomicAdd(&s_block_total, static_cast<uint32_t>(wave_count));
    __syncthreads();
  }
  if (tid == 0) {
    __hip_atomic_fetch_add(&p.state->total, static_cast<uint64_t>(s_block_total),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t prev = __hip_atomic_fetch_add(&p.state->done, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gridDim.x - 1) {
      const uint64_t total =
          __hip_atomic_load(&p.state->total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&p.state->count_out, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&p.state->total, uint64_t{0}, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&p.state->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&p.state->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int MODE, int U>
void* kernel_ptr() {
  return reinterpret_cast<void*>(&scan_kernel<MODE, U>);
}

void* pick(uint32_t mode, int unroll) {
#define MDRQ_PICK(U)                                             \
  if (unroll == U) {                                             \
    if (mode == kIds) return kernel_ptr<kIds, U>();              \
    if (mode == kBitmap) return kernel_ptr<kBitmap, U>();        \
    return kernel_ptr<kCount, U>();                              \
  }
  MDRQ_PICK(1)
  MDRQ_PICK(2)
  MDRQ_PICK(4)
  MDRQ_PICK(8)
#undef MDRQ_PICK
  return nullptr;
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

int scan_tile_rows(int unroll) { return kWavesPerBlock * 256 * unroll; }

int scan_blocks_per_cu(uint32_t mode, int unroll) {
  void* f = pick(mode, unroll);
  if (!f) return 0;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(f),
                                                   kBlock, 0) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

hipError_t launch_scan(const ScanParams& p, uint32_t mode, int unroll, int grid,
                       hipStream_t stream) {
  void* f = pick(mode, unroll);
  if (!f) return hipErrorInvalidValue;
  void* args[] = {const_cast<ScanParams*>(&p)};
  return hipLaunchKernel(reinterpret_cast<const void*>(f), dim3(grid), dim3(kBlock), args, 0,
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
