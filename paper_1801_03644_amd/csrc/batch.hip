// Batched shared scan for gfx950: many range queries answered by one pass over the
// columns.
//
// Each query is the paper's problem (section 2.1) on its own: a row qualifies iff
// lo_j <= x_j <= hi_j on each of the query's dimensions, and its result is the set
// of qualifying row identifiers.  The batch only shares the reading of the data: a
// tile of the union of the queried columns is loaded from HBM once and tested
// against every query of the batch, one predicate at a time with the early break of
// section 2.2.4 per query, the per-dimension results ANDed as in section 3.2.
//
// GPU design (the work is VALU-bound once many queries share a tile):
//  * Lane l of a wave holds rows 64e + l (e = 0..3) of a 256-row chunk, one dword
//    load per column and e.  Values become order-preserving uint32 keys once per
//    chunk (-0 mapped to +0), so one predicate on 64 rows is one subtract and one
//    unsigned compare:  lo <= x <= hi  <=>  key(x) - key(lo) <= key(hi) - key(lo).
//    The compare lands in a 64-bit wave mask, which is directly bitmap word e of the
//    chunk (bit l <=> row 64e + l).
//  * The union's keys sit in registers (D slots x 4); the query table sits in LDS.
//    Per query, predicates run in the query's order and a query stops as soon as its
//    four masks are all zero.
//  * Per (query, 256-row chunk) the four masks are written as bitmap words to
//    scratch; per (query, 4096-row tile) the count is accumulated in LDS and stored.
//  * A finishing launch takes one workgroup per query: it sums the query's tile
//    counts and, for identifier output, scans them in LDS and compacts the query's
//    bitmap into ascending identifiers (tiles without a hit are not read).
#include <cstring>

#include "mdrq_internal.h"

namespace mdrq {
namespace {

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Order-preserving key of a non-NaN float: unsigned key order equals float order, and
// -0 and +0 share one key.
__device__ __forceinline__ uint32_t dkey(float x) {
  uint32_t b = __float_as_uint(x);
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Evaluate one predicate of slot S on the four row groups of a chunk.
#define MDRQ_SLOT_CASE(S)                                              \
  case S:                                                              \
    m0 &= ballot(x[S][0] - klo <= kw);                                 \
    m1 &= ballot(x[S][1] - klo <= kw);                                 \
    m2 &= ballot(x[S][2] - klo <= kw);                                 \
    m3 &= ballot(x[S][3] - klo <= kw);                                 \
    break;

template <int D, int W>
__global__ void __launch_bounds__(W * 64) batch_scan_kernel(BatchParams bp) {
  extern __shared__ uint32_t lds[];
  const uint32_t group = blockIdx.y;
  const uint32_t q_beg = bp.group_first[group];
  const uint32_t q_end = bp.group_first[group + 1];
  const uint32_t nq = q_end - q_beg;
  // LDS: [0, nq) per-query tile counts, then the group's table words.
  uint32_t* s_cnt = lds;
  uint32_t* s_tab = lds + nq;
  const uint32_t t_beg = bp.group_table[group];
  const uint32_t t_len = bp.group_table[group + 1] - t_beg;
  for (uint32_t i = threadIdx.x; i < t_len; i += W * 64) s_tab[i] = bp.table[t_beg + i];
  for (uint32_t i = threadIdx.x; i < nq; i += W * 64) s_cnt[i] = 0;
  __syncthreads();

  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x / 64;
  constexpr uint32_t kChunksPerWave = 16 / W;   // a tile is 16 chunks of 256 rows
  for (uint64_t tile = blockIdx.x; tile < bp.n_tiles; tile += gridDim.x) {
#pragma unroll 1
    for (uint32_t cw = 0; cw < kChunksPerWave; ++cw) {
      const uint64_t chunk = tile * 16 + wave * kChunksPerWave + cw;
      const uint64_t row0 = chunk * 256;
      if (row0 >= bp.n_rows) break;
      // Slots >= D are never referenced by the table (n_slots <= D); they stay the
      // constant 0 so that their switch cases fold away.
      uint32_t x[kMaxSlots][4];
      uint64_t valid[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint64_t r = row0 + 64 * e + lane;
        valid[e] = ballot(r < bp.n_rows);
#pragma unroll
        for (int s = 0; s < kMaxSlots; ++s)
          x[s][e] = (s < D && s < static_cast<int>(bp.n_slots) && r < bp.n_rows)
                        ? dkey(bp.slot_cols[s][r]) : 0u;
      }
      const uint64_t word0 = row0 / 64;
#pragma unroll 1
      for (uint32_t qi = 0; qi < nq; ++qi) {
        const uint32_t* rec = s_tab + s_tab[qi];
        const uint32_t head = rec[0];
        const uint32_t np = head & 0xFFu;
        const uint32_t kind = (head >> 8) & 0x3u;
        uint64_t m0 = valid[0], m1 = valid[1], m2 = valid[2], m3 = valid[3];
#pragma unroll 1
        for (uint32_t pi = 0; pi < np; ++pi) {
          const uint32_t slot = __builtin_amdgcn_readfirstlane(rec[1 + 3 * pi]);
          const uint32_t klo = __builtin_amdgcn_readfirstlane(rec[2 + 3 * pi]);
          const uint32_t kw = __builtin_amdgcn_readfirstlane(rec[3 + 3 * pi]);
          switch (slot) {
            MDRQ_SLOT_CASE(0)
            MDRQ_SLOT_CASE(1)
            MDRQ_SLOT_CASE(2)
            MDRQ_SLOT_CASE(3)
            MDRQ_SLOT_CASE(4)
            MDRQ_SLOT_CASE(5)
            MDRQ_SLOT_CASE(6)
            MDRQ_SLOT_CASE(7)
            MDRQ_SLOT_CASE(8)
            MDRQ_SLOT_CASE(9)
            MDRQ_SLOT_CASE(10)
            MDRQ_SLOT_CASE(11)
            MDRQ_SLOT_CASE(12)
            MDRQ_SLOT_CASE(13)
            MDRQ_SLOT_CASE(14)
            MDRQ_SLOT_CASE(15)
            default:
              break;
          }
          if ((m0 | m1 | m2 | m3) == 0) break;
        }
        const uint32_t c = __popcll(m0) + __popcll(m1) + __popcll(m2) + __popcll(m3);
        if (c != 0 && lane == 0) atomicAdd(&s_cnt[qi], c);
        if (kind != kBatchCount) {
          const uint32_t out = head >> 16;
          uint64_t* words = bp.words + static_cast<uint64_t>(out) * bp.n_words + word0;
          const uint64_t mv = lane == 0 ? m0 : lane == 1 ? m1 : lane == 2 ? m2 : m3;
          if (lane < 4 && word0 + lane < bp.n_words) words[lane] = mv;
        }
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nq; i += W * 64) {
      bp.tile_counts[static_cast<uint64_t>(q_beg + i) * bp.n_tiles + tile] = s_cnt[i];
      s_cnt[i] = 0;
    }
    __syncthreads();
  }
}
#undef MDRQ_SLOT_CASE

// ---------------------------------------------------------------- per-query finish

constexpr uint32_t kFinThreads = 256;
constexpr uint32_t kFinWaves = kFinThreads / 64;
constexpr uint32_t kFinScan = 8 * kFinThreads;   // tile counts scanned in LDS at a time

__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t& excl, uint32_t* s_wave) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x / 64;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d);
    if (lane >= static_cast<uint32_t>(d)) incl += o;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint32_t base = 0, total = 0;
#pragma unroll
  for (uint32_t w = 0; w < kFinWaves; ++w) {
    base += w < wave ? s_wave[w] : 0u;
    total += s_wave[w];
  }
  __syncthreads();
  excl = base + incl - v;
  return total;
}

// Workgroup q: exact count of query q, then its output: the bitmap copied to the
// caller's buffer, or its ascending identifiers.  AUTO picks, from the exact count,
// whichever of the two is smaller and fits the buffer.
__global__ void __launch_bounds__(kFinThreads) batch_finish_kernel(BatchFinish f) {
  __shared__ uint32_t s_off[kFinScan + 1];
  __shared__ uint32_t s_wave[kFinWaves];
  const uint32_t q = blockIdx.x;
  const BatchOut o = f.outs[q];
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63;
  const uint32_t wave = tid / 64;
  const uint32_t* counts = f.tile_counts + static_cast<uint64_t>(q) * f.n_tiles;
  const uint64_t* words = f.words + static_cast<uint64_t>(o.out_index) * f.n_words;

  uint32_t kind = o.kind;
  if (kind == kBatchAuto) {
    uint64_t part = 0;
    for (uint64_t t = tid; t < f.n_tiles; t += kFinThreads) part += counts[t];
    uint32_t ignore;
    const uint64_t count = block_scan(static_cast<uint32_t>(part), ignore, s_wave);
    const uint64_t bitmap_bytes = 8 * f.n_words;
    const bool fits_bitmap = o.buf_bytes >= bitmap_bytes;
    kind = (fits_bitmap && (bitmap_bytes < 4 * count || o.buf_bytes < 4 * count)) ? kBatchBitmap
                                                                                 : kBatchIds;
  }
  if (kind == kBatchBitmap) {
    const uint64_t cap = o.buf_bytes / 8;
    const uint64_t n = cap < f.n_words ? cap : f.n_words;
    uint64_t* dst = static_cast<uint64_t*>(o.buf);
    for (uint64_t i = tid; i < n; i += kFinThreads) dst[i] = words[i];
  }
  uint32_t* ids = static_cast<uint32_t*>(o.buf);
  const uint64_t capacity = kind == kBatchIds ? o.buf_bytes / 4 : 0;
  uint64_t carry = 0;
  for (uint64_t t0 = 0; t0 < f.n_tiles; t0 += kFinScan) {
    const uint32_t nt = static_cast<uint32_t>(f.n_tiles - t0 < kFinScan ? f.n_tiles - t0 : kFinScan);
    uint32_t v[8];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t t = tid * 8 + i;
      v[i] = t < nt ? counts[t0 + t] : 0u;
      sum += v[i];
    }
    uint32_t excl;
    const uint32_t total = block_scan(sum, excl, s_wave);
    if (kind == kBatchIds && carry < capacity) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint32_t t = tid * 8 + i;
        if (t < nt) s_off[t] = excl;
        excl += v[i];
      }
      if (tid == 0) s_off[nt] = total;
      __syncthreads();
      // One tile = 64 words = one wave-wide load.
      for (uint32_t t = wave; t < nt; t += kFinWaves) {
        const uint32_t beg = s_off[t];
        if (s_off[t + 1] == beg) continue;
        const uint64_t off = carry + beg;
        if (off >= capacity) continue;
        const uint64_t w = (t0 + t) * 64 + lane;
        const uint64_t word = w < f.n_words ? words[w] : 0;
        const uint32_t k = __popcll(word);
        uint32_t incl = k;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t x = __shfl_up(incl, d);
          if (lane >= static_cast<uint32_t>(d)) incl += x;
        }
        uint64_t r = off + incl - k;
        uint64_t bits = word;
        const uint32_t row = static_cast<uint32_t>(w * 64);
        while (bits) {
          const uint32_t b = static_cast<uint32_t>(__builtin_ctzll(bits));
          if (r < capacity) ids[r] = row + b;
          ++r;
          bits &= bits - 1;
        }
      }
      __syncthreads();
    }
    carry += total;
  }
  if (tid == 0) {
    f.counts_out[q] = carry;
    f.kind_out[q] = kind;
  }
}

template <int D, int W>
const void* scan_fn() {
  return reinterpret_cast<const void*>(&batch_scan_kernel<D, W>);
}

const void* pick_batch(int d, int w) {
  if (w == 4) return d <= 4 ? scan_fn<4, 4>() : d <= 8 ? scan_fn<8, 4>() : scan_fn<16, 4>();
  return d <= 4 ? scan_fn<4, 8>() : d <= 8 ? scan_fn<8, 8>() : scan_fn<16, 8>();
}

}  // namespace

uint32_t batch_key(float x) {
  uint32_t b;
  std::memcpy(&b, &x, sizeof b);
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

int batch_blocks_per_cu(int n_slots, int waves, size_t lds_bytes) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, pick_batch(n_slots, waves), waves * 64,
                                                   lds_bytes) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

hipError_t launch_batch_scan(const BatchParams& bp, int n_slots, int waves, dim3 grid,
                             size_t lds_bytes, hipStream_t stream) {
  void* args[] = {const_cast<BatchParams*>(&bp)};
  return hipLaunchKernel(pick_batch(n_slots, waves), grid, dim3(waves * 64), args, lds_bytes,
                         stream);
}

hipError_t launch_batch_finish(const BatchFinish& f, uint32_t n_queries, hipStream_t stream) {
  if (n_queries == 0) return hipSuccess;
  void* args[] = {const_cast<BatchFinish*>(&f)};
  return hipLaunchKernel(reinterpret_cast<const void*>(&batch_finish_kernel), dim3(n_queries),
                         dim3(kFinThreads), args, 0, stream);
}

}  // namespace mdrq
