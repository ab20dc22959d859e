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
//  * Lane l of a wave holds rows 64g + l (g < RG) of a chunk of 64*RG rows, one dword
//    load per column and g.  Values become order-preserving uint32 keys once per
//    chunk (-0 mapped to +0), so one predicate on 64 rows is one subtract and one
//    unsigned compare:  lo <= x <= hi  <=>  key(x) - key(lo) <= key(hi) - key(lo).
//    The compare lands in a 64-bit wave mask, which is directly bitmap word g of the
//    chunk (bit l <=> row 64g + l).
//  * The union's keys sit in registers (D slots x RG) and the query table in LDS; a
//    predicate's register slot is found by uniform branches, either searched per
//    predicate (the query's own order) or walked slot by slot with each query's
//    predicates sorted by slot (fewer branches).  A query stops as soon as all its
//    masks are zero.  RG rows per lane amortise the per-predicate work.  A second
//    variant stages the keys in LDS instead, for unions wider than the registers hold.
//  * The bitmap scratch is zeroed first; per (query, chunk) only non-zero masks are
//    stored; per (query, 4096-row tile) the count is accumulated in LDS and stored.
//  * Finishing takes two launches: one workgroup per query sums its tile counts (the
//    exact count), resolves AUTO and, for identifier output, turns the tile counts into
//    output positions; then a grid of (tile range, query) workgroups copies bitmap
//    words or compacts the tiles with a hit into ascending identifiers.
#include <algorithm>
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

// One query-table predicate, one 16-byte entry: the register slot, key(lo), and
// key(hi) - key(lo) (register variants) or key(hi) (LDS variant).
struct TabPred {
  uint32_t slot, klo, kw, pad;
};

// Row of tile_counts that query q of the batch writes.
__device__ __forceinline__ uint64_t count_row(const BatchParams& bp, uint32_t q) {
  return bp.count_row ? bp.count_row[q] : q;
}

// Workgroups stride over the 4096-row tiles of [tile_begin, tile_end); within a tile, each wave takes chunks of
// 64*RG rows (lane l holds rows 64g + l, g < RG).  For each chunk every query of the
// workgroup's group is evaluated; non-zero wave masks are stored as bitmap words
// (the scratch was zeroed), and the chunk's count is added to the query's tile
// count in LDS.
//
// WALK: the host has sorted each query's predicates by slot, and the slots are walked
// in order (one uniform compare per slot and query) instead of searching each
// predicate's slot (up to one compare per slot and predicate).
template <int D, int W, int RG, bool WALK>
__global__ void __launch_bounds__(W * 64) batch_scan_kernel(BatchParams bp) {
  static_assert(W * RG <= 64, "a tile must hold at least one chunk per wave");
  extern __shared__ uint32_t lds[];
  const uint32_t group = blockIdx.y;
  const uint32_t q_beg = bp.group_first[group];
  const uint32_t q_end = bp.group_first[group + 1];
  const uint32_t nq = q_end - q_beg;
  // LDS: [0, nq) per-query tile counts, then the group's table words (16-byte aligned).
  uint32_t* s_cnt = lds;
  uint32_t* s_tab = lds + ((nq + 3) & ~3u);
  const uint32_t t_beg = bp.group_table[group];
  const uint32_t t_len = bp.group_table[group + 1] - t_beg;
  for (uint32_t i = threadIdx.x; i < t_len; i += W * 64) s_tab[i] = bp.table[t_beg + i];
  for (uint32_t i = threadIdx.x; i < nq; i += W * 64) s_cnt[i] = 0;
  __syncthreads();

  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x / 64;
  constexpr uint32_t kChunkRows = 64 * RG;
  constexpr uint32_t kChunksPerWave = 4096 / kChunkRows / W;
  for (uint64_t tile = bp.tile_begin + blockIdx.x; tile < bp.tile_end; tile += gridDim.x) {
#pragma unroll 1
    for (uint32_t cw = 0; cw < kChunksPerWave; ++cw) {
      const uint64_t row0 = tile * 4096 + (wave * kChunksPerWave + cw) * kChunkRows;
      if (row0 >= bp.n_rows) break;
      // Rows past the end get the key 0, below the key of every non-NaN float (bounds
      // are never NaN: the smallest, key(-inf), is 0x007FFFFF), so the first predicate
      // of every query rejects them.
      uint32_t x[D][RG];
      const bool full = row0 + kChunkRows <= bp.n_rows;
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        const uint64_t r = row0 + 64 * g + lane;
#pragma unroll
        for (int s = 0; s < D; ++s)
          x[s][g] = (s < static_cast<int>(bp.n_slots) && (full || r < bp.n_rows))
                        ? dkey(__builtin_nontemporal_load(&bp.slot_cols[s][r])) : 0u;
      }
      const uint64_t word0 = row0 / 64;
      // Records are contiguous: each is a 4-word header and 4 words per predicate.
      const uint32_t* rec = s_tab + s_tab[0];
#pragma unroll 1
      for (uint32_t qi = 0; qi < nq; ++qi) {
        const uint32_t head = __builtin_amdgcn_readfirstlane(rec[0]);
        const uint32_t np = head & 0xFFu;
        const uint32_t kind = (head >> 8) & 0x3u;
        const TabPred* tp = reinterpret_cast<const TabPred*>(rec + 4);
        rec += 4 + 4 * np;
        uint64_t m[RG];
        if (np != 0) {
#pragma unroll
          for (int g = 0; g < RG; ++g) m[g] = ~uint64_t{0};
        } else {  // no predicate: every row of the chunk that exists
#pragma unroll
          for (int g = 0; g < RG; ++g) m[g] = ballot(row0 + 64 * g + lane < bp.n_rows);
        }
        bool dead = false;
        if constexpr (WALK) {
          uint32_t pi = 0;
          uint32_t slot = np ? __builtin_amdgcn_readfirstlane(tp[0].slot) : static_cast<uint32_t>(D);
#pragma unroll
          for (int S = 0; S < D; ++S)
            if (slot == static_cast<uint32_t>(S)) {
              const uint32_t klo = __builtin_amdgcn_readfirstlane(tp[pi].klo);
              const uint32_t kw = __builtin_amdgcn_readfirstlane(tp[pi].kw);
#pragma unroll
              for (int g = 0; g < RG; ++g) m[g] &= ballot(x[S][g] - klo <= kw);
              ++pi;
              slot = pi < np ? __builtin_amdgcn_readfirstlane(tp[pi].slot) : static_cast<uint32_t>(D);
              // Early break of the whole chunk, tested after every second predicate.
              if (!(pi & 1) && pi < np) {
                uint64_t any = 0;
#pragma unroll
                for (int g = 0; g < RG; ++g) any |= m[g];
                if (any == 0) {
                  dead = true;
                  slot = static_cast<uint32_t>(D);
                }
              }
            }
        } else {
#pragma unroll 1
        for (uint32_t pi = 0; pi < np; ++pi) {
          const TabPred t = tp[pi];
          const uint32_t slot = __builtin_amdgcn_readfirstlane(t.slot);
          const uint32_t klo = __builtin_amdgcn_readfirstlane(t.klo);
          const uint32_t kw = __builtin_amdgcn_readfirstlane(t.kw);
          // Slot dispatch: register slots cannot be indexed at run time, so a flat
          // chain of uniform branches; each case updates the masks in place.
#pragma unroll
          for (int S = 0; S < D; ++S)
            if (slot == static_cast<uint32_t>(S)) {
#pragma unroll
              for (int g = 0; g < RG; ++g) m[g] &= ballot(x[S][g] - klo <= kw);
            }
          // Early break of the whole chunk, tested after every second predicate.
          if ((pi & 1) && pi + 1 < np) {
            uint64_t any = 0;
#pragma unroll
            for (int g = 0; g < RG; ++g) any |= m[g];
            if (any == 0) {
              dead = true;
              break;
            }
          }
        }
        }
        if (dead) continue;
        uint32_t c = 0;
#pragma unroll
        for (int g = 0; g < RG; ++g) c += __popcll(m[g]);
        if (c != 0) {
          if (lane == 0) atomicAdd(&s_cnt[qi], c);
          if (kind != kBatchCount) {
            uint64_t* words = bp.words + static_cast<uint64_t>(head >> 16) * bp.n_words + word0;
#pragma unroll
            for (int g = 0; g < RG; ++g)
              if (m[g] != 0 && lane == 0) words[g] = m[g];
          }
        }
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nq; i += W * 64) {
      bp.tile_counts[count_row(bp, q_beg + i) * bp.n_tiles + tile] = s_cnt[i];
      s_cnt[i] = 0;
    }
    __syncthreads();
  }
}

// The query table is read-only for the whole launch and every access to it is
// wave-uniform: reading it through the constant address space gives scalar loads.
typedef __attribute__((address_space(4))) const uint32_t cu32;
typedef __attribute__((address_space(4))) const TabPred ctabpred;

// ---------------------------------------------------------------- slot-mask variant

// lo <= x <= hi on order-preserving keys  <=>  med3(x, lo, hi) == x.  The result is
// folded into a per-lane word that stays zero while the row qualifies, so a range
// test is two vector instructions (v_med3_u32, then v_bitop3_b32 for acc |= m ^ x)
// and no scalar work.  gfx9 VOP3 reads at most one scalar operand, hence hi in a VGPR.
__device__ __forceinline__ uint32_t med3u(uint32_t x, uint32_t lo, uint32_t hi) {
  uint32_t r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=&v"(r) : "v"(x), "s"(lo), "v"(hi));
  return r;
}

// Order-preserving key from the raw bits of a float, -0 one below +0 (the rank
// variant's keys: three instructions).
__device__ __forceinline__ uint32_t rkey(uint32_t b) {
  return b ^ (static_cast<uint32_t>(static_cast<int32_t>(b) >> 31) | 0x80000000u);
}

// Order-preserving key from the raw bits of a non-NaN float (as dkey).
__device__ __forceinline__ uint32_t bkey(uint32_t b) {
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// As batch_scan_kernel, with fixed-size query records read by scalar loads: the
// header, the query's slot mask (bit S: a predicate on slot S; bit 16 + S: test for
// the early break after it), then (key(lo), key(hi)) for every slot S < D.  A query
// walks the slots in order and tests those in its mask; the record of the next query
// is loaded while the current one is tested.  A query without predicates carries
// [key(-inf), key(+inf)] on slot 0, which every row passes except those past the end.
template <int D>
struct RegRecord {
  static constexpr uint32_t kWords = 2 + 2 * D;
};

template <int D, int W, int RG>
__global__ void __launch_bounds__(W * 64) batch_reg_kernel(BatchParams bp) {
  static_assert(W * RG <= 64, "a tile must hold at least one chunk per wave");
  constexpr uint32_t R = RegRecord<D>::kWords;
  // Chunk marks instead of zeroed scratch rows, where scalar registers allow: with 12
  // or 16 slots the mark's address would push scalar spills into the query loop.
  constexpr bool kMarks = batch_reg_uses_marks(D);
  extern __shared__ uint32_t lds[];
  const uint32_t group = blockIdx.y;
  const uint32_t q_beg = bp.group_first[group];
  const uint32_t nq = bp.group_first[group + 1] - q_beg;
  cu32* recs = (cu32*)(bp.table) + bp.group_table[group];  // generic -> constant address space
  uint32_t* s_cnt = lds;
  for (uint32_t i = threadIdx.x; i < nq; i += W * 64) s_cnt[i] = 0;
  __syncthreads();

  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // wave-uniform
  const uint32_t ns = bp.n_slots;
  constexpr uint32_t kChunkRows = 64 * RG;
  constexpr uint32_t kChunksPerWave = 4096 / kChunkRows / W;
  for (uint64_t tile = bp.tile_begin + blockIdx.x; tile < bp.tile_end; tile += gridDim.x) {
#pragma unroll 1
    for (uint32_t cw = 0; cw < kChunksPerWave; ++cw) {
      const uint64_t row0 = tile * 4096 + (wave * kChunksPerWave + cw) * kChunkRows;
      if (row0 >= bp.n_rows) break;
      const bool full = row0 + kChunkRows <= bp.n_rows;
      // All loads of the chunk first (rows clamped into the column), keys after, so the
      // loads are in flight together.  Rows past the end get the key 0, below
      // key(-inf) = 0x007FFFFF, the smallest bound key: every predicate rejects them.
      uint32_t x[D][RG];
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        const uint64_t r = row0 + 64 * g + lane;
        const uint64_t rc = r < bp.n_rows ? r : bp.n_rows - 1;
#pragma unroll
        for (int s = 0; s < D; ++s)
          x[s][g] = s < static_cast<int>(ns)
                        ? __float_as_uint(__builtin_nontemporal_load(&bp.slot_cols[s][rc])) : 0u;
      }
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        const bool valid = full || row0 + 64 * g + lane < bp.n_rows;
#pragma unroll
        for (int s = 0; s < D; ++s) x[s][g] = valid ? bkey(x[s][g]) : 0u;
      }
      const uint64_t word0 = row0 / 64;

      auto load_rec = [&](uint32_t* rr, uint32_t qi) {
        cu32* p = recs + qi * R;
#pragma unroll
        for (uint32_t i = 0; i < R; ++i) rr[i] = p[i];
      };
      // The query's predicates in slot order; true if the whole chunk is rejected (an
      // early break clears the remaining mask, so the walk falls through its slots).
      auto walk = [&](const uint32_t* rr, uint32_t* acc) -> bool {
        uint32_t sm = rr[1];
#pragma unroll
        for (int S = 0; S < D; ++S) {
          if (sm & (1u << S)) {
            const uint32_t klo = rr[2 + 2 * S];
            const uint32_t khi = rr[3 + 2 * S];
            uint32_t t[RG];
#pragma unroll
            for (int g = 0; g < RG; ++g) t[g] = med3u(x[S][g], klo, khi);
#pragma unroll
            for (int g = 0; g < RG; ++g) acc[g] |= t[g] ^ x[S][g];
            if (sm & (0x10000u << S)) {
              uint32_t mn = acc[0];
#pragma unroll
              for (int g = 1; g < RG; ++g) mn = mn < acc[g] ? mn : acc[g];
              if (ballot(mn == 0) == 0) sm = 0;
            }
          }
        }
        return sm == 0;
      };
      auto process = [&](const uint32_t* rr, uint32_t qi) {
        uint32_t acc[RG];
#pragma unroll
        for (int g = 0; g < RG; ++g) acc[g] = 0;
        if (walk(rr, acc)) return;
        uint64_t m[RG];
        uint32_t c = 0;
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          m[g] = ballot(acc[g] == 0);
          c += __popcll(m[g]);
        }
        if (c == 0) return;
        const uint32_t head = rr[0];
        if (lane == 0) atomicAdd(&s_cnt[qi], c);
        if (((head >> 8) & 0x3u) != kBatchCount) {
          const uint64_t out = head >> 16;
          uint64_t* words = bp.words + out * bp.n_words + word0;
          if constexpr (kMarks) {
            // The non-zero words, and the chunk's mark: bit g <=> word g was stored.
            uint32_t stored = 0;
#pragma unroll
            for (int g = 0; g < RG; ++g)
              if (m[g] != 0) {
                stored |= 1u << g;
                if (lane == 0) words[g] = m[g];
              }
            if (lane == 0) bp.flags[out * bp.n_chunks + row0 / kChunkRows] = static_cast<uint16_t>(stored);
          } else {  // the rows were zeroed: the non-zero words only
#pragma unroll
            for (int g = 0; g < RG; ++g)
              if (m[g] != 0 && lane == 0) words[g] = m[g];
          }
        }
      };
      // Two record buffers in turn: the next record is loaded while one is tested.
      uint32_t ra[R], rb[R];
      load_rec(ra, 0);
#pragma unroll 1
      for (uint32_t qi = 0; qi < nq; qi += 2) {
        load_rec(rb, qi + 1 < nq ? qi + 1 : qi);
        process(ra, qi);
        if (qi + 1 >= nq) break;
        load_rec(ra, qi + 2 < nq ? qi + 2 : qi + 1);
        process(rb, qi + 1);
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nq; i += W * 64) {
      bp.tile_counts[count_row(bp, q_beg + i) * bp.n_tiles + tile] = s_cnt[i];
      s_cnt[i] = 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- rank variant

// 32 x 32 bit transpose within each half of the wave: on return lane 32 h + c holds in
// bit r what lane 32 h + r held in bit c.  One stage per index bit k (the stages
// commute): lanes r and r ^ 2^k trade the bits whose index differs from the lane's in
// bit k.  Stages 4 and 3 move whole bytes (one byte permute); stages 2..0 rotate the
// partner's word by 2^k and insert the moved bits.  Partners are fetched with DPP
// within a row of 16 lanes and with a swizzle across rows.
struct HalfTranspose {
  uint32_t m1, a1, m2, a2, m4, a4, s8, s16;
};

__device__ __forceinline__ HalfTranspose half_transpose_consts(uint32_t lane) {
  HalfTranspose c;
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4, b3 = lane & 8, b4 = lane & 16;
  c.m1 = b0 ? 0x55555555u : 0xAAAAAAAAu;
  c.a1 = b0 ? 1 : 31;   // rotate right by 1, or left by 1
  c.m2 = b1 ? 0x33333333u : 0xCCCCCCCCu;
  c.a2 = b1 ? 2 : 30;
  c.m4 = b2 ? 0x0F0F0F0Fu : 0xF0F0F0F0u;
  c.a4 = b2 ? 4 : 28;
  // Byte selectors over (partner, own): own bytes 0..3, partner bytes 4..7.
  c.s8 = b3 ? 0x03070105u : 0x06020400u;
  c.s16 = b4 ? 0x03020706u : 0x05040100u;
  return c;
}

__device__ __forceinline__ uint32_t bit_stage(uint32_t a, uint32_t p, uint32_t mask, uint32_t amt) {
  const uint32_t rot = __builtin_amdgcn_alignbit(p, p, amt);
  uint32_t r;  // (mask & rot) | (~mask & a) in one instruction
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(mask), "v"(rot), "v"(a));
  return r;
}

__device__ __forceinline__ uint32_t lane_xor16(uint32_t a) {  // swizzle: lane ^ 16 within 32
  return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(static_cast<int>(a), 0x401F));
}
__device__ __forceinline__ uint32_t lane_xor4(uint32_t a) {   // swizzle: lane ^ 4 within 32
  return static_cast<uint32_t>(__builtin_amdgcn_ds_swizzle(static_cast<int>(a), 0x101F));
}
__device__ __forceinline__ uint32_t lane_xor8(uint32_t a) {    // DPP row_ror:8
  return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(a), 0x128, 0xF, 0xF, false));
}
__device__ __forceinline__ uint32_t lane_xor2(uint32_t a) {    // DPP quad_perm [2, 3, 0, 1]
  return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(a), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ uint32_t lane_xor1(uint32_t a) {    // DPP quad_perm [1, 0, 3, 2]
  return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(a), 0xB1, 0xF, 0xF, false));
}

__device__ __forceinline__ uint32_t half_transpose(uint32_t a, const HalfTranspose& c) {
  a = __builtin_amdgcn_perm(lane_xor16(a), a, c.s16);
  a = __builtin_amdgcn_perm(lane_xor8(a), a, c.s8);
  a = bit_stage(a, lane_xor4(a), c.m4, c.a4);
  a = bit_stage(a, lane_xor2(a), c.m2, c.a2);
  a = bit_stage(a, lane_xor1(a), c.m1, c.a1);
  return a;
}

// Per group of at most 32 * SW queries and per column of the union, the host sorts the
// distinct interval ends of the group's predicates on that column (key(lo) and
// key(hi) + 1) into boundaries B[0..M), and tabulates, for every rank r in [0, M], the
// bitset of the group's queries that the column lets through when M' = r boundaries are
// <= key(x): query q with predicate [lo, hi] passes iff idx(key(lo)) < r <=
// idx(key(hi) + 1); a query without a predicate on the column always passes.  Each
// row then costs, per column, one binary search for its rank and an AND of SW table
// words -- shared by all the group's queries -- and each 32 queries a bit transpose
// per 64 rows.  Output words are stored with per-chunk marks (bp.flags), as in the
// slot-mask variant, so the words need no clearing.  Exact: the boundaries include
// every interval end, so each rank interval lies wholly inside or outside every
// predicate.  Rows past the end get the key 0, below every boundary (rank 0), where
// every predicate fails; a query without predicates carries [key(-inf), key(+inf)]
// on slot 0.
//
// The rank search is bucketed: the host maps a slot's keys monotonically to nb
// buckets, either by key (2^shift keys per bucket from the smallest boundary kmin) or
// by value (float (v - vlo) * scale, truncated), whichever leaves the fewest
// boundaries in the fullest bucket, and stores per bucket the range of its boundaries;
// a row then needs one bucket lookup and at most d binary-search steps (2^d - 1 being at
// least the fullest bucket's count), of which it reads only those inside its bucket.
//
// LDS layout of a group (words): per query, its kind and output row (kind | sparse << 2
// | row << 8), padded to 4 words; per slot a header (offset of its boundaries; M | d <<
// 12 | log2(nb) << 16 | shift << 24 | by value << 31; kmin or vlo; scale); then per slot
// the nb bucket words (index of the bucket's first end | index past its last << 16), the
// M boundaries and a word 0xFFFFFFFF, and, at a 4-word aligned offset, the table of
// (M + 1) x SW words.
template <int W, int RG, int SW, bool SPARSE>
__global__ void __launch_bounds__(W * 64) batch_rank_kernel(BatchParams bp) {
  static_assert(W * RG <= 64, "a tile must hold at least one chunk per wave");
  extern __shared__ uint32_t lds[];
  const uint32_t group = blockIdx.y;
  const uint32_t q_beg = bp.group_first[group];
  const uint32_t nq = bp.group_first[group + 1] - q_beg;
  const uint32_t t_beg = bp.group_table[group];
  const uint32_t t_len = bp.group_table[group + 1] - t_beg;
  const uint32_t ns = bp.n_slots;
  uint32_t* s_cnt = lds;
  uint32_t* s_tab = lds + ((nq + 3) & ~3u);
  for (uint32_t i = threadIdx.x; i < t_len; i += W * 64) s_tab[i] = bp.table[t_beg + i];
  for (uint32_t i = threadIdx.x; i < nq; i += W * 64) s_cnt[i] = 0;
  __syncthreads();
  const uint32_t* info = s_tab;                     // nq words
  const uint32_t* hdr = s_tab + ((nq + 3) & ~3u);   // 4 words per slot

  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const HalfTranspose tc = half_transpose_consts(lane);
  // Lane 32 h + c writes half h of query 32 w + c's words: its output row, and a mask
  // that drops the stores of count-only queries and of lanes past the group.
  // A sparse query (bit 2) stores its chunks with a hit in slots of its pool region.
  uint32_t* out[SW];
  uint32_t keep[SW], outi[SW];
  uint32_t sp = 0;   // bit w: the lane's query of word w has sparse scratch
#pragma unroll
  for (int w = 0; w < SW; ++w) {
    const uint32_t qi = 32 * w + (lane & 31);
    const uint32_t inf = qi < nq ? info[qi] : kBatchCount;
    keep[w] = (inf & 0x3u) != kBatchCount ? ~0u : 0u;
    outi[w] = keep[w] ? inf >> 8 : 0;
    const uint32_t sparse = SPARSE && keep[w] ? (inf >> 2) & 1u : 0u;
    sp |= sparse << w;
    out[w] = reinterpret_cast<uint32_t*>(bp.words + static_cast<uint64_t>(sparse ? 0u : outi[w]) * bp.n_words) +
             (lane >> 5);
  }
  constexpr uint32_t kChunkRows = 64 * RG;
  constexpr uint32_t kChunksPerWave = 4096 / kChunkRows / W;
  for (uint64_t tile = bp.tile_begin + blockIdx.x; tile < bp.tile_end; tile += gridDim.x) {
#pragma unroll 1
    for (uint32_t cw = 0; cw < kChunksPerWave; ++cw) {
      const uint64_t row0 = tile * 4096 + (wave * kChunksPerWave + cw) * kChunkRows;
      if (row0 >= bp.n_rows) break;
      const bool full = row0 + kChunkRows <= bp.n_rows;
      uint32_t acc[RG][SW];
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int w = 0; w < SW; ++w) acc[g][w] = ~0u;
#pragma unroll 1
      for (uint32_t s = 0; s < ns; ++s) {
        const uint4 h = *reinterpret_cast<const uint4*>(hdr + 4 * s);
        const uint32_t hw = __builtin_amdgcn_readfirstlane(h.y);   // uniform
        if (hw == 0) continue;  // no predicate of the group on this column
        if constexpr (SW <= 2) {
          // Early break per chunk and group (section 2.2.4): once no query of the group
          // accepts a row of the chunk, the remaining columns are not read.  (acc starts
          // all ones; each applied column clears the bits of queries beyond the group.)
          // Checked for groups of up to 64 queries, where a chunk can die: in larger
          // groups it hardly does and the test would only cost vector instructions.
          uint32_t any = 0;
#pragma unroll
          for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int w = 0; w < SW; ++w) any |= acc[g][w];
          if (__builtin_amdgcn_ballot_w64(any != 0) == 0) break;
        }
        const uint32_t M = hw & 0xFFFu, d = (hw >> 12) & 15u, nbm1 = (1u << ((hw >> 16) & 15u)) - 1;
        const uint32_t shift = (hw >> 24) & 31u;
        const bool by_value = hw >> 31;
        const uint32_t* B = s_tab + __builtin_amdgcn_readfirstlane(h.x);
        const uint32_t base = __builtin_amdgcn_readfirstlane(h.z);   // kmin, or vlo's bits
        const float scale = __uint_as_float(__builtin_amdgcn_readfirstlane(h.w));
        const uint32_t* bucket = B - (nbm1 + 1);   // per bucket: first end | past-last << 16
        const uint32_t* T = B + ((M + 1 + 3) & ~3u);
        // Keys are the raw order-preserving keys (-0 just below +0): the host places an
        // interval end at zero so that both zeros fall on the same side of it.  Bucket
        // of each row: by key, min((max(key, kmin) - kmin) >> shift, nb - 1), or by value,
        // trunc(clamp((v - vlo) * scale, 0, nb - 1)) in the host's float arithmetic.  A
        // chunk inside the data loads from one uniform base with lane offsets; in the
        // last chunk rows past the end take key 0 and bucket 0 (rank 0).
        uint32_t x[RG], bk[RG];
        const float vlo = __uint_as_float(base), top = static_cast<float>(nbm1);
        if (full) {
          const float* c = bp.slot_cols[s] + row0 + lane;
#pragma unroll
          for (int g = 0; g < RG; ++g) x[g] = __float_as_uint(__builtin_nontemporal_load(c + 64 * g));
          if (by_value) {
#pragma unroll
            for (int g = 0; g < RG; ++g) {
              const float t = (__uint_as_float(x[g]) - vlo) * scale;
              bk[g] = static_cast<uint32_t>(__builtin_amdgcn_fmed3f(t, 0.0f, top));
            }
#pragma unroll
            for (int g = 0; g < RG; ++g) x[g] = rkey(x[g]);
          } else {
#pragma unroll
            for (int g = 0; g < RG; ++g) {
              x[g] = rkey(x[g]);
              const uint32_t b = (x[g] > base ? x[g] - base : 0u) >> shift;
              bk[g] = b < nbm1 ? b : nbm1;
            }
          }
        } else {
#pragma unroll
          for (int g = 0; g < RG; ++g) {
            const uint64_t r = row0 + 64 * g + lane;
            const uint64_t rc = r < bp.n_rows ? r : bp.n_rows - 1;
            x[g] = __float_as_uint(__builtin_nontemporal_load(&bp.slot_cols[s][rc]));
          }
#pragma unroll
          for (int g = 0; g < RG; ++g) {
            const bool in = row0 + 64 * g + lane < bp.n_rows;
            const float t = (__uint_as_float(x[g]) - vlo) * scale;
            const uint32_t bv = static_cast<uint32_t>(__builtin_amdgcn_fmed3f(t, 0.0f, top));
            x[g] = in ? rkey(x[g]) : 0u;
            const uint32_t b = (x[g] > base ? x[g] - base : 0u) >> shift;
            bk[g] = !in ? 0u : by_value ? bv : b < nbm1 ? b : nbm1;
          }
        }
        // rank = number of ends <= key: the ends in lower buckets, then a binary search
        // of d steps within the row's bucket, the reads of all row groups of a step
        // issued together.  A probe past the bucket's last end would read an end of a
        // higher bucket, above every key of this one: such a probe reads the word
        // 0xFFFFFFFF after the ends instead, the same word for every lane (one broadcast,
        // no bank conflict), so a row in an empty bucket costs no conflicting reads.
        uint32_t pos[RG], lim[RG];
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          const uint32_t e = bucket[bk[g]];
          pos[g] = e & 0xFFFFu;
          lim[g] = e >> 16;
        }
#pragma unroll 1
        for (uint32_t step = (1u << d) >> 1; step > 0; step >>= 1) {
          uint32_t v[RG];
#pragma unroll
          for (int g = 0; g < RG; ++g) v[g] = B[pos[g] + step <= lim[g] ? pos[g] + step - 1 : M];
#pragma unroll
          for (int g = 0; g < RG; ++g) pos[g] = v[g] <= x[g] ? pos[g] + step : pos[g];
        }
        // One table row per row group: SW words, 4 * SW-byte aligned, in one LDS read.
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          const uint32_t* t = T + pos[g] * SW;
          if constexpr (SW == 4) {
            const uint4 r = *reinterpret_cast<const uint4*>(t);
            acc[g][0] &= r.x;
            acc[g][1] &= r.y;
            acc[g][2] &= r.z;
            acc[g][3] &= r.w;
          } else if constexpr (SW == 2) {
            const uint2 r = *reinterpret_cast<const uint2*>(t);
            acc[g][0] &= r.x;
            acc[g][1] &= r.y;
          } else {
#pragma unroll
            for (int w = 0; w < SW; ++w) acc[g][w] &= t[w];
          }
        }
      }
      // Per word of 32 queries and row group: a bit transpose within each half-wave
      // leaves in lane 32 h + c the 32 rows 64 g + 32 h + [0, 32) of query 32 w + c,
      // that is one half of its 64-row output word.  Counts are lane popcounts; words
      // are stored when not zero (the output was cleared before the scan).
      const uint64_t word0 = row0 / 64;
#pragma unroll
      for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int w = 0; w < SW; ++w) acc[g][w] = half_transpose(acc[g][w], tc);
#pragma unroll
      for (int w = 0; w < SW; ++w) {
        if (32 * w >= static_cast<int>(nq)) break;
        uint32_t cnt = 0, nz = 0;   // nz bit g: word g of the query is not zero
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          cnt += __builtin_popcount(acc[g][w]);
          nz |= (acc[g][w] != 0 ? 1u : 0u) << g;
        }
        nz = (nz | __shfl_xor(nz, 32)) & keep[w];   // lanes c and 32 + c: the two halves
        if (cnt != 0) atomicAdd(&s_cnt[32 * w + (lane & 31)], cnt);
        // Sparse query with a hit in this chunk: lane c takes a slot, lane 32 + c gets
        // it, both store their halves of all RG words there; no room: nothing stored.
        const bool sparse = SPARSE && ((sp >> w) & 1u);
        const bool take = sparse && nz != 0;
        uint32_t slot = 0;
        if constexpr (SPARSE) {
          if (take && lane < 32) slot = atomicAdd(&bp.slot_next[outi[w]], 1u);
          slot = __shfl(slot, lane & 31);
        }
        if (take) {
          if (slot < bp.sparse_cap[outi[w]]) {
            const uint64_t at = static_cast<uint64_t>(bp.sparse_base[outi[w]]) + slot;
            uint32_t* dst = reinterpret_cast<uint32_t*>(bp.pool + at * RG) + (lane >> 5);
#pragma unroll
            for (int g = 0; g < RG; ++g) dst[2 * g] = acc[g][w];
            if (lane < 32) bp.slots[static_cast<uint64_t>(outi[w]) * bp.n_chunks + row0 / kChunkRows] = slot + 1;
          }
        } else if (!sparse) {
          // Both halves of every non-zero word, and the chunk's mark (bit g <=> word g
          // was stored): the words themselves are not cleared before the scan.
#pragma unroll
          for (int g = 0; g < RG; ++g)
            if ((nz >> g) & 1u) out[w][(word0 + g) * 2] = acc[g][w];
          if (nz != 0 && lane < 32)
            bp.flags[static_cast<uint64_t>(outi[w]) * bp.n_chunks + row0 / kChunkRows] = static_cast<uint16_t>(nz);
        }
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nq; i += W * 64) {
      bp.tile_counts[count_row(bp, q_beg + i) * bp.n_tiles + tile] = s_cnt[i];
      s_cnt[i] = 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- LDS-staged variant


__device__ __forceinline__ TabPred load_pred(ctabpred* p) {
  TabPred t;
  t.slot = p->slot;
  t.klo = p->klo;
  t.kw = p->kw;
  t.pad = 0;
  return t;
}

// Keys per lane in LDS, as vectors of V = min(RG, 4) consecutive row groups.
template <int RG>
struct KeyVec;
template <>
struct KeyVec<1> {
  typedef uint32_t type;
};
template <>
struct KeyVec<2> {
  typedef uint2 type;
};
template <>
struct KeyVec<4> {
  typedef uint4 type;
};
template <>
struct KeyVec<8> {
  typedef uint4 type;
};

// As batch_scan_kernel, for unions of up to kMaxUnion columns: a chunk's keys are
// staged in LDS instead of registers, so a predicate's column is an LDS address
// (slot * stride) rather than a register slot found by branching.  Lane l writes and
// later reads only its own keys, so staging needs no barrier.  Wave layout: for slot
// s, row-group quad q and lane l, V keys at ((s * RG/V + q) * 64 + l) * V.
template <int W, int RG>
__global__ void __launch_bounds__(W * 64) batch_lds_kernel(BatchParams bp) {
  static_assert(W * RG <= 64, "a tile must hold at least one chunk per wave");
  constexpr int V = RG < 4 ? RG : 4;   // 1, 2 or 4
  constexpr int NQ = RG / V;
  typedef typename KeyVec<RG>::type vec;
  extern __shared__ uint32_t lds[];
  const uint32_t group = blockIdx.y;
  const uint32_t q_beg = bp.group_first[group];
  const uint32_t q_end = bp.group_first[group + 1];
  const uint32_t nq = q_end - q_beg;
  const uint32_t ns = bp.n_slots;
  cu32* gtab = (cu32*)(bp.table) + bp.group_table[group];  // generic -> constant address space
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x / 64;
  uint32_t* s_cnt = lds;
  uint32_t* keys = lds + ((nq + 3) & ~3u) + wave * ns * RG * 64 + lane * V;
  for (uint32_t i = threadIdx.x; i < nq; i += W * 64) s_cnt[i] = 0;
  __syncthreads();

  constexpr uint32_t kChunkRows = 64 * RG;
  constexpr uint32_t kChunksPerWave = 4096 / kChunkRows / W;
  for (uint64_t tile = bp.tile_begin + blockIdx.x; tile < bp.tile_end; tile += gridDim.x) {
#pragma unroll 1
    for (uint32_t cw = 0; cw < kChunksPerWave; ++cw) {
      const uint64_t row0 = tile * 4096 + (wave * kChunksPerWave + cw) * kChunkRows;
      if (row0 >= bp.n_rows) break;
      const bool full = row0 + kChunkRows <= bp.n_rows;
      // Stage the keys; rows past the end get 0xFFFFFFFF, above the key of every
      // non-NaN float, so the first predicate of every query rejects them.
#pragma unroll 1
      for (uint32_t s = 0; s < ns; ++s) {
        const float* col = bp.slot_cols[s];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          uint32_t k[V];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const uint64_t r = row0 + 64 * (q * V + v) + lane;
            k[v] = (full || r < bp.n_rows) ? dkey(__builtin_nontemporal_load(&col[r])) : 0xFFFFFFFFu;
          }
          vec kv;
          if constexpr (V == 1) {
            kv = k[0];
          } else if constexpr (V == 2) {
            kv = vec{k[0], k[1]};
          } else {
            kv = vec{k[0], k[1], k[2], k[3]};
          }
          *reinterpret_cast<vec*>(keys + (s * NQ + q) * 64 * V) = kv;
        }
      }
      const uint64_t word0 = row0 / 64;
      cu32* rec = gtab + gtab[0];
#pragma unroll 1
      for (uint32_t qi = 0; qi < nq; ++qi) {
        const uint32_t head = rec[0];
        const uint32_t np = head & 0xFFu;   // >= 1: the host gives an empty query an
                                            // always-true predicate
        const uint32_t kind = (head >> 8) & 0x3u;
        ctabpred* tp = reinterpret_cast<ctabpred*>(rec + 4);
        rec += 4 + 4 * np;
        // Two forms of the range test.  With four or more rows per lane: the median of
        // three folded into acc[g], which stays zero in lanes whose row passes every
        // predicate so far (vector work only).  With fewer: subtract and compare into
        // the wave masks m[g] (one scalar AND per test, but no per-predicate setup to
        // amortise over few rows).
        constexpr bool kMed3 = RG >= 4;
        uint32_t acc[RG];
        uint64_t m[RG];
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          acc[g] = 0;
          m[g] = ~uint64_t{0};
        }
        auto apply = [&](const TabPred& t) {
          const uint32_t* kp = keys + t.slot * (NQ * 64 * V);
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const vec kv = *reinterpret_cast<const vec*>(kp + q * 64 * V);
            uint32_t k[V];
            if constexpr (V == 1) {
              k[0] = kv;
            } else if constexpr (V == 2) {
              k[0] = kv.x;
              k[1] = kv.y;
            } else {
              k[0] = kv.x;
              k[1] = kv.y;
              k[2] = kv.z;
              k[3] = kv.w;
            }
            if constexpr (kMed3) {
              uint32_t r[V];
#pragma unroll
              for (int v = 0; v < V; ++v) r[v] = med3u(k[v], t.klo, t.kw);  // kw: key(hi)
#pragma unroll
              for (int v = 0; v < V; ++v) acc[q * V + v] |= r[v] ^ k[v];
            } else {
              const uint32_t w = t.kw - t.klo;
#pragma unroll
              for (int v = 0; v < V; ++v) m[q * V + v] &= ballot(k[v] - t.klo <= w);
            }
          }
        };
        auto all_rejected = [&]() {
          if constexpr (kMed3) {
            uint32_t mn = acc[0];
#pragma unroll
            for (int g = 1; g < RG; ++g) mn = mn < acc[g] ? mn : acc[g];
            return ballot(mn == 0) == 0;
          } else {
            uint64_t any = 0;
#pragma unroll
            for (int g = 0; g < RG; ++g) any |= m[g];
            return any == 0;
          }
        };
        // Predicates in the query's order, two at a time; the early break of the
        // whole chunk is tested after each pair.
        bool dead = false;
        uint32_t pi = 0;
#pragma unroll 1
        for (; pi + 1 < np; pi += 2) {
          const TabPred t0 = load_pred(tp + pi), t1 = load_pred(tp + pi + 1);
          apply(t0);
          apply(t1);
          if (pi + 2 < np && all_rejected()) {
            dead = true;
            break;
          }
        }
        if (dead) continue;
        if (pi < np) apply(load_pred(tp + pi));
        uint32_t c = 0;
#pragma unroll
        for (int g = 0; g < RG; ++g) {
          if constexpr (kMed3) m[g] = ballot(acc[g] == 0);
          c += __popcll(m[g]);
        }
        if (c != 0) {
          if (lane == 0) atomicAdd(&s_cnt[qi], c);
          if (kind != kBatchCount) {
            uint64_t* words = bp.words + static_cast<uint64_t>(head >> 16) * bp.n_words + word0;
#pragma unroll
            for (int g = 0; g < RG; ++g)
              if (m[g] != 0 && lane == 0) words[g] = m[g];
          }
        }
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nq; i += W * 64) {
      bp.tile_counts[count_row(bp, q_beg + i) * bp.n_tiles + tile] = s_cnt[i];
      s_cnt[i] = 0;
    }
    __syncthreads();
  }
}

// Zero a range of 64-bit words (the bitmap scratch before a shared scan).
__global__ void __launch_bounds__(256) zero_words_kernel(uint64_t* w, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 256;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride)
    w[i] = 0;
}

// p[0, n) = v.
__global__ void __launch_bounds__(256) fill_u16_kernel(uint16_t* p, uint64_t n, uint16_t v) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 256;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Zero rows rows[y] of row_words 64-bit words each (workgroup row y of the grid).
__global__ void __launch_bounds__(256) zero_rows_kernel(uint64_t* base, uint64_t row_words, const uint32_t* rows) {
  uint64_t* w = base + static_cast<uint64_t>(rows[blockIdx.y]) * row_words;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 256;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x; i < row_words; i += stride) w[i] = 0;
}

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

constexpr uint32_t kEmitTiles = 128;   // tiles per emit chunk (two per lane of one wave)
constexpr uint32_t kEmitStage = 2048;  // ids per wave staged in LDS (tiles of up to 4096)
// Tiles of at most this many ids skip the staging: their lanes hold one id or a few, so
// the direct writes of one step already fall on consecutive positions.
constexpr uint32_t kEmitDirect = 64;
static_assert(kEmitTiles == 2 * 64, "one wave sums an emit chunk, two tiles per lane");

// Inclusive prefix sum over the wave's lanes by DPP: shifts by 1, 2, 4, 8 within each
// row of 16 lanes, then row 0's and row 2's last lane added to rows 1 and 3, then lane
// 31 to rows 2 and 3 (lanes with no source add 0).
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
  // The row shifts read 0 where the source lane is outside the row (bound control), so
  // they need no zeroed register and can fold into the adds.
  v += static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x111, 0xF, 0xF, true));
  v += static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x112, 0xF, 0xF, true));
  v += static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x114, 0xF, 0xF, true));
  v += static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x118, 0xF, 0xF, true));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xA, 0xF, false));
  v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xC, 0xF, false));
  return v;
}

__device__ __forceinline__ uint64_t finish_row(const BatchFinish& f, uint32_t q) {
  return f.count_row ? f.count_row[q] : q;
}

// Pass 0, workgroup (x, q): one wave per emit chunk sums query q's tile counts over the
// chunk's tiles, into the query's row of chunk sums.  Every chunk's workgroup runs at
// once, so the count of a query no longer waits on one workgroup walking all its tiles.
__global__ void __launch_bounds__(kFinThreads) batch_chunk_kernel(BatchFinish f) {
  const uint32_t q = blockIdx.y;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t c = static_cast<uint64_t>(blockIdx.x) * kFinWaves + threadIdx.x / 64;
  const uint64_t n_emit = (f.n_tiles + kEmitTiles - 1) / kEmitTiles;
  if (c >= n_emit) return;
  const uint64_t row = finish_row(f, q);
  const uint32_t* counts = f.tile_counts + row * f.n_tiles;
  const uint64_t t = c * kEmitTiles + 2 * lane;
  const uint32_t v = (t < f.n_tiles ? counts[t] : 0u) + (t + 1 < f.n_tiles ? counts[t + 1] : 0u);
  const uint32_t total = __builtin_amdgcn_readlane(wave_incl_sum(v), 63);
  if (lane == 0) f.chunk_pos[row * n_emit + c] = total;
}

// Pass 1, workgroup q: the exact count of query q and its output kind (AUTO picks,
// from the exact count, whichever of bitmap and identifiers is smaller and fits the
// buffer); for identifier output the chunk sums are replaced, in place, by their
// exclusive prefix sums (each chunk's first output position).
__global__ void __launch_bounds__(kFinThreads) batch_count_kernel(BatchFinish f) {
  __shared__ uint32_t s_wave[kFinWaves];
  const uint32_t q = blockIdx.x;
  const BatchOut o = f.outs[q];
  const uint32_t tid = threadIdx.x;
  const uint64_t n_emit = (f.n_tiles + kEmitTiles - 1) / kEmitTiles;
  uint32_t* sums = f.chunk_pos + finish_row(f, q) * n_emit;
  uint64_t part = 0;
  for (uint64_t c = tid; c < n_emit; c += kFinThreads) part += sums[c];
  uint32_t ignore;
  const uint64_t count = block_scan(static_cast<uint32_t>(part), ignore, s_wave);
  uint32_t kind = o.kind;
  if (kind == kBatchAuto) {
    const uint64_t bitmap_bytes = 8 * f.n_words;
    const bool fits_bitmap = o.buf_bytes >= bitmap_bytes;
    kind = (fits_bitmap && (bitmap_bytes < 4 * count || o.buf_bytes < 4 * count)) ? kBatchBitmap
                                                                                 : kBatchIds;
  }
  const bool over = o.sparse && f.slot_next[o.out_index] > f.sparse_cap[o.out_index];
  if (tid == 0) {
    f.counts_out[q] = count;
    f.kind_out[q] = kind;
    if (f.over_out) f.over_out[q] = over ? 1u : 0u;
  }
  if (kind != kBatchIds || count == 0 || over) return;
  uint32_t carry = 0;
  for (uint64_t c0 = 0; c0 < n_emit; c0 += kFinScan) {
    const uint32_t nc = static_cast<uint32_t>(n_emit - c0 < kFinScan ? n_emit - c0 : kFinScan);
    uint32_t v[8];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t c = tid * 8 + i;
      v[i] = c < nc ? sums[c0 + c] : 0u;
      sum += v[i];
    }
    uint32_t excl;
    const uint32_t total = block_scan(sum, excl, s_wave);
    excl += carry;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t c = tid * 8 + i;
      if (c < nc) sums[c0 + c] = excl;
      excl += v[i];
    }
    carry += total;
  }
}

// Word w of query q's scratch row: zero unless the scan marked it as stored.  The word
// and its mark are loaded independently (both in bounds), then combined.
__device__ __forceinline__ uint64_t scratch_word(const BatchFinish& f, const uint64_t* words,
                                                 uint64_t out_index, uint64_t w) {
  const uint64_t v = words[w];
  if (!f.flags) return v;
  const uint32_t mark = f.flags[out_index * f.n_chunks + (w >> f.chunk_shift)];
  return (mark >> (w & ((1u << f.chunk_shift) - 1))) & 1u ? v : 0;
}

// Word w of a sparse query's scratch: in its chunk's slot if the chunk was stored, else
// zero.
__device__ __forceinline__ uint64_t sparse_word(const BatchFinish& f, uint32_t si, uint64_t w) {
  const uint32_t slot = f.slots[static_cast<uint64_t>(si) * f.n_chunks + (w >> f.chunk_shift)];
  if (slot == 0) return 0;
  const uint64_t at = (static_cast<uint64_t>(f.sparse_base[si]) + slot - 1) << f.chunk_shift;
  return f.pool[at + (w & ((1u << f.chunk_shift) - 1))];
}

// The caller's output buffer as global memory.  Its address comes from a table in memory,
// where the compiler cannot tell its address space; a generic (flat) store would also
// count against the wave's LDS wait counter, so every LDS read after it would wait for the
// store to complete.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* global_out(void* p) {
  return reinterpret_cast<__attribute__((address_space(1))) T*>(reinterpret_cast<uintptr_t>(p));
}

// Pass 2, workgroup (c, q): tiles [c * kEmitTiles, (c + 1) * kEmitTiles) of query q.
// Bitmap output copies the tiles' words; identifier output compacts each tile with a
// hit (one wave per tile) at the tile's first output position (its chunk's
// position plus the tile counts before it in the chunk), so the identifiers come
// out ascending.  Nothing beyond the caller's capacity is written.
__global__ void __launch_bounds__(kFinThreads) batch_emit_kernel(BatchFinish f) {
  const uint32_t q = blockIdx.y;
  const uint32_t kind = f.kind_out[q];
  const uint64_t count = f.counts_out[q];
  if (kind == kBatchCount || (kind == kBatchIds && count == 0)) return;
  const BatchOut o = f.outs[q];
  // A sparse query whose slots ran out is answered again by the host.
  if (o.sparse && f.slot_next[o.out_index] > f.sparse_cap[o.out_index]) return;
  const uint64_t t_beg = static_cast<uint64_t>(blockIdx.x) * kEmitTiles;
  if (t_beg >= f.n_tiles) return;
  const uint64_t t_end = t_beg + kEmitTiles < f.n_tiles ? t_beg + kEmitTiles : f.n_tiles;
  const uint64_t* words = f.words + static_cast<uint64_t>(o.sparse ? 0u : o.out_index) * f.n_words;
  const bool sparse = o.sparse != 0;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63;
  const uint32_t wave = tid / 64;
  if (kind == kBatchBitmap) {
    const uint64_t cap = o.buf_bytes / 8;
    const uint64_t lim = cap < f.n_words ? cap : f.n_words;
    const uint64_t w_end = t_end * 64 < lim ? t_end * 64 : lim;
    auto* dst = global_out<uint64_t>(o.buf);
    // Four words per lane loaded before any is stored, so that a store's completion (which
    // the next load's wait also covers) is not waited for once per word.
    for (uint64_t i0 = t_beg * 64 + tid; i0 < w_end; i0 += 4 * kFinThreads) {
      uint64_t v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint64_t i = i0 + static_cast<uint64_t>(j) * kFinThreads;
        v[j] = i >= w_end ? 0 : sparse ? sparse_word(f, o.out_index, i) : scratch_word(f, words, o.out_index, i);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint64_t i = i0 + static_cast<uint64_t>(j) * kFinThreads;
        if (i < w_end) dst[i] = v[j];
      }
    }
    return;
  }
  // The tiles' output positions (and the end of the last) into LDS in one pass.
  __shared__ uint32_t s_pos[kEmitTiles + 1];
  __shared__ uint16_t s_stage[kFinWaves][kEmitStage];
  if (wave == 0) {   // two tiles per lane; lanes past the last tile add zeros
    const uint64_t row = finish_row(f, q);
    const uint32_t* counts = f.tile_counts + row * f.n_tiles;
    const uint32_t base = f.chunk_pos[row * ((f.n_tiles + kEmitTiles - 1) / kEmitTiles) + blockIdx.x];
    const uint64_t t = t_beg + 2 * lane;
    const uint32_t a = t < t_end ? counts[t] : 0u;
    const uint32_t b = t + 1 < t_end ? counts[t + 1] : 0u;
    const uint32_t incl = wave_incl_sum(a + b);
    s_pos[2 * lane] = base + incl - (a + b);
    s_pos[2 * lane + 1] = base + incl - b;
    if (lane == 63) s_pos[kEmitTiles] = base + incl;
  }
  __syncthreads();
  auto* ids = global_out<uint32_t>(o.buf);
  const uint64_t capacity = o.buf_bytes / 4;
  // Tiles are taken per wave, so a tile's position and whether it has a hit inside the
  // caller's capacity are the same for all its lanes: kept in scalar registers.
  auto pos_of = [&](uint64_t t) {
    return static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(s_pos[static_cast<uint32_t>(t - t_beg)]));
  };
  auto hit = [&](uint64_t t) {
    const uint32_t a = pos_of(t);
    return pos_of(t + 1) != a && a < capacity;
  };
  // One tile = 64 words = one wave-wide load.  A word and its chunk's mark are loaded
  // as they are and combined only when the tile is written, so the loads of the wave's
  // next tile stay in flight while the current one is written.  (A chunk holds
  // 2^chunk_shift words and a tile 64, so a lane's bit in its chunk's mark is its lane
  // index modulo 2^chunk_shift.)
  const uint32_t mark_bit = lane & ((1u << f.chunk_shift) - 1);
  uint64_t next_word = 0;
  uint32_t next_mark = ~0u;   // all bits: no marks, a sparse query's word, or past the end
  auto load = [&](uint64_t t) {
    const uint64_t w = t * 64 + lane;
    next_word = 0;
    next_mark = ~0u;
    if (w >= f.n_words) return;
    if (sparse) {
      next_word = sparse_word(f, o.out_index, w);
    } else {
      next_word = words[w];
      if (f.flags) next_mark = f.flags[static_cast<uint64_t>(o.out_index) * f.n_chunks + (w >> f.chunk_shift)];
    }
  };
  uint64_t t = t_beg + static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(wave));
  if (t < t_end && hit(t)) load(t);
  for (; t < t_end; t += kFinWaves) {
    const bool use = hit(t);
    const uint64_t word = (next_mark >> mark_bit) & 1u ? next_word : 0;
    const uint64_t tn = t + kFinWaves;
    if (tn < t_end && hit(tn)) load(tn);
    if (!use) continue;
    const uint64_t beg = pos_of(t);
    const uint64_t w = t * 64 + lane;
    const uint32_t k = __popcll(word);
    const uint32_t incl = wave_incl_sum(k);
    const uint32_t total = __builtin_amdgcn_readlane(incl, 63);   // ids of the tile
    uint64_t bits = word;
    const uint32_t row = static_cast<uint32_t>(w * 64);
    if (total > kEmitDirect && total <= kEmitStage) {
      // Each lane's rows (16-bit offsets in the tile) into the wave's LDS buffer at
      // their places in the tile's output, then out to HBM in consecutive 64-lane runs.
      uint16_t* buf = s_stage[wave];
      uint32_t r = incl - k;
      const uint32_t off = lane * 64;
      while (bits) {
        buf[r++] = static_cast<uint16_t>(off + static_cast<uint32_t>(__builtin_ctzll(bits)));
        bits &= bits - 1;
      }
      const uint32_t tile_row = static_cast<uint32_t>(t * 4096);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (uint32_t i0 = 0; i0 < total; i0 += 256) {   // four runs' reads in flight
        uint32_t v[4];   // read unconditionally (index 0 past the end), so the reads go together
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t i = i0 + 64 * j + lane;
          v[j] = tile_row + buf[i < total ? i : 0u];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t i = i0 + 64 * j + lane;
          if (i < total && beg + i < capacity) ids[beg + i] = v[j];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else if (total > kEmitStage) {
      // A dense tile, word by word: lane l takes bit l of the word, whose place is the
      // word's offset plus the set bits below it, so each store is one run of ids.
      const uint32_t before = incl - k;
      const uint32_t tile_row = static_cast<uint32_t>(t * 4096);
      const uint32_t wlo = static_cast<uint32_t>(word);
      const uint32_t whi = static_cast<uint32_t>(word >> 32);
      for (uint32_t j = 0; j < 64; ++j) {
        const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(wlo), static_cast<int>(j)));
        const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(whi), static_cast<int>(j)));
        const uint32_t at = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(before), static_cast<int>(j)));
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
        const bool set = (((static_cast<uint64_t>(hi) << 32 | lo) >> lane) & 1u) != 0;
        const uint64_t r = beg + at + below;
        if (set && r < capacity) ids[r] = tile_row + 64 * j + lane;
      }
    } else {  // a sparse tile: each lane writes its ids directly
      uint64_t r = beg + incl - k;
      while (bits) {
        const uint32_t b = static_cast<uint32_t>(__builtin_ctzll(bits));
        if (r < capacity) ids[r] = row + b;
        ++r;
        bits &= bits - 1;
      }
    }
  }
}

template <int D, int W, int RG>
const void* scan_fn(bool walk) {
  return walk ? reinterpret_cast<const void*>(&batch_scan_kernel<D, W, RG, true>)
              : reinterpret_cast<const void*>(&batch_scan_kernel<D, W, RG, false>);
}

// Register budget: D slots x RG rows per lane stays at or below 128 VGPRs.
const void* pick_batch(int d, int w, int rg, bool walk) {
  const int dd = d <= 4 ? 4 : d <= 8 ? 8 : 16;
  if (dd == 4) {
    if (rg == 16) return scan_fn<4, 4, 16>(walk);
    if (rg == 8) return w == 8 ? scan_fn<4, 8, 8>(walk) : scan_fn<4, 4, 8>(walk);
    return w == 8 ? scan_fn<4, 8, 4>(walk) : scan_fn<4, 4, 4>(walk);
  }
  if (dd == 8) {
    if (rg == 16) return scan_fn<8, 4, 16>(walk);
    if (rg == 8) return w == 8 ? scan_fn<8, 8, 8>(walk) : scan_fn<8, 4, 8>(walk);
    return w == 8 ? scan_fn<8, 8, 4>(walk) : scan_fn<8, 4, 4>(walk);
  }
  if (rg >= 8) return w == 8 ? scan_fn<16, 8, 8>(walk) : scan_fn<16, 4, 8>(walk);
  return w == 8 ? scan_fn<16, 8, 4>(walk) : scan_fn<16, 4, 4>(walk);
}

template <int D, int W, int RG>
const void* reg_fn() {
  return reinterpret_cast<const void*>(&batch_reg_kernel<D, W, RG>);
}

const void* pick_reg(int d, int w, int rg) {
  const int dd = batch_reg_slots(d);
  if (dd == 4) {
    if (rg == 16) return reg_fn<4, 4, 16>();
    if (rg == 8) return w == 8 ? reg_fn<4, 8, 8>() : reg_fn<4, 4, 8>();
    return w == 8 ? reg_fn<4, 8, 4>() : reg_fn<4, 4, 4>();
  }
  if (dd == 8) {
    if (rg == 16) return reg_fn<8, 4, 16>();
    if (rg == 8) return w == 8 ? reg_fn<8, 8, 8>() : reg_fn<8, 4, 8>();
    return w == 8 ? reg_fn<8, 8, 4>() : reg_fn<8, 4, 4>();
  }
  if (dd == 12) {
    if (rg >= 8) return w == 8 ? reg_fn<12, 8, 8>() : reg_fn<12, 4, 8>();
    return w == 8 ? reg_fn<12, 8, 4>() : reg_fn<12, 4, 4>();
  }
  if (rg >= 8) return w == 8 ? reg_fn<16, 8, 8>() : reg_fn<16, 4, 8>();
  return w == 8 ? reg_fn<16, 8, 4>() : reg_fn<16, 4, 4>();
}

const void* pick_rank(int w, int rg, int sw, bool sparse) {
#define MDRQ_RANK(W_, RG_, SP_)                                                              \
  (sw <= 1 ? reinterpret_cast<const void*>(&batch_rank_kernel<W_, RG_, 1, SP_>)               \
   : sw == 2 ? reinterpret_cast<const void*>(&batch_rank_kernel<W_, RG_, 2, SP_>)             \
             : reinterpret_cast<const void*>(&batch_rank_kernel<W_, RG_, 4, SP_>))
  // Sparse scratch only with 8 row groups per lane (512-row chunks).
  if (sparse) return w == 8 ? MDRQ_RANK(8, 8, true) : MDRQ_RANK(4, 8, true);
  if (rg >= 8) return w == 8 ? MDRQ_RANK(8, 8, false) : MDRQ_RANK(4, 8, false);
  return w == 8 ? MDRQ_RANK(8, 4, false) : MDRQ_RANK(4, 4, false);
#undef MDRQ_RANK
}

const void* pick_lds(int w, int rg) {
  if (rg >= 8) return w == 8 ? reinterpret_cast<const void*>(&batch_lds_kernel<8, 8>)
                             : reinterpret_cast<const void*>(&batch_lds_kernel<4, 8>);
  if (rg == 4) return w == 8 ? reinterpret_cast<const void*>(&batch_lds_kernel<8, 4>)
                             : reinterpret_cast<const void*>(&batch_lds_kernel<4, 4>);
  if (rg == 2) return w == 8 ? reinterpret_cast<const void*>(&batch_lds_kernel<8, 2>)
                             : reinterpret_cast<const void*>(&batch_lds_kernel<4, 2>);
  return w == 8 ? reinterpret_cast<const void*>(&batch_lds_kernel<8, 1>)
                : reinterpret_cast<const void*>(&batch_lds_kernel<4, 1>);
}

int lds_rows(int rg) { return rg >= 8 ? 8 : rg >= 4 ? 4 : rg >= 2 ? 2 : 1; }

}  // namespace

uint32_t batch_key(float x) {
  uint32_t b;
  std::memcpy(&b, &x, sizeof b);
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

int batch_reg_slots(int n_slots) {
  return n_slots <= 4 ? 4 : n_slots <= 8 ? 8 : n_slots <= 12 ? 12 : 16;
}

size_t batch_lds_key_bytes(int n_slots, int waves, int rg) {
  return static_cast<size_t>(waves == 8 ? 8 : 4) * n_slots * lds_rows(rg) * 64 * 4;
}

int batch_rows_per_lane(int n_slots, int waves, int rg) {
  (void)n_slots;
  if (rg == 16 && waves == 8) rg = 8;
  if (n_slots > 8 && rg == 16) rg = 8;
  return rg == 16 || rg == 8 ? rg : 4;
}

namespace {
const void* pick_scan(int n_slots, int w, int rg, int lds_variant, int sw) {
  if (lds_variant == 1) return pick_lds(w, rg);
  if (lds_variant == 4) return pick_rank(w, rg >= 8 ? 8 : 4, sw, false);
  if (lds_variant == 5) return pick_rank(w, 8, sw, true);
  if (lds_variant == 3) return pick_reg(n_slots, w, batch_rows_per_lane(n_slots, w, rg));
  return pick_batch(n_slots, w, batch_rows_per_lane(n_slots, w, rg), lds_variant == 2);
}
}  // namespace

int batch_blocks_per_cu(int n_slots, int waves, int rg, int lds_variant, size_t lds_bytes, int sw) {
  int blocks = 0;
  const int w = waves == 8 ? 8 : 4;
  const void* fn = pick_scan(n_slots, w, rg, lds_variant, sw);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, w * 64, lds_bytes) != hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

hipError_t launch_zero_words(uint64_t* w, uint64_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
  zero_words_kernel<<<static_cast<uint32_t>(blocks), 256, 0, stream>>>(w, n);
  return hipGetLastError();
}

hipError_t launch_fill_u16(uint16_t* p, uint64_t n, uint16_t v, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 4096);
  fill_u16_kernel<<<static_cast<uint32_t>(blocks), 256, 0, stream>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_zero_rows(uint64_t* base, uint64_t row_words, const uint32_t* rows, uint32_t n_rows,
                            hipStream_t stream) {
  if (n_rows == 0 || row_words == 0) return hipSuccess;
  const uint64_t blocks = std::min<uint64_t>((row_words + 255) / 256, 256);
  zero_rows_kernel<<<dim3(static_cast<uint32_t>(blocks), n_rows), 256, 0, stream>>>(base, row_words, rows);
  return hipGetLastError();
}

hipError_t launch_batch_scan(const BatchParams& bp, int n_slots, int waves, int rg, int lds_variant,
                             dim3 grid, size_t lds_bytes, hipStream_t stream, int sw) {
  const int w = waves == 8 ? 8 : 4;
  // Zero the scratch rows, or only their chunk marks (slot-mask variant).
  const uint64_t n = bp.flags ? bp.n_zero : bp.n_words * bp.n_out;
  if (n) {
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
    zero_words_kernel<<<static_cast<uint32_t>(blocks), 256, 0, stream>>>(
        bp.flags ? reinterpret_cast<uint64_t*>(bp.flags) : bp.words, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  void* args[] = {const_cast<BatchParams*>(&bp)};
  const void* fn = pick_scan(n_slots, w, rg, lds_variant, sw);
  if (lds_bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds_bytes));
    if (e != hipSuccess) return e;
  }
  return hipLaunchKernel(fn, grid, dim3(w * 64), args, lds_bytes, stream);
}

hipError_t batch_launches(const BatchParams& bp, const BatchFinish& f, uint32_t n_queries, int n_slots, int waves,
                          int rg, int lds_variant, dim3 grid, size_t lds_bytes, int sw, BatchLaunches* L) {
  const int w = waves == 8 ? 8 : 4;
  L->bp = bp;
  L->fin = f;
  L->zero_ptr = bp.flags ? reinterpret_cast<uint64_t*>(bp.flags) : bp.words;
  L->zero_n = bp.flags ? bp.n_zero : bp.n_words * bp.n_out;
  L->zero_args[0] = &L->zero_ptr;
  L->zero_args[1] = &L->zero_n;
  L->scan_args[0] = &L->bp;
  L->fin_args[0] = &L->fin;
  auto node = [](const void* fn, dim3 g, uint32_t threads, size_t shmem, void** args) {
    hipKernelNodeParams k{};
    k.func = const_cast<void*>(fn);
    k.gridDim = g;
    k.blockDim = dim3(threads);
    k.sharedMemBytes = static_cast<unsigned int>(shmem);
    k.kernelParams = args;
    k.extra = nullptr;
    return k;
  };
  const uint64_t zb = std::max<uint64_t>(1, std::min<uint64_t>((L->zero_n + 255) / 256, 65536));
  L->zero = node(reinterpret_cast<const void*>(&zero_words_kernel), dim3(static_cast<uint32_t>(zb)), 256, 0,
                 L->zero_args);
  const void* fn = pick_scan(n_slots, w, rg, lds_variant, sw);
  if (lds_bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_bytes));
    if (e != hipSuccess) return e;
  }
  L->scan = node(fn, grid, static_cast<uint32_t>(w * 64), lds_bytes, L->scan_args);
  const uint32_t chunks = static_cast<uint32_t>(std::max<uint64_t>(1, batch_emit_chunks(f.n_tiles)));
  L->chunk = node(reinterpret_cast<const void*>(&batch_chunk_kernel), dim3((chunks + kFinWaves - 1) / kFinWaves, n_queries),
                  kFinThreads, 0, L->fin_args);
  L->count = node(reinterpret_cast<const void*>(&batch_count_kernel), dim3(n_queries), kFinThreads, 0, L->fin_args);
  L->emit = node(reinterpret_cast<const void*>(&batch_emit_kernel), dim3(chunks, n_queries), kFinThreads, 0,
                 L->fin_args);
  return hipSuccess;
}

uint64_t batch_emit_chunks(uint64_t n_tiles) { return (n_tiles + kEmitTiles - 1) / kEmitTiles; }

hipError_t launch_batch_finish(const BatchFinish& f, uint32_t n_queries, hipStream_t stream) {
  if (n_queries == 0) return hipSuccess;
  const uint32_t chunks = static_cast<uint32_t>(batch_emit_chunks(f.n_tiles));
  if (chunks) batch_chunk_kernel<<<dim3((chunks + kFinWaves - 1) / kFinWaves, n_queries), kFinThreads, 0, stream>>>(f);
  batch_count_kernel<<<n_queries, kFinThreads, 0, stream>>>(f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || f.n_tiles == 0) return e;
  batch_emit_kernel<<<dim3(chunks, n_queries), kFinThreads, 0, stream>>>(f);
  return hipGetLastError();
}

}  // namespace mdrq
