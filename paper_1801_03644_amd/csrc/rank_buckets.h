// Bucket maps of the rank variant's search (host side, plain C++: the kernel repeats
// the value map's float arithmetic exactly, and a CPU test checks these functions
// against brute force).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace mdrq {

constexpr uint32_t kRankBuckets = 1024;  // most buckets of a rank search

// Buckets of the rank search over sorted distinct interval ends, either by key (nb
// buckets of 2^shift keys from the smallest end, the last open above) or by value
// (bucket min(trunc(clamp((v - vlo) * scale, 0, nb - 1))) of a float v, in float
// arithmetic that the kernel repeats exactly; an end above key(+inf) goes to the last
// bucket).  Both maps are monotone in the key order, so an end in a lower bucket is
// below every key of a higher one.  The starts count the ends in lower buckets, and d
// is the number of binary-search steps that resolve the fullest bucket.  Of the maps
// and bucket counts (powers of two up to kRankBuckets) tried, the one with the fewest
// steps wins, key before value and the fewer buckets on a tie.
struct RankBuckets {
  uint32_t nb = 0, shift = 0, d = 0;
  bool by_value = false;
  float vlo = 0.0f, scale = 1.0f;
  std::vector<uint16_t> starts;
};

inline float key_value(uint32_t k) {  // the float of an order-preserving key (NaN above +inf)
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  float v;
  std::memcpy(&v, &b, sizeof v);
  return v;
}

inline uint32_t value_bucket(float v, float vlo, float scale, uint32_t nbm1) {
  if (v != v) return nbm1;  // NaN: an end above key(+inf)
  const float t = (v - vlo) * scale;
  // trunc(clamp(t, 0, nb - 1)); t is never NaN here (v, vlo finite or infinite, scale
  // finite and positive, and v - vlo is not inf - inf as vlo is finite)
  if (!(t > 0.0f)) return 0;
  return t < static_cast<float>(nbm1) ? static_cast<uint32_t>(t) : nbm1;
}

// Candidate bucket maps of sorted distinct ends, each with its search steps d (starts
// not built).  mode: 0 both maps, 1 by key only, 2 by value only (by key where that is
// impossible); max_nb: the most buckets (a power of two, 8 .. kRankBuckets); no more
// than about 4 per end are tried.  Because both maps are monotone and the ends sorted,
// the ends of a bucket are consecutive, so the fullest bucket is the longest run of
// equal bucket numbers: one pass per candidate, nothing allocated.  Halving the bucket
// count merges buckets in pairs under either map (the key map's shift grows by one,
// the value map's scale halves exactly), so d never falls as buckets are halved: each
// map is walked down from its most buckets and left once d has grown, and the last
// candidate kept is that map's fewest buckets with its fewest steps.
inline std::vector<RankBuckets> bucket_candidates(const std::vector<uint32_t>& ends, int mode,
                                                  uint32_t max_nb) {
  const uint32_t M = static_cast<uint32_t>(ends.size());
  const uint32_t kmin = ends.front(), span = ends.back() - kmin;
  std::vector<RankBuckets> out;
  uint32_t cap = 8;
  while (cap < max_nb && cap < 4 * M) cap *= 2;
  auto steps = [](uint32_t fullest) { return 32 - static_cast<uint32_t>(__builtin_clz(fullest)); };
  auto walk = [&](auto&& make, auto&& bucket_of) {
    uint32_t d_top = 0;
    for (uint32_t nb = cap; nb >= 8; nb /= 2) {
      RankBuckets m = make(nb);
      uint32_t fullest = 0, run = 0, prev = 0xFFFFFFFFu;
      for (uint32_t i = 0; i < M; ++i) {
        const uint32_t b = bucket_of(m, i);
        run = b == prev ? run + 1 : 1;
        prev = b;
        fullest = std::max(fullest, run);
      }
      m.d = steps(fullest);
      if (nb == cap) d_top = m.d;
      if (m.d > d_top) break;
      out.push_back(m);
    }
  };
  if (mode != 2)
    walk(
        [&](uint32_t nb) {
          RankBuckets m;
          m.nb = nb;
          while ((span >> m.shift) > nb - 1) ++m.shift;
          return m;
        },
        [&](const RankBuckets& m, uint32_t i) { return std::min<uint32_t>((ends[i] - kmin) >> m.shift, m.nb - 1); });
  if (mode == 1) return out;
  std::vector<float> vals(M);
  float vlo = std::numeric_limits<float>::infinity(), vhi = -vlo;
  for (uint32_t i = 0; i < M; ++i) {
    vals[i] = key_value(ends[i]);
    if (std::isfinite(vals[i])) {
      vlo = std::min(vlo, vals[i]);
      vhi = std::max(vhi, vals[i]);
    }
  }
  // The value map only where the host's float arithmetic on the ends cannot meet a
  // subnormal that a flush-to-zero mode of the calling thread could change: a span of
  // at least 2^-90 (scale at most 2^100) and a zero or normal lower end of at least
  // 2^-100 in magnitude.  A subnormal end or key then lands in the bucket it would get
  // exactly (the difference rounds to -vlo, or the product truncates to 0).
  const bool value_ok = vlo < vhi && std::isfinite(vhi - vlo) && vhi - vlo >= 0x1p-90f &&
                        (vlo == 0.0f || std::fabs(vlo) >= 0x1p-100f);
  if (!value_ok) return mode == 2 ? bucket_candidates(ends, 1, max_nb) : out;
  walk(
      [&](uint32_t nb) {
        RankBuckets m;
        m.nb = nb;
        m.by_value = true;
        m.vlo = vlo;
        m.scale = static_cast<float>(nb) / (vhi - vlo);
        return m;
      },
      [&](const RankBuckets& m, uint32_t i) { return value_bucket(vals[i], m.vlo, m.scale, m.nb - 1); });
  return out;
}

// The preferred candidate with at most cap buckets: the fewest steps, then the key map,
// then the fewest buckets.
inline RankBuckets pick_buckets(const std::vector<RankBuckets>& c, uint32_t cap) {
  RankBuckets best;
  for (const RankBuckets& m : c) {
    if (m.nb > cap) continue;
    if (best.nb == 0 || m.d < best.d ||
        (m.d == best.d && (m.by_value < best.by_value || (m.by_value == best.by_value && m.nb < best.nb))))
      best = m;
  }
  return best;
}

// The bucket starts of a chosen map: the number of ends in lower buckets.
inline void fill_starts(const std::vector<uint32_t>& ends, RankBuckets& rb) {
  const uint32_t M = static_cast<uint32_t>(ends.size());
  rb.starts.assign(rb.nb, 0);
  uint32_t next = 0;  // first bucket whose start is not yet set
  for (uint32_t i = 0; i < M; ++i) {
    const uint32_t b = rb.by_value ? value_bucket(key_value(ends[i]), rb.vlo, rb.scale, rb.nb - 1)
                                   : std::min<uint32_t>((ends[i] - ends[0]) >> rb.shift, rb.nb - 1);
    while (next <= b) rb.starts[next++] = static_cast<uint16_t>(i);
  }
  while (next < rb.nb) rb.starts[next++] = static_cast<uint16_t>(M);
}

inline RankBuckets rank_buckets(const std::vector<uint32_t>& ends, int mode, uint32_t max_nb) {
  RankBuckets rb = pick_buckets(bucket_candidates(ends, mode, max_nb), max_nb);
  fill_starts(ends, rb);
  return rb;
}

inline uint64_t align4(uint64_t x) { return (x + 3) & ~uint64_t{3}; }

// Words one column's tables take in a group's LDS image (see append_slot_tables).
inline uint64_t slot_table_words(uint32_t M, const RankBuckets& rb, uint32_t sw) {
  return rb.nb + align4(uint64_t{M} + 1) + align4(uint64_t{M + 1} * sw);
}

// Upper bound of slot_table_words over every set of at most max_ends distinct ends and
// every bucket map of at most nb buckets.
inline uint64_t slot_table_words_bound(uint32_t max_ends, uint32_t nb, uint32_t sw) {
  return nb + align4(uint64_t{max_ends} + 1) + align4(uint64_t{max_ends + 1} * sw);
}

// One query's interval on a column as order-preserving keys; has = false: the query
// does not restrict the column and passes at every rank.
struct KeyInterval {
  uint32_t klo = 0, khi = 0;
  bool has = false;
};

// The rank variant's keys: order-preserving keys of the raw bits, -0 (0x7FFFFFFF) one
// below +0 (0x80000000), so the kernel needs no zero test.  An interval [lo, hi] takes
// the key of -0 for a lower end at zero and the key of +0 for an upper end at zero, so
// both zeros fall inside exactly when zero does (-0 == +0).
inline uint32_t rank_key(float x) {
  uint32_t b;
  std::memcpy(&b, &x, sizeof b);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
inline KeyInterval rank_interval(float lo, float hi) {
  KeyInterval k;
  k.klo = lo == 0.0f ? 0x7FFFFFFFu : rank_key(lo);
  k.khi = hi == 0.0f ? 0x80000000u : rank_key(hi);
  k.has = true;
  return k;
}

// Append one column's tables to a group's words g (whose size is 4-word aligned on
// entry and stays so): per bucket one word holding the index of its first end (the
// number of ends in lower buckets) in the low 16 bits and the index past its last end
// in the high 16 bits, the M sorted distinct ends and one word 0xFFFFFFFF after them
// (4-word aligned), then the (M + 1) x sw table of query bitsets by rank.  A search
// within a bucket reads only the bucket's own ends; a probe it does not need reads the
// word after the ends instead, the same word for every lane.  Query q of qs passes at rank r
// (r ends <= the row's key) iff idx(klo) < r <= idx(khi + 1); its bit is toggled on at
// idx(klo) + 1 and off at idx(khi + 1) + 1, and a running XOR over the ranks fills the
// rows.  Returns the offset of the ends in g (the column header's first word).
inline uint32_t append_slot_tables(std::vector<uint32_t>& g, const std::vector<uint32_t>& ends,
                                   const RankBuckets& rb, const std::vector<KeyInterval>& qs,
                                   uint32_t sw) {
  const uint32_t M = static_cast<uint32_t>(ends.size());
  const size_t s0 = g.size();
  g.resize(s0 + rb.nb, 0u);
  for (uint32_t b = 0; b < rb.nb; ++b) {
    const uint32_t end = b + 1 < rb.nb ? rb.starts[b + 1] : M;
    g[s0 + b] = static_cast<uint32_t>(rb.starts[b]) | (end << 16);
  }
  const uint32_t at = static_cast<uint32_t>(g.size());
  g.insert(g.end(), ends.begin(), ends.end());
  g.push_back(0xFFFFFFFFu);
  g.resize(align4(g.size()), 0u);
  const size_t t0 = g.size();
  g.resize(t0 + static_cast<size_t>(M + 1) * sw, 0u);
  std::vector<uint32_t> toggle(static_cast<size_t>(M + 2) * sw, 0u), always(sw, 0u);
  for (size_t q = 0; q < qs.size(); ++q) {
    const uint32_t w = static_cast<uint32_t>(q / 32), m = 1u << (q % 32);
    if (!qs[q].has) {
      always[w] |= m;
      continue;
    }
    const uint32_t r_lo = static_cast<uint32_t>(std::lower_bound(ends.begin(), ends.end(), qs[q].klo) - ends.begin());
    const uint32_t r_hi = static_cast<uint32_t>(std::lower_bound(ends.begin(), ends.end(), qs[q].khi + 1) - ends.begin());
    if (r_lo >= r_hi) continue;  // an empty interval passes nowhere
    toggle[static_cast<size_t>(r_lo + 1) * sw + w] ^= m;
    toggle[static_cast<size_t>(r_hi + 1) * sw + w] ^= m;
  }
  for (uint32_t w = 0; w < sw; ++w) {
    uint32_t cur = 0;
    for (uint32_t r = 0; r <= M; ++r) {
      cur ^= toggle[static_cast<size_t>(r) * sw + w];
      g[t0 + static_cast<size_t>(r) * sw + w] = cur | always[w];
    }
  }
  g.resize(align4(g.size()), 0u);
  return at;
}

}  // namespace mdrq
