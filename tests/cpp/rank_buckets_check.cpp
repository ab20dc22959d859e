// Brute-force check of the rank variant's bucket maps (host side).  For random sorted
// sets of distinct interval ends -- uniform, log-spread of both signs, arbitrary bit
// patterns, a grid, with key(-inf) and key(+inf) + 1 mixed in -- and every mode and
// bucket cap: bucket numbers never decrease along the sorted ends (the map is
// monotone), the starts equal the number of ends in lower buckets, 2^d - 1 holds the
// fullest bucket and 2^(d-1) - 1 does not, the bucket count respects the cap, the
// key-only mode never picks the value map, and the choice equals an exhaustive search.  The kernel's value map repeats the host's
// float arithmetic, so a key between two ends lands in a bucket between theirs.
// The slot tables appended for the kernel are checked too: their size against the
// bound the host plans LDS with, the padding, and every query bitset row.
#include <cstdio>
#include <random>

#include "rank_buckets.h"

namespace {

uint32_t order_key(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  if (b == 0x80000000u) b = 0;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

}  // namespace

int main() {
  std::mt19937 rng(1);
  int bad = 0, value_maps = 0, key_maps = 0;
  for (int it = 0; it < 20000; ++it) {
    const int n = 1 + static_cast<int>(rng() % 300);
    std::vector<uint32_t> ends;
    const int kind = it % 4;
    for (int i = 0; i < n; ++i) {
      float v;
      if (kind == 0) {
        v = std::uniform_real_distribution<float>(0.0f, 1.0f)(rng);
      } else if (kind == 1) {
        v = std::exp(std::uniform_real_distribution<float>(-20.0f, 5.0f)(rng)) * ((rng() & 1) ? 1.0f : -1.0f);
      } else if (kind == 2) {
        const uint32_t b = static_cast<uint32_t>(rng());
        std::memcpy(&v, &b, 4);
        if (std::isnan(v)) v = 1.0f;
      } else {
        v = static_cast<float>(rng() % 1000000) * 1e-6f;
      }
      const uint32_t k = order_key(v);
      ends.push_back((rng() & 1) ? k : k + 1);  // key(lo) or key(hi) + 1
    }
    if (it % 7 == 0) ends.push_back(order_key(-INFINITY));
    if (it % 11 == 0) ends.push_back(order_key(INFINITY) + 1);
    std::sort(ends.begin(), ends.end());
    ends.erase(std::unique(ends.begin(), ends.end()), ends.end());
    const uint32_t M = static_cast<uint32_t>(ends.size());
    for (int mode = 0; mode < 3; ++mode)
      for (uint32_t cap : {256u, 1024u}) {
        const mdrq::RankBuckets rb = mdrq::rank_buckets(ends, mode, cap);
        (rb.by_value ? value_maps : key_maps)++;
        std::vector<uint32_t> bk(M);
        for (uint32_t i = 0; i < M; ++i)
          bk[i] = rb.by_value ? mdrq::value_bucket(mdrq::key_value(ends[i]), rb.vlo, rb.scale, rb.nb - 1)
                              : std::min<uint32_t>((ends[i] - ends[0]) >> rb.shift, rb.nb - 1);
        for (uint32_t i = 1; i < M; ++i)
          if (bk[i] < bk[i - 1]) {
            ++bad;
            break;
          }
        std::vector<uint32_t> occ(rb.nb, 0);
        for (uint32_t b : bk) ++occ[b];
        uint32_t below = 0, fullest = 0;
        for (uint32_t b = 0; b < rb.nb; ++b) {
          if (rb.starts[b] != below) {
            ++bad;
            break;
          }
          below += occ[b];
          fullest = std::max(fullest, occ[b]);
        }
        if (fullest > (1u << rb.d) - 1 || (rb.d > 1 && fullest <= (1u << (rb.d - 1)) - 1)) ++bad;
        if (rb.nb > cap || rb.nb < 8 || (rb.nb & (rb.nb - 1))) ++bad;
        if (mode == 1 && rb.by_value) ++bad;
        // The choice equals an exhaustive search over both maps and all bucket counts
        // up to the cap (and about 4 per end): fewest steps, then key, then fewest.
        uint32_t lim = 8;
        while (lim < cap && lim < 4 * M) lim *= 2;
        uint32_t best_d = 99, best_v = 2, best_nb = 0;
        float vlo = INFINITY, vhi = -INFINITY;
        for (uint32_t e : ends) {
          const float v = mdrq::key_value(e);
          if (std::isfinite(v)) {
            vlo = std::min(vlo, v);
            vhi = std::max(vhi, v);
          }
        }
        const bool value_ok = vlo < vhi && std::isfinite(vhi - vlo) && vhi - vlo >= 0x1p-90f &&
                              (vlo == 0.0f || std::fabs(vlo) >= 0x1p-100f);
        for (uint32_t v = 0; v < 2; ++v) {
          if ((v == 0 && mode == 2 && value_ok) || (v == 1 && (mode == 1 || !value_ok))) continue;
          for (uint32_t nb = 8; nb <= lim; nb *= 2) {
            std::vector<uint32_t> o(nb, 0);
            uint32_t shift = 0;
            while (((ends.back() - ends[0]) >> shift) > nb - 1) ++shift;
            const float scale = static_cast<float>(nb) / (vhi - vlo);
            for (uint32_t e : ends)
              ++o[v ? mdrq::value_bucket(mdrq::key_value(e), vlo, scale, nb - 1)
                    : std::min<uint32_t>((e - ends[0]) >> shift, nb - 1)];
            const uint32_t f = *std::max_element(o.begin(), o.end());
            const uint32_t d = 32 - static_cast<uint32_t>(__builtin_clz(f));
            if (d < best_d || (d == best_d && (v < best_v || (v == best_v && nb < best_nb)))) {
              best_d = d;
              best_v = v;
              best_nb = nb;
            }
          }
        }
        if (rb.d != best_d || rb.by_value != (best_v == 1) || rb.nb != best_nb) ++bad;
      }
  }
  // Slot tables of S queries (32 x sw per group, any S up to 128): the appended words
  // equal slot_table_words and stay within slot_table_words_bound(2 S) for adversarial
  // end sets (all but one end crowded into one bucket), each bucket word holds the
  // first and one-past-last index of the bucket's ends, and every bitset row says
  // exactly which queries pass at that rank.
  int tables = 0;
  for (int it = 0; it < 4000; ++it) {
    const uint32_t S = 1 + static_cast<uint32_t>(rng() % 128);
    const uint32_t sw = S <= 32 ? 1 : S <= 64 ? 2 : 4;
    const int kind = it % 3;
    std::vector<mdrq::KeyInterval> qs(S);
    const uint32_t base = order_key(0.5f);
    for (uint32_t q = 0; q < S; ++q) {
      if (rng() % 5 == 0) continue;  // no predicate on this column
      uint32_t a, b;
      if (kind == 0) {        // crowded: consecutive keys, one far outlier below
        a = base + static_cast<uint32_t>(rng() % (2 * S + 2));
        b = base + static_cast<uint32_t>(rng() % (2 * S + 2));
      } else if (kind == 1) { // spread
        a = order_key(std::uniform_real_distribution<float>(0.0f, 1.0f)(rng));
        b = order_key(std::uniform_real_distribution<float>(0.0f, 1.0f)(rng));
      } else {                // arbitrary keys of non-NaN floats, key(-inf) .. key(+inf)
        a = 0x007FFFFFu + static_cast<uint32_t>(rng()) % (0xFF800000u - 0x007FFFFFu);
        b = 0x007FFFFFu + static_cast<uint32_t>(rng()) % (0xFF800000u - 0x007FFFFFu);
      }
      if (rng() % 4) {
        if (a > b) std::swap(a, b);
      }
      qs[q] = mdrq::KeyInterval{a, b, true};
    }
    if (kind == 0) qs[0] = mdrq::KeyInterval{order_key(-1e30f), order_key(-1e30f), true};
    std::vector<uint32_t> ends;
    for (const auto& k : qs)
      if (k.has) {
        ends.push_back(k.klo);
        ends.push_back(k.khi + 1);
      }
    if (ends.empty()) continue;
    std::sort(ends.begin(), ends.end());
    ends.erase(std::unique(ends.begin(), ends.end()), ends.end());
    const uint32_t M = static_cast<uint32_t>(ends.size());
    for (uint32_t cap : {256u, 1024u}) {
      mdrq::RankBuckets rb = mdrq::rank_buckets(ends, it % 3, cap);
      std::vector<uint32_t> g(8, 0u);
      const uint32_t at = mdrq::append_slot_tables(g, ends, rb, qs, sw);
      const uint64_t words = g.size() - 8;
      ++tables;
      if (words != mdrq::slot_table_words(M, rb, sw) || g.size() % 4 ||
          (cap == 256 && words > mdrq::slot_table_words_bound(2 * S, 256, sw)) || at != 8 + rb.nb) {
        std::printf("size S=%u M=%u d=%u nb=%u words=%llu\n", S, M, rb.d, rb.nb,
                    static_cast<unsigned long long>(words));
        ++bad;
        continue;
      }
      for (uint32_t i = 0; i < M; ++i)
        if (g[at + i] != ends[i]) ++bad;
      if (g[at + M] != 0xFFFFFFFFu) ++bad;
      // bucket words: [first, past-last) of the ends the map puts in that bucket, and
      // a search of d steps within it stays inside it
      for (uint32_t b = 0; b < rb.nb; ++b) {
        uint32_t first = M, past = 0, n_in = 0;
        for (uint32_t i = 0; i < M; ++i) {
          const uint32_t bi = rb.by_value ? mdrq::value_bucket(mdrq::key_value(ends[i]), rb.vlo, rb.scale, rb.nb - 1)
                                          : std::min<uint32_t>((ends[i] - ends[0]) >> rb.shift, rb.nb - 1);
          if (bi == b) {
            first = std::min(first, i);
            past = std::max(past, i + 1);
            ++n_in;
          }
        }
        uint32_t below = 0;
        for (uint32_t i = 0; i < M; ++i) {
          const uint32_t bi = rb.by_value ? mdrq::value_bucket(mdrq::key_value(ends[i]), rb.vlo, rb.scale, rb.nb - 1)
                                          : std::min<uint32_t>((ends[i] - ends[0]) >> rb.shift, rb.nb - 1);
          below += bi < b ? 1u : 0u;
        }
        const uint32_t w = g[8 + b];
        if ((w & 0xFFFFu) != below || (w >> 16) != below + n_in || (n_in && (first != below || past != below + n_in)) ||
            n_in > (1u << rb.d) - 1) {
          if (bad < 5)
            std::printf("bucket b=%u nb=%u words %u/%u below=%u n_in=%u d=%u M=%u\n", b, rb.nb, w & 0xFFFFu,
                        w >> 16, below, n_in, rb.d, M);
          ++bad;
        }
      }
      const size_t t0 = at + mdrq::align4(M + 1);
      for (uint32_t r = 0; r <= M; ++r)
        for (uint32_t q = 0; q < S; ++q) {
          // rank r: the ends[0..r) are <= the key; the query passes iff
          // klo <= key <= khi, i.e. klo is among them and khi + 1 is not.
          bool pass = true;
          if (qs[q].has) {
            const uint32_t lo_idx = static_cast<uint32_t>(std::find(ends.begin(), ends.end(), qs[q].klo) - ends.begin());
            const uint32_t hi_idx = static_cast<uint32_t>(std::find(ends.begin(), ends.end(), qs[q].khi + 1) - ends.begin());
            pass = lo_idx < r && r <= hi_idx;
          }
          const bool got = (g[t0 + static_cast<size_t>(r) * sw + q / 32] >> (q % 32)) & 1u;
          if (got != pass) ++bad;
        }
    }
  }
  // The rank variant's interval keys: for every interval [lo, hi] and value x of a set
  // with both zeros, infinities, subnormals and their neighbours, lo <= x <= hi exactly
  // when klo <= rank_key(x) < khi + 1.
  {
    std::vector<float> vals = {0.0f, -0.0f, INFINITY, -INFINITY, 1e-45f, -1e-45f, 1.17549435e-38f,
                               -1.17549435e-38f, 1.0f, -1.0f, 0.5f, -2.5f, 3.4e38f, -3.4e38f};
    const size_t base_n = vals.size();
    for (size_t i = 0; i < base_n; ++i) {
      vals.push_back(std::nextafter(vals[i], INFINITY));
      vals.push_back(std::nextafter(vals[i], -INFINITY));
    }
    int checked = 0;
    for (float lo : vals)
      for (float hi : vals) {
        if (!(lo <= hi)) continue;
        const mdrq::KeyInterval k = mdrq::rank_interval(lo, hi);
        for (float x : vals) {
          const bool want = lo <= x && x <= hi;
          const uint32_t kx = mdrq::rank_key(x);
          const bool got = k.klo <= kx && kx < k.khi + 1;
          if (want != got) {
            if (bad < 5) std::printf("rank key: lo=%g hi=%g x=%g\n", lo, hi, x);
            ++bad;
          }
          ++checked;
        }
      }
    std::printf("rank interval checks %d\n", checked);
  }
  std::printf("bad=%d key_maps=%d value_maps=%d slot_tables=%d\n", bad, key_maps, value_maps, tables);
  return bad != 0 || value_maps == 0 || key_maps == 0;
}
