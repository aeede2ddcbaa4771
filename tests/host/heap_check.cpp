// Host-side checks of the workspace allocator (pgx::Heap) and the host bin
// tables, built with AddressSanitizer and UndefinedBehaviorSanitizer on the
// host code.  Needs no device: the Heap only does bookkeeping over a region,
// here a host buffer.  Exits non-zero on the first failed check.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_1705_03464_amd/csrc/pgx_host.hpp"

#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                  \
    }                                                                \
  } while (0)

int main() {
  // 1. random alloc / release sequences against a byte-level model: no two
  //    live blocks overlap, every block is 256-byte aligned within the
  //    region, in_use and the free runs account for every byte, and releasing
  //    everything coalesces the region back into one run
  const size_t region = (size_t)1 << 22;
  std::vector<char> buf(region + pgx::Heap::kAlign);
  char* base = buf.data() + (pgx::Heap::kAlign - (reinterpret_cast<uintptr_t>(buf.data()) % pgx::Heap::kAlign)) %
                                pgx::Heap::kAlign;
  std::mt19937_64 rng(12345);
  for (int trial = 0; trial < 50; ++trial) {
    pgx::Heap h;
    h.reset(base, region);
    std::vector<unsigned char> owner(region, 0);
    struct Blk { char* p; size_t n; unsigned char tag; };
    std::vector<Blk> live;
    for (int step = 0; step < 400; ++step) {
      const bool do_alloc = live.empty() || (rng() % 3 != 0);
      if (do_alloc) {
        const size_t n = 1 + rng() % (region / 16);
        void* q = h.try_alloc(n);
        if (!q) {
          CHECK(h.largest_free() < pgx::Heap::round(n));
          bool threw = false;
          try {
            h.alloc(n, "test");
          } catch (const pgx::Error& e) {
            threw = e.code == PGX_ENOSPACE;
          }
          CHECK(threw);
          continue;
        }
        char* p = static_cast<char*>(q);
        CHECK(p >= base && p + n <= base + region);
        CHECK((size_t)(p - base) % pgx::Heap::kAlign == 0);
        const unsigned char tag = (unsigned char)(1 + step % 250);
        for (size_t i = 0; i < pgx::Heap::round(n); ++i) {
          CHECK(owner[(size_t)(p - base) + i] == 0);
          owner[(size_t)(p - base) + i] = tag;
        }
        live.push_back({p, n, tag});
      } else {
        const size_t k = rng() % live.size();
        const Blk b = live[k];
        for (size_t i = 0; i < pgx::Heap::round(b.n); ++i) {
          CHECK(owner[(size_t)(b.p - base) + i] == b.tag);
          owner[(size_t)(b.p - base) + i] = 0;
        }
        h.release(b.p, b.n);
        live.erase(live.begin() + (long)k);
      }
      size_t used = 0, freeb = 0;
      for (const Blk& b : live) used += pgx::Heap::round(b.n);
      for (const auto& f : h.free_) freeb += f.second;
      CHECK(h.in_use == used);
      CHECK(used + freeb == h.size);
      // free runs are disjoint, sorted and never adjacent (coalesced)
      size_t end = 0;
      bool first = true;
      for (const auto& f : h.free_) {
        CHECK(first || f.first > end);
        end = f.first + f.second;
        first = false;
      }
    }
    for (const Blk& b : live) h.release(b.p, b.n);
    CHECK(h.in_use == 0 && h.free_.size() == 1 && h.free_.begin()->second == h.size);
  }
  // 2. the bin look-up tables and pair-bin volumes on random edge sets
  for (int trial = 0; trial < 200; ++trial) {
    const int nb = 1 + (int)(rng() % 20);
    std::vector<double> e(nb + 1);
    double x = 0.1 + (double)(rng() % 1000) * 1e-3;
    for (int i = 0; i <= nb; ++i) {
      e[i] = x;
      x += 0.05 + (double)(rng() % 1000) * 1e-2;
    }
    const double delta = 0.5 + (double)(rng() % 100) * 0.05;
    const int64_t entries = 1 + (int64_t)(e[nb] * e[nb] / (delta * delta)) + (int64_t)(rng() % 50);
    const std::vector<int16_t> lut = pgx::bin_lut(e, delta, entries);
    CHECK((int64_t)lut.size() == entries);
    for (int64_t q = 0; q < entries; ++q) {
      const int b = lut[q];
      CHECK(b >= -1 && b < nb);
      // entry q is the squared lattice length in units of delta^2, decided
      // on squares of edge / delta (the table's convention)
      const double lo = (e[0] / delta) * (e[0] / delta), hi = (e[nb] / delta) * (e[nb] / delta);
      if (b >= 0) {
        const double t0 = (e[b] / delta) * (e[b] / delta), t1 = (e[b + 1] / delta) * (e[b + 1] / delta);
        CHECK((double)q >= t0 && (b == nb - 1 ? (double)q < hi : (double)q < t1));
      } else {
        CHECK((double)q < lo || (double)q >= hi);
      }
    }
    const double s0 = e[0], s1 = e[nb];
    CHECK(pgx::vol_s_mu(s0, s1, 0.0, 1.0) > 0.0);
    const double D = s1 * 1.5;
    CHECK(pgx::vol_rp_pi(0.0, s1, 0.0, D, D) > 0.0);
  }
  std::printf("host checks passed\n");
  return 0;
}
