// Host-side helpers shared by the library's translation units: device buffers,
// error handling, bin tables and pair-bin volumes.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pgx.h"
#include "pgx_weight.hpp"

namespace pgx {

struct Error : std::runtime_error {
  pgx_status code;
  Error(pgx_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PGX_HIP(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::pgx::Error(e_ == hipErrorOutOfMemory ? PGX_ENOSPACE : PGX_EHIP,                \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

#define PGX_REQUIRE(cond, code, msg) \
  do {                               \
    if (!(cond)) throw ::pgx::Error(code, msg); \
  } while (0)

inline void launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(PGX_EHIP, std::string("launch ") + what + ": " + hipGetErrorString(e));
}

// ----------------------------------------------------------------------------
// Device memory placement.  A plan's buffers are hipMalloc allocations it owns,
// unless a Heap is current on the calling thread: then they are carved from
// the Heap's region of device memory (a workspace the caller owns, or the
// library's fixed scratch array), first fit, 256-byte aligned, and the plan
// calls neither hipMalloc nor hipFree.
// ----------------------------------------------------------------------------
struct Heap {
  static constexpr size_t kAlign = 256;
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length of each free run (coalesced)
  size_t in_use = 0, peak = 0;
  void reset(void* b, size_t n) {
    base = static_cast<char*>(b);
    size = n & ~(kAlign - 1);
    free_.clear();
    if (size) free_[0] = size;
    in_use = peak = 0;
  }
  static size_t round(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  void* try_alloc(size_t n) {
    n = round(n == 0 ? 1 : n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      in_use += n;
      peak = std::max(peak, in_use);
      return base + off;
    }
    return nullptr;
  }
  void* alloc(size_t n, const char* what) {
    void* q = try_alloc(n);
    if (!q)
      throw Error(PGX_ENOSPACE, std::string(what) + ": " + std::to_string(round(n)) +
                                    " bytes do not fit (largest free run " +
                                    std::to_string(largest_free()) + " of " + std::to_string(size) + ")");
    return q;
  }
  void release(void* q, size_t n) {
    if (!q) return;
    n = round(n == 0 ? 1 : n);
    size_t off = (size_t)(static_cast<char*>(q) - base);
    in_use -= n;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + n == nx->first) {  // merge with the run after
      n += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {  // merge with the run before
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += n;
        return;
      }
    }
    free_[off] = n;
  }
};

// A fixed-scratch session: every buffer a call touches is carved afresh from
// the session's Heap (whatever the buffer held before is set aside, not
// freed) and put back as it was when the session ends, so that the call
// allocates nothing and leaves the plan's own buffers unchanged.
struct DBuf;
struct Session {
  Heap heap;
  uint64_t id = 0;
  struct Saved {
    DBuf* d;
    void* p;
    size_t bytes;
    Heap* owner;
  };
  std::vector<Saved> saved;
  inline void restore();
};

inline thread_local Heap* t_heap = nullptr;        // workspace of the plan being called
inline thread_local Session* t_session = nullptr;  // fixed-scratch session of the call

// Free device memory available to the plan's buffers: the largest free run of
// the current Heap, or the device's free memory.
inline size_t free_device_bytes() {
  if (t_session) return t_session->heap.largest_free();
  if (t_heap) return t_heap->largest_free();
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return fr;
}
// Memory left to other users of the device when an optional store is
// allocated: 4 GiB from the HIP allocator, none inside a caller's workspace.
inline size_t spare_device_bytes() { return (t_heap || t_session) ? 0 : ((size_t)4 << 30); }

// Fault injection for tests of the error paths: while the environment
// variable PGX_DEBUG_FAIL_ALLOC holds n >= 1, the n-th device allocation from
// the HIP allocator (counted from the moment the variable took that value)
// fails as if the device were out of memory: a required buffer raises
// PGX_EHIP, an optional store is skipped.  Unset, it costs one getenv per
// allocation.
inline bool injected_alloc_failure() {
  static std::mutex m;
  static std::string last;
  static long long count = 0;
  const char* e = std::getenv("PGX_DEBUG_FAIL_ALLOC");
  std::lock_guard<std::mutex> g(m);
  const std::string cur = e ? e : "";
  if (cur != last) {
    last = cur;
    count = 0;
  }
  if (cur.empty()) return false;
  const long long n = std::atoll(cur.c_str());
  return n > 0 && ++count == n;
}

// Device allocation that only grows (see Heap for where it lives).
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Heap* owner = nullptr;  // the Heap the memory came from; null: hipMalloc
  uint64_t session = 0;   // id of the fixed-scratch session that carved it
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) {
      if (owner) owner->release(p, bytes);
      else (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
    owner = nullptr;
    session = 0;
  }
  void* ensure(size_t n) {
    if (n == 0) n = 1;
    if (t_session) {
      if (session == t_session->id && n <= bytes) return p;
      if (session != t_session->id) {
        t_session->saved.push_back(Session::Saved{this, p, bytes, owner});
      } else {
        t_session->heap.release(p, bytes);
      }
      p = t_session->heap.alloc(n, "fixed scratch");
      bytes = n;
      owner = &t_session->heap;
      session = t_session->id;
      return p;
    }
    if (n > bytes) {
      release();
      if (t_heap) {
        p = t_heap->alloc(n, "workspace");
        owner = t_heap;
      } else {
        if (injected_alloc_failure())
          throw Error(PGX_EHIP, "hipMalloc of " + std::to_string(n) +
                                    " bytes: injected failure (PGX_DEBUG_FAIL_ALLOC)");
        PGX_HIP(hipMalloc(&p, n));
      }
      bytes = n;
    }
    return p;
  }
  // Optional store: allocate n bytes only when they fit with the spare
  // memory left over (spare_device_bytes); false, with nothing allocated,
  // otherwise.
  bool try_ensure(size_t n) {
    if (n <= bytes && p) return true;
    if (t_session) return false;
    if (free_device_bytes() + bytes < n + spare_device_bytes()) return false;
    release();
    if (t_heap) {
      p = t_heap->try_alloc(n);
      if (!p) return false;
      owner = t_heap;
    } else if (injected_alloc_failure() || hipMalloc(&p, n) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return false;
    }
    bytes = n;
    return true;
  }
  template <typename V> V* as() const { return static_cast<V*>(p); }
  template <typename V> V* get(size_t count) { return static_cast<V*>(ensure(count * sizeof(V))); }
};

inline void Session::restore() {
  for (auto it = saved.rbegin(); it != saved.rend(); ++it) {
    it->d->p = it->p;
    it->d->bytes = it->bytes;
    it->d->owner = it->owner;
    it->d->session = 0;
  }
  saved.clear();
}

inline int grid_for(int64_t n, int threads = 256) {
  int64_t g = (n + threads - 1) / threads;
  return (int)(g < 1 ? 1 : g);
}

// ----------------------------------------------------------------------------
// Output-bin tables (host).  q = e / Delta, threshold t = q*q (FP64);
// an integer square sum m is in bin k iff t_k <= m < t_{k+1}.
// ----------------------------------------------------------------------------
inline std::vector<int16_t> bin_lut(const std::vector<double>& edges, double delta, int64_t n_entries) {
  std::vector<double> t(edges.size());
  for (size_t i = 0; i < edges.size(); ++i) {
    const double q = edges[i] / delta;
    t[i] = q * q;
  }
  std::vector<int16_t> lut((size_t)n_entries, -1);
  const int nb = (int)edges.size() - 1;
  for (int64_t m = 0; m < n_entries; ++m) {
    const double md = (double)m;
    if (md < t[0] || md >= t[nb]) continue;
    int b = 0;
    for (int e = 1; e < nb; ++e) b += (md >= t[e]) ? 1 : 0;
    lut[(size_t)m] = (int16_t)b;
  }
  return lut;
}

// classification on the host with the same semantics as the device routine
struct HostBins {
  int mode, n2;
  std::vector<int16_t> lut1, lut2;
  std::vector<double> mu2;
  // GSW: gsw_value parameters and the cuts r_perp >= r_cut, |r| <= r_max as
  // squared lattice lengths (r / cell)^2
  double g[4] = {1.0, 0.0, 0.0, 0.0};
  double rcut2 = 0.0, rmax2 = 0.0;
  int classify(int i, int j, int k) const {
    const int xy = i * i + j * j, kk = k * k;
    if (mode == 3) return ((double)xy >= rcut2 && (double)(xy + kk) <= rmax2) ? 0 : -1;
    if (mode == 2) {
      if (xy >= (int)lut1.size() || kk >= (int)lut2.size()) return -1;
      const int b1 = lut1[xy], b2 = lut2[kk];
      if (b1 < 0 || b2 < 0) return -1;
      return b1 * n2 + b2;
    }
    const int m = xy + kk;
    if (m >= (int)lut1.size()) return -1;
    const int b1 = lut1[m];
    if (b1 < 0) return -1;
    if (mode == 0) return b1;
    const double md = (double)m, kd = (double)kk;
    if (kd < mu2[0] * md || kd > mu2[n2] * md) return -1;
    int kb = 0;
    for (int e = 1; e < n2; ++e) kb += (kd >= mu2[e] * md) ? 1 : 0;
    return b1 * n2 + kb;
  }
  // weight of a classified offset: 1 for the indicator bins
  double weight(int i, int j, int k) const {
    return mode == 3 ? gsw_value(i * i + j * j, k * k, g) : 1.0;
  }
};

// ----------------------------------------------------------------------------
// Pair-bin volumes
// ----------------------------------------------------------------------------
inline double vol_s_mu(double s0, double s1, double m0, double m1) {
  return 4.0 * M_PI / 3.0 * (s1 * s1 * s1 - s0 * s0 * s0) * (m1 - m0);
}

// int_{r0}^{r1} 2 pi r * |[c, d] cap [0, sqrt(D^2 - r^2)]| dr  (one sign of pi)
inline double slab_piece(double r0, double r1, double D, double c, double d) {
  if (r1 <= r0) return 0.0;
  auto h = [&](double r) { return std::sqrt(std::max(D * D - r * r, 0.0)); };
  // r where the sphere height equals d and c
  const double rd = d < D ? std::sqrt(D * D - d * d) : 0.0;
  const double rc = c < D ? std::sqrt(D * D - c * c) : 0.0;
  std::vector<double> pts = {r0, r1, std::min(std::max(rd, r0), r1), std::min(std::max(rc, r0), r1)};
  std::sort(pts.begin(), pts.end());
  double total = 0.0;
  for (size_t k = 0; k + 1 < pts.size(); ++k) {
    const double a = pts[k], b = pts[k + 1];
    if (b <= a) continue;
    const double mid = 0.5 * (a + b);
    const double top = std::min(d, h(mid));
    if (top <= c) continue;
    if (h(mid) >= d) {
      total += M_PI * (d - c) * (b * b - a * a);
    } else {
      auto F = [&](double r) {
        const double u = std::max(D * D - r * r, 0.0);
        return -(2.0 * M_PI / 3.0) * u * std::sqrt(u) - M_PI * c * r * r;
      };
      total += F(b) - F(a);
    }
  }
  return total;
}

inline double vol_rp_pi(double r0, double r1, double p0, double p1, double D) {
  return 2.0 * slab_piece(r0, std::min(r1, D), D, p0, p1);
}

}  // namespace pgx
