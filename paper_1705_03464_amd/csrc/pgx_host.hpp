// Host-side helpers shared by the library's translation units: device buffers,
// error handling, bin tables and pair-bin volumes.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
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

// Owned device allocation that only grows.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void* ensure(size_t n) {
    if (n == 0) n = 1;
    if (n > bytes) {
      release();
      PGX_HIP(hipMalloc(&p, n));
      bytes = n;
    }
    return p;
  }
  template <typename V> V* as() const { return static_cast<V*>(p); }
  template <typename V> V* get(size_t count) { return static_cast<V*>(ensure(count * sizeof(V))); }
};

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
