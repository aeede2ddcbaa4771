// Smaller kernels: weights, deterministic FP64 reductions, the finalisation
// formulas, and the pieces of the plain one-field-at-a-time path.
#pragma once
#include "pgx_kernels.hpp"

namespace pgx {

constexpr double kPi = 3.14159265358979323846;

// ----------------------------------------------------------------------------
// small utilities
// ----------------------------------------------------------------------------
template <typename V>
static __global__ void k_fill_value(V* __restrict__ p, int64_t n, V v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// fs[f] = first index of the sorted keys with key >= f nn, for f in [0, F]
// (binary search; the field boundaries of a field-major catalogue)
static __global__ void k_field_starts(const int32_t* __restrict__ key, int64_t n, int64_t nn, int F,
                                      int32_t* __restrict__ fs) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f > F) return;
  const int64_t t = (int64_t)f * nn;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)key[mid] < t)
      lo = mid + 1;
    else
      hi = mid;
  }
  fs[f] = (int32_t)lo;
}

static __global__ void k_field_counts(const int32_t* __restrict__ line_start, int64_t nn, int F,
                               int64_t* __restrict__ counts) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < F) counts[f] = (int64_t)line_start[(int64_t)(f + 1) * nn] - line_start[(int64_t)f * nn];
}

static __global__ void k_export_pairs(const int32_t* __restrict__ key, const int32_t* __restrict__ pi,
                               const int32_t* __restrict__ pj, int64_t n, int64_t nn,
                               int32_t* __restrict__ f, int32_t* __restrict__ i, int32_t* __restrict__ j) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (f) f[p] = (int32_t)(key[p] / nn);
  if (i) i[p] = pi[p];
  if (j) j[p] = pj[p];
}

// weights must be finite and >= 0
static __global__ void k_validate_w(const float* __restrict__ w, int64_t n, int* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = w[i];
  if (!isfinite(v) || v < 0.0f) atomicOr(err, 4);
}

// ----------------------------------------------------------------------------
// weights
// ----------------------------------------------------------------------------
// pair weight w_i * w_j (exact in FP64 for FP32 weights), rounded to T
template <typename T>
static __global__ void k_gather_weights(const int32_t* __restrict__ idx, const float* __restrict__ w,
                                 int64_t n, T* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  out[p] = w ? (T)w[idx[p]] : (T)1;
}

// Deterministic block sum of a double per thread (fixed tree over 256 lanes).
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Segmented sums over the fields' contiguous ranges of the sorted pair list
// are split into K equal chunks per segment (K fixed by the plan's sizes, so
// the partition, hence the rounding, does not depend on the data): block
// (segment, chunk k) sums chunk k, and k_sum_chunks adds the K partial sums
// of each segment in order.  Enough blocks for the whole GPU even when a few
// fields hold hundreds of millions of pairs.
__host__ __device__ inline int reduce_chunks(int64_t segments) {
  const int64_t k = (4096 + segments - 1) / (segments > 0 ? segments : 1);
  return (int)(k < 1 ? 1 : (k > 256 ? 256 : k));
}
// bounds [cs, ce) of chunk k of K of the range [s, e)
__device__ __forceinline__ void chunk_of(int64_t s, int64_t e, int k, int K, int64_t& cs, int64_t& ce) {
  cs = s + (e - s) * k / K;
  ce = s + (e - s) * (k + 1) / K;
}
// out[i] = sum_{k < K} part[i K + k], in order
static __global__ void k_sum_chunks(const double* __restrict__ part, int64_t n, int K,
                                    double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  for (int k = 0; k < K; ++k) a += part[i * K + k];
  out[i] = a;
}

// Pair weights w_i w_j (FP64 products, unit without weights; also rounded
// to T into wt when it is given) and their partial sums over each field's
// range: block (f, k) of a grid (F, K) takes chunk k of field f.  fs: the
// field starts of the field-major pair catalogue.
template <typename T>
static __global__ void k_pair_wts(const int32_t* __restrict__ fs, const int32_t* __restrict__ pi,
                                  const int32_t* __restrict__ pj, const float* __restrict__ w,
                                  T* __restrict__ wt, double* __restrict__ wd, double* __restrict__ part) {
  __shared__ double sh[256];
  const int f = blockIdx.x, k = blockIdx.y, K = gridDim.y;
  int64_t cs, ce;
  chunk_of(fs[f], fs[f + 1], k, K, cs, ce);
  double acc = 0.0;
  for (int64_t p = cs + threadIdx.x; p < ce; p += 256) {
    const double d = w ? (double)w[pi[p]] * (double)w[pj[p]] : 1.0;
    wd[p] = d;
    if (wt) wt[p] = (T)d;
    acc += d;
  }
  const double r = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[(int64_t)f * K + k] = r;
}

// Largest disagreement between two sets of bin sums of the same estimator,
// in units of tol * max(|xi|, 1e-2) with xi = S / (n_b Wsum_f W_g) (fields
// with Wsum_f = 0 skipped).  One block; out[0] = the largest ratio.
static __global__ void k_xi_disagreement(const double* __restrict__ Sa, const double* __restrict__ Sb,
                                         const double* __restrict__ nb, const double* __restrict__ wsum,
                                         const double* __restrict__ wg, int F, int R, double tol,
                                         double* __restrict__ out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < F * R; i += 256) {
    const int f = i / R, b = i - f * R;
    const double norm = nb[b] * wsum[f] * wg[0];
    if (!(wsum[f] > 0.0) || !(norm > 0.0)) continue;
    const double xa = Sa[i] / norm, xb = Sb[i] / norm;
    const double r = fabs(xa - xb) / (tol * fmax(fabs(xa), 1e-2));
    m = r > m || r != r ? r : m;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double o = sh[threadIdx.x + s];
      if (o > sh[threadIdx.x] || o != o) sh[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Per-field scale of the pair fields in the transforms: 1 / Wsum_f rounded to
// FP32 (1 for empty fields), so that the two fields sharing a complex grid
// have unit mass each and neither one's rounding swamps the other's signal.
static __global__ void k_field_scale(const double* __restrict__ wsum, int F, float* __restrict__ fsc) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < F) fsc[f] = (float)(wsum[f] > 1e-30 ? 1.0 / wsum[f] : 1.0);
}

// Sum of galaxy weights in FP64, deterministic: kWtBlocks blocks each sum a
// fixed contiguous chunk (256 threads, fixed partition), then one block sums
// the partials in order.
constexpr int kWtBlocks = 256;
static __global__ void k_weight_partial(const float* __restrict__ w, int64_t n, double* __restrict__ part) {
  __shared__ double sh[256];
  const int64_t chunk = (n + kWtBlocks - 1) / kWtBlocks;
  const int64_t a = (int64_t)blockIdx.x * chunk, b = a + chunk < n ? a + chunk : n;
  double acc = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += 256) acc += w ? (double)w[i] : 1.0;
  const double r = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}
static __global__ void k_weight_total(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < kWtBlocks; i += 256) acc += part[i];
  const double r = block_sum256(acc, sh);
  if (threadIdx.x == 0) out[0] = r;
}
// ----------------------------------------------------------------------------
// bin partial reduction: part[slot][nblk][2][R] -> S[f][R] for the two fields
// of each slot (fixed order over blocks, deterministic)
// ----------------------------------------------------------------------------
static __global__ void k_reduce_bins(const double* __restrict__ part, int nblk, int R,
                              const int32_t* __restrict__ slot_fa, const int32_t* __restrict__ slot_fb,
                              double* __restrict__ S, const float* __restrict__ fscale = nullptr) {
  // one block per (entry i of the 2R partial row, slot); fixed partition and tree
  __shared__ double sh[256];
  const int slot = blockIdx.y, i = blockIdx.x;
  const double* p = part + (int64_t)slot * nblk * 2 * R + i;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) acc += p[(int64_t)b * 2 * R];
  const double r = block_sum256(acc, sh);
  if (threadIdx.x == 0) {
    const int half = i / R, bin = i % R;
    const int f = half == 0 ? slot_fa[slot] : slot_fb[slot];
    // undo the field's transform scale (the FP32 value the scatter applied)
    if (f >= 0) S[(int64_t)f * R + bin] = fscale ? r / (double)fscale[f] : r;
  }
}

// ----------------------------------------------------------------------------
// finalisation (FP64)
//   xi_gg[b] = Sgg[b] / (n_b Wg^2)
//   xi_pg[f,b] = S[f,b] / (n_b Wsum_f Wg)
//   xi_dp[f] = 2 Wsum_f L^3 / (Wg^2 V_f) - 1
//   b = xi_pg / xi_gg ; Q from the not-strictly-squeezed estimator (default),
//   the squeezed-limit estimator, or a constant xi_w.
// ----------------------------------------------------------------------------
struct FinalizeArgs {
  int F, R, qmode;
  double L, xi_w_const;
  const double* S;
  const double* Sgg;
  const double* nb;      // n_b as double
  const double* vol;     // V_f
  const double* wsum;
  const double* wg;      // [1]
  double* xi_gg;
  double* xi_pg;
  double* xi_dp;
  double* b_pg;
  double* q_eff;
};

__device__ __forceinline__ double q_estimator(double b, double x, double xw, int mode) {
  if (mode == 1) return ((1.0 + x) * b - 2.0) / (2.0 * x);
  return ((1.0 + x) * b - 2.0 - xw / (2.0 * x)) / (2.0 * x + 1.5 * xw);
}

static __global__ void k_finalize(FinalizeArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double wg = a.wg[0];
  if (i < a.R) a.xi_gg[i] = a.Sgg[i] / (a.nb[i] * wg * wg);
  if (i < a.F) a.xi_dp[i] = 2.0 * a.wsum[i] * a.L * a.L * a.L / (wg * wg * a.vol[i]) - 1.0;
  if (i >= a.F * a.R) return;
  const int f = i / a.R, b = i % a.R;
  const double xgg = a.Sgg[b] / (a.nb[b] * wg * wg);
  // an empty field (no pairs, or zero pair weight) has no correlation: NaN,
  // also where its grid partner's rounding left a nonzero sum
  const double xpg = a.wsum[f] > 0.0 ? a.S[i] / (a.nb[b] * a.wsum[f] * wg) : __builtin_nan("");
  const double x = 2.0 * a.wsum[f] * a.L * a.L * a.L / (wg * wg * a.vol[f]) - 1.0;
  const double bb = xpg / xgg;
  const double xw = a.qmode == 2 ? a.xi_w_const : xgg;
  a.xi_pg[i] = xpg;
  a.b_pg[i] = bb;
  a.q_eff[i] = q_estimator(bb, x, xw, a.qmode);
}

// ----------------------------------------------------------------------------
// Projected 2PCF (2PCF section, equation 2PCF_los_integrated_explicit): for
// pairs binned by (r_p, |pi|), the line-of-sight integral of the pair
// correlation over the pair sphere, averaged over each r_p annulus:
//   w_p[a] = sum_b xi(d_p)[a, b] V[a, b] / A_a,   A_a = pi (rp_{a+1}^2 - rp_a^2),
// with V the exact annulus-slab volume cut by the sphere (pieces of zero
// volume, whose xi(d_p) is 0/0, contribute nothing).  rp2 holds the squared
// r_p edges.  Its adjoint: g_xi(d_p)[a, b] = g_w[a] V[a, b] / A_a.
// ----------------------------------------------------------------------------
static __global__ void k_projected(const double* __restrict__ xi_dp, const double* __restrict__ vol,
                                   const double* __restrict__ rp2, int n1, int n2,
                                   double* __restrict__ wp) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n1) return;
  const double area = 3.14159265358979323846 * (rp2[a + 1] - rp2[a]);
  double acc = 0.0;
  for (int b = 0; b < n2; ++b) {
    const double v = vol[a * n2 + b];
    if (v > 0.0) acc += xi_dp[a * n2 + b] * v;
  }
  wp[a] = acc / area;
}
static __global__ void k_projected_adjoint(const double* __restrict__ g_wp, const double* __restrict__ vol,
                                           const double* __restrict__ rp2, int n1, int n2,
                                           double* __restrict__ g_xidp) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n1 * n2) return;
  const int a = f / n2;
  const double area = 3.14159265358979323846 * (rp2[a + 1] - rp2[a]);
  const double v = vol[f];
  g_xidp[f] = v > 0.0 ? g_wp[a] * v / area : 0.0;
}

// ----------------------------------------------------------------------------
// plain path
// ----------------------------------------------------------------------------
template <typename T>
static __global__ void k_fill_zero(C<T>* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = C<T>{0, 0};
}

// CIC scatter of the points in [s, e) with global atomics into the real part
template <typename T>
static __global__ void k_scatter_atomic(const int32_t* __restrict__ line_start, int64_t k0, int64_t k1,
                                 const int32_t* __restrict__ key, PointSet<T> ps, int N,
                                 C<T>* __restrict__ grid) {
  const int64_t s = line_start[k0], e = line_start[k1];
  const int64_t NN = (int64_t)N * N;
  for (int64_t p = s + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < e;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = (int64_t)key[p] % NN;
    const int y0 = (int)(l % N), z0 = (int)(l / N), x0 = ps.x0[p];
    const T fx = ps.fx[p], fy = ps.fy[p], fz = ps.fz[p], w = ps.wt[p];
    for (int c = 0; c < 8; ++c) {
      const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
      const T wx = ox ? fx : (T)1 - fx, wy = oy ? fy : (T)1 - fy, wz = oz ? fz : (T)1 - fz;
      const int64_t idx = ((int64_t)((z0 + oz) & (N - 1)) * N + ((y0 + oy) & (N - 1))) * N +
                          ((x0 + ox) & (N - 1));
      atomicAdd(&grid[idx].x, w * wx * wy * wz);
    }
  }
}

// Plain path, TSC: each point adds to the 27 nodes of its TSC footprint
// (tsc_axis on each axis) with global atomics.
template <typename T>
static __global__ void k_scatter_atomic_tsc(const int32_t* __restrict__ line_start, int64_t k0, int64_t k1,
                                            const int32_t* __restrict__ key, PointSet<T> ps, int N,
                                            C<T>* __restrict__ grid) {
  const int64_t s = line_start[k0], e = line_start[k1];
  const int64_t NN = (int64_t)N * N;
  for (int64_t p = s + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < e;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = (int64_t)key[p] % NN;
    int lx, ly, lz;
    T wx[3], wy[3], wz[3];
    tsc_axis<T>(ps.x0[p], ps.fx[p], lx, wx);
    tsc_axis<T>((int)(l % N), ps.fy[p], ly, wy);
    tsc_axis<T>((int)(l / N), ps.fz[p], lz, wz);
    const T w = ps.wt[p];
    for (int c = 0; c < 27; ++c) {
      const int ox = c % 3, oy = (c / 3) % 3, oz = c / 9;
      const int64_t idx = ((int64_t)((lz + oz) & (N - 1)) * N + ((ly + oy) & (N - 1))) * N +
                          ((lx + ox) & (N - 1));
      atomicAdd(&grid[idx].x, w * wx[ox] * wy[oy] * wz[oz]);
    }
  }
}

// a[i] *= conj(b[i]); with SELF, a[i] = |a[i]|^2 after zeroing a[0] (the k = 0 mode)
template <typename T, bool SELF>
static __global__ void k_mul_conj(C<T>* __restrict__ a, const C<T>* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if constexpr (SELF) {
      const C<T> v = a[i];
      a[i] = C<T>{v.x * v.x + v.y * v.y, (T)0};
    } else {
      a[i] = cmulc(a[i], b[i]);
    }
  }
}

template <typename T>
static __global__ void k_zero_dc(C<T>* a) {
  if (threadIdx.x == 0 && blockIdx.x == 0) a[0] = C<T>{0, 0};
}

// copy a full grid into another buffer
template <typename T>
static __global__ void k_copy(const C<T>* __restrict__ a, C<T>* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// bin sums over the window cube of a full grid (real part); partials per block
template <typename T, int RMAX>
static __global__ void k_bins_dense(const C<T>* __restrict__ h, int N, int pwx, int pwy, int pwz,
                             BinMap bm, int R, double* __restrict__ part) {
  __shared__ double acc[RMAX];
  for (int i = threadIdx.x; i < R; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  const int nx = win_len(pwx), ny = win_len(pwy), nz = win_len(pwz);
  const int64_t total = (int64_t)nx * ny * nz;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < total) {
    const int ix = (int)(q % nx), iy = (int)((q / nx) % ny), iz = (int)(q / ((int64_t)nx * ny));
    const int i = ix - pwx, j = iy - pwy, k = iz - pwz;
    const int b = classify_bin(bm, i, j, k);
    if (b >= 0) {
      const int64_t idx = ((int64_t)(k & (N - 1)) * N + (j & (N - 1))) * N + (i & (N - 1));
      atomicAdd(&acc[b], bin_weight(bm, i, j, k) * (double)h[idx].x);
    }
  }
  __syncthreads();
  double* dst = part + (int64_t)blockIdx.x * 2 * R;
  for (int i = threadIdx.x; i < 2 * R; i += blockDim.x) dst[i] = i < R ? acc[i] : 0.0;
}

}  // namespace pgx
