// Dual (gather) form of the forward estimator, the paper's own evaluation
// (Methodology, equation bpg_final): instead of one transform per pair field,
// one transform per pair of output bins.  For output bin b with lattice
// indicator S_b,
//   S_fb = sum_{s in b} IDFT(Z_f conj(G))(s) = sum_{p in f} w_p U_b(m_p),
//   U_b  = IDFT(S^_b G)  (= N^3 (S_b * g~), the bin kernel convolved with the
//                         DC-free galaxy field),
// with U_b(m_p) the CIC interpolation of U_b at the pair midpoint: the same
// identity as the adjoint of CIC assignment, exact on the grid.  The last
// inverse transform (along x) and that interpolation run together in a
// sweep along z that holds each point's four CIC lines in LDS.  Bins are
// packed in pairs (b1, b2) as U = U_b1 + i U_b2 (both real, since S_b is real
// and even and g is real).  The kernel columns S_b1 + i S_b2 come from the
// adjoint's kernel generator (x and y transforms of the window) with
// coefficients 1 / n_b, so that the two bins sharing a grid have comparable
// magnitudes; the per-field sums divide the scale out again.
//
// Adjoint.  With a_fb = dL/dS_fb:
//   pair side    dL/dw_p = sum_b a_{f(p)b} U_b(m_p), from the gathered values
//                the forward kept (no transform);
//   galaxy side  dL/dg' = sum_b S_b * Pi_b, Pi_b = sum_f a_fb rho_f, i.e. all
//                pairs scattered with the coefficients of their field for bin
//                b.  Bins travel in pairs again: Pi_b1 + i Pi_b2 is built
//                line by line (CIC in LDS, x transform), y and z transformed,
//                and its product with the conjugate spectrum of the bin
//                kernel pair, halved, is added to the same spectral
//                accumulator the per-field adjoint fills (real part of the
//                inverse transform = the sum over both bins).
// The Pi scatter needs all pairs grouped by their base line whatever their
// field: a second, line-major copy of the pair catalogue.
#pragma once

#include <climits>

#include "pgx_adjoint.hpp"
#include "pgx_kernels.hpp"

namespace pgx {

// z pass of the dual form.  Tile (xt, ky); for each slot (pair of bins): the
// forward z transform of the kernel columns (only the window planes
// pe = (z + pwz) mod N <= 2 pwz are present), times G, inverse z transform,
// stored dense.  Slot pipeline as in the forward cross-power pass: the next
// slot's kernel columns are loaded into the idle register set at the top of
// each trip, so the wait for them does not include the current slot's
// stores.
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_zconv(const C<T>* __restrict__ ky_in, int64_t ky_slot, int n_slots, int pwz,
        const C<T>* __restrict__ fg, C<T>* __restrict__ out, int64_t out_slot,
        const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr int64_t NN = (int64_t)N * N;
  constexpr bool PIPE = E <= 8;
  __shared__ C<T> tw_s[tw_lds_entries<Sh, kZTwReg>()];
  __shared__ C<T> lines[W][LL];
  int xt, ky;
  xcd_tile(xt, ky);
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  TwAuto<Sh, T, kZTwReg> twa;
  twa.init(tw_s, tw_g, t);
  const int64_t col = (int64_t)ky * N + xt * W + c;
  constexpr bool BUF = NN * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr uint32_t CB = sizeof(C<T>);
  constexpr uint32_t ZST = BUF ? (uint32_t)(TPL * NN * CB) : 0u;
  const int64_t tile = (int64_t)ky * N + xt * W;
  const uint32_t vo = (uint32_t)((c + (int64_t)t * NN) * CB);
  // kernel columns of one slot; planes outside the window, and every plane
  // when `take` is false, are zero
  auto load_k = [&](int slot, bool take, C<T>* k) {
    if constexpr (BUF) {
      const Buf<T> bk(ky_in + slot * ky_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int pe = (t + TPL * m + pwz) & (N - 1);
        k[m] = bk.load(take && pe <= 2 * pwz ? (uint32_t)((c + (int64_t)pe * NN) * CB) : kBufOff, 0u);
      }
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int pe = (t + TPL * m + pwz) & (N - 1);
        const bool ok = take && pe <= 2 * pwz;
        const C<T> b = ky_in[slot * ky_slot + col + (ok ? (int64_t)pe * NN : (int64_t)0)];
        k[m].x = ok ? b.x : (T)0;
        k[m].y = ok ? b.y : (T)0;
      }
    }
  };
  C<T> ka[E], kb[PIPE ? E : 1], g[E];
  load_k(0, true, ka);
  // G after the first columns (the same wait on entry as on later trips)
#pragma unroll
  for (int m = 0; m < E; ++m) {
    if constexpr (BUF) g[m] = Buf<T>(fg + tile).load(vo, (uint32_t)m * ZST);
    else g[m] = fg[col + (int64_t)(t + TPL * m) * NN];
  }
  auto body = [&](int slot, C<T>* v) {
    block_sync();
    twa.template fft<-1>(v, t, lines[c]);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmul(v[m], g[m]);
    block_sync();
    twa.template fft<1>(v, t, lines[c]);
    if constexpr (BUF) {
      const Buf<T> bo(out + slot * out_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) bo.store(v[m], vo, (uint32_t)m * ZST);
    } else {
      C<T>* dst = out + slot * out_slot + col;
#pragma unroll
      for (int m = 0; m < E; ++m) dst[(int64_t)(t + TPL * m) * NN] = v[m];
    }
  };
  if constexpr (PIPE) {
    auto trip = [&](int slot, const C<T>* cur, C<T>* nxt) {
      const bool more = slot + 1 < n_slots;
      load_k(more ? slot + 1 : slot, more, nxt);
      __builtin_amdgcn_sched_barrier(0);
      C<T> v[E];
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cur[m];
      body(slot, v);
    };
    int slot = 0;
    for (; slot + 1 < n_slots; slot += 2) {
      trip(slot, ka, kb);
      trip(slot + 1, kb, ka);
    }
    if (slot < n_slots) trip(slot, ka, kb);
  } else {
    for (int slot = 0; slot < n_slots; ++slot) {
      if (slot > 0) load_k(slot, true, ka);
      C<T> v[E];
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = ka[m];
      body(slot, v);
    }
  }
}

// Inverse x pass of the dual form fused with the CIC gather, as a sweep
// along z.  Block = (tile of YT base lines in y, segment of z, slot).  It
// keeps two z rows of YT + 1 lines in LDS (the lines y_base .. y_base + YT,
// inverse transformed along x): with row z0 and row z0 + 1 resident, every
// point whose base line is (y0, z0), y0 in the tile, finds all four lines of
// its CIC footprint in the block, and its value is written once (no
// atomics, deterministic).  Then row z0 + 2 replaces row z0, its global
// loads issued before the gather so they are in flight during it.  Points
// come from the line-major catalogue (x0, fractions; perm = field-major
// index of gv).  Bins b1 = b0 + 2 slot, b2 = b1 + 1 (< R).
template <typename T, typename Sh, int YT>
static __global__ void __launch_bounds__((YT + 1) * Sh::TPL)
k_xinv_gather_sweep(PointSet<T> ps, const int32_t* __restrict__ perm, int64_t P,
                    const C<T>* __restrict__ U, int64_t u_slot, int zlen, int b0, int R,
                    float* __restrict__ gv, const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>(), NG = YT + 1;
  constexpr int64_t NN = (int64_t)N * N;
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> rows[2][NG][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  const int g = threadIdx.x / TPL, t = threadIdx.x % TPL;
  // neighbouring y tiles share lines of every z row: they run on one XCD
  int ytile, zseg, slot;
  xcd_block3(ytile, zseg, slot);
  const int y_base = ytile * YT;
  const int y = (y_base + g) & (N - 1);  // the line this group transforms
  const int z_lo = zseg * zlen, z_hi = min(z_lo + zlen, N);
  const C<T>* us = U + (int64_t)slot * u_slot;
  const int b1 = b0 + 2 * slot, b2 = b1 + 1;
  float* g1 = gv + (int64_t)b1 * P;
  float* g2 = gv + (int64_t)b2 * P;
  // row z of this group's line into registers
  auto load_row = [&](int z, C<T>* v) {
    const C<T>* src = us + ((int64_t)(z & (N - 1)) * N + y) * N;
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = src[t + TPL * m];
  };
  // inverse transform of v in buffer `buf`, result stored there
  auto transform_into = [&](int buf, C<T>* v) {
    C<T>* line = rows[buf][g];
    line_fft<Sh, 1>(v, t, line, tw_s, wave_sync);
    wave_sync();  // this group has read its last-stage inputs
#pragma unroll
    for (int m = 0; m < E; ++m) line[lpad(t + TPL * m)] = v[m];
  };
  C<T> v[E];
  load_row(z_lo, v);
  block_sync();  // twiddles
  transform_into(0, v);
  load_row(z_lo + 1, v);
  block_sync();
  transform_into(1, v);
  block_sync();
  for (int z0 = z_lo; z0 < z_hi; ++z0) {
    const int cur = (z0 - z_lo) & 1;
    const bool more = z0 + 1 < z_hi;
    if (more) load_row(z0 + 2, v);  // in flight during the gather
    // gather: group g < YT serves base line (y_base + g, z0)
    const int y0 = y_base + g;
    if (g < YT && y0 < N) {
      const C<T>* a0 = rows[cur][g];
      const C<T>* a1 = rows[cur][g + 1];
      const C<T>* c0 = rows[cur ^ 1][g];
      const C<T>* c1 = rows[cur ^ 1][g + 1];
      const int key = z0 * N + y0;
      const int s = ps.line_start[key], e = ps.line_start[key + 1];
      for (int k = s + t; k < e; k += TPL) {
        const T fx = ps.fx[k], fy = ps.fy[k], fz = ps.fz[k];
        const int xa = ps.x0[k], xb = (xa + 1) & (N - 1);
        const int la = lpad(xa), lb = lpad(xb);
        const T w00 = ((T)1 - fy) * ((T)1 - fz), w10 = fy * ((T)1 - fz);
        const T w01 = ((T)1 - fy) * fz, w11 = fy * fz;
        const T ax = (T)1 - fx;
        const C<T> p00a = a0[la], p00b = a0[lb], p10a = a1[la], p10b = a1[lb];
        const C<T> p01a = c0[la], p01b = c0[lb], p11a = c1[la], p11b = c1[lb];
        const T sx = w00 * (ax * p00a.x + fx * p00b.x) + w10 * (ax * p10a.x + fx * p10b.x) +
                     w01 * (ax * p01a.x + fx * p01b.x) + w11 * (ax * p11a.x + fx * p11b.x);
        const T sy = w00 * (ax * p00a.y + fx * p00b.y) + w10 * (ax * p10a.y + fx * p10b.y) +
                     w01 * (ax * p01a.y + fx * p01b.y) + w11 * (ax * p11a.y + fx * p11b.y);
        const int64_t p = perm[k];
        g1[p] = (float)sx;
        if (b2 < R) g2[p] = (float)sy;
      }
    }
    block_sync();  // row z0 is no longer read
    if (more) {
      transform_into(cur, v);  // row z0 + 2 takes row z0's buffer
      block_sync();
    }
  }
}

// TSC weights along one axis of the nodes c - 1, c, c + 1 around the nearest
// node c of a point with CIC fraction f (c is the CIC corner plus one when
// f > 1/2; a point half-way takes the lower node).
template <typename T>
__device__ __forceinline__ void tsc_weights3(T f, T* w) {
  const T d = f > (T)0.5 ? f - (T)1 : f;
  w[0] = (T)0.5 * ((T)0.5 - d) * ((T)0.5 - d);
  w[1] = (T)0.75 - d * d;
  w[2] = (T)0.5 * ((T)0.5 + d) * ((T)0.5 + d);
}
// nearest node of a point with CIC corner a0 and fraction f
template <typename T>
__device__ __forceinline__ int tsc_nearest(int a0, T f, int N) {
  return (a0 + (f > (T)0.5 ? 1 : 0)) & (N - 1);
}

// Inverse x pass fused with the TSC gather, as a sweep along z (the TSC form
// of k_xinv_gather_sweep).  The line-major catalogue of a TSC plan is keyed
// by each point's nearest-node line, and a point reads the 3 x 3 lines around
// it.  Block = (tile of YT nearest-node lines in y, segment of z, slot); it
// keeps three z rows of YT + 2 lines (y_base - 1 .. y_base + YT) inverse
// transformed in LDS, so every point of a nearest-node line (y0, z0) of the
// tile finds its nine lines in the block; its value is written once.  Then
// row z0 + 2 replaces row z0 - 1, its global loads issued before the gather.
// Bins b1 = b0 + 2 slot, b2 = b1 + 1 (< R).
template <typename T, typename Sh, int YT>
static __global__ void __launch_bounds__((YT + 2) * Sh::TPL)
k_xinv_gather_sweep_tsc(PointSet<T> ps, const int32_t* __restrict__ perm, int64_t P,
                        const C<T>* __restrict__ U, int64_t u_slot, int zlen, int b0, int R,
                        float* __restrict__ gv, const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>(), NG = YT + 2;
  // stage twiddles in registers: the LDS holds only the three rows of lines
  __shared__ C<T> rows[3][NG][LL];
  const int g = threadIdx.x / TPL, t = threadIdx.x % TPL;
  TwReg<Sh, T> twr;
  twr.load(tw_g, t);
  // neighbouring y tiles share lines of every z row: they run on one XCD
  int ytile, zseg, slot;
  xcd_block3(ytile, zseg, slot);
  const int y_base = ytile * YT;
  const int y = (y_base - 1 + g) & (N - 1);  // the line this group transforms
  const int z_lo = zseg * zlen, z_hi = min(z_lo + zlen, N);
  const C<T>* us = U + (int64_t)slot * u_slot;
  const int b1 = b0 + 2 * slot, b2 = b1 + 1;
  float* g1 = gv + (int64_t)b1 * P;
  float* g2 = gv + (int64_t)b2 * P;
  auto load_row = [&](int z, C<T>* v) {
    const C<T>* src = us + ((int64_t)(z & (N - 1)) * N + y) * N;
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = src[t + TPL * m];
  };
  // ring slot of row z: rows z_lo - 1, z_lo, z_lo + 1, ... take slots 0, 1, 2, 0, ...
  auto ring = [&](int z) { return (z - z_lo + 1) % 3; };
  auto transform_into = [&](int buf, C<T>* v) {
    C<T>* line = rows[buf][g];
    line_fft_tw<Sh, 1, T>(v, t, line, twr, wave_sync);
    wave_sync();  // this group has read its last-stage inputs
#pragma unroll
    for (int m = 0; m < E; ++m) line[lpad(t + TPL * m)] = v[m];
  };
  C<T> v[E];
  load_row(z_lo - 1 + N, v);
  transform_into(ring(z_lo - 1), v);
  load_row(z_lo, v);
  transform_into(ring(z_lo), v);
  load_row(z_lo + 1, v);
  transform_into(ring(z_lo + 1), v);
  block_sync();
  for (int z0 = z_lo; z0 < z_hi; ++z0) {
    const bool more = z0 + 1 < z_hi;
    if (more) load_row(z0 + 2, v);  // in flight during the gather
    // gather: group g in [1, YT] serves nearest-node line (y_base + g - 1, z0)
    const int y0 = y_base + g - 1;
    if (g >= 1 && g <= YT && y0 < N) {
      const int rz[3] = {ring(z0 - 1), ring(z0), ring(z0 + 1)};
      const int key = z0 * N + y0;
      const int s = ps.line_start[key], e = ps.line_start[key + 1];
      for (int k = s + t; k < e; k += TPL) {
        T wx[3], wy[3], wz[3];
        int lx;
        tsc_axis<T>(ps.x0[k], ps.fx[k], lx, wx);
        tsc_weights3<T>(ps.fy[k], wy);
        tsc_weights3<T>(ps.fz[k], wz);
        T sx = (T)0, sy = (T)0;
#pragma unroll
        for (int jz = 0; jz < 3; ++jz)
#pragma unroll
          for (int jy = 0; jy < 3; ++jy) {
            const C<T>* a = rows[rz[jz]][g - 1 + jy];
            T ax = (T)0, ay = (T)0;
#pragma unroll
            for (int jx = 0; jx < 3; ++jx) {
              const C<T> c = a[lpad((lx + jx) & (N - 1))];
              ax += wx[jx] * c.x;
              ay += wx[jx] * c.y;
            }
            const T w = wz[jz] * wy[jy];
            sx += w * ax;
            sy += w * ay;
          }
        const int64_t p = perm[k];
        g1[p] = (float)sx;
        if (b2 < R) g2[p] = (float)sy;
      }
    }
    block_sync();  // row z0 - 1 is no longer read
    if (more) {
      transform_into(ring(z0 + 2), v);  // row z0 + 2 takes row z0 - 1's buffer
      block_sync();
    }
  }
}

// S[f][b] = sum over the pairs of field f of (w_i w_j) gv[b][p] (FP64 pair
// weights from k_pair_wts), divided by the bin's kernel scale (the FP32
// value the kernel generator applied).  Block (f, b, k) of a grid (F, R, K)
// writes the partial sum of chunk k of the field's range to
// part[(f R + b) K + k]; k_sum_chunks adds them in order (deterministic).
static __global__ void k_dual_reduce(const int32_t* __restrict__ line_start, int64_t nn,
                                     const double* __restrict__ wp, const float* __restrict__ gv,
                                     int64_t P, int R, const float* __restrict__ bscale,
                                     double* __restrict__ part) {
  __shared__ double sh[256];
  const int f = blockIdx.x, b = blockIdx.y, k = blockIdx.z, K = gridDim.z;
  int64_t cs, ce;
  chunk_of(line_start[(int64_t)f * nn], line_start[(int64_t)(f + 1) * nn], k, K, cs, ce);
  const float* g = gv + (int64_t)b * P;
  double acc = 0.0;
  for (int64_t p = cs + threadIdx.x; p < ce; p += 256) acc += wp[p] * (double)g[p];
  const double r = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[((int64_t)f * R + b) * K + k] = r / (double)bscale[b];
}

// ----------------------------------------------------------------------------
// Adjoint of the dual form
// ----------------------------------------------------------------------------
// line-major order of the pair catalogue: sort key (base line, x0) of each
// pair, so that within a base line the points run in x order
static __global__ void k_line_x_key(const int32_t* __restrict__ key, const int32_t* __restrict__ x0,
                                    int64_t P, int64_t nn, int n, int32_t* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) out[p] = (int32_t)((key[p] % nn) * n + x0[p]);
}
// TSC plans: the sort key (nearest-node line, nearest x node) of each pair,
// from its CIC corner and fractions (the same FP32 fractions, and the same
// rule for a point half-way, as the TSC weights)
template <typename T>
static __global__ void k_line_x_key_tsc(const int32_t* __restrict__ key, const int32_t* __restrict__ x0,
                                        const T* __restrict__ fx, const T* __restrict__ fy,
                                        const T* __restrict__ fz, int64_t P, int64_t nn, int n,
                                        int32_t* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int line = (int)(key[p] % nn);
  const int cy = tsc_nearest(line % n, fy[p], n), cz = tsc_nearest(line / n, fz[p], n);
  const int cx = tsc_nearest(x0[p], fx[p], n);
  out[p] = (int32_t)(((int64_t)cz * n + cy) * n + cx);
}
// base line of a sorted (line, x0) key
static __global__ void k_key_line(const int32_t* __restrict__ k, int64_t P, int n,
                                  int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P) out[i] = k[i] / n;
}
// field of each pair in line-major order (lp: line-major -> field-major index)
static __global__ void k_field_of(const int32_t* __restrict__ lp, const int32_t* __restrict__ key,
                                  int64_t P, int64_t nn, int32_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < P) out[k] = (int32_t)(key[lp[k]] / nn);
}

// Scatter coefficients of the bin pairs: coef[q*F + f] = (a_f,b1 / s_b1,
// a_f,b2 / s_b2) for b1 = 2q, b2 = 2q + 1 (zero past the last bin), with s_b
// the FP32 scale of bin b's kernel field, so that the products with the
// kernel spectra come out unscaled.
static __global__ void k_dual_coef(const double* __restrict__ a, int F, int R,
                                   const float* __restrict__ bscale, int Q,
                                   float2* __restrict__ coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Q * F) return;
  const int q = (int)(i / F), f = (int)(i - (int64_t)q * F);
  const int b1 = 2 * q, b2 = b1 + 1;
  float2 c;
  c.x = (float)(a[(int64_t)f * R + b1] / (double)bscale[b1]);
  c.y = b2 < R ? (float)(a[(int64_t)f * R + b2] / (double)bscale[b2]) : 0.0f;
  coef[i] = c;
}

// Pair side: acc[p] = sum_b a_{f(p)b} gv[b][p] / s_b  (= dL/dw_p before the
// normalisation terms), FP64 accumulation.
static __global__ void k_dual_pair_grad(const int32_t* __restrict__ key, int64_t P, int64_t nn,
                                        const double* __restrict__ a, int R,
                                        const float* __restrict__ gv,
                                        const float* __restrict__ bscale, float* __restrict__ acc) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double* ar = a + (int64_t)(key[p] / nn) * R;
  double s = 0.0;
  for (int b = 0; b < R; ++b) s += ar[b] * (double)gv[(int64_t)b * P + p] / (double)bscale[b];
  acc[p] = (float)s;
}

// The points whose CIC footprint reaches line (y, z): those of the four base
// lines (y, z), (y-1, z), (y, z-1), (y-1, z-1), taken as one index range
// (range q = base line q, whose y / z weight is the upper one when bit 0 /
// bit 1 of q is set).
struct LineRanges {
  int o1, o2, o3, n, d0, d1, d2, d3;
  template <typename T>
  __device__ __forceinline__ void init(const PointSet<T>& ps, int y, int z, int N) {
    const int ym = (y - 1) & (N - 1), zm = (z - 1) & (N - 1);
    const int k0 = z * N + y, k1 = z * N + ym, k2 = zm * N + y, k3 = zm * N + ym;
    const int s0 = ps.line_start[k0], e0 = ps.line_start[k0 + 1];
    const int s1 = ps.line_start[k1], e1 = ps.line_start[k1 + 1];
    const int s2 = ps.line_start[k2], e2 = ps.line_start[k2 + 1];
    const int s3 = ps.line_start[k3], e3 = ps.line_start[k3 + 1];
    o1 = e0 - s0;
    o2 = o1 + (e1 - s1);
    o3 = o2 + (e2 - s2);
    n = o3 + (e3 - s3);
    d0 = s0;
    d1 = s1 - o1;
    d2 = s2 - o2;
    d3 = s3 - o3;
  }
  // range and point of combined index i < n
  __device__ __forceinline__ int range(int i) const { return (i >= o1) + (i >= o2) + (i >= o3); }
  __device__ __forceinline__ int point(int i, int q) const {
    return i + (q == 0 ? d0 : q == 1 ? d1 : q == 2 ? d2 : d3);
  }
};

// CIC weights of point p on a line of its range q: the two x nodes
// (x0, x0 + 1) get w * (1 - fx) and w * fx, w = weight * y weight * z weight.
template <typename T>
__device__ __forceinline__ void cic_on_line(const PointSet<T>& ps, int p, int q, T& wa, T& wb,
                                            int& x0) {
  const T fy = ps.fy[p], fz = ps.fz[p], fx = ps.fx[p];
  const T wy = (q & 1) ? fy : (T)1 - fy;
  const T wz = (q & 2) ? fz : (T)1 - fz;
  const T w = (ps.wt ? ps.wt[p] : (T)1) * wy * wz;
  wa = w * ((T)1 - fx);
  wb = w * fx;
  x0 = ps.x0[p];
}

// Segmented inclusive sums over one wavefront (64 lanes, lane = threadIdx.x
// mod 64) whose keys ascend, so that equal keys form contiguous runs: after
// add(v), each lane holds the sum of v over the lanes of its run up to and
// including itself; `tail` marks the last lane of each run.  In-row steps
// use DPP row shifts (1, 2, 4, 8 lanes within rows of 16), then the running
// sums are carried across rows from lanes 15, 31 and 47 in turn (the usual
// wavefront scan); every step adds only where the source lane has the same
// key.  All 64 lanes must take part.
struct WaveRuns {
  uint32_t m;
  bool tail;
  __device__ __forceinline__ void init(int key) {
    const int lane = (int)(threadIdx.x & 63u);
    const int k1 = __builtin_amdgcn_update_dpp(INT_MIN, key, 0x111, 0xF, 0xF, false);
    const int k2 = __builtin_amdgcn_update_dpp(INT_MIN, key, 0x112, 0xF, 0xF, false);
    const int k4 = __builtin_amdgcn_update_dpp(INT_MIN, key, 0x114, 0xF, 0xF, false);
    const int k8 = __builtin_amdgcn_update_dpp(INT_MIN, key, 0x118, 0xF, 0xF, false);
    const int k15 = __builtin_amdgcn_readlane(key, 15);
    const int k31 = __builtin_amdgcn_readlane(key, 31);
    const int k47 = __builtin_amdgcn_readlane(key, 47);
    const int row = lane >> 4;
    m = (uint32_t)(k1 == key) | ((uint32_t)(k2 == key) << 1) | ((uint32_t)(k4 == key) << 2) |
        ((uint32_t)(k8 == key) << 3) | ((uint32_t)(row == 1 && key == k15) << 4) |
        ((uint32_t)(row == 2 && key == k31) << 5) | ((uint32_t)(row == 3 && key == k47) << 6);
    const int next = __builtin_amdgcn_ds_bpermute(((lane + 1) & 63) << 2, key);
    tail = lane == 63 || next != key;
  }
  __device__ __forceinline__ float add(float v) const {
    int b = __builtin_bit_cast(int, v);
    float s;
    s = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, b, 0x111, 0xF, 0xF, false));
    v += (m & 1u) ? s : 0.f;
    b = __builtin_bit_cast(int, v);
    s = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, b, 0x112, 0xF, 0xF, false));
    v += (m & 2u) ? s : 0.f;
    b = __builtin_bit_cast(int, v);
    s = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, b, 0x114, 0xF, 0xF, false));
    v += (m & 4u) ? s : 0.f;
    b = __builtin_bit_cast(int, v);
    s = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, b, 0x118, 0xF, 0xF, false));
    v += (m & 8u) ? s : 0.f;
    s = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 15));
    v += (m & 16u) ? s : 0.f;
    s = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 31));
    v += (m & 32u) ? s : 0.f;
    s = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 47));
    v += (m & 64u) ? s : 0.f;
    return v;
  }
};

// x pass of the Pi fields with the CIC scatter fused in.  Block = W lines
// (y, z), each for every slot of the batch in turn (bins 2(q0+slot),
// 2(q0+slot)+1): the line is built in LDS from the points whose CIC
// footprint reaches it, each weighted by its pair weight and its field's
// coefficient pair, transformed along x and written.  The first point of
// every thread (most lines have at most TPL points) stays in registers
// across the slots, with its coefficients for the next slot loaded one slot
// ahead; further points of crowded lines are read again per slot.  Every one
// of the N*N lines is written (zero lines transform to zero).  With HARM
// (the multipoles' adjoint) the slots hold (bin, harmonic) combos c = b nh + h
// and each pair's coefficient is also multiplied by its harmonic
// yl[h P + p] (line-major pair index p).
template <typename T, typename Sh, int W, bool HARM = false>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_xscatter_dual(PointSet<T> ps, const int32_t* __restrict__ lfield, const float2* __restrict__ coef,
                int F, int q0, int nq, C<T>* __restrict__ out, int64_t out_slot,
                const C<T>* __restrict__ tw_g, const float* __restrict__ yl = nullptr, int nh = 1,
                int64_t P = 0) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
  const int li = blockIdx.x * W + l;  // < N*N by the grid
  const int y = li % N, z = li / N;
  C<T>* line = lines[l];
  LineRanges lr;
  lr.init(ps, y, z, N);
  const bool has0 = t < lr.n;
  T wa0 = (T)0, wb0 = (T)0;
  int xa0 = 0, f0 = 0, p0 = 0;
  if (has0) {
    const int q = lr.range(t), p = lr.point(t, q);
    cic_on_line(ps, p, q, wa0, wb0, xa0);
    f0 = lfield[p];
    p0 = p;
  }
  // the pair's harmonic factors of the slot's two combos (multipoles)
  auto harm = [&](float2 c, int p, int slot) {
    if constexpr (HARM) {
      const int c1 = 2 * (q0 + slot);
      c.x *= yl[(int64_t)(c1 % nh) * P + p];
      c.y *= yl[(int64_t)((c1 + 1) % nh) * P + p];
    }
    return c;
  };
  const int xb0 = (xa0 + 1) & (N - 1);
  // one line per wavefront: contributions of points on the same x node are
  // summed across the wavefront first (the points of a base line run in x
  // order), and only the last lane of each run adds to LDS
  constexpr bool RUNS = TPL == 64 && std::is_same<T, float>::value;
  WaveRuns r0;
  if constexpr (RUNS) r0.init(has0 ? lr.range(t) * N + xa0 : 4 * N + t);
  float2 cn = has0 ? coef[(int64_t)q0 * F + f0] : float2{0.f, 0.f};
  for (int slot = 0; slot < nq; ++slot) {
    const float2 c0 = has0 ? harm(cn, p0, slot) : cn;
    if (has0 && slot + 1 < nq) cn = coef[(int64_t)(q0 + slot + 1) * F + f0];
    if (slot > 0) block_sync();  // the previous slot's transform has left the LDS line
#pragma unroll
    for (int m = 0; m < E; ++m) line[lpad(t + TPL * m)] = C<T>{0, 0};
    block_sync();
    const float2* cq = coef + (int64_t)(q0 + slot) * F;
    if constexpr (RUNS) {
      const T ax = r0.add(wa0 * (T)c0.x), ay = r0.add(wa0 * (T)c0.y);
      const T bx = r0.add(wb0 * (T)c0.x), by = r0.add(wb0 * (T)c0.y);
      if (has0 && r0.tail) {
        atomicAdd(&line[lpad(xa0)].x, ax);
        atomicAdd(&line[lpad(xa0)].y, ay);
        atomicAdd(&line[lpad(xb0)].x, bx);
        atomicAdd(&line[lpad(xb0)].y, by);
      }
      // crowded lines: further points, a wavefront-wide pass at a time
      for (int base = TPL; base < lr.n; base += TPL) {
        const int i = base + t;
        const bool act = i < lr.n;
        T wa = (T)0, wb = (T)0;
        int xa = 0, q = 0;
        float2 c = float2{0.f, 0.f};
        if (act) {
          q = lr.range(i);
          const int p = lr.point(i, q);
          cic_on_line(ps, p, q, wa, wb, xa);
          c = harm(cq[lfield[p]], p, slot);
        }
        WaveRuns r;
        r.init(act ? q * N + xa : 4 * N + t);
        const T sx = r.add(wa * (T)c.x), sy = r.add(wa * (T)c.y);
        const T tx = r.add(wb * (T)c.x), ty = r.add(wb * (T)c.y);
        if (act && r.tail) {
          const int xb = (xa + 1) & (N - 1);
          atomicAdd(&line[lpad(xa)].x, sx);
          atomicAdd(&line[lpad(xa)].y, sy);
          atomicAdd(&line[lpad(xb)].x, tx);
          atomicAdd(&line[lpad(xb)].y, ty);
        }
      }
    } else {
      if (has0) {
        atomicAdd(&line[lpad(xa0)].x, wa0 * (T)c0.x);
        atomicAdd(&line[lpad(xa0)].y, wa0 * (T)c0.y);
        atomicAdd(&line[lpad(xb0)].x, wb0 * (T)c0.x);
        atomicAdd(&line[lpad(xb0)].y, wb0 * (T)c0.y);
      }
      for (int i = t + TPL; i < lr.n; i += TPL) {
        const int q = lr.range(i), p = lr.point(i, q);
        T wa, wb;
        int xa;
        cic_on_line(ps, p, q, wa, wb, xa);
        const float2 c = harm(cq[lfield[p]], p, slot);
        const int xb = (xa + 1) & (N - 1);
        atomicAdd(&line[lpad(xa)].x, wa * (T)c.x);
        atomicAdd(&line[lpad(xa)].y, wa * (T)c.y);
        atomicAdd(&line[lpad(xb)].x, wb * (T)c.x);
        atomicAdd(&line[lpad(xb)].y, wb * (T)c.y);
      }
    }
    block_sync();
    C<T> v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = line[lpad(t + TPL * m)];
    block_sync();
    line_fft<Sh, -1>(v, t, line, tw_s, wave_sync);
    C<T>* o = out + (int64_t)slot * out_slot + (int64_t)li * N;
#pragma unroll
    for (int m = 0; m < E; ++m) o[t + TPL * m] = v[m];
  }
}

// z pass of the galaxy-side adjoint.  Tile (xt, ky); for each slot: forward z
// transform of the Pi columns (dense) and of the kernel columns (window
// planes only), acc += Pi^ conj(K^) / 2; then A += acc.  Slot pipeline: at
// the top of each trip the current slot's kernel columns and the next slot's
// Pi columns are issued, so both are in flight during the transforms.
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_zdual_acc(const C<T>* __restrict__ x, int64_t x_slot, int n_slots,
            const C<T>* __restrict__ ky_in, int64_t ky_slot, int pwz, C<T>* __restrict__ acc_out,
            const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr int64_t NN = (int64_t)N * N;
  constexpr bool PIPE = E <= 8;
  __shared__ C<T> tw_s[tw_lds_entries<Sh, kZTwReg>()];
  __shared__ C<T> lines[W][LL];
  int xt, ky;
  xcd_tile(xt, ky);
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  TwAuto<Sh, T, kZTwReg> twa;
  twa.init(tw_s, tw_g, t);
  const int64_t col = (int64_t)ky * N + xt * W + c;
  constexpr bool BUF = NN * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr uint32_t CB = sizeof(C<T>);
  constexpr uint32_t ZST = BUF ? (uint32_t)(TPL * NN * CB) : 0u;
  const int64_t tile = (int64_t)ky * N + xt * W;
  const uint32_t vo = (uint32_t)((c + (int64_t)t * NN) * CB);
  // Pi columns of one slot (zero when `take` is false)
  auto load_pi = [&](int slot, bool take, C<T>* v) {
    if constexpr (BUF) {
      const Buf<T> bi(x + slot * x_slot + tile);
      const uint32_t kill = take ? 0u : kBufOff;
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = bi.load((vo + (uint32_t)m * ZST) | kill, 0u);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const C<T> b = x[slot * x_slot + col + (int64_t)(t + TPL * m) * NN];
        v[m].x = take ? b.x : (T)0;
        v[m].y = take ? b.y : (T)0;
      }
    }
  };
  // kernel columns: only the window planes pe = (z + pwz) mod N <= 2 pwz
  auto load_k = [&](int slot, C<T>* k) {
    if constexpr (BUF) {
      const Buf<T> bk(ky_in + slot * ky_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int pe = (t + TPL * m + pwz) & (N - 1);
        k[m] = bk.load(pe <= 2 * pwz ? (uint32_t)((c + (int64_t)pe * NN) * CB) : kBufOff, 0u);
      }
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int pe = (t + TPL * m + pwz) & (N - 1);
        const bool ok = pe <= 2 * pwz;
        const C<T> b = ky_in[slot * ky_slot + col + (ok ? (int64_t)pe * NN : (int64_t)0)];
        k[m].x = ok ? b.x : (T)0;
        k[m].y = ok ? b.y : (T)0;
      }
    }
  };
  C<T> acc[E];
#pragma unroll
  for (int m = 0; m < E; ++m) acc[m] = C<T>{0, 0};
  auto body = [&](C<T>* v, C<T>* k) {
    block_sync();
    twa.template fft<-1>(v, t, lines[c]);
    block_sync();
    twa.template fft<-1>(k, t, lines[c]);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const C<T> pk = cmulc(v[m], k[m]);
      acc[m].x += (T)0.5 * pk.x;
      acc[m].y += (T)0.5 * pk.y;
    }
  };
  C<T> pa[E], pb[PIPE ? E : 1];
  load_pi(0, true, pa);
  if constexpr (PIPE) {
    auto trip = [&](int slot, const C<T>* cur, C<T>* nxt) {
      const bool more = slot + 1 < n_slots;
      C<T> k[E];
      load_k(slot, k);
      load_pi(more ? slot + 1 : slot, more, nxt);
      __builtin_amdgcn_sched_barrier(0);
      C<T> v[E];
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cur[m];
      body(v, k);
    };
    int slot = 0;
    for (; slot + 1 < n_slots; slot += 2) {
      trip(slot, pa, pb);
      trip(slot + 1, pb, pa);
    }
    if (slot < n_slots) trip(slot, pa, pb);
  } else {
    for (int slot = 0; slot < n_slots; ++slot) {
      if (slot > 0) load_pi(slot, true, pa);
      C<T> k[E];
      load_k(slot, k);
      body(pa, k);
    }
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
    C<T>* p = acc_out + col + (int64_t)(t + TPL * m) * NN;
    const C<T> o = *p;
    *p = C<T>{o.x + acc[m].x, o.y + acc[m].y};
  }
}

// The points whose TSC footprint reaches line (y, z) in a TSC plan's
// line-major catalogue (keyed by nearest-node line): those of the nine lines
// (y + dy, z + dz), dy, dz in {-1, 0, 1}, taken as one index range (range
// q = 3 (dz + 1) + dy + 1).
struct LineRanges9 {
  int o[9], d[9], n;
  // UNIFORM: the line is the same on every lane of the wavefront (one line
  // per wavefront), so the table is taken into scalar registers
  template <bool UNIFORM, typename T>
  __device__ __forceinline__ void init(const PointSet<T>& ps, int y, int z, int N) {
    n = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int yy = (y + q % 3 - 1) & (N - 1), zz = (z + q / 3 - 1) & (N - 1);
      const int k = zz * N + yy;
      int s = ps.line_start[k], e = ps.line_start[k + 1];
      if constexpr (UNIFORM) {
        s = __builtin_amdgcn_readfirstlane(s);
        e = __builtin_amdgcn_readfirstlane(e);
      }
      o[q] = n;
      d[q] = s - n;
      n += e - s;
    }
  }
  __device__ __forceinline__ int range(int i) const {
    int q = 0;
#pragma unroll
    for (int k = 1; k < 9; ++k) q += i >= o[k] ? 1 : 0;
    return q;
  }
  // (selects, not indexing: the tables stay in registers)
  __device__ __forceinline__ int point(int i, int q) const {
    int dq = d[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) dq = q == k ? d[k] : dq;
    return i + dq;
  }
};
template <typename T>
__device__ __forceinline__ T pick3(const T* w, int j) {
  return j == 0 ? w[0] : (j == 1 ? w[1] : w[2]);
}

// Pi scatter of the dual form's adjoint with TSC (the TSC form of
// k_xscatter_dual): every pair whose footprint reaches line (y, z) adds
// coef[slot][f] times its weight and its TSC weights along y, z (node offset
// from its nearest node: the range it came from) and x (three nodes) to the
// line in LDS; then the line is transformed along x and stored.  One line
// per wavefront at 512^3: runs of equal (range, nearest x node) are summed
// across the wavefront first (the catalogue is sorted that way within each
// line), and only the last lane of a run issues the LDS atomics.
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_xscatter_dual_tsc(PointSet<T> ps, const int32_t* __restrict__ lfield, const float2* __restrict__ coef,
                    int F, int q0, int nq, C<T>* __restrict__ out, int64_t out_slot,
                    const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr bool RUNS = TPL == 64 && std::is_same<T, float>::value;
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
  const int li = blockIdx.x * W + l;  // < N*N by the grid
  const int y = li % N, z = li / N;
  C<T>* line = lines[l];
  LineRanges9 lr;
  lr.template init<TPL == 64>(ps, y, z, N);
  // point i of the line's nine ranges: TSC weights of this line (its weight
  // times the y and z weights of the node offset its range stands for, times
  // the three x weights), first x node and field
  auto point_data = [&](int i, T* w, int& lx, int& q, int& f) {
    q = lr.range(i);
    const int p = lr.point(i, q);
    T wy[3], wz[3];
    tsc_weights3<T>(ps.fy[p], wy);
    tsc_weights3<T>(ps.fz[p], wz);
    // this line is node 1 - (q % 3) from the nearest node in y (range
    // q % 3 = 0 holds points whose nearest line is y - 1), likewise in z
    const T wyz = (ps.wt ? ps.wt[p] : (T)1) * pick3(wy, 2 - q % 3) * pick3(wz, 2 - q / 3);
    T wx[3];
    tsc_axis<T>(ps.x0[p], ps.fx[p], lx, wx);
    w[0] = wyz * wx[0];
    w[1] = wyz * wx[1];
    w[2] = wyz * wx[2];
    f = lfield[p];
  };
  // one trip of TPL points into the line: wavefront run sums over equal
  // (range, nearest x node), then the run's last lane adds to LDS
  auto add_trip = [&](bool act, const T* w, int lx, int q, float2 c) {
    T sx[3], sy[3];
    bool issue = act;
    if constexpr (RUNS) {
      WaveRuns r;
      r.init(act ? q * N + ((lx + 1) & (N - 1)) : 9 * N + t);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        sx[j] = r.add(w[j] * (T)c.x);
        sy[j] = r.add(w[j] * (T)c.y);
      }
      issue = act && r.tail;
    } else {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        sx[j] = w[j] * (T)c.x;
        sy[j] = w[j] * (T)c.y;
      }
    }
    if (issue) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        C<T>* a = &line[lpad((lx + j) & (N - 1))];
        atomicAdd(&a->x, sx[j]);
        atomicAdd(&a->y, sy[j]);
      }
    }
  };
  // the first two trips' point data stay in registers across the slots (most
  // lines have at most 2 TPL points in their nine ranges); only the field's
  // coefficients are read per slot
  T w0[3] = {(T)0, (T)0, (T)0}, w1[3] = {(T)0, (T)0, (T)0};
  int lx0 = 0, q0r = 0, f0 = 0, lx1 = 0, q1r = 0, f1 = 0;
  const bool a0 = t < lr.n, a1 = TPL + t < lr.n;
  if (a0) point_data(t, w0, lx0, q0r, f0);
  if (a1) point_data(TPL + t, w1, lx1, q1r, f1);
  for (int slot = 0; slot < nq; ++slot) {
    if (slot > 0) block_sync();  // the previous slot's transform has left the LDS line
#pragma unroll
    for (int m = 0; m < E; ++m) line[lpad(t + TPL * m)] = C<T>{0, 0};
    block_sync();
    const float2* cq = coef + (int64_t)(q0 + slot) * F;
    // every lane of a wavefront takes the same trips (RUNS: one line per wavefront)
    if (lr.n > 0) add_trip(a0, w0, lx0, q0r, a0 ? cq[f0] : float2{0.f, 0.f});
    if (lr.n > TPL) add_trip(a1, w1, lx1, q1r, a1 ? cq[f1] : float2{0.f, 0.f});
    for (int base = 2 * TPL; base < lr.n; base += TPL) {
      const int i = base + t;
      const bool act = i < lr.n;
      T w[3] = {(T)0, (T)0, (T)0};
      int lx = 0, q = 0, f = 0;
      if (act) point_data(i, w, lx, q, f);
      add_trip(act, w, lx, q, act ? cq[f] : float2{0.f, 0.f});
    }
    block_sync();
    C<T> v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = line[lpad(t + TPL * m)];
    block_sync();
    line_fft<Sh, -1>(v, t, line, tw_s, wave_sync);
    C<T>* o = out + (int64_t)slot * out_slot + (int64_t)li * N;
#pragma unroll
    for (int m = 0; m < E; ++m) o[t + TPL * m] = v[m];
  }
}

// ----------------------------------------------------------------------------
// Kernel spectra.  The bin kernels are even in each lattice axis (every bin
// depends on i'^2 + j'^2 and k'^2 only, and the window is symmetric), so the
// full transform of a bin-pair kernel column K^ = K^_b1 + i K^_b2 satisfies
// K^(kx, ky, kz) = K^(kx, N - ky, kz) = K^(kx, ky, N - kz).  The store keeps
// the rows ky, kz <= N/2 of every x frequency, per slot
//   ks[(kz (N/2 + 1) + ky) N + kx],
// filled once per plan from the x, y transformed window columns; the z passes
// that read it skip the kernel's z transform.
// ----------------------------------------------------------------------------

// Row order of the z passes that read the store: the rows ky and N - ky (the
// same kernel rows) are adjacent in the logical tile order, so they run on
// one XCD at about the same time and the second read of a kernel row is
// served by that XCD's L2.  XCD-contiguous ranges as in xcd_tile; the grid is
// (N / W, N).
__device__ __forceinline__ void xcd_mirror_tile(int& xt, int& ky) {
  const int nb = (int)(gridDim.x * gridDim.y), bid = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int lt = (bid & 7) * (nb >> 3) + (bid >> 3);
  const int n = (int)gridDim.y, rest = lt >> 1;
  xt = rest % (int)gridDim.x;
  const int p = rest / (int)gridDim.x;  // pair of rows, in [0, N/2)
  ky = (lt & 1) == 0 ? p : (p == 0 ? n / 2 : n - p);
}

// Fill the store: block (xt, ky <= N/2, slot) transforms the window column
// along z (planes pe = (z + pwz) mod N <= 2 pwz present) and keeps kz <= N/2.
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_kspec(const C<T>* __restrict__ ky_in, int64_t ky_slot, int pwz, C<T>* __restrict__ ks,
        int64_t ks_slot, const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>(), H = N / 2;
  constexpr int64_t NN = (int64_t)N * N;
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  const int ky = blockIdx.y, slot = blockIdx.z;
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int x = blockIdx.x * W + c;
  const C<T>* kin = ky_in + slot * ky_slot + (int64_t)ky * N + x;
  C<T> k[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int pe = (t + TPL * m + pwz) & (N - 1);
    const bool ok = pe <= 2 * pwz;
    const C<T> b = kin[ok ? (int64_t)pe * NN : (int64_t)0];
    k[m].x = ok ? b.x : (T)0;
    k[m].y = ok ? b.y : (T)0;
  }
  block_sync();
  line_fft<Sh, -1>(k, t, lines[c], tw_s, block_sync);
  C<T>* o = ks + slot * ks_slot + (int64_t)ky * N + x;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kz = t + TPL * m;
    if (kz <= H) o[(int64_t)kz * (H + 1) * N] = k[m];
  }
}

// Offset (elements) of kernel row (kz, ky) at x frequency x in one slot of
// the store.
template <int N>
__device__ __forceinline__ int64_t ks_index(int kz, int kyr, int x) {
  constexpr int H = N / 2;
  const int kzr = kz <= H ? kz : N - kz;
  return ((int64_t)kzr * (H + 1) + kyr) * N + x;
}

// z pass of the dual form on the kernel spectra: per slot, K^ G (K^ from the
// store), inverse z transform, stored dense.  Shapes of at most 8 elements
// per thread are held to 64 VGPRs (stage twiddles from the LDS table, no
// prefetch of the next slot), so two 16-wave blocks share a compute unit and
// one block's memory stream overlaps the other's transforms; at 512^3 that
// beats one block per unit with the next slot's kernel values prefetched in
// registers by about 14 %.
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL, Sh::E <= 8 ? 8 : 1)
k_zconv_ks(const C<T>* __restrict__ ks, int64_t ks_slot, int n_slots, const C<T>* __restrict__ fg,
           C<T>* __restrict__ out, int64_t out_slot, const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>(), H = N / 2;
  constexpr int64_t NN = (int64_t)N * N;
  __shared__ C<T> tw_s[tw_lds_entries<Sh, false>()];
  __shared__ C<T> lines[W][LL];
  int xt, ky;
  xcd_mirror_tile(xt, ky);
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  TwAuto<Sh, T, false> twa;
  twa.init(tw_s, tw_g, t);
  const int kyr = ky <= H ? ky : N - ky, x = xt * W + c;
  const int64_t col = (int64_t)ky * N + x;
  constexpr bool BUF = NN * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr bool BUFK = (int64_t)(H + 1) * (H + 1) * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr uint32_t CB = sizeof(C<T>);
  constexpr uint32_t ZST = BUF ? (uint32_t)(TPL * NN * CB) : 0u;
  const int64_t tile = (int64_t)ky * N + xt * W;
  const uint32_t vo = (uint32_t)((c + (int64_t)t * NN) * CB);
  auto load_k = [&](int slot, C<T>* k) {
    if constexpr (BUFK) {
      const Buf<T> bk(ks + slot * ks_slot);
#pragma unroll
      for (int m = 0; m < E; ++m) k[m] = bk.load((uint32_t)(ks_index<N>(t + TPL * m, kyr, x) * CB), 0u);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) k[m] = ks[slot * ks_slot + ks_index<N>(t + TPL * m, kyr, x)];
    }
  };
  C<T> g[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    if constexpr (BUF) g[m] = Buf<T>(fg + tile).load(vo, (uint32_t)m * ZST);
    else g[m] = fg[col + (int64_t)(t + TPL * m) * NN];
  }
  auto body = [&](int slot, C<T>* v) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmul(v[m], g[m]);
    block_sync();
    twa.template fft<1>(v, t, lines[c]);
    if constexpr (BUF) {
      const Buf<T> bo(out + slot * out_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) bo.store(v[m], vo, (uint32_t)m * ZST);
    } else {
      C<T>* dst = out + slot * out_slot + col;
#pragma unroll
      for (int m = 0; m < E; ++m) dst[(int64_t)(t + TPL * m) * NN] = v[m];
    }
  };
  for (int slot = 0; slot < n_slots; ++slot) {
    C<T> v[E];
    load_k(slot, v);
    body(slot, v);
  }
}

// Scale of the galaxy kernel in terms of the stored bin-pair spectra: the
// galaxy-side kernel of the adjoint is sum_b a_gg,b S_b, and slot q of the
// store holds (S^_b1 + i S^_b2) s_b (s_b the FP32 bin scale), so
// K^_g = sum_q (gc_q.x Re + gc_q.y Im) with gc_q = (a_gg,b1 / s_b1, a_gg,b2 / s_b2).
static __global__ void k_gal_coef(const double* __restrict__ agg, int R,
                                  const float* __restrict__ bscale, int Q,
                                  float2* __restrict__ gc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  const int b1 = 2 * q, b2 = b1 + 1;
  float2 c;
  c.x = (float)(agg[b1] / (double)bscale[b1]);
  c.y = b2 < R ? (float)(agg[b2] / (double)bscale[b2]) : 0.0f;
  gc[q] = c;
}

// z pass of the galaxy-side adjoint on the kernel spectra.  Per slot: forward
// z transform of the Pi columns, acc += Pi^ conj(K^) / 2, and the galaxy
// kernel's spectrum kg += gc.x Re K^ + gc.y Im K^ (each thread owns its
// column elements' entries, so no barrier guards them).  Then
//   A = acc + kg G   (first batch of bin pairs), A += acc + kg G (later ones),
// which also takes the place of the separate galaxy-kernel pass.
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL, Sh::E <= 8 ? 8 : 1)
k_zdual_acc_ks(const C<T>* __restrict__ x, int64_t x_slot, int n_slots,
               const C<T>* __restrict__ ks, int64_t ks_slot, const float2* __restrict__ gc,
               const C<T>* __restrict__ fg, int first, C<T>* __restrict__ acc_out,
               const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>(), H = N / 2;
  constexpr int64_t NN = (int64_t)N * N;
  // Shapes of at most 8 elements per thread run lean: the galaxy-kernel sum
  // in registers, stage twiddles from the LDS table, the kernel values loaded
  // after the transform and in two halves, no register prefetch of the next
  // slot; the kernel then fits 64 VGPRs without spills and about 75 KB of
  // LDS, so two blocks share a compute unit and one block's memory stream
  // overlaps the other's transforms (5.55 -> 4.14 ms per launch at 512^3
  // with 10 bin pairs).  Larger shapes keep the sum in LDS.
  constexpr bool LEAN = E <= 8;
  __shared__ C<T> tw_s[LEAN ? Sh::tw_entries() : tw_lds_entries<Sh, kZTwReg>()];
  __shared__ C<T> lines[W][LL];
  __shared__ T kgs[LEAN ? 1 : W][LEAN ? 1 : N];
  int xt, ky;
  xcd_mirror_tile(xt, ky);
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  TwAuto<Sh, T, !LEAN && kZTwReg> twa;
  twa.init(tw_s, tw_g, t);
  const int kyr = ky <= H ? ky : N - ky, xx = xt * W + c;
  const int64_t col = (int64_t)ky * N + xx;
  constexpr bool BUF = NN * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr bool BUFK = (int64_t)(H + 1) * (H + 1) * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr uint32_t CB = sizeof(C<T>);
  constexpr uint32_t ZST = BUF ? (uint32_t)(TPL * NN * CB) : 0u;
  const int64_t tile = (int64_t)ky * N + xt * W;
  const uint32_t vo = (uint32_t)((c + (int64_t)t * NN) * CB);
  auto load_pi = [&](int slot, bool take, C<T>* v) {
    if constexpr (BUF) {
      const Buf<T> bi(x + slot * x_slot + tile);
      const uint32_t kill = take ? 0u : kBufOff;
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = bi.load((vo + (uint32_t)m * ZST) | kill, 0u);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const C<T> b = x[slot * x_slot + col + (int64_t)(t + TPL * m) * NN];
        v[m].x = take ? b.x : (T)0;
        v[m].y = take ? b.y : (T)0;
      }
    }
  };
  // kernel values of elements m0 .. m0 + M - 1 of this thread's column.
  // Elements m < E/2 have kz < N/2 (stored row kz), the others kz >= N/2
  // (mirrored row N - kz); each half is one per-lane base offset plus a
  // scalar offset per element, so no per-element address stays live
  constexpr uint32_t KS = (uint32_t)((H + 1) * N);
  const uint32_t kb0 = (uint32_t)(((int64_t)t * KS + (int64_t)kyr * N + xx) * CB);
  const uint32_t kb1 = (uint32_t)(((int64_t)(TPL - t) * KS + (int64_t)kyr * N + xx) * CB);
  auto load_k = [&](int slot, int m0, auto& k) {
    constexpr int M = sizeof(k) / sizeof(k[0]);
    if constexpr (BUFK) {
      const Buf<T> bk(ks + slot * ks_slot);
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int mm = m0 + m;
        k[m] = 2 * mm < E ? bk.load(kb0, (uint32_t)mm * TPL * KS * CB)
                          : bk.load(kb1, (uint32_t)(E - 1 - mm) * TPL * KS * CB);
      }
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) k[m] = ks[slot * ks_slot + ks_index<N>(t + TPL * (m0 + m), kyr, xx)];
    }
  };
  C<T> acc[E];
  T kg[LEAN ? E : 1];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    acc[m] = C<T>{0, 0};
    if constexpr (LEAN) kg[m] = (T)0;
    else kgs[c][t + TPL * m] = (T)0;
  }
  // lean shapes take the kernel values in two halves, so that at most half
  // of them are live beside the transformed column and the accumulators
  constexpr int EH = LEAN && E % 2 == 0 ? E / 2 : E;
  for (int slot = 0; slot < n_slots; ++slot) {
    C<T> v[E];
    load_pi(slot, true, v);
    block_sync();
    twa.template fft<-1>(v, t, lines[c]);
    // the kernel values are loaded after the transform, so that they are not
    // held in registers during it
    const float2 q = gc[slot];
#pragma unroll
    for (int h = 0; h < E; h += EH) {
      C<T> k[EH];
      load_k(slot, h, k);
#pragma unroll
      for (int mm = 0; mm < EH; ++mm) {
        const int m = h + mm;
        const C<T> pk = cmulc(v[m], k[mm]);
        acc[m].x += (T)0.5 * pk.x;
        acc[m].y += (T)0.5 * pk.y;
        const T kv = (T)q.x * k[mm].x + (T)q.y * k[mm].y;
        if constexpr (LEAN) kg[m] += kv;
        else kgs[c][t + TPL * m] += kv;
      }
      if constexpr (EH < E) __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int64_t idx = col + (int64_t)(t + TPL * m) * NN;
    const C<T> g = fg[idx];
    T kgv;
    if constexpr (LEAN) kgv = kg[m];
    else kgv = kgs[c][t + TPL * m];
    C<T> r = C<T>{acc[m].x + kgv * g.x, acc[m].y + kgv * g.y};
    if (!first) {
      const C<T> o = acc_out[idx];
      r.x += o.x;
      r.y += o.y;
    }
    acc_out[idx] = r;
  }
}

// ----------------------------------------------------------------------------
// Multipoles in the angle between the pair axis and the pair-to-galaxy
// direction, by the dual form.  With P_l(a . b) = 4 pi / (2l + 1)
// sum_m Y_lm(a) Y_lm(b), the sum over the lattice vectors r of shell b
//   sum_p w_p sum_r (2l + 1) P_l(d^_p . r^) g'(m_p + r)
//     = 4 pi sum_m sum_p w_p Y_lm(d^_p) U_{b,lm}(m_p),
//   U_{b,lm} = IDFT(S^_{b,lm} G),  S_{b,lm}(r) = [r in b] Y_lm(r^),
// so each (bin, harmonic) combo is one more bin kernel of the dual form
// (generated with the harmonic factor), gathered at the midpoints like the
// bins, and the per-field sums weight each pair by Y_lm of its axis.
// ----------------------------------------------------------------------------

// yp[h P + p] = Y_h(axis of pair p) (FP32), the axis d = x_j - x_i with each
// component folded once into [-L/2, L/2), from the kept galaxy positions.
static __global__ void k_pair_harm(const int32_t* __restrict__ pi, const int32_t* __restrict__ pj,
                                   const double* __restrict__ x, const double* __restrict__ y,
                                   const double* __restrict__ z, int64_t P, double L, int nh,
                                   float* __restrict__ yp) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int i = pi[p], j = pj[p];
  const double h = 0.5 * L;
  auto fold = [&](double d) { return d >= h ? d - L : (d < -h ? d + L : d); };
  const double dx = fold(x[j] - x[i]), dy = fold(y[j] - y[i]), dz = fold(z[j] - z[i]);
  for (int k = 0; k < nh; ++k) yp[(int64_t)k * P + p] = (float)real_ylm_dir(k, dx, dy, dz);
}

// S[(f R + b) nl + il] = 4 pi sum_{h of degree 2 il} sum_{p in f}
//   w_p Y_h(d^_p) gv[b nh + h][p] / s_{b nh + h}
// (FP64 pair weights).  Block (f, b nl + il, k) of a grid (F, R nl, K) writes
// the partial sum of chunk k of the field's range to part[i K + k], i the
// output index; k_sum_chunks adds them in order (deterministic).
static __global__ void k_dual_reduce_mp(const int32_t* __restrict__ line_start, int64_t nn,
                                        const double* __restrict__ wp, const float* __restrict__ gv,
                                        const float* __restrict__ yp, int64_t P, int R, int nh, int nl,
                                        const float* __restrict__ bscale, double* __restrict__ part) {
  constexpr double PI = 3.14159265358979323846;
  __shared__ double sh[256];
  const int f = blockIdx.x, b = blockIdx.y / nl, il = blockIdx.y % nl, k = blockIdx.z, K = gridDim.z;
  const int h0 = il == 0 ? 0 : (il == 1 ? 1 : 6), h1 = il == 0 ? 1 : (il == 1 ? 6 : 15);
  int64_t s, e;
  chunk_of(line_start[(int64_t)f * nn], line_start[(int64_t)(f + 1) * nn], k, K, s, e);
  double acc = 0.0;
  for (int h = h0; h < h1; ++h) {
    const int c = b * nh + h;
    const float* g = gv + (int64_t)c * P;
    const float* yh = yp + (int64_t)h * P;
    double a = 0.0;
    for (int64_t p = s + threadIdx.x; p < e; p += 256) a += wp[p] * (double)yh[p] * (double)g[p];
    acc += a / (double)bscale[c];
  }
  const double r = block_sum256(acc, sh);
  if (threadIdx.x == 0) part[(((int64_t)f * R + b) * nl + il) * K + k] = 4.0 * PI * r;
}

// xi_l[f][b][il] = S / (n_b Wsum_f W_g), the normalisation of xi_pg.
static __global__ void k_finalize_mp(const double* __restrict__ S, const double* __restrict__ nb,
                                     const double* __restrict__ wsum, const double* __restrict__ wg,
                                     int F, int R, int nl, double* __restrict__ xi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)F * R * nl) return;
  const int f = (int)(i / ((int64_t)R * nl)), b = (int)((i / nl) % R);
  xi[i] = wsum[f] > 0.0 ? S[i] / (nb[b] * wsum[f] * wg[0]) : __builtin_nan("");
}

// ----------------------------------------------------------------------------
// Adjoint of the multipoles.  With a_{f,b,l} = dL/dS_l(f, b) and the
// combo coefficients A_{f,c} = 4 pi a_{f,b(c),l(c)} / s_c:
//   pair side    dL/dw_p = sum_c A_{f(p),c} Y_h(c)(d^_p) gv[c][p],
//   galaxy side  Pi_c = sum_p A_{f(p),c} Y_h(c)(d^_p) w_p CIC(m_p), through
//                the harmonic bin kernels exactly as the dual form's adjoint.
// ----------------------------------------------------------------------------

// degree index (0, 1, 2 for l = 0, 2, 4) of harmonic h
__device__ __forceinline__ int harm_degree_index(int h) { return h == 0 ? 0 : (h < 6 ? 1 : 2); }

// dL/dS_l(f, b) = g / (n_b Wsum_f W_g) and the explicit normalisation terms
// dL/dWsum_f = -sum g xi / Wsum_f, dL/dW_g = -sum g xi / W_g (one block of
// 256 threads; terms that are not finite, and empty fields, carry none).
static __global__ void k_finalize_adjoint_mp(const double* __restrict__ S, const double* __restrict__ g,
                                             const double* __restrict__ nb,
                                             const double* __restrict__ wsum,
                                             const double* __restrict__ wg, int F, int R, int nl,
                                             double* __restrict__ a, double* __restrict__ gws,
                                             double* __restrict__ gwg) {
  __shared__ double sh[256];
  const double w = wg[0];
  double wacc = 0.0;
  for (int f = threadIdx.x; f < F; f += 256) {
    const double ws = wsum[f];
    const bool ok = ws > 0.0;
    double gs = 0.0;
    for (int o = 0; o < R * nl; ++o) {
      const int64_t i = (int64_t)f * R * nl + o;
      const int b = o / nl;
      if (ok) {
        const double gi = fin0(g[i]);
        const double xi = S[i] / (nb[b] * ws * w);
        gs += -fin0(gi * xi / ws);
        wacc += -fin0(gi * xi / w);
        a[i] = gi / (nb[b] * ws * w);
      } else {
        a[i] = 0.0;
      }
    }
    gws[f] = ok ? gs : 0.0;
  }
  const double tot = block_sum256(wacc, sh);
  if (threadIdx.x == 0) gwg[0] = tot;
}

// coef[q F + f] = (A_{f,2q}, A_{f,2q+1}) (zero past the last combo)
static __global__ void k_mp_coef(const double* __restrict__ a, int F, int R, int nh, int nl,
                                 const float* __restrict__ bscale, int QC, float2* __restrict__ coef) {
  constexpr double PI = 3.14159265358979323846;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)QC * F) return;
  const int q = (int)(i / F), f = (int)(i - (int64_t)q * F);
  const int RC = R * nh;
  auto one = [&](int c) -> float {
    if (c >= RC) return 0.0f;
    const int b = c / nh, il = harm_degree_index(c % nh);
    return (float)(4.0 * PI * a[((int64_t)f * R + b) * nl + il] / (double)bscale[c]);
  };
  coef[i] = float2{one(2 * q), one(2 * q + 1)};
}

// pair side: acc[p] = sum_c A_{f(p),c} Y_h(c)(d^_p) gv[c][p], FP64 sum
static __global__ void k_mp_pair_grad(const int32_t* __restrict__ key, int64_t P, int64_t nn,
                                      const double* __restrict__ a, int R, int nh, int nl,
                                      const float* __restrict__ gv, const float* __restrict__ yp,
                                      const float* __restrict__ bscale, float* __restrict__ acc) {
  constexpr double PI = 3.14159265358979323846;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double* af = a + (int64_t)(key[p] / nn) * R * nl;
  double s = 0.0;
  for (int b = 0; b < R; ++b)
    for (int h = 0; h < nh; ++h) {
      const int c = b * nh + h;
      s += af[b * nl + harm_degree_index(h)] * (double)yp[(int64_t)h * P + p] *
           (double)gv[(int64_t)c * P + p] / (double)bscale[c];
    }
  acc[p] = (float)(4.0 * PI * s);
}

// line-major copy of the pair harmonics: yl[h P + k] = yp[h P + lp[k]]
static __global__ void k_harm_line_major(const int32_t* __restrict__ lp, const float* __restrict__ yp,
                                         int64_t P, int nh, float* __restrict__ yl) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const int64_t p = lp[k];
  for (int h = 0; h < nh; ++h) yl[(int64_t)h * P + k] = yp[(int64_t)h * P + p];
}

}  // namespace pgx
