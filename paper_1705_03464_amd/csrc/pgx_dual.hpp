// Dual (gather) form of the forward estimator, the paper's own evaluation
// (Methodology, equation bpg_final): instead of one transform per pair field,
// one transform per pair of output bins.  For output bin b with lattice
// indicator S_b,
//   S_fb = sum_{s in b} IDFT(Z_f conj(G))(s) = sum_{p in f} w_p U_b(m_p),
//   U_b  = IDFT(S^_b G)  (= N^3 (S_b * g~), the bin kernel convolved with the
//                         DC-free galaxy field),
// with U_b(m_p) the CIC interpolation of U_b at the pair midpoint: the same
// identity as the adjoint of CIC assignment, exact on the grid.  Bins are
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

#include "pgx_kernels.hpp"

namespace pgx {

// z pass of the dual form.  Tile (xt, ky); for each slot (pair of bins): the
// forward z transform of the kernel columns (only the window planes
// pe = (z + pwz) mod N <= 2 pwz are present), times G, inverse z transform,
// stored dense.
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_zconv(const C<T>* __restrict__ ky_in, int64_t ky_slot, int n_slots, int pwz,
        const C<T>* __restrict__ fg, C<T>* __restrict__ out, int64_t out_slot,
        const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr int64_t NN = (int64_t)N * N;
  __shared__ C<T> tw_s[tw_lds_entries<Sh, kZTwReg>()];
  __shared__ C<T> lines[W][LL];
  const int xt = blockIdx.x, ky = blockIdx.y;
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  TwAuto<Sh, T, kZTwReg> twa;
  twa.init(tw_s, tw_g, t);
  const int64_t col = (int64_t)ky * N + xt * W + c;
  constexpr bool BUF = NN * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr uint32_t CB = sizeof(C<T>);
  constexpr uint32_t ZST = BUF ? (uint32_t)(TPL * NN * CB) : 0u;
  const int64_t tile = (int64_t)ky * N + xt * W;
  const uint32_t vo = (uint32_t)((c + (int64_t)t * NN) * CB);
  C<T> g[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    if constexpr (BUF) g[m] = Buf<T>(fg + tile).load(vo, (uint32_t)m * ZST);
    else g[m] = fg[col + (int64_t)(t + TPL * m) * NN];
  }
  for (int slot = 0; slot < n_slots; ++slot) {
    C<T> v[E];
    if constexpr (BUF) {
      const Buf<T> bk(ky_in + slot * ky_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int pe = (t + TPL * m + pwz) & (N - 1);
        v[m] = bk.load(pe <= 2 * pwz ? (uint32_t)((c + (int64_t)pe * NN) * CB) : kBufOff, 0u);
      }
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int pe = (t + TPL * m + pwz) & (N - 1);
        const bool ok = pe <= 2 * pwz;
        const C<T> b = ky_in[slot * ky_slot + col + (ok ? (int64_t)pe * NN : (int64_t)0)];
        v[m].x = ok ? b.x : (T)0;
        v[m].y = ok ? b.y : (T)0;
      }
    }
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
  }
}

// CIC interpolation of the packed real-space grids U_q (q < n_slots, bins
// b0 + 2q and b0 + 2q + 1) at every pair midpoint: gv[b][p] (FP32, no pair
// weight).  One thread per pair; the lower CIC node is (x0, y0, z0) with
// (y0, z0) from the pair's sort key, weights (1 - f, f) per axis.
template <typename T>
static __global__ void k_dual_gather(const int32_t* __restrict__ key, const int32_t* __restrict__ x0,
                                     const T* __restrict__ fx, const T* __restrict__ fy,
                                     const T* __restrict__ fz, int64_t P, int N,
                                     const C<T>* __restrict__ U, int64_t u_slot, int n_slots,
                                     int b0, int R, float* __restrict__ gv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t NN = (int64_t)N * N;
  const int64_t line = key[p] % NN;
  const int z0 = (int)(line / N), y0 = (int)(line % N), xa = x0[p];
  const int z1 = (z0 + 1) & (N - 1), y1 = (y0 + 1) & (N - 1), xb = (xa + 1) & (N - 1);
  const T ax = fx[p], ay = fy[p], az = fz[p];
  const T wz[2] = {(T)1 - az, az}, wy[2] = {(T)1 - ay, ay};
  const int zz[2] = {z0, z1}, yy[2] = {y0, y1};
  for (int q = 0; q < n_slots; ++q) {
    const C<T>* u = U + q * u_slot;
    C<T> s{0, 0};
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) {
        const C<T>* row = u + ((int64_t)zz[dz] * N + yy[dy]) * N;
        const C<T> a = row[xa], b = row[xb];
        const T w = wz[dz] * wy[dy];
        s.x += w * (((T)1 - ax) * a.x + ax * b.x);
        s.y += w * (((T)1 - ax) * a.y + ax * b.y);
      }
    const int b1 = b0 + 2 * q, b2 = b1 + 1;
    gv[(int64_t)b1 * P + p] = (float)s.x;
    if (b2 < R) gv[(int64_t)b2 * P + p] = (float)s.y;
  }
}

// S[f][b] = sum over the pairs of field f of w_i w_j gv[b][p] (FP64, one
// 256-thread block per (field, bin), fixed partition: deterministic).
static __global__ void k_dual_reduce(const int32_t* __restrict__ line_start, int64_t nn,
                                     const int32_t* __restrict__ pi, const int32_t* __restrict__ pj,
                                     const float* __restrict__ w, const float* __restrict__ gv,
                                     int64_t P, int R, const float* __restrict__ bscale,
                                     double* __restrict__ S) {
  __shared__ double sh[256];
  const int f = blockIdx.x, b = blockIdx.y;
  const int64_t s = line_start[(int64_t)f * nn], e = line_start[(int64_t)(f + 1) * nn];
  const float* g = gv + (int64_t)b * P;
  double acc = 0.0;
  for (int64_t p = s + threadIdx.x; p < e; p += 256) {
    const double wp = w ? (double)w[pi[p]] * (double)w[pj[p]] : 1.0;
    acc += wp * (double)g[p];
  }
  const double r = block_sum256(acc, sh);
  // undo the bin's kernel scale (the FP32 value the kernel generator applied)
  if (threadIdx.x == 0) S[(int64_t)f * R + b] = r / (double)bscale[b];
}

// ----------------------------------------------------------------------------
// Adjoint of the dual form
// ----------------------------------------------------------------------------
// line-major order of the pair catalogue: base line of each pair (sort key)
static __global__ void k_line_of(const int32_t* __restrict__ key, int64_t P, int64_t nn,
                                 int32_t* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) out[p] = (int32_t)(key[p] % nn);
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

// x pass of the Pi fields with the CIC scatter fused in.  Block = W whole
// lines (all N*N lines of every slot are written: zero lines transform to
// zero); slot = blockIdx.z, bins (2(q0+slot), 2(q0+slot)+1).  The line is
// built in LDS from the points of the four base lines whose CIC footprint
// reaches it, each point weighted by its pair weight and its field's
// coefficient pair, then transformed along x.
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_xscatter_dual(PointSet<T> ps, const int32_t* __restrict__ lfield, const float2* __restrict__ coef,
                int F, int q0, C<T>* __restrict__ out, int64_t out_slot,
                const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
  const int li = blockIdx.x * W + l;  // < N*N by the grid
  const int slot = blockIdx.z;
  const float2* cq = coef + (int64_t)(q0 + slot) * F;
  C<T>* line = lines[l];
#pragma unroll
  for (int m = 0; m < E; ++m) line[lpad(t + TPL * m)] = C<T>{0, 0};
  const int y = li % N, z = li / N;
  block_sync();
  const int ym = (y - 1) & (N - 1), zm = (z - 1) & (N - 1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int by = (q & 1) ? ym : y, bz = (q & 2) ? zm : z;
    const int key = bz * N + by;
    const int s = ps.line_start[key], e = ps.line_start[key + 1];
    for (int p = s + t; p < e; p += TPL) {
      const T fy = ps.fy[p], fz = ps.fz[p], fx = ps.fx[p];
      const T wy = (q & 1) ? fy : (T)1 - fy;
      const T wz = (q & 2) ? fz : (T)1 - fz;
      const T w = ps.wt[p] * wy * wz;
      const float2 c = cq[lfield[p]];
      const T w0 = w * ((T)1 - fx), w1 = w * fx;
      const int x0 = ps.x0[p];
      C<T>* a0 = &line[lpad(x0)];
      C<T>* a1 = &line[lpad((x0 + 1) & (N - 1))];
      atomicAdd(&a0->x, w0 * (T)c.x);
      atomicAdd(&a0->y, w0 * (T)c.y);
      atomicAdd(&a1->x, w1 * (T)c.x);
      atomicAdd(&a1->y, w1 * (T)c.y);
    }
  }
  block_sync();
  C<T> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = line[lpad(t + TPL * m)];
  block_sync();
  line_fft<Sh, -1>(v, t, line, tw_s, block_sync);
  C<T>* o = out + (int64_t)slot * out_slot + (int64_t)li * N;
#pragma unroll
  for (int m = 0; m < E; ++m) o[t + TPL * m] = v[m];
}

// z pass of the galaxy-side adjoint.  Tile (xt, ky); for each slot: forward z
// transform of the Pi columns (dense) and of the kernel columns (window
// planes only), acc += Pi^ conj(K^) / 2; then A += acc.
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_zdual_acc(const C<T>* __restrict__ x, int64_t x_slot, int n_slots,
            const C<T>* __restrict__ ky_in, int64_t ky_slot, int pwz, C<T>* __restrict__ acc_out,
            const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr int64_t NN = (int64_t)N * N;
  __shared__ C<T> tw_s[tw_lds_entries<Sh, kZTwReg>()];
  __shared__ C<T> lines[W][LL];
  const int xt = blockIdx.x, ky = blockIdx.y;
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  TwAuto<Sh, T, kZTwReg> twa;
  twa.init(tw_s, tw_g, t);
  const int64_t col = (int64_t)ky * N + xt * W + c;
  constexpr bool BUF = NN * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr uint32_t CB = sizeof(C<T>);
  constexpr uint32_t ZST = BUF ? (uint32_t)(TPL * NN * CB) : 0u;
  const int64_t tile = (int64_t)ky * N + xt * W;
  const uint32_t vo = (uint32_t)((c + (int64_t)t * NN) * CB);
  C<T> acc[E];
#pragma unroll
  for (int m = 0; m < E; ++m) acc[m] = C<T>{0, 0};
  for (int slot = 0; slot < n_slots; ++slot) {
    C<T> v[E], k[E];
    if constexpr (BUF) {
      const Buf<T> bi(x + slot * x_slot + tile);
      const Buf<T> bk(ky_in + slot * ky_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        v[m] = bi.load(vo, (uint32_t)m * ZST);
        const int pe = (t + TPL * m + pwz) & (N - 1);
        k[m] = bk.load(pe <= 2 * pwz ? (uint32_t)((c + (int64_t)pe * NN) * CB) : kBufOff, 0u);
      }
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        v[m] = x[slot * x_slot + col + (int64_t)(t + TPL * m) * NN];
        const int pe = (t + TPL * m + pwz) & (N - 1);
        const bool ok = pe <= 2 * pwz;
        const C<T> b = ky_in[slot * ky_slot + col + (ok ? (int64_t)pe * NN : (int64_t)0)];
        k[m].x = ok ? b.x : (T)0;
        k[m].y = ok ? b.y : (T)0;
      }
    }
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
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
    C<T>* p = acc_out + col + (int64_t)(t + TPL * m) * NN;
    const C<T> o = *p;
    *p = C<T>{o.x + acc[m].x, o.y + acc[m].y};
  }
}

}  // namespace pgx
