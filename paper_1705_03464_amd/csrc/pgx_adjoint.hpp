// Adjoint of the correlation path: gradients of a scalar loss with respect to
// the per-galaxy weights.  With raw CIC densities rho_f (pair weights) and
// rho_g (galaxy weights), g' = rho_g - W_g / N^3, Z_f = DFT(rho_f),
// G = DFT(g') (its k = 0 mode is zero) and H_f = IDFT(Z_f conj(G)), the
// forward computes
//   S_fb = sum_{s in b} H_f(s),   xi_pg[f,b] = S_fb / (n_b Wsum_f W_g)
//   Sgg_b = sum_{s in b} IDFT(|G|^2)(s),   xi_gg[b] = Sgg_b / (n_b W_g^2).
// Given a_fb = dL/dS_fb and a_gb = dL/dSgg_b, with the symmetric kernels
// K_f(r) = sum_b a_fb w(r) 1[r in b] (w = 1 for the indicator bins, the
// Gaussian-sigmoid weight for the weighted bin) and K_g likewise (real
// transforms K^):
//   dL/drho_f      = IDFT(K^_f G)                       (per pair field)
//   dL/dg'         = IDFT(sum_f K^_f Z_f) + 2 IDFT(K^_g G)
// Two fields a, b travel in one complex grid: the transform of K_a + i K_b is
// K^_a + i K^_b, so IDFT((K^_a + i K^_b) G) = dL/drho_a + i dL/drho_b, and
// with A = Z conj(K^_a + i K^_b) / 2 summed over field pairs, plus K^_g G,
// dL/dg' = 2 Re IDFT(A) (the sum over k and -k is folded into the real part).
// Zeroing A(0) projects out the mean that g' removes from rho_g.  The CIC
// gathers of these fields at the pair midpoints / galaxies, times the partner
// weight, give the weight gradient; the explicit dependence of the
// normalisations on Wsum_f and W_g is added by the finalisation adjoint.
#pragma once
#include "pgx_misc.hpp"

namespace pgx {

struct AdjointArgs {
  int F, R, qmode;
  double L, xi_w_const;
  const double* S;
  const double* Sgg;
  const double* nb;
  const double* vol;
  const double* wsum;
  const double* wg;
  const double* g_b;     // [F][R] or null
  const double* g_q;     // [F][R] or null
  const double* g_xipg;  // [F][R] or null
  const double* g_xigg;  // [R] or null
  const double* g_xidp;  // [F] or null
  double* apg;           // out [F][R] dL/dS_fb
  double* agg;           // out [R]    dL/dSgg_b
  double* gws;           // out [F]    explicit dL/dWsum_f
  double* gwg;           // out [1]    explicit dL/dW_g
};

__device__ __forceinline__ double fin0(double v) { return isfinite(v) ? v : 0.0; }

// One block of 256 threads.  Finalisation adjoint of
//   b = xi_pg / xi_gg,  xi_dp = 2 Wsum L^3 / (Wg^2 V) - 1,
//   Q (not strictly squeezed): ((1+x) b - 2 - xw/(2x)) / (2x + 1.5 xw), xw = xi_gg
//   Q (squeezed): ((1+x) b - 2) / (2x);  Q (constant xi_w): xw = const.
// Terms that are not finite (empty fields, zero xi_gg) carry no gradient.
static __global__ void k_finalize_adjoint(AdjointArgs a) {
  __shared__ double sh[256];
  const int F = a.F, R = a.R;
  const double wg = a.wg[0];
  const double L3 = a.L * a.L * a.L;
  // per field: dL/dS_fb, explicit dL/dWsum_f (own thread loops, no races)
  double wg_acc = 0.0;
  for (int f = threadIdx.x; f < F; f += 256) {
    const double ws = a.wsum[f];
    const bool ok = ws > 0.0;
    const double x = 2.0 * ws * L3 / (wg * wg * a.vol[f]) - 1.0;
    double gx = a.g_xidp ? fin0(a.g_xidp[f]) : 0.0;
    double gws = 0.0;
    for (int b = 0; b < R; ++b) {
      const int i = f * R + b;
      double gpg = 0.0;
      if (ok) {
        const double xg = a.Sgg[b] / (a.nb[b] * wg * wg);
        const double xp = a.S[i] / (a.nb[b] * ws * wg);
        const double bb = xp / xg;
        const double gq = a.g_q ? fin0(a.g_q[i]) : 0.0;
        double dqdb, dqdx;
        if (a.qmode == 1) {
          dqdb = (1.0 + x) / (2.0 * x);
          dqdx = (2.0 - bb) / (2.0 * x * x);
        } else {
          const double xw = a.qmode == 2 ? a.xi_w_const : xg;
          const double num = (1.0 + x) * bb - 2.0 - xw / (2.0 * x);
          const double den = 2.0 * x + 1.5 * xw;
          dqdb = (1.0 + x) / den;
          dqdx = ((bb + xw / (2.0 * x * x)) * den - 2.0 * num) / (den * den);
        }
        const double gbt = (a.g_b ? fin0(a.g_b[i]) : 0.0) + fin0(gq * dqdb);
        gpg = (a.g_xipg ? fin0(a.g_xipg[i]) : 0.0) + fin0(gbt / xg);
        gx += fin0(gq * dqdx);
        // xi_pg = S / (n_b Wsum Wg)
        gws += -fin0(gpg * xp / ws);
        wg_acc += -fin0(gpg * xp / wg);
        a.apg[i] = gpg / (a.nb[b] * ws * wg);
      } else {
        a.apg[i] = 0.0;
      }
    }
    if (ok) {
      // xi_dp = 2 Wsum L^3 / (Wg^2 V) - 1
      gws += gx * (x + 1.0) / ws;
      wg_acc += -2.0 * gx * (x + 1.0) / wg;
    }
    a.gws[f] = ok ? gws : 0.0;
  }
  // per output bin: dL/dSgg_b
  for (int b = threadIdx.x; b < R; b += 256) {
    const double xg = a.Sgg[b] / (a.nb[b] * wg * wg);
    double ggg = a.g_xigg ? fin0(a.g_xigg[b]) : 0.0;
    for (int f = 0; f < F; ++f) {
      const double ws = a.wsum[f];
      if (!(ws > 0.0)) continue;
      const int i = f * R + b;
      const double x = 2.0 * ws * L3 / (wg * wg * a.vol[f]) - 1.0;
      const double xp = a.S[i] / (a.nb[b] * ws * wg);
      const double bb = xp / xg;
      const double gq = a.g_q ? fin0(a.g_q[i]) : 0.0;
      double dqdb = 0.0, dqdxw = 0.0;
      if (a.qmode == 1) {
        dqdb = (1.0 + x) / (2.0 * x);
      } else {
        const double xw = a.qmode == 2 ? a.xi_w_const : xg;
        const double num = (1.0 + x) * bb - 2.0 - xw / (2.0 * x);
        const double den = 2.0 * x + 1.5 * xw;
        dqdb = (1.0 + x) / den;
        if (a.qmode == 0) dqdxw = (-den / (2.0 * x) - 1.5 * num) / (den * den);
      }
      const double gbt = (a.g_b ? fin0(a.g_b[i]) : 0.0) + fin0(gq * dqdb);
      ggg += fin0(-gbt * bb / xg) + fin0(gq * dqdxw);
    }
    // xi_gg = Sgg / (n_b Wg^2)
    wg_acc += -2.0 * fin0(ggg * xg / wg);
    a.agg[b] = ggg / (a.nb[b] * wg * wg);
  }
  const double tot = block_sum256(wg_acc, sh);
  if (threadIdx.x == 0) a.gwg[0] = tot;
}

// ----------------------------------------------------------------------------
// Kernel fields on the output window, transformed along x.  Task = window line
// (pz, py) of a slot; values K_a(r) + i K_b(r) at the lattice offsets
// r = (x' , py - pwy, pz - pwz), |x'| <= pwx; zero elsewhere on the line.
// Output layout [slot][pz][py][kx].  fa/fb index rows of coef (F x R); a
// negative index means no field.
// ----------------------------------------------------------------------------
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_kgen_x(const double* __restrict__ coef, int R, const int32_t* __restrict__ slot_fa,
         const int32_t* __restrict__ slot_fb, int pwx, int pwy, int pwz, BinMap bm,
         C<T>* __restrict__ out, int64_t out_slot, const C<T>* __restrict__ tw_g,
         const float* __restrict__ fscale = nullptr, int nh = 0) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  const int slot = blockIdx.z;
  const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
  const int ny = win_len(pwy), nz = win_len(pwz);
  const int task = blockIdx.x * W + l;
  const bool active = task < ny * nz;
  const int py = active ? task % ny : 0, pz = active ? task / ny : 0;
  const int fa = slot_fa[slot], fb = slot_fb[slot];
  C<T> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    v[m] = C<T>{0, 0};
    const int xx = t + TPL * m;
    const int px = (xx + pwx) & (N - 1);
    if (active && px <= 2 * pwx) {
      const int b = classify_bin(bm, px - pwx, py - pwy, pz - pwz);
      if (b >= 0) {
        // coefficients of a field whose transform ran scaled by fscale[f] are
        // divided by it, so products with its spectrum come out unscaled
        const double sa = fscale && fa >= 0 ? (double)fscale[fa] : 1.0;
        const double sb = fscale && fb >= 0 ? (double)fscale[fb] : 1.0;
        const double wb = bin_weight(bm, px - pwx, py - pwy, pz - pwz);
        // multipole kernels (nh > 0): "field" fa is a (bin, harmonic) combo
        // c = b nh + h, and the kernel carries Y_h of the lattice direction
        const double ya = nh > 0 && fa >= 0 ? real_ylm_dir(fa % nh, px - pwx, py - pwy, pz - pwz) : 1.0;
        const double yb = nh > 0 && fb >= 0 ? real_ylm_dir(fb % nh, px - pwx, py - pwy, pz - pwz) : 1.0;
        v[m].x = fa >= 0 ? (T)(coef[(int64_t)fa * R + b] * wb * ya / sa) : (T)0;
        v[m].y = fb >= 0 ? (T)(coef[(int64_t)fb * R + b] * wb * yb / sb) : (T)0;
      }
    }
  }
  block_sync();
  line_fft<Sh, -1>(v, t, lines[l], tw_s, wave_sync);
  if (active) {
    C<T>* o = out + slot * out_slot + (int64_t)task * N;
#pragma unroll
    for (int m = 0; m < E; ++m) o[t + TPL * m] = v[m];
  }
}

// ----------------------------------------------------------------------------
// Backward z pass.  Tile (xt, ky).  For each slot:
//   Z  = forward z of the recomputed pair-field columns (x, y transformed)
//   Kp = forward z of the kernel columns (only the window planes are present)
//   acc += Z conj(Kp) / 2                       (galaxy-side accumulation)
//   column <- inverse z of Kp G                (pair-side adjoint, in place)
// then A += acc.  G is the galaxy spectrum with its k = 0 mode removed.
// Slot pipeline as in k_zcross: plane masks in LDS, the next slot's columns
// loaded into the idle register set at the top of each trip.  STORED mode
// reads Z from the spectra the forward kept (`spec`, by field-pair index)
// instead of transforming the recomputed columns.
// ----------------------------------------------------------------------------
// the STORED variant keeps its galaxy-side accumulator in registers (it has
// one transform less in flight than the recomputing variant)
constexpr bool kZbAccRegStored = true;

template <typename T, typename Sh, int W, bool STORED = false>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_zback(C<T>* x, int64_t x_slot, const uint8_t* __restrict__ pflag,
        const int32_t* __restrict__ slot_fp, int n_slots, const C<T>* __restrict__ ky_in,
        int64_t ky_slot, int pwz, const C<T>* __restrict__ fg, C<T>* __restrict__ acc_out,
        const C<T>* __restrict__ tw_g, const C<T>* __restrict__ spec = nullptr) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr int64_t NN = (int64_t)N * N;
  constexpr bool PIPE = E <= 8;  // register room for a second set of columns
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  __shared__ uint32_t pmask[kMaxSlots][TPL];
  // accumulator of the galaxy-side term: in LDS when it fits beside the line
  // buffers (each thread owns its entries; rows padded to an odd length so the
  // W columns fall on different banks), in registers otherwise
  constexpr bool ACC_LDS =
      !(STORED && kZbAccRegStored) &&
      (size_t)(W * (N + 1) + W * LL + Sh::tw_entries()) * sizeof(C<T>) +
              (size_t)kMaxSlots * TPL * sizeof(uint32_t) <= 160 * 1024;
  __shared__ C<T> accs[ACC_LDS ? W : 1][ACC_LDS ? N + 1 : 1];
  C<T> accr[ACC_LDS ? 1 : E];
  load_twiddles<T, Sh>(tw_s, tw_g);
  int xt = blockIdx.x, ky = blockIdx.y;
  if constexpr (narrow_tile<T, W>()) xcd_tile(xt, ky);
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  for (int i = threadIdx.x; i < n_slots * TPL; i += W * TPL) {
    const int s = i / TPL, tt = i - s * TPL;
    const uint8_t* pf = pflag + (int64_t)slot_fp[s] * N + tt;
    uint32_t mk = 0;
#pragma unroll
    for (int m = 0; m < E; ++m) mk |= (uint32_t)(pf[TPL * m] != 0) << m;
    pmask[s][tt] = mk;
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
    if constexpr (ACC_LDS) accs[c][t + TPL * m] = C<T>{0, 0};
    else accr[m] = C<T>{0, 0};
  }
  block_sync();
  const int64_t col = (int64_t)ky * N + xt * W + c;
  // buffer path for fields up to 2 GiB per slot (see k_zcross)
  constexpr bool BUF = NN * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr uint32_t CB = sizeof(C<T>);
  constexpr uint32_t ZST = BUF ? (uint32_t)(TPL * NN * CB) : 0u;  // TPL planes
  const int64_t tile = (int64_t)ky * N + xt * W;
  const uint32_t vo = (uint32_t)((c + (int64_t)t * NN) * CB);
  auto load_cols = [&](int slot, bool take, C<T>* dst) {
    if constexpr (STORED) {
      // the stored spectrum Z of this slot's field pair (dense)
      const C<T>* zs = spec + (int64_t)slot_fp[slot] * (NN * N);
      if constexpr (BUF) {
        const Buf<T> bz(zs + tile);
        const uint32_t kill = take ? 0u : kBufOff;
#pragma unroll
        for (int m = 0; m < E; ++m) dst[m] = bz.load((vo + (uint32_t)m * ZST) | kill, 0u);
      } else {
#pragma unroll
        for (int m = 0; m < E; ++m) dst[m] = zs[col + (int64_t)(t + TPL * m) * NN];
      }
      return;
    }
    const uint32_t mk = take ? pmask[slot][t] : 0u;
    if constexpr (BUF) {
      const Buf<T> bi(x + slot * x_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m)
        dst[m] = bi.load((mk >> m) & 1u ? vo + (uint32_t)m * ZST : kBufOff, 0u);
    } else {
      // absent planes read the tile's first element (valid), zeroed when taken
      const C<T>* src = x + slot * x_slot + col;
#pragma unroll
      for (int m = 0; m < E; ++m) dst[m] = src[(mk >> m) & 1u ? (int64_t)(t + TPL * m) * NN : 0];
    }
  };
  auto take_cols = [&](int slot, const C<T>* cur, C<T>* v) {
    if constexpr (BUF || STORED) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cur[m];
    } else {
      const uint32_t mk = pmask[slot][t];
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const bool ok = (mk >> m) & 1u;
        v[m].x = ok ? cur[m].x : (T)0;
        v[m].y = ok ? cur[m].y : (T)0;
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
  C<T> ca[E], cb[PIPE ? E : 1], g[E];
  load_cols(0, true, ca);
  // G after the first columns (see k_zcross)
#pragma unroll
  for (int m = 0; m < E; ++m) {
    if constexpr (BUF) g[m] = Buf<T>(fg + tile).load(vo, (uint32_t)m * ZST);
    else g[m] = fg[col + (int64_t)(t + TPL * m) * NN];
  }
  auto body = [&](int slot, C<T>* v, C<T>* k) {
    if constexpr (!STORED) {
      block_sync();
      line_fft<Sh, -1>(v, t, lines[c], tw_s, block_sync);
    }
    block_sync();
    line_fft<Sh, -1>(k, t, lines[c], tw_s, block_sync);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const C<T> zk = cmulc(v[m], k[m]);
      C<T>& a = ACC_LDS ? accs[c][t + TPL * m] : accr[ACC_LDS ? 0 : m];
      a.x += (T)0.5 * zk.x;
      a.y += (T)0.5 * zk.y;
      v[m] = cmul(k[m], g[m]);
    }
    block_sync();
    line_fft<Sh, 1>(v, t, lines[c], tw_s, block_sync);
    if constexpr (BUF) {
      const Buf<T> bo(x + slot * x_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) bo.store(v[m], vo, (uint32_t)m * ZST);
    } else {
      C<T>* xs = x + slot * x_slot + col;
#pragma unroll
      for (int m = 0; m < E; ++m) xs[(int64_t)(t + TPL * m) * NN] = v[m];
    }
  };
  if constexpr (PIPE) {
    auto trip = [&](int slot, const C<T>* cur, C<T>* nxt) {
      const bool more = slot + 1 < n_slots;
      C<T> k[E];
      load_k(slot, k);
      load_cols(more ? slot + 1 : slot, more, nxt);
      __builtin_amdgcn_sched_barrier(0);
      C<T> v[E];
      take_cols(slot, cur, v);
      body(slot, v, k);
    };
    int slot = 0;
    for (; slot + 1 < n_slots; slot += 2) {
      trip(slot, ca, cb);
      trip(slot + 1, cb, ca);
    }
    if (slot < n_slots) trip(slot, ca, cb);
  } else {
    for (int slot = 0; slot < n_slots; ++slot) {
      if (slot > 0) load_cols(slot, true, ca);
      C<T> v[E], k[E];
      load_k(slot, k);
      take_cols(slot, ca, v);
      body(slot, v, k);
    }
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
    C<T>* p = acc_out + col + (int64_t)(t + TPL * m) * NN;
    const C<T> o = *p, a = ACC_LDS ? accs[c][t + TPL * m] : accr[ACC_LDS ? 0 : m];
    *p = C<T>{o.x + a.x, o.y + a.y};
  }
}

// Galaxy term of the accumulation: A = K^_g G, with K^_g the forward z
// transform of the (x, y transformed) galaxy kernel column (real part).
template <typename T, typename Sh, int W>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_zinit(const C<T>* __restrict__ ky_in, int pwz, const C<T>* __restrict__ fg,
        C<T>* __restrict__ acc_out, const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr int64_t NN = (int64_t)N * N;
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  int xt = blockIdx.x, ky = blockIdx.y;
  if constexpr (narrow_tile<T, W>()) xcd_tile(xt, ky);
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int64_t col = (int64_t)ky * N + xt * W + c;
  C<T> k[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int z = t + TPL * m;
    const int pe = (z + pwz) & (N - 1);
    const bool ok = pe <= 2 * pwz;
    const C<T> b = ky_in[col + (ok ? (int64_t)pe * NN : (int64_t)0)];
    k[m].x = ok ? b.x : (T)0;
    k[m].y = ok ? b.y : (T)0;
  }
  block_sync();
  line_fft<Sh, -1>(k, t, lines[c], tw_s, block_sync);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int64_t idx = col + (int64_t)(t + TPL * m) * NN;
    const C<T> gv = fg[idx];
    acc_out[idx] = C<T>{k[m].x * gv.x, k[m].x * gv.y};
  }
}

// ----------------------------------------------------------------------------
// Inverse x pass fused with the CIC gather.  One task per non-empty line of a
// field pair (same task words as the forward scatter).  The line is inverse
// transformed, kept in LDS, and every point whose CIC footprint reaches the
// line takes its share (real part for field a, imaginary for b):
//   scale * wy * wz * ((1 - fx) line[x0] + fx line[x0 + 1]).
// With qs > 0 (CIC, every footprint line of every point among the tasks)
// the share of the line at offset (dy, dz) in {0, 1}^2 from the point's base
// line is stored to acc[(dy + 2 dz) qs + p]: each entry is written exactly
// once, no atomics, and the reader sums the four in a fixed order.  With
// qs = 0 (TSC) the shares are added to acc[p] with atomics.
// ----------------------------------------------------------------------------
template <typename T, typename Sh, int W, bool TSC = false>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_xgather(const int32_t* __restrict__ tasks, int n_tasks, PointSet<T> ps,
          const int32_t* __restrict__ slot_fa, const int32_t* __restrict__ slot_fb,
          const C<T>* __restrict__ in, T scale, float* __restrict__ acc, int64_t qs,
          const C<T>* __restrict__ tw_g, const float* __restrict__ fscale = nullptr) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr int64_t NN = (int64_t)N * N;
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
  const int task = blockIdx.x * W + l;
  const bool active = task < n_tasks;
  C<T>* line = lines[l];
  int slot = 0, y = 0, z = 0;
  if (active) {
    const int32_t word = tasks[task];
    slot = (int)(word / NN);
    const int li = (int)(word - (int64_t)slot * NN);
    y = li % N;
    z = li / N;
  }
  C<T> v[E];
  const C<T>* src = in + (int64_t)slot * NN * N + ((int64_t)z * N + y) * N;
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = active ? src[t + TPL * m] : C<T>{0, 0};
  block_sync();
  line_fft<Sh, 1>(v, t, line, tw_s, wave_sync);
  block_sync();
#pragma unroll
  for (int m = 0; m < E; ++m) line[lpad(t + TPL * m)] = v[m];
  block_sync();
  if (active) {
    const int ym = (y - 1) & (N - 1), zm = (z - 1) & (N - 1);
    const int fa = slot_fa[slot], fb = slot_fb[slot];
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      const int f = part == 0 ? fa : fb;
      if (f < 0) continue;
      const int64_t fbase = (int64_t)f * NN;
      // a field whose kernel coefficients were divided by fscale[f] gives
      // values scaled by 1 / fscale[f]: undo it here
      const T sc = scale * (fscale ? (T)fscale[f] : (T)1);
      // the base lines whose points read this line (as in the scatter)
      constexpr int NB = TSC ? 16 : 4;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        int by, bz;
        if constexpr (TSC) {
          by = (y + (q & 3) - 2) & (N - 1);
          bz = (z + (q >> 2) - 2) & (N - 1);
        } else {
          by = (q & 1) ? ym : y;
          bz = (q & 2) ? zm : z;
        }
        const int64_t key = fbase + (int64_t)bz * N + by;
        const int s = ps.line_start[key], e = ps.line_start[key + 1];
        for (int p = s + t; p < e; p += TPL) {
          const T fy = ps.fy[p], fz = ps.fz[p], fx = ps.fx[p];
          const int x0 = ps.x0[p];
          auto val = [&](int xx) {
            const C<T> a = line[lpad(xx & (N - 1))];
            return part == 0 ? a.x : a.y;
          };
          if constexpr (TSC) {
            const T wyz = tsc_line_weight<T>(by, fy, y, N) * tsc_line_weight<T>(bz, fz, z, N);
            if (wyz == (T)0) continue;
            T wx[3];
            int lx;
            tsc_axis<T>(x0, fx, lx, wx);
            const T g = wx[0] * val(lx) + wx[1] * val(lx + 1) + wx[2] * val(lx + 2);
            atomicAdd(&acc[p], (float)(sc * wyz * g));
          } else {
            const T wy = (q & 1) ? fy : (T)1 - fy;
            const T wz = (q & 2) ? fz : (T)1 - fz;
            const float g = (float)(sc * wy * wz * (((T)1 - fx) * val(x0) + fx * val(x0 + 1)));
            if (qs > 0)
              acc[q * qs + p] = g;
            else
              atomicAdd(&acc[p], g);
          }
        }
      }
    }
  }
}

// Sum of the nc components acc[c cs + p] (the gather's per-line shares, or
// one value), in FP64 and in component order.
__device__ __forceinline__ double acc_sum(const float* __restrict__ acc, int nc, int64_t cs, int64_t p) {
  double a = (double)acc[p];
  for (int c = 1; c < nc; ++c) a += (double)acc[c * cs + p];
  return a;
}

// Pair terms of the weight gradient: grad[i] += w_j g_p, grad[j] += w_i g_p
// with g_p = acc[p] + dL/dWsum_f (acc of nc components, stride cs).  Within a
// (field, line) the pairs keep the order of the pair search, which emits each
// galaxy's pairs together, so runs of one galaxy in adjacent lanes are
// summed across the wavefront first and only the last lane of each run adds
// to the galaxy's entry.
static __global__ void k_pair_grad(const int32_t* __restrict__ pkey, const int32_t* __restrict__ pi,
                                   const int32_t* __restrict__ pj, const float* __restrict__ acc,
                                   int nc, int64_t cs, int64_t n, int64_t nn, const double* __restrict__ gws,
                                   const float* __restrict__ w, double* __restrict__ grad) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = p < n;  // every lane of the wavefront takes part in the run sums
  const int lane = (int)(threadIdx.x & 63u);
  int i = -1 - lane, j = -1 - lane;  // idle lanes: keys no galaxy has
  double gi = 0.0, gj = 0.0;
  if (act) {
    const int f = (int)(pkey[p] / nn);
    const double gval = acc_sum(acc, nc, cs, p) + gws[f];
    i = pi[p];
    j = pj[p];
    const double wi = w ? (double)w[i] : 1.0, wj = w ? (double)w[j] : 1.0;
    gi = wj * gval;
    gj = wi * gval;
  }
  SegRuns ri;
  ri.init(i);
  const double si = ri.add(gi);
  if (act && ri.tail) atomicAdd(&grad[i], si);
  SegRuns rj;
  rj.init(j);
  const double sj = rj.add(gj);
  if (act && rj.tail) atomicAdd(&grad[j], sj);
}

// galaxy term: grad[idx[p]] += acc[p] + gwg (each galaxy appears once; acc
// of nc components, stride cs)
static __global__ void k_gal_grad(const int32_t* __restrict__ idx, const float* __restrict__ acc, int nc,
                                  int64_t cs, int64_t n, const double* __restrict__ gwg,
                                  double* __restrict__ grad) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  grad[idx[p]] += acc_sum(acc, nc, cs, p) + gwg[0];
}

static __global__ void k_grad_out(const double* __restrict__ g, int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)g[i];
}

}  // namespace pgx
