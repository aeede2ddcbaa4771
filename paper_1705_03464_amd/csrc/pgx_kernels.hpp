// Device kernels of the forward correlation path (templated on precision and
// line shape).  Grid layout: a field is an N^3 complex array indexed
// [z][y][x] with x fastest.  Two real pair fields travel as the real and
// imaginary parts of one complex field ("field pair"); by linearity the
// correlation of the complex field with the real galaxy field carries the
// two real correlations in its real and imaginary parts.
#pragma once
#include "pgx_fft.hpp"
#include "pgx_weight.hpp"
#include "pgx_harm.hpp"
#include "pgx_wave.hpp"

#include <type_traits>

namespace pgx {

// ----------------------------------------------------------------------------
// Point sets: points sorted by (set, base line), where the base line of a point
// is z0*N + y0 of its lower CIC corner.  line_start[set*N*N + l] is the first
// point whose key is >= set*N*N + l (size n_sets*N*N + 1).
// ----------------------------------------------------------------------------
template <typename T> struct PointSet {
  const int32_t* line_start;
  const int32_t* x0;   // lower CIC corner along x
  const T* fx;         // CIC fractions (u - floor(u)) per axis
  const T* fy;
  const T* fz;
  const T* wt;         // point weight
};

// Number of lines along each axis of the pruned output window [-w, w].
__host__ __device__ inline int win_len(int w) { return 2 * w + 1; }

// Block size helpers
template <typename Sh, int W> struct Blk {
  static constexpr int threads = W * Sh::TPL;
};

__device__ __forceinline__ void block_sync() { __syncthreads(); }
// Synchronisation of one wavefront around its own LDS accesses.  The
// x-direction kernels give each line TPL <= 64 consecutive threads, so every
// line lies within one wavefront and the exchanges between the stages of its
// transform need no block barrier: the LDS instructions of a wavefront
// complete in issue order, and the fences keep the compiler from moving LDS
// accesses across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, typename Sh>
__device__ __forceinline__ void load_twiddles(C<T>* tw_s, const C<T>* __restrict__ tw_g) {
  for (int i = threadIdx.x; i < Sh::tw_entries(); i += blockDim.x) tw_s[i] = tw_g[i];
}

// ----------------------------------------------------------------------------
// Buffer-resource access to one slot of a field (at most 2 GiB): a 32-bit
// per-lane byte offset plus a per-element scalar offset, so the strided
// element addresses cost no vector arithmetic.  The resource's record count
// is kBufRecords; a lane offset at or beyond it (kBufOff) is out of range:
// the hardware's range check returns zero for such a load and discards such
// a store, which gives masked accesses without branches.
// ----------------------------------------------------------------------------
constexpr uint32_t kBufRecords = 0x7FFFFFF0u;
constexpr uint32_t kBufOff = 0x80000000u;
typedef unsigned int pgx_v2u __attribute__((ext_vector_type(2)));
typedef unsigned int pgx_v4u __attribute__((ext_vector_type(4)));

template <typename T> struct Buf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Buf(const void* base) {
    r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)kBufRecords,
                                          0x00020000);
  }
  __device__ __forceinline__ C<T> load(uint32_t voff, uint32_t soff) const {
    if constexpr (sizeof(T) == 4) {
      return __builtin_bit_cast(C<T>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    } else {
      return __builtin_bit_cast(C<T>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
    }
  }
  __device__ __forceinline__ void store(C<T> v, uint32_t voff, uint32_t soff) const {
    if constexpr (sizeof(T) == 4) {
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(pgx_v2u, v), r, (int)voff, (int)soff, 0);
    } else {
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(pgx_v4u, v), r, (int)voff, (int)soff, 0);
    }
  }
};

// XCD-aware order of the (x tile, y) blocks of a z pass: the hardware hands
// block b to XCD b mod 8, so XCD k gets the contiguous range of logical tiles
// [k T/8, (k+1) T/8) (T = blocks in the grid, a multiple of 8 for every grid
// side used), and the tiles one XCD works on at a time share rows, hence its
// L2 and its address-translation caches.
__device__ __forceinline__ void xcd_tile(int& xt, int& ky) {
  const int nb = (int)(gridDim.x * gridDim.y), bid = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int lt = (bid & 7) * (nb >> 3) + (bid >> 3);
  xt = lt % (int)gridDim.x;
  ky = lt / (int)gridDim.x;
}

// XCD-aware order of a three-dimensional grid (blockIdx.x fastest in the
// logical order): XCD k takes the contiguous logical range [k nb/8,
// (k+1) nb/8), so blocks with neighbouring x indices run on one XCD at the
// same time and data they share is fetched from HBM once, into that XCD's
// L2.  A grid whose block count is not a multiple of 8 keeps the hardware
// order.
__device__ __forceinline__ void xcd_block3(int& bx, int& by, int& bz) {
  const int nx = (int)gridDim.x, ny = (int)gridDim.y;
  const int nb = nx * ny * (int)gridDim.z;
  const int bid = ((int)blockIdx.z * ny + (int)blockIdx.y) * nx + (int)blockIdx.x;
  const int lt = (nb & 7) == 0 ? (bid & 7) * (nb >> 3) + (bid >> 3) : bid;
  bx = lt % nx;
  by = (lt / nx) % ny;
  bz = lt / (nx * ny);
}

// Tiles of the strided and z passes narrower than one 128-byte row (the
// eight-column tiles of 1024^3 grids): two neighbouring tiles share every row's
// 128-byte lines, so they run in XCD order, on one XCD at the same time.
template <typename T, int W> constexpr bool narrow_tile() { return W * (int)sizeof(C<T>) < 128; }

// z passes: default twiddle source (registers when they fit; the autotuner
// also tries the LDS table), and the most slots one launch may carry (their
// plane masks are staged in LDS)
constexpr bool kZTwReg = true;
constexpr int kMaxSlots = 32;

// Twiddle source: kernels whose threads transform many lines (the z passes
// loop over a batch) keep their stage twiddles in registers when a thread has
// at most 8 elements; single-tile kernels and larger shapes read the LDS table
// (one coalesced table load per block, no register pressure).
// `fft<DIR>(v, t, line)` runs the line transform with it.
struct TwNone {};
template <typename Sh, typename T, bool PREFER_REG> struct TwAuto {
  static constexpr bool REG = PREFER_REG && Sh::E <= 8;
  typename std::conditional<REG, TwReg<Sh, T>, TwNone>::type reg;
  C<T>* lds;
  __device__ __forceinline__ void init(C<T>* lds_table, const C<T>* __restrict__ tw_g, int t) {
    lds = lds_table;
    if constexpr (REG) reg.load(tw_g, t);
    else load_twiddles<T, Sh>(lds_table, tw_g);
  }
  template <int DIR> __device__ __forceinline__ void fft(C<T>* v, int t, C<T>* line) const {
    if constexpr (REG) line_fft_tw<Sh, DIR, T>(v, t, line, reg, block_sync);
    else line_fft<Sh, DIR, T>(v, t, line, lds, block_sync);
  }
};
template <typename Sh, bool PREFER_REG> constexpr int tw_lds_entries() {
  return (PREFER_REG && Sh::E <= 8) ? 1 : Sh::tw_entries();
}

// TSC mass assignment (Implementation section, "Mass assignment function"):
// the point spreads over its nearest node c and both neighbours
// on each axis, weights 3/4 - d^2 (c) and (1/2 -+ d)^2 / 2 (c - 1, c + 1),
// d = u - c in [-1/2, 1/2].  From the CIC corner x0 and fraction f of the
// point set: c = x0, d = f when f <= 1/2, else c = x0 + 1, d = f - 1 (a
// point at exactly one half takes the lower node; both give the same
// weights).
template <typename T>
__device__ __forceinline__ void tsc_axis(int x0, T f, int& lo, T* w) {
  const bool up = f > (T)0.5;
  const T d = up ? f - (T)1 : f;
  lo = x0 + (up ? 1 : 0) - 1;
  w[0] = (T)0.5 * ((T)0.5 - d) * ((T)0.5 - d);
  w[1] = (T)0.75 - d * d;
  w[2] = (T)0.5 * ((T)0.5 + d) * ((T)0.5 + d);
}

// TSC weight along one axis of the point with CIC corner a0 and fraction f
// for grid index a (0 where a is not one of the three nodes of the point).
template <typename T>
__device__ __forceinline__ T tsc_line_weight(int a0, T f, int a, int N) {
  const bool up = f > (T)0.5;
  const T d = up ? f - (T)1 : f;
  const int j = ((a - a0 - (up ? 1 : 0) + N + 1) & (N - 1)) - 1;  // node - nearest node
  return j == 0 ? (T)0.75 - d * d
       : j == -1 ? (T)0.5 * ((T)0.5 - d) * ((T)0.5 - d)
       : j == 1 ? (T)0.5 * ((T)0.5 + d) * ((T)0.5 + d) : (T)0;
}

// ----------------------------------------------------------------------------
// (A) x pass with the CIC scatter fused in.  One task per non-empty line of a
// field pair.  The line is built in LDS from the points of the four base lines
// whose CIC footprint reaches it (LDS atomics), transformed along x and
// written once.  task word = slot * N*N + line (line = z*N + y).  When a line
// is one or more whole wavefronts, each wavefront first sums the
// contributions of adjacent points on the same x node (clustered catalogues
// put many points on one node, and same-address LDS atomics serialise), and
// only the last point of each run adds to the line.
// ----------------------------------------------------------------------------
template <typename T, typename Sh, int W, bool TSC = false>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_xscatter(const int32_t* __restrict__ tasks, int n_tasks, PointSet<T> ps,
           const int32_t* __restrict__ slot_fa, const int32_t* __restrict__ slot_fb,
           C<T>* __restrict__ out, const C<T>* __restrict__ tw_g,
           const float* __restrict__ fscale = nullptr) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr int64_t NN = (int64_t)N * N;
  constexpr bool kRuns = TPL % 64 == 0;
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
  const int task = blockIdx.x * W + l;
  const bool active = task < n_tasks;
  C<T>* line = lines[l];
#pragma unroll
  for (int m = 0; m < E; ++m) line[lpad(t + TPL * m)] = C<T>{0, 0};
  int slot = 0, y = 0, z = 0;
  if (active) {
    const int32_t word = tasks[task];
    slot = (int)(word / NN);
    const int li = (int)(word - (int64_t)slot * NN);
    y = li % N;
    z = li / N;
  }
  block_sync();
  if (active) {
    const int ym = (y - 1) & (N - 1), zm = (z - 1) & (N - 1);
    const int fa = slot_fa[slot], fb = slot_fb[slot];
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      const int f = part == 0 ? fa : fb;
      if (f < 0) continue;
      const int64_t fbase = (int64_t)f * NN;
      const T sc = fscale ? (T)fscale[f] : (T)1;
      // base lines (CIC corner rows) whose points reach this line: (y, z) and
      // their lower neighbours for CIC; y - 2 .. y + 1 by z - 2 .. z + 1 for
      // TSC, whose footprint of three rows starts one row below or at the
      // corner row
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
        // every lane of a wavefront takes the same trips (one line per wavefront)
        for (int b0 = s; b0 < e; b0 += TPL) {
          const int p = b0 + t;
          const bool ok = p < e;
          T lo = (T)0, mid = (T)0, hi = (T)0;
          int x0 = -1 - (int)(threadIdx.x & 63u);  // idle lanes: keys no node has
          if (ok) {
            const T fy = ps.fy[p], fz = ps.fz[p], fx = ps.fx[p];
            x0 = ps.x0[p];
            if constexpr (TSC) {
              const T w = ps.wt[p] * sc * tsc_line_weight<T>(by, fy, y, N) *
                          tsc_line_weight<T>(bz, fz, z, N);
              // nodes c - 1, c, c + 1 of the nearest node c; the run key is c
              T wx[3];
              int lx;
              tsc_axis<T>(x0, fx, lx, wx);
              x0 = (lx + 1) & (N - 1);
              lo = w * wx[0];
              mid = w * wx[1];
              hi = w * wx[2];
            } else {
              const T wy = (q & 1) ? fy : (T)1 - fy;
              const T wz = (q & 2) ? fz : (T)1 - fz;
              const T w = ps.wt[p] * sc * wy * wz;
              lo = w * ((T)1 - fx);
              hi = w * fx;
            }
          }
          bool issue = ok;
          if constexpr (kRuns) {
            SegRuns r;
            r.init(x0);
            lo = r.add(lo);
            if constexpr (TSC) mid = r.add(mid);
            hi = r.add(hi);
            issue = ok && r.tail;
          }
          if (issue) {
            auto at = [&](int xx) -> T* {
              C<T>* c = &line[lpad(xx & (N - 1))];
              return part == 0 ? &c->x : &c->y;
            };
            if constexpr (TSC) {
              atomicAdd(at(x0 - 1), lo);
              atomicAdd(at(x0), mid);
              atomicAdd(at(x0 + 1), hi);
            } else {
              atomicAdd(at(x0), lo);
              atomicAdd(at(x0 + 1), hi);
            }
          }
        }
      }
    }
  }
  block_sync();
  C<T> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = line[lpad(t + TPL * m)];
  block_sync();
  line_fft<Sh, -1>(v, t, line, tw_s, wave_sync);
  if (active) {
    C<T>* o = out + (int64_t)slot * NN * N + ((int64_t)z * N + y) * N;
#pragma unroll
    for (int m = 0; m < E; ++m) o[t + TPL * m] = v[m];
  }
}

// ----------------------------------------------------------------------------
// (B) strided pass: lines along an axis with element stride `es` (N for y,
// N*N for z) over tiles of W adjacent x positions.  Tile (xt, a): column base
// a*A + xt*W.  Input modes:
//   IN_DENSE   every element read;
//   IN_FLAGS   element e counts only when lflag[a*N + e] != 0, and the whole
//              tile is skipped when pflag[a] == 0 (a field written sparsely by
//              the x pass; its untouched elements hold stale data);
//   IN_WINDOW  only elements e with (e + pw) mod N <= 2 pw exist, stored at
//              position (e + pw) mod N of a window-sized input line.
// Output modes:
//   OUT_DENSE  every element written;
//   OUT_WINDOW only outputs e' with (e' + pw) mod N <= 2 pw, at position
//              (e' + pw) mod N of a window-sized output line;
//   OUT_FLAGS  only outputs whose line flag lflag[a*N + e'] is set (the tile is
//              skipped when pflag[a] == 0).
// Batched over blockIdx.z with per-slot strides; flags per field pair slot_fp.
// ----------------------------------------------------------------------------
enum { IN_DENSE = 0, IN_FLAGS = 1, IN_WINDOW = 2 };
enum { OUT_DENSE = 0, OUT_WINDOW = 1, OUT_FLAGS = 2 };

template <typename T, typename Sh, int W, int DIR, int IN, int OUT>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_strided(const C<T>* in, C<T>* out, int64_t in_slot, int64_t out_slot,
          int64_t in_A, int64_t out_A, int64_t in_es, int64_t out_es, int pw,
          const uint8_t* __restrict__ lflag, const uint8_t* __restrict__ pflag,
          int64_t flag_slot, const int32_t* __restrict__ slot_fp, const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  __shared__ C<T> tw_s[tw_lds_entries<Sh, false>()];
  __shared__ C<T> lines[W][LL];
  int xt = blockIdx.x, a = blockIdx.y, slot = blockIdx.z;
  if constexpr (narrow_tile<T, W>()) xcd_block3(xt, a, slot);
  const uint8_t* lf = nullptr;
  if constexpr (IN == IN_FLAGS || OUT == OUT_FLAGS) {
    const int64_t fp = slot_fp[slot];
    if (pflag[fp * N + a] == 0) return;  // whole plane empty
    lf = lflag + fp * flag_slot + (int64_t)a * N;
  }
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  TwAuto<Sh, T, false> twa;
  twa.init(tw_s, tw_g, t);
  // buffer path: tile base in a scalar resource, per-lane 32-bit offset,
  // per-element scalar offset (fields up to 2 GiB per slot)
  constexpr bool BUF = (int64_t)N * N * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  const C<T>* tin = in + slot * in_slot + a * in_A + xt * W;
  C<T> v[E];
  uint8_t fl[E];
  if constexpr (IN == IN_FLAGS || OUT == OUT_FLAGS) {
#pragma unroll
    for (int m = 0; m < E; ++m) fl[m] = lf[t + TPL * m];
  }
  if constexpr (BUF) {
    const Buf<T> bi(tin);
    const uint32_t vo = (uint32_t)((c + (int64_t)t * in_es) * (int64_t)sizeof(C<T>));
    const uint32_t st = (uint32_t)((int64_t)TPL * in_es * (int64_t)sizeof(C<T>));
#pragma unroll
    for (int m = 0; m < E; ++m) {
      if constexpr (IN == IN_FLAGS) {
        // absent lines read the tile's first element (valid, cached), then zero
        const C<T> x = bi.load(fl[m] ? vo + (uint32_t)m * st : 0u, 0u);
        v[m].x = fl[m] ? x.x : (T)0;
        v[m].y = fl[m] ? x.y : (T)0;
      } else if constexpr (IN == IN_WINDOW) {
        const int e = t + TPL * m;
        const int pe = (e + pw) & (N - 1);
        const bool ok = pe <= 2 * pw;
        const uint32_t o = (uint32_t)((c + (int64_t)pe * in_es) * (int64_t)sizeof(C<T>));
        const C<T> x = bi.load(ok ? o : 0u, 0u);
        v[m].x = ok ? x.x : (T)0;
        v[m].y = ok ? x.y : (T)0;
      } else {
        v[m] = bi.load(vo, (uint32_t)m * st);
      }
    }
  } else {
    const C<T>* src = tin + c;
    if constexpr (IN == IN_FLAGS || IN == IN_WINDOW) {
      // branch-free predicated loads: an absent element reads the tile's first
      // input element (a valid, cached address) and is replaced by zero
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int e = t + TPL * m;
        bool ok;
        int64_t off;
        if constexpr (IN == IN_FLAGS) {
          ok = fl[m] != 0;
          off = (int64_t)e * in_es;
        } else {
          const int pe = (e + pw) & (N - 1);
          ok = pe <= 2 * pw;
          off = (int64_t)pe * in_es;
        }
        const C<T> x = src[ok ? off : (int64_t)0];
        v[m].x = ok ? x.x : (T)0;
        v[m].y = ok ? x.y : (T)0;
      }
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = src[(int64_t)(t + TPL * m) * in_es];
    }
  }
  block_sync();
  twa.template fft<DIR>(v, t, lines[c]);
  C<T>* tout = out + slot * out_slot + a * out_A + xt * W;
  if constexpr (BUF) {
    const Buf<T> bo(tout);
    const uint32_t st = (uint32_t)((int64_t)TPL * out_es * (int64_t)sizeof(C<T>));
    const uint32_t vo = (uint32_t)((c + (int64_t)t * out_es) * (int64_t)sizeof(C<T>));
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + TPL * m;
      if constexpr (OUT == OUT_WINDOW) {
        const int pe = (e + pw) & (N - 1);
        if (pe <= 2 * pw)
          bo.store(v[m], (uint32_t)((c + (int64_t)pe * out_es) * (int64_t)sizeof(C<T>)), 0u);
      } else if constexpr (OUT == OUT_FLAGS) {
        if (fl[m]) bo.store(v[m], vo, (uint32_t)m * st);
      } else {
        bo.store(v[m], vo, (uint32_t)m * st);
      }
    }
  } else {
    C<T>* dst = tout + c;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int e = t + TPL * m;
      if constexpr (OUT == OUT_WINDOW) {
        const int pe = (e + pw) & (N - 1);
        if (pe <= 2 * pw) dst[(int64_t)pe * out_es] = v[m];
      } else if constexpr (OUT == OUT_FLAGS) {
        if (fl[m]) dst[(int64_t)e * out_es] = v[m];
      } else {
        dst[(int64_t)e * out_es] = v[m];
      }
    }
  }
}

// ----------------------------------------------------------------------------
// (C) z pass with the cross-power product fused in.  Tile (xt, ky); for each
// slot of the batch: forward transform along z, multiply by conj(Fg), inverse
// transform along z, store only the pruned window of z' (layout
// [pz][ky][kx], pz = (z' + pw) mod N).  Fg is read once per tile per batch.
// GAL mode (galaxy field): after the forward transform the k = 0 mode is set
// to zero, the spectrum is stored to `fg_out`, and the product is |Fg|^2.
// STORE mode also writes each pair-field spectrum (after the forward z
// transform) to `spec` at its field-pair index, for the adjoint.
// ----------------------------------------------------------------------------
template <typename T, typename Sh, int W, bool GAL, bool STORE = false, bool TWREG = kZTwReg>
static __global__ void __launch_bounds__(W * Sh::TPL, GAL && !TWREG && Sh::E <= 8 ? 8 : 1)
k_zcross(const C<T>* in, int64_t in_slot, const uint8_t* __restrict__ pflag,
         const int32_t* __restrict__ slot_fp, int n_slots, const C<T>* __restrict__ fg,
         C<T>* __restrict__ fg_out, C<T>* __restrict__ out, int64_t out_slot, int pw,
         const C<T>* __restrict__ tw_g, C<T>* __restrict__ spec = nullptr) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  constexpr int64_t NN = (int64_t)N * N;
  // slot pipeline when a thread has room for a second set of columns
  constexpr bool PIPE = !GAL && E <= 8;
  __shared__ C<T> tw_s[tw_lds_entries<Sh, TWREG>()];
  __shared__ C<T> lines[W][LL];
  __shared__ uint32_t pmask[GAL ? 1 : kMaxSlots][TPL];
  int xt = blockIdx.x, ky = blockIdx.y;
  if constexpr (narrow_tile<T, W>()) xcd_tile(xt, ky);
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  TwAuto<Sh, T, TWREG> twa;
  twa.init(tw_s, tw_g, t);
  if constexpr (!GAL) {
    // plane masks of the batch: bit m of pmask[s][t] = plane t + TPL m of
    // slot s holds data
    for (int i = threadIdx.x; i < n_slots * TPL; i += W * TPL) {
      const int s = i / TPL, tt = i - s * TPL;
      const uint8_t* pf = pflag + (int64_t)slot_fp[s] * N + tt;
      uint32_t mk = 0;
#pragma unroll
      for (int m = 0; m < E; ++m) mk |= (uint32_t)(pf[TPL * m] != 0) << m;
      pmask[s][tt] = mk;
    }
    block_sync();
  }
  const int64_t col = (int64_t)ky * N + xt * W + c;
  // buffer path (fields up to 2 GiB per slot): tile base in a scalar resource,
  // per-lane offset of the column, per-element scalar offset of the z plane
  constexpr bool BUF = NN * N * (int64_t)sizeof(C<T>) < ((int64_t)1 << 31);
  constexpr uint32_t CB = sizeof(C<T>);
  constexpr uint32_t ZST = BUF ? (uint32_t)(TPL * NN * CB) : 0u;  // TPL planes
  const int64_t tile = (int64_t)ky * N + xt * W;
  const uint32_t vo = (uint32_t)((c + (int64_t)t * NN) * CB);
  const int pw2 = 2 * pw + 1;
  // columns of one slot; absent planes are zero (buffer path: out-of-range
  // offset; pointer path: the tile's first element is read and zeroed when
  // the columns are taken)
  auto load_cols = [&](int slot, bool take, C<T>* dst) {
    if constexpr (GAL && BUF) {
      const Buf<T> bi(in + slot * in_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) dst[m] = bi.load(vo, (uint32_t)m * ZST);
    } else if constexpr (GAL) {
      const C<T>* src = in + slot * in_slot + col;
#pragma unroll
      for (int m = 0; m < E; ++m) dst[m] = src[(int64_t)(t + TPL * m) * NN];
    } else if constexpr (BUF) {
      const uint32_t mk = take ? pmask[slot][t] : 0u;
      const Buf<T> bi(in + slot * in_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m)
        dst[m] = bi.load((mk >> m) & 1u ? vo + (uint32_t)m * ZST : kBufOff, 0u);
    } else {
      const uint32_t mk = take ? pmask[slot][t] : 0u;
      const C<T>* src = in + slot * in_slot + col;
#pragma unroll
      for (int m = 0; m < E; ++m) dst[m] = src[(mk >> m) & 1u ? (int64_t)(t + TPL * m) * NN : 0];
    }
  };
  auto take_cols = [&](int slot, const C<T>* cur, C<T>* v) {
    if constexpr (GAL || BUF) {
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
  C<T> ca[E], cb[PIPE ? E : 1], g[E];
  load_cols(0, true, ca);
  // G after the first columns: on entry to the loop, as on every later trip
  // (where the previous slot's stores follow them), eight younger memory
  // operations follow the columns, so the wait for them is the same
  if constexpr (!GAL) {
    if constexpr (BUF) {
      const Buf<T> bg(fg + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) g[m] = bg.load(vo, (uint32_t)m * ZST);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) g[m] = fg[col + (int64_t)(t + TPL * m) * NN];
    }
  }
  auto body = [&](int slot, C<T>* v) {
    block_sync();
    twa.template fft<-1>(v, t, lines[c]);
    if constexpr (GAL) {
      if (col == 0 && t == 0) v[0] = C<T>{0, 0};  // kz = 0 of the (0,0) column
      if constexpr (BUF) {
        const Buf<T> bs(fg_out + tile);
#pragma unroll
        for (int m = 0; m < E; ++m) bs.store(v[m], vo, (uint32_t)m * ZST);
      } else {
#pragma unroll
        for (int m = 0; m < E; ++m) fg_out[col + (int64_t)(t + TPL * m) * NN] = v[m];
      }
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = C<T>{v[m].x * v[m].x + v[m].y * v[m].y, (T)0};
    } else {
      if constexpr (STORE) {
        // keep the pair-field spectrum (field pair slot_fp[slot], dense N^3)
        // for the adjoint
        C<T>* sp = spec + (int64_t)slot_fp[slot] * (NN * N);
        if constexpr (BUF) {
          const Buf<T> bs(sp + tile);
#pragma unroll
          for (int m = 0; m < E; ++m) bs.store(v[m], vo, (uint32_t)m * ZST);
        } else {
#pragma unroll
          for (int m = 0; m < E; ++m) sp[col + (int64_t)(t + TPL * m) * NN] = v[m];
        }
      }
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cmulc(v[m], g[m]);
    }
    block_sync();
    twa.template fft<1>(v, t, lines[c]);
    if constexpr (BUF) {
      // every lane issues its stores; those outside the window are discarded
      const Buf<T> bo(out + slot * out_slot + tile);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int pz = (t + TPL * m + pw) & (N - 1);
        bo.store(v[m], pz < pw2 ? (uint32_t)((c + (int64_t)pz * NN) * CB) : kBufOff, 0u);
      }
    } else {
      C<T>* dst = out + slot * out_slot + col;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int pz = (t + TPL * m + pw) & (N - 1);
        if (pz < pw2) dst[(int64_t)pz * NN] = v[m];
      }
    }
  };
  if constexpr (PIPE) {
    // the next slot's columns go into the idle register set at the top of
    // each trip, before the current ones are waited for: they are in flight
    // during both transforms (the last trip issues only out-of-range loads)
    auto trip = [&](int slot, const C<T>* cur, C<T>* nxt) {
      const bool more = slot + 1 < n_slots;
      load_cols(more ? slot + 1 : slot, more, nxt);
      // keep the arithmetic on the current columns (and its wait) after the
      // loads are issued
      __builtin_amdgcn_sched_barrier(0);
      C<T> v[E];
      take_cols(slot, cur, v);
      body(slot, v);
    };
    // two trips per loop pass, so the register sets keep their roles across
    // the back edge (no copies); an odd last slot runs after the loop
    int slot = 0;
    for (; slot + 1 < n_slots; slot += 2) {
      trip(slot, ca, cb);
      trip(slot + 1, cb, ca);
    }
    if (slot < n_slots) trip(slot, ca, cb);
  } else {
    for (int slot = 0; slot < n_slots; ++slot) {
      if (slot > 0) load_cols(slot, true, ca);
      C<T> v[E];
      take_cols(slot, ca, v);
      body(slot, v);
    }
  }
}

// ----------------------------------------------------------------------------
// Output-bin classification of a lattice offset (i', j', k') (signed).  All
// modes depend only on |k'| and on i'^2 + j'^2 (+ k'^2), so a displacement
// and its negative share a bin.
// ----------------------------------------------------------------------------
struct BinMap {
  int mode;             // 0 shell, 1 r_mu, 2 rp_pi, 3 Gaussian-sigmoid weight
  int n2;               // number of second-axis bins (1 for shell)
  const int16_t* lut1;  // shell/r_mu: indexed by m = i'^2+j'^2+k'^2 ; rp_pi: by i'^2+j'^2
  int lut1_n;
  const int16_t* lut2;  // rp_pi: indexed by k'^2
  int lut2_n;
  const double* mu2;    // r_mu: squared mu edges (n2 + 1)
  double g[4];          // Gaussian-sigmoid: gsw_value parameters
  double rcut2, rmax2;  // Gaussian-sigmoid: cuts as squared lattice lengths
};

__device__ __forceinline__ int classify_bin(const BinMap& bm, int i, int j, int k) {
  const int xy = i * i + j * j, kk = k * k;
  if (bm.mode == 3) return ((double)xy >= bm.rcut2 && (double)(xy + kk) <= bm.rmax2) ? 0 : -1;
  if (bm.mode == 2) {
    if (xy >= bm.lut1_n || kk >= bm.lut2_n) return -1;
    const int b1 = bm.lut1[xy], b2 = bm.lut2[kk];
    if (b1 < 0 || b2 < 0) return -1;
    return b1 * bm.n2 + b2;
  }
  const int m = xy + kk;
  if (m >= bm.lut1_n) return -1;
  const int b1 = bm.lut1[m];
  if (b1 < 0) return -1;
  if (bm.mode == 0) return b1;
  const double md = (double)m, kd = (double)kk;
  if (kd < bm.mu2[0] * md || kd > bm.mu2[bm.n2] * md) return -1;
  int kb = 0;
  for (int e = 1; e < bm.n2; ++e) kb += (kd >= bm.mu2[e] * md) ? 1 : 0;
  return b1 * bm.n2 + kb;
}

// weight of an offset classified into a bin: 1 for the indicator bins, the
// Gaussian-sigmoid value in mode 3
__device__ __forceinline__ double bin_weight(const BinMap& bm, int i, int j, int k) {
  return bm.mode == 3 ? gsw_value(i * i + j * j, k * k, bm.g) : 1.0;
}

// ----------------------------------------------------------------------------
// (E) last inverse pass along x over the pruned window lines (pz, py), with
// the bin reduction fused: FP64 bin sums in LDS, one partial row per block:
// part[slot][block][2][R] (real part -> field a, imaginary -> field b).
// ----------------------------------------------------------------------------
template <typename T, typename Sh, int W, int RMAX>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_xinv_bins(const C<T>* __restrict__ in, int64_t in_slot, int pwx, int pwy, int pwz, BinMap bm,
            int R, double* __restrict__ part, const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  __shared__ double acc[2 * RMAX];
  load_twiddles<T, Sh>(tw_s, tw_g);
  for (int i = threadIdx.x; i < 2 * R; i += blockDim.x) acc[i] = 0.0;
  const int slot = blockIdx.z;
  const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
  const int ny = win_len(pwy), nz = win_len(pwz);
  const int task = blockIdx.x * W + l;
  const bool active = task < ny * nz;
  const int py = active ? task % ny : 0, pz = active ? task / ny : 0;
  C<T> v[E];
  const C<T>* src = in + slot * in_slot + (int64_t)task * N;
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = active ? src[t + TPL * m] : C<T>{0, 0};
  block_sync();
  line_fft<Sh, 1>(v, t, lines[l], tw_s, wave_sync);
  if (active) {
    const int jj = py - pwy, kk = pz - pwz;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int px = (t + TPL * m + pwx) & (N - 1);
      if (px <= 2 * pwx) {
        const int b = classify_bin(bm, px - pwx, jj, kk);
        if (b >= 0) {
          const double wb = bin_weight(bm, px - pwx, jj, kk);
          atomicAdd(&acc[b], wb * (double)v[m].x);
          atomicAdd(&acc[R + b], wb * (double)v[m].y);
        }
      }
    }
  }
  block_sync();
  double* dst = part + ((int64_t)slot * gridDim.x + blockIdx.x) * 2 * R;
  for (int i = threadIdx.x; i < 2 * R; i += blockDim.x) dst[i] = acc[i];
}

// ----------------------------------------------------------------------------
// Plain path pieces (one field per complex grid, imaginary part zero)
// ----------------------------------------------------------------------------
// contiguous x pass over all lines of a dense field, in place
template <typename T, typename Sh, int W, int DIR>
static __global__ void __launch_bounds__(W * Sh::TPL)
k_xdense(C<T>* data, const C<T>* __restrict__ tw_g) {
  constexpr int N = Sh::n, E = Sh::E, TPL = Sh::TPL, LL = lds_line_elems<N>();
  __shared__ C<T> tw_s[Sh::tw_entries()];
  __shared__ C<T> lines[W][LL];
  load_twiddles<T, Sh>(tw_s, tw_g);
  const int t = threadIdx.x % TPL, l = threadIdx.x / TPL;
  C<T>* p = data + ((int64_t)blockIdx.x * W + l) * N;
  C<T> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = p[t + TPL * m];
  block_sync();
  line_fft<Sh, DIR>(v, t, lines[l], tw_s, wave_sync);
#pragma unroll
  for (int m = 0; m < E; ++m) p[t + TPL * m] = v[m];
}

}  // namespace pgx
