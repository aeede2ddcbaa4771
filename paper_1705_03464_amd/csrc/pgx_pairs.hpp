// Close-pair search on a cell list, integer pair-bin keys and CIC point data.
//
// The paper keeps every pair closer than the maximum pair separation (a
// close triplet gives three pairs) and places a pair at its midpoint
// (Implementation section, pair catalogue; Methodology, equation
// delta_pi_x).  Keys are decided with FP64 comparisons of squared
// separations against squared edges, evaluated with the same operation order
// as the reference definition and without fused multiply-add, so they are
// reproducible bit for bit:
//   d = x_j - x_i (i < j by catalogue index), folded once into [-L/2, L/2)
//   xy = dx*dx + dy*dy ; zz = dz*dz ; s2 = xy + zz
//   s/|mu| mode:  t1[b] <= s2 < t1[b+1] ;  k = largest with zz >= mu2[k]*s2,
//                 kept iff mu2[0]*s2 <= zz <= mu2[n2]*s2 (top edge closed)
//   r_p/|pi| mode: s2 < dmax^2 ; t1[b] <= xy < t1[b+1] ; t2[k] <= zz < t2[k+1]
//   key = b * n2 + k
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pgx {

struct PairCfg {
  double L, halfL, gscale;  // gscale = N / L
  double side;              // cell side (>= maximum pair separation)
  int nc, N, mode, n1, n2;
  int step1;                // largest power of two below n1 (binary search over t1)
  const double* t1;         // squared first-axis edges (n1 + 1)
  const double* t2;         // squared second-axis edges (mu^2 or pi^2) (n2 + 1)
  double dmax2;
};

__device__ __forceinline__ double fold(double d, double L, double h) {
#pragma clang fp contract(off)
  return d >= h ? d - L : (d < -h ? d + L : d);
}

// returns key >= 0 or -1
__device__ __forceinline__ int pair_key(const PairCfg& c, double dx, double dy, double dz) {
#pragma clang fp contract(off)
  const double xy = dx * dx + dy * dy;
  const double zz = dz * dz;
  const double s2 = xy + zz;
  if (c.mode == 0) {
    if (s2 < c.t1[0] || s2 >= c.t1[c.n1]) return -1;
    if (zz < c.t2[0] * s2 || zz > c.t2[c.n2] * s2) return -1;
    // the number of inner edges with s2 >= t1[e] (t1 ascending): binary search
    int b = 0;
    for (int step = c.step1; step > 0; step >>= 1)
      if (b + step < c.n1 && s2 >= c.t1[b + step]) b += step;
    int k = 0;
    for (int e = 1; e < c.n2; ++e) k += (zz >= c.t2[e] * s2) ? 1 : 0;
    return b * c.n2 + k;
  }
  if (s2 >= c.dmax2) return -1;
  if (xy < c.t1[0] || xy >= c.t1[c.n1]) return -1;
  if (zz < c.t2[0] || zz >= c.t2[c.n2]) return -1;
  int b = 0;
  for (int e = 1; e < c.n1; ++e) b += (xy >= c.t1[e]) ? 1 : 0;
  int k = 0;
  for (int e = 1; e < c.n2; ++e) k += (zz >= c.t2[e]) ? 1 : 0;
  return b * c.n2 + k;
}

// CIC data of a position u = x * (N / L): lower node and fraction
__device__ __forceinline__ void cic_of(double x, double gscale, int N, int& i0, double& f) {
#pragma clang fp contract(off)
  const double u = x * gscale;
  const double fl = floor(u);
  f = u - fl;
  i0 = ((int)fl) & (N - 1);
}

// validation: bit 1 non-finite position, bit 2 outside [0, L), bit 4 bad weight
static __global__ void k_validate(const double* __restrict__ x, const double* __restrict__ y,
                           const double* __restrict__ z, const float* __restrict__ w, int64_t n,
                           double L, int* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int e = 0;
  const double a = x[i], b = y[i], c = z[i];
  if (!isfinite(a) || !isfinite(b) || !isfinite(c)) e |= 1;
  else if (a < 0.0 || a >= L || b < 0.0 || b >= L || c < 0.0 || c >= L) e |= 2;
  if (w) {
    const float v = w[i];
    if (!isfinite(v) || v < 0.0f) e |= 4;
  }
  if (e) atomicOr(err, e);
}

static __global__ void k_cell_keys(const double* __restrict__ x, const double* __restrict__ y,
                            const double* __restrict__ z, int64_t n, double side, int nc,
                            int32_t* __restrict__ key, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int cx = min((int)(x[i] / side), nc - 1);
  int cy = min((int)(y[i] / side), nc - 1);
  int cz = min((int)(z[i] / side), nc - 1);
  key[i] = (cx * nc + cy) * nc + cz;
  idx[i] = (int32_t)i;
}

static __global__ void k_gather_pos(const int32_t* __restrict__ perm, const double* __restrict__ x,
                             const double* __restrict__ y, const double* __restrict__ z, int64_t n,
                             double* __restrict__ px, double* __restrict__ py, double* __restrict__ pz) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int i = perm[p];
  px[p] = x[i];
  py[p] = y[i];
  pz[p] = z[i];
}

// Counts of sorted keys (n < 2^31): only the ends of each run of equal keys
// touch the histogram (the first adds -p, the last p + 1), so equal keys do
// not contend for one address.
static __global__ void k_run_counts(const int32_t* __restrict__ key, int64_t n, int32_t* __restrict__ h) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t k = key[p];
  const bool first = p == 0 || key[p - 1] != k;
  const bool last = p == n - 1 || key[p + 1] != k;
  if (first && last)
    atomicAdd(&h[k], 1);
  else if (first)
    atomicAdd(&h[k], -(int32_t)p);
  else if (last)
    atomicAdd(&h[k], (int32_t)(p + 1));
}

// One wavefront per galaxy p (in cell order); its candidates are the galaxies
// of the 27 neighbour cells with a larger cell-order index, taken as one
// list: neighbour cells in order o = 0..26, each cell's candidates in cell
// order.  The lanes test 64 consecutive candidates of that list at a time;
// each kept pair gets its place from a ballot of the lanes (the kept lanes
// below it), so a galaxy's pairs are written contiguously and in list order
// (coalesced stores, and the same order as a serial loop over the list).
// COUNT: cnt[p] = number of kept pairs.  EMIT: pairs written at off[p] + rank:
// the sort key (field, base line of the midpoint) and the catalogue indices
// i < j only; the midpoint's CIC corner and fractions are recomputed after
// the sort by k_pair_cic, with coalesced stores.
constexpr int kPairWaves = 4;  // wavefronts per block
template <bool EMIT, typename T>
static __global__ void __launch_bounds__(64 * kPairWaves)
k_pairs(PairCfg c, const double* __restrict__ px, const double* __restrict__ py,
        const double* __restrict__ pz, const int32_t* __restrict__ perm,
        const int32_t* __restrict__ cell_of, const int32_t* __restrict__ cell_start, int64_t n,
        int64_t* __restrict__ cnt_off, int32_t* __restrict__ skey, int32_t* __restrict__ oi,
        int32_t* __restrict__ oj) {
#pragma clang fp contract(off)
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t NN = (int64_t)c.N * c.N;
  const int nc = c.nc;
  for (int64_t p = (int64_t)blockIdx.x * kPairWaves + (threadIdx.x >> 6); p < n;
       p += (int64_t)gridDim.x * kPairWaves) {
    const int cell = cell_of[p];
    const int cx = cell / (nc * nc), cy = (cell / nc) % nc, cz = cell % nc;
    // lane o < 27: candidates of neighbour cell o start at qs and number cn
    // (each pair once, by its lower cell-order index: past p)
    int qs = 0, cn = 0;
    if (lane < 27) {
      const int nx = (cx + lane / 9 - 1 + nc) % nc;
      const int ny = (cy + (lane / 3) % 3 - 1 + nc) % nc;
      const int nz = (cz + lane % 3 - 1 + nc) % nc;
      const int nb = (nx * nc + ny) * nc + nz;
      const int s = cell_start[nb], e = cell_start[nb + 1];
      qs = s > (int)p ? s : (int)p + 1;
      cn = e > qs ? e - qs : 0;
    }
    // exclusive prefix of the counts over the 27 cells
    int inc = cn;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
      const int u = __shfl_up(inc, d, 64);
      if (lane >= d) inc += u;
    }
    const int pre = inc - cn;
    const int total = __shfl(inc, 26, 64);
    const double ax = px[p], ay = py[p], az = pz[p];
    const int ia = perm[p];
    int64_t w = EMIT ? cnt_off[p] : 0;
    for (int base = 0; base < total; base += 64) {
      const int idx = base + lane;
      // the neighbour cell of list entry idx: the last o with pre[o] <= idx
      // (pre is non-decreasing in o: binary search over lanes 0..26)
      int o = 0;
#pragma unroll
      for (int step = 16; step > 0; step >>= 1) {
        const int k = o + step;
        const int pk = __shfl(pre, k < 27 ? k : 26, 64);
        o = (k < 27 && pk <= idx) ? k : o;
      }
      const int q = __shfl(qs, o, 64) + (idx - __shfl(pre, o, 64));
      int key = -1;
      int32_t okey = 0, oa = 0, ob = 0;
      if (idx < total) {
        const int ib_ = perm[q];
        const double bx = px[q], by = py[q], bz = pz[q];
        // i < j by catalogue index, d = x_j - x_i
        const bool fwd = ia < ib_;
        const double xi = fwd ? ax : bx, yi = fwd ? ay : by, zi = fwd ? az : bz;
        const double dx = fold((fwd ? bx : ax) - xi, c.L, c.halfL);
        const double dy = fold((fwd ? by : ay) - yi, c.L, c.halfL);
        const double dz = fold((fwd ? bz : az) - zi, c.L, c.halfL);
        key = pair_key(c, dx, dy, dz);
        if (EMIT && key >= 0) {
          double my = yi + 0.5 * dy, mz = zi + 0.5 * dz;
          my = my >= c.L ? my - c.L : (my < 0.0 ? my + c.L : my);
          mz = mz >= c.L ? mz - c.L : (mz < 0.0 ? mz + c.L : mz);
          int y0, z0;
          double fy, fz;
          cic_of(my, c.gscale, c.N, y0, fy);
          cic_of(mz, c.gscale, c.N, z0, fz);
          okey = (int32_t)((int64_t)key * NN + (int64_t)z0 * c.N + y0);
          oa = fwd ? ia : ib_;
          ob = fwd ? ib_ : ia;
        }
      }
      const uint64_t kept = __ballot(key >= 0);
      if (EMIT && key >= 0) {
        const int64_t at = w + __popcll(kept & below);
        skey[at] = okey;
        oi[at] = oa;
        oj[at] = ob;
      }
      w += __popcll(kept);
    }
    if (!EMIT && lane == 0) cnt_off[p] = w;
  }
}

// Each pair in sorted order: its members (i < j), gathered from the emission
// order through the sort's permutation and stored, and the CIC corner and
// fractions of its midpoint from their catalogue positions: the same FP64
// operations as the pair search (d = x_j - x_i folded once into [-L/2, L/2),
// m = x_i + d / 2 wrapped into [0, L)), so the result matches the key the
// search gave.
template <typename T>
static __global__ void k_pair_cic(PairCfg c, const double* __restrict__ x, const double* __restrict__ y,
                                  const double* __restrict__ z, const int32_t* __restrict__ perm,
                                  const int32_t* __restrict__ ui, const int32_t* __restrict__ uj, int64_t P,
                                  int32_t* __restrict__ opi, int32_t* __restrict__ opj,
                                  int32_t* __restrict__ ox0, T* __restrict__ ofx, T* __restrict__ ofy,
                                  T* __restrict__ ofz) {
#pragma clang fp contract(off)
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  // the pair's galaxies from the emission order (perm: sorted -> emitted)
  const int e = perm[p];
  const int i = ui[e], j = uj[e];
  opi[p] = i;
  opj[p] = j;
  const double xi = x[i], yi = y[i], zi = z[i];
  const double dx = fold(x[j] - xi, c.L, c.halfL);
  const double dy = fold(y[j] - yi, c.L, c.halfL);
  const double dz = fold(z[j] - zi, c.L, c.halfL);
  double mx = xi + 0.5 * dx, my = yi + 0.5 * dy, mz = zi + 0.5 * dz;
  mx = mx >= c.L ? mx - c.L : (mx < 0.0 ? mx + c.L : mx);
  my = my >= c.L ? my - c.L : (my < 0.0 ? my + c.L : my);
  mz = mz >= c.L ? mz - c.L : (mz < 0.0 ? mz + c.L : mz);
  int x0, y0, z0;
  double fx, fy, fz;
  cic_of(mx, c.gscale, c.N, x0, fx);
  cic_of(my, c.gscale, c.N, y0, fy);
  cic_of(mz, c.gscale, c.N, z0, fz);
  ox0[p] = x0;
  ofx[p] = (T)fx;
  ofy[p] = (T)fy;
  ofz[p] = (T)fz;
}

// galaxy CIC points: key = z0*N + y0
template <typename T>
static __global__ void k_gal_points(const double* __restrict__ x, const double* __restrict__ y,
                             const double* __restrict__ z, int64_t n, double gscale, int N,
                             int32_t* __restrict__ skey, int32_t* __restrict__ idx,
                             int32_t* __restrict__ ox0, T* __restrict__ ofx, T* __restrict__ ofy,
                             T* __restrict__ ofz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int x0, y0, z0;
  double fx, fy, fz;
  cic_of(x[i], gscale, N, x0, fx);
  cic_of(y[i], gscale, N, y0, fy);
  cic_of(z[i], gscale, N, z0, fz);
  skey[i] = z0 * N + y0;
  idx[i] = (int32_t)i;
  ox0[i] = x0;
  ofx[i] = (T)fx;
  ofy[i] = (T)fy;
  ofz[i] = (T)fz;
}

template <typename V>
static __global__ void k_gather(const int32_t* __restrict__ perm, const V* __restrict__ src, int64_t n,
                         V* __restrict__ dst) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  dst[p] = src[perm[p]];
}

// mark the (up to) four lines a point's CIC footprint touches, for the field
// pair of its field (fp = field / 2)
static __global__ void k_mark_lines(const int32_t* __restrict__ skey, int64_t n, int N, int tsc,
                             uint8_t* __restrict__ flags) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t NN = (int64_t)N * N;
  const int64_t k = skey[p];
  const int64_t f = k / NN, l = k % NN;
  const int y0 = (int)(l % N), z0 = (int)(l / N);
  uint8_t* fl = flags + (f >> 1) * NN;
  // the rows a point's footprint can reach: the corner row and the next
  // (CIC), one below to two above (TSC, three of those four rows)
  const int lo = tsc ? -1 : 0, hi = tsc ? 2 : 1;
  for (int dz = lo; dz <= hi; ++dz)
    for (int dy = lo; dy <= hi; ++dy)
      fl[(int64_t)((z0 + dz) & (N - 1)) * N + ((y0 + dy) & (N - 1))] = 1;
}

// plane flag = any line of the plane non-empty
static __global__ void k_plane_flags(const uint8_t* __restrict__ flags, int N, int64_t n_planes,
                              uint8_t* __restrict__ pflags) {
  const int64_t pl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pl >= n_planes) return;
  const uint8_t* f = flags + pl * N;
  int any = 0;
  for (int y = 0; y < N; ++y) any |= f[y];
  pflags[pl] = (uint8_t)(any ? 1 : 0);
}

// task words for the x pass: slot * N^2 + line, slot = fp % batch
constexpr int kTaskKeyBits = 30;
constexpr int32_t kTaskKeyMax = (1 << kTaskKeyBits) - 1;

static __global__ void k_emit_tasks(const uint8_t* __restrict__ flags, const int32_t* __restrict__ pos,
                             int64_t total, int N, int batch, int32_t* __restrict__ tasks) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total || !flags[i]) return;
  const int64_t NN = (int64_t)N * N;
  const int64_t fp = i / NN, l = i % NN;
  tasks[pos[i]] = (int32_t)((fp % batch) * NN + l);
}

// Sort key of each x-pass task: the number of points whose footprint reaches
// its line (both fields 2 fp, 2 fp + 1 of its field pair, from the field-major
// line starts), inverted so that an ascending sort puts the most crowded
// lines first.  rows = 2 (CIC: base lines y - 1 .. y by z - 1 .. z) or 4
// (TSC: y - 2 .. y + 1 by z - 2 .. z + 1).  key[pos[i]] for every flagged i.
static __global__ void k_task_cost(const uint8_t* __restrict__ flags, const int32_t* __restrict__ pos,
                                   int64_t total, int N, int F, int rows,
                                   const int32_t* __restrict__ line_start, int32_t* __restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total || !flags[i]) return;
  const int64_t NN = (int64_t)N * N;
  const int64_t fp = i / NN, l = i % NN;
  const int y = (int)(l % N), z = (int)(l / N);
  const int lo = rows == 4 ? -2 : -1;
  int64_t c = 0;
  for (int part = 0; part < 2; ++part) {
    const int64_t f = 2 * fp + part;
    if (f >= F) continue;
    for (int dz = 0; dz < rows; ++dz)
      for (int dy = 0; dy < rows; ++dy) {
        const int64_t k = f * NN + (int64_t)((z + lo + dz) & (N - 1)) * N + ((y + lo + dy) & (N - 1));
        c += line_start[k + 1] - line_start[k];
      }
  }
  key[pos[i]] = kTaskKeyMax - (int32_t)(c < kTaskKeyMax ? c : kTaskKeyMax);
}

static __global__ void k_iota(int32_t* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

}  // namespace pgx
