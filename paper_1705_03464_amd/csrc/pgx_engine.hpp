// Engine: device buffers and launch sequences of one plan, templated on the
// transform precision T and the grid side N.
#pragma once
#include "pgx_adjoint.hpp"
#include "pgx_dual.hpp"
#include "pgx_misc.hpp"
#include "pgx_pairs.hpp"
#include "pgx_prim.hpp"

#include <type_traits>

namespace pgx {

struct PlanCfg {
  double L = 0, pair_dmax = 0, xi_w_const = 0, smax = 0;
  int N = 0, precision = 1, pair_mode = 0, out_mode = 0, qeff_mode = 0, batch = 0;
  int assignment = 0;  // 0 CIC, 1 TSC
  std::vector<double> p1, p2, o1, o2;
  int F = 0, R = 0, n_fp = 0;
  int pw[3] = {0, 0, 0};
  HostBins bins;
  std::vector<int64_t> nb;   // lattice vectors per output bin (weight > 0)
  std::vector<double> nbw;   // normalisation per output bin: n_b, or sum of weights
  std::vector<double> vol;
};

// Per-kernel timing with HIP events recorded on the launch stream around each
// launch of the instrumented kernels, plus the algorithmic bytes each launch
// must move (reads + writes of the data it is defined on).
struct Profiler {
  struct Cat {
    std::string name;
    int64_t launches = 0;
    double bytes = 0.0, ms = 0.0;
  };
  bool on = false;
  std::vector<Cat> cats;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;

  int cat(const char* name) {
    for (size_t i = 0; i < cats.size(); ++i)
      if (cats[i].name == name) return (int)i;
    cats.push_back(Cat{name});
    return (int)cats.size() - 1;
  }
  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    PGX_HIP(hipEventCreate(&e));
    return e;
  }
  template <typename Fn> void run(const char* name, hipStream_t s, double bytes, Fn&& launch) {
    if (!on) {
      launch();
      return;
    }
    const int c = cat(name);
    hipEvent_t a = ev(), b = ev();
    PGX_HIP(hipEventRecord(a, s));
    launch();
    PGX_HIP(hipEventRecord(b, s));
    pending.push_back({c, {a, b}});
    cats[c].launches += 1;
    cats[c].bytes += bytes;
  }
  void collect() {
    for (auto& p : pending) {
      PGX_HIP(hipEventSynchronize(p.second.second));
      float ms = 0.f;
      PGX_HIP(hipEventElapsedTime(&ms, p.second.first, p.second.second));
      cats[p.first].ms += ms;
      pool.push_back(p.second.first);
      pool.push_back(p.second.second);
    }
    pending.clear();
  }
  void reset() {
    collect();
    cats.clear();
  }
  ~Profiler() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.second.first);
      (void)hipEventDestroy(p.second.second);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Captured launch sequences.  The forward and adjoint bodies are recorded
// once into a HIP graph on a private stream and replayed on the caller's
// stream; a body is captured on its second call with the same key (the first
// runs eagerly and makes every allocation), and the key changes whenever
// anything the recorded launches depend on may have changed (a new pair
// catalogue, a different batch schedule, null-ness of optional inputs).
struct GraphKey {
  uint64_t gen = 0;
  const void* p = nullptr;
  int flags = 0;
  bool operator==(const GraphKey& o) const { return gen == o.gen && p == o.p && flags == o.flags; }
};
struct Graphed {
  hipGraphExec_t exec = nullptr;
  GraphKey key, seen;
  bool has_seen = false;
  int64_t replays = 0;
  Graphed() = default;
  Graphed(const Graphed&) = delete;
  Graphed& operator=(const Graphed&) = delete;
  ~Graphed() { reset(); }
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    has_seen = false;
  }
};

struct EngineBase {
  virtual ~EngineBase() {
    gf.reset();
    gb.reset();
    if (cap) (void)hipStreamDestroy(cap);
  }
  Profiler prof;
  bool use_graphs = true;
  uint64_t gen = 0;  // bumped by every pair build
  hipStream_t cap = nullptr;
  Graphed gf, gb;

  // run body(stream) eagerly, or capture it once and replay it (see Graphed)
  template <typename Body> void graphed(Graphed& g, const GraphKey& key, hipStream_t s, Body&& body) {
    if (!use_graphs || prof.on) {
      body(s);
      return;
    }
    if (g.exec && g.key == key) {
      PGX_HIP(hipGraphLaunch(g.exec, s));
      ++g.replays;
      return;
    }
    if (!g.has_seen || !(g.seen == key)) {
      g.reset();
      body(s);
      g.seen = key;
      g.has_seen = true;
      return;
    }
    if (!cap) PGX_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    PGX_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
    try {
      body(cap);
    } catch (...) {
      (void)hipStreamEndCapture(cap, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    PGX_HIP(hipStreamEndCapture(cap, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    PGX_HIP(e);
    g.reset();
    g.exec = exec;
    g.key = key;
    PGX_HIP(hipGraphLaunch(exec, s));
    ++g.replays;
  }

  virtual void pairs_build(const double* x, const double* y, const double* z, const float* w,
                           int64_t n, hipStream_t s, int64_t* n_pairs, int64_t* counts,
                           double* wsum) = 0;
  virtual void pairs_export(int32_t* f, int32_t* i, int32_t* j, hipStream_t s) = 0;
  virtual void forward(const float* w, hipStream_t s, double* wsum, double* xi_gg, double* xi_pg,
                       double* xi_dp, double* b_pg, double* q_eff) = 0;
  virtual void backward(hipStream_t s, const double* g_b, const double* g_q, const double* g_xipg,
                        const double* g_xigg, const double* g_xidp, float* grad_w) = 0;
  virtual void autotune(hipStream_t s, int32_t* out) = 0;
  virtual void schedule_info(int32_t* out) const = 0;
  virtual void set_schedule(const int32_t* in, hipStream_t s) = 0;
  virtual double recheck_dual(hipStream_t s, bool fallback) = 0;
  virtual void multipoles(hipStream_t s, int lmax, double* xi) = 0;
  virtual void multipoles_backward(hipStream_t s, const double* g, float* grad_w) = 0;
  virtual void projected(hipStream_t s, const double* xi_dp, double* wp, bool adjoint) = 0;
  virtual int64_t gal_count() const = 0;
  virtual int64_t pair_count() const = 0;
  bool built = false;
  bool forward_done = false;
  // keep each pair-field spectrum from the forward for the adjoint (when the
  // device has room); the adjoint then skips recomputing them
  bool keep_spectra = false;
  bool spectra_valid = false;
  // autotuner: the dual form's largest xi disagreement with the per-field
  // transforms in units of 1e-5 max(|xi|, 1e-2) (-1 when not measured)
  double dual_disagreement = -1.0;
};

constexpr int kRMax = 640;  // largest number of output bins handled by the bin kernels

template <typename T, int N> struct Engine : EngineBase {
  using Sh = typename DefaultShape<T, N>::type;
  static constexpr int TPL = Sh::TPL;
  // strided passes: tiles of W adjacent columns (W complex = 128 B per row;
  // 64 B for 16-element shapes, whose 1024-thread blocks would cap registers
  // at 128 per thread); x-direction passes: WX whole lines per block
  static constexpr int W = Sh::E <= 8 ? (int)(128 / sizeof(C<T>)) : (int)(64 / sizeof(C<T>));
  static constexpr int NT = W * TPL;
  static constexpr int WX = (256 / TPL) > 1 ? (256 / TPL) : 1;
  static constexpr int NTX = WX * TPL;
  // dual form, fused inverse x + gather: base lines per y tile and z segments
  // per launch.  Small tiles (two z rows of 4 lines, 35 KB of LDS at 512^3)
  // let several blocks share a compute unit; measured at 512^3: 3.6 ms per
  // launch against 3.7 ms for 7 and 4.3 ms for 15 base lines per tile.  The
  // TSC sweep keeps three z rows of YTT + 2 lines and its stage twiddles in
  // registers: 52 KB with 2 base lines per tile, three blocks per compute unit
  // (5.6 ms per launch at 512^3, against 7.7 ms with the LDS twiddle table and
  // two blocks, and 10.2 ms for 3 base lines per tile).
  static constexpr int YTS = 3;
  static constexpr int YTT = 2;
  static constexpr int kZSeg = 8;
  // dual form, z passes: tile width of the second variant (half the columns,
  // so that two blocks share a compute unit)
  static constexpr int WH = W / 2 >= 4 ? W / 2 : W;
  static constexpr int64_t NN = (int64_t)N * N;
  static constexpr int64_t NC = NN * N;
  // second radix schedule of the y passes (autotuner candidate)
  using ShA = typename AltShape<T, N>::type;
  static constexpr int WA =
      (int)(128 / sizeof(C<T>)) * ShA::TPL <= 1024 ? (int)(128 / sizeof(C<T>)) : 1024 / ShA::TPL;
  static constexpr int NTA = WA * ShA::TPL;

  const PlanCfg& cfg;
  int B = 1;          // field pairs per batch
  int n_batches = 0;
  int64_t n_gal = 0, n_pairs = 0;
  int64_t gal_count() const override { return n_gal; }
  int64_t pair_count() const override { return n_pairs; }
  std::vector<int64_t> batch_task_off;  // host, n_batches + 1
  std::vector<int64_t> field_counts_h;  // host, pairs per field
  std::vector<int64_t> build_print;     // schedule and buffers of the last pair build
  // the line flags and x-pass task lists match the current catalogue
  bool tasks_ready = false;
  // the dual form's line-major copy of the pairs matches the current catalogue
  bool lm_ready = false;

  // kernel variants picked by the autotuner (0 = default): forward y pass,
  // inverse y pass (radix schedule), z pass (twiddle source; for the dual
  // form: tile width)
  int v_ypass = 0, v_yinv = 0, v_zpass = 0;
  // algorithm of the pair-field part of the forward: 0 = one transform per
  // field pair, 1 = dual form (one transform per pair of output bins, then a
  // gather at the pair midpoints)
  int algo = 0;
  // z-pass variant of the per-field transforms the autotuner found (the
  // schedule a failed re-check of the dual form falls back to)
  int pf_vz = 0;
  DBuf coef_id, bscale, bfa, bfb, GV;  // dual form: bin coefficients 1/norm_b (and their FP32 values), bin-pair slots, gathered values
  DBuf FSC;  // per-field FP32 transform scale 1 / Wsum_f
  // constant tables
  DBuf tw_alt;
  DBuf tw, lut1, lut2, mu2, nbd, vold, t1, t2, slot_fa, slot_fb, slot_fp, gslot_fa, gslot_fb,
      fidx, neg1;
  // catalogue
  DBuf g_key, g_ls, g_x0, g_fx, g_fy, g_fz, g_idx, g_wt, g_tasks;
  // field-major pair catalogue; p_fs holds the field boundaries (F + 1), p_ls
  // the (field, line) starts that only the per-field transforms read (built
  // with their task lists)
  DBuf p_key, p_ls, p_fs, p_i, p_j, p_x0, p_fx, p_fy, p_fz, p_wt;
  DBuf tasks_s, t_key, t_key2;  // the scatter's task order (most crowded line first) and its sort keys
  DBuf p_wd, wg_part;  // FP64 pair weights of the current forward; partial weight sums
  DBuf ws_part, red_part, mp_part;  // partial sums of the chunked segmented reductions
  // line-major copy of the pair catalogue (all fields together): line starts,
  // CIC corner and fractions, field, field-major index, weight (adjoint of the
  // dual form)
  DBuf l_ls, l_x0, l_fx, l_fy, l_fz, l_f, l_p, l_wt, dcoef;
  DBuf lflag, pflag, tasks;
  // scratch for the build
  DBuf s_tmp, s_k0, s_k1, s_v0, s_v1, s_cnt, s_off, s_px, s_py, s_pz, s_cell, s_cs, s_hist, s_err,
      s_i, s_j, s_x0, s_fx, s_fy, s_fz, s_pos;
  // forward work
  DBuf X, P1, P2, Fg, part, S, Sgg, wsum_d, wg_d, outs;
  // backward work
  DBuf KX, KY, Aacc, gbuf, gbuf_g, grad_d, apg, agg, gws, gwg, w_last;
  DBuf SPEC;  // kept pair-field spectra, one N^3 grid per field pair
  DBuf gup, gw_out;  // adjoint: copies of the upstream gradients, weight gradient
  bool w_given = false;
  // the last forward ran the dual form: its gathered values are in GV
  bool fwd_dual = false;
  DBuf S_ref, dis_d;  // autotuner: per-field bin sums, disagreement of the dual form
  // dual form: the bin-pair kernel fields after their x and y transforms
  // depend only on the binning; kept for the plan's lifetime when they fit
  DBuf KC;
  bool kc_tried = false, kc_valid = false;
  // dual form, z-pass variant 2: the full kernel spectra (rows ky, kz <= N/2
  // of every x frequency; the bin kernels are even in each axis), filled once
  // per plan, and the galaxy kernel's coefficients on them
  DBuf KS, gcoef;
  bool ks_tried = false, ks_valid = false;
  // multipoles of the pair axis against the pair-to-galaxy direction: the
  // galaxy positions of the last build (for the pair axes), the pair
  // harmonics, the gathered values of every (bin, harmonic) combo, tables
  DBuf pos_x, pos_y, pos_z, MPY, MPG, MPS, mp_coef, mp_scale, mp_fa, mp_fb, MPA, MPL, mp_cf;
  int mp_lmax = -1;  // lmax of the last multipoles call (-1: none since the last forward)

  // room for the kept spectra: already allocated, or fits in free device
  // memory with 4 GiB to spare
  C<T>* spectra_store() {
    const size_t need = (size_t)cfg.n_fp * (size_t)NC * sizeof(C<T>);
    if (need == 0) return nullptr;
    if (!SPEC.try_ensure(need)) return nullptr;
    return SPEC.as<C<T>>();
  }

  // Upper bound of the device memory the plan's buffers reach for a catalogue
  // of n galaxies and P pairs, summed over everything the pair build, the
  // forward, the adjoint and the autotuner hold at once: point and pair
  // records with their build scratch, per-(field, line) tables, batch slots
  // of up to twice the default batch, the galaxy spectrum and accumulator,
  // the dual form's gathered values and kernel stores, the kept spectra when
  // asked for; plus 10 % and 64 MiB for tables and first-fit fragmentation.
  // The multipoles' harmonic buffers are not included.
  static size_t memory_bound(const PlanCfg& c, int64_t n, int64_t P, bool spectra) {
    const double cb = (double)sizeof(C<T>), tb = (double)sizeof(T);
    const double F = c.F, R = c.R, Q = (c.R + 1) / 2, nfp = c.n_fp;
    const double nz = win_len(c.pw[2]), ny = win_len(c.pw[1]), nx = win_len(c.pw[0]);
    const double nd = (double)std::max<int64_t>(n, 1), pd = (double)std::max<int64_t>(P, 1);
    int nc = (int)std::floor(c.L / (c.smax * (1.0 + 1e-12)));
    const double ncell = std::max(27.0, (double)nc * nc * nc);
    double b = 0.0;
    // galaxies: positions kept for the multipoles, cell-list scratch, point
    // records, weights and gradients
    b += nd * (24.0 + 24.0 + 16.0 + 16.0 + 12.0 + 4.0 * tb + 4.0 + 3.0 * tb + 4.0 + 4.0 + 8.0 + 16.0);
    // pairs: build scratch (six int32 arrays over max(n, P)), radix-sort
    // temporaries, field-major records, FP64 weights, line-major copy, gradient
    b += std::max(nd, pd) * 24.0 + (std::max(nd, pd) * 8.0 + (32 << 20));
    b += pd * (16.0 + 4.0 * tb + 8.0 + 12.0 + 4.0 * tb + 16.0);
    // per-(field, line) starts, counting table, line flags, task positions
    const double fl = F * NN + 1.0, pl = nfp * NN + 1.0;
    // (and the task order's keys, sorted copies and sort temporaries)
    b += fl * 4.0 + (std::max({ncell, fl, (double)NN}) + 1.0) * 8.0 + pl * (1.0 + 4.0 + 4.0 + 24.0) + nfp * N +
         2.0 * (NN + 1.0) * 4.0;
    const double tiny = 16.0 * F * R * 8.0 + 4.0 * (F + R) * 8.0 + ((size_t)8 << 20);
    if (c.precision == PGX_FP64_PLAIN) {
      const double nblk = std::ceil(nx * ny * nz / 256.0);
      b += 2.0 * NC * cb + nblk * 2.0 * R * 8.0 + tiny;
    } else {
      const int b0 = std::max(1, std::min({c.batch > 0 ? c.batch : (N >= 512 ? 8 : (N >= 256 ? 16 : 32)),
                                           c.n_fp, kMaxSlots}));
      const double Bm = std::min<double>(kMaxSlots, 2.0 * b0);
      const double nblkE = std::ceil(ny * nz / (double)WX);
      // batch slots: transformed fields, pruned inverse z and y outputs, the
      // adjoint's kernel fields
      b += Bm * (NC + nz * NN + nz * ny * N + nz * ny * N + nz * NN) * cb;
      b += Bm * nblkE * 2.0 * R * 8.0;
      // galaxy spectrum, adjoint accumulator; dual form: gathered values,
      // kernel-field and kernel-spectrum stores
      b += 2.0 * NC * cb + R * pd * 4.0;
      b += Q * nz * NN * cb + Q * (N / 2 + 1.0) * (N / 2 + 1.0) * N * cb;
      if (spectra) b += nfp * NC * cb;
      b += 3.0 * F * R * reduce_chunks((int64_t)F * R) * 8.0 + tiny;
    }
    return (size_t)(1.1 * b) + ((size_t)64 << 20);
  }

  explicit Engine(const PlanCfg& c) : cfg(c) {
    static_assert(N % W == 0 && N % WA == 0, "tile width must divide N");
    static_assert((N / W) * N % 8 == 0 && (N / WH) * N % 8 == 0, "z-pass grids are whole XCD rounds");
    upload(tw, twiddles<Sh>());
    upload(tw_alt, twiddles<ShA>());
    upload(lut1, cfg.bins.lut1.empty() ? std::vector<int16_t>{-1} : cfg.bins.lut1);
    upload(lut2, cfg.bins.lut2.empty() ? std::vector<int16_t>{-1} : cfg.bins.lut2);
    upload(mu2, cfg.bins.mu2.empty() ? std::vector<double>{0.0} : cfg.bins.mu2);
    upload(nbd, cfg.nbw);
    upload(vold, cfg.vol);
    std::vector<double> a1(cfg.p1.size()), a2(cfg.p2.size());
    for (size_t i = 0; i < a1.size(); ++i) a1[i] = cfg.p1[i] * cfg.p1[i];
    for (size_t i = 0; i < a2.size(); ++i) a2[i] = cfg.p2[i] * cfg.p2[i];
    upload(t1, a1);
    upload(t2, a2);
    const int nfp = cfg.n_fp;
    B = std::max(1, std::min({default_batch(), nfp, kMaxSlots}));
    n_batches = (nfp + B - 1) / B;
    // slot j of the launch sequence holds field pair j, whatever the batch size
    std::vector<int32_t> fa((size_t)nfp + kMaxSlots, -1), fb((size_t)nfp + kMaxSlots, -1),
        fp((size_t)nfp + kMaxSlots, 0);
    for (int k = 0; k < nfp; ++k) {
      fa[k] = 2 * k;
      fb[k] = 2 * k + 1 < cfg.F ? 2 * k + 1 : -1;
      fp[k] = k;
    }
    upload(slot_fa, fa);
    upload(slot_fb, fb);
    upload(slot_fp, fp);
    // dual form: slot q holds output bins (2q, 2q + 1) with unit coefficients
    const int R = cfg.R, Q = (R + 1) / 2;
    std::vector<double> ci((size_t)R * R, 0.0);
    std::vector<float> bs((size_t)std::max(R, 1), 1.0f);
    for (int b = 0; b < R; ++b) {
      const double sc = cfg.nbw[b] > 0 ? 1.0 / cfg.nbw[b] : 1.0;
      bs[b] = (float)sc;
      ci[(size_t)b * R + b] = (double)bs[b];  // the generator casts to T: same value
    }
    upload(coef_id, ci);
    upload(bscale, bs);
    std::vector<int32_t> qa((size_t)Q + kMaxSlots, -1), qb((size_t)Q + kMaxSlots, -1);
    for (int q = 0; q < Q; ++q) {
      qa[q] = 2 * q;
      qb[q] = 2 * q + 1 < R ? 2 * q + 1 : -1;
    }
    upload(bfa, qa);
    upload(bfb, qb);
    upload(gslot_fa, std::vector<int32_t>{0});
    upload(gslot_fb, std::vector<int32_t>{-1});
    upload(neg1, std::vector<int32_t>{-1});
    std::vector<int32_t> fi(std::max(cfg.F, 1));
    for (int f = 0; f < (int)fi.size(); ++f) fi[f] = f;
    upload(fidx, fi);
    std::vector<int32_t> gt(NN);
    for (int64_t l = 0; l < NN; ++l) gt[l] = (int32_t)l;
    upload(g_tasks, gt);
    PGX_HIP(hipDeviceSynchronize());
  }

  // per-stage twiddles exp(-2 pi i r k / (Ns R)) at [twoff(s) + r Ns + k], FP64 rounded to T
  template <typename Shp> static std::vector<C<T>> twiddles() {
    std::vector<C<T>> h(Shp::tw_entries());
    for (int st = 1; st < Shp::stages; ++st) {
      const int R = Shp::radix(st), Ns = Shp::ns(st);
      for (int r = 0; r < R; ++r)
        for (int k = 0; k < Ns; ++k) {
          const double a = -2.0 * kPi * (double)(r * k) / (double)(Ns * R);
          h[Shp::twoff(st) + r * Ns + k] = C<T>{(T)std::cos(a), (T)std::sin(a)};
        }
    }
    return h;
  }

  template <typename V> static void upload(DBuf& d, const std::vector<V>& h) {
    d.ensure(h.size() * sizeof(V));
    if (!h.empty()) PGX_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  }

  BinMap binmap() const {
    BinMap bm;
    bm.mode = cfg.out_mode;
    bm.n2 = cfg.out_mode == 0 ? 1 : (int)cfg.o2.size() - 1;
    bm.lut1 = lut1.as<int16_t>();
    bm.lut1_n = (int)cfg.bins.lut1.size();
    bm.lut2 = lut2.as<int16_t>();
    bm.lut2_n = (int)cfg.bins.lut2.size();
    bm.mu2 = mu2.as<double>();
    for (int i = 0; i < 4; ++i) bm.g[i] = cfg.bins.g[i];
    bm.rcut2 = cfg.bins.rcut2;
    bm.rmax2 = cfg.bins.rmax2;
    return bm;
  }

  // ------------------------------------------------------------------------
  // pair catalogue
  // ------------------------------------------------------------------------
  // blocks of the pair search (one wavefront per galaxy, grid-stride)
  static int pair_blocks(int64_t n) {
    const int64_t b = (n + kPairWaves - 1) / kPairWaves;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 16));
  }

  void pairs_build(const double* x, const double* y, const double* z, const float* w, int64_t n,
                   hipStream_t s, int64_t* n_pairs_out, int64_t* counts, double* wsum) override {
    PGX_REQUIRE(n >= 0 && n < INT32_MAX, PGX_EINVAL, "n_gal must be in [0, 2^31)");
    PGX_REQUIRE(n == 0 || (x && y && z), PGX_EINVAL, "positions must not be NULL");
    built = false;
    forward_done = false;
    mp_lmax = -1;
    n_gal = n;
    const int F = cfg.F;
    // validate
    int* err = s_err.get<int>(1);
    k_fill_i32(err, 1, s);
    if (n > 0) {
      k_validate<<<grid_for(n), 256, 0, s>>>(x, y, z, w, n, cfg.L, err);
      launch_check("validate");
    }
    int herr = 0;
    PGX_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    PGX_HIP(hipStreamSynchronize(s));
    PGX_REQUIRE(!(herr & 1), PGX_EINVAL, "non-finite galaxy position");
    PGX_REQUIRE(!(herr & 2), PGX_EINVAL, "galaxy position outside [0, L)");
    PGX_REQUIRE(!(herr & 4), PGX_EINVAL, "weights must be finite and >= 0");
    if (n > 0) {
      // kept for the pair axes of the multipoles
      PGX_HIP(hipMemcpyAsync(pos_x.get<double>(n), x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      PGX_HIP(hipMemcpyAsync(pos_y.get<double>(n), y, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      PGX_HIP(hipMemcpyAsync(pos_z.get<double>(n), z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }

    // cell list: side >= maximum pair separation
    int nc = (int)std::floor(cfg.L / (cfg.smax * (1.0 + 1e-12)));
    PGX_REQUIRE(nc >= 3, PGX_EINVAL, "maximum pair separation must be < L/3");
    const double side = cfg.L / nc;
    const int64_t ncell = (int64_t)nc * nc * nc;
    int32_t* ck = s_k0.get<int32_t>(n);
    int32_t* ci = s_v0.get<int32_t>(n);
    int32_t* cks = s_k1.get<int32_t>(n);
    int32_t* perm = s_v1.get<int32_t>(n);
    if (n > 0) {
      k_cell_keys<<<grid_for(n), 256, 0, s>>>(x, y, z, n, side, nc, ck, ci);
      launch_check("cell_keys");
    }
    sort_pairs_i32(ck, cks, ci, perm, n, bits_for(ncell), s, s_tmp);
    int32_t* hist = s_hist.get<int32_t>(ncell + 1);
    int32_t* cstart = s_cs.get<int32_t>(ncell + 1);
    counts_to_starts(cks, n, ncell, hist, cstart, s);
    double* px = s_px.get<double>(n);
    double* py = s_py.get<double>(n);
    double* pz = s_pz.get<double>(n);
    if (n > 0) {
      k_gather_pos<<<grid_for(n), 256, 0, s>>>(perm, x, y, z, n, px, py, pz);
      launch_check("gather_pos");
    }
    PairCfg pc;
    pc.L = cfg.L;
    pc.halfL = cfg.L * 0.5;
    pc.gscale = (double)N / cfg.L;
    pc.side = side;
    pc.nc = nc;
    pc.N = N;
    pc.mode = cfg.pair_mode;
    pc.n1 = (int)cfg.p1.size() - 1;
    pc.n2 = (int)cfg.p2.size() - 1;
    pc.step1 = 0;  // smallest power of two with 2 step1 >= n1 (the steps cover n1 - 1)
    while (2 * pc.step1 < pc.n1) pc.step1 = pc.step1 ? 2 * pc.step1 : 1;
    pc.t1 = t1.as<double>();
    pc.t2 = t2.as<double>();
    pc.dmax2 = cfg.pair_dmax * cfg.pair_dmax;
    int64_t* cnt = s_cnt.get<int64_t>(n + 1);
    int64_t* off = s_off.get<int64_t>(n + 1);
    int64_t P = 0;
    if (n > 0) {
      k_pairs<false, T><<<pair_blocks(n), 64 * kPairWaves, 0, s>>>(pc, px, py, pz, perm, cks, cstart,
                                                                  n, cnt, nullptr, nullptr, nullptr);
      launch_check("pair_count");
      exscan_i64(cnt, off, n, s, s_tmp);
      int64_t last[2] = {0, 0};
      PGX_HIP(hipMemcpyAsync(&last[0], off + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      PGX_HIP(hipMemcpyAsync(&last[1], cnt + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      PGX_HIP(hipStreamSynchronize(s));
      P = last[0] + last[1];
    }
    PGX_REQUIRE(P < (int64_t)INT32_MAX, PGX_ENOTSUP, "pair count reaches 2^31");
    n_pairs = P;
    int32_t* uk = s_k0.get<int32_t>(P);
    int32_t* ui = s_i.get<int32_t>(P);
    int32_t* uj = s_j.get<int32_t>(P);
    if (P > 0) {
      k_pairs<true, T><<<pair_blocks(n), 64 * kPairWaves, 0, s>>>(pc, px, py, pz, perm, cks, cstart,
                                                                 n, off, uk, ui, uj);
      launch_check("pair_emit");
    }
    // bucket by (field, line)
    int32_t* iota = s_v0.get<int32_t>(P);
    if (P > 0) {
      k_iota<<<grid_for(P), 256, 0, s>>>(iota, P);
      launch_check("iota");
    }
    int32_t* sk = p_key.get<int32_t>(P);
    int32_t* pp = s_v1.get<int32_t>(P);
    const int64_t nkeys = (int64_t)F * NN;
    sort_pairs_i32(uk, sk, iota, pp, P, bits_for(nkeys), s, s_tmp);
    int32_t* ppi = p_i.get<int32_t>(P);
    int32_t* ppj = p_j.get<int32_t>(P);
    int32_t* px0 = p_x0.get<int32_t>(P);
    T* pfx = p_fx.get<T>(P);
    T* pfy = p_fy.get<T>(P);
    T* pfz = p_fz.get<T>(P);
    if (P > 0) {
      // galaxy indices in sorted order and the midpoints' CIC data, one pass
      k_pair_cic<T><<<grid_for(P), 256, 0, s>>>(pc, x, y, z, pp, ui, uj, P, ppi, ppj, px0, pfx, pfy, pfz);
      launch_check("pair_cic");
    }
    p_wt.get<T>(P);
    int32_t* pfs = p_fs.get<int32_t>(F + 1);
    k_field_starts<<<grid_for(F + 1), 256, 0, s>>>(sk, P, NN, F, pfs);
    launch_check("field_starts");
    {
      int64_t* cdev = s_cnt.get<int64_t>(std::max<int64_t>(n + 1, F));
      k_field_counts<<<grid_for(F), 256, 0, s>>>(pfs, 1, F, cdev);
      launch_check("field_counts");
      field_counts_h.assign(F, 0);
      PGX_HIP(hipMemcpyAsync(field_counts_h.data(), cdev, F * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      if (counts)
        PGX_HIP(hipMemcpyAsync(counts, cdev, F * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    }
    // galaxy point set
    int32_t* gk = s_k0.get<int32_t>(n);
    int32_t* gi = s_v0.get<int32_t>(n);
    int32_t* gx0 = s_x0.get<int32_t>(n);
    T* gfx = s_fx.get<T>(n);
    T* gfy = s_fy.get<T>(n);
    T* gfz = s_fz.get<T>(n);
    if (n > 0) {
      k_gal_points<T><<<grid_for(n), 256, 0, s>>>(x, y, z, n, (double)N / cfg.L, N, gk, gi, gx0,
                                                  gfx, gfy, gfz);
      launch_check("gal_points");
    }
    int32_t* gks = g_key.get<int32_t>(n);
    int32_t* gp = s_v1.get<int32_t>(n);
    sort_pairs_i32(gk, gks, gi, gp, n, bits_for(NN), s, s_tmp);
    // gp is the sorted catalogue index
    PGX_HIP(hipMemcpyAsync(g_idx.get<int32_t>(n), gp, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    gather(gp, gx0, g_x0.get<int32_t>(n), n, s);
    gather(gp, gfx, g_fx.get<T>(n), n, s);
    gather(gp, gfy, g_fy.get<T>(n), n, s);
    gather(gp, gfz, g_fz.get<T>(n), n, s);
    g_wt.get<T>(n);
    counts_to_starts(gks, n, NN, s_hist.get<int32_t>(NN + 1), g_ls.get<int32_t>(NN + 1), s);

    // line-major copy of the pairs (the dual form's): only when that
    // algorithm is in use (its entry points build it on demand)
    lm_ready = false;
    if constexpr (std::is_same<T, float>::value)
      if (algo == 1) line_major(s);
    // line flags and x-pass task lists of the per-field transforms: only
    // when that algorithm is in use (the schedule builds them on demand)
    tasks_ready = false;
    if constexpr (std::is_same<T, float>::value)
      if (algo == 0) schedule(B, s);
    if (wsum) {
      // weighted pair sum of every field, the numerator of xi(d_p) (the same
      // kernels and order as the forward's)
      double* wp = p_wd.get<double>(std::max<int64_t>(P, 1));
      const int K = reduce_chunks(F);
      double* part = ws_part.get<double>((int64_t)F * K);
      k_pair_wts<T><<<dim3(F, K), 256, 0, s>>>(p_fs.as<int32_t>(), p_i.as<int32_t>(), p_j.as<int32_t>(), w,
                                               nullptr, wp, part);
      k_sum_chunks<<<grid_for(F), 256, 0, s>>>(part, F, K, wsum);
      launch_check("field_wsum");
    }
    PGX_HIP(hipStreamSynchronize(s));
    if (n_pairs_out) *n_pairs_out = P;
    built = true;
    refresh_print();
  }

  // Recorded launch sequences stay valid when the new catalogue has the same
  // schedule (sizes, per-batch task counts, per-field counts) in the same
  // buffers, as when the same catalogue is rebuilt; otherwise the generation
  // moves on and they are recorded again.
  void refresh_print() {
    std::vector<int64_t> fpr = {n_gal, n_pairs, (int64_t)B, tasks_ready ? 1 : 0, lm_ready ? 1 : 0};
    if (tasks_ready) fpr.insert(fpr.end(), batch_task_off.begin(), batch_task_off.end());
    fpr.insert(fpr.end(), field_counts_h.begin(), field_counts_h.end());
    for (const DBuf* d : {&g_key, &g_ls, &g_x0, &g_fx, &g_fy, &g_fz, &g_idx, &g_wt, &g_tasks, &p_key,
                          &p_ls, &p_fs, &p_i, &p_j, &p_x0, &p_fx, &p_fy, &p_fz, &p_wt, &lflag, &pflag, &tasks, &tasks_s, &l_ls, &l_x0, &l_fx,
                          &l_fy, &l_fz, &l_f, &l_p, &l_wt})
      fpr.push_back((int64_t)(intptr_t)d->p);
    if (fpr != build_print) {
      build_print = fpr;
      ++gen;
    }
  }

  // Line-major copy of the pairs for the dual form: a stable sort of the
  // field-major order by (base line, x node), the CIC data and field of each
  // pair in that order, and the line starts.
  void line_major(hipStream_t s) {
    if constexpr (std::is_same<T, float>::value) {
      const int64_t P = n_pairs;
      int32_t* iota = s_v0.get<int32_t>(P);
      int32_t* lk = s_k0.get<int32_t>(P);
      int32_t* lks = s_i.get<int32_t>(P);
      int32_t* lln = s_j.get<int32_t>(P);
      int32_t* lp = l_p.get<int32_t>(P);
      const int32_t* sk = p_key.as<int32_t>();
      if (P > 0) {
        k_iota<<<grid_for(P), 256, 0, s>>>(iota, P);
        launch_check("iota");
        // CIC: by the corner's line and x node; TSC: by the nearest node's
        if (cfg.assignment == 1)
          k_line_x_key_tsc<T><<<grid_for(P), 256, 0, s>>>(sk, p_x0.as<int32_t>(), p_fx.as<T>(), p_fy.as<T>(),
                                                          p_fz.as<T>(), P, NN, N, lk);
        else
          k_line_x_key<<<grid_for(P), 256, 0, s>>>(sk, p_x0.as<int32_t>(), P, NN, N, lk);
        launch_check("line_x_key");
      }
      sort_pairs_i32(lk, lks, iota, lp, P, bits_for(NN * N), s, s_tmp);
      if (P > 0) {
        k_key_line<<<grid_for(P), 256, 0, s>>>(lks, P, N, lln);
        launch_check("key_line");
      }
      gather(lp, p_x0.as<int32_t>(), l_x0.get<int32_t>(P), P, s);
      gather(lp, p_fx.as<T>(), l_fx.get<T>(P), P, s);
      gather(lp, p_fy.as<T>(), l_fy.get<T>(P), P, s);
      gather(lp, p_fz.as<T>(), l_fz.get<T>(P), P, s);
      int32_t* lf = l_f.get<int32_t>(P);
      if (P > 0) {
        k_field_of<<<grid_for(P), 256, 0, s>>>(lp, sk, P, NN, lf);
        launch_check("field_of");
      }
      l_wt.get<T>(P);
      counts_to_starts(lln, P, NN, s_hist.get<int32_t>(NN + 1), l_ls.get<int32_t>(NN + 1), s);
    }
    lm_ready = true;
  }

  // Builds the line-major copy if the current catalogue has none yet (before
  // anything that records launches).
  void ensure_line_major(hipStream_t s) {
    if (!lm_ready) {
      line_major(s);
      refresh_print();
    }
  }

  // Non-empty lines of every field pair (a byte per grid line), non-empty
  // planes, and the exclusive scan of the line flags, from the field-major
  // catalogue: the input of the x-pass task lists.
  void line_flags(hipStream_t s) {
    // (field, line) starts of the field-major catalogue
    const int64_t nkeys = (int64_t)cfg.F * NN;
    counts_to_starts(p_key.as<int32_t>(), n_pairs, nkeys, s_hist.get<int32_t>(nkeys + 1),
                     p_ls.get<int32_t>(nkeys + 1), s);
    const int64_t nfl = (int64_t)cfg.n_fp * NN;
    // one extra zero entry so the exclusive scan over nfl + 1 entries yields the total
    uint8_t* lf = lflag.get<uint8_t>(nfl + 1);
    k_fill_u8(lf, nfl + 1, s);
    if (n_pairs > 0) {
      k_mark_lines<<<grid_for(n_pairs), 256, 0, s>>>(p_key.as<int32_t>(), n_pairs, N, cfg.assignment, lf);
      launch_check("mark_lines");
    }
    uint8_t* pf = pflag.get<uint8_t>((int64_t)cfg.n_fp * N);
    k_plane_flags<<<grid_for((int64_t)cfg.n_fp * N), 256, 0, s>>>(lf, N, (int64_t)cfg.n_fp * N, pf);
    launch_check("plane_flags");
    int32_t* pos = s_pos.get<int32_t>(nfl + 1);
    exscan_u8_i32(lf, pos, nfl + 1, s, s_tmp);  // entry nfl is the total
  }

  int default_batch() const {
    if (cfg.batch > 0) return cfg.batch;
    return N >= 512 ? 8 : (N >= 256 ? 16 : 32);
  }

  // Autotuner.  For each candidate batch size (half, equal to and twice the
  // default) it runs the forward launch sequence twice per variant set (once
  // to settle allocations, once timed with events per kernel): all passes in
  // their default variant, then all in the alternative one (y passes: second
  // radix schedule; z pass: twiddles from the LDS table instead of
  // registers).  Per pass it keeps the faster variant; the batch size with
  // the smallest modelled total wins.  Candidates whose batch buffers do not
  // fit in free device memory (with 4 GiB to spare) are skipped.
  void autotune(hipStream_t s, int32_t* out) override {
    PGX_REQUIRE(built, PGX_ESTATE, "pgx_pairs_build has not been called");
    if constexpr (!std::is_same<T, float>::value) {
      throw Error(PGX_ENOTSUP, "the autotuner tunes the FP32 batched path");
    } else {
      const int nfp = cfg.n_fp;
      const int b0 = std::max(1, std::min({default_batch(), nfp, kMaxSlots}));
      const int64_t slot_bytes =
          (NC + (int64_t)win_len(pwz()) * NN + (int64_t)win_len(pwz()) * win_len(pwy()) * N) *
          (int64_t)sizeof(C<T>);
      const double room = (double)free_device_bytes() + (double)(X.bytes + P1.bytes + P2.bytes) -
                          (double)spare_device_bytes();
      std::vector<int> cands;
      for (int b : {b0 / 2, b0, 2 * b0}) {
        const int bb = std::max(1, std::min({b, nfp, kMaxSlots}));
        if (std::find(cands.begin(), cands.end(), bb) != cands.end()) continue;
        if (bb != b0 && (double)bb * slot_bytes > room) continue;
        cands.push_back(bb);
      }
      const bool prof_on = prof.on;
      float* wl = w_given && n_gal > 0 ? w_last.as<float>() : nullptr;
      double best_ms = 1e300;
      int best[4] = {b0, 0, 0, 0};
      algo = 0;  // the per-field trials, whatever the schedule in use
      for (int b : cands) {
        double t[2][3] = {{0, 0, 0}, {0, 0, 0}}, other = 0;
        try {
          schedule(b, s);
          for (int v = 0; v < 2; ++v) {
            v_ypass = v_yinv = v_zpass = v;
            prof.reset();
            prof.on = false;
            weights(wl, s);
            forward_batched(s, nullptr, wl);
            prof.on = true;
            weights(wl, s);
            forward_batched(s, nullptr, wl);
            prof.collect();
            prof.on = false;
            for (const auto& c : prof.cats) {
              if (c.name == "ypass") t[v][0] = c.ms;
              else if (c.name == "yinv") t[v][1] = c.ms;
              else if (c.name == "zpass_cross") t[v][2] = c.ms;
              else if (v == 0) other += c.ms;
            }
          }
        } catch (const Error& e) {
          // a larger batch whose slots do not fit in the free runs of a
          // caller's workspace (its free total can exceed the largest run)
          prof.on = false;
          if (e.code != PGX_ENOSPACE || b == b0) throw;
          continue;
        }
        const int vy = t[1][0] < t[0][0], vi = t[1][1] < t[0][1], vz = t[1][2] < t[0][2];
        const double ms = other + t[vy][0] + t[vi][1] + t[vz][2];
        if (ms < best_ms) {
          best_ms = ms;
          best[0] = b;
          best[1] = vy;
          best[2] = vi;
          best[3] = vz;
        }
      }
      // the dual form (one transform per pair of output bins) at the chosen
      // batch size, when its gathered values fit (its z-pass variant is the
      // tile width of its z passes).  It is kept only if its xi agree with
      // the per-field transforms' within half of 1e-5 max(|xi|, 1e-2) on
      // every bin (so its error exceeds theirs by at most that): its FP32
      // rounding sits in the bin kernels' convolution at each pair midpoint,
      // which the few pairs of a sparse field do not average.
      int best_algo = 0, best_vz_dual = 0;
      dual_disagreement = -1.0;
      algo = 0;
      if (dual_fits()) {
        const int F = cfg.F, R = cfg.R;
        double* sref = S_ref.get<double>((int64_t)F * R);
        PGX_HIP(hipMemcpyAsync(sref, S.as<double>(), (size_t)F * R * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
        schedule(best[0], s);
        ensure_line_major(s);
        algo = 1;
        double dis[3] = {-1.0, -1.0, -1.0};
        for (int v = 0; v < 3; ++v) {
          // variant 2 reads the kernel-spectrum store: only when it fits
          if (v == 2 && !ensure_kernel_spectra(s)) break;
          v_zpass = v;
          prof.reset();
          prof.on = false;
          weights(wl, s);
          forward_batched(s, nullptr, wl);
          if (v != 1) {
            double* r = dis_d.get<double>(1);
            k_xi_disagreement<<<1, 256, 0, s>>>(sref, S.as<double>(), nbd.as<double>(),
                                                wsum_d.as<double>(), wg_d.as<double>(), F, R, 1e-5, r);
            launch_check("xi_disagreement");
            PGX_HIP(hipMemcpyAsync(&dis[v], r, sizeof(double), hipMemcpyDeviceToHost, s));
            PGX_HIP(hipStreamSynchronize(s));
            if (v == 0) dual_disagreement = dis[0];
            if (!(dis[v] <= 0.5)) {
              if (v == 0) break;
              continue;
            }
          }
          prof.on = true;
          weights(wl, s);
          forward_batched(s, nullptr, wl);
          prof.collect();
          prof.on = false;
          double ms = 0;
          for (const auto& c : prof.cats) ms += c.ms;
          if (ms < best_ms) {
            best_ms = ms;
            best_algo = 1;
            best_vz_dual = v;
          }
        }
        // the check of the variant in use (variants 0 and 1 differ only in
        // tile shape, not in arithmetic)
        if (best_algo == 1 && best_vz_dual == 2) dual_disagreement = dis[2];
        algo = 0;
      }
      prof.reset();
      prof.on = prof_on;
      schedule(best[0], s);
      v_ypass = best[1];
      v_yinv = best[2];
      v_zpass = best_algo == 1 ? best_vz_dual : best[3];
      pf_vz = best[3];
      algo = best_algo;
      ++gen;  // recorded launch sequences used the old schedule
      forward_done = false;
      spectra_valid = false;
      schedule_info(out);
    }
  }

  void set_schedule(const int32_t* in, hipStream_t s) override {
    PGX_REQUIRE(built, PGX_ESTATE, "pgx_pairs_build has not been called");
    PGX_REQUIRE(in[0] >= 1 && in[0] <= kMaxSlots, PGX_EINVAL, "batch size must be in [1, 32]");
    for (int i = 1; i < 5; ++i)
      PGX_REQUIRE(in[i] == 0 || in[i] == 1 || (i == 3 && in[i] == 2 && in[4] == 1), PGX_EINVAL,
                  "variants and algorithm are 0 or 1 (z-pass variant 2 with the dual form)");
    if constexpr (!std::is_same<T, float>::value) {
      throw Error(PGX_ENOTSUP, "schedules apply to the FP32 batched path");
    } else {
      schedule(in[0], s);
      v_ypass = in[1];
      v_yinv = in[2];
      v_zpass = in[3];
      pf_vz = in[4] == 0 ? in[3] : 0;
      algo = in[4];
      ++gen;
      forward_done = false;
      spectra_valid = false;
      if (v_zpass == 2)
        PGX_REQUIRE(ensure_kernel_spectra(s), PGX_ENOSPACE,
                    "the kernel spectra of z-pass variant 2 do not fit in free device memory");
    }
  }

  // The dual form's accuracy check again, on the weights of the last
  // forward (unit weights if none): the per-field transforms and the dual
  // form in its z-pass variant run the forward body once each, and their xi
  // are compared bin by bin as in the autotuner.  With `fallback` and a
  // disagreement above 0.5 the plan switches to the per-field transforms
  // (batch size and y variants kept, the per-field z variant the autotuner
  // found).  Returns -1 when the schedule in use is not the dual form.
  double recheck_dual(hipStream_t s, bool fallback) override {
    PGX_REQUIRE(built, PGX_ESTATE, "pgx_pairs_build has not been called");
    if constexpr (!std::is_same<T, float>::value) {
      throw Error(PGX_ENOTSUP, "the dual form runs on the FP32 batched path");
    } else {
      if (algo != 1) return -1.0;
      float* wl = w_given && n_gal > 0 ? w_last.as<float>() : nullptr;
      const int F = cfg.F, R = cfg.R, vz_dual = v_zpass;
      const bool prof_on = prof.on;
      prof.on = false;
      algo = 0;
      v_zpass = pf_vz;
      weights(wl, s);
      forward_batched(s, nullptr, wl);
      double* sref = S_ref.get<double>((int64_t)F * R);
      PGX_HIP(hipMemcpyAsync(sref, S.as<double>(), (size_t)F * R * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
      algo = 1;
      v_zpass = vz_dual;
      ensure_line_major(s);
      weights(wl, s);
      forward_batched(s, nullptr, wl);
      double* r = dis_d.get<double>(1);
      k_xi_disagreement<<<1, 256, 0, s>>>(sref, S.as<double>(), nbd.as<double>(), wsum_d.as<double>(),
                                          wg_d.as<double>(), F, R, 1e-5, r);
      launch_check("xi_disagreement");
      double dis = -1.0;
      PGX_HIP(hipMemcpyAsync(&dis, r, sizeof(double), hipMemcpyDeviceToHost, s));
      PGX_HIP(hipStreamSynchronize(s));
      prof.on = prof_on;
      dual_disagreement = dis;
      if (fallback && !(dis <= 0.5)) {
        algo = 0;
        v_zpass = pf_vz;
      }
      ++gen;  // recorded launch sequences may hold the other schedule
      forward_done = false;
      spectra_valid = false;
      return dis;
    }
  }

  void schedule_info(int32_t* out) const override {
    if (!out) return;
    out[0] = B;
    out[1] = v_ypass;
    out[2] = v_yinv;
    out[3] = v_zpass;
    out[4] = algo;
  }

  // Batch schedule for b field pairs per launch: per-batch task ranges and
  // the x-pass task words (slot within the batch, line) of every non-empty
  // line, from the line flags and their exclusive scan of the pair build.
  void schedule(int b, hipStream_t s) {
    const int nfp = cfg.n_fp;
    B = std::max(1, std::min({b, nfp, kMaxSlots}));
    n_batches = (nfp + B - 1) / B;
    if (!tasks_ready) line_flags(s);
    const int64_t nfl = (int64_t)nfp * NN;
    const uint8_t* lf = lflag.as<uint8_t>();
    const int32_t* pos = s_pos.as<int32_t>();
    std::vector<int32_t> hpos(n_batches + 1);
    for (int k = 0; k <= n_batches; ++k) {
      const int64_t e = std::min<int64_t>((int64_t)k * B, nfp) * NN;
      PGX_HIP(hipMemcpyAsync(&hpos[k], pos + e, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    PGX_HIP(hipStreamSynchronize(s));
    batch_task_off.assign(hpos.begin(), hpos.end());
    const int64_t ntk = std::max<int64_t>(hpos[n_batches], 1);
    int32_t* tk = tasks.get<int32_t>(ntk);
    k_emit_tasks<<<grid_for(nfl), 256, 0, s>>>(lf, pos, nfl, N, B, tk);
    launch_check("emit_tasks");
    // the scatter's copy: within each batch most crowded line first (stable,
    // so equal counts keep line order), so that a clustered catalogue's few
    // crowded lines start early instead of trailing the launch and the lines
    // sharing a block have similar point counts (6.6 against 7.8 ms per
    // launch on 3.6e8 HOD pairs).  The adjoint's gather keeps line order,
    // where the four lines that read a point's records run close together
    // and find them in cache (6.0 against 6.3 ms).
    int32_t* tks = tasks_s.get<int32_t>(ntk);
    PGX_HIP(hipMemcpyAsync(tks, tk, (size_t)ntk * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (hpos[n_batches] > 0) {
      int32_t* key = t_key.get<int32_t>(ntk);
      int32_t* key2 = t_key2.get<int32_t>(ntk);
      k_task_cost<<<grid_for(nfl), 256, 0, s>>>(lf, pos, nfl, N, cfg.F, cfg.assignment == 1 ? 4 : 2,
                                                p_ls.as<int32_t>(), key);
      launch_check("task_cost");
      for (int k = 0; k < n_batches; ++k) {
        const int64_t t0 = hpos[k], nt = hpos[k + 1] - t0;
        if (nt < 2) continue;
        sort_pairs_i32(key + t0, key2 + t0, tk + t0, tks + t0, nt, kTaskKeyBits, s, s_tmp);
      }
    }
    tasks_ready = true;
  }

  // pairs in the fields of batch k (host copy taken at build time)
  int64_t batch_points(int k) const {
    if (field_counts_h.empty()) return 0;
    int64_t n = 0;
    for (int f = 2 * k * B; f < std::min(2 * (k + 1) * B, cfg.F); ++f) n += field_counts_h[f];
    return n;
  }

  static int bits_for(int64_t nkeys) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < nkeys) ++b;
    return b;
  }

  template <typename V> void gather(const int32_t* perm, const V* src, V* dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_gather<V><<<grid_for(n), 256, 0, s>>>(perm, src, n, dst);
    launch_check("gather");
  }

  void k_fill_i32(int32_t* p, int64_t n, hipStream_t s) {
    k_fill_value<int32_t><<<grid_for(n), 256, 0, s>>>(p, n, 0);
    launch_check("fill");
  }
  void k_fill_u8(uint8_t* p, int64_t n, hipStream_t s) {
    k_fill_value<uint8_t><<<std::min(grid_for(n), 65536), 256, 0, s>>>(p, n, 0);
    launch_check("fill");
  }

  // starts[k] = first index of sorted keys with key >= k, for k in [0, nkeys]
  void counts_to_starts(const int32_t* sorted, int64_t n, int64_t nkeys, int32_t* hist,
                        int32_t* starts, hipStream_t s) {
    k_fill_value<int32_t><<<std::min(grid_for(nkeys + 1), 65536), 256, 0, s>>>(hist, nkeys + 1, 0);
    launch_check("fill");
    if (n > 0) {
      k_run_counts<<<grid_for(n), 256, 0, s>>>(sorted, n, hist);
      launch_check("histogram");
    }
    exscan_i32(hist, starts, nkeys + 1, s, s_tmp);
  }

  void pairs_export(int32_t* f, int32_t* i, int32_t* j, hipStream_t s) override {
    PGX_REQUIRE(built, PGX_ESTATE, "pgx_pairs_build has not been called");
    if (n_pairs == 0) return;
    k_export_pairs<<<grid_for(n_pairs), 256, 0, s>>>(p_key.as<int32_t>(), p_i.as<int32_t>(),
                                                     p_j.as<int32_t>(), n_pairs, NN, f, i, j);
    launch_check("export");
  }

  // ------------------------------------------------------------------------
  // forward
  // ------------------------------------------------------------------------
  void weights(const float* w, hipStream_t s) {
    const int F = cfg.F;
    if (n_gal > 0) {
      k_gather_weights<T><<<grid_for(n_gal), 256, 0, s>>>(g_idx.as<int32_t>(), w, n_gal, g_wt.as<T>());
      launch_check("gal_weights");
    }
    double* wp = p_wd.get<double>(std::max<int64_t>(n_pairs, 1));
    {
      // pair weights (FP64, and in T for the scatters) with their per-field sums
      const int K = reduce_chunks(F);
      double* part = ws_part.get<double>((int64_t)F * K);
      k_pair_wts<T><<<dim3(F, K), 256, 0, s>>>(p_fs.as<int32_t>(), p_i.as<int32_t>(), p_j.as<int32_t>(), w,
                                               n_pairs > 0 ? p_wt.as<T>() : nullptr, wp, part);
      k_sum_chunks<<<grid_for(F), 256, 0, s>>>(part, F, K, wsum_d.get<double>(F));
      launch_check("pair_weights");
    }
    k_field_scale<<<grid_for(F), 256, 0, s>>>(wsum_d.as<double>(), F, FSC.get<float>(std::max(F, 1)));
    launch_check("field_scale");
    double* wpart = wg_part.get<double>(kWtBlocks);
    k_weight_partial<<<kWtBlocks, 256, 0, s>>>(w, n_gal, wpart);
    k_weight_total<<<1, 256, 0, s>>>(wpart, wg_d.get<double>(1));
    launch_check("weight_total");
  }

  // x-pass scatter and its adjoint gather with the plan's mass assignment
  // (CIC, or TSC on the same point records)
  void xscatter(int grid, const int32_t* tk, int nt, const PointSet<T>& ps, const int32_t* fa,
                const int32_t* fb, C<T>* out, const C<T>* twp, const float* fsc, hipStream_t s) {
    if (cfg.assignment == 1)
      k_xscatter<T, Sh, WX, true><<<grid, NTX, 0, s>>>(tk, nt, ps, fa, fb, out, twp, fsc);
    else
      k_xscatter<T, Sh, WX><<<grid, NTX, 0, s>>>(tk, nt, ps, fa, fb, out, twp, fsc);
  }
  // (CIC: the four per-line shares of each point to acc[q qs + p], written
  // once each; TSC: added to acc[p] with atomics)
  void xgather(int grid, const int32_t* tk, int nt, const PointSet<T>& ps, const int32_t* fa,
               const int32_t* fb, const C<T>* in, T scale, float* acc, int64_t qs, const C<T>* twp,
               const float* fsc, hipStream_t s) {
    if (cfg.assignment == 1)
      k_xgather<T, Sh, WX, true><<<grid, NTX, 0, s>>>(tk, nt, ps, fa, fb, in, scale, acc, 0, twp, fsc);
    else
      k_xgather<T, Sh, WX><<<grid, NTX, 0, s>>>(tk, nt, ps, fa, fb, in, scale, acc, qs, twp, fsc);
  }

  PointSet<T> gal_set() const {
    return PointSet<T>{g_ls.as<int32_t>(), g_x0.as<int32_t>(), g_fx.as<T>(), g_fy.as<T>(),
                       g_fz.as<T>(), g_wt.as<T>()};
  }
  PointSet<T> pair_set() const {
    return PointSet<T>{p_ls.as<int32_t>(), p_x0.as<int32_t>(), p_fx.as<T>(), p_fy.as<T>(),
                       p_fz.as<T>(), p_wt.as<T>()};
  }
  PointSet<T> line_set() const {
    return PointSet<T>{l_ls.as<int32_t>(), l_x0.as<int32_t>(), l_fx.as<T>(), l_fy.as<T>(),
                       l_fz.as<T>(), l_wt.as<T>()};
  }

  void finalize(hipStream_t s, double* xi_gg, double* xi_pg, double* xi_dp, double* b_pg,
                double* q_eff, double* wsum) {
    const int F = cfg.F, R = cfg.R;
    // outputs not requested go to plan scratch
    double* base = outs.get<double>(3 * (int64_t)F * R + F + R + 8);
    FinalizeArgs a;
    a.F = F;
    a.R = R;
    a.qmode = cfg.qeff_mode;
    a.L = cfg.L;
    a.xi_w_const = cfg.xi_w_const;
    a.S = S.as<double>();
    a.Sgg = Sgg.as<double>();
    a.nb = nbd.as<double>();
    a.vol = vold.as<double>();
    a.wsum = wsum_d.as<double>();
    a.wg = wg_d.as<double>();
    a.xi_gg = xi_gg ? xi_gg : base;
    a.xi_pg = xi_pg;
    a.xi_dp = xi_dp ? xi_dp : base + R;
    a.b_pg = b_pg ? b_pg : base + R + F;
    a.q_eff = q_eff ? q_eff : base + R + F + (int64_t)F * R;
    k_finalize<<<grid_for((int64_t)F * R + F + R), 256, 0, s>>>(a);
    launch_check("finalize");
    if (wsum) PGX_HIP(hipMemcpyAsync(wsum, wsum_d.p, F * sizeof(double), hipMemcpyDeviceToDevice, s));
  }

  // projected 2PCF of (r_p, |pi|) pair bins from xi(d_p) (adjoint: the
  // gradient with respect to xi(d_p) from the one with respect to w_p)
  void projected(hipStream_t s, const double* in, double* out, bool adjoint) override {
    PGX_REQUIRE(cfg.pair_mode == PGX_PAIR_RP_PI, PGX_EINVAL,
                "the projected 2PCF needs pair bins in (r_p, |pi|)");
    PGX_REQUIRE(in != nullptr && out != nullptr, PGX_EINVAL, "NULL argument");
    const int n1 = (int)cfg.p1.size() - 1, n2 = (int)cfg.p2.size() - 1;
    if (adjoint)
      k_projected_adjoint<<<grid_for(n1 * n2), 256, 0, s>>>(in, vold.as<double>(), t1.as<double>(),
                                                             n1, n2, out);
    else
      k_projected<<<grid_for(n1), 256, 0, s>>>(in, vold.as<double>(), t1.as<double>(), n1, n2, out);
    launch_check("projected");
  }

  void forward(const float* w, hipStream_t s, double* wsum, double* xi_gg, double* xi_pg,
               double* xi_dp, double* b_pg, double* q_eff) override {
    PGX_REQUIRE(built, PGX_ESTATE, "pgx_pairs_build has not been called");
    PGX_REQUIRE(xi_pg != nullptr, PGX_EINVAL, "xi_pg must not be NULL");
    if (w && n_gal > 0) {
      int* err = s_err.get<int>(1);
      k_fill_i32(err, 1, s);
      k_validate_w<<<grid_for(n_gal), 256, 0, s>>>(w, n_gal, err);
      launch_check("validate_w");
      int herr = 0;
      PGX_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
      PGX_HIP(hipStreamSynchronize(s));
      PGX_REQUIRE(!herr, PGX_EINVAL, "weights must be finite and >= 0");
    }
    S.get<double>((int64_t)cfg.F * cfg.R);
    Sgg.get<double>(cfg.R);
    forward_done = false;
    mp_lmax = -1;
    spectra_valid = false;
    w_given = w != nullptr;
    float* wl = w_given && n_gal > 0 ? w_last.get<float>(n_gal) : nullptr;
    if (wl) PGX_HIP(hipMemcpyAsync(wl, w, n_gal * sizeof(float), hipMemcpyDeviceToDevice, s));
    C<T>* spec = nullptr;
    if constexpr (std::is_same<T, float>::value)
      spec = keep_spectra && algo == 0 ? spectra_store() : nullptr;  // the dual form has no pair-field spectra
    if constexpr (std::is_same<T, float>::value) {
      if (algo == 1) {
        ensure_line_major(s);
        ensure_dual_kernels(s);
      }
      if (algo == 0 && !tasks_ready) {
        schedule(B, s);
        refresh_print();
      }
    }
    // the recorded body reads the weights from the plan's copy
    GraphKey key;
    key.gen = gen;
    key.p = spec;
    key.flags = (w_given ? 1 : 0) | (n_gal > 0 ? 2 : 0) | (algo << 2) | (kc_valid ? 64 : 0) |
                (ks_valid ? 128 : 0);
    graphed(gf, key, s, [&](hipStream_t st) {
      weights(wl, st);
      if constexpr (std::is_same<T, float>::value)
        forward_batched(st, spec, wl);
      else
        forward_plain(st);
    });
    spectra_valid = spec != nullptr;
    fwd_dual = std::is_same<T, float>::value && algo == 1;
    finalize(s, xi_gg, xi_pg, xi_dp, b_pg, q_eff, wsum);
    forward_done = true;
  }

  // ------------------------------------------------------------------------
  // backward (batched FP32 path)
  // ------------------------------------------------------------------------
  void backward(hipStream_t s, const double* g_b, const double* g_q, const double* g_xipg,
                const double* g_xigg, const double* g_xidp, float* grad_w) override {
    PGX_REQUIRE(built && forward_done, PGX_ESTATE, "pgx_backward needs a preceding pgx_forward");
    PGX_REQUIRE(grad_w != nullptr || n_gal == 0, PGX_EINVAL, "grad_w must not be NULL");
    if constexpr (std::is_same<T, float>::value) {
      // the recorded body reads the upstream gradients from plan copies and
      // writes the weight gradient to a plan buffer
      const int F = cfg.F, R = cfg.R;
      const double* src[5] = {g_b, g_q, g_xipg, g_xigg, g_xidp};
      const int64_t len[5] = {(int64_t)F * R, (int64_t)F * R, (int64_t)F * R, R, F};
      double* up = gup.get<double>(3 * (int64_t)F * R + R + F);
      const double* cp[5];
      if (fwd_dual) ensure_dual_kernels(s);
      int flags = (spectra_valid ? 1 : 0) | (w_given ? 2 : 0) | (fwd_dual ? 256 : 0) | (kc_valid ? 512 : 0) |
                  (ks_valid ? 1024 : 0);
      double* dst = up;
      for (int i = 0; i < 5; ++i) {
        cp[i] = src[i] ? dst : nullptr;
        if (src[i]) {
          PGX_HIP(hipMemcpyAsync(dst, src[i], len[i] * sizeof(double), hipMemcpyDeviceToDevice, s));
          flags |= 4 << i;
        }
        dst += len[i];
      }
      float* gw = gw_out.get<float>(std::max<int64_t>(n_gal, 1));
      GraphKey key;
      key.gen = gen;
      key.p = spectra_valid ? SPEC.p : nullptr;
      key.flags = flags;
      graphed(gb, key, s, [&](hipStream_t st) {
        backward_batched(st, cp[0], cp[1], cp[2], cp[3], cp[4], gw);
      });
      if (n_gal > 0)
        PGX_HIP(hipMemcpyAsync(grad_w, gw, n_gal * sizeof(float), hipMemcpyDeviceToDevice, s));
    } else {
      throw Error(PGX_ENOTSUP, "the adjoint is implemented on the FP32 batched path");
    }
  }

  void backward_batched(hipStream_t s, const double* g_b, const double* g_q, const double* g_xipg,
                        const double* g_xigg, const double* g_xidp, float* grad_w) {
    const int F = cfg.F, R = cfg.R;
    const int ny = win_len(pwy()), nz = win_len(pwz());
    const int nblkK = (ny * nz + WX - 1) / WX;
    const int64_t kx_slot = (int64_t)nz * ny * N, ky_slot = (int64_t)nz * NN;
    const double cb = (double)sizeof(C<T>);
    const C<T>* twp = tw.as<C<T>>();
    BinMap bm = binmap();
    C<T>* kx = KX.get<C<T>>((int64_t)B * kx_slot);
    C<T>* ky = KY.get<C<T>>((int64_t)B * ky_slot);
    C<T>* x = X.get<C<T>>((int64_t)B * NC);
    C<T>* A = Aacc.get<C<T>>(NC);
    const C<T>* fg = Fg.as<C<T>>();
    // pair-side values: the dual form writes one per pair; the per-field
    // gather (CIC) writes one share per footprint line, summed by the reader
    const int gcomp = !fwd_dual && cfg.assignment == 0 ? 4 : 1;
    const int64_t gstride = std::max<int64_t>(n_pairs, 1);
    float* gb = gbuf.get<float>(gcomp * gstride);
    double* gd = grad_d.get<double>(std::max<int64_t>(n_gal, 1));
    AdjointArgs aa;
    aa.F = F;
    aa.R = R;
    aa.qmode = cfg.qeff_mode;
    aa.L = cfg.L;
    aa.xi_w_const = cfg.xi_w_const;
    aa.S = S.as<double>();
    aa.Sgg = Sgg.as<double>();
    aa.nb = nbd.as<double>();
    aa.vol = vold.as<double>();
    aa.wsum = wsum_d.as<double>();
    aa.wg = wg_d.as<double>();
    aa.g_b = g_b;
    aa.g_q = g_q;
    aa.g_xipg = g_xipg;
    aa.g_xigg = g_xigg;
    aa.g_xidp = g_xidp;
    aa.apg = apg.get<double>((int64_t)F * R);
    aa.agg = agg.get<double>(R);
    aa.gws = gws.get<double>(F);
    aa.gwg = gwg.get<double>(1);
    k_finalize_adjoint<<<1, 256, 0, s>>>(aa);
    launch_check("finalize_adjoint");
    if (gcomp == 1)
      k_fill_value<float><<<grid_for(gstride), 256, 0, s>>>(gb, gstride, 0.f);
    k_fill_value<double><<<grid_for(std::max<int64_t>(n_gal, 1)), 256, 0, s>>>(gd, std::max<int64_t>(n_gal, 1), 0.0);
    launch_check("fill");
    // galaxy kernel field -> A = K^_g G (on the kernel-spectrum path of the
    // dual form the z pass of the pairs computes K^_g G from the stored
    // spectra instead)
    const bool ksp = fwd_dual && ks_path() && n_pairs > 0;
    if (!ksp) {
    prof.run("bwd_kgen", s, (double)kx_slot * cb, [&] {
      k_kgen_x<T, Sh, WX><<<dim3(nblkK, 1, 1), NTX, 0, s>>>(aa.agg, R, gslot_fa.as<int32_t>(),
                                                             gslot_fb.as<int32_t>(), pwx(), pwy(),
                                                             pwz(), bm, kx, kx_slot, twp);
      launch_check("kgen(gal)");
    });
    prof.run("bwd_kgen_y", s, (double)(kx_slot + ky_slot) * cb, [&] {
      k_strided<T, Sh, W, -1, IN_WINDOW, OUT_DENSE><<<dim3(N / W, nz, 1), NT, 0, s>>>(
          kx, ky, kx_slot, ky_slot, (int64_t)ny * N, NN, N, N, pwy(), nullptr, nullptr, 0, nullptr,
          twp);
      launch_check("kgen_y(gal)");
    });
    prof.run("bwd_zinit", s, (double)ky_slot * cb + 2.0 * NC * cb, [&] {
      k_zinit<T, Sh, W><<<dim3(N / W, N, 1), NT, 0, s>>>(ky, pwz(), fg, A, twp);
      launch_check("zinit");
    });
    }
    if (fwd_dual) {
      backward_dual_pairs(s, aa.apg, aa.agg, x, A, gb, twp, bm);
    } else {
      for (int k = 0; k < n_batches; ++k) {
        const int nb = std::min(B, cfg.n_fp - k * B);
        const int64_t t0 = batch_task_off[k], nt = batch_task_off[k + 1] - t0;
        const int32_t* fa = slot_fa.as<int32_t>() + (int64_t)k * B;
        const int32_t* fb = slot_fb.as<int32_t>() + (int64_t)k * B;
        const int32_t* fp = slot_fp.as<int32_t>() + (int64_t)k * B;
        const double pts = (double)batch_points(k) * (4 + 4 * sizeof(T));
        prof.run("bwd_kgen", s, (double)nb * kx_slot * cb, [&] {
          k_kgen_x<T, Sh, WX><<<dim3(nblkK, 1, nb), NTX, 0, s>>>(aa.apg, R, fa, fb, pwx(), pwy(),
                                                                  pwz(), bm, kx, kx_slot, twp,
                                                                  FSC.as<float>());
          launch_check("kgen");
        });
        prof.run("bwd_kgen_y", s, (double)nb * (kx_slot + ky_slot) * cb, [&] {
          k_strided<T, Sh, W, -1, IN_WINDOW, OUT_DENSE><<<dim3(N / W, nz, nb), NT, 0, s>>>(
              kx, ky, kx_slot, ky_slot, (int64_t)ny * N, NN, N, N, pwy(), nullptr, nullptr, 0,
              nullptr, twp);
          launch_check("kgen_y");
        });
        if (spectra_valid) {
          // Z from the spectra the forward kept: no scatter, y pass or forward z
          prof.run("bwd_zpass", s,
                   (double)nb * (2.0 * NC + ky_slot) * cb + 3.0 * NC * cb, [&] {
            k_zback<T, Sh, W, true><<<dim3(N / W, N, 1), NT, 0, s>>>(
                x, NC, pflag.as<uint8_t>(), fp, nb, ky, ky_slot, pwz(), fg, A, twp, SPEC.as<C<T>>());
            launch_check("zback(kept)");
          });
        } else {
          if (nt > 0) {
            prof.run("bwd_xscatter", s, pts + (double)nt * N * cb, [&] {
              xscatter((int)((nt + WX - 1) / WX), tasks_s.as<int32_t>() + t0, (int)nt, pair_set(), fa, fb,
                       x, twp, FSC.as<float>(), s);
              launch_check("xscatter(bwd)");
            });
          }
          prof.run("bwd_ypass", s, (double)nt * N * cb + (double)nb * NC * cb, [&] {
            ypass_launch(v_ypass, x, nb, fp, s);
            launch_check("ypass(bwd)");
          });
          prof.run("bwd_zpass", s,
                   (double)nb * (2.0 * NC + ky_slot) * cb + 3.0 * NC * cb, [&] {
            k_zback<T, Sh, W><<<dim3(N / W, N, 1), NT, 0, s>>>(x, NC, pflag.as<uint8_t>(), fp, nb, ky,
                                                                ky_slot, pwz(), fg, A, twp);
            launch_check("zback");
          });
        }
        prof.run("bwd_yinv", s, (double)nb * NC * cb + (double)nt * N * cb, [&] {
          k_strided<T, Sh, W, 1, IN_DENSE, OUT_FLAGS><<<dim3(N / W, N, nb), NT, 0, s>>>(
              x, x, NC, NC, NN, NN, N, N, 0, lflag.as<uint8_t>(), pflag.as<uint8_t>(), NN, fp, twp);
          launch_check("yinv(bwd)");
        });
        if (nt > 0) {
          // point records (x0, fractions) read, the per-line shares written
          const double gpts = (double)batch_points(k) * (4.0 + 3.0 * sizeof(T) + 4.0 * gcomp);
          prof.run("bwd_xgather", s, gpts + (double)nt * N * cb, [&] {
            xgather((int)((nt + WX - 1) / WX), tasks.as<int32_t>() + t0, (int)nt, pair_set(), fa, fb, x,
                    (T)1, gb, gstride, twp, FSC.as<float>(), s);
            launch_check("xgather");
          });
        }
      }
    }
    galaxy_adjoint_tail(s, A, gb, gcomp, gd, aa.gws, aa.gwg, grad_w, twp);
  }

  // Galaxy side and weight chain of the adjoint, after A holds the spectral
  // accumulation: dL/drho_g = 2 Re IDFT(A) with A(0) removed, gathered at the
  // galaxies; then the per-galaxy gradient from the pair terms (gb, pair
  // weights w_i w_j, dL/dWsum_f) and the galaxy terms (dL/dW_g).
  // gb: the pair-side values, gcomp components of stride max(n_pairs, 1).
  void galaxy_adjoint_tail(hipStream_t s, C<T>* A, const float* gb, int gcomp, double* gd,
                           const double* gws_d, const double* gwg_d, float* grad_w, const C<T>* twp) {
    const double cb = (double)sizeof(C<T>);
    // galaxy-side values: one share per footprint line (CIC), or one sum (TSC)
    const int ggcomp = cfg.assignment == 0 ? 4 : 1;
    const int64_t ggstride = std::max<int64_t>(n_gal, 1);
    float* gbg = gbuf_g.get<float>(ggcomp * ggstride);
    if (ggcomp == 1) {
      k_fill_value<float><<<grid_for(ggstride), 256, 0, s>>>(gbg, ggstride, 0.f);
      launch_check("fill");
    }
    // galaxy side: dL/drho_g = 2 Re IDFT(A) with A(0) removed
    k_zero_dc<T><<<1, 64, 0, s>>>(A);
    prof.run("bwd_gal_zinv", s, 2.0 * NC * cb, [&] {
      k_strided<T, Sh, W, 1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, 1), NT, 0, s>>>(
          A, A, 0, 0, N, N, NN, NN, 0, nullptr, nullptr, 0, nullptr, twp);
      launch_check("gal_zinv");
    });
    prof.run("bwd_gal_yinv", s, 2.0 * NC * cb, [&] {
      k_strided<T, Sh, W, 1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, 1), NT, 0, s>>>(
          A, A, 0, 0, NN, NN, N, N, 0, nullptr, nullptr, 0, nullptr, twp);
      launch_check("gal_yinv");
    });
    prof.run("bwd_gal_xgather", s, (double)NC * cb + (double)n_gal * (4 + 4 * sizeof(T)), [&] {
      xgather((int)(NN / WX), g_tasks.as<int32_t>(), (int)NN, gal_set(), gslot_fa.as<int32_t>(),
              gslot_fb.as<int32_t>(), A, (T)2, gbg, ggstride, twp, nullptr, s);
      launch_check("gal_xgather");
    });
    const float* wl = w_given ? w_last.as<float>() : nullptr;
    if (n_pairs > 0) {
      k_pair_grad<<<grid_for(n_pairs), 256, 0, s>>>(p_key.as<int32_t>(), p_i.as<int32_t>(),
                                                    p_j.as<int32_t>(), gb, gcomp, std::max<int64_t>(n_pairs, 1),
                                                    n_pairs, NN, gws_d, wl, gd);
      launch_check("pair_grad");
    }
    if (n_gal > 0) {
      k_gal_grad<<<grid_for(n_gal), 256, 0, s>>>(g_idx.as<int32_t>(), gbg, ggcomp, ggstride, n_gal, gwg_d, gd);
      k_grad_out<<<grid_for(n_gal), 256, 0, s>>>(gd, n_gal, grad_w);
      launch_check("grad_out");
    }
  }

  // Pair-field part of the adjoint after a dual-form forward (see
  // pgx_dual.hpp): the pair side from the values the forward gathered, the
  // galaxy side through the per-bin pair fields, accumulated into A.
  void backward_dual_pairs(hipStream_t s, const double* apg, const double* agg, C<T>* x, C<T>* A,
                           float* gb, const C<T>* twp, const BinMap& bm) {
    const int R = cfg.R, F = cfg.F, Q = (R + 1) / 2;
    if (n_pairs == 0) return;  // A holds the galaxy term alone
    const bool ksp = ks_path();
    float2* gcf = ksp ? gcoef.get<float2>(Q) : nullptr;
    if (ksp) {
      k_gal_coef<<<(Q + 255) / 256, 256, 0, s>>>(agg, R, bscale.as<float>(), Q, gcf);
      launch_check("gal_coef");
    }
    const int nz = win_len(pwz());
    const int64_t ky_slot = (int64_t)nz * NN;
    C<T>* kc = kernel_store();
    const double cb = (double)sizeof(C<T>);
    float2* cf = dcoef.get<float2>((int64_t)Q * F);
    k_dual_coef<<<grid_for((int64_t)Q * F), 256, 0, s>>>(apg, F, R, bscale.as<float>(), Q, cf);
    launch_check("dual_coef");
    prof.run("bwd_dual_pairs", s, (double)n_pairs * (8.0 + 4.0 * R), [&] {
      k_dual_pair_grad<<<grid_for(n_pairs), 256, 0, s>>>(p_key.as<int32_t>(), n_pairs, NN, apg, R,
                                                         GV.as<float>(), bscale.as<float>(), gb);
      launch_check("dual_pair_grad");
    });
    gather(l_p.as<int32_t>(), p_wt.as<T>(), l_wt.as<T>(), n_pairs, s);
    const double pts = (double)n_pairs * (12.0 + 4.0 * sizeof(T)) + (double)NN * 4.0;
    for (int q0 = 0; q0 < Q; q0 += B) {
      const int nq = std::min(B, Q - q0);
      C<T>* ky = ksp ? nullptr : dual_kernels(s, q0, nq, kc, twp, bm, "bwd_dual_kgen", "bwd_dual_kgen_y");
      prof.run("bwd_dual_xscatter", s, (double)nq * ((double)NC * cb + pts), [&] {
        if (cfg.assignment == 1)
          k_xscatter_dual_tsc<T, Sh, WX><<<(int)(NN / WX), NTX, 0, s>>>(line_set(), l_f.as<int32_t>(), cf, F,
                                                                      q0, nq, x, NC, twp);
        else
          k_xscatter_dual<T, Sh, WX><<<(int)(NN / WX), NTX, 0, s>>>(line_set(), l_f.as<int32_t>(), cf, F,
                                                                   q0, nq, x, NC, twp);
        launch_check("xscatter(dual adjoint)");
      });
      prof.run("bwd_dual_ypass", s, 2.0 * nq * NC * cb, [&] {
        k_strided<T, Sh, W, -1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, nq), NT, 0, s>>>(
            x, x, NC, NC, NN, NN, N, N, 0, nullptr, nullptr, 0, nullptr, twp);
        launch_check("ypass(dual adjoint)");
      });
      if (ksp) {
        // Pi columns, every stored kernel row once, G, and A written (read
        // too after the first batch)
        const double bytes = ((double)nq * (NC + ks_slot()) + (q0 == 0 ? 2.0 : 3.0) * NC) * cb;
        prof.run("bwd_dual_zacc", s, bytes, [&] {
          k_zdual_acc_ks<T, Sh, W><<<dim3(N / W, N, 1), NT, 0, s>>>(
              x, NC, nq, KS.as<C<T>>() + q0 * ks_slot(), ks_slot(), gcf + q0, Fg.as<C<T>>(),
              q0 == 0 ? 1 : 0, A, twp);
          launch_check("zacc(ks)");
        });
        continue;
      }
      prof.run("bwd_dual_zacc", s, (double)nq * (NC + ky_slot) * cb + 2.0 * NC * cb, [&] {
        if (v_zpass == 0)
          k_zdual_acc<T, Sh, W><<<dim3(N / W, N, 1), NT, 0, s>>>(x, NC, nq, ky, ky_slot, pwz(), A, twp);
        else
          k_zdual_acc<T, Sh, WH><<<dim3(N / WH, N, 1), WH * TPL, 0, s>>>(x, NC, nq, ky, ky_slot, pwz(),
                                                                      A, twp);
        launch_check("zacc(dual adjoint)");
      });
    }
    if (kc) kc_valid = true;
  }

  // forward y pass over the flagged lines of a batch, in radix schedule v
  void ypass_launch(int v, C<T>* x, int nb, const int32_t* fp, hipStream_t s) {
    const uint8_t* lf = lflag.as<uint8_t>();
    const uint8_t* pf = pflag.as<uint8_t>();
    if (v == 0)
      k_strided<T, Sh, W, -1, IN_FLAGS, OUT_DENSE><<<dim3(N / W, N, nb), NT, 0, s>>>(
          x, x, NC, NC, NN, NN, N, N, 0, lf, pf, NN, fp, tw.as<C<T>>());
    else
      k_strided<T, ShA, WA, -1, IN_FLAGS, OUT_DENSE><<<dim3(N / WA, N, nb), NTA, 0, s>>>(
          x, x, NC, NC, NN, NN, N, N, 0, lf, pf, NN, fp, tw_alt.as<C<T>>());
  }

  int pwx() const { return cfg.pw[0]; }
  int pwy() const { return cfg.pw[1]; }
  int pwz() const { return cfg.pw[2]; }

  // whether the dual form fits: its per-pair, per-bin gathered values must
  // fit in half the free device memory
  bool dual_fits() const {
    const double fr = (double)free_device_bytes();
    const double need = (double)cfg.R * (double)std::max<int64_t>(n_pairs, 1) * 4.0;
    // from the HIP allocator: at most half the free memory; in a workspace:
    // whatever is free
    return need < (t_heap ? fr + (double)GV.bytes : 0.5 * (fr + (double)GV.bytes));
  }

  // Dual form of the pair-field part (see pgx_dual.hpp): for each batch of B
  // bin pairs, the kernel fields S_b1 + i S_b2 (x, y transforms of the
  // window, from the store when kept), the z pass with G, the inverse y
  // transform, and the inverse x transform swept along z with the gather at
  // every pair midpoint; then the per-field sums.
  // Kernel-field store of the dual form (all (R+1)/2 bin pairs, y
  // transformed): one allocation attempt per plan, at the first dual-form
  // body (an eager run, never a graph capture), kept when it fits in free
  // memory with 4 GiB to spare; null otherwise (the kernel fields are then
  // generated per call).
  C<T>* kernel_store() {
    if (!kc_tried) {
      kc_tried = true;
      const int Q = (cfg.R + 1) / 2;
      const size_t need = (size_t)Q * (size_t)win_len(pwz()) * (size_t)NN * sizeof(C<T>);
      (void)KC.try_ensure(need);
    }
    return KC.as<C<T>>();
  }

  // y-transformed kernel fields of bin pairs q0 .. q0 + nq - 1: from the
  // store when it holds them, else generated (into the store when there is
  // one, else into the work buffer KY)
  C<T>* dual_kernels(hipStream_t s, int q0, int nq, C<T>* kc, const C<T>* twp, const BinMap& bm,
                     const char* nx, const char* ny_name) {
    const int R = cfg.R;
    const int ny = win_len(pwy()), nz = win_len(pwz());
    const int nblkK = (ny * nz + WX - 1) / WX;
    const int64_t kx_slot = (int64_t)nz * ny * N, ky_slot = (int64_t)nz * NN;
    const double cb = (double)sizeof(C<T>);
    C<T>* ky = kc ? kc + (int64_t)q0 * ky_slot : KY.get<C<T>>((int64_t)B * ky_slot);
    if (kc && kc_valid) return ky;
    C<T>* kx = KX.get<C<T>>((int64_t)B * kx_slot);
    prof.run(nx, s, (double)nq * kx_slot * cb, [&] {
      k_kgen_x<T, Sh, WX><<<dim3(nblkK, 1, nq), NTX, 0, s>>>(
          coef_id.as<double>(), R, bfa.as<int32_t>() + q0, bfb.as<int32_t>() + q0, pwx(), pwy(),
          pwz(), bm, kx, kx_slot, twp);
      launch_check("kgen(dual)");
    });
    prof.run(ny_name, s, (double)nq * (kx_slot + ky_slot) * cb, [&] {
      k_strided<T, Sh, W, -1, IN_WINDOW, OUT_DENSE><<<dim3(N / W, nz, nq), NT, 0, s>>>(
          kx, ky, kx_slot, ky_slot, (int64_t)ny * N, NN, N, N, pwy(), nullptr, nullptr, 0,
          nullptr, twp);
      launch_check("kgen_y(dual)");
    });
    return ky;
  }

  // Multipoles of xi_pg in the angle between the pair axis and the
  // pair-to-galaxy direction (even l <= lmax) over the shell bins, by the
  // dual form: one bin kernel per (bin, harmonic) combo c = b nh + h, carrying
  // Y_h(r^) and 1 / n_b; z transform times G, inverse y, inverse x fused with
  // the gather at the midpoints; per-field sums weighted by Y_h of each pair
  // axis.  Uses the weights and galaxy spectrum of the last forward.  Eager
  // launches (not recorded).
  void multipoles(hipStream_t s, int lmax, double* xi) override {
    PGX_REQUIRE(lmax == 0 || lmax == 2 || lmax == 4, PGX_EINVAL, "lmax must be 0, 2 or 4");
    PGX_REQUIRE(cfg.assignment == 0, PGX_ENOTSUP, "the multipoles use the CIC footprint");
    PGX_REQUIRE(xi != nullptr, PGX_EINVAL, "xi_l must not be NULL");
    if constexpr (!std::is_same<T, float>::value) {
      throw Error(PGX_ENOTSUP, "multipoles are implemented on the FP32 batched path");
    } else {
      PGX_REQUIRE(cfg.out_mode == 0, PGX_EINVAL, "multipoles are taken over shell output bins");
      PGX_REQUIRE(cfg.o1[0] > 0.0, PGX_EINVAL, "the first shell edge must be > 0 for multipoles");
      PGX_REQUIRE(built && forward_done, PGX_ESTATE, "pgx_multipoles needs a preceding pgx_forward");
      ensure_line_major(s);
      const int R = cfg.R, F = cfg.F, nh = harm_count(lmax), nl = lmax / 2 + 1;
      const int RC = R * nh, QC = (RC + 1) / 2;
      // combo tables: coefficient 1 / n_b (FP32 value) for bin b(c) = c / nh
      std::vector<double> ci((size_t)RC * R, 0.0);
      std::vector<float> bs((size_t)RC, 1.0f);
      for (int c = 0; c < RC; ++c) {
        const int b = c / nh;
        bs[c] = (float)(cfg.nbw[b] > 0 ? 1.0 / cfg.nbw[b] : 1.0);
        ci[(size_t)c * R + b] = (double)bs[c];
      }
      std::vector<int32_t> qa((size_t)QC + kMaxSlots, -1), qb((size_t)QC + kMaxSlots, -1);
      for (int q = 0; q < QC; ++q) {
        qa[q] = 2 * q;
        qb[q] = 2 * q + 1 < RC ? 2 * q + 1 : -1;
      }
      upload(mp_coef, ci);
      upload(mp_scale, bs);
      upload(mp_fa, qa);
      upload(mp_fb, qb);
      const int64_t P = n_pairs;
      float* yp = MPY.get<float>(std::max<int64_t>((int64_t)nh * P, 1));
      float* gv = MPG.get<float>(std::max<int64_t>((int64_t)RC * P, 1));
      double* Sm = MPS.get<double>((int64_t)F * R * nl);
      if (P > 0) {
        k_pair_harm<<<grid_for(P), 256, 0, s>>>(p_i.as<int32_t>(), p_j.as<int32_t>(), pos_x.as<double>(),
                                                pos_y.as<double>(), pos_z.as<double>(), P, cfg.L, nh, yp);
        launch_check("pair_harm");
        const int ny = win_len(pwy()), nz = win_len(pwz());
        const int nblkK = (ny * nz + WX - 1) / WX;
        const int64_t kx_slot = (int64_t)nz * ny * N, ky_slot = (int64_t)nz * NN;
        C<T>* kx = KX.get<C<T>>((int64_t)B * kx_slot);
        C<T>* ky = KY.get<C<T>>((int64_t)B * ky_slot);
        C<T>* x = X.get<C<T>>((int64_t)B * NC);
        const C<T>* fg = Fg.as<C<T>>();
        const C<T>* twp = tw.as<C<T>>();
        const BinMap bm = binmap();
        for (int q0 = 0; q0 < QC; q0 += B) {
          const int nq = std::min(B, QC - q0);
          k_kgen_x<T, Sh, WX><<<dim3(nblkK, 1, nq), NTX, 0, s>>>(
              mp_coef.as<double>(), R, mp_fa.as<int32_t>() + q0, mp_fb.as<int32_t>() + q0, pwx(), pwy(),
              pwz(), bm, kx, kx_slot, twp, nullptr, nh);
          launch_check("kgen(multipoles)");
          k_strided<T, Sh, W, -1, IN_WINDOW, OUT_DENSE><<<dim3(N / W, nz, nq), NT, 0, s>>>(
              kx, ky, kx_slot, ky_slot, (int64_t)ny * N, NN, N, N, pwy(), nullptr, nullptr, 0, nullptr, twp);
          launch_check("kgen_y(multipoles)");
          k_zconv<T, Sh, W><<<dim3(N / W, N, 1), NT, 0, s>>>(ky, ky_slot, nq, pwz(), fg, x, NC, twp);
          launch_check("zconv(multipoles)");
          k_strided<T, Sh, W, 1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, nq), NT, 0, s>>>(
              x, x, NC, NC, NN, NN, N, N, 0, nullptr, nullptr, 0, nullptr, twp);
          launch_check("yinv(multipoles)");
          k_xinv_gather_sweep<T, Sh, YTS><<<dim3((N + YTS - 1) / YTS, kZSeg, nq), (YTS + 1) * TPL, 0, s>>>(
              line_set(), l_p.as<int32_t>(), P, x, NC, N / kZSeg, 2 * q0, RC, gv, twp);
          launch_check("xinv_gather(multipoles)");
        }
      }
      {
        const int K = reduce_chunks((int64_t)F * R * nl);
        double* part = mp_part.get<double>((int64_t)F * R * nl * K);
        k_dual_reduce_mp<<<dim3(F, R * nl, K), 256, 0, s>>>(p_fs.as<int32_t>(), 1, p_wd.as<double>(), gv, yp,
                                                            P, R, nh, nl, mp_scale.as<float>(), part);
        k_sum_chunks<<<grid_for((int64_t)F * R * nl), 256, 0, s>>>(part, (int64_t)F * R * nl, K, Sm);
        launch_check("reduce(multipoles)");
      }
      k_finalize_mp<<<grid_for((int64_t)F * R * nl), 256, 0, s>>>(Sm, nbd.as<double>(), wsum_d.as<double>(),
                                                                  wg_d.as<double>(), F, R, nl, xi);
      launch_check("finalize(multipoles)");
      mp_lmax = lmax;
    }
  }

  // Adjoint of the last multipoles call: dL/dw for upstream gradients g of
  // xi_l [F][R][lmax/2 + 1].  Pair side from the gathered values of that
  // call; galaxy side through the harmonic bin kernels (Pi scatter with each
  // pair's harmonic, y pass, z pass accumulating into A), then the galaxy
  // side and weight chain of the main adjoint.  Eager launches.
  void multipoles_backward(hipStream_t s, const double* g, float* grad_w) override {
    if constexpr (!std::is_same<T, float>::value) {
      throw Error(PGX_ENOTSUP, "multipoles are implemented on the FP32 batched path");
    } else {
      PGX_REQUIRE(built && forward_done && mp_lmax >= 0, PGX_ESTATE,
                  "pgx_multipoles_backward needs a preceding pgx_multipoles after the last pgx_forward");
      ensure_line_major(s);
      PGX_REQUIRE(g != nullptr, PGX_EINVAL, "g_xi_l must not be NULL");
      PGX_REQUIRE(grad_w != nullptr || n_gal == 0, PGX_EINVAL, "grad_w must not be NULL");
      const int lmax = mp_lmax, R = cfg.R, F = cfg.F, nh = harm_count(lmax), nl = lmax / 2 + 1;
      const int RC = R * nh, QC = (RC + 1) / 2;
      const int64_t P = n_pairs;
      const double cb = (double)sizeof(C<T>);
      (void)cb;
      const C<T>* twp = tw.as<C<T>>();
      C<T>* A = Aacc.get<C<T>>(NC);
      C<T>* x = X.get<C<T>>((int64_t)B * NC);
      float* gb = gbuf.get<float>(std::max<int64_t>(P, 1));
      double* gd = grad_d.get<double>(std::max<int64_t>(n_gal, 1));
      double* a = MPA.get<double>((int64_t)F * R * nl);
      double* gws_d = gws.get<double>(F);
      double* gwg_d = gwg.get<double>(1);
      k_finalize_adjoint_mp<<<1, 256, 0, s>>>(MPS.as<double>(), g, nbd.as<double>(), wsum_d.as<double>(),
                                               wg_d.as<double>(), F, R, nl, a, gws_d, gwg_d);
      launch_check("finalize_adjoint(multipoles)");
      k_fill_value<float><<<grid_for(std::max<int64_t>(P, 1)), 256, 0, s>>>(gb, std::max<int64_t>(P, 1), 0.f);
      k_fill_value<double><<<grid_for(std::max<int64_t>(n_gal, 1)), 256, 0, s>>>(gd, std::max<int64_t>(n_gal, 1), 0.0);
      // A = 0 (the multipoles have no galaxy auto-correlation term)
      k_fill_value<T><<<std::min(grid_for(2 * NC), 65536), 256, 0, s>>>(reinterpret_cast<T*>(A), 2 * NC, (T)0);
      launch_check("fill");
      if (P > 0) {
        k_mp_pair_grad<<<grid_for(P), 256, 0, s>>>(p_key.as<int32_t>(), P, NN, a, R, nh, nl, MPG.as<float>(),
                                                   MPY.as<float>(), mp_scale.as<float>(), gb);
        launch_check("pair_grad(multipoles)");
        float2* cf = mp_cf.get<float2>((int64_t)QC * F);
        k_mp_coef<<<grid_for((int64_t)QC * F), 256, 0, s>>>(a, F, R, nh, nl, mp_scale.as<float>(), QC, cf);
        launch_check("coef(multipoles)");
        float* yl = MPL.get<float>((int64_t)nh * P);
        k_harm_line_major<<<grid_for(P), 256, 0, s>>>(l_p.as<int32_t>(), MPY.as<float>(), P, nh, yl);
        launch_check("harm_line_major");
        gather(l_p.as<int32_t>(), p_wt.as<T>(), l_wt.as<T>(), P, s);
        const int ny = win_len(pwy()), nz = win_len(pwz());
        const int nblkK = (ny * nz + WX - 1) / WX;
        const int64_t kx_slot = (int64_t)nz * ny * N, ky_slot = (int64_t)nz * NN;
        C<T>* kx = KX.get<C<T>>((int64_t)B * kx_slot);
        C<T>* ky = KY.get<C<T>>((int64_t)B * ky_slot);
        const BinMap bm = binmap();
        for (int q0 = 0; q0 < QC; q0 += B) {
          const int nq = std::min(B, QC - q0);
          k_kgen_x<T, Sh, WX><<<dim3(nblkK, 1, nq), NTX, 0, s>>>(
              mp_coef.as<double>(), R, mp_fa.as<int32_t>() + q0, mp_fb.as<int32_t>() + q0, pwx(), pwy(),
              pwz(), bm, kx, kx_slot, twp, nullptr, nh);
          launch_check("kgen(multipoles adjoint)");
          k_strided<T, Sh, W, -1, IN_WINDOW, OUT_DENSE><<<dim3(N / W, nz, nq), NT, 0, s>>>(
              kx, ky, kx_slot, ky_slot, (int64_t)ny * N, NN, N, N, pwy(), nullptr, nullptr, 0, nullptr, twp);
          launch_check("kgen_y(multipoles adjoint)");
          k_xscatter_dual<T, Sh, WX, true><<<(int)(NN / WX), NTX, 0, s>>>(
              line_set(), l_f.as<int32_t>(), cf, F, q0, nq, x, NC, twp, yl, nh, P);
          launch_check("xscatter(multipoles adjoint)");
          k_strided<T, Sh, W, -1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, nq), NT, 0, s>>>(
              x, x, NC, NC, NN, NN, N, N, 0, nullptr, nullptr, 0, nullptr, twp);
          launch_check("ypass(multipoles adjoint)");
          k_zdual_acc<T, Sh, W><<<dim3(N / W, N, 1), NT, 0, s>>>(x, NC, nq, ky, ky_slot, pwz(), A, twp);
          launch_check("zacc(multipoles adjoint)");
        }
      }
      galaxy_adjoint_tail(s, A, gb, 1, gd, gws_d, gwg_d, grad_w, twp);
    }
  }

  // fill the kernel-field store (when there is one) before a recorded body
  // uses it, so that the body's launch sequence is the same from the first call
  void ensure_dual_kernels(hipStream_t s) {
    C<T>* kc = kernel_store();
    if (kc && !kc_valid) {
      const int Q = (cfg.R + 1) / 2;
      const BinMap bm = binmap();
      for (int q0 = 0; q0 < Q; q0 += B)
        dual_kernels(s, q0, std::min(B, Q - q0), kc, tw.as<C<T>>(), bm, "dual_kgen", "dual_kgen_y");
      kc_valid = true;
    }
    if (v_zpass == 2) ensure_kernel_spectra(s);
  }

  static constexpr int64_t ks_slot() { return (int64_t)(N / 2 + 1) * (N / 2 + 1) * N; }

  // The kernel-spectrum store: allocated once when free memory holds it with
  // 4 GiB to spare, filled once per plan (from the window columns, kept or
  // regenerated).  Returns whether it is ready.
  bool ensure_kernel_spectra(hipStream_t s) {
    if (ks_valid) return true;
    const int Q = (cfg.R + 1) / 2;
    if (!ks_tried) {
      ks_tried = true;
      const size_t need = (size_t)Q * (size_t)ks_slot() * sizeof(C<T>);
      (void)KS.try_ensure(need);
    }
    if (!KS.p) return false;
    C<T>* kc = kernel_store();
    const BinMap bm = binmap();
    const int64_t ky_slot = (int64_t)win_len(pwz()) * NN;
    for (int q0 = 0; q0 < Q; q0 += B) {
      const int nq = std::min(B, Q - q0);
      const C<T>* ky = dual_kernels(s, q0, nq, kc, tw.as<C<T>>(), bm, "dual_kgen", "dual_kgen_y");
      k_kspec<T, Sh, W><<<dim3(N / W, N / 2 + 1, nq), NT, 0, s>>>(ky, ky_slot, pwz(),
                                                                  KS.as<C<T>>() + q0 * ks_slot(),
                                                                  ks_slot(), tw.as<C<T>>());
      launch_check("kspec");
    }
    if (kc) kc_valid = true;
    ks_valid = true;
    return true;
  }

  // the dual form's z passes read the kernel-spectrum store
  bool ks_path() const { return algo == 1 && v_zpass == 2 && ks_valid; }

  void forward_dual_pairs(hipStream_t s, C<T>* x, const C<T>* fg, const C<T>* twp, const BinMap& bm,
                          double* Sd, const float* wl) {
    const int R = cfg.R, F = cfg.F, Q = (R + 1) / 2;
    const int nz = win_len(pwz());
    const int64_t ky_slot = (int64_t)nz * NN;
    const double cb = (double)sizeof(C<T>);
    float* gv = GV.get<float>(std::max<int64_t>((int64_t)R * n_pairs, 1));
    C<T>* kc = kernel_store();
    const bool ksp = ks_path();
    for (int q0 = 0; q0 < Q; q0 += B) {
      const int nq = std::min(B, Q - q0);
      if (ksp) {
        // every stored kernel row once (the reads for the mirrored rows
        // ky, N - ky and planes kz, N - kz are meant to hit the caches)
        const double kb = (double)nq * (double)ks_slot();
        prof.run("dual_zconv", s, (kb + (double)NC + (double)nq * NC) * cb, [&] {
          k_zconv_ks<T, Sh, W><<<dim3(N / W, N, 1), NT, 0, s>>>(KS.as<C<T>>() + q0 * ks_slot(), ks_slot(),
                                                                nq, fg, x, NC, twp);
          launch_check("zconv(ks)");
        });
      } else {
        C<T>* ky = dual_kernels(s, q0, nq, kc, twp, bm, "dual_kgen", "dual_kgen_y");
        prof.run("dual_zconv", s, (double)(nq * ky_slot + NC + nq * NC) * cb, [&] {
          if (v_zpass == 0)
            k_zconv<T, Sh, W><<<dim3(N / W, N, 1), NT, 0, s>>>(ky, ky_slot, nq, pwz(), fg, x, NC, twp);
          else
            k_zconv<T, Sh, WH><<<dim3(N / WH, N, 1), WH * TPL, 0, s>>>(ky, ky_slot, nq, pwz(), fg, x,
                                                                    NC, twp);
          launch_check("zconv");
        });
      }
      prof.run("dual_yinv", s, 2.0 * nq * NC * cb, [&] {
        k_strided<T, Sh, W, 1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, nq), NT, 0, s>>>(
            x, x, NC, NC, NN, NN, N, N, 0, nullptr, nullptr, 0, nullptr, twp);
        launch_check("yinv(dual)");
      });
      if (n_pairs > 0) {
        const int zlen = N / kZSeg;
        // the y-transformed grids once, the point records, the gathered values
        const double bytes = (double)nq * NC * cb + (double)n_pairs * (20.0 + 8.0 * nq) + (double)NN * 4.0;
        prof.run("dual_xinv_gather", s, bytes, [&] {
          if (cfg.assignment == 1)
            k_xinv_gather_sweep_tsc<T, Sh, YTT><<<dim3((N + YTT - 1) / YTT, kZSeg, nq), (YTT + 2) * TPL, 0, s>>>(
                line_set(), l_p.as<int32_t>(), n_pairs, x, NC, zlen, 2 * q0, R, gv, twp);
          else
            k_xinv_gather_sweep<T, Sh, YTS><<<dim3((N + YTS - 1) / YTS, kZSeg, nq), (YTS + 1) * TPL, 0, s>>>(
                line_set(), l_p.as<int32_t>(), n_pairs, x, NC, zlen, 2 * q0, R, gv, twp);
          launch_check("xinv_gather(dual)");
        });
      }
    }
    const int K = reduce_chunks((int64_t)F * R);
    double* part = red_part.get<double>((int64_t)F * R * K);
    k_dual_reduce<<<dim3(F, R, K), 256, 0, s>>>(p_fs.as<int32_t>(), 1, p_wd.as<double>(), gv, n_pairs,
                                                R, bscale.as<float>(), part);
    k_sum_chunks<<<grid_for((int64_t)F * R), 256, 0, s>>>(part, (int64_t)F * R, K, Sd);
    launch_check("reduce(dual)");
    if (kc) kc_valid = true;
  }

  void forward_batched(hipStream_t s, C<T>* spec, const float* wl) {
    const int R = cfg.R;
    // bin sums: allocated here too, since the autotuner runs this body
    // without a preceding pgx_forward
    double* Sd = S.get<double>((int64_t)cfg.F * R);
    double* Sggd = Sgg.get<double>(R);
    const int ny = win_len(pwy()), nz = win_len(pwz());
    const int nblkE = (ny * nz + WX - 1) / WX;
    const int64_t p1_slot = (int64_t)nz * NN;
    const int64_t p2_slot = (int64_t)nz * ny * N;
    C<T>* x = X.get<C<T>>((int64_t)B * NC);
    C<T>* p1 = P1.get<C<T>>((int64_t)B * p1_slot);
    C<T>* p2 = P2.get<C<T>>((int64_t)B * p2_slot);
    C<T>* fg = Fg.get<C<T>>(NC);
    double* pt = part.get<double>((int64_t)B * nblkE * 2 * R);
    const C<T>* twp = tw.as<C<T>>();
    BinMap bm = binmap();
    // ---- galaxy field: spectrum (DC removed) and auto-correlation
    const double cb = (double)sizeof(C<T>);
    prof.run("gal_xscatter", s, (double)n_gal * (4 + 4 * sizeof(T)) + (double)NC * cb, [&] {
      xscatter((int)(NN / WX), g_tasks.as<int32_t>(), (int)NN, gal_set(), gslot_fa.as<int32_t>(),
               gslot_fb.as<int32_t>(), x, twp, nullptr, s);
      launch_check("xscatter(gal)");
    });
    prof.run("gal_ypass", s, 2.0 * NC * cb, [&] {
      k_strided<T, Sh, W, -1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, 1), NT, 0, s>>>(
          x, x, 0, 0, NN, NN, N, N, 0, nullptr, nullptr, 0, nullptr, twp);
      launch_check("ypass(gal)");
    });
    prof.run("gal_zpass", s, 2.0 * NC * cb + (double)p1_slot * cb, [&] {
      k_zcross<T, Sh, W, true, false, false><<<dim3(N / W, N, 1), NT, 0, s>>>(x, 0, nullptr, nullptr, 1, nullptr,
                                                                               fg, p1, 0, pwz(), twp);
      launch_check("zcross(gal)");
    });
    prof.run("gal_yinv", s, (double)(p1_slot + p2_slot) * cb, [&] {
      k_strided<T, Sh, W, 1, IN_DENSE, OUT_WINDOW><<<dim3(N / W, nz, 1), NT, 0, s>>>(
          p1, p2, p1_slot, p2_slot, NN, (int64_t)ny * N, N, N, pwy(), nullptr, nullptr, 0, nullptr,
          twp);
      launch_check("yinv(gal)");
    });
    prof.run("gal_xinv_bins", s, (double)p2_slot * cb, [&] {
      k_xinv_bins<T, Sh, WX, kRMax><<<dim3(nblkE, 1, 1), NTX, 0, s>>>(p2, p2_slot, pwx(), pwy(),
                                                                     pwz(), bm, R, pt, twp);
      launch_check("xinv_bins(gal)");
    });
    k_reduce_bins<<<dim3(2 * R, 1), 256, 0, s>>>(pt, nblkE, R, gslot_fa.as<int32_t>(),
                                                           gslot_fb.as<int32_t>(), Sggd);
    launch_check("reduce(gal)");
    if (algo == 1) {
      forward_dual_pairs(s, x, fg, twp, bm, Sd, wl);
      return;
    }
    // ---- pair fields, B field pairs per batch
    for (int k = 0; k < n_batches; ++k) {
      const int nb = std::min(B, cfg.n_fp - k * B);
      const int64_t t0 = batch_task_off[k], nt = batch_task_off[k + 1] - t0;
      const int32_t* fa = slot_fa.as<int32_t>() + (int64_t)k * B;
      const int32_t* fb = slot_fb.as<int32_t>() + (int64_t)k * B;
      const int32_t* fp = slot_fp.as<int32_t>() + (int64_t)k * B;
      const double pts = (double)batch_points(k) * (4 + 4 * sizeof(T));
      if (nt > 0) {
        prof.run("xscatter", s, pts + (double)nt * N * cb, [&] {
          xscatter((int)((nt + WX - 1) / WX), tasks_s.as<int32_t>() + t0, (int)nt, pair_set(), fa, fb, x,
                   twp, FSC.as<float>(), s);
          launch_check("xscatter");
        });
      }
      prof.run("ypass", s, (double)nt * N * cb + (double)nb * NC * cb, [&] {
        ypass_launch(v_ypass, x, nb, fp, s);
        launch_check("ypass");
      });
      prof.run("zpass_cross", s,
               (double)(nb + 1) * NC * cb + (double)nb * p1_slot * cb + (spec ? (double)nb * NC * cb : 0.0),
               [&] {
        const dim3 gz(N / W, N, 1);
        const uint8_t* pf = pflag.as<uint8_t>();
        if (spec && v_zpass == 0)
          k_zcross<T, Sh, W, false, true, true><<<gz, NT, 0, s>>>(x, NC, pf, fp, nb, fg, nullptr, p1,
                                                                  p1_slot, pwz(), twp, spec);
        else if (spec)
          k_zcross<T, Sh, W, false, true, false><<<gz, NT, 0, s>>>(x, NC, pf, fp, nb, fg, nullptr, p1,
                                                                   p1_slot, pwz(), twp, spec);
        else if (v_zpass == 0)
          k_zcross<T, Sh, W, false, false, true><<<gz, NT, 0, s>>>(x, NC, pf, fp, nb, fg, nullptr, p1,
                                                                   p1_slot, pwz(), twp);
        else
          k_zcross<T, Sh, W, false, false, false><<<gz, NT, 0, s>>>(x, NC, pf, fp, nb, fg, nullptr,
                                                                    p1, p1_slot, pwz(), twp);
        launch_check("zcross");
      });
      prof.run("yinv", s, (double)nb * (p1_slot + p2_slot) * cb, [&] {
        if (v_yinv == 0)
          k_strided<T, Sh, W, 1, IN_DENSE, OUT_WINDOW><<<dim3(N / W, nz, nb), NT, 0, s>>>(
              p1, p2, p1_slot, p2_slot, NN, (int64_t)ny * N, N, N, pwy(), nullptr, nullptr, 0,
              nullptr, twp);
        else
          k_strided<T, ShA, WA, 1, IN_DENSE, OUT_WINDOW><<<dim3(N / WA, nz, nb), NTA, 0, s>>>(
              p1, p2, p1_slot, p2_slot, NN, (int64_t)ny * N, N, N, pwy(), nullptr, nullptr, 0,
              nullptr, tw_alt.as<C<T>>());
        launch_check("yinv");
      });
      prof.run("xinv_bins", s, (double)nb * p2_slot * cb, [&] {
        k_xinv_bins<T, Sh, WX, kRMax><<<dim3(nblkE, 1, nb), NTX, 0, s>>>(p2, p2_slot, pwx(), pwy(),
                                                                        pwz(), bm, R, pt, twp);
        launch_check("xinv_bins");
      });
      k_reduce_bins<<<dim3(2 * R, nb), 256, 0, s>>>(pt, nblkE, R, fa, fb, Sd, FSC.as<float>());
      launch_check("reduce");
    }
  }

  // one field at a time, full transforms, global-atomic scatter, FP64 or FP32
  void scatter_plain(const PointSet<T>& ps, const int32_t* key, const int32_t* ls, int64_t k0,
                     int64_t k1, C<T>* grid, hipStream_t s) {
    k_fill_zero<T><<<4096, 256, 0, s>>>(grid, NC);
    launch_check("fill_zero");
    if (cfg.assignment == 1)
      k_scatter_atomic_tsc<T><<<2048, 256, 0, s>>>(ls, k0, k1, key, ps, N, grid);
    else
      k_scatter_atomic<T><<<2048, 256, 0, s>>>(ls, k0, k1, key, ps, N, grid);
    launch_check("scatter_atomic");
  }

  void fft3(C<T>* g, int dir, hipStream_t s) {
    const C<T>* twp = tw.as<C<T>>();
    if (dir < 0) {
      k_xdense<T, Sh, WX, -1><<<(int)(NN / WX), NTX, 0, s>>>(g, twp);
      k_strided<T, Sh, W, -1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, 1), NT, 0, s>>>(
          g, g, 0, 0, NN, NN, N, N, 0, nullptr, nullptr, 0, nullptr, twp);
      k_strided<T, Sh, W, -1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, 1), NT, 0, s>>>(
          g, g, 0, 0, N, N, NN, NN, 0, nullptr, nullptr, 0, nullptr, twp);
    } else {
      k_strided<T, Sh, W, 1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, 1), NT, 0, s>>>(
          g, g, 0, 0, N, N, NN, NN, 0, nullptr, nullptr, 0, nullptr, twp);
      k_strided<T, Sh, W, 1, IN_DENSE, OUT_DENSE><<<dim3(N / W, N, 1), NT, 0, s>>>(
          g, g, 0, 0, NN, NN, N, N, 0, nullptr, nullptr, 0, nullptr, twp);
      k_xdense<T, Sh, WX, 1><<<(int)(NN / WX), NTX, 0, s>>>(g, twp);
    }
    launch_check("fft3");
  }

  void bins_plain(const C<T>* h, const int32_t* fa, double* out, hipStream_t s) {
    const int R = cfg.R;
    const int64_t cube = (int64_t)win_len(pwx()) * win_len(pwy()) * win_len(pwz());
    const int nblk = grid_for(cube);
    double* pt = part.get<double>((int64_t)nblk * 2 * R);
    k_bins_dense<T, kRMax><<<nblk, 256, 0, s>>>(h, N, pwx(), pwy(), pwz(), binmap(), R, pt);
    launch_check("bins_dense");
    k_reduce_bins<<<dim3(2 * R, 1), 256, 0, s>>>(pt, nblk, R, fa, neg1.as<int32_t>(), out);
    launch_check("reduce_plain");
  }

  void forward_plain(hipStream_t s) {
    S.get<double>((int64_t)cfg.F * cfg.R);
    Sgg.get<double>(cfg.R);
    C<T>* g = Fg.get<C<T>>(NC);
    C<T>* h = X.get<C<T>>(NC);
    scatter_plain(gal_set(), g_key.as<int32_t>(), g_ls.as<int32_t>(), 0, NN, g, s);
    fft3(g, -1, s);
    k_zero_dc<T><<<1, 64, 0, s>>>(g);
    k_copy<T><<<4096, 256, 0, s>>>(g, h, NC);
    k_mul_conj<T, true><<<4096, 256, 0, s>>>(h, nullptr, NC);
    launch_check("gal_product");
    fft3(h, 1, s);
    bins_plain(h, gslot_fa.as<int32_t>(), Sgg.as<double>(), s);
    for (int f = 0; f < cfg.F; ++f) {
      scatter_plain(pair_set(), p_key.as<int32_t>(), p_fs.as<int32_t>(), f, f + 1, h, s);
      fft3(h, -1, s);
      k_mul_conj<T, false><<<4096, 256, 0, s>>>(h, g, NC);
      launch_check("product");
      fft3(h, 1, s);
      bins_plain(h, fidx.as<int32_t>() + f, S.as<double>(), s);
    }
  }
};

}  // namespace pgx
