// C-ABI of the pair-galaxy correlation library: plan creation and validation,
// output-bin tables, pair-bin volumes, and dispatch to the engines.
#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <utility>

#include "pgx_engine.hpp"

namespace pgx {
EngineBase* make_engine_f32(const PlanCfg& c);
EngineBase* make_engine_f64(const PlanCfg& c);
size_t memory_bound_f32(const PlanCfg& c, int64_t n, int64_t P, bool spectra);
size_t memory_bound_f64(const PlanCfg& c, int64_t n, int64_t P, bool spectra);
}  // namespace pgx

struct pgx_plan {
  pgx::PlanCfg cfg;
  bool keep_spectra = false;
  bool use_graphs = true;
  // caller-owned workspace (null base: the plan allocates its own memory);
  // declared before the engine, whose buffers it may hold, so that it
  // outlives them
  pgx::Heap ws;
  mutable std::string last_error;  // message of the last failed call on this plan
  std::unique_ptr<pgx::EngineBase> eng;  // created on first device use
  pgx::EngineBase& engine() {
    if (!eng) {
      pgx::EngineBase* e = cfg.precision == PGX_FP32_BATCHED ? pgx::make_engine_f32(cfg)
                                                             : pgx::make_engine_f64(cfg);
      PGX_REQUIRE(e != nullptr, PGX_ENOTSUP, "unsupported grid size");
      eng.reset(e);
    }
    return *eng;
  }
};

namespace {

thread_local std::string g_last_error;

pgx_status fail(const pgx_plan* plan, pgx_status code, const std::string& msg) {
  g_last_error = msg;
  if (plan) plan->last_error = msg;
  return code;
}
pgx_status fail(pgx_status code, const std::string& msg) { return fail(nullptr, code, msg); }

// The plan's workspace is the current Heap for the duration of a call.
struct HeapScope {
  pgx::Heap* prev;
  explicit HeapScope(const pgx_plan* plan) : prev(pgx::t_heap) {
    pgx::t_heap = (plan && plan->ws.base) ? const_cast<pgx::Heap*>(&plan->ws) : nullptr;
  }
  ~HeapScope() { pgx::t_heap = prev; }
};

template <typename F> pgx_status guarded(const pgx_plan* plan, F&& f) {
  try {
    HeapScope hs(plan);
    f();
    return PGX_OK;
  } catch (const pgx::Error& e) {
    return fail(plan, e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(plan, PGX_ENOSPACE, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(plan, PGX_EHIP, e.what());
  } catch (...) {
    return fail(plan, PGX_EHIP, "unknown error");
  }
}
template <typename F> pgx_status guarded(F&& f) {
  return guarded(static_cast<const pgx_plan*>(nullptr), std::forward<F>(f));
}

// ----------------------------------------------------------------------------
// Fixed scratch of the allocation-free forward: one array per device, its
// address looked up once per device (the array's host-side name is not a
// device address).
// ----------------------------------------------------------------------------
constexpr size_t kFixedScratchBytes = (size_t)96 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
std::atomic<uint64_t> g_session_id{0};

void* fixed_scratch() {
  int dev = 0;
  PGX_HIP(hipGetDevice(&dev));
  PGX_REQUIRE(dev >= 0 && dev < kMaxDevices, PGX_ENOTSUP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    PGX_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    PGX_REQUIRE(ptr != nullptr, PGX_EHIP, "no device address for the fixed scratch");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// Bytes the FP64 plain forward takes from the fixed scratch: the galaxy
// spectrum and the field grid (complex FP64, N^3 each), bin partials, pair
// weights, per-field sums, the finalisation's spare outputs, each carved on a
// 256-byte boundary.
size_t fixed_forward_bytes(const pgx::PlanCfg& c, int64_t n_gal, int64_t n_pairs) {
  auto r = [](double b) { return (size_t)(std::ceil(std::max(b, 1.0) / 256.0) * 256.0); };
  const double N = c.N, F = c.F, R = c.R;
  const double cube = (2.0 * c.pw[0] + 1) * (2.0 * c.pw[1] + 1) * (2.0 * c.pw[2] + 1);
  const double nblk = std::ceil(cube / 256.0);
  const double K = pgx::reduce_chunks(c.F);
  size_t b = 2 * r(N * N * N * 16.0);  // galaxy spectrum, field grid
  b += r(nblk * 2 * R * 8) + r(F * R * 8) + r(R * 8);
  b += r(std::max<double>((double)n_pairs, 1.0) * 8) + r(F * K * 8) + r(F * 8) + r(F * 4);
  b += r(pgx::kWtBlocks * 8.0) + r(8) + r((3 * F * R + F + R + 8) * 8) + r(4);
  b += r(std::max<double>((double)n_gal, 1.0) * 4);  // copy of the weights
  return b;
}

// A fixed-scratch session for the duration of one call (restores the plan's
// buffers on exit, also after an error).
struct SessionScope {
  pgx::Session sess;
  SessionScope(void* base, size_t bytes) {
    sess.heap.reset(base, bytes);
    sess.id = ++g_session_id;
    pgx::t_session = &sess;
  }
  ~SessionScope() {
    sess.restore();
    pgx::t_session = nullptr;
  }
};

std::vector<double> edges(const double* p, int n, const char* name) {
  PGX_REQUIRE(n >= 1 && p != nullptr, PGX_EINVAL, std::string(name) + ": need n >= 1 and edges");
  std::vector<double> v(p, p + n + 1);
  for (int i = 0; i <= n; ++i)
    PGX_REQUIRE(std::isfinite(v[i]), PGX_EINVAL, std::string(name) + ": non-finite edge");
  for (int i = 0; i < n; ++i)
    PGX_REQUIRE(v[i] < v[i + 1], PGX_EINVAL, std::string(name) + ": edges must be strictly ascending");
  return v;
}

void build_cfg(const pgx_params* p, pgx::PlanCfg& c) {
  PGX_REQUIRE(p != nullptr, PGX_EINVAL, "params is NULL");
  PGX_REQUIRE(std::isfinite(p->L) && p->L > 0, PGX_EINVAL, "L must be finite and > 0");
  const int N = p->N;
  PGX_REQUIRE(N >= 64 && N <= 1024 && (N & (N - 1)) == 0, PGX_ENOTSUP,
              "N must be a power of two in [64, 1024]");
  PGX_REQUIRE(p->precision == PGX_FP64_PLAIN || p->precision == PGX_FP32_BATCHED, PGX_EINVAL,
              "unknown precision");
  PGX_REQUIRE(p->pair_mode == PGX_PAIR_S_MU || p->pair_mode == PGX_PAIR_RP_PI, PGX_EINVAL,
              "unknown pair_mode");
  PGX_REQUIRE(p->out_mode >= PGX_OUT_SHELL && p->out_mode <= PGX_OUT_GSW, PGX_EINVAL,
              "unknown out_mode");
  PGX_REQUIRE(p->qeff_mode >= PGX_QEFF_NOTSQ && p->qeff_mode <= PGX_QEFF_CONST_XIW, PGX_EINVAL,
              "unknown qeff_mode");
  PGX_REQUIRE(p->assignment == PGX_ASSIGN_CIC || p->assignment == PGX_ASSIGN_TSC, PGX_EINVAL,
              "unknown assignment");
  c.L = p->L;
  c.N = N;
  c.precision = p->precision;
  c.pair_mode = p->pair_mode;
  c.out_mode = p->out_mode;
  c.qeff_mode = p->qeff_mode;
  c.assignment = p->assignment;
  c.xi_w_const = p->xi_w_const;
  c.batch = p->batch;
  c.pair_dmax = p->pair_dmax;
  c.p1 = edges(p->p1_edges, p->n_p1, "p1_edges");
  c.p2 = edges(p->p2_edges, p->n_p2, "p2_edges");
  const bool gsw = c.out_mode == PGX_OUT_GSW;
  if (gsw) {
    const double w[5] = {p->w_sigma, p->w_rs, p->w_s0, p->w_rcut, p->w_rmax};
    for (double v : w) PGX_REQUIRE(std::isfinite(v), PGX_EINVAL, "weighting parameters must be finite");
    PGX_REQUIRE(p->w_sigma > 0 && p->w_s0 > 0 && p->w_rcut >= 0 && p->w_rcut < p->w_rmax, PGX_EINVAL,
                "weighting parameters need w_sigma > 0, w_s0 > 0, 0 <= w_rcut < w_rmax");
    c.o1 = {p->w_rcut, p->w_rmax};  // radial extent: the window and the cut test
  } else {
    c.o1 = edges(p->o1_edges, p->n_o1, "o1_edges");
    if (c.out_mode != PGX_OUT_SHELL) c.o2 = edges(p->o2_edges, p->n_o2, "o2_edges");
  }
  PGX_REQUIRE(c.p1[0] >= 0, PGX_EINVAL, "p1_edges must be >= 0");
  PGX_REQUIRE(c.p2[0] >= 0, PGX_EINVAL, "p2_edges must be >= 0");
  PGX_REQUIRE(c.o1[0] >= 0, PGX_EINVAL, "o1_edges must be >= 0");
  if (c.pair_mode == PGX_PAIR_S_MU) {
    PGX_REQUIRE(c.p2.back() <= 1.0, PGX_EINVAL, "|mu| edges must lie in [0, 1]");
    c.smax = c.p1.back();
  } else {
    PGX_REQUIRE(std::isfinite(c.pair_dmax) && c.pair_dmax > 0, PGX_EINVAL, "pair_dmax must be > 0");
    c.smax = std::min(c.pair_dmax, std::hypot(c.p1.back(), c.p2.back()));
  }
  PGX_REQUIRE(c.smax > 0 && c.smax < c.L / 3.0, PGX_EINVAL,
              "maximum pair separation must be in (0, L/3)");
  if (c.out_mode == PGX_OUT_R_MU) {
    PGX_REQUIRE(c.o2[0] >= 0 && c.o2.back() <= 1.0, PGX_EINVAL, "output |mu| edges must lie in [0, 1]");
  } else if (c.out_mode == PGX_OUT_RP_PI) {
    PGX_REQUIRE(c.o2[0] >= 0, PGX_EINVAL, "output |pi| edges must be >= 0");
  }
  const double delta = c.L / N;
  double top1 = c.o1.back();
  double topz = c.out_mode == PGX_OUT_RP_PI ? c.o2.back() : top1;
  PGX_REQUIRE(top1 < c.L / 2 && topz < c.L / 2, PGX_EINVAL, "output bins must stay below L/2");
  const int w1 = (int)std::floor(top1 / delta), wz = (int)std::floor(topz / delta);
  PGX_REQUIRE(w1 <= N / 2 - 1 && wz <= N / 2 - 1, PGX_EINVAL, "output window reaches N/2");
  c.pw[0] = w1;
  c.pw[1] = w1;
  c.pw[2] = wz;
  const int n_p1 = (int)c.p1.size() - 1, n_p2 = (int)c.p2.size() - 1;
  c.F = n_p1 * n_p2;
  c.n_fp = (c.F + 1) / 2;
  const int n_o2 = (c.out_mode == PGX_OUT_SHELL || gsw) ? 1 : (int)c.o2.size() - 1;
  c.R = ((int)c.o1.size() - 1) * n_o2;
  PGX_REQUIRE(c.R <= pgx::kRMax, PGX_ENOTSUP, "too many output bins");
  PGX_REQUIRE((int64_t)c.F * N * N + 1 < (int64_t)INT32_MAX, PGX_ENOTSUP, "n_fields * N^2 too large");
  // bin tables
  pgx::HostBins& hb = c.bins;
  hb.mode = c.out_mode;
  hb.n2 = n_o2;
  if (gsw) {
    hb.g[0] = delta;
    hb.g[1] = p->w_s0;
    hb.g[2] = p->w_rs;
    hb.g[3] = 1.0 / (2.0 * p->w_sigma * p->w_sigma);
    const double qc = p->w_rcut / delta, qm = p->w_rmax / delta;
    hb.rcut2 = qc * qc;
    hb.rmax2 = qm * qm;
  } else if (c.out_mode == PGX_OUT_RP_PI) {
    hb.lut1 = pgx::bin_lut(c.o1, delta, (int64_t)2 * w1 * w1 + 1);
    hb.lut2 = pgx::bin_lut(c.o2, delta, (int64_t)wz * wz + 1);
  } else {
    hb.lut1 = pgx::bin_lut(c.o1, delta, (int64_t)3 * w1 * w1 + 1);
    if (c.out_mode == PGX_OUT_R_MU) {
      hb.mu2.resize(c.o2.size());
      for (size_t i = 0; i < c.o2.size(); ++i) hb.mu2[i] = c.o2[i] * c.o2[i];
    }
  }
  c.nb.assign(c.R, 0);
  c.nbw.assign(c.R, 0.0);
  for (int k = -wz; k <= wz; ++k)
    for (int j = -w1; j <= w1; ++j)
      for (int i = -w1; i <= w1; ++i) {
        const int b = hb.classify(i, j, k);
        if (b >= 0) {
          c.nb[b] += 1;
          c.nbw[b] += hb.weight(i, j, k);
        }
      }
  // pair-bin volumes
  c.vol.clear();
  for (int a = 0; a < n_p1; ++a)
    for (int b = 0; b < n_p2; ++b)
      c.vol.push_back(c.pair_mode == PGX_PAIR_S_MU
                          ? pgx::vol_s_mu(c.p1[a], c.p1[a + 1], c.p2[b], c.p2[b + 1])
                          : pgx::vol_rp_pi(c.p1[a], c.p1[a + 1], c.p2[b], c.p2[b + 1], c.pair_dmax));
}

}  // namespace

extern "C" {

pgx_status pgx_plan_create(const pgx_params* params, pgx_plan** out) {
  if (!out) return fail(PGX_EINVAL, "out is NULL");
  *out = nullptr;
  return guarded([&] {
    std::unique_ptr<pgx_plan> p(new pgx_plan());
    build_cfg(params, p->cfg);
    *out = p.release();
  });
}

pgx_status pgx_plan_destroy(pgx_plan* plan) {
  return guarded([&] { delete plan; });
}

pgx_status pgx_plan_info(const pgx_plan* plan, int32_t* n_fields, int32_t* n_out, int32_t* window) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  if (n_fields) *n_fields = plan->cfg.F;
  if (n_out) *n_out = plan->cfg.R;
  if (window)
    for (int i = 0; i < 3; ++i) window[i] = plan->cfg.pw[i];
  return PGX_OK;
}

pgx_status pgx_out_counts(const pgx_plan* plan, int64_t* n_b) {
  if (!plan || !n_b) return fail(plan, PGX_EINVAL, "NULL argument");
  for (int b = 0; b < plan->cfg.R; ++b) n_b[b] = plan->cfg.nb[b];
  return PGX_OK;
}

pgx_status pgx_out_norms(const pgx_plan* plan, double* norm) {
  if (!plan || !norm) return fail(plan, PGX_EINVAL, "NULL argument");
  for (int b = 0; b < plan->cfg.R; ++b) norm[b] = plan->cfg.nbw[b];
  return PGX_OK;
}

pgx_status pgx_field_volumes(const pgx_plan* plan, double* vol) {
  if (!plan || !vol) return fail(plan, PGX_EINVAL, "NULL argument");
  for (int f = 0; f < plan->cfg.F; ++f) vol[f] = plan->cfg.vol[f];
  return PGX_OK;
}

pgx_status pgx_pairs_build(pgx_plan* plan, const double* x, const double* y, const double* z,
                           const float* w, int64_t n_gal, void* stream, int64_t* n_pairs,
                           int64_t* counts, double* wsum) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    plan->engine().pairs_build(x, y, z, w, n_gal, (hipStream_t)stream, n_pairs, counts, wsum);
  });
}

pgx_status pgx_pairs_export(pgx_plan* plan, int32_t* field, int32_t* i, int32_t* j, void* stream) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] { plan->engine().pairs_export(field, i, j, (hipStream_t)stream); });
}

pgx_status pgx_forward(pgx_plan* plan, const float* w, void* stream, double* wsum, double* xi_gg,
                       double* xi_pg, double* xi_dp, double* b_pg, double* q_eff) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    auto& e = plan->engine();
    e.keep_spectra = plan->keep_spectra;
    e.use_graphs = plan->use_graphs;
    e.forward(w, (hipStream_t)stream, wsum, xi_gg, xi_pg, xi_dp, b_pg, q_eff);
  });
}

pgx_status pgx_backward(pgx_plan* plan, void* stream, const double* g_b_pg, const double* g_q_eff,
                        const double* g_xi_pg, const double* g_xi_gg, const double* g_xi_dp,
                        float* grad_w) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    auto& e = plan->engine();
    e.use_graphs = plan->use_graphs;
    e.backward((hipStream_t)stream, g_b_pg, g_q_eff, g_xi_pg, g_xi_gg, g_xi_dp, grad_w);
  });
}

pgx_status pgx_projected(pgx_plan* plan, void* stream, const double* xi_dp, double* w_p) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] { plan->engine().projected((hipStream_t)stream, xi_dp, w_p, false); });
}

pgx_status pgx_projected_backward(pgx_plan* plan, void* stream, const double* g_w_p, double* g_xi_dp) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] { plan->engine().projected((hipStream_t)stream, g_w_p, g_xi_dp, true); });
}

pgx_status pgx_multipoles(pgx_plan* plan, void* stream, int32_t lmax, double* xi_l) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] { plan->engine().multipoles((hipStream_t)stream, lmax, xi_l); });
}

pgx_status pgx_multipoles_backward(pgx_plan* plan, void* stream, const double* g_xi_l, float* grad_w) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] { plan->engine().multipoles_backward((hipStream_t)stream, g_xi_l, grad_w); });
}

pgx_status pgx_keep_spectra(pgx_plan* plan, int32_t enable) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] { plan->keep_spectra = enable != 0; });
}

pgx_status pgx_autotune(pgx_plan* plan, void* stream, int32_t* schedule) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] { plan->engine().autotune((hipStream_t)stream, schedule); });
}

pgx_status pgx_schedule(pgx_plan* plan, int32_t* schedule) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  if (!schedule) return fail(plan, PGX_EINVAL, "schedule is NULL");
  return guarded(plan, [&] { plan->engine().schedule_info(schedule); });
}

pgx_status pgx_dual_check(pgx_plan* plan, double* disagreement) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  if (!disagreement) return fail(plan, PGX_EINVAL, "disagreement is NULL");
  return guarded(plan, [&] { *disagreement = plan->eng ? plan->eng->dual_disagreement : -1.0; });
}

pgx_status pgx_dual_recheck(pgx_plan* plan, void* stream, int32_t fallback, double* disagreement) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  if (!disagreement) return fail(plan, PGX_EINVAL, "disagreement is NULL");
  return guarded(plan, [&] {
    *disagreement = plan->engine().recheck_dual((hipStream_t)stream, fallback != 0);
  });
}

pgx_status pgx_set_schedule(pgx_plan* plan, void* stream, const int32_t* schedule) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  if (!schedule) return fail(plan, PGX_EINVAL, "schedule is NULL");
  return guarded(plan, [&] { plan->engine().set_schedule(schedule, (hipStream_t)stream); });
}

pgx_status pgx_use_graphs(pgx_plan* plan, int32_t enable) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] { plan->use_graphs = enable != 0; });
}

pgx_status pgx_graph_replays(pgx_plan* plan, int64_t* forward, int64_t* backward) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    const int64_t f = plan->eng ? plan->eng->gf.replays : 0;
    const int64_t b = plan->eng ? plan->eng->gb.replays : 0;
    if (forward) *forward = f;
    if (backward) *backward = b;
  });
}

pgx_status pgx_profile(pgx_plan* plan, int32_t enable) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    auto& pr = plan->engine().prof;
    pr.reset();
    pr.on = enable != 0;
  });
}

pgx_status pgx_profile_read(pgx_plan* plan, int32_t k, const char** name, int64_t* launches,
                            double* ms, double* bytes) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    auto& pr = plan->engine().prof;
    pr.collect();
    PGX_REQUIRE(k >= 0 && k < (int32_t)pr.cats.size(), PGX_EINVAL, "no such profile entry");
    const auto& c = pr.cats[k];
    if (name) *name = c.name.c_str();
    if (launches) *launches = c.launches;
    if (ms) *ms = c.ms;
    if (bytes) *bytes = c.bytes;
  });
}

#ifndef PGX_SOURCE_SHA256
#define PGX_SOURCE_SHA256 "unknown"
#endif
const char* pgx_build_digest(void) { return PGX_SOURCE_SHA256; }

const char* pgx_last_error(const pgx_plan* plan) {
  return plan ? plan->last_error.c_str() : g_last_error.c_str();
}

pgx_status pgx_workspace_bytes(const pgx_plan* plan, int64_t n_gal, int64_t n_pairs, size_t* bytes) {
  if (!plan || !bytes) return fail(plan, PGX_EINVAL, "NULL argument");
  if (n_gal < 0 || n_pairs < 0) return fail(plan, PGX_EINVAL, "negative size");
  return guarded(plan, [&] {
    *bytes = plan->cfg.precision == PGX_FP32_BATCHED
                 ? pgx::memory_bound_f32(plan->cfg, n_gal, n_pairs, plan->keep_spectra)
                 : pgx::memory_bound_f64(plan->cfg, n_gal, n_pairs, false);
  });
}

pgx_status pgx_set_workspace(pgx_plan* plan, void* ws, size_t bytes) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  if (ws && (reinterpret_cast<uintptr_t>(ws) & (pgx::Heap::kAlign - 1)) != 0)
    return fail(plan, PGX_EINVAL, "workspace must be 256-byte aligned");
  if (ws && bytes < pgx::Heap::kAlign) return fail(plan, PGX_EINVAL, "workspace too small");
  return guarded(plan, [&] {
    if (plan->eng) PGX_HIP(hipDeviceSynchronize());
    {
      HeapScope hs(plan);  // the old buffers go back where they came from
      plan->eng.reset();
    }
    plan->ws.reset(ws, ws ? bytes : 0);
  });
}

pgx_status pgx_workspace_used(const pgx_plan* plan, size_t* in_use, size_t* peak) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  if (in_use) *in_use = plan->ws.in_use;
  if (peak) *peak = plan->ws.peak;
  return PGX_OK;
}

pgx_status pgx_forward_fixed(pgx_plan* plan, const float* w, void* stream, double* wsum,
                             double* xi_gg, double* xi_pg, double* xi_dp, double* b_pg,
                             double* q_eff) {
  if (!plan) return fail(PGX_EINVAL, "plan is NULL");
  return guarded(plan, [&] {
    PGX_REQUIRE(plan->cfg.precision == PGX_FP64_PLAIN, PGX_ENOTSUP,
                "pgx_forward_fixed serves PGX_FP64_PLAIN plans");
    auto& e = plan->engine();
    PGX_REQUIRE(e.built, PGX_ESTATE, "pgx_pairs_build has not been called");
    const size_t need = fixed_forward_bytes(plan->cfg, e.gal_count(), e.pair_count());
    PGX_REQUIRE(need <= kFixedScratchBytes, PGX_ENOSPACE,
                "pgx_forward_fixed: the forward needs " + std::to_string(need) +
                    " bytes of work memory, the fixed scratch holds " +
                    std::to_string(kFixedScratchBytes));
    void* base = fixed_scratch();
    const bool ug = e.use_graphs;
    e.use_graphs = false;  // eager: nothing recorded points into the scratch
    try {
      SessionScope ss(base, kFixedScratchBytes);
      e.forward(w, (hipStream_t)stream, wsum, xi_gg, xi_pg, xi_dp, b_pg, q_eff);
    } catch (...) {
      e.use_graphs = ug;
      e.forward_done = false;
      throw;
    }
    e.use_graphs = ug;
    e.forward_done = false;  // its state lived in the scratch
  });
}

}  // extern "C"
