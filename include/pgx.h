/*
 * pgx.h - pair-galaxy cross-correlation on one AMD Instinct MI355X (gfx950).
 *
 * Computes, for a periodic box of galaxies, the estimator of Yuan, Eisenstein
 * & Garrison (2017), "Using galaxy pairs to investigate the three-point
 * correlation function in the squeezed limit":
 *   - close galaxy pairs binned by separation (s, |mu|) or (r_p, |pi|), each
 *     bin a "pair field" of pair midpoints (Implementation section, pair
 *     catalogue; Methodology, equation delta_pi_x);
 *   - each pair field's cross-correlation with the galaxy field on an N^3
 *     grid, averaged over lattice-vector bins: xi_pg(f, b); the galaxy
 *     auto-correlation xi_gg(b) (Methodology, equation bpg_initial with the
 *     weight W taken as the normalised indicator of one separation bin);
 *   - xi(d_p) of each pair bin from weighted pair counts (2PCF section,
 *     equation 2PCF_d_collapsed), b_pg = xi_pg / xi_gg (Introduction, eq. 1)
 *     and Q_eff (Methodology, equations Qeff and Qeff_notsq).
 *
 * Conventions
 *   - Lengths in the caller's unit (Mpc/h).  Line of sight = z axis.
 *   - Grid node (a, b, c) sits at (a, b, c) * L / N; cloud-in-cell assignment
 *     unless the plan asks for TSC.
 *   - Pair (i, j), i < j by catalogue index, has d = x_j - x_i folded once
 *     into [-L/2, L/2); position x_i + d/2 wrapped into [0, L); weight w_i w_j.
 *   - Bins are half-open [e_k, e_{k+1}) and decided on squares against e*e in
 *     FP64; the top |mu| edge is closed.  Field index f = b1 * n_p2 + b2,
 *     output bin index b = o1 * n_o2 + o2 (n_o2 = 1 for shells).
 *   - Arrays marked "device" are HIP device memory owned by the caller; the
 *     library never frees them.  Work memory: by default the plan allocates
 *     its own (grown on demand, released by pgx_plan_destroy); with a
 *     workspace attached (pgx_set_workspace) every device buffer of the plan
 *     is placed in that caller-owned region instead and the plan calls
 *     neither hipMalloc nor hipFree.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *     on it; calls that return host values synchronise it (stated below).
 *   - Every call returns a pgx_status; no exception or abort crosses the ABI.
 *     On a non-OK status pgx_last_error(plan) describes the failure.
 *   - A plan is not thread-safe: use one plan per host thread and stream.
 *   - Fault injection, for tests of the error paths: while the environment
 *     variable PGX_DEBUG_FAIL_ALLOC holds n >= 1, the n-th allocation from the
 *     HIP allocator (counted from when the variable took that value) fails as
 *     an out-of-memory error would: calls needing that buffer return
 *     PGX_EHIP, optional stores are skipped.  The plan stays usable.
 */
#ifndef PGX_H
#define PGX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pgx_plan pgx_plan;

typedef enum {
  PGX_OK = 0,
  PGX_EINVAL = 1,   /* invalid argument or input data */
  PGX_ENOSPACE = 2, /* device memory exhausted */
  PGX_EHIP = 3,     /* HIP runtime error */
  PGX_ENOTSUP = 4,  /* unsupported size (N not a power of two in [64, 1024], too many pairs) */
  PGX_ESTATE = 5    /* call out of order (e.g. forward before pgx_pairs_build) */
} pgx_status;

typedef enum { PGX_PAIR_S_MU = 0, PGX_PAIR_RP_PI = 1 } pgx_pair_mode;
typedef enum { PGX_OUT_SHELL = 0, PGX_OUT_R_MU = 1, PGX_OUT_RP_PI = 2, PGX_OUT_GSW = 3 } pgx_out_mode;
typedef enum { PGX_FP64_PLAIN = 0, PGX_FP32_BATCHED = 1 } pgx_precision;
typedef enum { PGX_QEFF_NOTSQ = 0, PGX_QEFF_SQUEEZED = 1, PGX_QEFF_CONST_XIW = 2 } pgx_qeff_mode;
typedef enum { PGX_ASSIGN_CIC = 0, PGX_ASSIGN_TSC = 1 } pgx_assignment;

/*
 * Plan parameters.  Edge arrays are HOST arrays of n+1 strictly ascending
 * values, copied at plan creation.
 *   pair_mode S_MU : p1 = s edges (> 0 at the top), p2 = |mu| edges in [0, 1].
 *   pair_mode RP_PI: p1 = r_p edges, p2 = |pi| edges (>= 0), pair_dmax = sphere
 *                    radius (pairs kept iff |d| < pair_dmax).
 *   out_mode SHELL : o1 = r edges (o2 ignored); R_MU: o1 = r, o2 = |mu| in
 *                    [0, 1]; RP_PI: o1 = r_p, o2 = |pi|.
 *            GSW   : one output "bin" weighted by the paper's Gaussian-sigmoid
 *                    weighting function (Section "weighting", equation
 *                    weighting): with r_perp, r_par the lattice offset's
 *                    components across and along the line of sight (z),
 *                    W = sigmoid(w_s0 (r_perp - w_rs)) exp(-(r_perp^2 +
 *                    r_par^2) / (2 w_sigma^2)) where r_perp >= w_rcut and
 *                    |r| <= w_rmax, 0 elsewhere (the normalisation constant
 *                    cancels; w_rmax cuts the Gaussian tail off the lattice
 *                    window).  xi = sum_r W(r) C(r) / sum_r W(r), so b_pg is
 *                    the paper's estimator (equation bpg_initial) with W.
 *                    o1 / o2 are ignored (may be NULL).
 *   Requirements: the maximum pair separation < L/3 (cell list with at least
 *   3 cells per side); the largest output edge (w_rmax for GSW) < L/2, with
 *   w_sigma > 0, w_s0 > 0, 0 <= w_rcut < w_rmax; N a power of two in
 *   [64, 1024]; n_fields * N^2 < 2^31.
 *   precision FP64_PLAIN: one field at a time in FP64 (transforms, sums).
 *             FP32_BATCHED: fields paired into complex grids, FP32 transforms
 *             and products, FP64 bin sums, normalisations and ratios.
 *   qeff_mode NOTSQ (default, equation Qeff_notsq with xi(d_w) := xi_gg(b)),
 *             SQUEEZED (equation Qeff), CONST_XIW (Qeff_notsq with xi(d_w) =
 *             xi_w_const, the paper's weighting-function table value).
 *   batch: field pairs per batch on the batched path (0 = automatic).
 *   assignment: mass assignment of galaxies and pair midpoints to the grid.
 *             CIC (default; every path), or TSC, the paper's triangular-
 *             shaped cloud (Implementation section, "Mass assignment
 *             function": the point spreads over its nearest node and both
 *             neighbours on each axis with weights 3/4 - d^2 and
 *             (1/2 -+ d)^2 / 2, d the offset from that node in cells; ties
 *             at d = 1/2 go to the lower node).  On FP32_BATCHED plans TSC
 *             runs in both evaluations, forward and adjoint (the dual form
 *             keys its line-major pair catalogue by each midpoint's nearest
 *             node and gathers over the 3 x 3 lines around it); the
 *             multipoles refuse TSC plans (ENOTSUP).
 */
typedef struct {
  double L;
  int32_t N;
  int32_t precision;
  int32_t pair_mode;
  int32_t n_p1;
  const double* p1_edges;
  int32_t n_p2;
  const double* p2_edges;
  double pair_dmax;
  int32_t out_mode;
  int32_t n_o1;
  const double* o1_edges;
  int32_t n_o2;
  const double* o2_edges;
  int32_t qeff_mode;
  double xi_w_const;
  int32_t batch;
  /* out_mode GSW only */
  double w_sigma, w_rs, w_s0, w_rcut, w_rmax;
  int32_t assignment;
} pgx_params;

/* Create a plan.  Validates the parameters (PGX_EINVAL / PGX_ENOTSUP) and
 * builds the host-side bin tables; touches no device.  Device tables and
 * work memory are created on the current HIP device at the first
 * pgx_pairs_build, and the plan stays bound to that device. */
pgx_status pgx_plan_create(const pgx_params* params, pgx_plan** out);

/* Release the plan and all device memory it owns.  NULL is accepted. */
pgx_status pgx_plan_destroy(pgx_plan* plan);

/* Sizes: number of pair fields F, output bins R, and the half-widths of the
 * lattice window holding every output bin (window[3], in grid cells). */
pgx_status pgx_plan_info(const pgx_plan* plan, int32_t* n_fields, int32_t* n_out,
                         int32_t* window);

/* Exact lattice-vector count n_b of every output bin (HOST array [R]); for
 * GSW the number of lattice vectors with W > 0. */
pgx_status pgx_out_counts(const pgx_plan* plan, int64_t* n_b);

/* Normalisation of every output bin (HOST array [R]), the denominator of xi:
 * n_b for the indicator bins, sum_r W(r) over the lattice window for GSW
 * (FP64). */
pgx_status pgx_out_norms(const pgx_plan* plan, double* norm);

/* Volume of every pair bin (HOST array [F]) used by xi(d_p): the exact
 * (s, |mu|) shell-sector volume, or the (r_p, |pi|) annulus-slab volume cut by
 * the sphere |d| < pair_dmax, both signs of mu or pi included. */
pgx_status pgx_field_volumes(const pgx_plan* plan, double* vol);

/*
 * Pair catalogue (steps: validate, cell list, close-pair search with integer
 * keys, bucketing by field and grid line) and the galaxy point set.  Every
 * unordered pair closer than the largest pair separation is kept (a close
 * triplet gives three pairs) and sits at its midpoint (Implementation
 * section, pair catalogue; Methodology, equation delta_pi_x).
 *   x, y, z: device FP64 [n_gal] positions in [0, L).
 *   w:       device FP32 [n_gal] galaxy weights (>= 0, finite) or NULL (unit
 *            weights); read only for validation and wsum.
 *   n_pairs: HOST out, total number of pairs (this call synchronises stream).
 *   counts:  device int64 [F] out (nullable), pairs per field.
 *   wsum:    device FP64 [F] out (nullable), sum of pair weights w_i w_j per
 *            field (the weighted pair count of xi(d_p), 2PCF section).
 * Inputs are not referenced after the call returns.  Errors: EINVAL for
 * non-finite or out-of-box positions, invalid weights, n_gal < 0 or >= 2^31;
 * ENOTSUP when the pair count reaches 2^31; ENOSPACE when the workspace (if
 * attached) is too small.
 */
pgx_status pgx_pairs_build(pgx_plan* plan, const double* x, const double* y, const double* z,
                           const float* w, int64_t n_gal, void* stream, int64_t* n_pairs,
                           int64_t* counts, double* wsum);

/* Copy the bucketed pair list to device arrays [n_pairs]: field index, and the
 * catalogue indices i < j.  Order: by field, then by grid line of the
 * midpoint's lower CIC corner, then by search order (deterministic). */
pgx_status pgx_pairs_export(pgx_plan* plan, int32_t* field, int32_t* i, int32_t* j, void* stream);

/*
 * Forward estimator for the catalogue of the last pgx_pairs_build.
 *   w: device FP32 [n_gal] galaxy weights (>= 0, finite) or NULL for unit
 *      weights.  Pair weights are w_i w_j.
 *   Outputs (device FP64, each nullable except xi_pg): wsum [F] (sum of pair
 *   weights per field), xi_gg [R], xi_pg [F][R], xi_dp [F], b_pg [F][R],
 *   q_eff [F][R].  Empty pair fields give NaN rows of xi_pg, b_pg, q_eff.
 *   The call keeps what pgx_backward needs inside the plan.  Errors: ESTATE
 *   before pgx_pairs_build.
 */
pgx_status pgx_forward(pgx_plan* plan, const float* w, void* stream, double* wsum, double* xi_gg,
                       double* xi_pg, double* xi_dp, double* b_pg, double* q_eff);

/*
 * Adjoint of pgx_forward: gradient of a scalar loss with respect to the
 * galaxy weights w of the last pgx_forward call.  Hand-written chain rule
 * through the finalisation, the bin sums, the inverse and forward transforms,
 * the cross-power product and the mass assignment (which becomes a gather at
 * the pair midpoints and galaxies); the paper has no gradients, its HOD
 * derivatives are numerical (HOD dependency section).
 *   g_b_pg, g_q_eff, g_xi_pg [F][R], g_xi_gg [R], g_xi_dp [F]: device FP64
 *   upstream gradients dL/d(output), each nullable (= zero).  Entries of
 *   outputs that were not finite (empty fields) are ignored.
 *   grad_w: device FP32 [n_gal] out, dL/dw_i (unit weights when the forward
 *   had w = NULL: the derivative at w = 1).
 * Implemented for PGX_FP32_BATCHED plans (PGX_ENOTSUP otherwise); ESTATE
 * without a preceding pgx_forward on the same catalogue.
 */
pgx_status pgx_backward(pgx_plan* plan, void* stream, const double* g_b_pg, const double* g_q_eff,
                        const double* g_xi_pg, const double* g_xi_gg, const double* g_xi_dp,
                        float* grad_w);

/*
 * Projected two-point correlation of the pairs (2PCF section, equation
 * 2PCF_los_integrated_explicit): for a plan with pair_mode RP_PI, the
 * line-of-sight integral of the pair correlation xi(d_p) inside the pair
 * sphere, averaged over each r_p annulus,
 *   w_p[a] = sum_b xi_dp[a n_p2 + b] V[a n_p2 + b] / (pi (rp_{a+1}^2 - rp_a^2)),
 * V the exact annulus-slab volumes of pgx_field_volumes (pieces of zero volume
 * contribute nothing).  With one |pi| bin covering the sphere and a thin
 * annulus this is the paper's 2 d_par,max (xi - like) column with the
 * annulus volume taken exactly (its printed Delta V_perp misses a factor
 * d_perp).
 *   xi_dp: device FP64 [F] (as pgx_forward returns it); w_p: device FP64
 *   [n_p1] out.
 * pgx_projected_backward: the adjoint, g_xi_dp[f] = g_w_p[a(f)] V_f / A_a
 * (device FP64 [n_p1] in, [F] out).  Errors: EINVAL for other pair modes or
 * NULL arrays.
 */
pgx_status pgx_projected(pgx_plan* plan, void* stream, const double* xi_dp, double* w_p);
pgx_status pgx_projected_backward(pgx_plan* plan, void* stream, const double* g_w_p, double* g_xi_dp);

/*
 * Multipoles of the pair-galaxy cross-correlation in the angle between the
 * pair axis and the pair-to-galaxy direction: the other reading of the
 * pair-orientation cosine, the pair axis against the direction to the
 * galaxy instead of against the z line of sight, with the cosine
 * mu' = d^ . r^ expanded in Legendre polynomials.  Over the lattice vectors
 * r of output shell b:
 *   xi_l[f][b] = (2l + 1) / (n_b Wsum_f) sum_{p in f} w_p sum_{r in b}
 *                P_l(d^_p . r^) (CIC interpolation of delta_g at m_p + r),
 * for l = 0, 2, .., lmax (even l: the pair axis has no sign; d = x_j - x_i,
 * minimum image; a pair with d = 0 counts for l = 0 only).  l = 0 is xi_pg.
 * Computed by the dual form with the addition theorem (one bin kernel per
 * shell and harmonic Y_lm, gathered at the midpoints, per-field sums
 * weighted by Y_lm of each pair axis), from the weights and galaxy
 * spectrum of the last pgx_forward; eager launches.
 *   lmax: 0, 2 or 4.
 *   xi_l: device FP64 out [F][R][lmax/2 + 1]; NaN rows for empty fields.
 * Device memory: n_pairs x R x (number of harmonics: 1, 6, 15) FP32 for the
 * gathered values.  Errors: EINVAL for another lmax, an output mode other
 * than shells, or a first shell edge of 0; ESTATE without a preceding
 * pgx_forward; ENOTSUP on FP64 plans.
 */
pgx_status pgx_multipoles(pgx_plan* plan, void* stream, int32_t lmax, double* xi_l);

/*
 * Adjoint of the last pgx_multipoles call (after the last pgx_forward):
 * gradient of a scalar loss with respect to the galaxy weights, by the same
 * hand-written chain as pgx_backward through the harmonic bin kernels (pair
 * side from the values that call gathered; galaxy side through the pair
 * fields weighted by each pair axis's harmonics) and the normalisations
 * Wsum_f, W_g.
 *   g_xi_l: device FP64 [F][R][lmax/2 + 1] upstream gradient (entries of
 *   empty fields and non-finite entries are ignored).
 *   grad_w: device FP32 [n_gal] out.
 * Eager launches.  Errors: ESTATE without a pgx_multipoles after the last
 * pgx_forward or pgx_pairs_build; EINVAL for NULL arguments; ENOTSUP on
 * FP64 plans.
 */
pgx_status pgx_multipoles_backward(pgx_plan* plan, void* stream, const double* g_xi_l, float* grad_w);

/*
 * Spectrum keeping for the adjoint.  With enable = 1, each later pgx_forward
 * on an FP32 batched plan also writes every pair-field spectrum (one complex
 * N^3 grid per two fields: n_fields/2 rounded up, 1 GiB each at N = 512) into
 * plan-owned device memory, when the device has room for it plus 4 GiB;
 * pgx_backward then reads them instead of recomputing the pair-field
 * transforms.  Results are identical either way (the same kernels produce
 * the same spectra); only time and memory differ.  When the memory is not
 * available the forward silently recomputes as with enable = 0.  The memory
 * is held until the plan is destroyed.  Default 0.  No device work.
 */
pgx_status pgx_keep_spectra(pgx_plan* plan, int32_t enable);

/*
 * Autotuner for the FP32 batched path.  Times the forward launch sequence on
 * the current pair catalogue (so call it after pgx_pairs_build) for candidate
 * batch sizes (half, equal to and twice the default field pairs per launch,
 * those whose buffers fit in free device memory) and, per pass, two kernel
 * variants: the y passes in their default or second radix schedule (16
 * elements per thread, fewer exchange stages), the z pass with its stage
 * twiddles in registers or in the LDS table.  Then it times the dual form of
 * the pair-field part (the paper's own evaluation, Methodology, equation
 * bpg_final: one transform per pair of output bins, the bin kernel convolved
 * with the galaxy field, interpolated at every pair midpoint; the same
 * estimator exactly, up to floating-point rounding) when its per-pair values
 * (n_pairs x n_out FP32) fit in half the free device memory, with its two z
 * passes in tiles of the default width or half of it, or reading the bin
 * kernels' full spectra from a per-plan store (the kernels are even in each
 * lattice axis, so the rows ky, kz <= N/2 of every x frequency hold them:
 * (n_out + 1) / 2 x (N/2 + 1)^2 x N complex FP32, 2.7 GB at 512^3 with 20
 * bins, allocated when it fits with 4 GiB to spare; the z passes then skip
 * the kernel's z transform); the dual form is a
 * candidate only when its xi agree with the per-field transforms' within
 * half of 1e-5 max(|xi|, 1e-2) on every bin (pgx_dual_check).  It keeps the fastest
 * combination for later calls.  Results differ between schedules only by
 * floating-point rounding.  It runs the forward eagerly several times
 * (about sixteen forward passes' worth of device time), discards the state of
 * the last pgx_forward (a pgx_backward must follow a new pgx_forward), clears
 * the kernel-timing counters and invalidates the launch graphs.
 *   schedule: host int32[5] out (nullable): field pairs (or bin pairs) per
 *   batch, forward y-pass variant, inverse y-pass variant, z-pass variant
 *   (0 = default; for the dual form: 1 = half-width z-pass tiles, 2 = z passes
 *   on the stored kernel spectra), algorithm
 *   (0 = one transform per field pair, 1 = dual form).  pgx_backward runs
 *   the adjoint of the algorithm the preceding pgx_forward used.
 * Errors: ESTATE before pgx_pairs_build; ENOTSUP on FP64 plans.
 */
pgx_status pgx_autotune(pgx_plan* plan, void* stream, int32_t* schedule);
/* The schedule in use: host int32[5] as filled by pgx_autotune.  Creates the
 * device state of the plan if it does not exist yet. */
pgx_status pgx_schedule(pgx_plan* plan, int32_t* schedule);
/* The accuracy check of the dual form in the last pgx_autotune: its largest
 * xi disagreement with the per-field transforms on the tuned catalogue, in
 * units of 1e-5 max(|xi|, 1e-2) over every bin of every non-empty field (the
 * autotuner keeps the dual form only when it is at most 0.5); -1 when not
 * measured (no autotune yet, FP64 plan, or the dual form did not fit).  The
 * FP32 rounding of the dual form sits in the bin kernels' convolution at
 * each pair midpoint, which the few pairs of a sparse field do not average,
 * so on sparse catalogues it can exceed the per-field transforms' error.
 *   disagreement: host double out.  No device work. */
pgx_status pgx_dual_check(pgx_plan* plan, double* disagreement);
/* The dual form's accuracy check of pgx_dual_check taken again on the
 * weights of the last pgx_forward (unit weights if none), for callers whose
 * weights have moved since pgx_autotune (an HOD fit): the forward runs once
 * with the per-field transforms and once in the dual form of the schedule in
 * use, and their xi are compared as in the autotuner.  The result becomes
 * what pgx_dual_check reports.
 *   fallback:     nonzero: when the disagreement exceeds 0.5, switch the plan
 *                 to the per-field transforms (the batch size and y-pass
 *                 variants kept, the per-field z-pass variant of the last
 *                 pgx_autotune, 0 after pgx_set_schedule).
 *   disagreement: host double out, in units of 1e-5 max(|xi|, 1e-2); -1 when
 *                 the schedule in use is not the dual form (nothing runs).
 * Synchronises the stream.  Discards the state of the last pgx_forward (a
 * pgx_backward must follow a new pgx_forward) and invalidates the launch
 * graphs.  Errors: ESTATE before pgx_pairs_build; ENOTSUP on FP64 plans. */
pgx_status pgx_dual_recheck(pgx_plan* plan, void* stream, int32_t fallback, double* disagreement);
/* Apply a schedule (host int32[5] as above, e.g. one found by an earlier
 * pgx_autotune): batch size in [1, 32] (clamped to the number of field
 * pairs), variants and algorithm 0 or 1, z-pass variant 2 with algorithm 1
 * (fills the kernel-spectrum store on the stream).  Same side effects as
 * pgx_autotune apart from the timing runs.  Errors: EINVAL for values out of
 * range, ENOSPACE when the kernel-spectrum store does not fit, ESTATE before
 * pgx_pairs_build, ENOTSUP on FP64 plans. */
pgx_status pgx_set_schedule(pgx_plan* plan, void* stream, const int32_t* schedule);

/*
 * Launch graphs.  With enable = 1 (the default) the device work of
 * pgx_forward (weights, galaxy side, every batch of pair fields) and of
 * pgx_backward is recorded into a HIP graph the second time it runs with the
 * same catalogue, batch schedule and optional-input pattern, and replayed on
 * the caller's stream from then on (the caller's weights and upstream
 * gradients are first copied into plan buffers; results are copied out).
 * Validation and the finalisation run outside the graph.  A new
 * pgx_pairs_build or pgx_autotune invalidates the graphs.  While kernel timing
 * (pgx_profile) is on, the work runs eagerly.  No device work.
 */
pgx_status pgx_use_graphs(pgx_plan* plan, int32_t enable);
/* Number of graph replays of the forward and adjoint bodies since the plan
 * was created (host counters; either pointer may be NULL). */
pgx_status pgx_graph_replays(pgx_plan* plan, int64_t* forward, int64_t* backward);

/*
 * Kernel timing.  pgx_profile(plan, 1) clears the counters and starts
 * recording a pair of HIP events on the launch stream around every launch of
 * the transform-pass kernels (the events bracket exactly one kernel each);
 * pgx_profile(plan, 0) stops.  pgx_profile_read returns, for entry k (one per
 * kernel kind, in order of first launch): its name (owned by the plan, valid
 * until the next pgx_profile call), the number of launches, the summed
 * event-measured time in ms, and the summed algorithmic bytes of those
 * launches (the bytes each launch has to read and write: its input lines,
 * the galaxy spectrum where it is read, its output lines).  It synchronises
 * the recorded events.  EINVAL when k is out of range.
 */
pgx_status pgx_profile(pgx_plan* plan, int32_t enable);
pgx_status pgx_profile_read(pgx_plan* plan, int32_t k, const char** name, int64_t* launches,
                            double* ms, double* bytes);

/* SHA-256 (hex) of the sources this library was built from (kernel and host
 * headers, HIP translation units and this header), for tying a measurement to
 * the code that produced it. */
const char* pgx_build_digest(void);

/* Message for the last non-OK status returned by a call on `plan`; with
 * plan = NULL, the last one on this thread (e.g. of pgx_plan_create).  The
 * string is owned by the plan (or the thread) and valid until its next
 * failing call. */
const char* pgx_last_error(const pgx_plan* plan);

/*
 * Caller-owned workspace.
 * pgx_workspace_bytes: an upper bound of the device memory the plan's buffers
 * reach for a catalogue of n_gal galaxies and n_pairs pairs (n_pairs from a
 * pgx_pairs_build or an estimate): the pair build, pgx_forward, pgx_backward
 * and pgx_autotune with their batch slots (up to twice the default batch),
 * the galaxy spectrum, the dual form's gathered values and kernel stores,
 * and the kept spectra when pgx_keep_spectra is on; 10 % and 64 MiB are
 * added for small tables and first-fit fragmentation.  pgx_multipoles needs
 * n_pairs x (h + n_out h) x 4 bytes more (h harmonics: 1, 6, 15 for lmax 0,
 * 2, 4).  No device work.
 * pgx_set_workspace: from now on every device buffer of the plan is carved
 * from [ws, ws + bytes) (first fit, 256-byte aligned), a region of device
 * memory the caller allocated on the plan's device and keeps alive until the
 * plan is destroyed or another workspace is set; the plan then calls neither
 * hipMalloc nor hipFree.  Optional stores (kernel stores of the dual form,
 * kept spectra) are made only when they fit in the free part of it.  Setting
 * (or clearing, ws = NULL) a workspace discards the plan's device state: the
 * next call must be pgx_pairs_build.  A call that needs more than the free
 * part returns ENOSPACE.  Errors: EINVAL when ws is not 256-byte aligned.
 * pgx_workspace_used: bytes of the workspace in use now and at most so far.
 */
pgx_status pgx_workspace_bytes(const pgx_plan* plan, int64_t n_gal, int64_t n_pairs, size_t* bytes);
pgx_status pgx_set_workspace(pgx_plan* plan, void* ws, size_t bytes);
pgx_status pgx_workspace_used(const pgx_plan* plan, size_t* in_use, size_t* peak);

/*
 * Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * it): pgx_forward of a PGX_FP64_PLAIN plan, the same arguments and results
 * (to the rounding of the scatter's atomic additions), with all its work
 * memory (two complex FP64 N^3 grids, bin partials, pair weights, sums) in a
 * fixed array of 96 MiB that the library holds on each device it runs on
 * until the process ends; the call makes no hipMalloc or hipFree and leaves
 * the plan's own buffers as they were.  The array keeps the last call's
 * contents and every call on one device shares it: calls that overlap on one
 * device race.  Runs eagerly (no launch graph).  It needs a preceding
 * pgx_pairs_build (whose pair catalogue it reads).  Errors: ENOTSUP for other
 * precisions; ENOSPACE when the work exceeds the array (N = 128 needs 64 MiB
 * for the grids, leaving room for about 3.5e6 pairs; N >= 256 never fits);
 * ESTATE before pgx_pairs_build.
 */
pgx_status pgx_forward_fixed(pgx_plan* plan, const float* w, void* stream, double* wsum,
                             double* xi_gg, double* xi_pg, double* xi_dp, double* b_pg,
                             double* q_eff);

#ifdef __cplusplus
}
#endif

#endif /* PGX_H */
