"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle on the
same seeded catalogues.

Bars: pair keys and counts bit-exact; FP32 path |dxi| <= 1e-5 max(|xi|, 1e-2)
(1e-5 relative where |xi| > 1e-2, the same bound in absolute terms below);
FP64 plain path 1e-9 relative with a 1e-12 floor.
"""
import functools
import os
import sys

import numpy as np
import pytest

from oracle.pairs import pairs_for
from oracle.pipeline import forward as oracle_forward
from synth import get_config
from synth.catalog import Catalog
from synth.configs import Workload, linbins, logbins

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_03464_amd import load_library
    load_library()


def dev(cat):
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    return f(cat.x), f(cat.y), f(cat.z)


# The three FP32 evaluations as (z-pass variant, algorithm): per-field
# transforms, the dual form, the dual form on the stored kernel spectra.
ALGOS = {0: (0, 0), 1: (0, 1), 2: (2, 1)}


def run(wl, cat, precision, w=None, batch=0, algo=None, autotune=False):
    from paper_1705_03464_amd import Plan
    plan = Plan.from_workload(wl, precision=precision, batch=batch)
    P, counts = plan.pairs_build(*dev(cat))
    if algo is not None:
        zp, al = ALGOS[algo]
        plan.set_schedule(plan.schedule()["batch"], 0, 0, zp, al)
    if autotune:
        _say(f"  autotuned {plan.autotune()}")
    wt = None if w is None else torch.as_tensor(np.asarray(w, np.float32), device="cuda")
    out = plan.forward(wt)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    return plan, P, counts.cpu().numpy(), out


def xi_err_ok(got, exp, rel=1e-5, floor=1e-2):
    got = np.asarray(got); exp = np.asarray(exp)
    fin = np.isfinite(exp)
    assert np.array_equal(fin, np.isfinite(got)), "NaN pattern differs"
    assert np.array_equal(np.isnan(exp), np.isnan(got)), "empty fields must give NaN"
    d = np.abs(got[fin] - exp[fin])
    bound = rel * np.maximum(np.abs(exp[fin]), floor)
    worst = float(np.max(d / bound)) if d.size else 0.0
    return worst


def assert_fp32_parity(out, ref, rel=1e-5):
    w_gg = xi_err_ok(out["xi_gg"], ref["xi_gg"], rel)
    w_pg = xi_err_ok(out["xi_pg"], ref["xi_pg"], rel)
    _say(f"  worst |dxi| / (1e-5 max(|xi|,1e-2)): gg {w_gg:.3f} pg {w_pg:.3f}")
    assert w_gg <= 1.0 and w_pg <= 1.0
    # bins wholly outside the pair sphere have zero volume: NaN on both sides
    assert np.allclose(out["xi_dp"], ref["xi_dp"], rtol=1e-12, atol=1e-12, equal_nan=True)
    assert np.allclose(out["wsum"], ref["wsum"], rtol=1e-13, atol=0)
    # b and Q where both correlations are well above the noise bar
    m = (np.abs(ref["xi_pg"]) > 1e-2) & (np.abs(ref["xi_gg"])[None, :] > 1e-2)
    if m.any():
        assert np.allclose(out["b_pg"][m], ref["b_pg"][m], rtol=3e-5)
    # Q_eff (equation Qeff_notsq) there too, where its denominators are not
    # small: the bound propagates b's 3e-5 through each term's magnitude
    x = np.broadcast_to(ref["xi_dp"][:, None], ref["b_pg"].shape)
    xw = np.broadcast_to(ref["xi_gg"][None, :], ref["b_pg"].shape)
    with np.errstate(invalid="ignore", divide="ignore"):
        den = 2.0 * x + 1.5 * xw
        mq = m & np.isfinite(x) & (np.abs(x) > 1e-2) & (np.abs(den) > 1e-2)
        scale = (np.abs((1.0 + x) * ref["b_pg"]) + 2.0 + np.abs(xw / (2.0 * x))) / np.abs(den)
    if mq.any():
        dq = np.abs(out["q_eff"][mq] - ref["q_eff"][mq])
        assert np.all(dq <= 3e-5 * scale[mq] + 1e-12), float(np.max(dq / (3e-5 * scale[mq])))


def assert_fp64_parity(out, ref):
    for k in ("xi_gg", "xi_pg", "b_pg", "q_eff", "xi_dp"):
        fin = np.isfinite(ref[k])
        assert np.array_equal(fin, np.isfinite(out[k])), k
        assert np.allclose(out[k][fin], ref[k][fin], rtol=1e-9, atol=1e-12), k


def clustered_catalog(L, n_halo, n_field, seed, sat=8, spread=1.5):
    rng = np.random.default_rng(seed)
    c = rng.random((n_halo, 3)) * L
    s = np.repeat(c, sat, axis=0) + rng.normal(0, spread, (n_halo * sat, 3))
    pos = np.mod(np.concatenate([c, s, rng.random((n_field, 3)) * L]), L)
    pos[pos >= L] = 0.0
    n = pos.shape[0]
    return Catalog(L, pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.zeros(n),
                   np.zeros(n, np.int8))


# ------------------------------------------------------------------ pairs
def test_pairs_bitexact_cfg0():
    wl = get_config("cfg0")
    cat = wl.catalog()
    _say(f"pairs cfg0: n_gal={cat.n}")
    ref = pairs_for(cat, wl)
    plan, P, counts, _ = run(wl, cat, "fp64")
    assert P == ref["key"].size
    assert np.array_equal(counts, ref["counts"])
    f, i, j = (t.cpu().numpy().astype(np.int64) for t in plan.pairs_export())
    got = np.stack([f, i, j], 1)
    exp = np.stack([ref["key"], ref["i"], ref["j"]], 1)
    got = got[np.lexsort(got.T[::-1])]
    exp = exp[np.lexsort(exp.T[::-1])]
    assert np.array_equal(got, exp)


def test_pairs_rp_pi_and_mu_edges():
    L = 60.0
    wl = Workload(name="t", L=L, N=64, precision="fp32", pair_mode="rp_pi",
                  p1_edges=linbins(0.0, 12.0, 5), p2_edges=linbins(0.0, 12.0, 3), pair_dmax=12.0,
                  out_mode="rp_pi", o1_edges=linbins(0.0, 25.0, 5), o2_edges=linbins(0.0, 25.0, 4),
                  catalog_kw={})
    cat = clustered_catalog(L, 60, 1500, seed=3)
    # exact edge cases: on-edge separations, pairs along z, across the boundary
    extra = np.array([[1.0, 1.0, 1.0], [3.4, 1.0, 1.0], [10.0, 10.0, 10.0], [10.0, 10.0, 14.8],
                      [59.5, 30.0, 30.0], [0.5, 30.0, 30.0]])
    for a, k in zip("xyz", range(3)):
        setattr(cat, a, np.concatenate([getattr(cat, a), extra[:, k]]))
    cat.halo_mass = np.zeros(cat.x.size); cat.kind = np.zeros(cat.x.size, np.int8)
    ref = pairs_for(cat, wl, method="brute")
    plan, P, counts, _ = run(wl, cat, "fp32")
    assert np.array_equal(counts, ref["counts"])
    f, i, j = (t.cpu().numpy().astype(np.int64) for t in plan.pairs_export())
    got = np.stack([f, i, j], 1); exp = np.stack([ref["key"], ref["i"], ref["j"]], 1)
    assert np.array_equal(got[np.lexsort(got.T[::-1])], exp[np.lexsort(exp.T[::-1])])


def test_pairs_deterministic():
    wl = get_config("cfg0")
    cat = wl.catalog()
    plan, P, _, _ = run(wl, cat, "fp32")
    a = [t.cpu().numpy() for t in plan.pairs_export()]
    plan.pairs_build(*dev(cat))
    b = [t.cpu().numpy() for t in plan.pairs_export()]
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


# ------------------------------------------------------------------ forward, cfg0
def test_forward_fp64_plain_cfg0():
    wl = get_config("cfg0")
    cat = wl.catalog()
    _say("forward fp64 cfg0")
    ref = oracle_forward(cat, wl)
    _, _, counts, out = run(wl, cat, "fp64")
    assert np.array_equal(counts, ref["counts"])
    assert_fp64_parity(out, ref)


def test_forward_fp32_cfg0():
    wl = get_config("cfg0")
    cat = wl.catalog()
    _say("forward fp32 cfg0")
    ref = oracle_forward(cat, wl)
    _, _, _, out = run(wl, cat, "fp32")
    assert_fp32_parity(out, ref)


# ------------------------------------------------------------------ small grids, all modes
SMALL = [
    # (N, L, pair_mode, p1, p2, dmax, out_mode, o1, o2)
    (64, 100.0, "s_mu", linbins(0.5, 8.0, 3), linbins(0.0, 1.0, 3), 0.0, "shell",
     logbins(6.0, 40.0, 7), None),
    (64, 100.0, "s_mu", logbins(0.5, 8.0, 4), linbins(0.0, 1.0, 2), 0.0, "r_mu",
     logbins(6.0, 40.0, 5), linbins(0.0, 1.0, 4)),
    (128, 160.0, "rp_pi", linbins(0.0, 10.0, 3), linbins(0.0, 10.0, 3), 10.0, "rp_pi",
     linbins(0.0, 60.0, 6), linbins(0.0, 45.0, 5)),
    (256, 300.0, "s_mu", logbins(0.5, 10.0, 7), linbins(0.0, 1.0, 1), 0.0, "shell",
     logbins(10.0, 80.0, 20), None),
]


@pytest.mark.parametrize("case", range(len(SMALL)))
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_forward_small_grids(case, precision):
    N, L, pm, p1, p2, dmax, om, o1, o2 = SMALL[case]
    wl = Workload(name="t", L=L, N=N, precision=precision, pair_mode=pm, p1_edges=p1,
                  p2_edges=p2, pair_dmax=dmax, out_mode=om, o1_edges=o1, o2_edges=o2,
                  catalog_kw={})
    cat = clustered_catalog(L, int(0.02 * L ** 2), int(0.8 * L ** 2), seed=case)
    w = np.random.default_rng(case).uniform(0.3, 1.7, cat.n).astype(np.float32).astype(np.float64)
    _say(f"small case {case} N={N} {pm}/{om} F={wl.n_fields} n_gal={cat.n} {precision}")
    ref = oracle_forward(cat, wl, w=w)
    _, _, counts, out = run(wl, cat, precision, w=w, batch=2)
    assert np.array_equal(counts, ref["counts"])
    if precision == "fp64":
        assert_fp64_parity(out, ref)
    else:
        assert_fp32_parity(out, ref)


@pytest.mark.parametrize("algo", [0, 1, 2])
def test_empty_field_gives_nan_rows(algo):
    L = 100.0
    wl = Workload(name="t", L=L, N=64, precision="fp32", pair_mode="s_mu",
                  p1_edges=np.array([0.5, 1.0, 2.0, 9.0]), p2_edges=np.array([0.0, 1.0]),
                  out_mode="shell", o1_edges=logbins(6.0, 40.0, 4), o2_edges=None, catalog_kw={})
    rng = np.random.default_rng(0)
    # a sparse uniform catalogue: no pair closer than 1.0 is likely at this density
    pos = rng.random((300, 3)) * L
    cat = Catalog(L, pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.zeros(300),
                  np.zeros(300, np.int8))
    ref = oracle_forward(cat, wl)
    _, _, counts, out = run(wl, cat, "fp32", algo=algo)
    assert np.array_equal(counts, ref["counts"])
    for f in range(wl.n_fields):
        if counts[f] == 0:
            assert np.all(np.isnan(out["xi_pg"][f])) and np.all(np.isnan(out["b_pg"][f]))
    assert_fp32_parity(out, ref)


@pytest.mark.parametrize("algo", [0, 1, 2])
def test_catalogue_without_pairs(algo):
    """Galaxies but no close pair at all: every pair field is empty (NaN
    rows), xi_gg still meets the oracle, and the adjoint runs (galaxy term
    only) and meets the oracle's gradient."""
    from oracle import grad as OG
    L = 100.0
    wl = Workload(name="t", L=L, N=64, precision="fp32", pair_mode="s_mu",
                  p1_edges=np.array([0.5, 1.0, 2.0]), p2_edges=np.array([0.0, 1.0]),
                  out_mode="shell", o1_edges=logbins(6.0, 40.0, 4), o2_edges=None, catalog_kw={})
    g = np.arange(4) * 25.0 + 3.0
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")  # 64 galaxies 25 apart: no pair within 2
    cat = Catalog(L, X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy(), np.zeros(64),
                  np.zeros(64, np.int8))
    ref = oracle_forward(cat, wl)
    plan, P, counts, out = run(wl, cat, "fp32", algo=algo)
    assert P == 0 and not counts.any()
    assert np.all(np.isnan(out["xi_pg"]))
    assert xi_err_ok(out["xi_gg"], ref["xi_gg"]) <= 1.0
    w = np.random.default_rng(1).uniform(0.5, 1.5, 64).astype(np.float32).astype(np.float64)
    gg = np.random.default_rng(2).normal(size=wl.n_out)
    gref, _ = OG.weight_gradient(cat, wl, w, g_xigg=gg)
    plan.forward(torch.as_tensor(w, dtype=torch.float32, device="cuda"))
    gw = plan.backward(g_xi_gg=torch.as_tensor(gg, device="cuda")).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gw - gref) <= 1e-3 * np.linalg.norm(gref)


def test_no_galaxies_is_rejected_cleanly_or_empty():
    from paper_1705_03464_amd import PgxError
    wl = get_config("cfg0")
    cat = wl.catalog()
    bad = cat.subset(np.arange(50))
    bad.x = bad.x.copy(); bad.x[3] = wl.L  # outside [0, L)
    with pytest.raises(PgxError) as e:
        run(wl, bad, "fp32")
    assert e.value.code == 1


# ------------------------------------------------------------------ full-size workloads
def test_cfg2_full_size_sampled_fields():
    wl = get_config("cfg2")
    cat = wl.catalog()
    _say(f"cfg2 n_gal={cat.n}")
    pairs = pairs_for(cat, wl)
    fields = [0, 41, 80, 119, 159]
    ref = oracle_forward(cat, wl, pairs=pairs, fields=fields)
    _, P, counts, out = run(wl, cat, "fp32")
    assert P == pairs["key"].size
    assert np.array_equal(counts, pairs["counts"])
    sub = dict(ref); o = dict(out)
    for k in ("xi_pg", "b_pg", "q_eff", "xi_dp", "wsum"):
        sub[k] = ref[k][fields]; o[k] = out[k][fields]
    assert_fp32_parity(o, sub)


def test_cfg1_full_size_bench_configuration():
    """The 512^3 production workload in the launch configuration the bench times
    (the autotuned schedule): all pair counts bit-exact, xi_gg and the 10 most
    and 10 least populated pair fields (xi_pg, b_pg, Q_eff) against the FP64
    oracle."""
    wl = get_config("cfg1")
    cat = wl.catalog()
    _say(f"cfg1 n_gal={cat.n}")
    pairs = pairs_for(cat, wl)
    _, P, counts, out = run(wl, cat, "fp32", autotune=True)
    assert P == pairs["key"].size
    assert np.array_equal(counts, pairs["counts"])
    # the 10 most and the 10 least populated non-empty fields
    order = [int(f) for f in np.argsort(pairs["counts"], kind="stable") if pairs["counts"][f] > 0]
    fields = sorted(set(order[:10] + order[-10:]))
    ref = oracle_forward(cat, wl, pairs=pairs, fields=fields)
    sub = dict(ref); o = dict(out)
    for k in ("xi_pg", "b_pg", "q_eff", "xi_dp", "wsum"):
        sub[k] = ref[k][fields]; o[k] = out[k][fields]
    assert_fp32_parity(o, sub)


@functools.lru_cache(maxsize=1)
def _crowded_case():
    base = get_config("cfg4")
    wl = base.scaled(name="hod250", L=250.0, o1_edges=logbins(10.0, 80.0, 12),
                     catalog_kw=dict(base.catalog_kw, n_halos=625), weighted=False)
    cat = wl.catalog()
    w = np.random.default_rng(5).uniform(0.3, 1.7, cat.n).astype(np.float32).astype(np.float64)
    _say(f"512^3 crowded nodes: n_gal={cat.n}")
    pairs = pairs_for(cat, wl)
    fields = [0, wl.n_fields - 1]
    ref = oracle_forward(cat, wl, w=w, pairs=pairs, fields=fields)
    return wl, cat, w, pairs, fields, ref


@pytest.mark.parametrize("algo", [0, 1, 2])
def test_512_crowded_nodes(algo):
    """HOD candidates (50 per halo, NFW profiles) at 512^3 in a 250 Mpc/h box:
    up to ~2500 pair midpoints and ~40 galaxies share one grid node, so the
    scatters' wavefront run sums (active when a line is a whole wavefront, as
    at this grid) merge long runs.  Weighted; counts bit-exact, xi_gg and the
    smallest- and largest-separation fields against the oracle for the
    per-field transforms and both dual-form variants."""
    wl, cat, w, pairs, fields, ref = _crowded_case()
    _, P, counts, out = run(wl, cat, "fp32", w=w, algo=algo)
    _say(f"  algorithm {ALGOS[algo]}: {P} pairs, fields {fields}")
    assert P == pairs["key"].size
    assert np.array_equal(counts, pairs["counts"])
    sub = dict(ref); o = dict(out)
    for k in ("xi_pg", "b_pg", "q_eff", "xi_dp", "wsum"):
        sub[k] = ref[k][fields]; o[k] = out[k][fields]
    assert_fp32_parity(o, sub)


def test_forward_1024_redshift_space_sampled():
    """1024^3 grid with the (r_p, |pi|) binning of the redshift-space workload,
    on a reduced catalogue: counts bit-exact, xi_gg and three sampled fields."""
    wl = get_config("cfg3").scaled(catalog_kw=dict(get_config("cfg3").catalog_kw, n_halos=20000,
                                                   n_field=200000))
    cat = wl.catalog()
    _say(f"1024^3 n_gal={cat.n}")
    pairs = pairs_for(cat, wl)
    fields = [0, 37, 100]
    ref = oracle_forward(cat, wl, pairs=pairs, fields=fields)
    _, P, counts, out = run(wl, cat, "fp32")
    assert np.array_equal(counts, pairs["counts"])
    sub = dict(ref); o = dict(out)
    for k in ("xi_pg", "b_pg", "q_eff", "xi_dp", "wsum"):
        sub[k] = ref[k][fields]; o[k] = out[k][fields]
    assert_fp32_parity(o, sub)


def test_fp64_plain_512_matches_fp32_batched():
    """The one-field-at-a-time FP64 path at the production grid (the
    reference leg of the benchmark) against the batched FP32 path, which the
    test above holds to the oracle at this size."""
    wl = get_config("cfg1")
    cat = wl.catalog()
    _say(f"cfg1 fp64 plain vs fp32 batched: n_gal={cat.n}")
    _, _, _, o32 = run(wl, cat, "fp32")
    _, _, _, o64 = run(wl, cat, "fp64")
    for k in ("xi_gg", "xi_pg"):
        worst = xi_err_ok(o64[k], o32[k], rel=1e-5)
        _say(f"  {k}: worst |d| / (1e-5 max(|xi|,1e-2)) = {worst:.3f}")
        assert worst <= 1.0


@pytest.mark.parametrize("out_mode", ["shell", "gsw"])
def test_fp64_plain_tsc_vs_oracle(out_mode):
    """The paper's TSC mass assignment on the FP64 plain path against the
    oracle's TSC at the FP64 bar; with out_mode gsw this is the paper's
    estimator literally (its weighting function and its assignment)."""
    from dataclasses import replace
    L = 200.0
    o1 = np.array([15.0, 10.0, 0.8, 5.0, 60.0]) if out_mode == "gsw" else logbins(10.0, 60.0, 4)
    wl = Workload(name="tsc", L=L, N=64, precision="fp64", pair_mode="s_mu",
                  p1_edges=logbins(0.5, 8.0, 3), p2_edges=linbins(0.0, 1.0, 2), out_mode=out_mode,
                  o1_edges=o1, o2_edges=None, catalog_kw={}, qeff_mode="const", xi_w_const=0.362,
                  assignment="tsc")
    cat = clustered_catalog(L, 300, 12000, seed=17, sat=8, spread=1.5)
    w = np.random.default_rng(17).uniform(0.4, 1.6, cat.n).astype(np.float32).astype(np.float64)
    ref = oracle_forward(cat, wl, w=w)
    _, P, counts, out = run(wl, cat, "fp64", w=w)
    _say(f"TSC {out_mode}: n_gal={cat.n} pairs={P}")
    assert np.array_equal(counts, ref["counts"])
    assert_fp64_parity(out, ref)
    # the option takes effect: CIC gives other values
    cic = oracle_forward(cat, replace(wl, assignment="cic"), w=w)
    fin = np.isfinite(ref["xi_pg"])
    assert np.max(np.abs(ref["xi_pg"][fin] - cic["xi_pg"][fin])) > 1e-4 * np.max(np.abs(ref["xi_pg"][fin]))
