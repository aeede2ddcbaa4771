"""The paper's TSC mass assignment (Implementation section, "Mass assignment
function") on the batched FP32 path: forward against the oracle at the FP32
bar and the adjoint against the oracle's adjoint and its finite differences
at the gradient bar, for galaxies and pair midpoints alike, in all three
evaluations (per-field transforms; the dual form on the window columns and
on the kernel-spectrum store, whose line-major catalogue is keyed by each
midpoint's nearest node).  The multipoles refuse TSC plans."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import grad as OG  # noqa: E402
from oracle.pipeline import forward as oracle_forward  # noqa: E402
from synth import get_config  # noqa: E402
from synth.configs import Workload, linbins, logbins  # noqa: E402
from test_gpu_grad import grad_close, mask_ill_conditioned_q, upstream  # noqa: E402
from test_gpu_parity import ALGOS, assert_fp32_parity, clustered_catalog  # noqa: E402

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


CASES = {
    # clustered box at 64^3 and 128^3, (s, |mu|) pairs, shells / (r, |mu|)
    "s_mu-64": dict(L=120.0, N=64, pair_mode="s_mu", p1_edges=logbins(0.5, 9.0, 3),
                    p2_edges=linbins(0.0, 1.0, 2), out_mode="shell", o1_edges=logbins(6.0, 40.0, 6),
                    o2_edges=None),
    "r_mu-128": dict(L=200.0, N=128, pair_mode="s_mu", p1_edges=logbins(0.5, 9.0, 2),
                     p2_edges=linbins(0.0, 1.0, 3), out_mode="r_mu", o1_edges=logbins(8.0, 60.0, 5),
                     o2_edges=linbins(0.0, 1.0, 3)),
    "rp_pi-64": dict(L=120.0, N=64, pair_mode="rp_pi", p1_edges=linbins(0.0, 8.0, 3),
                     p2_edges=linbins(0.0, 8.0, 2), pair_dmax=9.0, out_mode="rp_pi",
                     o1_edges=linbins(0.0, 30.0, 4), o2_edges=linbins(0.0, 30.0, 3)),
}


def case(name, seed=21):
    kw = dict(CASES[name])
    wl = Workload(name=name, precision="fp32", catalog_kw={}, assignment="tsc", **kw)
    cat = clustered_catalog(wl.L, 120, 2500, seed=seed, sat=6, spread=1.5)
    w = np.random.default_rng(seed).uniform(0.5, 1.5, cat.n).astype(np.float32).astype(np.float64)
    return wl, cat, w


@pytest.mark.parametrize("algo", [0, 1, 2])
@pytest.mark.parametrize("name", list(CASES))
def test_tsc_forward_against_oracle(name, algo):
    from paper_1705_03464_amd import Plan
    wl, cat, w = case(name)
    ref = oracle_forward(cat, wl, w=w)
    plan = Plan.from_workload(wl, precision="fp32", batch=2)
    P, counts = plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    _say(f"TSC {name}: n_gal={cat.n} pairs={P} evaluation {ALGOS[algo]}")
    assert np.array_equal(counts.cpu().numpy(), ref["counts"])
    plan.set_schedule(2, 0, 0, *ALGOS[algo])
    out = {k: v.cpu().numpy() for k, v in plan.forward(dev(w, torch.float32)).items()}
    assert_fp32_parity(out, ref)
    # the scheme is applied: CIC gives a different xi_gg
    ref_c = oracle_forward(cat, wl.scaled(assignment="cic"), w=w, fields=[])
    assert np.max(np.abs(ref_c["xi_gg"] - ref["xi_gg"])) > 1e-3 * np.max(np.abs(ref["xi_gg"]))


@pytest.mark.parametrize("keep,algo", [(False, 0), (True, 0), (False, 1), (False, 2)])
@pytest.mark.parametrize("name", ["s_mu-64", "rp_pi-64"])
def test_tsc_adjoint_against_oracle(name, keep, algo):
    from paper_1705_03464_amd import Plan
    wl, cat, w = case(name, seed=22)
    g = upstream(wl.n_fields, wl.n_out, 5)
    g = mask_ill_conditioned_q(g, wl, oracle_forward(cat, wl, w=w))
    ref, _ = OG.weight_gradient(cat, wl, w, **g)
    plan = Plan.from_workload(wl, precision="fp32", batch=2)
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.set_schedule(2, 0, 0, *ALGOS[algo])
    plan.keep_spectra(keep)
    for call in range(2):
        plan.forward(dev(w, torch.float32))
        gw = plan.backward(g_b_pg=dev(g["g_b"]), g_q_eff=dev(g["g_q"]), g_xi_pg=dev(g["g_xipg"]),
                           g_xi_gg=dev(g["g_xigg"]), g_xi_dp=dev(g["g_xidp"]))
        gw = gw.cpu().numpy().astype(np.float64)
        _say(f"TSC adjoint {name}, evaluation {ALGOS[algo]}, kept spectra {keep}, call {call}:")
        assert grad_close(gw, ref)


def test_tsc_adjoint_against_finite_differences():
    from paper_1705_03464_amd import Plan
    wl, cat, w = case("s_mu-64", seed=23)
    g = upstream(wl.n_fields, wl.n_out, 6)
    g["g_b"] = np.zeros_like(g["g_b"])
    g["g_q"] = np.zeros_like(g["g_q"])
    plan = Plan.from_workload(wl, precision="fp32", batch=2)
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.forward(dev(w, torch.float32))
    gw = plan.backward(g_b_pg=dev(g["g_b"]), g_q_eff=dev(g["g_q"]), g_xi_pg=dev(g["g_xipg"]),
                       g_xi_gg=dev(g["g_xigg"]), g_xi_dp=dev(g["g_xidp"])).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(3)
    idx = np.concatenate([np.argsort(-np.abs(gw))[:6], rng.choice(cat.n, 6, replace=False)])
    fd = OG.fd_weight_gradient(cat, wl, w, idx, h=1e-3, **g)
    err = np.abs(gw[idx] - fd)
    _say(f"TSC fd max abs err {err.max():.3e} scale {np.abs(gw).max():.3e}")
    assert np.all(err <= 1e-3 * np.abs(gw).max())


def test_tsc_plans_tune_both_evaluations_and_refuse_multipoles():
    """The autotuner measures the TSC dual form against the TSC per-field
    transforms (its check is reported); the multipoles refuse TSC plans."""
    from paper_1705_03464_amd import PgxError, Plan
    wl, cat, w = case("s_mu-64", seed=24)
    plan = Plan.from_workload(wl, precision="fp32", batch=2)
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.forward(dev(w, torch.float32))
    sched = plan.autotune()
    _say(f"  TSC autotuned {sched}, dual-form check {plan.dual_check():.3f}")
    assert plan.dual_check() >= 0.0
    plan.forward(dev(w, torch.float32))
    with pytest.raises(PgxError) as e:
        plan.multipoles(2)
    assert e.value.code == 4


def test_tsc_hod_subset_matches_the_fp64_plain_path():
    """The tiny HOD subset with TSC: the FP32 batched forward against the FP64
    plain path on the same plan parameters (both TSC)."""
    from paper_1705_03464_amd import Plan
    wl = get_config("cfg4tiny").scaled(assignment="tsc")
    cat = wl.catalog()
    out = {}
    for prec in ("fp32", "fp64"):
        plan = Plan.from_workload(wl, precision=prec)
        plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
        out[prec] = {k: v.cpu().numpy() for k, v in plan.forward().items()}
        plan.close()
    ref = oracle_forward(cat, wl)
    for k in ("xi_gg", "xi_pg"):
        fin = np.isfinite(ref[k])
        assert np.allclose(out["fp64"][k][fin], ref[k][fin], rtol=1e-9, atol=1e-12)
        d = np.abs(out["fp32"][k][fin] - ref[k][fin])
        floor = 2.0 ** -23 * float(np.max(np.abs(ref["xi_pg"][np.isfinite(ref["xi_pg"])])))
        assert np.all(d <= np.maximum(1e-5 * np.abs(ref[k][fin]), floor)), k


@pytest.mark.parametrize("algo", [0, 2])
def test_tsc_at_512_against_oracle(algo):
    """512^3 (lines of one wavefront: the scatters' run sums over three x
    nodes are active): the production catalogue with 4 s-bins and 6 shells,
    forward at the FP32 bar and adjoint at the gradient bar against the
    oracle, per-field and in the dual form on the kernel-spectrum store."""
    from paper_1705_03464_amd import Plan
    base = get_config("cfg1")
    wl = base.scaled(name="cfg1-tsc", p1_edges=logbins(0.5, 10.0, 4), p2_edges=linbins(0.0, 1.0, 1),
                     out_mode="shell", o1_edges=logbins(10.0, 80.0, 6), o2_edges=None, assignment="tsc")
    cat = wl.catalog()
    w = np.random.default_rng(11).uniform(0.5, 1.5, cat.n).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(12)
    g = dict(g_xipg=rng.normal(size=(wl.n_fields, wl.n_out)), g_xigg=rng.normal(size=wl.n_out),
             g_xidp=rng.normal(size=wl.n_fields))
    ref, rout = OG.weight_gradient(cat, wl, w, **g)
    plan = Plan.from_workload(wl, precision="fp32")
    P, counts = plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    _say(f"TSC 512^3: n_gal={cat.n} pairs={P}")
    assert np.array_equal(counts.cpu().numpy(), rout["counts"])
    plan.set_schedule(4, 0, 0, *ALGOS[algo])
    plan.keep_spectra(True)
    out = {k: v.cpu().numpy() for k, v in plan.forward(dev(w, torch.float32)).items()}
    assert_fp32_parity(out, rout)
    gw = plan.backward(g_xi_pg=dev(g["g_xipg"]), g_xi_gg=dev(g["g_xigg"]),
                       g_xi_dp=dev(g["g_xidp"])).cpu().numpy().astype(np.float64)
    assert grad_close(gw, ref)
