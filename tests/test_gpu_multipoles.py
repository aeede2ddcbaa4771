"""GPU multipoles of xi_pg in the angle between the pair axis and the
pair-to-galaxy direction (pgx_multipoles) against the oracle's addition-theorem
route (itself pinned to the definition on the CPU).

Bar: the FP32 bar of xi_pg, |d| <= 1e-5 max(|xi_l|, 1e-2), per multipole.
"""
import sys
import time

import numpy as np
import pytest

from oracle import multipoles as OM
from oracle.pipeline import forward as oracle_forward, galaxy_side
from synth import get_config
from synth.configs import Workload, linbins, logbins

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_parity import ALGOS, clustered_catalog, xi_err_ok  # noqa: E402

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


def small(seed=21):
    L = 120.0
    wl = Workload(name="mp", L=L, N=64, precision="fp32", pair_mode="s_mu",
                  p1_edges=logbins(0.5, 9.0, 3), p2_edges=linbins(0.0, 1.0, 2), out_mode="shell",
                  o1_edges=logbins(6.0, 50.0, 5), o2_edges=None, catalog_kw={})
    cat = clustered_catalog(L, 250, 6000, seed=seed, sat=6, spread=2.0)
    w = np.random.default_rng(seed).uniform(0.4, 1.6, cat.n).astype(np.float32).astype(np.float64)
    return wl, cat, w


def oracle_multipoles(wl, cat, w, ells):
    ref = oracle_forward(cat, wl, w=w)
    gal = galaxy_side(cat, wl, w=w)
    return OM.multipoles_fft(cat, wl, ref["pairs"], gal["dg"], ells=ells, Fg=gal["Fg"]), ref


@pytest.mark.parametrize("algo", [0, 1])
@pytest.mark.parametrize("batch", [2, 16])
def test_multipoles_small_grid_vs_oracle(algo, batch):
    """lmax = 4 after a forward of either algorithm, several combo batches
    (batch 2) or one (batch 16)."""
    from paper_1705_03464_amd import Plan
    wl, cat, w = small()
    exp, ref = oracle_multipoles(wl, cat, w, OM.EVEN_L)
    plan = Plan.from_workload(wl, precision="fp32", batch=batch)
    P, _ = plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.set_schedule(batch, 0, 0, *ALGOS[algo])
    out = {k: v.cpu().numpy() for k, v in plan.forward(dev(w, torch.float32)).items()}
    got = plan.multipoles(4).cpu().numpy()
    _say(f"multipoles 64^3 algorithm {algo} batch {batch}: pairs={P} "
         f"max |xi_0| {np.nanmax(np.abs(exp[..., 0])):.3f} |xi_2| {np.nanmax(np.abs(exp[..., 1])):.3f} "
         f"|xi_4| {np.nanmax(np.abs(exp[..., 2])):.3f}")
    assert got.shape == (wl.n_fields, wl.n_out, 3)
    for il, l in enumerate(OM.EVEN_L):
        worst = xi_err_ok(got[..., il], exp[..., il])
        _say(f"  l={l}: worst |d| / (1e-5 max(|xi|,1e-2)) = {worst:.3f}")
        assert worst <= 1.0, l
    # l = 0 is the shell estimator: the forward's xi_pg of the same plan
    assert xi_err_ok(got[..., 0], out["xi_pg"]) <= 1.0
    assert xi_err_ok(out["xi_pg"], ref["xi_pg"]) <= 1.0


def test_multipoles_lower_lmax_is_a_prefix():
    from paper_1705_03464_amd import Plan
    wl, cat, w = small(seed=5)
    plan = Plan.from_workload(wl, precision="fp32", batch=4)
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.forward(dev(w, torch.float32))
    m4 = plan.multipoles(4).cpu().numpy()
    m2 = plan.multipoles(2).cpu().numpy()
    m0 = plan.multipoles(0).cpu().numpy()
    assert xi_err_ok(m2, m4[..., :2]) <= 1.0
    assert xi_err_ok(m0, m4[..., :1]) <= 1.0


def test_multipoles_validation():
    from paper_1705_03464_amd import PgxError, Plan
    wl, cat, w = small(seed=6)
    plan = Plan.from_workload(wl, precision="fp32")
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    with pytest.raises(PgxError) as e:
        plan.multipoles(2)  # no forward yet
    assert e.value.code == 5
    plan.forward()
    for bad in (1, 3, 6, -2):
        with pytest.raises(PgxError) as e:
            plan.multipoles(bad)
        assert e.value.code == 1
    rmu = Plan(wl.L, wl.N, wl.p1_edges, wl.p2_edges, logbins(6.0, 50.0, 5), linbins(0.0, 1.0, 2),
               out_mode="r_mu", precision="fp32")
    rmu.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    rmu.forward()
    with pytest.raises(PgxError) as e:
        rmu.multipoles(2)
    assert e.value.code == 1
    zero = Plan(wl.L, wl.N, wl.p1_edges, wl.p2_edges, np.array([0.0, 10.0, 30.0]), precision="fp32")
    zero.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    zero.forward()
    with pytest.raises(PgxError) as e:
        zero.multipoles(2)
    assert e.value.code == 1


def test_multipoles_production_512():
    """The 512^3 production catalogue with its 20 shells, lmax = 2 (120 bin
    kernels): l = 0 against the forward's xi_pg (the dual form's bins), every
    multipole of a non-empty field finite, and the time of one call."""
    from paper_1705_03464_amd import Plan
    wl = get_config("cfg1")
    cat = wl.catalog()
    plan = Plan.from_workload(wl, precision="fp32")
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.set_schedule(16, 0, 0, *ALGOS[1])
    out = {k: v.cpu().numpy() for k, v in plan.forward().items()}
    plan.multipoles(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m = plan.multipoles(2).cpu().numpy()
    dt = time.perf_counter() - t0
    worst0 = xi_err_ok(m[..., 0], out["xi_pg"], 2e-5)
    _say(f"cfg1 multipoles lmax 2: {dt * 1e3:.1f} ms per call; l=0 vs xi_pg worst / (2e-5 max) = {worst0:.3f}; "
         f"|xi_2| max {np.nanmax(np.abs(m[..., 1])):.3f}")
    assert worst0 <= 1.0
    assert np.all(np.isfinite(m[np.isfinite(out["xi_pg"])]))


def small_fd(seed=33):
    L = 120.0
    wl = Workload(name="mpfd", L=L, N=64, precision="fp32", pair_mode="s_mu",
                  p1_edges=logbins(0.5, 9.0, 2), p2_edges=linbins(0.0, 1.0, 2), out_mode="shell",
                  o1_edges=logbins(6.0, 40.0, 4), o2_edges=None, catalog_kw={})
    cat = clustered_catalog(L, 150, 1500, seed=seed, sat=6, spread=2.0)
    w = np.random.default_rng(seed).uniform(0.5, 1.5, cat.n).astype(np.float32).astype(np.float64)
    return wl, cat, w


@pytest.mark.parametrize("lmax", [2, 4])
def test_multipole_gradient_matches_oracle_finite_differences(lmax):
    """dL/dw of L = sum g xi_l through pgx_multipoles_backward against central
    differences of the oracle's multipoles (the 1e-3 gradient bar, relative
    to the largest gradient entry)."""
    from paper_1705_03464_amd import Plan
    wl, cat, w = small_fd()
    ells = OM.EVEN_L[: lmax // 2 + 1]
    ref = oracle_forward(cat, wl, w=w)
    plan = Plan.from_workload(wl, precision="fp32", batch=4)
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.forward(dev(w, torch.float32))
    xi = plan.multipoles(lmax).cpu().numpy()
    g = np.random.default_rng(lmax).normal(size=xi.shape)
    g[~np.isfinite(xi)] = 0.0
    gw = plan.multipoles_backward(dev(g)).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(7)
    idx = np.concatenate([np.argsort(-np.abs(gw))[:6], rng.choice(cat.n, 6, replace=False)])
    fd = OM.fd_weight_gradient(cat, wl, w, idx, g, ref["pairs"], ells=ells, h=1e-3)
    err = np.abs(gw[idx] - fd)
    _say(f"multipole adjoint lmax {lmax}: pairs={ref['pairs']['key'].size} fd max abs err {err.max():.3e} "
         f"scale {np.abs(gw).max():.3e}")
    assert np.all(err <= 1e-3 * np.abs(gw).max())


def test_multipole_autograd_and_state():
    from paper_1705_03464_amd import PgxError, Plan, pair_galaxy_multipoles
    wl, cat, w = small_fd(seed=34)
    plan = Plan.from_workload(wl, precision="fp32", batch=4)
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.forward(dev(w, torch.float32))
    with pytest.raises(PgxError) as e:
        plan.multipoles_backward(torch.zeros(wl.n_fields, wl.n_out, 2, dtype=torch.float64, device="cuda"))
    assert e.value.code == 5  # no multipoles after the forward
    wt = dev(w, torch.float32).requires_grad_(True)
    xi = pair_galaxy_multipoles(plan, wt, 2)
    G = dev(np.random.default_rng(2).normal(size=tuple(xi.shape)))
    loss = (torch.where(torch.isfinite(xi), xi, torch.zeros_like(xi)) * G).sum()
    loss.backward()
    plan.forward(dev(w, torch.float32))
    xi2 = plan.multipoles(2)
    Gm = torch.where(torch.isfinite(xi2), G, torch.zeros_like(G))
    direct = plan.multipoles_backward(Gm).cpu().numpy().astype(np.float64)
    got = wt.grad.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - direct)) <= 1e-5 * np.max(np.abs(direct))
    plan.forward(dev(w, torch.float32))
    with pytest.raises(PgxError) as e:
        plan.multipoles_backward(Gm)  # a new forward invalidates the multipoles
    assert e.value.code == 5


def test_multipoles_empty_fields_and_their_adjoint_128():
    """A sparse catalogue on a 128^3 grid: pair fields without pairs give NaN
    rows (as xi_pg does), the others meet the oracle, and the adjoint
    ignores whatever upstream gradient sits on the NaN rows."""
    from paper_1705_03464_amd import Plan
    L = 200.0
    wl = Workload(name="mpe", L=L, N=128, precision="fp32", pair_mode="s_mu",
                  p1_edges=np.array([0.1, 0.3, 3.0, 9.0]), p2_edges=linbins(0.0, 1.0, 2), out_mode="shell",
                  o1_edges=logbins(6.0, 40.0, 4), o2_edges=None, catalog_kw={})
    cat = clustered_catalog(L, 60, 3000, seed=44, sat=4, spread=2.5)
    w = np.random.default_rng(44).uniform(0.5, 1.5, cat.n).astype(np.float32).astype(np.float64)
    exp, ref = oracle_multipoles(wl, cat, w, (0, 2))
    plan = Plan.from_workload(wl, precision="fp32", batch=4)
    P, counts = plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.forward(dev(w, torch.float32))
    got = plan.multipoles(2).cpu().numpy()
    counts = counts.cpu().numpy()
    _say(f"multipoles 128^3 sparse: pairs={P} per field {counts.tolist()}")
    assert np.any(counts == 0) and np.any(counts > 0)
    assert np.all(np.isnan(got[counts == 0]))
    for il in range(2):
        assert xi_err_ok(got[..., il], exp[..., il]) <= 1.0, il
    g = np.random.default_rng(5).normal(size=got.shape)
    g0 = np.where(np.isfinite(got), g, 0.0)
    a = plan.multipoles_backward(dev(g)).cpu().numpy()
    b = plan.multipoles_backward(dev(g0)).cpu().numpy()
    assert np.all(np.isfinite(a))
    assert np.max(np.abs(a - b)) <= 1e-6 * max(np.max(np.abs(b)), 1e-30)
