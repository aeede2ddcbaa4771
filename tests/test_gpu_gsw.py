"""The paper's Gaussian-sigmoid weighting function as one weighted output
bin (out_mode "gsw"), through the C-ABI on the device, against the oracle:
forward (both FP32 algorithms and the FP64 path), adjoint (both algorithms),
and the 512^3 production catalogue against the FP64 path."""
import sys

import numpy as np
import pytest

from oracle import grad as OG
from oracle.pipeline import forward as oracle_forward
from synth import get_config
from synth.configs import Workload, linbins, logbins

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from test_gpu_parity import ALGOS, assert_fp32_parity, assert_fp64_parity, clustered_catalog, xi_err_ok  # noqa: E402

PAR = np.array([15.0, 10.0, 0.8, 5.0, 60.0])  # sigma, r_s, s_0, r_cut, r_max (L = 200, 64^3)


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def small(precision="fp32"):
    L = 200.0
    wl = Workload(name="gsw", L=L, N=64, precision=precision, pair_mode="s_mu",
                  p1_edges=logbins(0.5, 8.0, 3), p2_edges=linbins(0.0, 1.0, 3),
                  out_mode="gsw", o1_edges=PAR, o2_edges=None, catalog_kw={},
                  qeff_mode="const", xi_w_const=0.362)
    cat = clustered_catalog(L, 600, 24000, seed=12, sat=8, spread=1.5)
    w = np.random.default_rng(12).uniform(0.3, 1.7, cat.n).astype(np.float32).astype(np.float64)
    return wl, cat, w


@pytest.mark.parametrize("algo", [0, 1, 2])
def test_gsw_forward_small_grid(algo):
    from paper_1705_03464_amd import Plan
    wl, cat, w = small()
    ref = oracle_forward(cat, wl, w=w)
    plan = Plan.from_workload(wl, precision="fp32", batch=2)
    P, counts = plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.set_schedule(2, 0, 0, *ALGOS[algo])
    out = {k: v.cpu().numpy() for k, v in plan.forward(dev(w, torch.float32)).items()}
    _say(f"gsw 64^3 algorithm {algo}: n_gal={cat.n} pairs={P} xi_gg={ref['xi_gg'][0]:.4f}")
    assert np.array_equal(counts.cpu().numpy(), ref["counts"])
    assert np.allclose(plan.out_norms(), ref["norm_b"], rtol=1e-12)
    assert_fp32_parity(out, ref)
    fin = np.isfinite(ref["q_eff"])
    assert np.allclose(out["q_eff"][fin], ref["q_eff"][fin], rtol=1e-4, atol=1e-6)


def test_gsw_forward_small_grid_fp64():
    from paper_1705_03464_amd import Plan
    wl, cat, w = small("fp64")
    ref = oracle_forward(cat, wl, w=w)
    plan = Plan.from_workload(wl, precision="fp64")
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    out = {k: v.cpu().numpy() for k, v in plan.forward(dev(w, torch.float32)).items()}
    assert_fp64_parity(out, ref)


@pytest.mark.parametrize("algo", [0, 1, 2])
def test_gsw_adjoint_small_grid(algo):
    from paper_1705_03464_amd import Plan
    wl, cat, w = small()
    rng = np.random.default_rng(3)
    g = dict(g_b=rng.normal(size=(wl.n_fields, 1)), g_xipg=rng.normal(size=(wl.n_fields, 1)),
             g_xigg=rng.normal(size=1), g_xidp=rng.normal(size=wl.n_fields))
    ref, _ = OG.weight_gradient(cat, wl, w, **g)
    plan = Plan.from_workload(wl, precision="fp32", batch=2)
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.set_schedule(2, 0, 0, *ALGOS[algo])
    plan.forward(dev(w, torch.float32))
    gw = plan.backward(g_b_pg=dev(g["g_b"]), g_xi_pg=dev(g["g_xipg"]), g_xi_gg=dev(g["g_xigg"]),
                       g_xi_dp=dev(g["g_xidp"])).cpu().numpy().astype(np.float64)
    l2 = np.linalg.norm(gw - ref) / np.linalg.norm(ref)
    mx = np.max(np.abs(gw - ref)) / np.max(np.abs(ref))
    _say(f"  gsw adjoint algorithm {algo}: rel l2 {l2:.2e} rel max {mx:.2e}")
    assert l2 <= 1e-3 and mx <= 1e-3


def test_gsw_production_512_against_fp64():
    """The production catalogue with the paper's d_p,max = 10 weighting
    function: both FP32 algorithms against the FP64 plain path."""
    from paper_1705_03464_amd import Plan
    wl = get_config("cfg1w")
    cat = wl.catalog()
    p64 = Plan.from_workload(wl, precision="fp64")
    p64.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    ref = {k: v.cpu().numpy() for k, v in p64.forward().items()}
    p64.close()
    for algo in (0, 1, 2):
        plan = Plan.from_workload(wl, precision="fp32")
        plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
        plan.set_schedule(16, 0, 0, *ALGOS[algo])
        out = {k: v.cpu().numpy() for k, v in plan.forward().items()}
        plan.close()
        for k in ("xi_gg", "xi_pg"):
            worst = xi_err_ok(out[k], ref[k], 1e-5)
            _say(f"  cfg1w algorithm {algo} {k}: worst / (1e-5 max(|xi|,1e-2)) vs FP64 = {worst:.3f}")
            assert worst <= 1.0, (algo, k)
        _say(f"  cfg1w b_pg range {np.nanmin(out['b_pg']):.3f}..{np.nanmax(out['b_pg']):.3f}")
