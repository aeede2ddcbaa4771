"""The production-size code paths against the oracle (not against another
HIP path): the adjoint at 256^3 and 512^3 (three-stage line transforms,
buffer-resource addressing, kept spectra, graph replays) for all three
evaluations, and the l = 2 multipole at 512^3 on sampled fields.

Few-field workloads keep the oracle affordable: the production catalogues
with 4 logarithmic s-bins and one |mu| bin, and 6 output shells over
10-80 Mpc/h.  Gradient bar: ||dg||_2 <= 1e-3 ||g||_2 and
max |dg| <= 1e-3 max |g|."""
import functools
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import grad as OG  # noqa: E402
from oracle import multipoles as OM  # noqa: E402
from oracle.pairs import pairs_for  # noqa: E402
from oracle.pipeline import galaxy_side  # noqa: E402
from synth import get_config  # noqa: E402
from synth.configs import linbins, logbins  # noqa: E402
from test_gpu_parity import ALGOS, xi_err_ok  # noqa: E402

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


def few_field(name):
    base = get_config(name)
    return base.scaled(name=f"{name}-few", p1_edges=logbins(0.5, 10.0, 4), p2_edges=linbins(0.0, 1.0, 1),
                       out_mode="shell", o1_edges=logbins(10.0, 80.0, 6), o2_edges=None)


@functools.lru_cache(maxsize=2)
def oracle_case(name):
    wl = few_field(name)
    cat = wl.catalog()
    w = np.random.default_rng(11).uniform(0.5, 1.5, cat.n).astype(np.float32).astype(np.float64)
    pairs = pairs_for(cat, wl)
    rng = np.random.default_rng(12)
    g_xipg = rng.normal(size=(wl.n_fields, wl.n_out))
    g_xigg = rng.normal(size=wl.n_out)
    g_xidp = rng.normal(size=wl.n_fields)
    grad, out = OG.weight_gradient(cat, wl, w, g_xipg=g_xipg, g_xigg=g_xigg, g_xidp=g_xidp,
                                   pairs=pairs)
    return wl, cat, w, pairs, (g_xipg, g_xigg, g_xidp), grad, out


@pytest.mark.parametrize("name", ["cfg2", "cfg1"])
@pytest.mark.parametrize("algo", [0, 1, 2])
def test_adjoint_at_production_grid_against_oracle(name, algo):
    from paper_1705_03464_amd import Plan
    wl, cat, w, pairs, (gp, gg, gd), ref, rout = oracle_case(name)
    _say(f"adjoint {wl.name} N={wl.N} algorithm {ALGOS[algo]}: n_gal={cat.n}, pairs={pairs['key'].size}")
    plan = Plan.from_workload(wl, precision="fp32")
    P, counts = plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    assert P == pairs["key"].size and np.array_equal(counts.cpu().numpy(), pairs["counts"])
    zp, al = ALGOS[algo]
    plan.set_schedule(plan.schedule()["batch"], 0, 0, zp, al)
    plan.keep_spectra(True)
    wt = dev(w, torch.float32)
    # eager, then recorded, then replayed (the graphs are captured on the
    # second call with the same key)
    for call in range(3):
        out = plan.forward(wt)
        g = plan.backward(g_xi_pg=dev(gp), g_xi_gg=dev(gg), g_xi_dp=dev(gd)).cpu().numpy().astype(np.float64)
        d = g - ref
        l2 = np.linalg.norm(d) / np.linalg.norm(ref)
        mx = np.abs(d).max() / np.abs(ref).max()
        _say(f"  call {call}: rel l2 {l2:.2e}, rel max {mx:.2e}; xi_pg worst "
             f"{xi_err_ok(out['xi_pg'].cpu().numpy(), rout['xi_pg']):.3f} of the 1e-5 bar")
        assert l2 <= 1e-3 and mx <= 1e-3
    fr, br = plan.graph_replays()
    _say(f"  graph replays (fwd, bwd): {fr}, {br}")
    assert fr >= 1 and br >= 1
    plan.close()


def test_multipole_l2_at_512_against_oracle():
    """l = 0 and l = 2 of the 512^3 production catalogue's pair fields in the
    angle between the pair axis and the pair-to-galaxy direction, against the
    oracle's addition-theorem route on three sampled fields (6 shells)."""
    from paper_1705_03464_amd import Plan
    base = get_config("cfg1")
    wl = base.scaled(name="cfg1-mp", out_mode="shell", o1_edges=logbins(10.0, 80.0, 6), o2_edges=None)
    cat = wl.catalog()
    pairs = pairs_for(cat, wl)
    order = [int(f) for f in np.argsort(pairs["counts"], kind="stable") if pairs["counts"][f] > 0]
    fields = [order[-1], order[len(order) // 2], order[0]]
    sub = dict(pairs)
    sel = np.isin(pairs["key"], fields)
    for k in ("key", "i", "j", "w", "mid"):
        sub[k] = pairs[k][sel]
    gal = galaxy_side(cat, wl)
    exp = OM.multipoles_fft(cat, wl, sub, gal["dg"], ells=(0, 2), Fg=gal["Fg"])
    plan = Plan.from_workload(wl, precision="fp32")
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.forward(None)
    got = plan.multipoles(2).cpu().numpy()
    plan.close()
    for il in range(2):
        worst = xi_err_ok(got[fields, :, il], exp[fields, :, il])
        _say(f"  multipole l={2 * il} fields {fields} (pairs {[int(pairs['counts'][f]) for f in fields]}): "
             f"worst {worst:.3f} of the 1e-5 bar")
        assert worst <= 1.0
