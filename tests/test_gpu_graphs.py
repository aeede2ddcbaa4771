"""Graph-recorded forward and adjoint against eager runs of the same plan
configuration: every replay, with eager torch work and synchronisations in
between, matches the eager result (the pair-field CIC scatter accumulates
with atomics, so runs agree to rounding, not bit for bit)."""
import sys

import numpy as np
import pytest

from synth import get_config

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_parity import ALGOS  # noqa: E402

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


def close(a, b, rel=1e-6):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    fa, fb = np.isfinite(a), np.isfinite(b)
    assert np.array_equal(fa, fb)
    d = np.abs(a[fa] - b[fa])
    return bool(np.all(d <= rel * np.maximum(np.abs(b[fa]), 1e-2)))


def eager_work():
    x = torch.randn(1 << 20, device="cuda")
    y = (x * 2.0).sum()
    torch.cuda.synchronize()
    return float(y)


def make(wl, cat, graphs, keep=False, algo=0):
    from paper_1705_03464_amd import Plan
    plan = Plan.from_workload(wl, precision="fp32", batch=2)
    plan.use_graphs(graphs)
    plan.keep_spectra(keep)
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    zp, al = ALGOS[algo]
    plan.set_schedule(2, 0, 0, zp, al)
    return plan


@pytest.mark.parametrize("algo", [0, 1, 2])
@pytest.mark.parametrize("name", ["cfg4tiny", "cfg2"])
def test_forward_graph_replays_match_eager(name, algo):
    wl = get_config(name)
    cat = wl.catalog()
    _say(f"{name}: n_gal={cat.n} N={wl.N}")
    w = dev(np.random.default_rng(11).uniform(0.5, 1.5, cat.n), torch.float32)
    pe = make(wl, cat, graphs=False, algo=algo)
    ref = {k: v.cpu().numpy() for k, v in pe.forward(w).items()}
    pg = make(wl, cat, graphs=True, algo=algo)
    for i in range(4):
        out = {k: v.cpu().numpy() for k, v in pg.forward(w).items()}
        eager_work()
        for k in ("xi_gg", "xi_pg", "b_pg", "xi_dp"):
            assert close(out[k], ref[k]), (i, k)
    f, b = pg.graph_replays()
    _say(f"  forward replays {f}")
    assert f == 3 and b == 0
    assert pe.graph_replays() == (0, 0)


@pytest.mark.parametrize("keep,algo", [(False, 0), (True, 0), (False, 1), (False, 2)])
def test_adjoint_graph_replays_match_eager(keep, algo):
    wl = get_config("cfg4tiny")
    cat = wl.catalog()
    rng = np.random.default_rng(12)
    w = dev(rng.uniform(0.5, 1.5, cat.n), torch.float32)
    g_xipg = dev(rng.normal(size=(wl.n_fields, wl.n_out)))
    g_xigg = dev(rng.normal(size=wl.n_out))

    def run(plan):
        plan.forward(w)
        return plan.backward(g_xi_pg=g_xipg, g_xi_gg=g_xigg).cpu().numpy().astype(np.float64)

    ref = run(make(wl, cat, graphs=False, keep=keep, algo=algo))
    pg = make(wl, cat, graphs=True, keep=keep, algo=algo)
    for i in range(4):
        gw = run(pg)
        eager_work()
        d = np.linalg.norm(gw - ref) / np.linalg.norm(ref)
        _say(f"  replay {i}: rel l2 {d:.2e}")
        assert d <= 1e-6
    f, b = pg.graph_replays()
    assert f == 3 and b == 3
