"""The allocation-free forward (pgx_forward_fixed) against pgx_forward on the
same FP64 plain plan, through the C-ABI: two calls in a row, the second on a
smaller catalogue, each to the FP64 bar (1e-9 relative, 1e-12 floor); the
plan's own forward still works afterwards and sizes beyond the fixed scratch
are refused."""
import sys

import numpy as np
import pytest

from synth.catalog import Catalog
from synth.configs import linbins, logbins

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


def _catalog(L, n_halo, n_field, seed):
    rng = np.random.default_rng(seed)
    c = rng.random((n_halo, 3)) * L
    s = np.repeat(c, 8, axis=0) + rng.normal(0.0, 1.5, (n_halo * 8, 3))
    pos = np.mod(np.concatenate([c, s, rng.random((n_field, 3)) * L]), L)
    pos[pos >= L] = 0.0
    n = pos.shape[0]
    return Catalog(L, pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.zeros(n),
                   np.zeros(n, np.int8))


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _same(a, b, what):
    for k in ("wsum", "xi_gg", "xi_pg", "xi_dp", "b_pg", "q_eff"):
        x = a[k].cpu().numpy(); y = b[k].cpu().numpy()
        fin = np.isfinite(y)
        assert np.array_equal(fin, np.isfinite(x)), (what, k)
        assert np.allclose(x[fin], y[fin], rtol=1e-9, atol=1e-12), (what, k)


def test_fixed_scratch_forward_matches_forward_twice():
    from paper_1705_03464_amd import Plan
    L = 100.0
    plan = Plan(L, 64, linbins(0.5, 8.0, 3), linbins(0.0, 1.0, 2), logbins(6.0, 40.0, 7),
                precision="fp64")
    for call, (n_halo, n_field, seed, weighted) in enumerate([(200, 8000, 0, True), (90, 3000, 1, False)]):
        cat = _catalog(L, n_halo, n_field, seed)
        _say(f"fixed-scratch forward, call {call}: n_gal={cat.n}, weighted={weighted}")
        P, _ = plan.pairs_build(_dev(cat.x), _dev(cat.y), _dev(cat.z))
        w = None
        if weighted:
            w = _dev(np.random.default_rng(7).uniform(0.5, 1.5, cat.n), torch.float32)
        ref = plan.forward(w)
        got = plan.forward_fixed(w)
        torch.cuda.synchronize()
        _say(f"  {P} pairs; comparing with pgx_forward")
        _same(got, ref, f"call {call}")
    # the plan's own forward is unaffected by the fixed-scratch calls
    again = plan.forward(None)
    torch.cuda.synchronize()
    _same(again, ref, "forward after the fixed-scratch calls")
    plan.close()


def test_fixed_scratch_forward_refuses_what_does_not_fit():
    from paper_1705_03464_amd import Plan, PgxError
    L = 400.0
    plan = Plan(L, 256, linbins(0.5, 8.0, 2), [0.0, 1.0], logbins(10.0, 60.0, 5), precision="fp64")
    cat = _catalog(L, 50, 2000, 3)
    plan.pairs_build(_dev(cat.x), _dev(cat.y), _dev(cat.z))
    with pytest.raises(PgxError) as e:
        plan.forward_fixed(None)
    assert e.value.code == 2 and "fixed scratch" in str(e.value)
    plan.close()
