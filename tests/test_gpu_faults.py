"""Error paths forced from the host.  An injected failure of each device
allocation in turn (PGX_DEBUG_FAIL_ALLOC = n) during a pair build, forward
and adjoint must come back through the C-ABI as PGX_EHIP with a message, and
the same plan must then rebuild and give the results of a plan that never
failed.  Every failure is raised on the host before the allocation it
replaces: no kernel runs with a missing buffer."""
import os
import sys

import numpy as np
import pytest

from synth import get_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

VAR = "PGX_DEBUG_FAIL_ALLOC"


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(plan, cat, w, g):
    dev = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    out = {k: v.cpu().numpy() for k, v in plan.forward(w).items()}
    grad = plan.backward(g_xi_pg=g).cpu().numpy()
    torch.cuda.synchronize()
    return out, grad


def test_injected_allocation_failures_are_reported_and_recovered():
    from paper_1705_03464_amd import Plan, PgxError
    wl = get_config("cfg4tiny")
    cat = wl.catalog()
    rng = np.random.default_rng(3)
    w = torch.as_tensor(rng.uniform(0.5, 1.5, cat.n).astype(np.float32), device="cuda")
    g = torch.as_tensor(rng.normal(size=(wl.n_fields, wl.n_out)), device="cuda")
    os.environ.pop(VAR, None)
    ref_plan = Plan.from_workload(wl, precision="fp32")
    ref, ref_grad = _run(ref_plan, cat, w, g)
    ref_plan.close()
    failures = 0
    for n in range(1, 400):
        plan = Plan.from_workload(wl, precision="fp32")
        os.environ[VAR] = str(n)
        try:
            _run(plan, cat, w, g)
            hit = None
        except PgxError as e:
            hit = e
        finally:
            os.environ.pop(VAR, None)
        if hit is None:
            _say(f"  allocation {n}: past the last allocation of the run ({failures} injected failures)")
            plan.close()
            break
        assert hit.code == 3 and "injected" in str(hit), str(hit)
        failures += 1
        # the same plan rebuilds and matches a plan that never failed
        out, grad = _run(plan, cat, w, g)
        plan.close()
        for k in ("xi_gg", "xi_pg", "b_pg"):
            assert np.allclose(out[k], ref[k], rtol=1e-6, atol=1e-12, equal_nan=True), (n, k)
        assert np.allclose(grad, ref_grad, rtol=1e-5, atol=1e-6 * np.abs(ref_grad).max()), n
    assert failures >= 10


def test_invalid_inputs_are_rejected_and_the_plan_stays_usable():
    """Non-finite or out-of-box positions and negative or non-finite weights
    give PGX_EINVAL with a message; a rejected pair build leaves the plan
    without a catalogue (PGX_ESTATE until the next build); the plan then runs
    a valid catalogue."""
    from paper_1705_03464_amd import Plan, PgxError
    wl = get_config("cfg4tiny")
    cat = wl.catalog()
    dev = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    plan = Plan.from_workload(wl, precision="fp32")
    for bad in (np.nan, np.inf, -1e-9, wl.L):
        x = cat.x.copy()
        x[7] = bad
        with pytest.raises(PgxError) as e:
            plan.pairs_build(dev(x), dev(cat.y), dev(cat.z))
        assert e.value.code == 1, (bad, str(e.value))
    P, _ = plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    assert P > 0
    for bad in (-0.5, np.nan, np.inf):
        w = np.ones(cat.n, np.float32)
        w[11] = bad
        with pytest.raises(PgxError) as e:
            plan.forward(dev(w, torch.float32))
        assert e.value.code == 1, (bad, str(e.value))
        with pytest.raises(PgxError) as e:
            plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z), w=dev(w, torch.float32), with_wsum=True)
        assert e.value.code == 1, (bad, str(e.value))
        # a rejected build leaves no catalogue behind: a forward now asks for one
        with pytest.raises(PgxError) as e:
            plan.forward()
        assert e.value.code == 5, str(e.value)
        plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    plan.pairs_build(dev(cat.x), dev(cat.y), dev(cat.z))
    out = plan.forward()
    assert np.isfinite(out["xi_gg"].cpu().numpy()).all()
    plan.close()
