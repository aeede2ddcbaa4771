"""Pins of the oracle's TSC mass assignment (the paper's scheme): the 1-D
weights against their moments and the on-node values, the 3-D assignment
against the CIC assignment averaged over a unit box of shifts (TSC is CIC
convolved with one more cell-wide box), the interpolation (gather) against
the polynomials it reproduces and as the adjoint of the assignment, and the
oracle's weight gradient with TSC against finite differences."""
import numpy as np

from oracle import grad as G
from oracle.cic import cic_assign, tsc_assign, tsc_gather, tsc_weights_1d
from synth.catalog import Catalog
from synth.configs import Workload, linbins


def test_tsc_weights_moments_and_on_node_values():
    u = np.concatenate([np.random.default_rng(0).random(500) * 64, [3.0, 3.5, 7.25, 0.0, 63.999]])
    lo, w = tsc_weights_1d(u)
    nodes = lo[:, None] + np.arange(3)[None, :]
    assert np.allclose(w.sum(1), 1.0, atol=1e-15)
    assert np.allclose((w * nodes).sum(1), u, atol=1e-12)                       # centroid
    assert np.allclose((w * (nodes - u[:, None]) ** 2).sum(1), 0.25, atol=1e-12)  # variance 3/12
    assert np.all(w >= 0)
    lo, w = tsc_weights_1d(np.array([5.0]))
    assert lo[0] == 4 and np.allclose(w[0], [0.125, 0.75, 0.125], atol=0)


def test_tsc_is_cic_averaged_over_a_unit_box_of_shifts():
    L, N = 16.0, 16
    pos = np.array([[3.3, 7.9, 12.02], [0.4, 15.7, 8.5], [5.0, 6.0, 7.0]])
    w = np.array([1.0, 0.6, 1.7])
    tsc = tsc_assign(pos, w, N, L)
    n = 40  # midpoint rule per axis on (-1/2, 1/2) cells
    t = (np.arange(n) + 0.5) / n - 0.5
    acc = np.zeros((N, N, N))
    d = L / N
    for a in t:
        for b in t:
            for c in t:
                acc += cic_assign(np.mod(pos + d * np.array([a, b, c]), L), w, N, L)
    acc /= n ** 3
    assert np.isclose(tsc.sum(), w.sum(), rtol=1e-14)
    assert np.max(np.abs(tsc - acc)) <= 1e-3 * np.max(tsc)


def test_tsc_gather_reproduces_linear_fields_and_shifts_the_square():
    """On nodes a = 0..N-1 along x the interpolated field a is u itself and
    a^2 is u^2 + 1/4 (the weights' variance), for points whose footprint
    does not wrap; constants are reproduced everywhere."""
    N, L = 32, 32.0
    rng = np.random.default_rng(4)
    pos = np.stack([2.0 + rng.random(300) * (N - 5.0), rng.random(300) * L, rng.random(300) * L], 1)
    a = np.arange(N, dtype=np.float64)
    lin = np.broadcast_to(a[:, None, None], (N, N, N))
    u = pos[:, 0] * (N / L)
    assert np.allclose(tsc_gather(lin, pos, N, L), u, atol=1e-12)
    assert np.allclose(tsc_gather(lin ** 2, pos, N, L), u * u + 0.25, atol=1e-10)
    assert np.allclose(tsc_gather(np.full((N, N, N), 2.5), rng.random((50, 3)) * L, N, L), 2.5, atol=1e-14)


def test_p13_tsc_assign_gather_adjoint():
    rng = np.random.default_rng(1)
    N, L = 12, 30.0
    pos = rng.random((200, 3)) * L
    v = rng.normal(size=200)
    fld = rng.normal(size=(N, N, N))
    assert np.isclose(np.sum(tsc_assign(pos, v, N, L) * fld), np.sum(v * tsc_gather(fld, pos, N, L)),
                      rtol=1e-13)


def test_p14_tsc_adjoint_matches_finite_differences():
    L = 40.0
    wl = Workload(name="t", L=L, N=16, precision="fp64", pair_mode="s_mu",
                  p1_edges=linbins(0.5, 6.0, 3), p2_edges=np.array([0.0, 0.5, 1.0]), out_mode="shell",
                  o1_edges=linbins(5.0, 17.0, 3), o2_edges=None, catalog_kw={}, assignment="tsc")
    rng = np.random.default_rng(0)
    c = rng.random((100, 3)) * L
    pos = np.mod(np.concatenate([c, np.repeat(c, 3, axis=0) + rng.normal(0, 1.5, (300, 3))]), L)
    cat = Catalog(L, pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.zeros(400), np.zeros(400, np.int8))
    w = rng.uniform(0.5, 1.5, cat.n)
    g = dict(g_xipg=rng.normal(size=(wl.n_fields, wl.n_out)), g_xigg=rng.normal(size=wl.n_out),
             g_b=rng.normal(size=(wl.n_fields, wl.n_out)), g_xidp=rng.normal(size=wl.n_fields))
    grad, out = G.weight_gradient(cat, wl, w, **g)
    idx = rng.choice(cat.n, 12, replace=False)
    fd = G.fd_weight_gradient(cat, wl, w, idx, h=1e-4, pairs=out["pairs"], **g)
    assert np.allclose(grad[idx], fd, rtol=2e-5, atol=1e-7 * np.abs(grad).max())
    # the TSC gradient differs from the CIC one (the scheme is used)
    wl_c = wl.scaled(assignment="cic")
    grad_c, _ = G.weight_gradient(cat, wl_c, w, pairs=out["pairs"], **g)
    assert np.max(np.abs(grad - grad_c)) > 1e-3 * np.abs(grad).max()
