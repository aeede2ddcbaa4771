"""Gradient pins of the oracle: adjoint dot products, finite differences,
direct-sum vs FFT adjoint, scale invariance and the HOD weight Jacobian."""
import numpy as np
import pytest

from oracle import grad as G
from oracle.cic import cic_assign, cic_gather
from synth import get_config
from synth.configs import HOD_FIDUCIAL, Workload, linbins, logbins


def tiny(N=16, L=40.0, out=None):
    return Workload(name="t", L=L, N=N, precision="fp64", pair_mode="s_mu",
                    p1_edges=linbins(0.5, 6.0, 3), p2_edges=np.array([0.0, 0.5, 1.0]),
                    out_mode="shell", o1_edges=out if out is not None else linbins(5.0, 17.0, 3),
                    o2_edges=None, catalog_kw={})


def clustered(n=400, L=40.0, seed=0):
    rng = np.random.default_rng(seed)
    c = rng.random((n // 4, 3)) * L
    s = np.repeat(c, 3, axis=0) + rng.normal(0, 1.5, (3 * (n // 4), 3))
    pos = np.mod(np.concatenate([c, s]), L)
    from synth.catalog import Catalog
    k = np.zeros(pos.shape[0], np.int8)
    return Catalog(L, pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.zeros(pos.shape[0]), k)


def upstream(F, R, seed=3):
    rng = np.random.default_rng(seed)
    return dict(g_b=rng.normal(size=(F, R)), g_q=rng.normal(size=(F, R)),
                g_xipg=rng.normal(size=(F, R)), g_xigg=rng.normal(size=R),
                g_xidp=rng.normal(size=F))


def test_p13_cic_scatter_gather_adjoint():
    rng = np.random.default_rng(0)
    N, L = 12, 30.0
    pos = rng.random((200, 3)) * L
    v = rng.normal(size=200)
    Fld = rng.normal(size=(N, N, N))
    lhs = np.sum(cic_assign(pos, v, N, L) * Fld)
    rhs = np.sum(v * cic_gather(Fld, pos, N, L))
    assert np.isclose(lhs, rhs, rtol=1e-13)


def test_p13_correlation_adjoints():
    rng = np.random.default_rng(1)
    N = 10
    k = rng.normal(size=(N, N, N)); d = rng.normal(size=(N, N, N)); y = rng.normal(size=(N, N, N))
    # <corr(k, d), y> = <d, conv(k, y)>   (the map d -> sum_r k(r) d(x+r) and its transpose)
    assert np.isclose(np.sum(G._corr_sum(k, d) * y), np.sum(d * G._conv_sum(k, y)), rtol=1e-12)
    assert np.allclose(G._corr_sum(k, d), G._corr_sum_direct(k, d), atol=1e-11)
    assert np.allclose(G._conv_sum(k, d), G._conv_sum_direct(k, d), atol=1e-11)


def test_p14_adjoint_matches_finite_differences():
    wl = tiny()
    cat = clustered()
    rng = np.random.default_rng(8)
    w = rng.uniform(0.5, 1.5, cat.n)
    g = upstream(wl.n_fields, wl.n_out)
    grad, out = G.weight_gradient(cat, wl, w, **g)
    assert np.all(np.isfinite(out["xi_pg"]))
    idx = rng.choice(cat.n, 12, replace=False)
    fd = G.fd_weight_gradient(cat, wl, w, idx, h=1e-4, pairs=out["pairs"], **g)
    assert np.allclose(grad[idx], fd, rtol=2e-5, atol=1e-7 * np.abs(grad).max())


def test_p14_direct_sum_adjoint_equals_fft_adjoint():
    wl = tiny(N=10, L=25.0, out=linbins(4.0, 10.0, 2))
    cat = clustered(n=160, L=25.0, seed=2)
    w = np.random.default_rng(2).uniform(0.5, 1.5, cat.n)
    g = upstream(wl.n_fields, wl.n_out, seed=4)
    a, _ = G.weight_gradient(cat, wl, w, method="fft", **g)
    b, _ = G.weight_gradient(cat, wl, w, method="direct", **g)
    assert np.allclose(a, b, rtol=1e-9, atol=1e-12 * np.abs(a).max())


def test_p12_scale_invariance():
    wl = tiny()
    cat = clustered(seed=5)
    w = np.random.default_rng(5).uniform(0.5, 1.5, cat.n)
    g = upstream(wl.n_fields, wl.n_out, seed=6)
    grad, _ = G.weight_gradient(cat, wl, w, **g)
    assert abs(np.dot(w, grad)) <= 1e-9 * np.sum(np.abs(w * grad))


def test_hod_jacobian_matches_fd():
    rng = np.random.default_rng(0)
    M = 10 ** rng.uniform(12.8, 15.0, 300)
    kind = rng.integers(1, 3, 300).astype(np.int8)
    th = np.array([HOD_FIDUCIAL[k] for k in ("logMcut", "logM1", "sigma", "alpha")])
    J = G.hod_weight_jacobian(M, kind, th)
    for k in range(4):
        h = 1e-6
        tp = th.copy(); tp[k] += h
        tm = th.copy(); tm[k] -= h
        fd = (G.hod_weights(M, kind, tp) - G.hod_weights(M, kind, tm)) / (2 * h)
        assert np.allclose(J[:, k], fd, rtol=1e-5, atol=1e-9)
    w = G.hod_weights(M, kind, th)
    # central occupation is 1/2 at M = Mcut; satellites vanish below M0 = Mcut
    assert np.isclose(G.hod_weights(np.array([10 ** 13.35]), np.array([1]), th)[0], 0.5)
    assert G.hod_weights(np.array([10 ** 13.3]), np.array([2]), th)[0] == 0.0
    assert np.all(w >= 0)
