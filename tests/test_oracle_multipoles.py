"""Pins of the multipole oracle (pair axis against the pair-to-galaxy
direction): the harmonics against the addition theorem, the FFT route
against the direct definition, l = 0 against the shell estimator, a single
pair and a single galaxy against the closed form, and invariance under a
quarter turn of the box."""
import numpy as np
import pytest

from oracle import multipoles as OM
from oracle.pipeline import forward, galaxy_side
from synth.catalog import Catalog
from synth.configs import Workload, logbins


def small(L=60.0, N=32, seed=0, step=None):
    rng = np.random.default_rng(seed)
    c = rng.random((30, 3)) * L
    pos = np.mod(np.concatenate([c, np.repeat(c, 5, 0) + rng.normal(0, 1.5, (150, 3)),
                                 rng.random((300, 3)) * L]), L)
    if step is not None:  # positions on a grid of exactly representable values
        pos = np.mod(np.round(pos / step) * step, L)
    n = pos.shape[0]
    cat = Catalog(L, pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.zeros(n),
                  np.zeros(n, np.int8))
    wl = Workload(name="t", L=L, N=N, precision="fp64", pair_mode="s_mu",
                  p1_edges=logbins(0.5, 6.0, 2), p2_edges=np.array([0.0, 1.0]), out_mode="shell",
                  o1_edges=logbins(3.0, 12.0, 3), o2_edges=None, catalog_kw={})
    return cat, wl


def test_harmonics_satisfy_the_addition_theorem():
    rng = np.random.default_rng(1)
    a = OM.unit(rng.normal(size=(200, 3)))
    b = OM.unit(rng.normal(size=(200, 3)))
    for l in OM.EVEN_L:
        lhs = 4 * np.pi / (2 * l + 1) * np.sum(OM.real_sph_harm(l, a) * OM.real_sph_harm(l, b), axis=0)
        assert np.allclose(lhs, OM.legendre(l, np.sum(a * b, axis=1)), rtol=0, atol=1e-13), l
    # a zero vector contributes to l = 0 only
    z = np.zeros((1, 3))
    assert np.all(OM.real_sph_harm(2, z) == 0) and np.all(OM.real_sph_harm(4, z) == 0)


def test_legendre_closed_forms():
    x = np.linspace(-1, 1, 11)
    assert np.allclose(OM.legendre(2, x), np.polynomial.legendre.legval(x, [0, 0, 1]), atol=1e-15)
    assert np.allclose(OM.legendre(4, x), np.polynomial.legendre.legval(x, [0, 0, 0, 0, 1]), atol=1e-15)


def test_fft_route_matches_definition_and_monopole_is_shell_estimator():
    cat, wl = small()
    ref = forward(cat, wl)
    gal = galaxy_side(cat, wl)
    xf = OM.multipoles_fft(cat, wl, ref["pairs"], gal["dg"], ells=OM.EVEN_L, Fg=gal["Fg"])
    xd = OM.multipoles_direct(cat, wl, ref["pairs"], gal["dg"], ells=OM.EVEN_L)
    scale = np.nanmax(np.abs(xd))
    assert np.array_equal(np.isnan(xf), np.isnan(xd))
    assert np.nanmax(np.abs(xf - xd)) <= 1e-12 * scale
    assert np.nanmax(np.abs(xf[:, :, 0] - ref["xi_pg"])) <= 1e-12 * np.nanmax(np.abs(ref["xi_pg"]))
    # the clustered catalogue is anisotropic about its close pairs: the
    # quadrupole is not negligible (so the pins above exercise it)
    assert np.nanmax(np.abs(xf[:, :, 1])) > 0.05 * np.nanmax(np.abs(xf[:, :, 0]))


@pytest.mark.parametrize("axis", [(0, 0, 1), (1, 0, 0), (0, 1, 1)])
def test_single_pair_single_galaxy_closed_form(axis):
    """One pair whose midpoint sits on a node, delta_g a unit spike at the
    lattice vector r0 from it: xi_l(b(r0)) = (2l + 1) P_l(d^ . r0^) / n_b."""
    L, N = 32.0, 32
    wl = Workload(name="t", L=L, N=N, precision="fp64", pair_mode="s_mu",
                  p1_edges=np.array([0.5, 4.0]), p2_edges=np.array([0.0, 1.0]), out_mode="shell",
                  o1_edges=np.array([2.0, 4.0, 7.0]), o2_edges=None, catalog_kw={})
    mid = np.array([10.0, 11.0, 12.0])
    d = np.asarray(axis, np.float64)
    d = 1.5 * d / np.linalg.norm(d)
    pos = np.stack([mid - 0.5 * d, mid + 0.5 * d])
    cat = Catalog(L, pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.zeros(2), np.zeros(2, np.int8))
    pairs = dict(i=np.array([0]), j=np.array([1]), key=np.array([0]), mid=mid[None, :],
                 w=np.array([0.7]), counts=np.array([1]), wsum=np.array([0.7]))
    r0 = np.array([3, -1, 4])
    dg = np.zeros((N, N, N))
    node = np.rint(mid).astype(int)
    dg[tuple((node + r0) % N)] = 1.0
    xd = OM.multipoles_direct(cat, wl, pairs, dg, ells=OM.EVEN_L)
    xf = OM.multipoles_fft(cat, wl, pairs, dg, ells=OM.EVEN_L)
    counts = OM._shell_table(wl)[2]
    b = 1  # |r0| = sqrt(26) in [4, 7)
    mu = float(np.dot(d / np.linalg.norm(d), r0 / np.linalg.norm(r0)))
    for il, l in enumerate(OM.EVEN_L):
        exp = np.zeros(2)
        exp[b] = (2 * l + 1) * OM.legendre(l, mu) / counts[b]
        assert np.allclose(xd[0, :, il], exp, rtol=1e-12, atol=1e-15), l
        assert np.allclose(xf[0, :, il], exp, rtol=1e-12, atol=1e-14), l


def test_quarter_turn_invariance():
    """(x, y, z) -> (L - y, x, z) maps the lattice and the CIC weights onto
    themselves and turns every pair axis and lattice vector alike, so the
    multipoles do not change (positions on a representable grid make the
    turn exact)."""
    cat, wl = small(step=1.0 / 64)
    L = cat.L
    rot = Catalog(L, np.mod(L - cat.y, L), cat.x.copy(), cat.z.copy(), cat.halo_mass, cat.kind)
    out = []
    for c in (cat, rot):
        ref = forward(c, wl)
        gal = galaxy_side(c, wl)
        out.append(OM.multipoles_fft(c, wl, ref["pairs"], gal["dg"], ells=OM.EVEN_L, Fg=gal["Fg"]))
    assert np.array_equal(np.isnan(out[0]), np.isnan(out[1]))
    assert np.nanmax(np.abs(out[0] - out[1])) <= 1e-11 * np.nanmax(np.abs(out[0]))


def test_finite_differences_of_a_linear_functional_are_exact_in_g():
    """The oracle's finite-difference gradient of J = sum g xi_l is linear in
    g: doubling g doubles it, and g = 0 gives 0 (a check of the helper the
    GPU adjoint test uses)."""
    cat, wl = small()
    ref = forward(cat, wl)
    w = np.random.default_rng(3).uniform(0.5, 1.5, cat.n)
    g = np.random.default_rng(4).normal(size=(wl.n_fields, wl.n_out, 2))
    idx = [0, 5, 40]
    a = OM.fd_weight_gradient(cat, wl, w, idx, g, ref["pairs"])
    b = OM.fd_weight_gradient(cat, wl, w, idx, 2 * g, ref["pairs"])
    assert np.allclose(b, 2 * a, rtol=1e-9, atol=1e-12)
    assert np.all(OM.fd_weight_gradient(cat, wl, w, idx, 0 * g, ref["pairs"]) == 0)
