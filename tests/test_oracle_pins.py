"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute force
or a library routine on a special case, a closed form, an invariant, or an
identity the paper states.  No GPU, no product code.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import cKDTree

from oracle import bins as B
from oracle import finalize as FZ
from oracle.cic import cic_assign, cic_gather, overdensity
from oracle.corr import direct_corr, fft_corr
from oracle.pairs import bruteforce_pairs, celllist_pairs, classify, min_image
from oracle.pipeline import forward
from synth import get_config
from synth.configs import Workload, linbins, logbins


def small_workload(L=100.0, N=32, p1=None, p2=None, o1=None, o2=None, pair_mode="s_mu",
                   out_mode="shell", dmax=0.0, qeff="notsq"):
    return Workload(name="t", L=L, N=N, precision="fp64", pair_mode=pair_mode,
                    p1_edges=np.asarray(p1 if p1 is not None else linbins(0.5, 10.0, 5)),
                    p2_edges=np.asarray(p2 if p2 is not None else [0.0, 1.0]),
                    out_mode=out_mode,
                    o1_edges=np.asarray(o1 if o1 is not None else logbins(10.0, 40.0, 6)),
                    o2_edges=None if o2 is None else np.asarray(o2),
                    catalog_kw={}, pair_dmax=dmax, qeff_mode=qeff)


# ---------------------------------------------------------------- P1 pairs
def test_p1_bruteforce_equals_celllist_cfg0():
    wl = get_config("cfg0")
    c = wl.catalog()
    a = celllist_pairs(c.x, c.y, c.z, None, c.L, wl.pair_mode, wl.p1_edges, wl.p2_edges)
    b = bruteforce_pairs(c.x, c.y, c.z, None, c.L, wl.pair_mode, wl.p1_edges, wl.p2_edges,
                         chunk=256)
    assert np.array_equal(a["i"], b["i"]) and np.array_equal(a["j"], b["j"])
    assert np.array_equal(a["key"], b["key"])
    assert np.array_equal(a["counts"], b["counts"])
    assert a["counts"].sum() > 10000


def test_p1_counts_match_periodic_kdtree():
    """Per-s-bin pair counts from scipy's periodic kd-tree (cumulative counts)."""
    rng = np.random.default_rng(5)
    L = 60.0
    pos = rng.random((3000, 3)) * L
    pos[:200] = pos[200:400] + rng.normal(0, 1.0, (200, 3))  # clustered copies
    pos = np.mod(pos, L)
    edges = np.array([0.7, 1.5, 3.0, 5.0, 9.0])
    res = celllist_pairs(pos[:, 0], pos[:, 1], pos[:, 2], None, L, "s_mu", edges, [0.0, 1.0])
    tree = cKDTree(pos, boxsize=L)
    cum = np.array([len(tree.query_pairs(r=e * (1 - 1e-12))) for e in edges])
    assert np.array_equal(res["counts"], np.diff(cum))


def test_p1_mu_bins_match_kdtree_on_projected_sets():
    """|mu| split: pairs with |d_z| >= mu s counted by kd-tree on anisotropic rescaling
    is awkward, so check the mu-bin counts sum to the s-bin counts and agree
    with a pure-Python per-pair evaluation of acos-free definitions."""
    rng = np.random.default_rng(7)
    L = 40.0
    pos = rng.random((400, 3)) * L
    s_e = np.array([1.0, 4.0, 9.0])
    mu_e = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
    res = bruteforce_pairs(pos[:, 0], pos[:, 1], pos[:, 2], None, L, "s_mu", s_e, mu_e)
    exp = np.zeros(8, int)
    for i in range(400):
        for j in range(i + 1, 400):
            d = [pos[j, a] - pos[i, a] for a in range(3)]
            d = [v - L if v >= L / 2 else (v + L if v < -L / 2 else v) for v in d]
            s = math.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
            if not (1.0 <= s < 9.0):
                continue
            sb = 0 if s < 4.0 else 1
            mu = abs(d[2]) / s
            mb = min(int(mu / 0.25), 3)
            exp[sb * 4 + mb] += 1
    assert np.array_equal(res["counts"], exp)


def test_p1_edge_cases():
    L = 30.0  # 3 cells of 10 for s_max = 10
    e = np.array([1.0, 5.0, 10.0])
    mu = np.array([0.0, 0.5, 1.0])
    # (a) separation exactly on an edge goes to the upper bin: d = (3, 4, 0) -> s = 5
    # (b) mu = 1 (pair along z) goes to the last mu bin
    # (c) pair across the periodic boundary: x = 29.5 and 0.5 -> d = +1
    # (d) s = 10 exactly is excluded (top edge open)
    x = np.array([1.0, 4.0, 10.0, 10.0, 29.5, 0.5, 20.0, 20.0])
    y = np.array([1.0, 5.0, 10.0, 10.0, 15.0, 15.0, 25.0, 25.0])
    z = np.array([1.0, 1.0, 10.0, 12.0, 5.0, 5.0, 1.0, 11.0])
    res = bruteforce_pairs(x, y, z, None, L, "s_mu", e, mu)
    got = {(int(i), int(j)): int(k) for i, j, k in zip(res["i"], res["j"], res["key"])}
    assert got[(0, 1)] == 1 * 2 + 0          # s = 5 -> bin 1, mu = 0 -> bin 0
    assert got[(2, 3)] == 0 * 2 + 1          # s = 2 along z -> mu = 1 -> last bin
    assert got[(4, 5)] == 0 * 2 + 0          # across the boundary, s = 1
    assert (6, 7) not in got                 # s = 10 excluded
    mid = {(int(i), int(j)): m for i, j, m in zip(res["i"], res["j"], res["mid"])}
    assert mid[(4, 5)][0] == 0.0             # midpoint of 29.5 and 30.5 wraps to 0
    cl = celllist_pairs(x, y, z, None, L, "s_mu", e, mu)
    assert np.array_equal(cl["key"], res["key"])


def test_p1_rp_pi_sphere_cut():
    L = 100.0
    x = np.array([10.0, 13.0, 50.0, 50.0, 70.0, 70.0])
    y = np.array([10.0, 14.0, 50.0, 50.0, 70.0, 74.0])
    z = np.array([10.0, 10.0, 50.0, 55.0, 70.0, 99.0])
    e_rp = linbins(0.0, 30.0, 6)
    e_pi = linbins(0.0, 30.0, 3)
    res = bruteforce_pairs(x, y, z, None, L, "rp_pi", e_rp, e_pi, dmax=30.0)
    got = {(int(i), int(j)): int(k) for i, j, k in zip(res["i"], res["j"], res["key"])}
    assert got[(0, 1)] == 1 * 3 + 0     # r_p = 5 (on edge -> bin 1), pi = 0
    assert got[(2, 3)] == 0 * 3 + 0     # r_p = 0, pi = 5
    # pair (4,5): r_p = 4, pi = 29 -> |d| = 29.27 < 30 -> kept, pi bin 2
    assert got[(4, 5)] == 0 * 3 + 2
    z2 = z.copy(); z2[5] = 99.9  # pi = 29.9, |d| = 30.17 > 30 -> dropped
    res2 = bruteforce_pairs(x, y, z2, None, L, "rp_pi", e_rp, e_pi, dmax=30.0)
    assert not any((int(i), int(j)) == (4, 5) for i, j in zip(res2["i"], res2["j"]))


def test_min_image_and_midpoint_wrap():
    L = 10.0
    d = min_image(np.array([5.0, -5.0, 4.999, -5.001, 9.0]), L)
    assert np.array_equal(d, [-5.0, -5.0, 4.999, 10.0 - 5.001, -1.0])


# ---------------------------------------------------------------- P2 lattice counts
@pytest.mark.parametrize("mode", ["shell", "r_mu", "rp_pi"])
def test_p2_lattice_counts_bruteforce(mode):
    L, N = 100.0, 32
    o1 = logbins(6.0, 40.0, 7) if mode != "rp_pi" else linbins(0.0, 40.0, 5)
    o2 = None if mode == "shell" else (linbins(0.0, 1.0, 4) if mode == "r_mu" else linbins(0.0, 30.0, 3))
    table = B.lattice_table(mode, o1, o2, L, N)
    assert np.array_equal(table[2], B.bin_counts_bruteforce(mode, o1, o2, L, N))


def test_p2_shell_counts_closed_form():
    """n_b from an independent loop: for each (i', j') count k' with
    t_lo <= i'^2 + j'^2 + k'^2 < t_hi in closed form."""
    L, N = 250.0, 128
    edges = logbins(10.0, 60.0, 15)
    table = B.lattice_table("shell", edges, None, L, N)
    delta = L / N
    t = (edges / delta) ** 2
    W = int(edges[-1] / delta) + 1

    def count_le(T, base):  # number of integers k with base + k^2 < T
        if T - base <= 0:
            return 0
        r = math.isqrt(max(int(math.ceil(T - base)) - 1, 0))
        while base + r * r >= T:
            r -= 1
        while base + (r + 1) ** 2 < T:
            r += 1
        return 2 * r + 1 if r >= 0 else 0

    exp = np.zeros(edges.size - 1, np.int64)
    for i in range(-W, W + 1):
        for j in range(-W, W + 1):
            base = i * i + j * j
            cum = [count_le(tb, base) for tb in t]
            exp += np.diff(cum)
    assert np.array_equal(table[2], exp)


# P2 for the two-dimensional output bins: closed-form lattice counts, written
# without the oracle's classifier.  The grid spacing is 1 (L = N) and every
# edge is chosen so that lattice vectors lie exactly on it, so a flipped
# comparison (>= against >, < against <=) on either axis changes a count.
def _r2(n):
    """Number of integer (a, b) with a^2 + b^2 = n (sum-of-two-squares count)."""
    if n < 0:
        return 0
    c = 0
    for a in range(-math.isqrt(n), math.isqrt(n) + 1):
        b2 = n - a * a
        b = math.isqrt(b2)
        if b * b == b2:
            c += 1 if b == 0 else 2
    return c


def test_p2_rp_pi_counts_closed_form_on_edges():
    """(r_p, |pi|) bins: the count of bin (b, k) is the number of (i', j') in
    the annulus e_b <= r_p < e_{b+1} (a sum of r2(n) over n in [e_b^2,
    e_{b+1}^2)) times the number of k' in the slab p_k <= |k'| < p_{k+1}
    (2 (p_{k+1} - p_k) integers, one fewer when p_k = 0).  Integer edges put
    vectors such as (3, 4, k') and (0, 5, k') exactly on r_p = 5 and k' = +-2
    exactly on |pi| = 2."""
    L = N = 64
    rp = np.array([0.0, 3.0, 5.0, 8.0, 13.0])
    pi = np.array([0.0, 2.0, 4.0, 7.0])
    got = B.lattice_table("rp_pi", rp, pi, float(L), N)[2]
    ann = [sum(_r2(n) for n in range(int(rp[b]) ** 2, int(rp[b + 1]) ** 2)) for b in range(rp.size - 1)]
    slab = [2 * int(pi[k + 1] - pi[k]) - (1 if pi[k] == 0 else 0) for k in range(pi.size - 1)]
    exp = np.array([a * s for a in ann for s in slab], np.int64)
    assert np.array_equal(got, exp), (got, exp)
    # the edges are hit: vectors with r_p exactly 5 and 8, |k'| exactly 2, 4, 7
    assert _r2(25) > 0 and _r2(64) > 0 and _r2(169) > 0


def test_p2_r_mu_counts_closed_form_on_edges():
    """(r, |mu|) bins: every lattice vector with i'^2 + j'^2 + k'^2 = m and
    k'^2 = K has the same bin, and there are r2(m - K) (times 2 for the sign
    of k' when K > 0) of them.  The shell is decided on m against the
    integer squares of the r edges; |mu| on K >= mu_e^2 m, the squares taken
    in FP64 as the bins are defined (ties go to the upper bin, mu = 1 to the
    last).  Here the r edges are integers and the |mu| edges 1/3, 0.6 and
    6/7 are ones whose FP64 squares make K = mu_e^2 m exact for vectors such
    as (2, 2, 1), (0, 4, 3) and (2, 3, 6); those ties are checked to be
    exact in rational arithmetic too, so this count does not rest on the
    rounding of the products."""
    from fractions import Fraction
    L = N = 64
    r = np.array([2.0, 3.0, 5.0, 7.0, 9.0, 10.0, 14.0])
    mu = np.array([0.0, 1.0 / 3.0, 0.6, 6.0 / 7.0, 1.0])
    got = B.lattice_table("r_mu", r, mu, float(L), N)[2]
    n2 = mu.size - 1
    exp = np.zeros((r.size - 1) * n2, np.int64)
    ties = 0
    W = int(r[-1])
    for m in range(W * W + 1):
        sb = [b for b in range(r.size - 1) if int(r[b]) ** 2 <= m < int(r[b + 1]) ** 2]
        if not sb:
            continue
        for k in range(0, math.isqrt(m) + 1):
            K = k * k
            n = _r2(m - K) * (2 if k > 0 else 1)
            if n == 0:
                continue
            # largest e with K >= mu_e^2 m (FP64 squares); the top edge is closed
            e = max(i for i in range(n2 + 1) if K >= (mu[i] * mu[i]) * m)
            for i in range(n2 + 1):
                tie = K == (mu[i] * mu[i]) * m
                ties += int(tie and 0 < i < n2)
                exact = Fraction(K) >= Fraction(float(mu[i])) ** 2 * m
                assert exact == (K >= (mu[i] * mu[i]) * m), (m, K, i)
            exp[sb[0] * n2 + min(e, n2 - 1)] += n
    assert ties >= 3
    assert np.array_equal(got, exp), (got, exp)


# ---------------------------------------------------------------- P3 node-placed special case
def test_p3_node_placed_equals_integer_histogram():
    rng = np.random.default_rng(11)
    L, N = 64.0, 32
    delta = L / N
    g_nodes = rng.integers(0, N, size=(700, 3))
    g_nodes[:100] = (g_nodes[100:200] + rng.integers(-2, 3, size=(100, 3))) % N
    p_nodes = rng.integers(0, N, size=(90, 3))
    gpos = g_nodes * delta
    ppos = p_nodes * delta
    rho_g = cic_assign(gpos, None, N, L)
    rho_p = cic_assign(ppos, None, N, L)
    # node placement -> CIC reduces to nearest grid point with unit mass
    assert np.allclose(rho_g.sum(), 700) and rho_g.max() >= 1 and np.all(np.mod(rho_g, 1) == 0)
    dg = overdensity(rho_g, 700.0)
    dp = overdensity(rho_p, 90.0)
    C = fft_corr(dp, dg)
    o1 = linbins(4.0, 30.0, 5)
    table = B.lattice_table("shell", o1, None, L, N)
    xi = B.bin_average(C, table, 5)
    # integer histogram of displacements node_g - node_p over all (pair, galaxy)
    dd = np.zeros((N, N, N), np.int64)
    for p in p_nodes:
        r = (g_nodes - p) % N
        np.add.at(dd, (r[:, 0], r[:, 1], r[:, 2]), 1)
    idx, b, n_b = table
    DD = np.bincount(b, weights=dd[idx], minlength=5)
    exp = N ** 3 * DD / (90 * 700 * n_b) - 1.0
    assert np.allclose(xi, exp, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- P4 FFT vs direct grid sum
@pytest.mark.parametrize("N", [8, 12])
def test_p4_fft_equals_direct_sum(N):
    rng = np.random.default_rng(N)
    a = rng.normal(size=(N, N, N))
    b = rng.normal(size=(N, N, N)) + 0.3 * np.roll(a, (1, 0, 2), axis=(0, 1, 2))
    assert np.allclose(fft_corr(a, b), direct_corr(a, b), rtol=0, atol=1e-12)


def test_p4_direct_sum_sign_convention():
    """C(r) is the galaxy field displaced by +r from the pair field."""
    N = 8
    a = np.zeros((N, N, N)); b = np.zeros((N, N, N))
    a[1, 2, 3] = 1.0
    b[3, 2, 2] = 1.0   # b at a + (2, 0, -1)
    C = fft_corr(a, b)
    k = np.unravel_index(np.argmax(C), C.shape)
    assert k == (2, 0, N - 1)
    assert np.isclose(C[k], 1.0 / N ** 3)


# ---------------------------------------------------------------- P5 paper identities
def test_p5_parseval_and_dual():
    rng = np.random.default_rng(3)
    L, N = 80.0, 32
    gpos = rng.random((1500, 3)) * L
    ppos = np.mod(gpos[:200] + rng.normal(0, 2.0, (200, 3)), L)
    pw = rng.random(200) + 0.5
    rho_g = cic_assign(gpos, None, N, L)
    rho_p = cic_assign(ppos, pw, N, L)
    dg = overdensity(rho_g, 1500.0)
    dp = overdensity(rho_p, pw.sum())
    o1 = linbins(6.0, 30.0, 4)
    table = B.lattice_table("shell", o1, None, L, N)
    idx, b, n_b = table
    C = fft_corr(dp, dg)
    xi = B.bin_average(C, table, 4)
    Fp = np.fft.fftn(dp); Fg = np.fft.fftn(dg)
    for bb in range(4):
        S = np.zeros((N, N, N))
        sel = b == bb
        S[tuple(a[sel] for a in idx)] = 1.0 / n_b[bb]
        St = np.fft.fftn(S)
        # (i) equation bpg_initial numerator in Fourier space: sum_k W(k) Re(conj(dg) dp)
        # with W(k) the transform of the bin indicator (real part: symmetric bins)
        lhs = np.sum(St.conj() * np.conj(Fp) * Fg).real / N ** 6
        assert np.isclose(lhs, xi[bb], rtol=1e-12, atol=1e-14)
        # (ii) the paper's evaluate-at-midpoints form (equation bpg_final numerator):
        # sum_x rho_p(x) (K_b * dg)(x) == sum_pairs w_p CIC-gather(K_b * dg)(m_p)
        Kd = np.real(np.fft.ifftn(np.conj(St) * Fg))  # sum_r S(r) dg(x + r)
        lhs2 = np.sum(rho_p * Kd)
        rhs2 = np.sum(pw * cic_gather(Kd, ppos, N, L))
        assert np.isclose(lhs2, rhs2, rtol=1e-12)
        nbar_p = pw.sum() / N ** 3
        assert np.isclose(lhs2 / nbar_p / N ** 3, xi[bb], rtol=1e-10, atol=1e-13)


# ---------------------------------------------------------------- P6 b == 1 when p := g
def test_p6_pair_field_equal_galaxy_field_gives_b_one():
    rng = np.random.default_rng(2)
    L, N = 100.0, 32
    pos = rng.random((2000, 3)) * L
    pos[:500] = np.mod(pos[500:1000] + rng.normal(0, 3, (500, 3)), L)
    rho = cic_assign(pos, None, N, L)
    d = overdensity(rho, 2000.0)
    table = B.lattice_table("shell", logbins(8.0, 40.0, 6), None, L, N)
    xi = B.bin_average(fft_corr(d, d), table, 6)
    fin = FZ.finalize(xi, xi[None, :], np.array([10.0]), 2000.0, L, np.array([1.0]))
    assert np.allclose(fin["b_pg"], 1.0, rtol=1e-13)


# ---------------------------------------------------------------- P7 linearity over mu
def test_p7_mu_split_linearity():
    wl_split = get_config("cfg0").scaled(p2_edges=linbins(0.0, 1.0, 4), N=64)
    wl_merged = get_config("cfg0").scaled(N=64)
    c = get_config("cfg0").catalog()
    a = forward(c, wl_split)
    m = forward(c, wl_merged)
    for sb in range(5):
        rows = slice(sb * 4, sb * 4 + 4)
        ws = a["wsum"][rows]
        comb = np.nansum(ws[:, None] * a["xi_pg"][rows], axis=0) / ws.sum()
        assert np.allclose(comb, m["xi_pg"][sb], rtol=1e-10, atol=1e-13)
        assert a["counts"][rows].sum() == m["counts"][sb]


# ---------------------------------------------------------------- P8 DC mode
def test_p8_galaxy_dc_vanishes():
    c = get_config("cfg0").catalog()
    rho = cic_assign(c.positions(), None, 64, c.L)
    d = overdensity(rho, float(c.n))
    F = np.fft.rfftn(d)
    assert abs(F[0, 0, 0]) <= 1e-12 * math.sqrt(d.size) * d.std() * math.sqrt(d.size)
    assert np.isclose(rho.sum(), c.n, rtol=1e-13)


# ---------------------------------------------------------------- P9 Poisson null
def test_p9_poisson_null():
    L, N = 100.0, 32
    o1 = linbins(12.0, 48.0, 6)  # beyond CIC self-count support
    table = B.lattice_table("shell", o1, None, L, N)
    xs = []
    for seed in range(20):
        rng = np.random.default_rng(100 + seed)
        pos = rng.random((4000, 3)) * L
        ppos = rng.random((600, 3)) * L
        dg = overdensity(cic_assign(pos, None, N, L), 4000.0)
        dp = overdensity(cic_assign(ppos, None, N, L), 600.0)
        xs.append(np.concatenate([B.bin_average(fft_corr(dg, dg), table, 6),
                                  B.bin_average(fft_corr(dp, dg), table, 6)]))
    xs = np.array(xs)
    mean = xs.mean(0)
    sem = xs.std(0, ddof=1) / math.sqrt(xs.shape[0])
    z = mean / sem
    assert np.all(np.abs(z) < 4.0)
    assert 0.2 < np.mean(z ** 2) < 3.0


# ---------------------------------------------------------------- P10 continuum consistency
def test_p10_grid_xi_matches_pair_counts():
    rng = np.random.default_rng(9)
    L, N = 120.0, 64
    nh = 300
    centres = rng.random((nh, 3)) * L
    sats = np.repeat(centres, 8, axis=0) + rng.normal(0, 6.0, (nh * 8, 3))
    pos = np.mod(np.concatenate([centres, sats, rng.random((3000, 3)) * L]), L)
    n = pos.shape[0]
    edges = linbins(10.0, 30.0, 4)
    table = B.lattice_table("shell", edges, None, L, N)
    d = overdensity(cic_assign(pos, None, N, L), float(n))
    xi_grid = B.bin_average(fft_corr(d, d), table, 4)
    tree = cKDTree(pos, boxsize=L)
    cum = np.array([tree.count_neighbors(tree, r) for r in edges], float)
    DD = np.diff(cum)  # ordered pairs
    RR = n * (n - 1) * (4 * math.pi / 3) * np.diff(edges ** 3) / L ** 3
    xi_pc = DD / RR - 1.0
    assert np.all(np.abs(xi_grid - xi_pc) < 0.1 * np.abs(xi_pc) + 0.01)


# ---------------------------------------------------------------- P11 finalize algebra
def test_p11_qeff_roundtrip_and_limits():
    rng = np.random.default_rng(1)
    q = rng.normal(1.0, 0.3, 50)
    x = rng.uniform(0.2, 50, 50)
    xw = rng.uniform(0.01, 0.4, 50)
    for mode in ("notsq", "squeezed"):
        b = FZ.b_from_q(q, x, xw, mode)
        assert np.allclose(FZ.q_eff(b, x, xw, mode), q, rtol=1e-13)
    b = rng.uniform(0.5, 3, 50)
    assert np.allclose(FZ.q_eff(b, x, 0.0, "notsq"), FZ.q_eff(b, x, xw, "squeezed"), rtol=1e-13)
    big = 1e9
    assert np.allclose(FZ.q_eff(b, big, xw, "notsq"), b / 2, rtol=1e-6)
    # paper's worked statement: b_pg = 2 (1 + Q xi)/(1 + xi) at Q = 1 gives b = 2
    assert np.allclose(FZ.b_from_q(1.0, x, 0.0, "squeezed"), 2.0)


def test_p11_xi_dp_unclustered_is_zero():
    """Uniform catalogue: Wsum ~ N^2 V / (2 L^3) -> xi_dp ~ 0 (statistical)."""
    rng = np.random.default_rng(4)
    L = 80.0
    pos = rng.random((6000, 3)) * L
    e = np.array([2.0, 5.0, 9.0])
    res = celllist_pairs(pos[:, 0], pos[:, 1], pos[:, 2], None, L, "s_mu", e, [0.0, 1.0])
    vol = FZ.field_volumes("s_mu", e, [0.0, 1.0])
    x = FZ.xi_dp(res["wsum"], 6000.0, L, vol)
    sig = 1.0 / np.sqrt(res["counts"])
    assert np.all(np.abs(x) < 4 * sig + 2e-3)


def test_volume_rp_pi_closed_form_vs_quadrature():
    D = 30.0
    for (a, b, c, d) in [(0.0, 5.0, 0.0, 10.0), (20.0, 25.0, 10.0, 30.0), (26.0, 30.0, 0.0, 30.0),
                         (10.0, 15.0, 20.0, 30.0), (0.0, 30.0, 0.0, 30.0)]:
        v = FZ.volume_rp_pi(a, b, c, d, D)
        f = lambda z, r: 2 * math.pi * r * (r * r + z * z < D * D)
        q = 2 * integrate.dblquad(f, a, b, lambda r: c, lambda r: d, epsabs=1e-10)[0]
        assert abs(v - q) < 1e-3 * max(q, 1.0)
    full = FZ.volume_rp_pi(0.0, 30.0, 0.0, 30.0, 30.0)
    assert math.isclose(full, 4 * math.pi / 3 * 27000.0, rel_tol=1e-12)
    assert math.isclose(FZ.volume_s_mu(1.0, 2.0, 0.0, 1.0), 4 * math.pi / 3 * 7.0, rel_tol=1e-15)


# ---------------------------------------------------------------- P15 symmetries
def test_p15_shift_and_swap_symmetry():
    wl = get_config("cfg0").scaled(N=64, out_mode="r_mu", o1_edges=logbins(10.0, 60.0, 6),
                                   o2_edges=linbins(0.0, 1.0, 3))
    c = get_config("cfg0").catalog()
    a = forward(c, wl)
    cs = c.subset(np.arange(c.n))
    delta = c.L / wl.N
    cs.x = np.mod(c.x + 5 * delta, c.L); cs.y = np.mod(c.y + 3 * delta, c.L)
    b = forward(cs, wl)
    sw = c.subset(np.arange(c.n)); sw.x, sw.y = c.y.copy(), c.x.copy()
    s = forward(sw, wl)
    assert np.allclose(a["xi_gg"], b["xi_gg"], rtol=1e-9, atol=1e-12)
    assert np.allclose(a["xi_pg"], b["xi_pg"], rtol=1e-8, atol=1e-11, equal_nan=True)
    assert np.allclose(a["xi_pg"], s["xi_pg"], rtol=1e-8, atol=1e-11, equal_nan=True)
    assert np.array_equal(a["counts"], s["counts"])


# ---------------------------------------------------------------- CIC by hand
def test_cic_weights_by_hand():
    L, N = 16.0, 8  # Delta = 2
    rho = cic_assign(np.array([[0.5, 2.0, 15.0]]), np.array([2.0]), N, L)
    # x: u = 0.25 -> nodes 0 (0.75), 1 (0.25); y: u = 1 exactly -> node 1 only;
    # z: u = 7.5 -> nodes 7 (0.5) and 0 (0.5, periodic)
    exp = {(0, 1, 7): 2 * 0.75 * 0.5, (0, 1, 0): 2 * 0.75 * 0.5,
           (1, 1, 7): 2 * 0.25 * 0.5, (1, 1, 0): 2 * 0.25 * 0.5}
    nz = {tuple(int(v) for v in k): rho[tuple(k)] for k in np.argwhere(rho != 0)}
    assert nz.keys() == exp.keys()
    for k, v in exp.items():
        assert nz[k] == v


# ---------------------------------------------------------------- PW: the paper's weighting function
from synth.configs import GSW_DP10, GSW_DP30, gsw_params  # noqa: E402


def test_pw_lattice_support_closed_form():
    """The weighted bin holds exactly the lattice vectors with r_perp >= r_cut
    and |r| <= r_max: for each (i', j') with i'^2 + j'^2 >= t_cut there are
    2 floor(sqrt(t_max - i'^2 - j'^2)) + 1 values of k' (t = (r / Delta)^2)."""
    L, N = 200.0, 64
    par = np.array([15.0, 10.0, 0.8, 5.0, 60.0])
    delta = L / N
    tc, tm = (par[3] / delta) ** 2, (par[4] / delta) ** 2
    w = int(np.floor(par[4] / delta))
    exp = 0
    for i in range(-w, w + 1):
        for j in range(-w, w + 1):
            xy = i * i + j * j
            if xy >= tc and xy <= tm:
                exp += 2 * math.isqrt(int(math.floor(tm - xy))) + 1
    table = B.lattice_table("gsw", par, None, L, N)
    assert table[2].tolist() == [exp]
    assert np.array_equal(table[2], B.bin_counts_bruteforce("gsw", par, None, L, N))


@pytest.mark.parametrize("row", [GSW_DP10, GSW_DP30])
def test_pw_small_jump_at_the_cavity(row):
    """The paper picks the parameters so that W's jump at r_cut is small
    (Section "weighting", figure of the weighting functions): on the r_perp
    axis W(r_cut) is under 1e-2 of W's maximum, for both rows of its table.
    A sigmoid of the wrong sign or centre fails this."""
    L, N = 1000.0, 8192  # fine lattice along the axis
    delta = L / N
    par = gsw_params(row)
    i = np.arange(0, int(par[4] / delta))
    W = B.gsw_weight(i, 0 * i, 0 * i, par, L, N)
    icut = int(np.ceil(par[3] / delta))
    assert W[icut] < 1e-2 * W.max()
    # and the peak sits outside the cavity, beyond r_s
    assert i[np.argmax(W)] * delta > par[1]


def test_pw_depends_on_r_perp_and_r_par_only():
    """W is a function of r_perp (x, y) and |r_par| (z): equal for (3, 4, k)
    and (5, 0, k) and (0, -5, k), even in k, and not symmetric between the
    transverse and the line-of-sight axes."""
    L, N = 100.0, 64
    par = np.array([12.0, 6.0, 0.7, 3.0, 40.0])
    for k in (0, 2, 7):
        a = B.gsw_weight(3, 4, k, par, L, N)
        assert np.isclose(a, B.gsw_weight(5, 0, k, par, L, N), rtol=1e-14)
        assert np.isclose(a, B.gsw_weight(0, -5, -k, par, L, N), rtol=1e-14)
    assert not np.isclose(B.gsw_weight(5, 0, 0, par, L, N), B.gsw_weight(0, 0, 5, par, L, N))


def test_pw_flat_limit_is_the_region_mean():
    """With a very wide Gaussian and a steep sigmoid centred inside the
    cavity, W is 1 on its support: the weighted bin is then the plain mean of
    C over {r_perp >= r_cut, |r| <= r_max}, taken here with a boolean mask."""
    rng = np.random.default_rng(4)
    L, N = 100.0, 32
    C = rng.normal(size=(N, N, N))
    par = np.array([1e9, 1.0, 1e3, 7.0, 30.0])
    table = B.lattice_table("gsw", par, None, L, N)
    bw = B.lattice_weights("gsw", par, None, L, N, table)
    got = B.bin_average(C, table, 1, bw)[0]
    a = np.arange(N)
    a = np.where(a < N // 2, a, a - N) * (L / N)
    X, Y, Z = np.meshgrid(a, a, a, indexing="ij")
    mask = (X * X + Y * Y >= 7.0 ** 2) & (X * X + Y * Y + Z * Z <= 30.0 ** 2)
    assert np.isclose(got, C[mask].mean(), rtol=1e-12)


def test_pw_pair_field_equal_galaxy_field_gives_b_one():
    """P6 with the weighting function: the weighted estimator is normalised
    so that a pair field equal to the galaxy field has b_pg = 1."""
    rng = np.random.default_rng(2)
    L, N = 100.0, 32
    pos = rng.random((2000, 3)) * L
    pos[:500] = np.mod(pos[500:1000] + rng.normal(0, 3, (500, 3)), L)
    d = overdensity(cic_assign(pos, None, N, L), 2000.0)
    par = np.array([12.0, 6.0, 0.7, 3.0, 40.0])
    table = B.lattice_table("gsw", par, None, L, N)
    bw = B.lattice_weights("gsw", par, None, L, N, table)
    xi = B.bin_average(fft_corr(d, d), table, 1, bw)
    fin = FZ.finalize(xi, xi[None, :], np.array([10.0]), 2000.0, L, np.array([1.0]), "const", 0.362)
    assert np.allclose(fin["b_pg"], 1.0, rtol=1e-13)


# ---------------------------------------------------------------- projected 2PCF (HOD-fit loss)
def test_projected_2pcf_thin_annulus_is_the_paper_column():
    """The projected correlation per r_p bin is xi(d_p) V / A (V the annulus-
    slab volume cut by the pair sphere, A the annulus area).  For a thin
    annulus V / A is the column length 2 d_par,max = 2 sqrt(d_max^2 - d_perp^2)
    of the paper's equation 2PCF_los_integrated_explicit."""
    dmax = 30.0
    for r in (1.0, 10.0, 25.0, 29.0):
        e = np.array([r, r + 1e-4])
        V = FZ.field_volumes("rp_pi", e, np.array([0.0, dmax]), dmax)[0]
        A = math.pi * (e[1] ** 2 - e[0] ** 2)
        assert np.isclose(V / A, 2.0 * math.sqrt(dmax * dmax - r * r), rtol=1e-4)
        # xi(d_p) = 1 in the annulus: w_p is the column length itself
        assert np.isclose(FZ.projected_2pcf([1.0], [V], e, 1)[0], V / A, rtol=1e-14)


def test_projected_2pcf_over_several_pi_bins_is_that_of_the_merged_bin():
    """Splitting the |pi| range into slabs does not change w_p: sum_b xi_b V_b
    = (2 sum_b Wsum_b L^3 / W_g^2) - sum_b V_b, the merged bin's xi V; slabs
    wholly outside the sphere (zero volume, xi = 0/0) add nothing."""
    dmax, L, wg = 20.0, 500.0, 1.0e4
    rp = np.array([0.0, 5.0, 12.0, 19.0])
    pi_split = np.array([0.0, 4.0, 11.0, 19.5, 25.0])
    Vs = FZ.field_volumes("rp_pi", rp, pi_split, dmax)
    Vm = FZ.field_volumes("rp_pi", rp, np.array([0.0, 25.0]), dmax)
    rng = np.random.default_rng(3)
    ws = rng.uniform(10.0, 100.0, Vs.size) * (Vs > 0)
    with np.errstate(invalid="ignore", divide="ignore"):
        xs = FZ.xi_dp(ws, wg, L, Vs)
    xm = FZ.xi_dp(ws.reshape(3, 4).sum(axis=1), wg, L, Vm)
    assert np.any(Vs == 0.0) and np.any(np.isnan(xs))
    assert np.allclose(FZ.projected_2pcf(xs, Vs, rp, 4), FZ.projected_2pcf(xm, Vm, rp, 1),
                       rtol=1e-12)


def test_projected_2pcf_of_a_poisson_catalogue_is_zero():
    """Uniform random galaxies: every r_p bin's projected correlation is
    consistent with zero (within 4 Poisson standard deviations)."""
    from oracle.pairs import pairs_for
    from synth.catalog import Catalog
    rng = np.random.default_rng(9)
    L, n, dmax = 100.0, 20000, 10.0
    pos = rng.random((n, 3)) * L
    cat = Catalog(L, pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.zeros(n), np.zeros(n, np.int8))
    rp = linbins(0.0, 8.0, 4)
    wl = Workload(name="t", L=L, N=64, precision="fp64", pair_mode="rp_pi", p1_edges=rp,
                  p2_edges=np.array([0.0, dmax]), pair_dmax=dmax, out_mode="shell",
                  o1_edges=logbins(5.0, 20.0, 2), o2_edges=None, catalog_kw={})
    pr = pairs_for(cat, wl)
    V = FZ.field_volumes("rp_pi", rp, np.array([0.0, dmax]), dmax)
    xdp = FZ.xi_dp(pr["wsum"], float(n), L, V)
    A = np.pi * (rp[1:] ** 2 - rp[:-1] ** 2)
    wp = FZ.projected_2pcf(xdp, V, rp, 1)
    expected = n * n / 2.0 * V / L ** 3
    sd = np.sqrt(expected) / expected * V / A
    assert np.all(np.abs(wp) < 4.0 * sd), (wp, sd)
