"""Multipoles of the pair-galaxy correlation in the angle between the pair
axis and the pair-to-galaxy direction (oracle, FP64, test infrastructure).

The build's cross-correlation bins the pair orientation about the z line of
sight.  This module computes the other reading of the pair-orientation cosine:
mu' = d^ . r^, between the pair axis d (pair catalogue conventions, d = x_j -
x_i) and the pair-to-galaxy separation r.  It expands the dependence on mu' in
Legendre multipoles.  Over the lattice vectors r of shell b:

  xi_l(f, b) = (2l + 1) / (n_b Wsum_f) sum_{p in f} w_p sum_{r in b}
               P_l(d^_p . r^) sum_nodes K(node - m_p) delta_g(node + r),

with K the CIC weights of the pair midpoint m_p and delta_g the galaxy
overdensity.  For l = 0 this is the shell estimator xi_pg exactly.  The mean of
P_l over the directions of a shell is zero for l > 0, so an isotropic
delta_g gives xi_l = 0.  The (2l + 1) normalisation makes
xi(mu') = sum_l xi_l P_l(mu') for an anisotropy that is a polynomial in mu'.
Only even l is meaningful: the pair axis has no sign.  A pair with d = 0
contributes to l = 0 only.

Two routes:
  multipoles_direct  the definition above, looped over pairs and lattice
                     vectors (small inputs);
  multipoles_fft     the addition theorem
                     P_l(a . b) = 4 pi / (2l + 1) sum_m Y_lm(a) Y_lm(b)
                     (real spherical harmonics).  One CIC pair field per
                     (f, l, m) with weights w_p Y_lm(d^_p), its FFT
                     cross-correlation with delta_g, then the Y_lm(r^)
                     weighted shell sums.
The tests pin the second route against the first on small inputs.
"""
from __future__ import annotations

import numpy as np

from . import bins as _bins
from .cic import cic_assign, cic_nodes
from .corr import irfftn, rfftn
from .pairs import min_image

EVEN_L = (0, 2, 4)


def legendre(l: int, x):
    x = np.asarray(x, np.float64)
    if l == 0:
        return np.ones_like(x)
    if l == 2:
        return 0.5 * (3.0 * x * x - 1.0)
    if l == 4:
        x2 = x * x
        return (35.0 * x2 * x2 - 30.0 * x2 + 3.0) / 8.0
    raise ValueError(l)


def real_sph_harm(l: int, u: np.ndarray) -> np.ndarray:
    """Real spherical harmonics Y_lm(u), m = -l..l (rows), for unit vectors
    u (n, 3); the Cartesian polynomial forms.  A zero vector gives 0 for
    l > 0."""
    u = np.asarray(u, np.float64).reshape(-1, 3)
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    pi = np.pi
    if l == 0:
        return np.full((1, x.size), 0.5 / np.sqrt(pi))
    if l == 2:
        a = 0.5 * np.sqrt(15.0 / pi)
        return np.stack([a * x * y, a * y * z, 0.25 * np.sqrt(5.0 / pi) * (2 * z * z - x * x - y * y),
                         a * x * z, 0.5 * a * (x * x - y * y)])
    if l == 4:
        x2, y2, z2 = x * x, y * y, z * z
        r2 = x2 + y2 + z2  # 1 for unit vectors, 0 for the zero vector
        return np.stack([
            0.75 * np.sqrt(35.0 / pi) * x * y * (x2 - y2),
            0.75 * np.sqrt(35.0 / (2 * pi)) * (3 * x2 - y2) * y * z,
            0.75 * np.sqrt(5.0 / pi) * x * y * (7 * z2 - r2),
            0.75 * np.sqrt(5.0 / (2 * pi)) * y * z * (7 * z2 - 3 * r2),
            3.0 / 16.0 * np.sqrt(1.0 / pi) * (35 * z2 * z2 - 30 * z2 * r2 + 3 * r2 * r2),
            0.75 * np.sqrt(5.0 / (2 * pi)) * x * z * (7 * z2 - 3 * r2),
            3.0 / 8.0 * np.sqrt(5.0 / pi) * (x2 - y2) * (7 * z2 - r2),
            0.75 * np.sqrt(35.0 / (2 * pi)) * (x2 - 3 * y2) * x * z,
            3.0 / 16.0 * np.sqrt(35.0 / pi) * (x2 * (x2 - 3 * y2) - y2 * (3 * x2 - y2)),
        ])
    raise ValueError(l)


def unit(v: np.ndarray) -> np.ndarray:
    """v / |v| row-wise; zero rows stay zero."""
    v = np.asarray(v, np.float64).reshape(-1, 3)
    n = np.sqrt(np.sum(v * v, axis=1))
    out = np.zeros_like(v)
    nz = n > 0
    out[nz] = v[nz] / n[nz, None]
    return out


def pair_axes(cat, pairs) -> np.ndarray:
    """Unit pair axes d^ = (x_j - x_i) / |x_j - x_i|, minimum image."""
    pos = cat.positions()
    L = cat.L
    d = np.stack([min_image(pos[pairs["j"], k] - pos[pairs["i"], k], L) for k in range(3)], axis=1)
    return unit(d)


def _shell_table(wl):
    if wl.out_mode != "shell":
        raise ValueError("multipoles are taken over shell output bins")
    if float(wl.o1_edges[0]) <= 0.0:
        raise ValueError("the first shell edge must be > 0 (r^ is undefined at r = 0)")
    table = _bins.lattice_table("shell", wl.o1_edges, None, wl.L, wl.N)
    return table


def _offsets(table, N):
    idx = table[0]
    return np.stack([np.where(a < N // 2, a, a - N) for a in idx], axis=1).astype(np.float64)


def multipoles_direct(cat, wl, pairs, dg, ells=(0, 2), w=None):
    """The definition, looped over pairs: xi_l[f, b, il] (NaN rows for empty
    fields).  dg is the galaxy overdensity grid, pairs as from oracle.pairs
    (with w the pair weights)."""
    N = wl.N
    table = _shell_table(wl)
    idx, b, counts = table
    R = counts.size
    rhat = unit(_offsets(table, N))
    axes = pair_axes(cat, pairs)
    i0, fr = cic_nodes(pairs["mid"], N, wl.L)
    F = wl.n_fields
    S = np.zeros((F, R, len(ells)))
    ws = np.zeros(F)
    for p in range(pairs["key"].size):
        f = pairs["key"][p]
        wp = pairs["w"][p]
        ws[f] += wp
        # CIC-smeared delta_g at m_p + r for every table vector r
        g = np.zeros(b.size)
        for ox in (0, 1):
            wx = fr[p, 0] if ox else 1.0 - fr[p, 0]
            for oy in (0, 1):
                wy = fr[p, 1] if oy else 1.0 - fr[p, 1]
                for oz in (0, 1):
                    wz = fr[p, 2] if oz else 1.0 - fr[p, 2]
                    g += wx * wy * wz * dg[(i0[p, 0] + ox + idx[0]) % N, (i0[p, 1] + oy + idx[1]) % N,
                                           (i0[p, 2] + oz + idx[2]) % N]
        mu = rhat @ axes[p]
        for il, l in enumerate(ells):
            if l > 0 and not np.any(axes[p]):
                continue
            S[f, :, il] += wp * (2 * l + 1) * np.bincount(b, weights=legendre(l, mu) * g, minlength=R)
    with np.errstate(invalid="ignore", divide="ignore"):
        xi = S / (counts[None, :, None] * ws[:, None, None])
    xi[ws == 0] = np.nan
    return xi


def multipoles_fft(cat, wl, pairs, dg, ells=(0, 2), Fg=None):
    """The addition-theorem route: xi_l[f, b, il]."""
    N, L = wl.N, wl.L
    table = _shell_table(wl)
    idx, b, counts = table
    R = counts.size
    rhat = unit(_offsets(table, N))
    axes = pair_axes(cat, pairs)
    if Fg is None:
        Fg = rfftn(dg)
    F = wl.n_fields
    xi = np.full((F, R, len(ells)), np.nan)
    for f in range(F):
        sel = pairs["key"] == f
        ws = float(np.sum(pairs["w"][sel]))
        if ws == 0.0:
            continue
        for il, l in enumerate(ells):
            Yd = real_sph_harm(l, axes[sel])
            Yr = real_sph_harm(l, rhat)
            S = np.zeros(R)
            for m in range(2 * l + 1):
                rho = cic_assign(pairs["mid"][sel], pairs["w"][sel] * Yd[m], N, L)
                # C(r) = sum_x rho(x) delta_g(x + r)
                C = irfftn(np.conj(rfftn(rho)) * Fg, rho.shape)
                S += np.bincount(b, weights=Yr[m] * C[idx], minlength=R)
            xi[f, :, il] = 4.0 * np.pi * S / (counts * ws)
    return xi


def multipoles_for_weights(cat, wl, w, pairs, ells=(0, 2)):
    """xi_l for galaxy weights w (pair weights w_i w_j, galaxy overdensity
    with weights w), reusing an existing pair catalogue's (i, j, key, mid)."""
    from .pipeline import galaxy_side
    w = np.asarray(w, np.float64)
    p = dict(pairs)
    p["w"] = w[p["i"]] * w[p["j"]]
    gal = galaxy_side(cat, wl, w=w)
    return multipoles_fft(cat, wl, p, gal["dg"], ells=ells, Fg=gal["Fg"])


def fd_weight_gradient(cat, wl, w, idx, g, pairs, ells=(0, 2), h=1e-3):
    """Central differences of J(w) = sum g xi_l(w) (non-finite entries of
    xi_l or g count as 0) at the weight coordinates idx."""
    w = np.asarray(w, np.float64)
    g = np.where(np.isfinite(g), g, 0.0)

    def J(wv):
        xi = multipoles_for_weights(cat, wl, wv, pairs, ells)
        return float(np.sum(np.where(np.isfinite(xi), xi, 0.0) * g))

    out = np.zeros(len(idx))
    for k, i in enumerate(idx):
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        out[k] = (J(wp) - J(wm)) / (2 * h)
    return out
