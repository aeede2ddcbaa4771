"""Seeded halo-model galaxy catalogues in a periodic box.

Stand-ins for the paper's HOD mock LRG catalogues built on N-body FoF halos
(Implementation section, "Mock LRG and LRG pair catalogue"), which are not
available here.  Every draw comes from one ``numpy.random.Generator`` (PCG64)
seeded by the caller, in a fixed order, so a (recipe, seed) pair always gives
the same arrays.  Lengths are in Mpc/h, masses in Msun/h, velocities in km/s.

Recipe pieces:
  * halo masses: log-uniform, or a power law dn/dM ~ M^-slope on [M_lo, M_hi]
    sampled by its inverse CDF;
  * halo centres: uniform, or a Soneira-Peebles hierarchy (clustered);
  * galaxies: one central at each halo centre, satellites on an isotropic NFW
    profile (concentration c, r_vir = 2 (M/1e15)^(1/3)), either Poisson(M/M_sat)
    per halo or a fixed number of weighted candidates per halo;
  * optional uniform field galaxies;
  * optional redshift-space shift along z by v/(aH) (the paper's RSD shift,
    Implementation section, equation RSD, with the aH factor for comoving
    coordinates).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

G_NEWTON = 4.30091e-9  # Mpc (km/s)^2 / Msun


@dataclass
class Catalog:
    """SoA galaxy catalogue. ``kind``: 0 field, 1 central, 2 satellite."""
    L: float
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    halo_mass: np.ndarray
    kind: np.ndarray
    w: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def positions(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    def subset(self, idx) -> "Catalog":
        return Catalog(self.L, self.x[idx].copy(), self.y[idx].copy(), self.z[idx].copy(),
                       self.halo_mass[idx].copy(), self.kind[idx].copy(),
                       None if self.w is None else self.w[idx].copy(), dict(self.meta))


def _nfw_mu(x):
    return np.log1p(x) - x / (1.0 + x)


def nfw_radius(u: np.ndarray, c: float) -> np.ndarray:
    """Radius in units of r_vir/c ... returned as fraction of r_vir.

    Solves mu(x) = u * mu(c) for x in [0, c] by bisection (mu is monotone),
    where mu(x) = ln(1+x) - x/(1+x) is the NFW enclosed-mass shape.
    """
    target = u * _nfw_mu(c)
    lo = np.zeros_like(target)
    hi = np.full_like(target, c)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        f = _nfw_mu(mid) - target
        hi = np.where(f > 0, mid, hi)
        lo = np.where(f > 0, lo, mid)
    return 0.5 * (lo + hi) / c


def _unit_vectors(rng, n):
    v = rng.normal(size=(n, 3))
    nrm = np.linalg.norm(v, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return v / nrm


def _points_in_ball(rng, n, radius):
    d = _unit_vectors(rng, n)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    return d * r[:, None]


def soneira_peebles(rng, n_points, L, R0=50.0, eta=4, lam=1.9, levels=4):
    """Clustered centres from a Soneira-Peebles hierarchy in a periodic box.

    Each cluster starts with a sphere of radius R0 at a uniform position; at
    each level every sphere spawns ``eta`` sub-sphere centres placed uniformly
    inside it, with radius divided by ``lam``.  After ``levels`` levels a
    cluster holds eta**levels points.  Enough clusters are drawn to cover
    ``n_points`` and a seeded random subset of that size is kept.
    """
    per = eta ** levels
    n_cl = int(math.ceil(n_points / per))
    centres = rng.random((n_cl, 3)) * L
    radius = R0
    pts = centres
    for _ in range(levels):
        parent = np.repeat(pts, eta, axis=0)
        pts = parent + _points_in_ball(rng, parent.shape[0], radius)
        radius = radius / lam
    pts = np.mod(pts, L)
    keep = rng.permutation(pts.shape[0])[:n_points]
    return pts[keep]


def _halo_masses(rng, n, dist, m_lo, m_hi, slope):
    u = rng.random(n)
    if dist == "loguniform":
        return 10.0 ** (np.log10(m_lo) + u * (np.log10(m_hi) - np.log10(m_lo)))
    if dist == "powerlaw":
        a = 1.0 - slope  # dn/dM ~ M^-slope  ->  CDF ~ M^(1-slope)
        lo, hi = m_lo ** a, m_hi ** a
        return (lo + u * (hi - lo)) ** (1.0 / a)
    raise ValueError(dist)


def make_catalog(*, L: float, n_halos: int, mass_dist: str = "loguniform",
                 m_lo: float = 1e13, m_hi: float = 1e15, slope: float = 1.9,
                 placement: str = "uniform", sp_R0: float = 50.0,
                 sat_mode: str = "poisson", m_sat: float = 10 ** 13.5,
                 n_candidates: int = 49, concentration: float = 5.0,
                 n_field: int = 0, rsd: bool = False, aH: Optional[float] = None,
                 sigma_bulk: float = 300.0, seed: int = 0) -> Catalog:
    rng = np.random.default_rng(seed)
    if placement == "uniform":
        centres = rng.random((n_halos, 3)) * L
    elif placement == "sp":
        centres = soneira_peebles(rng, n_halos, L, R0=sp_R0)
    else:
        raise ValueError(placement)
    mass = _halo_masses(rng, n_halos, mass_dist, m_lo, m_hi, slope)
    rvir = 2.0 * (mass / 1e15) ** (1.0 / 3.0)
    if sat_mode == "poisson":
        nsat = rng.poisson(mass / m_sat)
    elif sat_mode == "candidates":
        nsat = np.full(n_halos, n_candidates, dtype=np.int64)
    else:
        raise ValueError(sat_mode)
    host = np.repeat(np.arange(n_halos), nsat)
    u = rng.random(host.shape[0])
    rfrac = nfw_radius(u, concentration)
    dirs = _unit_vectors(rng, host.shape[0])
    sat_pos = centres[host] + dirs * (rfrac * rvir[host])[:, None]
    field_pos = rng.random((n_field, 3)) * L

    pos = np.concatenate([centres, sat_pos, field_pos], axis=0)
    hm = np.concatenate([mass, mass[host], np.zeros(n_field)])
    kind = np.concatenate([np.ones(n_halos, np.int8), np.full(host.shape[0], 2, np.int8),
                           np.zeros(n_field, np.int8)])
    meta = {"seed": seed, "n_halos": n_halos, "n_sat": int(host.shape[0]),
            "n_field": n_field, "halo_index": np.concatenate(
                [np.arange(n_halos), host, np.full(n_field, -1)])}
    if rsd:
        if aH is None:
            raise ValueError("rsd needs aH")
        v_bulk = rng.normal(0.0, sigma_bulk, n_halos)
        sig_sat = np.sqrt(G_NEWTON * mass[host] / (2.0 * rvir[host]))
        v_sat = v_bulk[host] + rng.normal(0.0, 1.0, host.shape[0]) * sig_sat
        v_field = rng.normal(0.0, sigma_bulk, n_field)
        vlos = np.concatenate([v_bulk, v_sat, v_field])
        pos[:, 2] = pos[:, 2] + vlos / aH
        meta["v_los"] = vlos
    pos = np.mod(pos, L)
    # np.mod can return exactly L for tiny negative inputs; fold those to 0.
    pos[pos >= L] = 0.0
    return Catalog(L, np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
                   np.ascontiguousarray(pos[:, 2]), hm, kind, None, meta)


def flat_lcdm_aH(z: float, omega_m: float = 0.31) -> float:
    """a(z) H(z) in h km/s/Mpc for flat LCDM: 100 E(z) / (1+z)."""
    E = math.sqrt(omega_m * (1 + z) ** 3 + (1 - omega_m))
    return 100.0 * E / (1.0 + z)
