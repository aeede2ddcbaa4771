"""Mass assignment on a periodic N^3 grid (oracle, FP64).

The paper assigns galaxies and pairs to a 512^3 grid with a triangular-shaped
cloud (Implementation section, "Mass assignment function"); this project uses
CIC by default and offers TSC as a scheme.
Node (a, b, c) sits at position (a, b, c) * L/N.  CIC: a point at
u = x*(N/L) (FP64) with i0 = floor(u), f = u - i0 gives weight (1 - f) to
node i0 and f to node i0 + 1 along each axis, indices taken mod N.  TSC: see
tsc_weights_1d.  Arrays are indexed [ix, iy, iz].
"""
from __future__ import annotations

import numpy as np


def cic_nodes(pos: np.ndarray, N: int, L: float):
    """Per point: base node (n,3) int64 and fractions (n,3) FP64."""
    u = np.asarray(pos, np.float64) * (N / L)
    i0 = np.floor(u)
    f = u - i0
    return np.mod(i0.astype(np.int64), N), f


def cic_assign(pos: np.ndarray, weights, N: int, L: float) -> np.ndarray:
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    wt = np.ones(pos.shape[0]) if weights is None else np.asarray(weights, np.float64)
    i0, f = cic_nodes(pos, N, L)
    rho = np.zeros((N, N, N))
    for ox in (0, 1):
        wx = f[:, 0] if ox else 1.0 - f[:, 0]
        ix = (i0[:, 0] + ox) % N
        for oy in (0, 1):
            wy = f[:, 1] if oy else 1.0 - f[:, 1]
            iy = (i0[:, 1] + oy) % N
            for oz in (0, 1):
                wz = f[:, 2] if oz else 1.0 - f[:, 2]
                iz = (i0[:, 2] + oz) % N
                np.add.at(rho, (ix, iy, iz), wt * wx * wy * wz)
    return rho


def cic_gather(field: np.ndarray, pos: np.ndarray, N: int, L: float) -> np.ndarray:
    """Adjoint of cic_assign with unit weights: sum_nodes K(node - x) field[node]."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    i0, f = cic_nodes(pos, N, L)
    out = np.zeros(pos.shape[0])
    for ox in (0, 1):
        wx = f[:, 0] if ox else 1.0 - f[:, 0]
        ix = (i0[:, 0] + ox) % N
        for oy in (0, 1):
            wy = f[:, 1] if oy else 1.0 - f[:, 1]
            iy = (i0[:, 1] + oy) % N
            for oz in (0, 1):
                wz = f[:, 2] if oz else 1.0 - f[:, 2]
                iz = (i0[:, 2] + oz) % N
                out += field[ix, iy, iz] * wx * wy * wz
    return out


def overdensity(rho: np.ndarray, wsum: float) -> np.ndarray:
    """delta = rho / rhobar - 1 with rhobar = (sum of weights) / N^3."""
    rhobar = wsum / rho.size
    return rho / rhobar - 1.0


def tsc_weights_1d(u: np.ndarray):
    """Triangular-shaped-cloud weights along one axis (the paper's mass
    assignment, Implementation section, "Mass assignment function"): the
    point at u (grid units) spreads over the nearest node c = round(u) and
    its two neighbours with the quadratic B-spline W(s) = 3/4 - s^2 for
    |s| <= 1/2 and (3/2 - |s|)^2 / 2 for 1/2 <= |s| <= 3/2, s = node - u.
    Ties (u exactly half-way) go to the lower node, where both choices give
    the same weights.  Returns the lowest node c - 1 (int64) and the three
    weights (n, 3)."""
    u = np.asarray(u, np.float64)
    i0 = np.floor(u)
    f = u - i0
    c = np.where(f <= 0.5, i0, i0 + 1.0)
    d = u - c  # in [-1/2, 1/2]
    w = np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], axis=-1)
    return (c - 1).astype(np.int64), w


def tsc_assign(pos: np.ndarray, weights, N: int, L: float) -> np.ndarray:
    """TSC density on the periodic N^3 grid (node (a, b, c) at (a, b, c) L/N)."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    wt = np.ones(pos.shape[0]) if weights is None else np.asarray(weights, np.float64)
    u = pos * (N / L)
    lo, ws = zip(*(tsc_weights_1d(u[:, k]) for k in range(3)))
    rho = np.zeros((N, N, N))
    for ox in range(3):
        for oy in range(3):
            for oz in range(3):
                np.add.at(rho, ((lo[0] + ox) % N, (lo[1] + oy) % N, (lo[2] + oz) % N),
                          wt * ws[0][:, ox] * ws[1][:, oy] * ws[2][:, oz])
    return rho


def tsc_gather(field: np.ndarray, pos: np.ndarray, N: int, L: float) -> np.ndarray:
    """Adjoint of tsc_assign with unit weights: the TSC interpolation
    sum_nodes W(node - u) field[node] at every point."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    u = pos * (N / L)
    lo, ws = zip(*(tsc_weights_1d(u[:, k]) for k in range(3)))
    out = np.zeros(pos.shape[0])
    for ox in range(3):
        for oy in range(3):
            for oz in range(3):
                out += (field[(lo[0] + ox) % N, (lo[1] + oy) % N, (lo[2] + oz) % N]
                        * ws[0][:, ox] * ws[1][:, oy] * ws[2][:, oz])
    return out


def assign(pos, weights, N, L, scheme="cic"):
    """Mass assignment by scheme "cic" or "tsc"."""
    if scheme == "cic":
        return cic_assign(pos, weights, N, L)
    if scheme == "tsc":
        return tsc_assign(pos, weights, N, L)
    raise ValueError(scheme)


def gather(field, pos, N, L, scheme="cic"):
    """Interpolation at the points, the adjoint of `assign` by scheme."""
    if scheme == "cic":
        return cic_gather(field, pos, N, L)
    if scheme == "tsc":
        return tsc_gather(field, pos, N, L)
    raise ValueError(scheme)
