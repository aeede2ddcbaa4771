"""Lattice-vector binning of a correlation grid (oracle, FP64).

Taking the weight W of the paper's equation bpg_initial to be the normalised
indicator of one separation bin turns the estimator into the bin average
xi[b] = n_b^-1 sum_{r in b} C(r), with n_b the number of lattice vectors in
the bin.  Lattice vector r = Delta * (i', j', k') with Delta = L/N and
i' = i for i < N/2, i - N otherwise.  Classification is done on integers
against FP64 thresholds q*q, q = e/Delta:
  shell   m = i'^2 + j'^2 + k'^2, bin b iff t_b <= m < t_{b+1};
  r_mu    shell bin on m, then |mu| = |k'|/sqrt(m) about the z line of sight:
          largest k with k'^2 >= (mu_k*mu_k)*m, top edge closed;
  rp_pi   r_p bin on i'^2 + j'^2, |pi| bin on k'^2 (both half-open).
The paper's own W (Section "weighting", equation weighting), out_mode "gsw",
is one weighted bin: xi = sum_r W(r) C(r) / sum_r W(r) over the lattice
vectors with r_perp >= r_cut (squares against the FP64 threshold, as above)
and |r| <= r_max; its parameters (sigma, r_s, s_0, r_cut, r_max) travel in
o1_edges.
"""
from __future__ import annotations

import numpy as np


def _thresholds(edges, L, N):
    delta = L / N
    q = np.asarray(edges, np.float64) / delta
    return q * q


def gsw_weight(ip, jp, kp, params, L, N):
    """The paper's Gaussian-sigmoid weighting function (Section "weighting",
    equation weighting) at lattice offsets, without its normalisation
    constant (it cancels in every ratio): a sigmoid in the distance r_perp
    across the line of sight (x, y), centred at r_s with slope s_0, times an
    isotropic Gaussian of width sigma in (r_perp, r_par), r_par along z.  The
    cavity r_perp < r_cut and the cut |r| > r_max are the classification's."""
    sigma, rs, s0 = float(params[0]), float(params[1]), float(params[2])
    delta = L / N
    ip = np.asarray(ip, np.float64); jp = np.asarray(jp, np.float64); kp = np.asarray(kp, np.float64)
    rperp = delta * np.sqrt(ip * ip + jp * jp)
    rpar = delta * np.abs(kp)
    sig = 1.0 / (1.0 + np.exp(-s0 * (rperp - rs)))
    return sig * np.exp(-0.5 * (rperp * rperp + rpar * rpar) / (sigma * sigma))


def window(out_mode, o1_edges, o2_edges, L, N):
    """Half-widths (wx, wy, wz) of the lattice cube that holds every bin."""
    delta = L / N
    if out_mode == "gsw":
        w = int(np.floor(o1_edges[4] / delta))
        return (w, w, w)
    if out_mode in ("shell", "r_mu"):
        w = int(np.floor(o1_edges[-1] / delta))
        return (w, w, w)
    wxy = int(np.floor(o1_edges[-1] / delta))
    wz = int(np.floor(o2_edges[-1] / delta))
    return (wxy, wxy, wz)


def classify_lattice(ip, jp, kp, out_mode, o1_edges, o2_edges, L, N):
    """Bin index (or -1) for integer lattice offsets."""
    ip = np.asarray(ip, np.int64); jp = np.asarray(jp, np.int64); kp = np.asarray(kp, np.int64)
    if out_mode == "gsw":
        tc, tm = _thresholds([o1_edges[3], o1_edges[4]], L, N)
        xy = (ip * ip + jp * jp).astype(np.float64)
        m = xy + (kp * kp).astype(np.float64)
        return np.where((xy >= tc) & (m <= tm), 0, -1)
    t1 = _thresholds(o1_edges, L, N)
    if out_mode == "shell" or out_mode == "r_mu":
        m = ip * ip + jp * jp + kp * kp
        mf = m.astype(np.float64)
        ok = (mf >= t1[0]) & (mf < t1[-1])
        b = np.searchsorted(t1, mf, side="right") - 1
        if out_mode == "shell":
            return np.where(ok, b, -1)
        mu = np.asarray(o2_edges, np.float64)
        m2 = mu * mu
        n2 = mu.size - 1
        kk2 = (kp * kp).astype(np.float64)
        k = np.zeros(m.shape, np.int64)
        for e in range(n2 + 1):
            k += (kk2 >= m2[e] * mf)
        ok &= (kk2 >= m2[0] * mf) & (kk2 <= m2[-1] * mf)
        k = np.minimum(k - 1, n2 - 1)
        return np.where(ok, b * n2 + k, -1)
    if out_mode == "rp_pi":
        t2 = _thresholds(o2_edges, L, N)
        n2 = len(o2_edges) - 1
        rp = (ip * ip + jp * jp).astype(np.float64)
        pz = (kp * kp).astype(np.float64)
        ok = (rp >= t1[0]) & (rp < t1[-1]) & (pz >= t2[0]) & (pz < t2[-1])
        b = np.searchsorted(t1, rp, side="right") - 1
        k = np.searchsorted(t2, pz, side="right") - 1
        return np.where(ok, b * n2 + k, -1)
    raise ValueError(out_mode)


def n_out(out_mode, o1_edges, o2_edges):
    if out_mode == "gsw":
        return 1
    n1 = len(o1_edges) - 1
    return n1 if out_mode == "shell" else n1 * (len(o2_edges) - 1)


def lattice_table(out_mode, o1_edges, o2_edges, L, N):
    """(grid indices tuple, bin ids, counts n_b) over the window cube."""
    wx, wy, wz = window(out_mode, o1_edges, o2_edges, L, N)
    if max(wx, wy, wz) >= N // 2:
        raise ValueError("output bins reach N/2 (need r_max < L/2)")
    I, J, K = np.meshgrid(np.arange(-wx, wx + 1), np.arange(-wy, wy + 1), np.arange(-wz, wz + 1),
                          indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    b = classify_lattice(I, J, K, out_mode, o1_edges, o2_edges, L, N)
    sel = b >= 0
    I, J, K, b = I[sel], J[sel], K[sel], b[sel]
    R = n_out(out_mode, o1_edges, o2_edges)
    counts = np.bincount(b, minlength=R).astype(np.int64)
    return (np.mod(I, N), np.mod(J, N), np.mod(K, N)), b, counts


def lattice_weights(out_mode, o1_edges, o2_edges, L, N, table):
    """Weight of every entry of `table` (1 for the indicator bins, W for
    "gsw") and the normalisation of every bin (their sums)."""
    idx, b, counts = table
    R = counts.size
    if out_mode != "gsw":
        return np.ones(b.size), counts.astype(np.float64)
    # the table holds grid indices; back to signed offsets
    off = [np.where(a < N // 2, a, a - N) for a in idx]
    w = gsw_weight(off[0], off[1], off[2], o1_edges, L, N)
    return w, np.bincount(b, weights=w, minlength=R)


def bin_average(C: np.ndarray, table, R: int, weights=None) -> np.ndarray:
    """Per-bin average of C over the table's lattice vectors, weighted by
    `weights` = (per-entry weights, per-bin sums) when given."""
    idx, b, counts = table
    if weights is None:
        sums = np.bincount(b, weights=C[idx], minlength=R)
        norm = counts
    else:
        w, norm = weights
        sums = np.bincount(b, weights=w * C[idx], minlength=R)
    with np.errstate(invalid="ignore", divide="ignore"):
        return sums / norm


def bin_counts_bruteforce(out_mode, o1_edges, o2_edges, L, N):
    """n_b by direct enumeration of all N^3 minimum-image lattice vectors."""
    a = np.arange(N)
    a = np.where(a < N // 2, a, a - N)
    I, J, K = np.meshgrid(a, a, a, indexing="ij")
    b = classify_lattice(I.ravel(), J.ravel(), K.ravel(), out_mode, o1_edges, o2_edges, L, N)
    R = n_out(out_mode, o1_edges, o2_edges)
    return np.bincount(b[b >= 0], minlength=R).astype(np.int64)
