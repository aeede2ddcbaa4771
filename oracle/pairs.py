"""Close-pair catalogue with integer bin keys (oracle, FP64, test infrastructure).

Follows the paper's pair catalogue rule (Implementation section, "Mock LRG
and LRG pair catalogue"): every unordered pair closer than the maximum pair
separation is kept, so a close triplet yields three pairs.  The pair's
position is its midpoint (Methodology, equation delta_pi_x); in a periodic
box that is x_i plus half the minimum-image separation, wrapped into [0, L).

Conventions fixed here (the paper is silent on them):
  * pair (i, j) has i < j by catalogue index and d = x_j - x_i, each
    component folded once into [-L/2, L/2): d >= L/2 -> d - L,
    d < -L/2 -> d + L;
  * s^2 = (dx*dx + dy*dy) + dz*dz in this order, FP64, no fused multiply-add;
  * bins are half-open [e_b, e_{b+1}) and tested on squares against e_b*e_b,
    so a value on an edge lands in the upper bin;
  * |mu| = |d_z|/s about the z line of sight; bin k is the largest k with
    dz*dz >= (mu_k*mu_k)*s^2, the top edge is closed (|mu| = 1 goes to the
    last bin);
  * r_p / pi mode: r_p^2 = dx*dx + dy*dy, |pi| = |dz|, kept iff s^2 < dmax^2
    and both fall in their half-open edge ranges;
  * key = b * n2 + k.
"""
from __future__ import annotations

import numpy as np


def min_image(d: np.ndarray, L: float) -> np.ndarray:
    h = L * 0.5
    return np.where(d >= h, d - L, np.where(d < -h, d + L, d))


def classify(dx, dy, dz, mode, p1_edges, p2_edges, dmax=None):
    """Return (keep mask, key) for separation components (FP64 arrays)."""
    e1 = np.asarray(p1_edges, np.float64)
    e2 = np.asarray(p2_edges, np.float64)
    n1, n2 = e1.size - 1, e2.size - 1
    xy = dx * dx + dy * dy
    zz = dz * dz
    s2 = xy + zz
    if mode == "s_mu":
        t1 = e1 * e1
        keep = (s2 >= t1[0]) & (s2 < t1[-1])
        b = np.searchsorted(t1, s2, side="right") - 1
        m2 = e2 * e2
        # count of mu edges satisfied; the predicate is monotone in k
        k = np.zeros(s2.shape, np.int64)
        for kk in range(n2 + 1):
            k += (zz >= m2[kk] * s2)
        keep &= (zz >= m2[0] * s2) & (zz <= m2[-1] * s2)
        k = np.minimum(k - 1, n2 - 1)
    elif mode == "rp_pi":
        if dmax is None:
            raise ValueError("rp_pi needs dmax")
        t1 = e1 * e1
        t2 = e2 * e2
        keep = (s2 < dmax * dmax) & (xy >= t1[0]) & (xy < t1[-1]) & (zz >= t2[0]) & (zz < t2[-1])
        b = np.searchsorted(t1, xy, side="right") - 1
        k = np.searchsorted(t2, zz, side="right") - 1
    else:
        raise ValueError(mode)
    key = np.where(keep, b * n2 + k, -1)
    return keep, key


def _emit(i, j, x, y, z, w, L, mode, p1_edges, p2_edges, dmax):
    dx = min_image(x[j] - x[i], L)
    dy = min_image(y[j] - y[i], L)
    dz = min_image(z[j] - z[i], L)
    keep, key = classify(dx, dy, dz, mode, p1_edges, p2_edges, dmax)
    i, j, key = i[keep], j[keep], key[keep]
    dx, dy, dz = dx[keep], dy[keep], dz[keep]
    mid = np.stack([x[i] + 0.5 * dx, y[i] + 0.5 * dy, z[i] + 0.5 * dz], axis=1)
    mid = np.where(mid >= L, mid - L, np.where(mid < 0.0, mid + L, mid))
    if w is None:
        wp = np.ones(i.shape[0])
    else:
        wp = w[i].astype(np.float64) * w[j].astype(np.float64)
    return i, j, key, mid, wp


def _finish(parts, n_fields):
    if parts:
        i = np.concatenate([p[0] for p in parts])
        j = np.concatenate([p[1] for p in parts])
        key = np.concatenate([p[2] for p in parts])
        mid = np.concatenate([p[3] for p in parts])
        wp = np.concatenate([p[4] for p in parts])
    else:
        i = j = key = np.zeros(0, np.int64)
        mid = np.zeros((0, 3))
        wp = np.zeros(0)
    order = np.lexsort((j, i))
    i, j, key, mid, wp = i[order], j[order], key[order], mid[order], wp[order]
    counts = np.bincount(key, minlength=n_fields).astype(np.int64)
    wsum = np.zeros(n_fields)
    np.add.at(wsum, key, wp)
    return dict(i=i, j=j, key=key, mid=mid, w=wp, counts=counts, wsum=wsum)


def bruteforce_pairs(x, y, z, w, L, mode, p1_edges, p2_edges, dmax=None, chunk=64):
    """O(N^2) enumeration of all i<j (chunked over i)."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64); z = np.asarray(z, np.float64)
    n = x.size
    n_fields = (len(p1_edges) - 1) * (len(p2_edges) - 1)
    parts = []
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        ii = np.arange(a, b)
        jj = np.arange(a + 1, n)
        I, J = np.meshgrid(ii, jj, indexing="ij")
        m = J > I
        parts.append(_emit(I[m], J[m], x, y, z, w, L, mode, p1_edges, p2_edges, dmax))
    return _finish(parts, n_fields)


def max_separation(mode, p1_edges, p2_edges, dmax=None):
    if mode == "s_mu":
        return float(p1_edges[-1])
    return float(min(dmax, np.hypot(p1_edges[-1], p2_edges[-1])))


def celllist_pairs(x, y, z, w, L, mode, p1_edges, p2_edges, dmax=None, max_cand=20_000_000):
    """Cell-list enumeration: cells of side >= s_max, the 27 neighbour cells.

    Written independently of the brute-force loop so the two can check each
    other's candidate enumeration (they share only ``classify``).
    """
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64); z = np.asarray(z, np.float64)
    n = x.size
    n_fields = (len(p1_edges) - 1) * (len(p2_edges) - 1)
    smax = max_separation(mode, p1_edges, p2_edges, dmax)
    nc = int(np.floor(L / smax))
    if nc < 3:
        raise ValueError("cell list needs at least 3 cells per side")
    side = L / nc
    c = np.stack([np.minimum((v / side).astype(np.int64), nc - 1) for v in (x, y, z)], axis=1)
    cid = (c[:, 0] * nc + c[:, 1]) * nc + c[:, 2]
    order = np.argsort(cid, kind="stable")
    cnt = np.bincount(cid, minlength=nc ** 3)
    start = np.concatenate([[0], np.cumsum(cnt)])
    parts = []
    offs = [(a, b, d) for a in (-1, 0, 1) for b in (-1, 0, 1) for d in (-1, 0, 1)]
    for (ox, oy, oz) in offs:
        nb = (((c[:, 0] + ox) % nc) * nc + (c[:, 1] + oy) % nc) * nc + (c[:, 2] + oz) % nc
        ncand = cnt[nb]
        # process galaxies in batches so the candidate arrays stay bounded
        csum = np.cumsum(ncand)
        lo = 0
        while lo < n:
            base = csum[lo - 1] if lo > 0 else 0
            hi = int(np.searchsorted(csum, base + max_cand, side="right"))
            hi = max(hi, lo + 1)
            hi = min(hi, n)
            gi = np.arange(lo, hi)
            reps = ncand[gi]
            I = np.repeat(gi, reps)
            # position of each candidate inside its neighbour cell
            first = np.repeat(start[nb[gi]], reps)
            within = np.arange(I.size) - np.repeat(np.cumsum(reps) - reps, reps)
            J = order[first + within]
            m = J > I
            if m.any():
                parts.append(_emit(I[m], J[m], x, y, z, w, L, mode, p1_edges, p2_edges, dmax))
            lo = hi
    return _finish(parts, n_fields)


def pairs_for(cat, wl, method="auto"):
    """Pairs of a synth catalogue under a workload's pair binning."""
    dmax = wl.pair_dmax if wl.pair_mode == "rp_pi" else None
    args = (cat.x, cat.y, cat.z, cat.w, cat.L, wl.pair_mode, wl.p1_edges, wl.p2_edges, dmax)
    if method == "brute" or (method == "auto" and cat.n <= 4000):
        return bruteforce_pairs(*args)
    return celllist_pairs(*args)
