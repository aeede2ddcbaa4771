"""Finalisation: xi(d_p), b_pg, Q_eff (oracle, FP64).

  xi_dp[f] = 2 Wsum_f L^3 / ((sum w)^2 V_f) - 1
      the paper's pair-count 2PCF (2PCF section, equation 2PCF_d_collapsed,
      xi = 2 N_p / (nbar_g N_g dV) - 1 with nbar_g = N_g / L^3), with counts
      replaced by weight sums and the thin-shell volume 4 pi d^2 dd replaced by
      the exact volume V_f of the pair bin;
  b_pg = xi_pg / xi_gg   (Introduction, eq. 1);
  Q_eff, not strictly squeezed (Methodology, equation Qeff_notsq, the one the
      paper uses for its results):
      Q = ((1 + xi_dp) b - 2 - xi_w / (2 xi_dp)) / (2 xi_dp + 1.5 xi_w)
  Q_eff, squeezed limit (Methodology, equation Qeff):
      Q = ((1 + xi_dp) b - 2) / (2 xi_dp)
  b_pg from Q (forward relations, equations bpg_squeezed and
      bpg_notsq_dw) are provided for the round-trip checks.
Projected 2PCF (2PCF section, equation 2PCF_los_integrated_explicit): the
  line-of-sight integral of xi(d_p) inside the pair sphere per r_p annulus,
      w_p[a] = sum_b xi_dp[a, b] V[a, b] / (pi (rp_{a+1}^2 - rp_a^2)),
  pieces of zero volume (wholly outside the sphere) contributing nothing.
xi_w is the paper's xi(d_w) (equation xi_dw).  For a thin-shell bin W the
ratio int W xi^2 / int W xi tends to xi at the shell radius, so the default
reading takes xi_w = xi_gg[b]; a constant xi_w can be given instead.
"""
from __future__ import annotations

import math

import numpy as np


def volume_s_mu(s_lo, s_hi, mu_lo, mu_hi):
    """Volume of {s in [s_lo, s_hi), |mu| in [mu_lo, mu_hi]} (both signs of mu)."""
    return (4.0 * math.pi / 3.0) * (s_hi ** 3 - s_lo ** 3) * (mu_hi - mu_lo)


def _slab_integral(r0, r1, D, c, d):
    """int_{r0}^{r1} 2 pi r * len([c, d] cap [0, sqrt(D^2 - r^2)]) dr (one sign of pi)."""
    if r1 <= r0:
        return 0.0
    total = 0.0
    # breakpoints where sqrt(D^2 - r^2) crosses d and c
    bd = math.sqrt(max(D * D - d * d, 0.0)) if d < D else 0.0
    bc = math.sqrt(max(D * D - c * c, 0.0)) if c < D else 0.0
    pts = sorted({r0, r1, min(max(bd, r0), r1), min(max(bc, r0), r1)})
    for a, b in zip(pts[:-1], pts[1:]):
        if b <= a:
            continue
        m = 0.5 * (a + b)
        h = math.sqrt(max(D * D - m * m, 0.0))
        top = min(d, h)
        if top <= c:
            continue
        if top == d:  # constant length d - c on this piece
            total += math.pi * (d - c) * (b * b - a * a)
        else:  # length sqrt(D^2 - r^2) - c
            F = lambda r: -(2.0 * math.pi / 3.0) * (max(D * D - r * r, 0.0)) ** 1.5 - math.pi * c * r * r
            total += F(b) - F(a)
    return total


def volume_rp_pi(rp_lo, rp_hi, pi_lo, pi_hi, dmax):
    """Volume of {r_p in [rp_lo, rp_hi), |pi| in [pi_lo, pi_hi), |d| < dmax}, both signs of pi."""
    return 2.0 * _slab_integral(rp_lo, min(rp_hi, dmax), dmax, pi_lo, pi_hi)


def field_volumes(mode, p1_edges, p2_edges, dmax=None):
    e1 = np.asarray(p1_edges, np.float64)
    e2 = np.asarray(p2_edges, np.float64)
    out = []
    for b in range(e1.size - 1):
        for k in range(e2.size - 1):
            if mode == "s_mu":
                out.append(volume_s_mu(e1[b], e1[b + 1], e2[k], e2[k + 1]))
            else:
                out.append(volume_rp_pi(e1[b], e1[b + 1], e2[k], e2[k + 1], dmax))
    return np.array(out)


def xi_dp(wsum, wg, L, volumes):
    return 2.0 * np.asarray(wsum) * L ** 3 / (wg * wg * np.asarray(volumes)) - 1.0


def projected_2pcf(xdp, volumes, rp_edges, n_p2):
    """w_p per r_p annulus from xi(d_p) of (r_p, |pi|) pair bins (field index
    a * n_p2 + b)."""
    e = np.asarray(rp_edges, np.float64)
    n1 = e.size - 1
    x = np.asarray(xdp, np.float64).reshape(n1, n_p2)
    v = np.asarray(volumes, np.float64).reshape(n1, n_p2)
    col = np.where(v > 0.0, np.nan_to_num(x) * v, 0.0).sum(axis=1)
    return col / (math.pi * (e[1:] ** 2 - e[:-1] ** 2))


def q_eff(b, xdp, xi_w, mode="notsq"):
    b = np.asarray(b, np.float64)
    xdp = np.asarray(xdp, np.float64)
    xi_w = np.asarray(xi_w, np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        if mode == "squeezed":
            return ((1.0 + xdp) * b - 2.0) / (2.0 * xdp)
        return ((1.0 + xdp) * b - 2.0 - xi_w / (2.0 * xdp)) / (2.0 * xdp + 1.5 * xi_w)


def b_from_q(q, xdp, xi_w, mode="notsq"):
    if mode == "squeezed":
        return 2.0 * (1.0 + q * xdp) / (1.0 + xdp)
    return (2.0 + xi_w / (2.0 * xdp) + q * (2.0 * xdp + 1.5 * xi_w)) / (1.0 + xdp)


def finalize(xi_gg, xi_pg, wsum, wg, L, volumes, qeff_mode="notsq", xi_w_const=0.0):
    xi_gg = np.asarray(xi_gg, np.float64)
    xi_pg = np.asarray(xi_pg, np.float64)
    xdp = xi_dp(wsum, wg, L, volumes)
    with np.errstate(invalid="ignore", divide="ignore"):
        b = xi_pg / xi_gg[None, :]
    if qeff_mode == "const":
        xi_w = np.full_like(b, xi_w_const)
        mode = "notsq"
    else:
        xi_w = np.broadcast_to(xi_gg[None, :], b.shape)
        mode = qeff_mode
    q = q_eff(b, xdp[:, None], xi_w, mode)
    return dict(xi_dp=xdp, b_pg=b, q_eff=q)
