"""Gradients of the estimator w.r.t. per-galaxy weights and HOD parameters
(oracle, FP64, test infrastructure).

The paper fits HODs with numerical derivatives (HOD dependency section,
emulator equations 2pf_emulate_1st/2nd); here the chain is written out by
hand.  Upstream gradients g_b, g_q, g_xipg (F x R), g_xigg (R) and g_xidp (F)
define the scalar J = <g_b, b> + <g_q, Q> + <g_xipg, xi_pg> + <g_xigg, xi_gg>
+ <g_xidp, xi_dp>; the functions return dJ/dw.  Entries that are not finite in
the forward (empty fields) carry no gradient.

Chain, with c_f = N_c / Wsum_f and c_g = N_c / W_g:
  xi_pg[f,b] = (N_c n_b)^-1 sum_{r in b} sum_x d_f(x) d_g(x + r)
  xi_gg[b]   = (N_c n_b)^-1 sum_{r in b} sum_x d_g(x) d_g(x + r)
  d_f = c_f rho_f - 1,   d_g = c_g rho_g - 1
  kappa_f(r) = sum_b gbar_pg[f,b] w(r) 1[r in b] / (N_c norm_b), kappa_g likewise
  (w = 1, norm_b = n_b for the indicator bins; W and sum W for the weighted one)
  dJ/dd_f(x) = sum_r kappa_f(r) d_g(x + r)
  dJ/dd_g(y) = sum_f sum_r kappa_f(r) d_f(y - r)
               + sum_r kappa_g(r) [d_g(y - r) + d_g(y + r)]
  dJ/drho = c * dJ/dd,   dJ/dWsum_f += -(N_c / Wsum_f^2) <dJ/dd_f, rho_f>
  rho_f = sum_pairs w_i w_j K(x - m_ij), rho_g = sum_i w_i K(x - x_i)
The lattice sums are evaluated either by FFT or directly (tiny grids only).
"""
from __future__ import annotations

import numpy as np

from . import bins as _bins
from .cic import assign, gather
from .corr import irfftn, rfftn
from .finalize import field_volumes, xi_dp as _xi_dp
from .pipeline import forward


# ----------------------------------------------------------------------------
# HOD occupation weights (smooth version of the paper's equation hod)
# ----------------------------------------------------------------------------
LN10 = np.log(10.0)


def _sigmoid(t):
    return 1.0 / (1.0 + np.exp(-t))


def hod_weights(halo_mass, kind, theta, n_candidates=49, per_candidate=True):
    """Occupation weights for central (kind 1) and satellite (kind 2) candidates.

    theta = (logMcut, logM1, sigma, alpha), log10 masses; M0 = Mcut (kappa = 1).
      central:   w = sigmoid((ln M - ln Mcut) / sigma)
      satellite: w = (max(M - M0, 0) / M1)^alpha * sigmoid(...) [/ K_h]
    The satellite term divides by the number of candidates per halo when
    ``per_candidate`` (the paper assigns satellites with per-particle
    probability <n_sat>/n_particle).  Field galaxies (kind 0) get weight 1.
    """
    logMcut, logM1, sigma, alpha = [float(t) for t in theta]
    M = np.asarray(halo_mass, np.float64)
    lnM = np.log(np.where(M > 0, M, 1.0))
    s = _sigmoid((lnM - logMcut * LN10) / sigma)
    M0 = 10.0 ** logMcut
    M1 = 10.0 ** logM1
    base = np.maximum(M - M0, 0.0) / M1
    pos = base > 0
    powv = np.where(pos, np.exp(alpha * np.log(np.where(pos, base, 1.0))), 0.0)
    sat = powv * s / (n_candidates if per_candidate else 1.0)
    w = np.where(kind == 1, s, np.where(kind == 2, sat, 1.0))
    return w


def hod_weight_jacobian(halo_mass, kind, theta, n_candidates=49, per_candidate=True):
    """d w_i / d theta_k, analytic, shape (n, 4)."""
    logMcut, logM1, sigma, alpha = [float(t) for t in theta]
    M = np.asarray(halo_mass, np.float64)
    lnM = np.log(np.where(M > 0, M, 1.0))
    t = (lnM - logMcut * LN10) / sigma
    s = _sigmoid(t)
    ds = s * (1.0 - s)
    ds_dlogMcut = ds * (-LN10 / sigma)
    ds_dsigma = ds * (-t / sigma)
    M0 = 10.0 ** logMcut
    M1 = 10.0 ** logM1
    base = np.maximum(M - M0, 0.0) / M1
    pos = base > 0
    lb = np.log(np.where(pos, base, 1.0))
    powv = np.where(pos, np.exp(alpha * lb), 0.0)
    # d base/d logMcut = -M0 ln10 / M1 ; d base / d logM1 = -base ln10
    dpow_dbase = np.where(pos, alpha * np.exp((alpha - 1.0) * lb), 0.0)
    dpow_dlogMcut = dpow_dbase * (-M0 * LN10 / M1)
    dpow_dlogM1 = dpow_dbase * (-base * LN10)
    dpow_dalpha = powv * lb
    k = (n_candidates if per_candidate else 1.0)
    J = np.zeros((M.size, 4))
    cen = kind == 1
    sat = kind == 2
    J[cen, 0] = ds_dlogMcut[cen]
    J[cen, 2] = ds_dsigma[cen]
    J[sat, 0] = (dpow_dlogMcut * s + powv * ds_dlogMcut)[sat] / k
    J[sat, 1] = (dpow_dlogM1 * s)[sat] / k
    J[sat, 2] = (powv * ds_dsigma)[sat] / k
    J[sat, 3] = (dpow_dalpha * s)[sat] / k
    return J


# ----------------------------------------------------------------------------
# finalisation adjoint
# ----------------------------------------------------------------------------
def _z(a, shape):
    return np.zeros(shape) if a is None else np.nan_to_num(np.asarray(a, np.float64), nan=0.0)


def finalize_adjoint(out, wl, g_b=None, g_q=None, g_xipg=None, g_xigg=None, g_xidp=None):
    """Returns (gbar_pg [F,R], gbar_gg [R], gbar_wsum [F], gbar_wg)."""
    xi_gg = out["xi_gg"]; xi_pg = out["xi_pg"]; b = out["b_pg"]
    x = out["xi_dp"][:, None]
    F, R = xi_pg.shape
    g_b = _z(g_b, (F, R)); g_q = _z(g_q, (F, R)); g_xipg = _z(g_xipg, (F, R))
    g_xigg = _z(g_xigg, (R,)); g_xidp = _z(g_xidp, (F,))
    mode = wl.qeff_mode
    with np.errstate(invalid="ignore", divide="ignore"):
        if mode == "squeezed":
            dq_db = (1.0 + x) / (2.0 * x)
            dq_dx = (2.0 - b) / (2.0 * x * x)
            dq_dxw = np.zeros_like(b)
        else:
            xw = wl.xi_w_const if mode == "const" else xi_gg[None, :]
            num = (1.0 + x) * b - 2.0 - xw / (2.0 * x)
            den = 2.0 * x + 1.5 * xw
            dq_db = (1.0 + x) / den
            dq_dx = ((b + xw / (2.0 * x * x)) * den - 2.0 * num) / (den * den)
            dq_dxw = (-den / (2.0 * x) - 1.5 * num) / (den * den)
            if mode == "const":
                dq_dxw = np.zeros_like(b)
        gbt = g_b + g_q * dq_db
        gpg = g_xipg + gbt / xi_gg[None, :]
        ggg = g_xigg + np.nansum(-gbt * b / xi_gg[None, :] + g_q * dq_dxw, axis=0)
        gx = g_xidp + np.nansum(g_q * dq_dx, axis=1)
    finite = np.isfinite(xi_pg)
    gpg = np.where(finite, gpg, 0.0)
    gx = np.where(np.isfinite(out["xi_dp"]) & (out["wsum"] > 0), gx, 0.0)
    # xi_dp = 2 Wsum L^3 / (Wg^2 V) - 1
    with np.errstate(invalid="ignore", divide="ignore"):
        gws = np.where(out["wsum"] > 0, gx * (out["xi_dp"] + 1.0) / out["wsum"], 0.0)
    gwg = float(np.sum(gx * -2.0 * (out["xi_dp"] + 1.0) / out["wg"]))
    return np.nan_to_num(gpg), np.nan_to_num(ggg), gws, gwg


# ----------------------------------------------------------------------------
# weight gradient
# ----------------------------------------------------------------------------
def _kappa_grid(gbar, table, N, R, bw):
    """kappa(r) = dJ/dC(r) = gbar_b w(r) / (N^3 norm_b) for r in bin b (w = 1
    and norm_b = n_b for the indicator bins)."""
    idx, b, counts = table
    w, norm = bw
    k = np.zeros((N, N, N))
    with np.errstate(invalid="ignore", divide="ignore"):
        per_bin = np.where(norm > 0, gbar / (N ** 3 * norm), 0.0)
    k[idx] = per_bin[b] * w
    return k


def _corr_sum(kappa, d):
    """out(x) = sum_r kappa(r) d(x + r)."""
    return irfftn(np.conj(rfftn(kappa)) * rfftn(d), d.shape)


def _conv_sum(kappa, d):
    """out(y) = sum_r kappa(r) d(y - r)."""
    return irfftn(rfftn(kappa) * rfftn(d), d.shape)


def _corr_sum_direct(kappa, d):
    N = d.shape[0]
    out = np.zeros_like(d)
    for r in np.argwhere(kappa != 0):
        out += kappa[tuple(r)] * np.roll(d, shift=(-r[0], -r[1], -r[2]), axis=(0, 1, 2))
    return out


def _conv_sum_direct(kappa, d):
    out = np.zeros_like(d)
    for r in np.argwhere(kappa != 0):
        out += kappa[tuple(r)] * np.roll(d, shift=(r[0], r[1], r[2]), axis=(0, 1, 2))
    return out


def weight_gradient(cat, wl, w, g_b=None, g_q=None, g_xipg=None, g_xigg=None, g_xidp=None,
                    method="fft", pairs=None):
    """dJ/dw for every galaxy (FP64)."""
    N, L = wl.N, wl.L
    w = np.asarray(w, np.float64)
    out = forward(cat, wl, pairs=pairs, w=w)
    pairs = out["pairs"]
    gpg, ggg, gws, gwg = finalize_adjoint(out, wl, g_b, g_q, g_xipg, g_xigg, g_xidp)
    table = _bins.lattice_table(wl.out_mode, wl.o1_edges, wl.o2_edges, L, N)
    bw = _bins.lattice_weights(wl.out_mode, wl.o1_edges, wl.o2_edges, L, N, table)
    R = table[2].size
    Nc = N ** 3
    corr = _corr_sum if method == "fft" else _corr_sum_direct
    conv = _conv_sum if method == "fft" else _conv_sum_direct
    pos = cat.positions()
    wg = out["wg"]
    scheme = getattr(wl, "assignment", "cic")
    rho_g = assign(pos, w, N, L, scheme)
    dg = rho_g * (Nc / wg) - 1.0
    E = np.zeros((N, N, N))
    kg = _kappa_grid(ggg, table, N, R, bw)
    E += conv(kg, dg) + corr(kg, dg)
    grad = np.zeros(cat.n)
    for f in range(wl.n_fields):
        sel = pairs["key"] == f
        ws = out["wsum"][f]
        if ws <= 0 or not np.any(gpg[f] != 0) and gws[f] == 0:
            continue
        mid = pairs["mid"][sel]
        pw = pairs["w"][sel]
        rho_f = assign(mid, pw, N, L, scheme)
        df = rho_f * (Nc / ws) - 1.0
        kf = _kappa_grid(gpg[f], table, N, R, bw)
        D = corr(kf, dg)
        E += conv(kf, df)
        drho_f = D * (Nc / ws)
        gws_f = gws[f] - (Nc / ws ** 2) * float(np.sum(D * rho_f))
        gath = gather(drho_f, mid, N, L, scheme) + gws_f
        ii = pairs["i"][sel]; jj = pairs["j"][sel]
        np.add.at(grad, ii, w[jj] * gath)
        np.add.at(grad, jj, w[ii] * gath)
    drho_g = E * (Nc / wg)
    gwg_tot = gwg - (Nc / wg ** 2) * float(np.sum(E * rho_g))
    grad += gather(drho_g, pos, N, L, scheme) + gwg_tot
    return grad, out


def objective(out, g_b=None, g_q=None, g_xipg=None, g_xigg=None, g_xidp=None):
    """J = sum of upstream-weighted outputs (finite entries only)."""
    J = 0.0
    for g, key in ((g_b, "b_pg"), (g_q, "q_eff"), (g_xipg, "xi_pg"), (g_xigg, "xi_gg"),
                   (g_xidp, "xi_dp")):
        if g is None:
            continue
        v = out[key]
        m = np.isfinite(v) & np.isfinite(g)
        J += float(np.sum(np.asarray(g)[m] * v[m]))
    return J


def fd_weight_gradient(cat, wl, w, idx, h=1e-3, pairs=None, **g):
    """Central differences dJ/dw_i for i in idx, step h * max(|w_i|, 0.1)
    (an absolute floor so that zero weights get a usable step)."""
    w = np.asarray(w, np.float64)
    out0 = forward(cat, wl, pairs=pairs, w=w)
    pairs = out0["pairs"]
    res = []
    for i in idx:
        step = h * max(abs(w[i]), 0.1)
        wp = w.copy(); wp[i] += step
        wm = w.copy(); wm[i] -= step
        Jp = objective(forward(cat, wl, pairs=pairs, w=wp), **g)
        Jm = objective(forward(cat, wl, pairs=pairs, w=wm), **g)
        res.append((Jp - Jm) / (2 * step))
    return np.array(res)
