"""End-to-end oracle forward: catalogue -> xi_gg, xi_pg, xi_dp, b_pg, Q_eff.

Plain definitions in the paper's order: pair catalogue, mass assignment of
galaxies and of each pair bin's midpoints, overdensities, the grid
correlation of each pair field with the galaxy field, bin averages, then the
finalisation formulas.  FP64 throughout; ``scipy.fft`` is the FFT primitive.
"""
from __future__ import annotations

import numpy as np

from . import bins as _bins
from .cic import assign, overdensity
from .corr import irfftn, rfftn
from .finalize import field_volumes, finalize
from .pairs import pairs_for


def weights_or_ones(cat):
    return np.ones(cat.n) if cat.w is None else np.asarray(cat.w, np.float64)


def galaxy_side(cat, wl, w=None):
    """delta_g spectrum, lattice table and xi_gg."""
    N, L = wl.N, wl.L
    w = weights_or_ones(cat) if w is None else np.asarray(w, np.float64)
    wg = float(np.sum(w))
    rho_g = assign(cat.positions(), w, N, L, getattr(wl, "assignment", "cic"))
    dg = overdensity(rho_g, wg)
    Fg = rfftn(dg)
    table = _bins.lattice_table(wl.out_mode, wl.o1_edges, wl.o2_edges, L, N)
    R = _bins.n_out(wl.out_mode, wl.o1_edges, wl.o2_edges)
    bw = _bins.lattice_weights(wl.out_mode, wl.o1_edges, wl.o2_edges, L, N, table)
    Cgg = irfftn(Fg * np.conj(Fg), dg.shape) / dg.size
    xi_gg = _bins.bin_average(Cgg, table, R, bw)
    return dict(wg=wg, dg=dg, Fg=Fg, table=table, R=R, bw=bw, xi_gg=xi_gg, w=w)


def pair_field_xi(pairs, f, gal, wl):
    """xi_pg[f, :] for one pair field (NaN row when the field is empty)."""
    N, L = wl.N, wl.L
    sel = pairs["key"] == f
    ws = float(np.sum(pairs["w"][sel]))
    if ws == 0.0:
        return np.full(gal["R"], np.nan)
    rho_f = assign(pairs["mid"][sel], pairs["w"][sel], N, L, getattr(wl, "assignment", "cic"))
    df = overdensity(rho_f, ws)
    C = irfftn(np.conj(rfftn(df)) * gal["Fg"], df.shape) / df.size
    return _bins.bin_average(C, gal["table"], gal["R"], gal["bw"])


def forward(cat, wl, pairs=None, fields=None, w=None):
    """Full oracle forward.  ``fields`` restricts which xi_pg rows are computed
    (others NaN); finalisation is then only meaningful on those rows.  ``w``
    overrides the catalogue weights (pair weights and sums follow from it)."""
    gal = galaxy_side(cat, wl, w=w)
    if pairs is None:
        pairs = pairs_for(cat, wl)
    if w is not None:
        pairs = dict(pairs)
        ww = np.asarray(w, np.float64)
        pairs["w"] = ww[pairs["i"]] * ww[pairs["j"]]
        wsum = np.zeros(wl.n_fields)
        np.add.at(wsum, pairs["key"], pairs["w"])
        pairs["wsum"] = wsum
    F = wl.n_fields
    xi_pg = np.full((F, gal["R"]), np.nan)
    for f in (range(F) if fields is None else fields):
        xi_pg[f] = pair_field_xi(pairs, f, gal, wl)
    dmax = wl.pair_dmax if wl.pair_mode == "rp_pi" else None
    vol = field_volumes(wl.pair_mode, wl.p1_edges, wl.p2_edges, dmax)
    fin = finalize(gal["xi_gg"], xi_pg, pairs["wsum"], gal["wg"], wl.L, vol,
                   wl.qeff_mode, wl.xi_w_const)
    return dict(counts=pairs["counts"], wsum=pairs["wsum"], wg=gal["wg"], xi_gg=gal["xi_gg"],
                xi_pg=xi_pg, volumes=vol, n_b=gal["table"][2], norm_b=gal["bw"][1], pairs=pairs,
                **fin)
