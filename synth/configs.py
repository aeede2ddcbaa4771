"""Named workloads: catalogue recipe + grid + pair/output binning.

Sizes follow the five benchmark workloads of this project (plain FP64 at
128^3, production FP32 at 512^3, batched 256^3, redshift-space 1024^3, and the
weighted 512^3 HOD-fit case) plus a tiny 64^3 case for brute-force gradient
checks.  Pair modes: "s_mu" (separation s, |mu| = |d_z|/s w.r.t. the z line of
sight) and "rp_pi" (r_p, |pi| = |d_z| inside a sphere |d| < dmax).  Output
modes: "shell", "r_mu", "rp_pi", and "gsw" (the paper's Gaussian-sigmoid
weighting function as one weighted output bin; o1_edges then holds its
parameters sigma, r_s, s_0, r_cut and the cut radius r_max).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Callable, Optional

import numpy as np

from .catalog import Catalog, flat_lcdm_aH, make_catalog


def logbins(lo, hi, n):
    return np.logspace(np.log10(lo), np.log10(hi), n + 1)


def linbins(lo, hi, n):
    return np.linspace(lo, hi, n + 1)


@dataclass
class Workload:
    name: str
    L: float
    N: int
    precision: str            # "fp64" | "fp32"
    pair_mode: str            # "s_mu" | "rp_pi"
    p1_edges: np.ndarray      # s or r_p edges
    p2_edges: np.ndarray      # |mu| or |pi| edges
    out_mode: str             # "shell" | "r_mu" | "rp_pi"
    o1_edges: np.ndarray
    o2_edges: Optional[np.ndarray]
    catalog_kw: dict
    pair_dmax: float = 0.0    # rp_pi only
    qeff_mode: str = "notsq"
    xi_w_const: float = 0.0
    weighted: bool = False
    assignment: str = "cic"   # mass assignment: "cic" or "tsc"
    seed: int = 1000
    description: str = ""

    @property
    def n_fields(self) -> int:
        return (len(self.p1_edges) - 1) * (len(self.p2_edges) - 1)

    @property
    def n_out(self) -> int:
        if self.out_mode == "gsw":
            return 1
        n2 = 1 if self.o2_edges is None else len(self.o2_edges) - 1
        return (len(self.o1_edges) - 1) * n2

    def catalog(self, seed: Optional[int] = None) -> Catalog:
        return make_catalog(L=self.L, seed=self.seed if seed is None else seed, **self.catalog_kw)

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


_AH_Z05 = flat_lcdm_aH(0.5, 0.31)

# The paper's weighting-function table: (sigma, r_s, s_0, r_cut) and xi(d_w)
# for maximum pair separations 10 and 30 Mpc/h; the cut radius of the lattice
# window is 5 sigma (the Gaussian is down to 4e-6 there).
GSW_DP10 = dict(sigma=30.0, rs=20.0, s0=0.8, rcut=10.0, xi_dw=0.362)
GSW_DP30 = dict(sigma=50.0, rs=35.0, s0=0.5, rcut=20.0, xi_dw=0.104)


def gsw_params(t, rmax_sigmas=5.0):
    return np.array([t["sigma"], t["rs"], t["s0"], t["rcut"], rmax_sigmas * t["sigma"]])

_CFG1_CAT = dict(n_halos=40000, mass_dist="powerlaw", m_lo=1e13, m_hi=2e15, slope=1.9,
                 placement="sp", sat_mode="poisson", n_field=800000)

CONFIGS = {
    "cfg0": Workload(
        name="cfg0", L=250.0, N=128, precision="fp64", pair_mode="s_mu",
        p1_edges=linbins(0.5, 10.0, 5), p2_edges=np.array([0.0, 1.0]),
        out_mode="shell", o1_edges=logbins(10.0, 60.0, 15), o2_edges=None,
        catalog_kw=dict(n_halos=200, mass_dist="loguniform", m_lo=1e13, m_hi=1e15,
                        placement="uniform", sat_mode="poisson", n_field=15000),
        seed=1000, description="plain FP64, L=250, 128^3, 5 linear s-bins, 15 log r-bins"),
    "cfg1": Workload(
        name="cfg1", L=1000.0, N=512, precision="fp32", pair_mode="s_mu",
        p1_edges=logbins(0.5, 10.0, 20), p2_edges=linbins(0.0, 1.0, 10),
        out_mode="shell", o1_edges=logbins(10.0, 80.0, 20), o2_edges=None,
        catalog_kw=dict(_CFG1_CAT), seed=1001,
        description="production FP32, L=1000, 512^3, 20 log s x 10 |mu| fields, 20 log r-bins"),
    "cfg2": Workload(
        name="cfg2", L=500.0, N=256, precision="fp32", pair_mode="s_mu",
        p1_edges=logbins(0.5, 10.0, 20), p2_edges=linbins(0.0, 1.0, 8),
        out_mode="shell", o1_edges=logbins(10.0, 80.0, 20), o2_edges=None,
        catalog_kw=dict(_CFG1_CAT, n_halos=5000, n_field=100000), seed=1002,
        description="batched FP32, L=500, 256^3, 160 fields, 20 log r-bins"),
    "cfg3": Workload(
        name="cfg3", L=2000.0, N=1024, precision="fp32", pair_mode="rp_pi",
        p1_edges=linbins(0.0, 30.0, 16), p2_edges=linbins(0.0, 30.0, 8), pair_dmax=30.0,
        out_mode="rp_pi", o1_edges=linbins(0.0, 80.0, 24), o2_edges=linbins(0.0, 80.0, 24),
        catalog_kw=dict(_CFG1_CAT, n_halos=320000, n_field=6400000, rsd=True, aH=_AH_Z05),
        seed=1003, description="redshift space, L=2000, 1024^3, 16 r_p x 8 pi fields, 24x24 (r_p,pi)"),
    "cfg4": Workload(
        name="cfg4", L=1000.0, N=512, precision="fp32", pair_mode="s_mu",
        p1_edges=logbins(0.5, 10.0, 20), p2_edges=np.array([0.0, 1.0]),
        out_mode="shell", o1_edges=logbins(10.0, 80.0, 20), o2_edges=None,
        catalog_kw=dict(_CFG1_CAT, sat_mode="candidates", n_candidates=49, n_field=0),
        weighted=True, seed=1004,
        description="weighted HOD candidates, L=1000, 512^3, 20 s-bins x 20 r-bins, fwd+bwd"),
    "cfg1w": Workload(
        name="cfg1w", L=1000.0, N=512, precision="fp32", pair_mode="s_mu",
        p1_edges=logbins(0.5, 10.0, 20), p2_edges=linbins(0.0, 1.0, 10),
        out_mode="gsw", o1_edges=gsw_params(GSW_DP10), o2_edges=None,
        qeff_mode="const", xi_w_const=GSW_DP10["xi_dw"],
        catalog_kw=dict(_CFG1_CAT), seed=1001,
        description="production catalogue, L=1000, 512^3, 20 log s x 10 |mu| fields, the paper's "
                    "weighting function for d_p,max = 10 (one weighted bin, Q_eff with its xi(d_w))"),
    "cfg4tiny": Workload(
        name="cfg4tiny", L=125.0, N=64, precision="fp32", pair_mode="s_mu",
        p1_edges=logbins(0.5, 10.0, 20), p2_edges=np.array([0.0, 1.0]),
        out_mode="shell", o1_edges=logbins(10.0, 60.0, 20), o2_edges=None,
        catalog_kw=dict(_CFG1_CAT, n_halos=40, sat_mode="candidates", n_candidates=49,
                        n_field=0, placement="uniform"),
        weighted=True, seed=1104,
        description="tiny weighted case for brute-force gradients: L=125, 64^3, ~2k candidates"),
}


def get_config(name: str) -> Workload:
    return CONFIGS[name]


# Fiducial HOD of the paper (Implementation section, equation hod) and the
# alpha = 1.05 refit row of the HOD-parameter table (HOD dependency section).
HOD_FIDUCIAL = dict(logMcut=13.35, logM1=13.8, sigma=0.85, alpha=1.0, kappa=1.0)
HOD_TARGET = dict(logMcut=13.35 - 0.086, logM1=13.8 - 0.018, sigma=0.85 - 0.16,
                  alpha=1.05, kappa=1.0)
