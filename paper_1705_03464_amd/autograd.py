"""torch.autograd wrapper of the forward/adjoint pair and the smooth HOD
occupation weights (the paper's HOD form, Implementation section, equation
hod, with a logistic step for the central occupation)."""
from __future__ import annotations

import math

import torch

from ._lib import Plan

LN10 = math.log(10.0)


class PairGalaxyXi(torch.autograd.Function):
    """(xi_gg, xi_pg, xi_dp, b_pg, q_eff) = f(w) for the plan's catalogue.

    Differentiable in the galaxy weights w (float32, one per galaxy).  The
    plan keeps the state of its last forward, so each forward must be followed
    by its backward before the plan runs another forward.
    """

    @staticmethod
    def forward(ctx, w: torch.Tensor, plan: Plan):
        # a backward will follow: let the plan keep the pair-field spectra
        plan.keep_spectra(bool(ctx.needs_input_grad[0]))
        out = plan.forward(w.detach().contiguous())
        ctx.plan = plan
        ctx.count = plan.forward_count
        return out["xi_gg"], out["xi_pg"], out["xi_dp"], out["b_pg"], out["q_eff"]

    @staticmethod
    def backward(ctx, g_xigg, g_xipg, g_xidp, g_b, g_q):
        plan = ctx.plan
        if plan.forward_count != ctx.count:
            raise RuntimeError("the plan ran another forward before this backward")
        grad = plan.backward(g_b_pg=g_b, g_q_eff=g_q, g_xi_pg=g_xipg, g_xi_gg=g_xigg, g_xi_dp=g_xidp)
        return grad, None


def pair_galaxy_xi(plan: Plan, w: torch.Tensor):
    """Differentiable forward; returns a dict of the five outputs."""
    xi_gg, xi_pg, xi_dp, b_pg, q_eff = PairGalaxyXi.apply(w, plan)
    return dict(xi_gg=xi_gg, xi_pg=xi_pg, xi_dp=xi_dp, b_pg=b_pg, q_eff=q_eff)


class MultipoleXi(torch.autograd.Function):
    """xi_l [F][R][lmax/2 + 1] = f(w): the multipoles of xi_pg in the angle
    between the pair axis and the pair-to-galaxy direction, differentiable in
    the galaxy weights (forward, then pgx_multipoles; the backward is
    pgx_multipoles_backward)."""

    @staticmethod
    def forward(ctx, w: torch.Tensor, plan: Plan, lmax: int):
        plan.keep_spectra(False)
        plan.forward(w.detach().contiguous())
        out = plan.multipoles(lmax)
        ctx.plan = plan
        ctx.count = plan.forward_count
        return out

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        if plan.forward_count != ctx.count:
            raise RuntimeError("the plan ran another forward before this backward")
        return plan.multipoles_backward(g), None, None


def pair_galaxy_multipoles(plan: Plan, w: torch.Tensor, lmax: int = 2) -> torch.Tensor:
    """Differentiable multipoles xi_l, l = 0, 2, .., lmax."""
    return MultipoleXi.apply(w, plan, lmax)


def hod_weights(theta: torch.Tensor, halo_mass: torch.Tensor, kind: torch.Tensor,
                n_candidates: int = 49, per_candidate: bool = True) -> torch.Tensor:
    """Occupation weights of central (kind 1) and satellite (kind 2) candidates.

    theta = (log10 Mcut, log10 M1, sigma, alpha), with M0 = Mcut (kappa = 1):
      central    w = sigmoid((ln M - ln Mcut) / sigma)
      satellite  w = (max(M - M0, 0) / M1)^alpha sigmoid(...) / n_candidates
    (the division mirrors the paper's per-particle satellite probability
    <n_sat> / n_particle).  Other kinds get weight 1.  Returns float32.
    """
    lmc, lm1, sig, alpha = theta[0], theta[1], theta[2], theta[3]
    M = halo_mass.to(torch.float64)
    lnM = torch.log(torch.where(M > 0, M, torch.ones_like(M)))
    s = torch.sigmoid((lnM - lmc.to(torch.float64) * LN10) / sig.to(torch.float64))
    M0 = torch.pow(torch.tensor(10.0, dtype=torch.float64, device=M.device), lmc.to(torch.float64))
    M1 = torch.pow(torch.tensor(10.0, dtype=torch.float64, device=M.device), lm1.to(torch.float64))
    base = (M - M0) / M1
    pos = base > 0
    safe = torch.where(pos, base, torch.ones_like(base))
    powv = torch.where(pos, torch.exp(alpha.to(torch.float64) * torch.log(safe)), torch.zeros_like(base))
    sat = powv * s / (n_candidates if per_candidate else 1.0)
    w = torch.where(kind == 1, s, torch.where(kind == 2, sat, torch.ones_like(s)))
    return w.to(torch.float32)
