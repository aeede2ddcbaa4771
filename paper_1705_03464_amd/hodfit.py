"""Gradient-based HOD fit on the adjoint (replaces the paper's emulator and
Powell / Nelder-Mead / BFGS fits of its HOD-dependency section with gradient
descent on the HOD parameters, through the hand-written adjoint).

Loss terms:
  * pair-galaxy bias: sum over (pair bin, output bin) of (b_pg - target)^2
    over the entries finite in both, from a plan binned by (s, |mu|);
  * projected 2PCF (Section "2PCF", equation 2PCF_los_integrated_explicit):
    w(d_perp) is the line-of-sight integral of the pair correlation inside the
    pair sphere.  From a plan binned by (r_p, |pi|) with one |pi| bin over the
    sphere, each field's xi(d_p) is the pair-count correlation over its
    annulus-slab volume V_f (exact, cut by the sphere), so the projected
    correlation averaged over the annulus of area A_f is
        w_f = xi(d_p)_f V_f / A_f,
    the paper's 2 d_par,max (2 sigma_p / (n_g N_g dV_perp) - 1) with the
    thin-annulus volume replaced by the exact one; the library computes it
    (pgx_projected) and its adjoint.  Its term is
    sum_f ((w_f - target_f) / scale_f)^2.
Both plans hold the same candidate catalogue; the weights come from
``hod_weights`` and the gradients flow through ``pair_galaxy_xi``.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from ._lib import Plan
from .autograd import hod_weights, pair_galaxy_xi


class _Projected(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi_dp: torch.Tensor, plan: Plan):
        ctx.plan = plan
        return plan.projected(xi_dp.detach())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.projected_backward(g.contiguous()), None


def projected_2pcf(plan: Plan, xi_dp: torch.Tensor) -> torch.Tensor:
    """w_p per r_p annulus of an (r_p, |pi|) plan, computed by the library
    (pgx_projected), differentiable in xi_dp."""
    return _Projected.apply(xi_dp, plan)


class HodFit:
    """Loss of the HOD parameters theta = (log10 Mcut, log10 M1, sigma, alpha).

    plan_b: plan for b_pg (pairs built on the candidates); target_b: its target
    b_pg [F, R] (NaN entries ignored); mask_b (optional, bool [F, R]): the
    entries the loss uses, e.g. those whose xi_gg is well away from zero (b_pg
    divides by it).  plan_w (optional): plan with pair mode
    (r_p, |pi|), one |pi| bin, on the same candidates;
    target_w [F_w] and scale_w [F_w] (1 if None); lam weighs that term.
    """

    def __init__(self, plan_b: Plan, halo_mass: torch.Tensor, kind: torch.Tensor,
                 target_b: torch.Tensor, plan_w: Optional[Plan] = None,
                 target_w: Optional[torch.Tensor] = None, scale_w: Optional[torch.Tensor] = None,
                 lam: float = 1.0, n_candidates: int = 49,
                 mask_b: Optional[torch.Tensor] = None):
        self.plan_b, self.plan_w = plan_b, plan_w
        self.hm, self.kind = halo_mass, kind
        self.target_b = target_b
        self.mask_b = torch.isfinite(target_b)
        if mask_b is not None:
            self.mask_b = self.mask_b & mask_b
        self.lam = float(lam)
        self.n_candidates = n_candidates
        if plan_w is not None:
            self.target_w = target_w
            self.scale_w = torch.ones_like(target_w) if scale_w is None else scale_w

    def weights(self, theta: torch.Tensor) -> torch.Tensor:
        return hod_weights(theta, self.hm, self.kind, n_candidates=self.n_candidates)

    def loss(self, theta: torch.Tensor):
        """(total loss, b_pg term, w term) as float64 tensors."""
        w = self.weights(theta)
        out = pair_galaxy_xi(self.plan_b, w)
        d = out["b_pg"] - self.target_b
        m = self.mask_b & torch.isfinite(d)
        lb = (d[m] ** 2).sum()
        lw = torch.zeros((), dtype=torch.float64, device=lb.device)
        if self.plan_w is not None:
            ow = pair_galaxy_xi(self.plan_w, w)
            wp = projected_2pcf(self.plan_w, ow["xi_dp"])
            r = (wp - self.target_w) / self.scale_w
            mw = torch.isfinite(r)
            lw = (r[mw] ** 2).sum()
        return lb + self.lam * lw, lb, lw


def fit(hf: HodFit, theta0, steps: int = 50, lr: float = 0.01, callback=None, recheck_every: int = 0):
    """Adam on theta (float64) for `steps` steps; returns (theta, history of
    (total, b term, w term) per step, before each update).

    The autotuner checks the dual form's accuracy on the weights it sees; an
    HOD fit moves them.  With `recheck_every` = k > 0, after every k-th step's
    gradient each plan that runs the dual form takes that check again on the
    step's weights and falls back to the per-field transforms when it fails
    (Plan.dual_recheck)."""
    theta = torch.tensor(np.asarray(theta0, np.float64), dtype=torch.float64,
                         device=hf.target_b.device, requires_grad=True)
    opt = torch.optim.Adam([theta], lr=lr)
    hist = []
    for k in range(steps):
        opt.zero_grad()
        total, lb, lw = hf.loss(theta)
        total.backward()
        hist.append((float(total), float(lb), float(lw)))
        if callback is not None:
            callback(k, theta.detach().cpu().numpy(), hist[-1])
        if recheck_every > 0 and (k + 1) % recheck_every == 0:
            for p in (hf.plan_b, hf.plan_w):
                if p is not None:
                    p.dual_recheck(fallback=True)
        opt.step()
    return theta.detach(), hist
