"""torch.autograd.Function wrappers over the library's hand-written adjoints.

LatCombo:    Y = ROM apply of X (eq. romstiffnessmatrix) on the packed layout, with gradients
             with respect to X and to the per-cell Lame parameters (mu, lam); the principal set
             is frozen (the arg-max of the greedy is piecewise constant).
LatResidual: r = sum_s A^s f^{int,s}(u^s) (eq. residualvector, eq. internalloadvec), with
             gradients with respect to u and (mu, lam); the tangent used in the reverse pass is
             the exact Jacobian of the residual.
Both forward and backward run entirely in liblat kernels; torch only routes tensors.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import binding as B


@dataclasses.dataclass
class RomState:
    """The ROM operator at one displacement: principal stacks, coefficients, greedy outputs."""
    plan: B.Plan
    K: torch.Tensor
    S: torch.Tensor
    n_r: int
    alpha: torch.Tensor
    K_mu: Optional[torch.Tensor] = None
    K_lam: Optional[torch.Tensor] = None
    delta: Optional[torch.Tensor] = None      # greedy residuals (snapshot matrix after selection)
    Z: Optional[torch.Tensor] = None
    R: Optional[torch.Tensor] = None
    nu: Optional[torch.Tensor] = None
    snap_mu: Optional[torch.Tensor] = None
    snap_lam: Optional[torch.Tensor] = None
    # what the state was built from (LatCombo rebuilds it for other Lame parameters)
    u_global: Optional[torch.Tensor] = None
    mu: Optional[torch.Tensor] = None
    lam: Optional[torch.Tensor] = None
    tol: float = 0.0
    cap: Optional[int] = None
    snap_rule: int = B.RULE_FULL
    # precision of the combination in the forward and transposed applies (lat_apply_combo's prec)
    prec: int = B.F64
    refine_tol: float = 1e-6


def build_rom_state(plan: B.Plan, u_global, mu, lam, tol, cap=None, for_adjoint=True, snap_rule=B.RULE_FULL,
                    prec=B.F64, refine_tol=1e-6):
    """Snapshots -> greedy -> alpha -> principal operators (and, for the adjoint, the Lame parts)."""
    r = plan.residual_tangent(u_global, mu, lam, snap_rule=snap_rule, f=False, energy=False, snap=True)
    g = plan.select_principal(r["snap"], tol, cap=cap, keep_Z=for_adjoint)
    n_r = int(g["n_r"].item())
    ops = plan.principal_ops(u_global, mu, lam, g["S"], n_r, parts=for_adjoint)
    st = RomState(plan=plan, K=ops["K"], S=g["S"], n_r=n_r, alpha=g["alpha"], u_global=u_global,
                  mu=mu.detach().clone(), lam=lam.detach().clone(), tol=tol, cap=cap, snap_rule=snap_rule, prec=prec,
                  refine_tol=refine_tol)
    if for_adjoint:
        ones = torch.ones_like(mu)
        zeros = torch.zeros_like(mu)
        sm = plan.residual_tangent(u_global, ones, zeros, snap_rule=snap_rule, f=False, energy=False)["snap"]
        sl = plan.residual_tangent(u_global, zeros, ones, snap_rule=snap_rule, f=False, energy=False)["snap"]
        st.K_mu, st.K_lam = ops["K_mu"], ops["K_lam"]
        st.delta, st.Z, st.R, st.nu = r["snap"], g["Z"], g["R"], g["nu"]
        st.snap_mu, st.snap_lam = sm, sl
    return st


class LatCombo(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, mu, lam, state: RomState, m: int):
        if state.mu is None or not (torch.equal(mu, state.mu) and torch.equal(lam, state.lam)):
            # the operator depends on (mu, lam): a state built for other values is rebuilt at these
            if state.u_global is None:
                raise RuntimeError("RomState does not record its displacement; build it with build_rom_state")
            state = build_rom_state(state.plan, state.u_global, mu.detach(), lam.detach(), state.tol, state.cap,
                                    for_adjoint=state.K_mu is not None, snap_rule=state.snap_rule, prec=state.prec,
                                    refine_tol=state.refine_tol)
        ctx.state, ctx.m = state, m
        ctx.save_for_backward(X)
        return state.plan.apply_combo(state.K, state.n_r, state.alpha, X.contiguous(), m, prec=state.prec,
                                      refine_tol=state.refine_tol)

    @staticmethod
    def backward(ctx, Ybar):
        st, m = ctx.state, ctx.m
        (X,) = ctx.saved_tensors
        P = st.plan
        want_lame = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        if want_lame and st.K_mu is None:
            raise RuntimeError("RomState was built without adjoint data (for_adjoint=False)")
        r = P.apply_combo_adjoint(st.K, st.n_r, st.alpha, X.contiguous(), Ybar.contiguous(), m,
                                  K_mu=st.K_mu if want_lame else None, K_lam=st.K_lam if want_lame else None,
                                  S=st.S, want_xbar=ctx.needs_input_grad[0], want_alpha_bar=want_lame, prec=st.prec,
                                  refine_tol=st.refine_tol)
        mu_bar = lam_bar = None
        if want_lame:
            mu_bar, lam_bar = r["mu_bar"], r["lam_bar"]
            P.alpha_adjoint(st.delta, st.Z, st.R, st.nu, st.S, st.n_r, st.alpha, r["alpha_bar"], st.snap_mu,
                            st.snap_lam, mu_bar, lam_bar)
        return r["Xbar"], mu_bar, lam_bar, None, None


class LatResidual(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u_global, mu, lam, plan: B.Plan):
        ctx.plan = plan
        ctx.save_for_backward(u_global, mu, lam)
        f = plan.residual_tangent(u_global.contiguous(), mu.contiguous(), lam.contiguous(), f=True, energy=False,
                                  snap=False)["f"]
        return plan.assemble(f, plan.dim)[: plan.nglobal * plan.dim].view(plan.nglobal, plan.dim)

    @staticmethod
    def backward(ctx, rbar):
        P = ctx.plan
        u, mu, lam = ctx.saved_tensors
        w = P.gather(rbar.contiguous(), P.dim)
        r = P.residual_adjoint(u, mu, lam, w, local=True, glob=True, lame=True)
        ub = r["ubar_global"][: P.nglobal * P.dim].view(P.nglobal, P.dim)
        return ub, r["mu_bar"], r["lam_bar"], None


def rom_apply(X, mu, lam, state: RomState, m: int):
    return LatCombo.apply(X, mu, lam, state, m)


def residual(u_global, mu, lam, plan: B.Plan):
    return LatResidual.apply(u_global, mu, lam, plan)
