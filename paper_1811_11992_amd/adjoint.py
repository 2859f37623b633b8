"""Differentiation form: cumulative oil production as a torch.autograd.Function.

J_obj(ln k, ln A) = sum_n dt_n q_oil(u^n) over the implicit steps of a run.
A step whose Newton iteration fails is retried with half the step size (at
most four times), and the step sizes that succeeded are recorded: they are
the step sequence the objective and its gradient refer to.  The forward pass
keeps the state only every ``checkpoint_every`` steps; the backward pass
walks the segments in reverse, recomputes each segment's states from its
checkpoint with the recorded step sizes (the kernels are bitwise
deterministic, so the recomputed states are the forward states) and runs
``isc_adjoint`` step by step.
"""
from __future__ import annotations

import math

import torch

from . import isc


def _solve_step(ctx: isc.Context, u: torch.Tensor, dt: float, tol: float, max_newton: int, lin):
    """One implicit step from u (returned new tensor) in parity mode: Newton
    to tol, then one extra iteration so that the state sits at the root to
    rounding.  A failure raises (the caller may retry a shorter step)."""
    u_old = u
    u = u.clone()
    for _ in range(max_newton + 1):
        st, info = ctx.isc_newton_step(u, u_old, dt, tol, lin)
        if st != isc.ISC_OK:
            raise isc.IscError(st, "Newton step failed in the differentiation form")
        if info.converged:
            st, info = ctx.isc_newton_step(u, u_old, dt, 0.0, lin)
            if st != isc.ISC_OK:
                raise isc.IscError(st, "extra Newton iteration failed")
            return u
    raise isc.IscError(isc.ISC_ERR_NEWTON_NOCONV, f"no convergence in {max_newton} Newton iterations")


_RETRYABLE = (isc.ISC_ERR_NEWTON_NOCONV, isc.ISC_ERR_LINEAR_NOCONV, isc.ISC_ERR_NONFINITE, isc.ISC_ERR_SINGULAR)


def _step_with_cuts(ctx: isc.Context, u: torch.Tensor, dt: float, tol: float, lin, max_cuts: int = 4):
    """An implicit step of at most dt: the step is halved after a failure, at
    most max_cuts times.  Returns (new state, step size used)."""
    for cut in range(max_cuts + 1):
        try:
            return _solve_step(ctx, u, dt, tol, 12, lin), dt
        except isc.IscError as e:
            if cut == max_cuts or e.status not in _RETRYABLE:
                raise
            dt *= 0.5
    raise AssertionError("unreachable")


class OilProduction(torch.autograd.Function):
    """J = OilProduction.apply(logk, lnA, ctx, u0, dt, nsteps[, checkpoint_every, tol, progress, lin]);
    progress (optional) is called with a short text after every step of each pass; lin
    (optional, FP64) are the linear-solver options of the forward steps (default
    BILU(0)-GMRES(30) to 1e-8)."""

    @staticmethod
    def forward(fctx, logk, lnA, ctx: isc.Context, u0, dt: float, nsteps: int, checkpoint_every: int = 5,
                tol: float = 1e-10, progress=None, lin=None):
        A = torch.exp(lnA.detach().double()).cpu().tolist()
        ctx.isc_set_params(logk=logk.detach().double().contiguous(), A=A)
        lin = lin if lin is not None else isc.solve_opts()
        u = u0.detach().double().contiguous().clone()
        ckpt = {0: u.clone()}
        J = 0.0
        dts = []
        for n in range(1, nsteps + 1):
            u, dt_n = _step_with_cuts(ctx, u, dt, tol, lin)
            dts.append(dt_n)
            J += dt_n * ctx.isc_oil_rate(u)
            if progress:
                progress(f"forward step {n} (dt {dt_n:g} s)")
            if n % checkpoint_every == 0 and n < nsteps:
                ckpt[n] = u.clone()
        fctx.isc_ctx, fctx.dts, fctx.nsteps, fctx.tol, fctx.A = ctx, dts, nsteps, tol, A
        fctx.progress = progress
        fctx.lin = lin
        fctx.ckpt = ckpt
        fctx.logk = logk.detach().double().contiguous()
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(fctx, gJ):
        ctx: isc.Context = fctx.isc_ctx
        dts, nsteps, tol = fctx.dts, fctx.nsteps, fctx.tol
        ctx.isc_set_params(logk=fctx.logk, A=fctx.A)
        lin = fctx.lin
        n8 = (ctx.n, 8)
        g_logk = torch.zeros(ctx.n, dtype=torch.float64, device=ctx.device)
        g_A = [0.0] * 4
        lam_next = None
        lam = torch.empty(n8, dtype=torch.float64, device=ctx.device)
        starts = sorted(fctx.ckpt)
        for s0 in reversed(starts):
            s1 = min(nsteps, next((s for s in starts if s > s0), nsteps))
            states = [fctx.ckpt[s0]]
            for k in range(s0, s1):
                states.append(_solve_step(ctx, states[-1], dts[k], tol, 12, lin))
                if fctx.progress:
                    fctx.progress(f"recomputed step {k + 1}")
            for n in range(s1, s0, -1):
                lam_n = torch.empty(n8, dtype=torch.float64, device=ctx.device)
                dt_next = dts[n] if n < nsteps else dts[n - 1]   # ignored at the last step (no lam_next)
                g_A, _ = ctx.isc_adjoint(states[n - s0], states[n - 1 - s0], dts[n - 1], lam_next, dt_next, lam_n,
                                         g_logk, g_A)
                lam_next = lam_n
                if fctx.progress:
                    fctx.progress(f"adjoint step {n}")
        del lam
        g = float(gJ)
        grad_logk = (g * g_logk).to(fctx.logk.dtype)
        grad_lnA = torch.tensor([g * ga * a for ga, a in zip(g_A, fctx.A)], dtype=torch.float64)
        return grad_logk, grad_lnA, None, None, None, None, None, None, None, None


def cumulative_oil(ctx: isc.Context, logk, lnA, u0, dt, nsteps, checkpoint_every=5, tol=1e-10):
    return OilProduction.apply(logk, lnA, ctx, u0, dt, nsteps, checkpoint_every, tol)


def log_frequency_factors(fluid) -> torch.Tensor:
    return torch.tensor([math.log(a) for a in fluid.Afreq[:]], dtype=torch.float64)
