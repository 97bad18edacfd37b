"""Differentiable rollouts: the HIP step and step-adjoint wrapped in a torch.autograd.Function.

The forward pass advances the state with `sph_step`, keeping only a checkpoint of the state
every K steps (the paper's gradient checkpointing, Sec. 3: only particle data are retained,
intermediate pair quantities are recomputed).  A one-step rollout and the summation density
hand their backward the sort and neighbour lists that their forward built (retained in the
plan's workspace, reused while nothing has overwritten them), as the paper's backward reuses
the forward's adjacency.  The backward pass is `sph_rollout_backward`:
segment by segment in reverse, it recomputes the segment from its checkpoint (keeping each
step's sorted state and neighbour lists in the plan's tape) and applies the one-step
vector-Jacobian product (Sec. 2.2) to every step in reverse.  The plan's tape_depth must be
at least K.
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

import torch

from .lib import FLAG_NONFINITE, Plan, SphError

ERR_CAPACITY, ERR_NONFINITE = -3, -4


def check_status(plan: Plan, what: str) -> None:
    """Read (and clear) the plan's device status words; raise SphError if any simulation reports
    a non-finite value, a neighbour-list overflow or a particle that outran its list skin.
    Synchronises the stream."""
    st = plan.poll()
    bad = [(k, int(w)) for k, w in enumerate(st) if w]
    if bad:
        code = ERR_NONFINITE if any(w & FLAG_NONFINITE for _, w in bad) else ERR_CAPACITY
        raise SphError(code, "%s: device status of (simulation, flags): %s" % (what, bad[:8]))


class SPHRollout(torch.autograd.Function):
    """(x0, v0, rho0) -> (x_T, v_T, rho_T) after `nsteps` steps of the plan's simulations."""

    @staticmethod
    def forward(ctx, x0: torch.Tensor, v0: torch.Tensor, rho0: torch.Tensor, plan: Plan, nsteps: int,
                ckpt_every: int, check: bool = True):
        K = max(1, int(ckpt_every))
        nseg = math.ceil(nsteps / K) if nsteps > 0 else 0
        x, v, rho = x0.detach().clone(), v0.detach().clone(), rho0.detach().clone()
        ckpts = [plan.empty_state() for _ in range(nseg)]
        ctx.retained = (-1, 0)
        if nsteps > 0:
            plan.step(x, v, rho, nsteps, ckpts, K)
            if nsteps == 1:
                # the sort and lists of the initial state, reused by the backward while they last
                ctx.retained = plan.retained_lists()
            if check:
                check_status(plan, "rollout forward")
        ctx.plan, ctx.nsteps, ctx.K, ctx.nseg, ctx.check = plan, int(nsteps), K, nseg, bool(check)
        flat = [t for c in ckpts for t in c]
        ctx.save_for_backward(*flat)
        return x, v, rho

    @staticmethod
    def backward(ctx, gx: Optional[torch.Tensor], gv: Optional[torch.Tensor], grho: Optional[torch.Tensor]):
        plan: Plan = ctx.plan
        flat = ctx.saved_tensors
        ckpts = [tuple(flat[3 * k:3 * k + 3]) for k in range(ctx.nseg)]
        ref = plan.empty_state()
        cx = gx.detach().clone().contiguous() if gx is not None else torch.zeros_like(ref[0])
        cv = gv.detach().clone().contiguous() if gv is not None else torch.zeros_like(ref[1])
        cr = grho.detach().clone().contiguous() if grho is not None else torch.zeros_like(ref[2])
        if ctx.nsteps == 1 and ctx.retained[0] >= 0:
            # one step: its adjoint on the forward's retained lists (a plain step adjoint if they
            # have been overwritten since)
            plan.step_adjoint(*ckpts[0], cx, cv, cr, retained=ctx.retained)
            if ctx.check:
                check_status(plan, "rollout backward")
        elif ctx.nsteps > 0:
            plan.rollout_backward(ckpts, ctx.nsteps, ctx.K, cx, cv, cr)
            if ctx.check:
                check_status(plan, "rollout backward")
        return cx, cv, cr, None, None, None, None


def rollout(plan: Plan, x0, v0, rho0, nsteps: int, ckpt_every: int = 8, check: bool = True) -> Tuple[torch.Tensor, ...]:
    """Differentiable T-step rollout of all simulations of `plan`.  With `check` (default) the
    forward and the backward each end by reading the device status words and raise SphError if a
    simulation went non-finite, overflowed its neighbour lists or outran its list skin (a
    synchronisation each); check=False leaves the status words for the caller's own poll()."""
    return SPHRollout.apply(x0, v0, rho0, plan, nsteps, ckpt_every, check)


class SPHDensitySum(torch.autograd.Function):
    """(x, v, rho) -> summation density rho_i = sum_j m W_ij (Sec. 2.3); differentiable in x
    through `sph_density_adjoint` (the density depends on nothing else)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, v: torch.Tensor, rho: torch.Tensor, plan: Plan):
        xs, vs, rs = x.detach().contiguous(), v.detach().contiguous(), rho.detach().contiguous()
        _, _, rho_sum = plan.rhs(xs, vs, rs, rho_sum=True)
        ctx.plan = plan
        ctx.retained = plan.retained_lists()  # the lists of this state, reused by the backward
        ctx.save_for_backward(xs, vs, rs)
        return rho_sum

    @staticmethod
    def backward(ctx, g: Optional[torch.Tensor]):
        xs, vs, rs = ctx.saved_tensors
        if g is None:
            return None, None, None, None
        return ctx.plan.density_adjoint(xs, vs, rs, g.detach().contiguous(), retained=ctx.retained), None, None, None


def density_sum(plan: Plan, x, v, rho) -> torch.Tensor:
    """Differentiable summation density of all simulations of `plan` (original order)."""
    return SPHDensitySum.apply(x, v, rho, plan)


class SPHShift(torch.autograd.Function):
    """(x, v, rho) -> (x + dr, v, rho): particle shifting as a differentiable post-processing step
    (`sph_shift` / `sph_shift_adjoint`)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, v: torch.Tensor, rho: torch.Tensor, plan: Plan, beta: float):
        xs = x.detach().clone()
        plan.shift(xs, v.detach(), rho.detach(), beta)
        ctx.plan, ctx.beta = plan, float(beta)
        ctx.save_for_backward(x.detach(), v.detach(), rho.detach())
        return xs, v.detach().clone(), rho.detach().clone()

    @staticmethod
    def backward(ctx, gx, gv, grho):
        x, v, rho = ctx.saved_tensors
        cx = gx.detach().clone().contiguous() if gx is not None else torch.zeros_like(x)
        cv = gv.detach().clone().contiguous() if gv is not None else torch.zeros_like(v)
        cr = grho.detach().clone().contiguous() if grho is not None else torch.zeros_like(rho)
        ctx.plan.shift_adjoint(x, v, rho, cx, cv, cr, ctx.beta)
        return cx, cv, cr, None, None


def shift(plan: Plan, x, v, rho, beta: float) -> Tuple[torch.Tensor, ...]:
    """Differentiable particle shift of all simulations of `plan`."""
    return SPHShift.apply(x, v, rho, plan, beta)
