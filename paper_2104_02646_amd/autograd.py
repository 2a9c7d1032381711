"""Differentiable rollout as a torch.autograd.Function.

The paper wraps each simulation kernel as a PyTorch autograd operation and lets
the tape carry the program flow (App. A; App. C).  Here the whole T-step rollout
is one operation: the forward runs ``gsim_rollout`` (storing a checkpoint every K
steps in a buffer owned by this call), the backward runs the checkpointed
adjoint ``gsim_rollout_backward`` (recompute each K-step segment, then its
adjoint steps), so a long rollout's gradient needs only ceil(T/K) saved states.
Both passes are HIP kernels in libgsim; this module only moves tensors.
"""
from __future__ import annotations

import torch

from . import gsim

_PARAM_KEYS = ("mu", "lam", "ktri", "mass", "contact", "act", "hact")
_INPUT_KEYS = ("air",)  # inputs without a gradient


class SimRollout(torch.autograd.Function):
    """(x0, v0, mu, lam, ktri, mass, contact, act, hact) -> (xT, vT) after n_steps steps.

    States are SoA [3, n_particles]; contact is [n_bodies, 4] = (k_e, k_d, k_f, mu_f);
    act / hact (tet / hinge actuation) are [n] for one value over the whole rollout
    or [n_steps, n] for a value per step, and their gradients have the same shape;
    air [n_bodies, 2] = (k_drag, k_lift) of bodies with lift/drag is an input
    without a gradient.  Pass None for parameters the model does not have
    (mu/lam without tets, ktri without triangles) or does not actuate."""

    @staticmethod
    def forward(ctx, model, n_steps, x0, v0, mu, lam, ktri, mass, contact, act, hact, air):
        vals = (mu, lam, ktri, mass, contact, act, hact)
        params = {k: v.detach().contiguous() for k, v in zip(_PARAM_KEYS, vals) if v is not None}
        if air is not None:
            params["air"] = air.detach().contiguous()
        ckpt = model.new_checkpoints()
        xT, vT = model.rollout(params, x0.detach().contiguous(), v0.detach().contiguous(), int(n_steps), ckpt=ckpt)
        ctx.model, ctx.n_steps, ctx.params, ctx.ckpt = model, int(n_steps), params, ckpt
        ctx.present = tuple(v is not None for v in vals)
        return xT, vT

    @staticmethod
    def backward(ctx, gx, gv):
        m = ctx.model
        gx = torch.zeros(3, m.np, dtype=m.dtype, device=m.device) if gx is None else gx.contiguous()
        gv = torch.zeros(3, m.np, dtype=m.dtype, device=m.device) if gv is None else gv.contiguous()
        grads = {k: torch.zeros_like(ctx.params[k]) for k, p in zip(_PARAM_KEYS, ctx.present) if p}
        xb0, vb0 = m.rollout_backward(ctx.params, ctx.n_steps, gx, gv, grads, ckpt=ctx.ckpt)
        out = [grads.get(k) if p else None for k, p in zip(_PARAM_KEYS, ctx.present)]
        return (None, None, xb0, vb0, *out, None)


def rollout(model, params, x0, v0, n_steps):
    """Differentiable rollout: params is a dict of (possibly requires_grad) tensors."""
    return SimRollout.apply(model, n_steps, x0, v0, *(params.get(k) for k in _PARAM_KEYS + _INPUT_KEYS))


class Controller(torch.autograd.Function):
    """W [n_signals, n] -> act [n_steps, n], the open-loop actuation controller
    (sinusoids of the simulation time -> bias-free linear layer -> tanh; App. "MPC
    controller architecture").  Forward and backward are the HIP kernels behind
    ``gsim_controller_forward`` / ``gsim_controller_backward``; feed the result to
    ``rollout`` as per-step ``act`` (or ``hact``) rows."""

    @staticmethod
    def forward(ctx, W, omega, dt, n_steps, t0, scale):
        W = W.detach().contiguous()
        ctx.save_for_backward(W)
        ctx.args = (float(omega), float(dt), int(t0), float(scale))
        return gsim.controller_forward(W, omega, dt, int(n_steps), t0=int(t0), scale=scale)

    @staticmethod
    def backward(ctx, g):
        (W,) = ctx.saved_tensors
        omega, dt, t0, scale = ctx.args
        gW = gsim.controller_backward(W, g.contiguous(), omega, dt, t0=t0, scale=scale)
        return gW, None, None, None, None, None


def controller(W, omega, dt, n_steps, t0=0, scale=1.0):
    """Differentiable per-step actuation rows from controller weights W."""
    return Controller.apply(W, omega, dt, n_steps, t0, scale)


class RigidRollout(torch.autograd.Function):
    """(s0 [nb, 13], mass [nb], inertia [nb, 6], contact [nb, 4]) -> final state after
    n_steps rigid-body steps (App. A.1 "Rigid bodies"); the forward stores every
    state (13 numbers per body per step) and the backward is the reverse-pass kernel
    over them."""

    @staticmethod
    def forward(ctx, model, n_steps, s0, mass, inertia, contact):
        params = {"mass": mass.detach().contiguous(), "inertia": inertia.detach().contiguous(),
                  "contact": contact.detach().contiguous()}
        traj = model.rollout(params, s0.detach().contiguous(), int(n_steps))
        ctx.model, ctx.n_steps, ctx.params, ctx.traj = model, int(n_steps), params, traj
        return traj[-1].clone()

    @staticmethod
    def backward(ctx, g):
        m = ctx.model
        grads = m.zero_grads()
        s0b = m.rollout_backward(ctx.params, ctx.traj, ctx.n_steps, g.contiguous(), grads)
        return None, None, s0b, grads["mass"], grads["inertia"], grads["contact"]


def rigid_rollout(model, params, s0, n_steps):
    """Differentiable rigid rollout: params = {mass, inertia, contact} tensors."""
    return RigidRollout.apply(model, n_steps, s0, params["mass"], params["inertia"], params["contact"])


class SoftSilhouette(torch.autograd.Function):
    """x [3, n_verts] (SoA positions) -> soft silhouette image [H, W] through the
    renderer's mesh and a 3x4 camera matrix P (the paper's pixel losses; SoftRas
    silhouette).  Forward and backward are the renderer's HIP kernels."""

    @staticmethod
    def forward(ctx, renderer, P, sigma, x):
        x = x.detach().contiguous()
        ctx.save_for_backward(x)
        ctx.renderer, ctx.P, ctx.sigma = renderer, P, sigma
        return renderer.forward(x, P, sigma)

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        return None, None, None, ctx.renderer.backward(x, ctx.P, ctx.sigma, g.contiguous())


def render(renderer, x, P, sigma):
    """Differentiable soft silhouette of positions x [3, n_verts]."""
    return SoftSilhouette.apply(renderer, P, sigma, x)
