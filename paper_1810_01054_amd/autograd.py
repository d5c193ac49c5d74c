"""torch.autograd wrappers over whole rollouts (the paper's memo-based
gradient evaluation, here a library-owned tape with checkpoint + recompute).

``rollout(sim, state0, act, T, ckpt_k)`` returns the final state; its
backward runs ``mpm_rollout_backward`` over the tape of that same rollout.
``rollout_ctrl`` is the closed-loop form (actuation from a tanh layer over
the component means of the state, mpm_rollout_ctrl); ``rollout_materials``
also differentiates a per-particle material field (mpm_set_materials).
A context keeps one tape, so a second rollout (or a set_materials call) on
the same simulator makes the first one's backward raise instead of
returning wrong gradients: each forward records the library's tape
generation (mpm_tape_generation) and the backward compares it.

Device-side errors (a particle left the grid, det F <= 0, a non-finite
value) are sticky in the context and reported by the next synchronising
call.  With ``check_errors=True`` the wrappers synchronise after the
rollout and after its reverse pass and raise such an error at once (this
costs the host/device overlap of one synchronisation per call).
"""
from __future__ import annotations

from typing import Optional

import torch

from .sim import Simulator, act_bank_backward, act_bank_forward


def _record(ctx, sim: Simulator, T: int, check_errors: bool):
    if check_errors:
        sim.sync_errors()
    ctx.sim, ctx.T, ctx.gen, ctx.check = sim, T, sim.tape_generation(), check_errors


def _seed_adjoint(ctx, gx, gv, gC, gF):
    sim = ctx.sim
    if sim.tape_generation() != ctx.gen:
        raise RuntimeError("the simulator ran another rollout (or changed its material "
                           "field) since this one; its tape is gone (use one Simulator "
                           "per live graph)")
    ref = sim.empty_state()
    return tuple(torch.zeros_like(r) if t is None else t.contiguous()
                 for t, r in zip((gx, gv, gC, gF), ref))


class MPMRolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim: Simulator, T: int, ckpt_k: int, check_errors: bool,
                x0, v0, C0, F0, act):
        sT = sim.rollout(tuple(t.contiguous() for t in (x0, v0, C0, F0)),
                         act.contiguous() if act is not None else None, T, ckpt_k)
        _record(ctx, sim, T, check_errors)
        ctx.has_act = act is not None
        return sT

    @staticmethod
    def backward(ctx, gx, gv, gC, gF):
        g = _seed_adjoint(ctx, gx, gv, gC, gF)
        g0, g_act = ctx.sim.rollout_backward(g, ctx.T)
        if ctx.check:
            ctx.sim.sync_errors()
        return (None, None, None, None, *g0, g_act if ctx.has_act else None)


class MPMRolloutCtrlFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim: Simulator, T: int, ckpt_k: int, check_errors: bool, comp_id,
                n_comp: int, x0, v0, C0, F0, W, b, target):
        sT, act = sim.rollout_ctrl(tuple(t.contiguous() for t in (x0, v0, C0, F0)), T,
                                   comp_id, n_comp, W.contiguous(), b.contiguous(),
                                   target.contiguous(), ckpt_k)
        _record(ctx, sim, T, check_errors)
        ctx.nz = W.shape[1]
        ctx.mark_non_differentiable(act)
        return (*sT, act)

    @staticmethod
    def backward(ctx, gx, gv, gC, gF, _gact):
        g = _seed_adjoint(ctx, gx, gv, gC, gF)
        g0, _, g_W, g_b = ctx.sim.rollout_ctrl_backward(g, ctx.T, ctx.nz)
        if ctx.check:
            ctx.sim.sync_errors()
        return (None, None, None, None, None, None, *g0, g_W, g_b, None)


class MPMRolloutMatFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim: Simulator, T: int, ckpt_k: int, check_errors: bool,
                x0, v0, C0, F0, act, E_p, rho_p):
        sim.set_materials(E_p.contiguous(), rho_p.contiguous())
        sT = sim.rollout(tuple(t.contiguous() for t in (x0, v0, C0, F0)),
                         act.contiguous() if act is not None else None, T, ckpt_k)
        _record(ctx, sim, T, check_errors)
        ctx.has_act = act is not None
        return sT

    @staticmethod
    def backward(ctx, gx, gv, gC, gF):
        g = _seed_adjoint(ctx, gx, gv, gC, gF)
        g0, g_act = ctx.sim.rollout_backward(g, ctx.T)
        g_E, g_rho = ctx.sim.material_grad()
        if ctx.check:
            ctx.sim.sync_errors()
        return (None, None, None, None, *g0, g_act if ctx.has_act else None, g_E, g_rho)


class ActBankFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T: int, dt: float, freq, amp, phase):
        ctx.save_for_backward(freq, amp, phase)
        ctx.T, ctx.dt = T, dt
        return act_bank_forward(T, dt, freq.contiguous(), amp.contiguous(),
                                phase.contiguous())

    @staticmethod
    def backward(ctx, g_act):
        freq, amp, phase = ctx.saved_tensors
        ga, gp = act_bank_backward(ctx.T, ctx.dt, freq, amp, phase, g_act.contiguous())
        return None, None, None, ga, gp


def rollout(sim: Simulator, state0, act: Optional[torch.Tensor], T: int,
            ckpt_k: int = 32, check_errors: bool = False):
    """Differentiable T-substep rollout: returns (xT, vT, CT, FT)."""
    x0, v0, C0, F0 = state0
    return MPMRolloutFn.apply(sim, T, ckpt_k, check_errors, x0, v0, C0, F0, act)


def rollout_ctrl(sim: Simulator, state0, T: int, comp_id, n_comp: int, W, b, target,
                 ckpt_k: int = 32, check_errors: bool = False):
    """Differentiable closed-loop rollout a^n = tanh(W z^n + b): returns
    (xT, vT, CT, FT, act) with gradients to the initial state, W and b
    (act, the controller's output, carries none)."""
    x0, v0, C0, F0 = state0
    return MPMRolloutCtrlFn.apply(sim, T, ckpt_k, check_errors, comp_id, n_comp,
                                  x0, v0, C0, F0, W, b, target)


def rollout_materials(sim: Simulator, state0, act: Optional[torch.Tensor], T: int,
                      E_p, rho_p, ckpt_k: int = 32, check_errors: bool = False):
    """Differentiable rollout over a per-particle material field (E_p,
    rho_p [N]): returns (xT, vT, CT, FT) with gradients to the initial
    state, the actuation, E_p and rho_p (system identification, co-design)."""
    x0, v0, C0, F0 = state0
    return MPMRolloutMatFn.apply(sim, T, ckpt_k, check_errors, x0, v0, C0, F0, act,
                                 E_p, rho_p)


def act_bank(T: int, dt: float, freq, amp, phase):
    """Differentiable sinusoid actuation schedule act[T][n_act]."""
    return ActBankFn.apply(T, dt, freq, amp, phase)
