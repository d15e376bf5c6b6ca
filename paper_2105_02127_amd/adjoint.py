"""Reverse-mode differentiation of an SSP-RK3 rollout of the TENO residual.

The stencil selection of every stage and the step sizes are frozen at the
values of the forward pass.  For fixed selection the reconstruction is linear
in the cell averages, so the step map is differentiable wherever the HLL flux
is, and its vector-Jacobian product is what `teno_vjp_rk_step` computes on the
device (the HLL flux differentiated in reverse mode, the reconstruction
transposed into per-tile sums formed in a fixed order and a reverse-stencil
gather; no floating-point atomics, so reruns are bit-identical).

Memory: U is checkpointed every `checkpoint_every` steps; the backward pass
recomputes one segment at a time (its stage states, flags and, unless
`keep_face_states` is off, the face states of every stage, which spares the
adjoint a reconstruction per stage) and walks it backwards.  With
`checkpoint_every=None` the forward pass keeps all of that for every step
instead, and the backward pass recomputes nothing: about
96 n_cell + 8 face_state_doubles * 3 bytes per step (2.5 + 15 GB for 200
steps of TENO4 on 131,072 cells), which one GPU's HBM holds.
"""
from __future__ import annotations

import torch

from . import teno


def forward_rollout(solver: "teno.Solver", U0: torch.Tensor, n_steps: int, cfl: float = 0.4,
                    dts: torch.Tensor | None = None, checkpoint_every: int = 20,
                    flags_out: torch.Tensor | None = None,
                    frozen_flags: torch.Tensor | None = None):
    """Advances U0 by n_steps.  dts (device float64[n_steps]) is computed with
    the constant-CFL rule when None, otherwise replayed.  flags_out (int16
    [n_steps, 3, n_cell]) receives every stage's selection; frozen_flags of
    the same shape replays a recorded selection instead.  Returns (U, dts,
    checkpoints) where checkpoints[k] is U at step k * checkpoint_every."""
    U = U0.detach().clone()
    if dts is None:
        dts = torch.empty(n_steps, dtype=torch.float64, device=U.device)
        fixed = False
    else:
        fixed = True
    ckpts = []
    for s in range(n_steps):
        if s % checkpoint_every == 0:
            ckpts.append(U.clone())
        dt = dts[s:s + 1]
        if not fixed:
            solver.max_dt(U, cfl, dt)
        if frozen_flags is not None:
            solver.rk_step(U, dt, flags3=frozen_flags[s], frozen=True)
        else:
            solver.rk_step(U, dt, flags3=None if flags_out is None else flags_out[s])
    return U, dts, ckpts


class RK3Rollout(torch.autograd.Function):
    """U_final = rollout(U0); backward gives d(loss)/d(U0) with frozen dt and
    selection."""

    @staticmethod
    def forward(ctx, U0, solver, n_steps, cfl, checkpoint_every, dts, keep_face_states=True):
        ctx.solver = solver
        ctx.n_steps = n_steps
        ctx.K = checkpoint_every
        ctx.keep = keep_face_states
        if checkpoint_every is None:
            U, dts_used, kept = _forward_keep_all(solver, U0, n_steps, cfl, dts, keep_face_states)
            ctx.kept = kept
            ctx.ckpts = None
        else:
            U, dts_used, ckpts = forward_rollout(solver, U0, n_steps, cfl, dts, checkpoint_every)
            ctx.ckpts = ckpts
        if dts is not None:
            dts_used = dts_used.clone()
        ctx.dts = dts_used
        ctx.mark_non_differentiable(dts_used)
        return U, dts_used

    @staticmethod
    def backward(ctx, grad_U, grad_dts):
        sv, n, K = ctx.solver, ctx.n_steps, ctx.K
        lam = grad_U.detach().contiguous().clone()
        if K is None:                      # everything kept: no recompute
            stages, flags, fs = ctx.kept
            for s in reversed(range(n)):
                sv.vjp_rk_step(stages[s], flags[s], ctx.dts[s:s + 1], lam, lam,
                               face_states=None if fs is None else fs[s])
            ctx.kept = None
            return lam, None, None, None, None, None, None
        nc = lam.shape[0]
        dev = lam.device
        stages = torch.empty((K, 3, nc, 4), dtype=torch.float64, device=dev)
        flags = torch.empty((K, 3, nc), dtype=torch.int16, device=dev)
        fs = sv.empty_face_states(K) if ctx.keep else None
        for seg in reversed(range(len(ctx.ckpts))):
            s0 = seg * K
            s1 = min(n, s0 + K)
            U = ctx.ckpts[seg].clone()
            for s in range(s0, s1):     # recompute the segment, keeping its stages
                sv.rk_step(U, ctx.dts[s:s + 1], flags3=flags[s - s0], stages=stages[s - s0],
                           face_states=None if fs is None else fs[s - s0])
            for s in reversed(range(s0, s1)):
                sv.vjp_rk_step(stages[s - s0], flags[s - s0], ctx.dts[s:s + 1], lam, lam,
                               face_states=None if fs is None else fs[s - s0])
        return lam, None, None, None, None, None, None


def _forward_keep_all(solver, U0, n_steps, cfl, dts, keep_face_states):
    """Forward rollout that keeps every step's stage inputs, flags and (when
    keep_face_states) face states for the backward pass."""
    U = U0.detach().clone()
    nc, dev = U.shape[0], U.device
    fixed = dts is not None
    if not fixed:
        dts = torch.empty(n_steps, dtype=torch.float64, device=dev)
    stages = torch.empty((n_steps, 3, nc, 4), dtype=torch.float64, device=dev)
    flags = torch.empty((n_steps, 3, nc), dtype=torch.int16, device=dev)
    fs = solver.empty_face_states(n_steps) if keep_face_states else None
    for s in range(n_steps):
        dt = dts[s:s + 1]
        if not fixed:
            solver.max_dt(U, cfl, dt)
        solver.rk_step(U, dt, flags3=flags[s], stages=stages[s],
                       face_states=None if fs is None else fs[s])
    return U, dts, (stages, flags, fs)


def rollout(solver, U0, n_steps, cfl=0.4, checkpoint_every=20, dts=None, keep_face_states=True):
    """Differentiable rollout: returns (U_final, dts).  keep_face_states
    trades 3 * face_state_doubles * 8 bytes per checkpointed step of device
    memory for one reconstruction per stage of the backward pass.
    checkpoint_every=None keeps every step and recomputes nothing."""
    return RK3Rollout.apply(U0, solver, n_steps, cfl, checkpoint_every, dts, keep_face_states)


def pressure_squared_loss(U, weights, gamma=1.4):
    """sum_i w_i p_i^2 with p from the conservative variables."""
    r, mx, my, e = U[:, 0], U[:, 1], U[:, 2], U[:, 3]
    p = (gamma - 1.0) * (e - 0.5 * (mx * mx + my * my) / r)
    return (weights * p * p).sum()
