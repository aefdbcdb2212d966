"""Differentiable rollouts: gradients of a final-position loss with respect to
the viscosity nu, the sound speed c0 (equation-of-state stiffness) and the
initial velocities, by the library's hand-written one-step adjoint with
checkpointed recomputation.

Every numerical step runs in the HIP library; this module only sequences the
calls and keeps checkpoints (device tensors).

Orders.  Step n reads its input state in order pi_n, sorts it (perm_n) and
writes its output in sorted order sigma_n, which is the input order of step
n + 1.  The one-step adjoint takes cotangents in sigma_n and returns them in
pi_n = sigma_(n-1), so the reverse sweep chains without any reordering.  The
first input order is the binning order, i.e. particle id order.
"""
from __future__ import annotations

import copy
from dataclasses import dataclass

import torch

from . import nauticle as N


@dataclass
class _StepRecord:
    """What the adjoint of one step needs: the sorted input state, the
    neighbour structure (lists, counts, perm) and the step's fields."""

    sorted: N.State
    cells: N.Cells
    fields: N.Fields


class Rollout:
    """n_steps of one case, differentiable in (v0, nu, c0).

    ``case`` is a workloads.Case (its nu and c0 are the defaults), ``target``
    the final cell-relative state the loss compares against (any order; it
    is matched by id)."""

    def __init__(self, case, n_steps: int, checkpoint_every: int = 20, device="cuda:0", max_nbr=None):
        self.case = case
        self.n_steps = int(n_steps)
        self.K = max(1, int(checkpoint_every))
        self.device = torch.device(device)
        self.max_nbr = max_nbr
        self._problems = {}

    # one prepared workspace per (nu, c0): the constants live in the case table
    def problem(self, nu: float, c0: float) -> N.Problem:
        key = (float(nu), float(c0))
        if key not in self._problems:
            c = copy.copy(self.case)
            c.nu, c.c0 = key
            self._problems[key] = N.Problem([c], device=self.device, max_nbr=self.max_nbr)
        return self._problems[key]

    def initial_state(self, prob: N.Problem, v0: torch.Tensor) -> N.State:
        """Binned initial positions with velocities v0 ((n, dim), id order)."""
        st = prob.state_from_cases()
        for k in range(prob.dim):
            st.vel[k].copy_(v0[:, k])
        return st

    def run(self, nu: float, c0: float, v0: torch.Tensor) -> N.State:
        prob = self.problem(nu, c0)
        st = self.initial_state(prob, v0)
        prob.step(st, self.n_steps)
        return st

    def loss(self, nu, c0, v0, target: N.State) -> float:
        prob = self.problem(nu, c0)
        st = self.run(nu, c0, v0)
        loss, _ = prob.position_loss(st, target, grad=False)
        return float(loss.item())

    def forward(self, nu: float, c0: float, v0: torch.Tensor):
        """Runs the rollout keeping a checkpoint (a copy of the state) every
        K steps; returns (final state, prepared problem, checkpoints)."""
        prob = self.problem(nu, c0)
        st = self.initial_state(prob, v0)
        ckpt = []
        for s in range(self.n_steps):
            if s % self.K == 0:
                ckpt.append((s, st.clone()))
            prob.step(st, 1)
        return st, prob, ckpt

    def vjp(self, prob: N.Problem, ckpt, lam_x, lam_v):
        """Reverse sweep from cotangents (lam_x, lam_v: per-axis device FP32,
        in the final state's order) of the final positions and velocities:
        each segment is recomputed from its checkpoint, storing every step's
        sorted state, lists and fields, then the one-step adjoints run in
        reverse.  Returns (dL/dv0 (n, dim) in id order, dL/dnu, dL/dc0)."""
        lam_x = [t.clone() for t in lam_x]
        lam_v = [t.clone() for t in lam_v]
        dnu = torch.zeros(1, dtype=torch.float64, device=self.device)
        dc0 = torch.zeros(1, dtype=torch.float64, device=self.device)
        out_x = [torch.empty_like(t) for t in lam_x]
        out_v = [torch.empty_like(t) for t in lam_x]
        for s0, st0 in reversed(ckpt):
            s1 = min(s0 + self.K, self.n_steps)
            records = []
            cur = st0.clone()
            for _ in range(s0, s1):
                rec = _StepRecord(prob.new_state(), prob.new_cells(), prob.new_fields())
                prob.build_cells(cur, rec.sorted, rec.cells)
                prob.density(rec.sorted, rec.cells, rec.fields)
                prob.forces(rec.sorted, cur, rec.cells, rec.fields)  # integrates into cur
                records.append(rec)
            for rec in reversed(records):
                prob.adjoint(rec.sorted, rec.cells, rec.fields, lam_x, lam_v, out_x, out_v, dnu, dc0)
                lam_x, out_x = out_x, lam_x
                lam_v, out_v = out_v, lam_v
        prob.check()
        gv0 = torch.stack(lam_v, dim=1)[: self.case.n]
        return gv0, float(dnu.item()), float(dc0.item())

    def loss_and_grad(self, nu: float, c0: float, v0: torch.Tensor, target: N.State):
        """(loss, dL/dv0 (n, dim) in id order, dL/dnu, dL/dc0) of the
        position loss against ``target`` (nauticle_position_loss, which also
        gives the loss's derivative in the final positions)."""
        st, prob, ckpt = self.forward(nu, c0, v0)
        loss, lam_x = prob.position_loss(st, target, grad=True)
        lam_v = [torch.zeros_like(t) for t in lam_x]
        gv0, dnu, dc0 = self.vjp(prob, ckpt, lam_x, lam_v)
        return float(loss.item()), gv0, dnu, dc0


class NauticleRollout(torch.autograd.Function):
    """r_T = NauticleRollout.apply(v0, nu, c0, rollout): the final absolute
    FP32 positions ((n, dim), particle id order) of ``rollout``'s n_steps,
    differentiable in v0 ((n, dim) float32, id order), nu and c0 (0-d
    tensors).  The forward pass keeps only the checkpoints; the backward
    pass seeds the positions' cotangent from grad_output (brought into the
    final state's order by the library), recomputes each segment and runs
    the hand-written adjoint.  Any loss built on r_T composes with it.  A
    particle that left the box across a periodic face comes back shifted by
    a box length; the shift has derivative one."""

    @staticmethod
    def forward(ctx, v0, nu, c0, rollout: Rollout):
        st, prob, ckpt = rollout.forward(float(nu), float(c0), v0.detach())
        pos = prob.unbin_by_id(st)
        ctx.rollout, ctx.prob, ctx.ckpt, ctx.final = rollout, prob, ckpt, st
        ctx.v0_dtype = v0.dtype
        ctx.nu_like = (nu.dtype, nu.device)
        ctx.c0_like = (c0.dtype, c0.device)
        return torch.stack(pos, dim=1)[: rollout.case.n]

    @staticmethod
    def backward(ctx, g):
        prob, n = ctx.prob, ctx.rollout.case.n
        g = g.to(torch.float32)
        gk = []
        for k in range(prob.dim):
            t = torch.zeros(max(prob.n, 1), dtype=torch.float32, device=prob.device)
            t[:n] = g[:, k]
            gk.append(t)
        lam_x = prob.gather_by_id(ctx.final, gk)
        lam_v = [torch.zeros_like(t) for t in lam_x]
        gv0, dnu, dc0 = ctx.rollout.vjp(prob, ctx.ckpt, lam_x, lam_v)
        return (gv0.to(ctx.v0_dtype), torch.tensor(dnu, dtype=ctx.nu_like[0], device=ctx.nu_like[1]),
                torch.tensor(dc0, dtype=ctx.c0_like[0], device=ctx.c0_like[1]), None)
