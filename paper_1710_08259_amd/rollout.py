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


_ALIGN_WORDS = 64  # each array of a record starts on a 256-byte boundary


def _record_arrays(prob: N.Problem):
    """The (name, words) of one step's record, in the order they are laid
    out: the sorted state, the cell table with its neighbour lists, the
    fields."""
    n = max(prob.n, 1)
    nc = max(prob.n_cells, 1)
    cont = prob.model == N.MODEL_CONTINUITY
    d = prob.dim
    out = [("cell", n)] + [("off", n)] * d + [("vel", n)] * d + [("id", n)] + ([("rho", n)] if cont else [])
    out += [("key", n), ("perm", n), ("cell_start", nc), ("cell_end", nc), ("nbr", prob.max_nbr * n),
            ("nbr_count", n)]
    out += [("f_rho", n), ("f_p", n), ("f_s", n), ("f_inv_rho", n)] + [("f_acc", n)] * d
    out += [("f_drho", n)] if cont else []
    return out


def _padded(words: int) -> int:
    return (words + _ALIGN_WORDS - 1) // _ALIGN_WORDS * _ALIGN_WORDS


def record_bytes(prob: N.Problem) -> int:
    """Device bytes of one step's record: the sorted state, the cell table
    with its neighbour lists, and the fields."""
    return 4 * sum(_padded(w) for _, w in _record_arrays(prob))


def _alloc_records(prob: N.Problem, count: int) -> list:
    """`count` step records carved out of one device allocation."""
    layout = _record_arrays(prob)
    words = sum(_padded(w) for _, w in layout)
    buf = torch.empty(count * words, dtype=torch.int32, device=prob.device)
    n = max(prob.n, 1)
    recs = []
    for r in range(count):
        at = r * words
        arrays = {}
        for name, w in layout:
            t = buf[at: at + w]
            at += _padded(w)
            arrays.setdefault(name, []).append(t)
        f = lambda name: [t.view(torch.float32) for t in arrays.get(name, [])]
        one = lambda name, flt=False: (f(name)[0] if flt else arrays[name][0]) if name in arrays else None
        st = N.State(one("cell"), f("off"), f("vel"), one("id"), one("rho", True))
        cells = N.Cells(one("key"), one("perm"), one("cell_start"), one("cell_end"),
                        one("nbr").view(N._list_shape(prob.max_nbr, n)), one("nbr_count"), prob.max_nbr)
        fields = N.Fields(one("f_rho", True), one("f_p", True), one("f_s", True), one("f_inv_rho", True), f("f_acc"),
                          one("f_drho", True))
        recs.append(_StepRecord(st, cells, fields))
    return recs


class _Records(list):
    """Every step's record, kept by the forward pass."""


class _Checkpoints(list):
    """(step, state) every K steps; the reverse sweep recomputes the rest."""


class Rollout:
    """n_steps of one case, differentiable in (v0, nu, c0).

    ``case`` is a workloads.Case (its nu and c0 are the defaults), ``target``
    the final cell-relative state the loss compares against (any order; it
    is matched by id).

    ``keep_records``: True keeps every step's record (sorted state, lists,
    fields) from the forward pass, so the reverse sweep runs the adjoint
    passes only; False keeps a checkpoint every ``checkpoint_every`` steps
    and recomputes each segment's records before its sweep (one more
    forward in all, in the memory of one segment).  None (the default)
    keeps the records when all of them take at most half the device memory
    free at the forward pass.  Both give bitwise the same results."""

    def __init__(self, case, n_steps: int, checkpoint_every: int = 20, device="cuda:0", max_nbr=None,
                 keep_records=None):
        self.case = case
        self.n_steps = int(n_steps)
        self.K = max(1, int(checkpoint_every))
        self.device = torch.device(device)
        self.max_nbr = max_nbr
        self.keep_records = keep_records
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

    def keeps_records(self, prob: N.Problem) -> bool:
        if self.keep_records is not None:
            return bool(self.keep_records)
        free, _ = torch.cuda.mem_get_info(self.device)
        return record_bytes(prob) * self.n_steps <= free // 2

    @staticmethod
    def _record_steps(prob: N.Problem, st: N.State, count: int) -> list:
        """`count` steps, as nauticle_step runs them, each leaving its record
        (st is advanced in place)."""
        recs = _alloc_records(prob, count)
        for rec in recs:
            prob.step_record(st, rec.sorted, rec.cells, rec.fields)
        return recs

    def forward(self, nu: float, c0: float, v0: torch.Tensor):
        """Runs the rollout keeping either every step's record or a
        checkpoint (a copy of the state) every K steps (see keep_records);
        returns (final state, prepared problem, what was kept)."""
        prob = self.problem(nu, c0)
        st = self.initial_state(prob, v0)
        if self.keeps_records(prob):
            kept = _Records(self._record_steps(prob, st, self.n_steps))
            return st, prob, kept
        kept = _Checkpoints()
        for s in range(self.n_steps):
            if s % self.K == 0:
                kept.append((s, st.clone()))
            prob.step(st, 1)
        return st, prob, kept

    def vjp(self, prob: N.Problem, kept, lam_x, lam_v):
        """Reverse sweep from cotangents (lam_x, lam_v: per-axis device FP32,
        in the final state's order) of the final positions and velocities:
        the one-step adjoints run in reverse over the kept records, or, from
        checkpoints, over each segment's records recomputed first.  Returns
        (dL/dv0 (n, dim) in id order, dL/dnu, dL/dc0)."""
        lam_x = [t.clone() for t in lam_x]
        lam_v = [t.clone() for t in lam_v]
        dnu = torch.zeros(1, dtype=torch.float64, device=self.device)
        dc0 = torch.zeros(1, dtype=torch.float64, device=self.device)
        out_x = [torch.empty_like(t) for t in lam_x]
        out_v = [torch.empty_like(t) for t in lam_x]

        def sweep(records):
            nonlocal lam_x, lam_v, out_x, out_v
            for rec in reversed(records):
                prob.adjoint(rec.sorted, rec.cells, rec.fields, lam_x, lam_v, out_x, out_v, dnu, dc0)
                lam_x, out_x = out_x, lam_x
                lam_v, out_v = out_v, lam_v

        if isinstance(kept, _Records):
            sweep(kept)
        else:
            for s0, st0 in reversed(kept):
                s1 = min(s0 + self.K, self.n_steps)
                cur = st0.clone()
                sweep(self._record_steps(prob, cur, s1 - s0))
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
    tensors).  The forward pass keeps every step's record, or only
    checkpoints (``rollout.keep_records``); the backward pass seeds the
    positions' cotangent from grad_output (brought into the final state's
    order by the library), recomputes the segments if only checkpoints were
    kept, and runs the hand-written adjoint.  Any loss built on r_T composes with it.  A
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
