"""The 3-D adjoint against the FP64 oracle, and the differentiable rollout
that returns the final positions (NauticleRollout) against the oracle's
reverse sweep from the same cotangents.

Bars (derived with the 2-D ones): one step -- lam_x 1e-4 of its largest
element (its terms hold F'/r and differences of A between neighbours, which
cancel), lam_v 1e-5 (no kernel Hessian), dL/dnu and dL/dc0 1e-4 relative;
rollouts of 15-20 FP32 steps -- 1e-2 relative, the rollout-gradient bar.
The measured errors are printed."""
import copy

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import f32, nauticle, u32
from tests.oracle_helpers import domain_of, params_of, v64, x64

pytestmark = pytest.mark.gpu


def _walls_case():
    c = WL.dam_break_case(dx=0.02, h_over_dx=1.2, c0=10.0, nu=1e-3, fluid=(0.2, 0.16, 0.24),
                          tank=(0.32, 0.16, 0.3), layers=3)
    rng = np.random.default_rng(41)
    v = rng.normal(0, 0.2, c.vel.shape).astype(np.float32)
    v[c.fixed_mask()] = 0.0
    pos = c.pos + (rng.uniform(-0.05, 0.05, c.pos.shape) * 0.02).astype(np.float32)
    pos[c.fixed_mask()] = c.pos[c.fixed_mask()]
    return WL.scaled(c, vel=v, pos=pos.astype(np.float32), dt=2e-4, name="tank_3d")


CASES_3D = {
    "periodic_16x15x14": lambda: WL.lattice_case(3, (16, 15, 14), 0.01, 1.2, 0.1, 0.2, seed=37, c0=10.0,
                                                 nu=2e-3, dt=2e-4),
    "walls": _walls_case,
}


def _one_step_vjp(N, case, seed):
    """One-step VJP through nauticle_sph_adjoint on random cotangents;
    returns the GPU's and the oracle's (lam_x, lam_v, dnu, dc0)."""
    d = case.dim
    prob = N.Problem([case])
    st = prob.state_from_cases()
    prob.build_cells(st)
    prob.density()
    n = case.n
    rng = np.random.default_rng(seed)
    lx_in = rng.normal(size=(n, d))
    lv_in = rng.normal(size=(n, d))
    torch.cuda.synchronize()
    perm = u32(prob.cells.perm)[:n]
    # cotangents of the step's outputs live in the output (sorted) order
    lxn = [torch.from_numpy(lx_in[perm, k].astype(np.float32)).cuda() for k in range(d)]
    lvn = [torch.from_numpy(lv_in[perm, k].astype(np.float32)).cuda() for k in range(d)]
    lx = [torch.empty(n, device="cuda") for _ in range(d)]
    lv = [torch.empty(n, device="cuda") for _ in range(d)]
    dnu = torch.zeros(1, dtype=torch.float64, device="cuda")
    dc0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    prob.adjoint(prob.sorted, prob.cells, prob.fields, lxn, lvn, lx, lv, dnu, dc0)
    torch.cuda.synchronize()
    prob.check()
    gx = np.stack([f32(t) for t in lx], 1)
    gv = np.stack([f32(t) for t in lv], 1)
    # the cotangents are rounded to FP32 for the GPU: the oracle takes the same values
    lx64 = lx_in.astype(np.float32).astype(np.float64)
    lv64 = lv_in.astype(np.float32).astype(np.float64)
    ox, ov, onu, oc0 = O.step_vjp(domain_of(case), params_of(case), x64(case), v64(case), lx64, lv64,
                                  fixed=case.fixed_mask())
    return (gx, gv, dnu.item(), dc0.item()), (ox, ov, onu, oc0)


@pytest.mark.parametrize("name", list(CASES_3D))
def test_adjoint_one_step_3d_matches_oracle_vjp(name):
    """Every particle's lam_x and lam_v, and the constants' cotangents, of
    one 3-D step (z terms of every sum, the 3-D F'/r Hessian, fixed walls
    with zero cotangents) against the oracle element by element."""
    N = nauticle()
    case = CASES_3D[name]()
    (gx, gv, gnu, gc0), (ox, ov, onu, oc0) = _one_step_vjp(N, case, seed=7)
    ex = np.abs(gx - ox).max() / np.abs(ox).max()
    ev = np.abs(gv - ov).max() / np.abs(ov).max()
    enu = abs(gnu - onu) / abs(onu)
    ec0 = abs(gc0 - oc0) / abs(oc0)
    print(f"{name} ({case.n} particles, {case.n_fixed} fixed): adjoint x {ex:.2e} v {ev:.2e} "
          f"nu {enu:.2e} c0 {ec0:.2e}")
    assert ex < 1e-4 and ev < 1e-5 and enu < 1e-4 and ec0 < 1e-4
    fixed = case.fixed_mask()
    if fixed.any():
        assert np.all(gx[fixed] == 0.0) and np.all(gv[fixed] == 0.0)


def test_adjoint_one_step_262k_matches_oracle_vjp():
    """The differentiation workload itself (64^3 = 262,144 particles, 3-D
    periodic, in the launch configuration of the rollout): one step's VJP
    of every particle against the oracle."""
    N = nauticle()
    case = WL.periodic_3d_262k()
    (gx, gv, gnu, gc0), (ox, ov, onu, oc0) = _one_step_vjp(N, case, seed=11)
    ex = np.abs(gx - ox).max() / np.abs(ox).max()
    ev = np.abs(gv - ov).max() / np.abs(ov).max()
    enu = abs(gnu - onu) / abs(onu)
    ec0 = abs(gc0 - oc0) / abs(oc0)
    print(f"262k one-step adjoint: x {ex:.2e} v {ev:.2e} nu {enu:.2e} c0 {ec0:.2e}")
    assert ex < 1e-4 and ev < 1e-5 and enu < 1e-4 and ec0 < 1e-4


def test_rollout_gradient_3d_matches_oracle():
    """20 steps of a 3-D periodic box, checkpoints every 6 (a partial last
    segment), loss against a target run with nu x 1.5 and c0 x 0.8: the
    loss, every element of dL/dv0, dL/dnu and dL/dc0 against the oracle's
    rollout gradient."""
    nauticle()
    from paper_1710_08259_amd.rollout import Rollout

    case = WL.lattice_case(3, (12, 11, 10), 0.01, 1.2, 0.1, 0.2, seed=43, c0=8.0, nu=2e-3, dt=2e-4)
    steps, K = 20, 6
    ro = Rollout(case, steps, checkpoint_every=K)
    v0 = torch.from_numpy(case.vel).cuda()
    target = ro.run(case.nu * 1.5, case.c0 * 0.8, v0)
    L, gv0, gnu, gc0 = ro.loss_and_grad(case.nu, case.c0, v0, target)
    dom, prm = domain_of(case), params_of(case)
    tgt = copy.copy(prm)
    tgt.nu, tgt.c0 = prm.nu * 1.5, prm.c0 * 0.8
    xt, _, _, _, _ = O.step(dom, tgt, x64(case), v64(case), n_steps=steps)
    Lo, gvo, gnuo, gc0o = O.rollout_grad(dom, prm, x64(case), v64(case), xt, steps, checkpoint_every=K)
    gv = gv0.cpu().numpy()
    e_L = abs(L - Lo) / Lo
    e_v = np.abs(gv - gvo).max() / np.abs(gvo).max()
    e_nu = abs(gnu - gnuo) / abs(gnuo)
    e_c0 = abs(gc0 - gc0o) / abs(gc0o)
    print(f"3-D rollout grad vs oracle: L {e_L:.2e} v0 {e_v:.2e} nu {e_nu:.2e} c0 {e_c0:.2e}")
    assert e_L < 1e-3 and e_v < 1e-2 and e_nu < 1e-2 and e_c0 < 1e-2


@pytest.mark.parametrize("dim", [2, 3])
def test_autograd_rollout_returns_final_positions_and_their_vjp(dim):
    """NauticleRollout.apply(v0, nu, c0, rollout) returns r_T in id order:
    against the oracle's rollout positions; a loss that is not the position
    MSE, sum(w * r_T) + sum(r_T^2) / 2, backpropagates through the adjoint
    to v0, nu and c0 as the oracle's reverse sweep from the same cotangent
    (w + r_T) does."""
    nauticle()
    from paper_1710_08259_amd.rollout import NauticleRollout, Rollout

    if dim == 2:
        case = WL.lattice_case(2, (16, 16), 0.01, 1.3, 0.05, 0.2, seed=31, c0=8.0, dt=2e-4)
    else:
        case = WL.lattice_case(3, (10, 10, 9), 0.01, 1.2, 0.05, 0.2, seed=47, c0=8.0, dt=2e-4)
    steps, K = 15, 4
    ro = Rollout(case, steps, checkpoint_every=K)
    v0 = torch.from_numpy(case.vel).cuda().requires_grad_(True)
    nu = torch.tensor(case.nu, dtype=torch.float64, requires_grad=True)
    c0 = torch.tensor(case.c0, dtype=torch.float64, requires_grad=True)
    r_T = NauticleRollout.apply(v0, nu, c0, ro)
    assert r_T.shape == (case.n, dim) and r_T.dtype == torch.float32
    w = torch.from_numpy(np.random.default_rng(53).normal(size=(case.n, dim)).astype(np.float32)).cuda()
    loss = (w * r_T).sum() + 0.5 * (r_T * r_T).sum()
    loss.backward()

    dom, prm = domain_of(case), params_of(case)
    xT, _, _, _, _ = O.step(dom, prm, x64(case), v64(case), n_steps=steps)
    r = r_T.detach().cpu().numpy().astype(np.float64)
    L = float(np.max(case.length()[:dim]))
    e_x = np.abs(O.min_image(dom, r - xT)).max() / L
    seed = w.cpu().numpy().astype(np.float64) + r  # d loss / d r_T, as the GPU's backward received it
    _, lvo, dnuo, dc0o = O.rollout_vjp(dom, prm, x64(case), v64(case), steps, seed, np.zeros_like(seed),
                                       checkpoint_every=K)
    gv = v0.grad.cpu().numpy()
    e_v = np.abs(gv - lvo).max() / np.abs(lvo).max()
    e_nu = abs(nu.grad.item() - dnuo) / abs(dnuo)
    e_c0 = abs(c0.grad.item() - dc0o) / abs(dc0o)
    print(f"{dim}-D NauticleRollout: r_T {e_x:.2e} (of L); grads vs oracle sweep: v0 {e_v:.2e} "
          f"nu {e_nu:.2e} c0 {e_c0:.2e}")
    assert e_x < 1e-6
    assert e_v < 1e-2 and e_nu < 1e-2 and e_c0 < 1e-2
    assert nu.grad.dtype == torch.float64 and nu.grad.device == nu.device


def test_autograd_rollout_position_mse_equals_the_fused_loss_gradient():
    """The position MSE written in torch on r_T (minimum image against the
    target's r_T) gives the gradients of Rollout.loss_and_grad, which seeds
    the same sweep from nauticle_position_loss."""
    nauticle()
    from paper_1710_08259_amd.rollout import NauticleRollout, Rollout

    case = WL.lattice_case(2, (16, 16), 0.01, 1.3, 0.05, 0.2, seed=59, c0=8.0)
    steps = 12
    ro = Rollout(case, steps, checkpoint_every=5)
    v0d = torch.from_numpy(case.vel).cuda()
    target_state = ro.run(case.nu * 1.5, case.c0 * 0.8, v0d)
    L_ref, gv_ref, gnu_ref, gc0_ref = ro.loss_and_grad(case.nu, case.c0, v0d, target_state)
    with torch.no_grad():
        tgt = NauticleRollout.apply(v0d, torch.tensor(case.nu * 1.5, dtype=torch.float64),
                                    torch.tensor(case.c0 * 0.8, dtype=torch.float64), ro)
    v0 = v0d.clone().requires_grad_(True)
    nu = torch.tensor(case.nu, dtype=torch.float64, requires_grad=True)
    c0 = torch.tensor(case.c0, dtype=torch.float64, requires_grad=True)
    r_T = NauticleRollout.apply(v0, nu, c0, ro)
    Lbox = torch.tensor(case.length()[:2], dtype=torch.float32, device="cuda")
    d = r_T - tgt
    d = d - Lbox * torch.round(d / Lbox)
    loss = (d * d).sum() / (case.n * 2)
    loss.backward()
    e_L = abs(loss.item() - L_ref) / L_ref
    e_v = (v0.grad - gv_ref).abs().max().item() / gv_ref.abs().max().item()
    e_nu = abs(nu.grad.item() - gnu_ref) / abs(gnu_ref)
    e_c0 = abs(c0.grad.item() - gc0_ref) / abs(gc0_ref)
    print(f"torch MSE on r_T vs fused loss: L {e_L:.2e} v0 {e_v:.2e} nu {e_nu:.2e} c0 {e_c0:.2e}")
    # the two differ only in how the displacement is rounded (absolute FP32
    # positions here, cell-relative offsets there)
    assert e_L < 1e-3 and e_v < 1e-3 and e_nu < 1e-3 and e_c0 < 1e-3
