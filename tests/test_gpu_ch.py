"""Parity of nauticle_ch_steps (Example 1b: Cahn-Hilliard with sph_L0 and
its adaptive time step, on fixed particles) with the FP64 oracle.

Tolerances: one step's mu and cdot within 1e-5 of their largest value (the
Laplacian's ~12 FP32 pair terms of random sign, each with relative error
~1e-6 from the FP32 distance, against the largest sum), c within 1e-6 of
its range; the device clock (time, dt) within 1e-5; a 50-step rollout
within 5e-4 (diffusive dynamics damp the per-step differences)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import f32, nauticle, u32
from tests.oracle_helpers import domain_of, params_of

pytestmark = pytest.mark.gpu


def _setup(N, case):
    prob = N.Problem([case], max_nbr=64)
    st = prob.state_from_cases()
    prob.build_cells(st)
    torch.cuda.synchronize()
    prob.check()
    perm = u32(prob.cells.perm)[: case.n]
    c = torch.from_numpy(np.ascontiguousarray(case.coef[perm])).cuda()
    clock = torch.tensor([0.0, case.dt], dtype=torch.float64, device="cuda")
    mu = torch.empty_like(c)
    cdot = torch.empty_like(c)
    return prob, perm, c, clock, mu, cdot


def _to_input(a, perm):
    out = np.empty_like(a)
    out[perm] = a
    return out


def test_one_step_matches_oracle():
    N = nauticle()
    case = WL.ch_sphere()
    prob, perm, c, clock, mu, cdot = _setup(N, case)
    prob.ch_steps(c, clock, 1, mu, cdot)
    torch.cuda.synchronize()
    prob.check()
    dom, prm = domain_of(case), params_of(case)
    c1, t1, dt1, mu_r, cd_r = O.ch_steps(dom, prm, case.pos.astype(np.float64), case.coef.astype(np.float64),
                                         0.0, case.dt, 1)
    mu_g = _to_input(f32(mu)[: case.n], perm)
    cd_g = _to_input(f32(cdot)[: case.n], perm)
    c_g = _to_input(f32(c)[: case.n], perm)
    e_mu = np.abs(mu_g - mu_r).max() / np.abs(mu_r).max()
    e_cd = np.abs(cd_g - cd_r).max() / np.abs(cd_r).max()
    e_c = np.abs(c_g - c1).max() / 2.0
    t_g, dt_g = clock.cpu().numpy()
    print(f"mu {e_mu:.2e} cdot {e_cd:.2e} c {e_c:.2e} time {t_g} dt {dt_g} vs {t1} {dt1}")
    assert e_mu < 1e-5 and e_cd < 1e-5 and e_c < 1e-6
    assert t_g == pytest.approx(t1, rel=1e-12)
    assert dt_g == pytest.approx(dt1, rel=1e-5)


def test_fifty_steps_with_the_adaptive_dt_match_oracle():
    N = nauticle()
    case = WL.ch_sphere(dx=0.1, seed=4)
    prob, perm, c, clock, mu, cdot = _setup(N, case)
    steps = 50
    prob.ch_steps(c, clock, steps, mu, cdot)
    torch.cuda.synchronize()
    prob.check()
    dom, prm = domain_of(case), params_of(case)
    c_r, t_r, dt_r, _, _ = O.ch_steps(dom, prm, case.pos.astype(np.float64), case.coef.astype(np.float64),
                                      0.0, case.dt, steps)
    c_g = _to_input(f32(c)[: case.n], perm)
    t_g, dt_g = clock.cpu().numpy()
    err = np.abs(c_g - c_r).max() / 2.0
    print(f"{steps} steps: c {err:.2e}, time {t_g:.6f} vs {t_r:.6f}, dt {dt_g:.6e} vs {dt_r:.6e}")
    assert err < 5e-4
    assert t_g == pytest.approx(t_r, rel=5e-4) and dt_g == pytest.approx(dt_r, rel=5e-4)
    # the phase mass is conserved (the Laplacian's pair terms cancel)
    assert abs(c_g.sum() - case.coef.astype(np.float64).sum()) < 1e-4 * np.abs(case.coef).sum()
    assert np.abs(c_g - case.coef).max() > 1e-2  # it evolved


def test_ch_entry_point_refuses_other_tables_and_ch_tables_refuse_nauticle_step():
    N = nauticle()
    lat = WL.periodic_2d_4096()
    prob = N.Problem([lat])
    st = prob.state_from_cases()
    prob.build_cells(st)
    c = torch.zeros(prob.n, device="cuda")
    clock = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(N.NauticleError) as e:
        prob.ch_steps(c, clock, 1)
    assert e.value.status == N.ERR_INVALID_ARG
    ch = N.Problem([WL.ch_sphere(dx=0.2)], max_nbr=64)
    s2 = ch.state_from_cases()
    with pytest.raises(N.NauticleError) as e:
        ch.step(s2, 1)
    assert e.value.status == N.ERR_INVALID_ARG
    torch.cuda.synchronize()
