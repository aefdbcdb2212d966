"""Parity of the HIP path with the FP64 oracle for symmetric (mirror) faces
and for Example 1a's model (continuity, linear equation of state, momentum
with the artificial viscosity), through the C-ABI.

Bit-exact: neighbour counts and sets, each entry's image axes and cell
offsets.  Floating point: per-step fields within 1e-5 of their scale,
positions and velocities within 5e-4 after a rollout."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import case_absolute_from_state, f32, nauticle, norms, stack, u32
from tests.oracle_helpers import domain_of, params_of, x64

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-5
TOL_ROLLOUT = 5e-4
SYM, CUT, PER = WL.SYMMETRIC, WL.CUTOFF, WL.PERIODIC


def _ex1a_moving(scale, seed):
    """Example 1a's column with random velocities and densities (so that
    every term of the continuity and momentum sums is exercised)."""
    c = WL.ex1a_dam_break(scale)
    rng = np.random.default_rng(seed)
    return WL.scaled(c, vel=rng.normal(0, 0.5, c.vel.shape).astype(np.float32),
                     rho=(c.rho0 * (1 + 0.01 * rng.standard_normal(c.n))).astype(np.float32),
                     name=f"ex1a_moving_{scale:g}")


CASES = {
    "mirror_2d": WL.mirror_box_case(2, (SYM, SYM, CUT), 11, n=700),
    "mirror_3d_cutoff_y": WL.mirror_box_case(3, (SYM, CUT, SYM), 12),
    "mirror_3d_periodic_y": WL.mirror_box_case(3, (SYM, PER, SYM), 13, n=3000),
    "mirror_2d_periodic_x": WL.mirror_box_case(2, (PER, SYM, CUT), 16, n=700),
    "mirror_2d_continuity": WL.mirror_box_case(2, (SYM, SYM, CUT), 14, n=700, model=WL.CONTINUITY),
    "mirror_3d_continuity": WL.mirror_box_case(3, (SYM, PER, SYM), 15, n=3000, model=WL.CONTINUITY),
    "ex1a_moving_2": _ex1a_moving(2.0, 3),
}
NAMES = list(CASES)
CONT_NAMES = [k for k, c in CASES.items() if c.model == WL.CONTINUITY]
SUM_NAMES = [k for k, c in CASES.items() if c.model == WL.SUMMATION]


def _max_nbr(case):
    # the crowded corners hold up to ~210 neighbours and images
    return 256


def _search(N, case):
    prob = N.Problem([case], max_nbr=_max_nbr(case))
    st = prob.state_from_cases()
    prob.build_cells(st)
    torch.cuda.synchronize()
    prob.check()
    return prob, st


def _inverse(perm):
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0], dtype=perm.dtype)
    return inv


@pytest.mark.parametrize("name", NAMES)
def test_mirror_lists_are_bit_exact(name):
    """Counts, and per particle the multiset of (neighbour, image axes), equal
    the oracle's FP32 lists; on other axes the stored offset is the folded
    cell difference; an image entry's particle and neighbour share the
    boundary cell of that axis."""
    N = nauticle()
    case = CASES[name]
    prob, st = _search(N, case)
    n, dim = case.n, case.dim
    cell_in = u32(st.cell)[:n]
    off_in = stack(st.off, n)
    perm = u32(prob.cells.perm)[:n]
    cnt_ref, lst_ref, mir_ref = O.neighbours_f32(domain_of(case), case.h, cell_in, off_in,
                                                 max_nbr=_max_nbr(case), mirrors=True)
    cnt = u32(prob.cells.nbr_count)[:n]
    np.testing.assert_array_equal(cnt, cnt_ref[perm])
    assert (cnt <= _max_nbr(case)).all()
    ent = u32(prob.cells.entries())[:, :n]
    j = ent & ((1 << 26) - 1)
    code = [((ent >> (26 + 2 * k)) & 3).astype(np.int64) for k in range(3)]
    nc = case.ncell
    coords = np.stack([cell_in % nc[0], (cell_in // nc[0]) % nc[1], cell_in // (nc[0] * nc[1])],
                      axis=1).astype(np.int64)
    n_images = 0
    for p in range(n):
        k = cnt[p]
        i = perm[p]
        nb = perm[j[:k, p]]
        mask = np.zeros(k, np.int64)
        for a in range(dim):
            mask |= (code[a][:k, p] == N.MIRROR_CODE).astype(np.int64) << a
        got = sorted(zip(nb.tolist(), mask.tolist()))
        want = sorted(zip(lst_ref[i, :k].tolist(), mir_ref[i, :k].astype(np.int64).tolist()))
        assert got == want, p
        n_images += int((mask != 0).sum())
        for a in range(dim):
            img = code[a][:k, p] == N.MIRROR_CODE
            # images: same boundary cell along a
            assert np.all(coords[nb[img], a] == coords[i, a])
            assert np.all((coords[i, a] == 0) | (coords[i, a] == nc[a] - 1)) or not img.any()
            dc = coords[nb[~img], a] - coords[i, a]
            if case.boundary[a] == PER:
                dc = (dc + nc[a] // 2) % nc[a] - nc[a] // 2
            np.testing.assert_array_equal(dc, code[a][:k, p][~img] - 1)
    assert n_images > 0


@pytest.mark.parametrize("name", SUM_NAMES)
def test_summation_model_with_symmetric_faces_matches_oracle(name):
    N = nauticle()
    case = CASES[name]
    prob, _ = _search(N, case)
    prob.density()
    prob.forces()
    torch.cuda.synchronize()
    prob.check()
    inv = _inverse(u32(prob.cells.perm)[: case.n])
    rho_g = f32(prob.fields.rho)[: case.n][inv]
    p_g = f32(prob.fields.p)[: case.n][inv]
    a_g = stack(prob.fields.acc, case.n)[inv]
    dom, prm = domain_of(case), params_of(case)
    x, v = x64(case), case.vel.astype(np.float64)
    rho, p = O.density(dom, prm, x)
    a = O.forces(dom, prm, x, v, rho, p)
    S = norms(case, rho, p, a)
    err = (np.abs(rho_g - rho).max() / S["rho"], np.abs(p_g - p).max() / S["p"], np.abs(a_g - a).max() / S["a"])
    print(f"{name}: rho {err[0]:.2e} p {err[1]:.2e} a {err[2]:.2e}")
    assert max(err) < TOL_STEP


def _continuity_reference(case):
    dom, prm = domain_of(case), params_of(case)
    x, v = x64(case), case.vel.astype(np.float64)
    rho = case.rho.astype(np.float64)
    drho = O.continuity(dom, prm, x, v, rho)
    rn = rho + prm.dt * drho
    p = np.array([O.linear_eos(prm, r) for r in rn])
    a = O.momentum(dom, prm, x, v, rn, p)
    return drho, rn, p, a


@pytest.mark.parametrize("name", CONT_NAMES)
def test_continuity_and_momentum_match_oracle(name):
    """One continuity pass (drho, rho' = rho + dt drho, p = c^2 (rho' -
    rho0)) and one momentum pass (pressure + artificial viscosity + g) on
    the same inputs as the oracle's eq1..eq5."""
    N = nauticle()
    case = CASES[name]
    prob, _ = _search(N, case)
    prob.continuity()
    prob.forces()
    torch.cuda.synchronize()
    prob.check()
    n = case.n
    inv = _inverse(u32(prob.cells.perm)[:n])
    drho_g = f32(prob.fields.drho)[:n][inv]
    rho_g = f32(prob.fields.rho)[:n][inv]
    p_g = f32(prob.fields.p)[:n][inv]
    a_g = stack(prob.fields.acc, n)[inv]
    drho, rn, p, a = _continuity_reference(case)
    S = norms(case, rn, p, a)
    s_drho = case.rho0 * float(np.abs(case.vel).max()) / case.h
    err = dict(drho=np.abs(drho_g - drho).max() / s_drho, rho=np.abs(rho_g - rn).max() / S["rho"],
               p=np.abs(p_g - p).max() / S["p"], a=np.abs(a_g - a).max() / S["a"])
    print(name, {k: f"{e:.2e}" for k, e in err.items()})
    assert max(err.values()) < TOL_STEP
    assert np.abs(drho).max() > 1e-3 * s_drho  # the sums are not trivially zero


def test_ex1a_rollout_matches_oracle():
    """Example 1a's dam break (h = 0.125 m, 2,170 particles) for 60 steps of
    1/2 ms through nauticle_step, against the oracle's eq1..eq7."""
    N = nauticle()
    case = WL.ex1a_dam_break(2.0)
    prob = N.Problem([case], max_nbr=64)
    st = prob.state_from_cases()
    steps = 60
    prob.step(st, steps)
    torch.cuda.synchronize()
    prob.check()
    n = case.n
    ids = u32(st.id)[:n]
    x_g = np.empty((n, 2))
    v_g = np.empty((n, 2))
    r_g = np.empty(n)
    x_g[ids] = case_absolute_from_state(case, u32(st.cell)[:n], stack(st.off, n))
    v_g[ids] = stack(st.vel, n)
    r_g[ids] = f32(st.rho)[:n]
    dom, prm = domain_of(case), params_of(case)
    x, v, rho, _, _, _ = O.step_ex1a(dom, prm, x64(case), np.zeros((n, 2)), case.rho.astype(np.float64),
                                     n_steps=steps)
    err_x = np.abs(x_g - x).max() / norms(case)["x"]
    err_v = np.abs(v_g - v).max() / np.abs(v).max()
    err_r = np.abs(r_g - rho).max() / case.rho0
    print(f"ex1a {steps} steps: err x {err_x:.2e} v {err_v:.2e} rho {err_r:.2e}")
    assert err_x < TOL_ROLLOUT and err_v < TOL_ROLLOUT and err_r < TOL_ROLLOUT
    assert v[:, 1].mean() < 0  # the column is falling


@pytest.mark.parametrize("name", ["mirror_2d_continuity", "ex1a_moving_2", "mirror_2d"])
def test_step_equals_separate_passes_bitwise(name):
    N = nauticle()
    case = CASES[name]
    cont = case.model == WL.CONTINUITY
    prob = N.Problem([case], max_nbr=_max_nbr(case))
    st0 = prob.state_from_cases()
    st1 = st0.clone()
    prob.step(st1, 1)
    torch.cuda.synchronize()
    f_step = [f32(t).copy() for t in (prob.fields.rho, prob.fields.p, *prob.fields.acc)]
    sorted_ = prob.new_state()
    nxt = prob.new_state()
    prob.build_cells(st0, sorted_)
    if cont:
        prob.continuity(sorted_)
    else:
        prob.density(sorted_)
    prob.forces(sorted_, nxt)
    torch.cuda.synchronize()
    prob.check()
    f_sep = [f32(t) for t in (prob.fields.rho, prob.fields.p, *prob.fields.acc)]
    for a, b in zip(f_step, f_sep):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
    n = case.n
    np.testing.assert_array_equal(u32(st1.cell)[:n], u32(nxt.cell)[:n])
    np.testing.assert_array_equal(stack(st1.off, n).view(np.uint32), stack(nxt.off, n).view(np.uint32))
    np.testing.assert_array_equal(stack(st1.vel, n).view(np.uint32), stack(nxt.vel, n).view(np.uint32))
    if cont:
        np.testing.assert_array_equal(f32(st1.rho)[:n].view(np.uint32), f32(nxt.rho)[:n].view(np.uint32))


def test_entry_points_refuse_what_they_do_not_cover():
    N = nauticle()
    prob = N.Problem([CASES["mirror_2d"]])
    st = prob.state_from_cases()
    prob.build_cells(st)
    with pytest.raises(N.NauticleError) as e:
        prob.continuity()  # summation model
    assert e.value.status == N.ERR_INVALID_ARG
    z = [torch.zeros(prob.n, device="cuda") for _ in range(2)]
    d = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(N.NauticleError) as e:  # adjoint with symmetric faces
        prob.adjoint(prob.sorted, prob.cells, prob.fields, z, z, [t.clone() for t in z], [t.clone() for t in z],
                     d, d.clone())
    assert e.value.status == N.ERR_INVALID_ARG
    cp = N.Problem([CASES["mirror_2d_continuity"]])
    s2 = cp.state_from_cases()
    s2.rho = None
    with pytest.raises(N.NauticleError) as e:  # the continuity model needs rho
        cp.build_cells(s2)
    assert e.value.status == N.ERR_INVALID_ARG
    torch.cuda.synchronize()
