"""Parity at the full sizes of the measured workloads, in the launch
configuration bench.py times (default tuning and list capacity), on what
the oracle can compute for a sample, and through properties that hold at
any size.

- 3-D periodic lattice, 8,388,608 particles: binning, keys, permutation and
  cell table bit-exact for every particle; neighbour counts and sets
  bit-exact for 4096 sampled particles; density, pressure and acceleration
  of one nauticle_step within 1e-5 of their scale, and the updated
  positions and velocities within 1e-5, for 2048 sampled particles
  (velocities against max |v'| or dt times the acceleration scale, the
  larger: from rest v' is dt a).
- The same recipe at 66,846,720 particles, the largest lattice under the
  26-bit index limit of a list entry: the same one-step checks.
- 3-D dam break, 1,595,308 particles (571,308 fixed): the same one-step
  checks on a sample drawn from the fluid and the walls, and the 500th
  step's fields on the state the GPU reached after 499 steps.
- Both, over 10 and 50 steps, every particle's position and velocity
  against the oracle's rollout.
- The 8.4M lattice recipe with cells for a skin of 0.1 2h, stepped 20 times
  with Verlet lists against 20 plain steps on the same table: positions and
  velocities of every particle within the rollout bar 5e-4 (the plain path
  being pinned to the oracle above and in the rollout tests)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import case_absolute_from_state, decode_nbr, f32, nauticle, norms, stack, u32
from tests.oracle_helpers import domain_of, params_of, v64, x64

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-5
TOL_ROLLOUT = 5e-4


def _one_step_sampled(N, case, n_nbr_sample, n_field_sample, seed):
    prob = N.Problem([case])  # the bench's configuration: default tuning and max_nbr
    st = prob.state_from_cases()
    torch.cuda.synchronize()
    n = case.n
    dom, prm = domain_of(case), params_of(case)
    cell_in = u32(st.cell)[:n].copy()
    off_in = stack(st.off, n).copy()
    # binning, bit-exact for every particle
    cell_ref, off_ref = O.bin_f32(dom, case.pos)
    np.testing.assert_array_equal(cell_in, cell_ref)
    np.testing.assert_array_equal(off_in.view(np.uint32), off_ref.view(np.uint32))
    print(f"{case.name}: {n} particles binned bit-exactly", flush=True)
    prob.step(st, 1)
    torch.cuda.synchronize()
    prob.check()
    # keys, permutation and cell table, bit-exact for every particle
    ks, perm_ref, start, end = O.sort_keys(cell_in, case.n_cells)
    perm = u32(prob.cells.perm)[:n]
    np.testing.assert_array_equal(u32(prob.cells.key)[:n], ks)
    np.testing.assert_array_equal(perm, perm_ref)
    np.testing.assert_array_equal(u32(prob.cells.cell_start)[: case.n_cells], start)
    np.testing.assert_array_equal(u32(prob.cells.cell_end)[: case.n_cells], end)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(n, dtype=perm.dtype)
    rng = np.random.default_rng(seed)
    # neighbour counts and sets of a sample, bit-exact
    sample = np.sort(rng.choice(n, n_nbr_sample, replace=False))
    cnt_ref, lst_ref = O.neighbours_f32(dom, case.h, cell_in, off_in, max_nbr=prob.max_nbr, which=sample)
    cnt = u32(prob.cells.nbr_count)[:n][inv[sample]]
    np.testing.assert_array_equal(cnt, cnt_ref)
    ent = u32(prob.cells.entries())[:, :n][:, inv[sample]]
    j, _ = decode_nbr(ent)
    for s in range(sample.size):
        k = cnt[s]
        assert sorted(perm[j[:k, s]].tolist()) == sorted(lst_ref[s, :k].tolist()), sample[s]
    print(f"{case.name}: keys, permutation, cell table and {n_nbr_sample} sampled lists bit-exact "
          f"({cnt.mean():.1f} neighbours each)", flush=True)
    # the step's fields for a sample, against the oracle evaluated one particle at a time
    fixed = case.fixed_mask()
    fs = np.sort(rng.choice(n, n_field_sample, replace=False))
    if case.n_fixed:  # make sure walls are in the sample
        fs = np.unique(np.concatenate([fs, rng.choice(np.flatnonzero(fixed), n_field_sample // 8, replace=False)]))
    x, v = x64(case), v64(case)
    rho_r, p_r = O.density(dom, prm, x, which=fs)
    a_r = O.forces_at(dom, prm, x, v, fs, fixed=fixed)
    rho_g = f32(prob.fields.rho)[:n][inv[fs]]
    p_g = f32(prob.fields.p)[:n][inv[fs]]
    a_g = stack(prob.fields.acc, n)[inv[fs]]
    S = norms(case, rho_r, p_r, a_r)
    fl = ~fixed[fs]
    err = dict(rho=np.abs(rho_g - rho_r).max() / S["rho"], p=np.abs(p_g - p_r).max() / S["p"],
               a=np.abs(a_g[fl] - a_r[fl]).max() / S["a"])
    assert np.all(a_g[~fl] == 0.0)
    # the update: v' = v + dt a, x' = x + dt v' (positions wrap on periodic axes)
    ids = u32(st.id)[:n]
    where = np.empty(n, np.int64)
    where[ids] = np.arange(n)
    xs_g = case_absolute_from_state(case, u32(st.cell)[:n][where[fs]], stack(st.off, n)[where[fs]])
    vs_g = stack(st.vel, n)[where[fs]]
    a_full = np.where(fl[:, None], a_r, 0.0)
    v1 = np.where(fl[:, None], v[fs] + case.dt * a_full, 0.0)
    x1 = x[fs] + case.dt * v1
    err["x"] = np.abs(O.min_image(dom, xs_g - x1)).max() / S["x"]
    # after one step v' - v = dt a: velocities take the scale of dt a where that is the larger
    # (a fluid at rest), else their own
    err["v"] = np.abs(vs_g - v1).max() / max(np.abs(v1).max(), case.dt * S["a"])
    print(f"{case.name}: {fs.size} sampled particles, " + ", ".join(f"err {k} {e:.2e}" for k, e in err.items()),
          flush=True)
    for k, e in err.items():
        assert e < TOL_STEP, k


def test_periodic_lattice_8388608_one_step_sampled():
    N = nauticle()
    _one_step_sampled(N, WL.periodic_3d_8m(), 4096, 2048, seed=101)


def test_largest_table_66846720_one_step_sampled():
    """The largest lattice of the recipe under the 26-bit index limit of a
    list entry (512 x 512 x 255 sites, 99.6 % of 2^26 particles; ~49 GiB of
    device memory): the same checks, where list offsets pass 2^32 bytes."""
    N = nauticle()
    case = WL.lattice_case(3, (512, 512, 255), 0.01, 1.2, 0.05, 0.05, seed=3, c0=10.0, nu=1e-3, dt=1e-4,
                           name="periodic_3d_66846720")
    assert case.n < (1 << 26)
    _one_step_sampled(N, case, 2048, 1024, seed=103)
    torch.cuda.empty_cache()


def test_dam_break_1595308_one_step_sampled():
    N = nauticle()
    _one_step_sampled(N, WL.dam_break_3d(), 4096, 2048, seed=102)


def _positions_by_id(case, st):
    n = case.n
    x = np.empty((n, 3))
    v = np.empty((n, 3))
    ids = u32(st.id)[:n]
    x[ids] = case_absolute_from_state(case, u32(st.cell)[:n], stack(st.off, n))
    v[ids] = stack(st.vel, n)
    return x, v


def test_verlet_steps_at_8388608_track_the_plain_steps():
    N = nauticle()
    base = WL.periodic_3d_8m()
    # the same lattice recipe with cells of at least 2h + skin: plain steps (a build every step)
    # and Verlet steps on that one table
    case = WL.lattice_case(3, (256, 256, 128), 0.01, 1.2, 0.05, 0.05, seed=3, c0=10.0, nu=1e-3, dt=1e-4,
                           skin=0.1 * 2.0 * base.h)
    steps = 20
    plain = N.Problem([case])
    st_p = plain.state_from_cases()
    plain.step(st_p, steps)
    torch.cuda.synchronize()
    plain.check()
    x_p, v_p = _positions_by_id(case, st_p)
    del plain, st_p
    torch.cuda.empty_cache()
    ver = N.Problem([case])
    st_v = ver.state_from_cases()
    builds = ver.step_verlet(st_v, steps)
    torch.cuda.synchronize()
    ver.check()
    x_v, v_v = _positions_by_id(case, st_v)
    dom = domain_of(case)
    err_x = np.abs(O.min_image(dom, x_v - x_p)).max() / float(case.length()[0])
    err_v = np.abs(v_v - v_p).max() / np.abs(v_p).max()
    print(f"8.4M, {steps} steps: Verlet builds {builds}, err x {err_x:.2e} v {err_v:.2e}", flush=True)
    assert builds < steps
    assert err_x < TOL_ROLLOUT and err_v < TOL_ROLLOUT


def test_dam_break_step_500_on_the_evolved_state_sampled():
    """After 499 steps the column has collapsed into an irregular layout.
    The 500th step's fields, for a sample, against the oracle evaluated on
    the GPU's own state at that time (read back exactly: cell-relative FP32
    is exact in FP64)."""
    N = nauticle()
    case = WL.dam_break_3d()
    prob = N.Problem([case])
    st = prob.state_from_cases()
    prob.step(st, 499)
    torch.cuda.synchronize()
    prob.check()
    n = case.n
    ids = u32(st.id)[:n].copy()
    x = np.empty((n, 3))
    v = np.empty((n, 3))
    x[ids] = case_absolute_from_state(case, u32(st.cell)[:n], stack(st.off, n))
    v[ids] = stack(st.vel, n)
    fixed = case.fixed_mask()
    x0 = x64(case)
    assert np.abs(x[fixed] - x0[fixed]).max() < 1e-6 and np.all(v[fixed] == 0.0)  # walls stay
    assert np.abs(x[~fixed] - x0[~fixed]).max() > 0.05  # the column has moved
    prob.step(st, 1)
    torch.cuda.synchronize()
    prob.check()
    perm = u32(prob.cells.perm)[:n]
    sorted_ids = ids[perm]  # particle id at each sorted position of step 500
    where = np.empty(n, np.int64)
    where[sorted_ids] = np.arange(n)
    rng = np.random.default_rng(103)
    fs = np.sort(rng.choice(np.flatnonzero(~fixed), 2048, replace=False))
    dom, prm = domain_of(case), params_of(case)
    rho_r, p_r = O.density(dom, prm, x, which=fs)
    a_r = O.forces_at(dom, prm, x, v, fs, fixed=fixed)
    rho_g = f32(prob.fields.rho)[:n][where[fs]]
    p_g = f32(prob.fields.p)[:n][where[fs]]
    a_g = stack(prob.fields.acc, n)[where[fs]]
    S = norms(case, rho_r, p_r, a_r)
    err = dict(rho=np.abs(rho_g - rho_r).max() / S["rho"], p=np.abs(p_g - p_r).max() / S["p"],
               a=np.abs(a_g - a_r).max() / S["a"])
    print(f"dam break, step 500 on the evolved state: " + ", ".join(f"err {k} {e:.2e}" for k, e in err.items())
          + f"; max |v| {np.abs(v).max():.3f} m/s", flush=True)
    for k, e in err.items():
        assert e < TOL_STEP, k


@pytest.mark.parametrize("which,steps", [("lattice_8388608", 10), ("dam_break_1595308", 50)])
def test_full_size_rollout_matches_the_oracle_for_every_particle(which, steps):
    """Multi-step rollouts at full size in the bench's configuration, every
    particle against the oracle's rollout from the same FP32 inputs: the
    8.4M lattice over 10 steps, the dam break over 50 (the column starts to
    fall; walls stay).  Positions against the largest displacement over the
    rollout (a bar relative to the box length would hide every error),
    velocities against max |v|; the rollout bar 5e-4."""
    N = nauticle()
    case = WL.periodic_3d_8m() if which.startswith("lattice") else WL.dam_break_3d()
    prob = N.Problem([case])
    st = prob.state_from_cases()
    prob.step(st, steps)
    torch.cuda.synchronize()
    prob.check()
    x_g, v_g = _positions_by_id(case, st)
    del prob, st
    torch.cuda.empty_cache()
    print(f"{case.name}: {steps} GPU steps done; oracle rollout of {case.n} particles ...", flush=True)
    dom, prm = domain_of(case), params_of(case)
    x0 = x64(case)
    x, v, _, _, _ = O.step(dom, prm, x0, v64(case), fixed=case.fixed_mask(), n_steps=steps)
    moved = np.abs(O.min_image(dom, x - x0)).max()
    err_x = np.abs(O.min_image(dom, x_g - x)).max() / moved
    err_v = np.abs(v_g - v).max() / np.abs(v).max()
    fixed = case.fixed_mask()
    print(f"{case.name}, {steps} steps, all {case.n} particles: err x {err_x:.2e} of the largest "
          f"displacement ({moved:.3e} m), v {err_v:.2e} of max |v| ({np.abs(v).max():.3e} m/s)", flush=True)
    assert err_x < TOL_ROLLOUT and err_v < TOL_ROLLOUT
    if fixed.any():
        assert np.all(v_g[fixed] == 0.0) and np.abs(x_g[fixed] - x0[fixed]).max() < 1e-6
