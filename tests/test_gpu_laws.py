"""Parity of the pair-law pass (nauticle_interact / nauticle_step_law) with
the FP64 oracle: Example 2's DEM contact law in a box with symmetric faces,
and the social force model in a room walled by fixed people.

Tolerances: the DEM overlap delta = R_i + R_j - r is a difference of
nearly equal FP32 lengths, with an absolute error of about 2u(R_i + R_j) ~
1e-9 m.  Through f ~ delta^(3/2) that is a relative force error of about
1.5e-9 / delta, 1e-5 at the tested overlaps of ~1e-4 m, more for grazing
contacts; and the damping term's delta^(1/4) has an unbounded slope at
delta = 0.  The social force's exp((R_ij - d)/B) turns the FP32 distance
error, about u (cs + d) ~ 1.4e-7 m in the cell frame, into a relative
error of 1.4e-7 / B ~ 2e-6 per term (B = 0.08 m), on terms several times
the net acceleration.  The per-step bars are therefore 1e-4 of the largest
acceleration for both laws, rollouts 5e-4."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import case_absolute_from_state, nauticle, stack, u32
from tests.oracle_helpers import domain_of, params_of

pytestmark = pytest.mark.gpu

TOL_DEM = 1e-4
TOL_SOCIAL = 1e-4
TOL_ROLLOUT = 5e-4


def _dem_case():
    return WL.dem_damper(spacing=2 * 0.004 * 0.985, jitter=0.05, v_sigma=0.1, seed=3, name="dem_overlapping")


def _social_case():
    c = WL.social_room(width=20.0, density=1.4, c_max=50.0, seed=5)
    rng = np.random.default_rng(6)
    v = rng.normal(0, 0.4, c.vel.shape).astype(np.float32)
    v[c.fixed_mask()] = 0.0
    return WL.scaled(c, vel=v, name="social_moving")


CASES = {"dem": _dem_case(), "social": _social_case()}


def _oracle_acc(case, x=None, v=None):
    dom, prm = domain_of(case), params_of(case)
    x = case.pos.astype(np.float64) if x is None else x
    v = case.vel.astype(np.float64) if v is None else v
    if case.model == WL.DEM:
        return O.dem(dom, prm, x, v, case.radius, case.pmass, case.coef, fixed=case.fixed_mask())
    return O.social(dom, prm, x, v, case.radius, case.pmass, case.coef, case.v0, case.goal,
                    fixed=case.fixed_mask())


def _run_pass(N, case):
    prob = N.Problem([case], max_nbr=64)
    st = prob.state_from_cases()
    attrs = prob.law_attrs()
    prob.build_cells(st)
    prob.interact(attrs)
    torch.cuda.synchronize()
    prob.check()
    perm = u32(prob.cells.perm)[: case.n]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(case.n, dtype=perm.dtype)
    return prob, stack(prob.fields.acc, case.n)[inv]


@pytest.mark.parametrize("name", list(CASES))
def test_pair_law_pass_matches_oracle(name):
    N = nauticle()
    case = CASES[name]
    _, a_g = _run_pass(N, case)
    a = _oracle_acc(case)
    scale = float(np.abs(a).max())
    err = np.abs(a_g - a).max() / scale
    print(f"{name}: max |a| {scale:.3e}, err {err:.2e}")
    assert err < (TOL_DEM if case.model == WL.DEM else TOL_SOCIAL)
    if case.model == WL.DEM:
        assert scale > 50.0  # contacts (and images) act
    else:
        assert np.all(a_g[case.fixed_mask()] == 0.0)


U32 = 2.0 ** -24  # unit roundoff of FP32


@pytest.mark.parametrize("name", list(CASES))
def test_pair_law_pass_matches_oracle_per_particle(name):
    """Each particle's acceleration against the size of the terms it is a
    sum of (the oracle's sum_j |F_ij| / m_i + |own term| + |g|, floored at
    1e-6 of the largest such size), so that errors on weakly loaded
    particles count as much as on the busiest.  Bar 1e-4 (module
    docstring).  DEM contacts whose FP32 force is ill-conditioned are left
    out and counted: grazing contacts (overlap delta below 2e-3 of R_i + R_j:
    the FP32 overlap carries an absolute error of about 2u (R_i + R_j), the
    rounding of r and of R_i + R_j, so a relative error 2u / ratio, which
    delta^(3/2) amplifies 1.5x: 9e-5 of that contact's force at the
    threshold, more below it), and nearly normal sliding contacts (|v_t|
    below 1e4 u |v_j - v_i|: the friction direction's FP32 error
    ~u |v_j - v_i| / |v_t| times c_f |f_n| would pass 1e-4 of the sum)."""
    N = nauticle()
    case = CASES[name]
    _, a_g = _run_pass(N, case)
    law = "dem" if case.model == WL.DEM else "social"
    dom, prm = domain_of(case), params_of(case)
    a, diag = O.law_diag(law, dom, prm, case.pos.astype(np.float64), case.vel.astype(np.float64), case.radius,
                         case.pmass, case.coef, v0=case.v0, goal=case.goal, fixed=case.fixed_mask())
    size = diag[:, 0]
    scale = np.maximum(size, 1e-6 * size.max())
    keep = ~case.fixed_mask()
    if law == "dem":
        grazing = diag[:, 1] < 2e-3
        normal = diag[:, 2] < 1e4 * U32
        keep &= ~grazing & ~normal
        print(f"dem: {case.n} spheres, left out: {int(grazing.sum())} with a grazing contact, "
              f"{int((normal & ~grazing).sum())} more with a nearly normal sliding contact")
        assert keep.sum() > case.n // 2
    e = np.abs(a_g - a).max(axis=1) / scale
    worst = int(np.argmax(np.where(keep, e, 0.0)))
    print(f"{name}: per-particle err max {e[keep].max():.2e} (particle {worst}, |a| {np.abs(a[worst]).max():.3e}, "
          f"size {size[worst]:.3e}), median {np.median(e[keep]):.2e}; over all particles {e.max():.2e}")
    assert e[keep].max() < (TOL_DEM if law == "dem" else TOL_SOCIAL)


@pytest.mark.parametrize("name,steps", [("dem", 150), ("dem_friction", 40), ("social", 150)])
def test_pair_law_rollout_matches_oracle(name, steps):
    """Rollouts through nauticle_step_law: DEM without and with Coulomb
    friction (c_f = 0.3), and the social force.  With friction the rollout
    is held to the bar for 40 steps; beyond ~50 steps sliding contacts come
    to rest and the friction direction, which jumps at v_t = 0, chatters, so
    the dynamics amplify rounding (see the next test)."""
    N = nauticle()
    case = CASES["dem" if name.startswith("dem") else name]
    if name == "dem":
        case = WL.scaled(case, law=(0.0,))
    prob = N.Problem([case], max_nbr=64)
    st = prob.state_from_cases()
    attrs = prob.law_attrs()
    prob.step_law(st, attrs, steps)
    torch.cuda.synchronize()
    prob.check()
    n = case.n
    ids = u32(st.id)[:n]
    x_g = np.empty((n, case.dim))
    v_g = np.empty((n, case.dim))
    x_g[ids] = case_absolute_from_state(case, u32(st.cell)[:n], stack(st.off, n))
    v_g[ids] = stack(st.vel, n)
    dom, prm = domain_of(case), params_of(case)
    law = "dem" if case.model == WL.DEM else "social"
    x, v, _ = O.step_law(law, dom, prm, case.pos.astype(np.float64), case.vel.astype(np.float64), case.radius,
                         case.pmass, case.coef, v0=case.v0, goal=case.goal, fixed=case.fixed_mask(),
                         n_steps=steps)
    L = float(np.max(case.length()[: case.dim]))
    err_x = np.abs(x_g - x).max() / L
    err_v = np.abs(v_g - v).max() / np.abs(v).max()
    print(f"{name} {steps} steps: err x {err_x:.2e} (of L) v {err_v:.2e} (of max |v|)")
    assert err_x < TOL_ROLLOUT and err_v < TOL_ROLLOUT


def test_dem_friction_rollout_150_steps_within_the_oracles_own_sensitivity():
    """150 DEM steps with Coulomb friction.  Contacts that come to rest make
    the friction direction v_t/|v_t| chatter from step to step, and the
    rollout amplifies rounding: the FP64 oracle itself, started from
    positions moved by the FP32 offset resolution (u times the cell edge),
    ends ~1e-3 of max |v| away from its unperturbed run.  The GPU's rollout
    is held to 3x the largest such divergence of three perturbed oracle
    runs (and to the plain bar where that is larger)."""
    N = nauticle()
    case = CASES["dem"]
    steps = 150
    prob = N.Problem([case], max_nbr=64)
    st = prob.state_from_cases()
    attrs = prob.law_attrs()
    prob.step_law(st, attrs, steps)
    torch.cuda.synchronize()
    prob.check()
    n = case.n
    ids = u32(st.id)[:n]
    x_g = np.empty((n, case.dim))
    v_g = np.empty((n, case.dim))
    x_g[ids] = case_absolute_from_state(case, u32(st.cell)[:n], stack(st.off, n))
    v_g[ids] = stack(st.vel, n)
    dom, prm = domain_of(case), params_of(case)
    x0, v0 = case.pos.astype(np.float64), case.vel.astype(np.float64)

    def run(x):
        return O.step_law("dem", dom, prm, x, v0, case.radius, case.pmass, case.coef, fixed=case.fixed_mask(),
                          n_steps=steps)
    x, v, _ = run(x0)
    L = float(np.max(case.length()[: case.dim]))
    vmax = np.abs(v).max()
    rng = np.random.default_rng(17)
    sens_x = sens_v = 0.0
    for _ in range(3):
        xp, vp, _ = run(x0 + rng.uniform(-1, 1, x0.shape) * 2.0 ** -24 * case.cell_size[0])
        sens_x = max(sens_x, np.abs(xp - x).max() / L)
        sens_v = max(sens_v, np.abs(vp - v).max() / vmax)
    err_x = np.abs(x_g - x).max() / L
    err_v = np.abs(v_g - v).max() / vmax
    print(f"dem with friction, {steps} steps: err x {err_x:.2e} v {err_v:.2e}; the oracle's own divergence "
          f"under rounding-sized perturbations x {sens_x:.2e} v {sens_v:.2e}")
    assert err_x < max(3 * sens_x, TOL_ROLLOUT) and err_v < max(3 * sens_v, TOL_ROLLOUT)


@pytest.mark.parametrize("name", list(CASES))
def test_step_law_equals_separate_passes_bitwise(name):
    N = nauticle()
    case = CASES[name]
    prob = N.Problem([case], max_nbr=64)
    attrs = prob.law_attrs()
    st0 = prob.state_from_cases()
    st1 = st0.clone()
    prob.step_law(st1, attrs, 1)
    torch.cuda.synchronize()
    a_step = [t.cpu().numpy().copy() for t in prob.fields.acc]
    sorted_ = prob.new_state()
    nxt = prob.new_state()
    prob.build_cells(st0, sorted_)
    prob.interact(attrs, sorted_, nxt)
    torch.cuda.synchronize()
    prob.check()
    for a, b in zip(a_step, prob.fields.acc):
        np.testing.assert_array_equal(a.view(np.uint32), b.cpu().numpy().view(np.uint32))
    n = case.n
    np.testing.assert_array_equal(u32(st1.cell)[:n], u32(nxt.cell)[:n])
    np.testing.assert_array_equal(stack(st1.off, n).view(np.uint32), stack(nxt.off, n).view(np.uint32))
    np.testing.assert_array_equal(stack(st1.vel, n).view(np.uint32), stack(nxt.vel, n).view(np.uint32))


def test_radius_above_h_is_reported():
    """A DEM radius larger than h (contacts could reach past the stencil)
    sets the attribute error, read by nauticle_check."""
    N = nauticle()
    case = CASES["dem"]
    prob = N.Problem([case], max_nbr=64)
    st = prob.state_from_cases()
    attrs = prob.law_attrs()
    attrs.radius[5] = case.h * 1.5
    prob.build_cells(st)
    prob.interact(attrs)
    with pytest.raises(N.NauticleError) as e:
        prob.check()
    assert e.value.status == N.ERR_ATTRIBUTE


def test_pair_law_entry_points_refuse_other_tables():
    N = nauticle()
    lat = WL.periodic_2d_4096()
    prob = N.Problem([lat])
    st = prob.state_from_cases()
    prob.build_cells(st)
    z = torch.zeros(prob.n, device="cuda")
    attrs = N.LawAttrs(z, z + 1, z)
    with pytest.raises(N.NauticleError) as e:
        prob.interact(attrs)
    assert e.value.status == N.ERR_INVALID_ARG
    dem = N.Problem([CASES["dem"]], max_nbr=64)
    s2 = dem.state_from_cases()
    with pytest.raises(N.NauticleError) as e:
        dem.step(s2, 1)  # pair-law tables step with step_law
    assert e.value.status == N.ERR_INVALID_ARG
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", list(CASES))
def test_pair_law_steps_are_identical_under_every_tuning(name, tmp_path):
    """The launch shape distributes the work and never changes a value; the
    autotuner times pair-law tables with their own steps and caches a pick."""
    from paper_1710_08259_amd import autotune

    N = nauticle()
    case = CASES[name]
    runs = []
    for t in (N.Tuning(), N.Tuning(block=64), N.Tuning(block=128, persistent=1, groups_per_cu=4)):
        prob = N.Problem([case], max_nbr=64, tuning=t)
        st = prob.state_from_cases()
        prob.step_law(st, prob.law_attrs(), 5)
        torch.cuda.synchronize()
        prob.check()
        runs.append([u32(st.cell)[: case.n], stack(st.off, case.n).view(np.uint32), stack(st.vel, case.n).view(np.uint32)])
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            np.testing.assert_array_equal(a, b)
    best, timings = autotune.tune([case], steps=2, candidates=(N.Tuning(), N.Tuning(block=64)),
                                  cache_path=str(tmp_path / "t.json"), max_nbr=64)
    assert best in timings and autotune.bucket([case]).startswith(f"m{case.model}-")
