"""Pins of the oracle's symmetric (mirror) faces and of Example 1a's operator
set (continuity, linear equation of state, momentum with the artificial
viscosity Pi_ij, the eq1..eq7 step), against facts that the paper and the
mathematics fix (no GPU).  Each test says which plausible mistake it would
catch."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.oracle_helpers import domain_of, params_of


def _mirror_layout(dim, boundary, seed, n=500, on_face=True):
    """Random particles in a box with symmetric faces, crowded near the faces
    and corners (a third of them within 2h of a face, some exactly on one),
    with random velocities and densities."""
    rng = np.random.default_rng(seed)
    h = 0.02
    ncell = (6, 5, 4)[:dim] + (1,) * (3 - dim)
    cs = tuple(float(np.float32(2.0 * h * 1.07)) for _ in range(dim)) + (1.0,) * (3 - dim)
    L = np.array([ncell[k] * cs[k] for k in range(3)])
    x = rng.uniform(0, 1, (n, dim)) * L[:dim]
    near = rng.random(n) < 0.35
    for k in range(dim):
        side = rng.random(n) < 0.5
        d = rng.uniform(0, 2.0 * h, n)
        pick = near & (rng.random(n) < 0.6)
        x[pick & side, k] = d[pick & side]
        x[pick & ~side, k] = L[k] - d[pick & ~side]
    if on_face:
        x[:3, 0] = 0.0  # exactly on the lower x face: their own image coincides
    x = np.clip(x, 0.0, np.nextafter(L[:dim], 0)).astype(np.float32).astype(np.float64)
    dom = O.Domain(dim=dim, n=ncell, cs=cs, origin=(0.0, 0.0, 0.0),
                   periodic=tuple(b == WL.PERIODIC for b in boundary),
                   symmetric=tuple(b == WL.SYMMETRIC for b in boundary))
    prm = O.Params(h=h, mass=1000.0 * (0.8 * h) ** dim, rho0=1000.0, c0=20.0, gamma=7.0, nu=1e-3,
                   dt=1e-4, g=(0.0, -9.81, 0.0)[:dim] + (0.0,) * (3 - dim), alpha_av=0.1)
    v = rng.normal(0, 0.5, (n, dim))
    rho = 1000.0 * (1.0 + 0.02 * rng.standard_normal(n))
    return dom, prm, x, v, rho


_MIRROR_CASES = [
    (2, (WL.SYMMETRIC, WL.SYMMETRIC, WL.CUTOFF), 1),
    (3, (WL.SYMMETRIC, WL.CUTOFF, WL.SYMMETRIC), 2),
    (3, (WL.SYMMETRIC, WL.PERIODIC, WL.SYMMETRIC), 3),
    (2, (WL.PERIODIC, WL.SYMMETRIC, WL.CUTOFF), 4),
]


def _doubled(dom, x, v, rho):
    """The box doubled across the lower face of every symmetric axis, with
    the particles' mirror copies (positions reflected, normal velocity
    reversed) and periodic faces on the doubled axes."""
    axes = [k for k in range(dom.dim) if dom.symmetric[k]]
    xs, vs, rs = [], [], []
    for flips in itertools.product((False, True), repeat=len(axes)):
        xc, vc = x.copy(), v.copy()
        for k, f in zip(axes, flips):
            if f:
                xc[:, k] = 2.0 * dom.origin[k] - xc[:, k]
                vc[:, k] = -vc[:, k]
        xs.append(xc)
        vs.append(vc)
        rs.append(rho)
    n = list(dom.n)
    origin = list(dom.origin)
    periodic = list(dom.periodic)
    for k in axes:
        n[k] *= 2
        origin[k] = dom.origin[k] - dom.n[k] * dom.cs[k]
        periodic[k] = True
    big = O.Domain(dim=dom.dim, n=tuple(n), cs=dom.cs, origin=tuple(origin), periodic=tuple(periodic),
                   symmetric=(False, False, False))
    return big, np.concatenate(xs), np.concatenate(vs), np.concatenate(rs)


@pytest.mark.parametrize("dim,boundary,seed", _MIRROR_CASES)
def test_symmetric_faces_equal_the_doubled_periodic_box(dim, boundary, seed):
    """A box with symmetric faces is the periodic box twice as long, filled
    with the particles and their mirror copies: every operator must agree on
    the original particles.  Catches a wrong image position, an unreflected
    or wrongly reflected velocity, a missed corner image, a dropped
    self-image, or an image counted twice."""
    dom, prm, x, v, rho = _mirror_layout(dim, boundary, seed)
    big, X, V, R = _doubled(dom, x, v, rho)
    n = x.shape[0]
    orig = np.arange(n)

    r_s, p_s, c_s = O.density(dom, prm, x, counts=True)
    r_b, p_b, c_b = O.density(big, prm, X, which=orig, counts=True)
    np.testing.assert_array_equal(c_s, c_b)
    assert (c_s > 0).all()
    np.testing.assert_allclose(r_s, r_b, rtol=1e-13)

    P_b = np.concatenate([p_s] * (X.shape[0] // n))
    Rs_b = np.concatenate([r_s] * (X.shape[0] // n))
    a_s = O.forces(dom, prm, x, v, r_s, p_s)
    a_b = O.forces(big, prm, X, V, Rs_b, P_b, which=orig)
    scale = np.abs(a_s).max()
    np.testing.assert_allclose(a_s, a_b, rtol=0, atol=1e-12 * scale)

    d_s = O.continuity(dom, prm, x, v, rho)
    d_b = O.continuity(big, prm, X, V, R, which=orig)
    np.testing.assert_allclose(d_s, d_b, rtol=0, atol=1e-12 * np.abs(d_s).max())
    assert np.abs(d_s).max() > 0

    p = np.array([O.linear_eos(prm, r) for r in rho])
    m_s = O.momentum(dom, prm, x, v, rho, p)
    m_b = O.momentum(big, prm, X, V, R, np.concatenate([p] * (X.shape[0] // n)), which=orig)
    np.testing.assert_allclose(m_s, m_b, rtol=0, atol=1e-12 * np.abs(m_s).max())


@pytest.mark.parametrize("dim,boundary,seed", _MIRROR_CASES)
def test_fp32_mirror_lists_cell_grid_equal_brute_force(dim, boundary, seed):
    """The cell-grid FP32 lists (a cell beyond a symmetric face standing for
    the boundary cell's image) count exactly what the brute force over every
    particle and every one of its reflections finds."""
    dom, prm, x, _, _ = _mirror_layout(dim, boundary, seed)
    cell, off = O.bin_f32(dom, x.astype(np.float32))
    grid = O.neighbours_f32(dom, prm.h, cell, off)
    brute = O.neighbours_f32(dom, prm.h, cell, off, brute=True)
    np.testing.assert_array_equal(grid, brute)


@pytest.mark.parametrize("dim,boundary,seed", _MIRROR_CASES)
def test_fp32_mirror_lists_match_exact_image_distances(dim, boundary, seed):
    """Every (neighbour, reflected axes) entry of the FP32 lists is an image
    within 2h of the particle in exact arithmetic on the absolute positions,
    and every such image is listed, except pairs within 1e-5 of the cut-off.
    Pins the FP32 image arithmetic (-off_j against the particle shifted by 0
    or 2 cells) against geometry."""
    dom, prm, x, _, _ = _mirror_layout(dim, boundary, seed)
    x32 = x.astype(np.float32)
    cell, off = O.bin_f32(dom, x32)
    cnt, lst, mir = O.neighbours_f32(dom, prm.h, cell, off, max_nbr=256, mirrors=True)
    L = np.array([dom.n[k] * dom.cs[k] for k in range(3)])
    X = x32.astype(np.float64)
    R = 2.0 * prm.h
    axes = [k for k in range(dim) if dom.symmetric[k]]
    n = X.shape[0]
    for i in range(n):
        got = {(int(j), int(m)) for j, m in zip(lst[i, : cnt[i]], mir[i, : cnt[i]])}
        assert len(got) == cnt[i]  # no entry twice
        want, near = set(), set()
        for choice in itertools.product((0, 1, 2), repeat=len(axes)):
            Y = X.copy()
            mask = 0
            for k, c in zip(axes, choice):
                if c == 1:
                    Y[:, k] = -Y[:, k]
                elif c == 2:
                    Y[:, k] = 2.0 * L[k] - Y[:, k]
                if c:
                    mask |= 1 << k
            d = Y - X[i]
            for k in range(dim):
                if dom.periodic[k]:
                    d[:, k] -= L[k] * np.rint(d[:, k] / L[k])
            r = np.sqrt((d ** 2).sum(1))
            for j in np.nonzero(r < R * (1 + 1e-5))[0]:
                if j == i and mask == 0:
                    continue
                (near if abs(r[j] - R) < 1e-5 * R else want).add((int(j), mask))
        assert want <= got, (i, want - got)
        assert got <= want | near, (i, got - want - near)


def _cutoff_lattice(dim, side, hr=1.3):
    case = WL.lattice_case(dim, side, 0.01, hr, 0.0, 0.0, seed=0)
    case = WL.scaled(case, boundary=(WL.CUTOFF,) * 3)
    sp = [case.length()[k] / side[k] for k in range(dim)]
    grids = np.meshgrid(*[(np.arange(side[k]) + 0.5) * sp[k] for k in range(dim)], indexing="ij")
    x = np.stack([g.ravel(order="F") for g in grids], axis=1)
    L = case.length()[:dim]
    interior = np.all((x > 2.01 * case.h) & (x < L - 2.01 * case.h), axis=1)
    return case, x, interior, sp[0]


def _lattice_kappa(dim, h_over_dx):
    """kappa = -sum over lattice vectors u (|u| < 2h) of F(|u|) u_x^2, times
    the cell volume (dx = 1): the lattice's second gradient moment, which the
    continuous kernel makes exactly 1."""
    h = h_over_dx
    rng = range(-3 * int(h) - 2, 3 * int(h) + 3)
    s = 0.0
    for k in itertools.product(rng, repeat=dim):
        r = float(np.sqrt(sum(c * c for c in k)))
        if 0.0 < r < 2 * h:
            s += -O.F(dim, h, r) * k[0] ** 2
    return s


@pytest.mark.parametrize("dim,side", [(2, (24, 24)), (3, (12, 12, 12))])
def test_continuity_of_a_linear_velocity_field_is_minus_rho0_kappa_trace(dim, side):
    """v = A x on a regular lattice at uniform density: every interior
    particle gets drho/dt = -rho0 kappa tr(A), kappa the lattice's gradient
    moment (-> 1 as h/dx grows, i.e. drho/dt = -rho div v).  Catches a wrong
    sign, a missing m/rho_j weight, or a wrong vector in the dot product."""
    case, x, interior, dx = _cutoff_lattice(dim, side)
    dom, prm = domain_of(case), params_of(case)
    A = np.array([[0.7, -0.3, 0.2], [0.4, -1.1, 0.5], [0.1, 0.6, 0.25]])[:dim, :dim]
    v = x @ A.T
    rho = np.full(case.n, 1015.0)  # uniform but not rho0: m/rho_j and rho_i cancel
    drho = O.continuity(dom, prm, x, v, rho)
    kappa = _lattice_kappa(dim, case.h / dx)
    expect = -prm.rho0 * kappa * np.trace(A)
    np.testing.assert_allclose(drho[interior], expect, rtol=1e-9)
    assert abs(kappa - 1.0) < 0.05


def test_continuity_vanishes_for_rigid_motion():
    """A rigid translation plus rotation has no divergence and no pair has
    (v_j - v_i) . r_ij != 0: drho/dt = 0 for every particle, boundary ones
    too, at any density field."""
    case, x, _, _ = _cutoff_lattice(2, (20, 18))
    dom, prm = domain_of(case), params_of(case)
    rng = np.random.default_rng(5)
    xj = x + rng.uniform(-0.2, 0.2, x.shape) * 0.01
    omega = 3.0
    v = np.array([0.4, -0.25]) + omega * np.stack([-xj[:, 1], xj[:, 0]], axis=1)
    rho = 1000.0 * (1.0 + 0.05 * rng.standard_normal(case.n))
    drho = O.continuity(dom, prm, xj, v, rho)
    scale = prm.rho0 * omega * 10
    assert np.abs(drho).max() < 1e-11 * scale


def _pair(u, wy, rho1=1000.0, rho2=1100.0, p1=0.0, p2=0.0):
    h = 0.02
    dom = O.Domain(dim=2, n=(6, 6, 1), cs=(0.05, 0.05, 1.0), periodic=(False, False, False))
    prm = O.Params(h=h, mass=0.4, rho0=1000.0, c0=50.0, gamma=1.0, nu=0.0, alpha_av=0.1,
                   g=(0.0, 0.0, 0.0))
    x = np.array([[0.12, 0.13], [0.12 + h, 0.13]])  # r_12 = (-h, 0), q = 1
    v = np.array([[u, 0.0], [0.0, wy]])
    rho = np.array([rho1, rho2])
    p = np.array([p1, p2])
    return dom, prm, x, v, rho, p


@pytest.mark.parametrize("u", [0.8, -0.8])
def test_two_particle_closed_forms(u):
    """Two particles a distance h apart along x, particle 1 moving along x
    at u (approaching when u > 0), particle 2 moving across at wy, densities
    1000 and 1100.  By hand, with F = F(h) < 0 and r_12 = (-h, 0):
      drho_1 = -rho_1 u h F m / rho_2,   drho_2 = -rho_2 u h F m / rho_1
      (compression while approaching);
      Pi_12 = alpha c u / rho_1 and Pi_21 = alpha c u / rho_2 when u > 0,
      else 0 (Pi uses rho_i, not a mean), so
      a_1 = (alpha c u h m F / rho_1, 0),  a_2 = (-alpha c u h m F / rho_2, 0);
    and with pressures only, a_1 = (p1/rho1^2 + p2/rho2^2) m F h (x axis)."""
    dom, prm, x, v, rho, p = _pair(u, 0.37)
    h, m, c = prm.h, prm.mass, prm.c0
    F = O.F(2, h, h)
    assert F < 0
    drho = O.continuity(dom, prm, x, v, rho)
    np.testing.assert_allclose(drho, [-rho[0] * u * h * F * m / rho[1], -rho[1] * u * h * F * m / rho[0]],
                               rtol=1e-13)
    a = O.momentum(dom, prm, x, v, rho, p)
    if u > 0:
        expect = np.array([[0.1 * c * u * h * m * F / rho[0], 0.0], [-0.1 * c * u * h * m * F / rho[1], 0.0]])
        assert a[0, 0] < 0 < a[1, 0]  # the approaching pair is braked and pushed apart
    else:
        expect = np.zeros((2, 2))
    np.testing.assert_allclose(a, expect, rtol=1e-13, atol=1e-300)
    dom, prm, x, v, rho, p = _pair(0.0, 0.0, p1=2000.0, p2=500.0)
    a = O.momentum(dom, prm, x, v, rho, p)
    s = p[0] / rho[0] ** 2 + p[1] / rho[1] ** 2
    np.testing.assert_allclose(a[0], [s * m * F * h, 0.0], rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(a[1], [-s * m * F * h, 0.0], rtol=1e-13, atol=1e-300)
    assert a[0, 0] < 0  # positive pressure pushes particle 1 (the left one) to -x


def test_artificial_viscosity_dissipates_and_conserves_momentum_at_uniform_density():
    """At uniform density the Pi_ij terms are equal and opposite (sum of m a
    is N m g) and their power sum_i m v_i . a_i is negative; with p = 0 the
    pressure terms vanish, so this isolates Pi."""
    case = WL.lattice_case(2, (18, 16), 0.01, 1.3, 0.2, 0.5, seed=21, g=(0.0, -9.81, 0.0))
    dom, prm = domain_of(case), params_of(case)
    prm.alpha_av = 0.1
    x = case.pos.astype(np.float64)
    v = case.vel.astype(np.float64)
    rho = np.full(case.n, 1000.0)
    a = O.momentum(dom, prm, x, v, rho, np.zeros(case.n))
    g = np.array(case.g[:2])
    total = case.mass * (a - g).sum(0)
    assert np.abs(total).max() < 1e-11 * case.mass * np.abs(a - g).sum()
    power = case.mass * ((a - g) * v).sum()
    assert power < 0.0
    prm.alpha_av = 0.0
    a0 = O.momentum(dom, prm, x, v, rho, np.zeros(case.n))
    np.testing.assert_allclose(a0, np.broadcast_to(g, a0.shape), rtol=0, atol=0)


def test_linear_equation_of_state():
    prm = O.Params(h=0.25, mass=1.0, rho0=1000.0, c0=50.0)
    assert O.linear_eos(prm, 1000.0) == 0.0
    assert O.linear_eos(prm, 1001.0) == pytest.approx(2500.0, rel=1e-15)
    assert O.linear_eos(prm, 990.0) == pytest.approx(-25000.0, rel=1e-15)


def test_ex1a_isolated_particle_closed_form():
    """One particle far from every face: no neighbour and no image, so its
    density stays, p = c^2 (rho - rho0), a = g and (x, v) follow the
    semi-implicit Euler closed form."""
    dom = O.Domain(dim=2, n=(8, 8, 1), cs=(0.5, 0.5, 1.0), periodic=(False, False, False),
                   symmetric=(True, True, False))
    prm = O.Params(h=0.25, mass=51.6, rho0=1000.0, c0=50.0, dt=1e-3, g=(0.0, -9.81, 0.0), alpha_av=0.1)
    x0 = np.array([[2.1, 2.3]])
    v0 = np.array([[0.3, -0.2]])
    n = 12
    x, v, rho, drho, p, a = O.step_ex1a(dom, prm, x0, v0, np.array([1003.0]), n_steps=n)
    assert rho[0] == 1003.0 and drho[0] == 0.0
    assert p[0] == pytest.approx(2500.0 * 3.0, rel=1e-12)
    g = np.array(prm.g[:2])
    np.testing.assert_allclose(a[0], g, rtol=1e-15)
    np.testing.assert_allclose(v[0], v0[0] + n * prm.dt * g, rtol=1e-13)
    np.testing.assert_allclose(x[0], x0[0] + n * prm.dt * v0[0] + prm.dt ** 2 * g * n * (n + 1) / 2,
                               rtol=1e-12)


def test_particle_at_a_face_is_pushed_back_by_its_image():
    """A particle at rest near a symmetric face, above rho0 (positive
    pressure), is repelled by its own mirror image: its acceleration points
    away from the face and is exactly normal to it."""
    dom = O.Domain(dim=2, n=(8, 8, 1), cs=(0.5, 0.5, 1.0), periodic=(False, False, False),
                   symmetric=(True, True, False))
    prm = O.Params(h=0.25, mass=51.6, rho0=1000.0, c0=50.0, g=(0.0, 0.0, 0.0), alpha_av=0.1)
    x = np.array([[0.2, 2.0]])
    rho = np.array([1010.0])
    p = np.array([O.linear_eos(prm, 1010.0)])
    a = O.momentum(dom, prm, x, np.zeros_like(x), rho, p)
    assert a[0, 0] > 0 and a[0, 1] == 0.0
    # approaching the face: its image approaches too, Pi brakes the motion
    a = O.momentum(dom, prm, x, np.array([[-1.0, 0.0]]), np.array([1000.0]), np.zeros(1))
    assert a[0, 0] > 0 and a[0, 1] == 0.0
    # sliding along the face: free slip, no tangential drag from the image
    a = O.momentum(dom, prm, x, np.array([[0.0, 1.0]]), np.array([1000.0]), np.zeros(1))
    assert a[0, 0] == 0.0 and a[0, 1] == 0.0


def test_ex1a_step_takes_the_equations_in_the_papers_order():
    """One step is eq1 (drho from the old state), eq2 (rho updated), eq3 (p
    from the NEW rho), eq4-5 (a from the new rho and p, old x and v), eq6
    (v), eq7 (x with the new v).  Using the old rho in the momentum
    equation, or the old v in eq7, fails this."""
    case = WL.ex1a_dam_break(scale=2.0)
    dom, prm = domain_of(case), params_of(case)
    x0 = case.pos.astype(np.float64)
    rng = np.random.default_rng(8)
    v0 = rng.normal(0, 0.3, x0.shape)
    rho0 = 1000.0 * (1.0 + 0.01 * rng.standard_normal(case.n))
    x1, v1, rho1, drho, p1, a = O.step_ex1a(dom, prm, x0, v0, rho0, n_steps=1)
    d = O.continuity(dom, prm, x0, v0, rho0)
    np.testing.assert_allclose(drho, d, rtol=1e-15)
    r = rho0 + prm.dt * d
    np.testing.assert_allclose(rho1, r, rtol=1e-15)
    pp = prm.c0 ** 2 * (r - prm.rho0)
    np.testing.assert_allclose(p1, pp, rtol=1e-12, atol=1e-12 * np.abs(pp).max())
    am = O.momentum(dom, prm, x0, v0, r, pp)
    np.testing.assert_allclose(a, am, rtol=1e-12, atol=1e-12 * np.abs(am).max())
    np.testing.assert_allclose(v1, v0 + prm.dt * am, rtol=1e-13, atol=1e-15)
    # particles pushed across a face are shifted periodically (Sec. 3.2.1)
    L = case.length()[:2]
    np.testing.assert_allclose(x1, np.mod(x0 + prm.dt * (v0 + prm.dt * am), L), rtol=1e-13, atol=1e-12)


def test_ex1a_dam_break_column_starts_to_collapse():
    """The paper's configuration after 50 steps: the column has sunk and
    spread along the floor (mean velocity down, the right edge moving out),
    no particle has left the box, and the density stays within a few per
    cent of rho0 (weak compressibility at c = 50 m/s)."""
    case = WL.ex1a_dam_break()
    dom, prm = domain_of(case), params_of(case)
    x0 = case.pos.astype(np.float64)
    x, v, rho, _, _, _ = O.step_ex1a(dom, prm, x0, np.zeros_like(x0), case.rho.astype(np.float64),
                                     n_steps=50)
    L = case.length()[:2]
    assert np.all(x >= 0) and np.all(x < L)
    assert v[:, 1].mean() < 0
    right = x0[:, 0] > x0[:, 0].max() - 0.3
    assert v[right, 0].mean() > 0
    assert np.abs(rho / prm.rho0 - 1).max() < 0.05


def test_step_vjp_refuses_symmetric_faces():
    dom, prm, x, v, _ = _mirror_layout(2, (WL.SYMMETRIC, WL.SYMMETRIC, WL.CUTOFF), 1, n=50)
    with pytest.raises(ValueError):
        O.step_vjp(dom, prm, x, v, np.zeros_like(x), np.zeros_like(x))
