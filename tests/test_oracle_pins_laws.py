"""Pins of the oracle's pair laws on the shared neighbour loop: the DEM
contact law of Example 2 and the social force model (no GPU).  Each test
names the plausible mistake it catches."""
import math

import numpy as np
import pytest

from oracle import oracle as O

E_STEEL_PAPER = 2.06e6   # the Young modulus as printed in Example 2's table (Pa)
NU = 0.33


def _dem_box(n_cells=(6, 6, 6), cs=0.01, symmetric=True, periodic=False):
    return O.Domain(dim=3, n=n_cells, cs=(cs,) * 3, periodic=(periodic,) * 3,
                    symmetric=(symmetric and not periodic,) * 3)


def _pair(ri, rj, mi, mj, Ei, Ej, nui, nuj, delta, v_i=(0, 0, 0), v_j=(0, 0, 0), cf=0.0):
    dom = _dem_box(symmetric=False)
    prm = O.Params(h=0.005, mass=1.0, g=(0.0, 0.0, 0.0), law=(cf,))
    dist = ri + rj - delta
    x = np.array([[0.03, 0.03, 0.03], [0.03 + dist, 0.03, 0.03]])
    v = np.array([v_i, v_j], dtype=float)
    R = np.array([ri, rj])
    m = np.array([mi, mj])
    q = np.array([(1 - nui ** 2) / Ei, (1 - nuj ** 2) / Ej])
    return O.dem(dom, prm, x, v, R, m, q)


def _hertz(ri, rj, mi, mj, Ei, Ej, nui, nuj):
    """Stiffness and damping coefficient, computed by hand from the printed
    effective quantities (E' as the printed fraction, not via q)."""
    Rs = ri * rj / (ri + rj)
    ms = mi * mj / (mi + mj)
    Es = Ei * Ej / (Ej * (1 - nui ** 2) + Ei * (1 - nuj ** 2))
    k = 4.0 / 3.0 * math.sqrt(Rs) * Es
    return k, math.sqrt(ms * k) / 8.0


def test_dem_static_overlap_is_hertzian_and_repulsive():
    """Two unlike spheres (radii, masses and materials differ) overlapping by
    delta: the force is k delta^(3/2) along the line of centres, pushing
    them apart, equal and opposite.  Catches a wrong effective radius, mass
    or modulus, a wrong exponent, or an attractive sign."""
    args = (0.004, 0.003, 2.1e-3, 0.9e-3, 2.06e6, 3.1e6, 0.33, 0.25)
    for delta in (1e-5, 2e-4, 6e-4):
        a = _pair(*args, delta=delta)
        k, _ = _hertz(*args)
        f = k * delta ** 1.5
        np.testing.assert_allclose(a[0], [-f / args[2], 0, 0], rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(a[1], [f / args[3], 0, 0], rtol=1e-12, atol=1e-300)


def test_dem_no_force_without_contact():
    a = _pair(0.004, 0.004, 2e-3, 2e-3, 2e6, 2e6, 0.3, 0.3, delta=-1e-4, v_i=(1, 2, 3))
    assert np.all(a == 0.0)


@pytest.mark.parametrize("u", [0.3, -0.3])
def test_dem_damping_grows_with_the_approach_rate(u):
    """Sphere 1 moving towards (u > 0) or away from (u < 0) sphere 2:
    f_n = k delta^(3/2) + c delta^(1/4) u, c = sqrt(m' k) / 8."""
    args = (0.004, 0.004, 2.1e-3, 2.1e-3, 2.06e6, 2.06e6, 0.33, 0.33)
    delta = 3e-4
    a = _pair(*args, delta=delta, v_i=(u, 0, 0))
    k, c = _hertz(*args)
    fn = k * delta ** 1.5 + c * delta ** 0.25 * u
    np.testing.assert_allclose(a[0, 0], -fn / args[2], rtol=1e-12)
    np.testing.assert_allclose(a[1, 0], fn / args[3], rtol=1e-12)


def test_dem_friction_drags_along_the_relative_tangential_motion():
    """Sphere 2 sliding past sphere 1 along +y: on 1 a tangential force
    c_f |f_n| along +y (dragged along), on 2 along -y; normal part as in the
    static test.  Catches a friction force against the wrong velocity or
    with the wrong magnitude."""
    args = (0.004, 0.004, 2.1e-3, 2.1e-3, 2.06e6, 2.06e6, 0.33, 0.33)
    delta = 3e-4
    cf = 0.4
    a = _pair(*args, delta=delta, v_j=(0, 0.7, 0), cf=cf)
    k, _ = _hertz(*args)
    fn = k * delta ** 1.5
    np.testing.assert_allclose(a[0], [-fn / args[2], cf * fn / args[2], 0], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(a[1], [fn / args[3], -cf * fn / args[3], 0], rtol=1e-12, atol=1e-300)


def test_dem_pair_forces_conserve_momentum():
    """Random overlapping packing in a periodic box, unlike radii and
    masses: sum_i m_i a_i = N-weighted gravity (Newton's third law for the
    normal, damping and friction parts)."""
    rng = np.random.default_rng(3)
    dom = _dem_box(n_cells=(5, 5, 5), cs=0.01, periodic=True)
    n = 300
    x = rng.uniform(0, 0.05, (n, 3))
    v = rng.normal(0, 0.2, (n, 3))
    R = rng.uniform(0.003, 0.005, n)
    m = 7850 * 4 / 3 * np.pi * R ** 3
    q = (1 - rng.uniform(0.2, 0.4, n) ** 2) / rng.uniform(1e6, 3e6, n)
    prm = O.Params(h=0.005, mass=1.0, g=(0.0, 0.0, -9.81), law=(0.3,))
    a = O.dem(dom, prm, x, v, R, m, q)
    F = (m[:, None] * (a - np.array(prm.g)))
    assert np.abs(F).sum() > 0
    assert np.abs(F.sum(0)).max() < 1e-11 * np.abs(F).sum()


def test_dem_sphere_rests_on_a_symmetric_floor_at_the_hertz_height():
    """A sphere touching the floor meets its own mirror image (R' = R/2,
    m' = m/2, overlap 2R - 2z).  At the height z* where k (2R - 2z*)^(3/2) =
    m g it is in equilibrium; lower it is pushed up, never sideways."""
    dom = _dem_box(n_cells=(6, 6, 6), cs=0.01)
    R, rho = 0.004, 7850.0
    m = rho * 4 / 3 * np.pi * R ** 3
    q = (1 - NU ** 2) / E_STEEL_PAPER
    prm = O.Params(h=0.005, mass=m, g=(0.0, 0.0, -9.81), law=(0.3,))
    k = 4.0 / 3.0 * math.sqrt(R / 2) * (1.0 / (2 * q))
    overlap = (m * 9.81 / k) ** (2.0 / 3.0)
    z = R - overlap / 2
    x = np.array([[0.031, 0.027, z]])
    a = O.dem(dom, prm, x, np.zeros((1, 3)), [R], [m], [q])
    assert abs(a[0, 2]) < 1e-9 * 9.81 and a[0, 0] == 0.0 and a[0, 1] == 0.0
    a = O.dem(dom, prm, x - [0, 0, 1e-5], np.zeros((1, 3)), [R], [m], [q])
    assert a[0, 2] > 0


def test_dem_bounce_loses_energy():
    """A sphere dropped on the symmetric floor bounces back (the contact is
    repulsive) lower than it fell (the damping term dissipates)."""
    dom = _dem_box(n_cells=(4, 4, 12), cs=0.01)
    R = 0.004
    m = 7850 * 4 / 3 * np.pi * R ** 3
    q = (1 - NU ** 2) / E_STEEL_PAPER
    prm = O.Params(h=0.005, mass=m, g=(0.0, 0.0, -9.81), dt=2e-6, law=(0.0,))
    x = np.array([[0.02, 0.02, R + 0.002]])
    v = np.zeros((1, 3))
    top = []
    for _ in range(30):
        x, v, _ = O.step_law("dem", dom, prm, x, v, [R], [m], [q], n_steps=1000)
        top.append((x[0, 2], v[0, 2]))
    zs = np.array([t[0] for t in top])
    vz = np.array([t[1] for t in top])
    assert (vz > 0).any()                       # it came back up
    assert zs.max() < R + 0.002                 # but not as high
    assert zs.min() > R - 0.002                 # and never fell through


def _social_case():
    dom = O.Domain(dim=2, n=(10, 10, 1), cs=(1.0, 1.0, 1.0), periodic=(False,) * 3)
    prm = O.Params(h=0.5, mass=1.0, g=(0.0, 0.0, 0.0), law=(2000.0, 0.08, 1.2e5, 0.5))
    return dom, prm


def test_social_isolated_person_relaxes_towards_the_goal():
    """No neighbour: a = (v0 e0 - v) / tau with e0 pointing at the goal."""
    dom, prm = _social_case()
    x = np.array([[2.0, 3.0]])
    v = np.array([[0.2, -0.1]])
    goal = np.array([[5.0, 7.0]])
    a = O.social(dom, prm, x, v, [0.3], [70.0], [0.0], [1.3], goal)
    e0 = np.array([3.0, 4.0]) / 5.0
    np.testing.assert_allclose(a[0], (1.3 * e0 - v[0]) / 0.5, rtol=1e-14)


@pytest.mark.parametrize("d", [0.45, 0.7])
def test_social_pair_term_closed_form(d):
    """Two people at rest with no desired speed (v0 = 0):
    a_1 = -(1/m_1) [A exp((R_12 - d)/B) + k max(R_12 - d, 0) - c_12] n_12,
    c_12 the mean of c_1 and c_2; the body force only when they touch
    (d < R_1 + R_2 = 0.55).  Catches a body force without contact, a wrong
    exponent sign, or c not averaged."""
    dom, prm = _social_case()
    x = np.array([[3.0, 3.0], [3.0 + d, 3.0]])
    R = np.array([0.3, 0.25])
    m = np.array([70.0, 55.0])
    c = np.array([40.0, 10.0])
    a = O.social(dom, prm, x, np.zeros((2, 2)), R, m, c, [0.0, 0.0], x)
    A, B, k = prm.law[:3]
    s = A * math.exp((0.55 - d) / B) + (k * (0.55 - d) if d < 0.55 else 0.0) - 25.0
    np.testing.assert_allclose(a[0], [-s / m[0], 0.0], rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(a[1], [s / m[1], 0.0], rtol=1e-13, atol=1e-300)


def test_social_pair_terms_cancel_and_walls_stay():
    """Random crowd: the pair forces are equal and opposite, so
    sum_i m_i (a_i - relaxation_i) = 0; with some people fixed (walls), those
    get a = 0."""
    rng = np.random.default_rng(9)
    dom, prm = _social_case()
    n = 200
    x = rng.uniform(0.5, 9.5, (n, 2))
    R = 0.002 * rng.uniform(50, 100, n) + 0.15
    m = (R - 0.15) / 0.002
    c = rng.uniform(0, 50, n)
    v = rng.normal(0, 0.5, (n, 2))
    v0 = rng.uniform(0.6, 1.5, n)
    goal = rng.uniform(0, 10, (n, 2))
    a = O.social(dom, prm, x, v, R, m, c, v0, goal)
    e = goal - x
    own = (v0[:, None] * e / np.linalg.norm(e, axis=1)[:, None] - v) / prm.law[3]
    F = m[:, None] * (a - own)
    assert np.abs(F).sum() > 0
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).sum()
    fixed = np.zeros(n, np.uint8)
    fixed[:20] = 1
    a = O.social(dom, prm, x, v, R, m, c, v0, goal, fixed=fixed)
    assert np.all(a[:20] == 0.0)


def test_dem_sphere_sliding_on_a_symmetric_floor_feels_no_friction():
    """A sphere pressed into the floor and sliding along it meets its own
    image, whose velocity differs only in the normal component: v_t = 0, so
    the symmetric face is frictionless (free slip), whatever c_f."""
    dom = _dem_box(n_cells=(6, 6, 6), cs=0.01)
    R = 0.004
    m = 7850 * 4 / 3 * np.pi * R ** 3
    q = (1 - NU ** 2) / E_STEEL_PAPER
    prm = O.Params(h=0.005, mass=m, g=(0.0, 0.0, 0.0), law=(0.8,))
    x = np.array([[0.031, 0.027, R - 2e-4]])
    v = np.array([[0.7, -0.3, -0.2]])
    a = O.dem(dom, prm, x, v, [R], [m], [q])
    assert a[0, 0] == 0.0 and a[0, 1] == 0.0 and a[0, 2] > 0
