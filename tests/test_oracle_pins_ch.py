"""Pins of the oracle's Example 1b (no GPU): the SPH Laplacian sph_L0
(eq. diffop3 as the example discretises it) and the Cahn-Hilliard steps
with the adaptive time step.  Each test names the mistake it catches."""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.oracle_helpers import domain_of, params_of


def _plane_lattice(side=24, hr=1.3):
    """A square lattice in the plane z = 0 of a 3-D periodic box, the kernel
    normalised in 2-D (as Example 1b's surface kernel)."""
    dx = 0.01
    h = hr * dx
    nxy = int(side * dx / (2 * h))
    cs = side * dx / nxy
    g = np.meshgrid((np.arange(side) + 0.5) * dx, (np.arange(side) + 0.5) * dx, indexing="ij")
    x = np.stack([g[0].ravel(), g[1].ravel(), np.full(side * side, 0.5 * cs)], axis=1)
    dom = O.Domain(dim=3, n=(nxy, nxy, 3), cs=(cs, cs, cs), periodic=(False, False, False))
    prm = O.Params(h=h, mass=dx * dx * 1000.0, rho0=1000.0)
    interior = np.all((x[:, :2] > 2.01 * h) & (x[:, :2] < side * dx - 2.01 * h), axis=1)
    return dom, prm, x, interior, dx


def _kappa2(hr):
    """-sum over 2-D lattice vectors u (|u| < 2h) of F_2D(|u|) u_x^2 (dx = 1)."""
    s = 0.0
    for k in itertools.product(range(-6, 7), repeat=2):
        r = math.hypot(*k)
        if 0.0 < r < 2 * hr:
            s += -O.F(2, hr, r) * k[0] ** 2
    return s


def test_laplacian_of_constant_linear_and_quadratic_fields_on_a_plane():
    """L(1) = 0 exactly; L(a x + b y) = 0 and L(x^2) = 2 kappa on interior
    particles, kappa the lattice moment (-> 1).  Catches a wrong sign, a
    missing factor 2 or V = m/rho0, or a 3-D normalisation of the surface
    kernel."""
    dom, prm, x, interior, dx = _plane_lattice()
    n = x.shape[0]
    assert np.all(O.laplacian(dom, prm, x, np.ones(n), kdim=2) == 0.0)
    L = O.laplacian(dom, prm, x, 0.3 * x[:, 0] - 1.2 * x[:, 1], kdim=2)
    assert np.abs(L[interior]).max() < 1e-10
    L = O.laplacian(dom, prm, x, x[:, 0] ** 2, kdim=2)
    kappa = _kappa2(prm.h / dx)
    np.testing.assert_allclose(L[interior], 2.0 * kappa, rtol=1e-9)
    assert abs(kappa - 1.0) < 0.05


def test_laplacian_of_z_on_a_sphere_is_the_laplace_beltrami_value():
    """On a sphere of radius R the surface Laplacian of z is -2 z / R^2 (the
    l = 1 harmonic).  The chord distances bring it in through the sphere's
    curvature alone, so a flat-space or wrongly signed operator fails."""
    case = WL.ch_sphere()
    dom, prm = domain_of(case), params_of(case)
    x = case.pos.astype(np.float64)
    z = x[:, 2]
    L = O.laplacian(dom, prm, x, z, kdim=2)
    lam = -(L @ z) / (z @ z)
    assert lam * 2.0 ** 2 == pytest.approx(2.0, rel=0.05)


def _ch(n_steps=5, c=None, dt=0.003):
    case = WL.ch_sphere(dx=0.14, seed=2)
    dom, prm = domain_of(case), params_of(case)
    x = case.pos.astype(np.float64)
    c0 = case.coef.astype(np.float64) if c is None else c
    return case, dom, prm, x, c0, O.ch_steps(dom, prm, x, c0, 0.0, dt, n_steps)


def test_cahn_hilliard_conserves_the_phase_mass():
    """sum_i c_i V is conserved: the Laplacian's pair terms are antisymmetric.
    A one-sided or non-symmetric operator drifts."""
    case, dom, prm, x, c0, (c, t, dt, mu, cdot) = _ch(n_steps=20)
    assert abs(c.sum() - c0.sum()) < 1e-11 * np.abs(c0).sum()
    assert np.abs(c - c0).max() > 1e-3   # it did evolve
    assert abs(cdot.sum()) < 1e-11 * np.abs(cdot).sum()


def test_cahn_hilliard_pure_phases_are_stationary():
    """c = +-1 everywhere: mu = c^3 - c = 0, so cdot = 0 and c stays; dt then
    goes to its gradient limit 0.1 gamma / (2h)^2."""
    for val in (1.0, -1.0):
        case, dom, prm, x, c0, (c, t, dt, mu, cdot) = _ch(n_steps=3, c=np.full(_ch_n(), val))
        assert np.all(c == val) and np.all(cdot == 0.0) and np.all(mu == 0.0)
        assert dt == pytest.approx(0.1 * prm.law[1] / (4 * prm.h ** 2), rel=1e-15)


def _ch_n():
    return WL.ch_sphere(dx=0.14, seed=2).n


def test_cahn_hilliard_step_follows_the_listed_equations():
    """One step is eq1-eq5 in order: time advances by the old dt; mu from c;
    cdot = D L(mu); c += old dt cdot; then dt = 0.1 min(1/max|cdot|, dt_g)."""
    case, dom, prm, x, c0, (c, t, dt, mu, cdot) = _ch(n_steps=1, dt=0.003)
    D, gamma, fac = prm.law[:3]
    lc = O.laplacian(dom, prm, x, c0, kdim=2)
    mu_ref = c0 ** 3 - c0 - gamma * lc
    np.testing.assert_allclose(mu, mu_ref, rtol=1e-12, atol=1e-12)
    cd = D * O.laplacian(dom, prm, x, mu_ref, kdim=2)
    np.testing.assert_allclose(cdot, cd, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(c, c0 + 0.003 * cd, rtol=1e-12, atol=1e-15)
    assert t == 0.003
    assert dt == pytest.approx(fac * min(1.0 / np.abs(cd).max(), gamma / (4 * prm.h ** 2)), rel=1e-14)
