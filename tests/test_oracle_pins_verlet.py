"""Pins of the oracle's Verlet-list rollout (neighbour lists reused between
builds; the paper reruns the search only when the layout has changed,
Sec. 4).

- pair_keys, the pair set the lists are checked with, against a plain loop
  over pairs and reflections on a tiny case with a periodic and a symmetric
  axis;
- the rollout with the list equals the plain rollout bit for bit (the steps
  never read the list), skips builds on a lively case, and never finds a
  pair inside 2h missing from the list;
- the displacement rule is what keeps the list whole: two particles
  approaching head-on from just beyond 2h + skin are caught by the rule at
  half the skin, and a rule at the full skin (a planted mistake) lets them
  into the support unlisted;
- with skin 0 every step of a moving system builds."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.oracle_helpers import domain_of, params_of


def _loop_keys(dom, x, radius):
    n, d = x.shape
    L = dom.length()
    keys = set()
    choices = [(0, 1, 2) if dom.symmetric[k] else (0,) for k in range(d)]
    for combo in itertools.product(*choices):
        code = sum(c * 3 ** k for k, c in enumerate(combo))
        for i in range(n):
            for j in range(n):
                if i == j and code == 0:
                    continue
                r2 = 0.0
                for k in range(d):
                    xj = x[j, k]
                    if combo[k] == 1:
                        xj = 2.0 * dom.origin[k] - xj
                    elif combo[k] == 2:
                        xj = 2.0 * (dom.origin[k] + L[k]) - xj
                    t = xj - x[i, k]
                    if dom.periodic[k]:
                        t -= L[k] * round(t / L[k])
                    r2 += t * t
                if r2 < radius * radius:
                    keys.add((i * n + j) * 27 + code)
    return np.array(sorted(keys), dtype=np.int64)


def test_pair_keys_equal_a_loop_over_pairs_and_reflections():
    dom = O.Domain(dim=2, n=(4, 3, 1), cs=(0.1, 0.1, 1.0), periodic=(True, False, False),
                   symmetric=(False, True, False))
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 1.0, (40, 2)) * np.array([0.4, 0.3])
    x[0] = [0.005, 0.004]    # near a periodic seam and a symmetric face: its own reflection counts
    x[1] = [0.395, 0.2995]
    keys = O.pair_keys(dom, x, 0.09)
    np.testing.assert_array_equal(keys, _loop_keys(dom, x, 0.09))
    assert np.any(keys % 27 != 0) and np.any(keys // 27 % 40 == keys // 27 // 40)  # images, self-images


def _lively_2d(skin):
    return WL.lattice_case(2, (24, 24), 0.01, 1.3, 0.05, 0.5, seed=9, c0=10.0, skin=skin)


def test_verlet_rollout_is_the_plain_rollout_and_skips_builds():
    c = _lively_2d(0.004)
    dom, prm = domain_of(c), params_of(c)
    steps = 40
    x, v, _, builds, when = O.verlet_steps(dom, prm, c.pos, c.vel, c.skin, steps)
    x2, v2, _, _, _ = O.step(dom, prm, c.pos.astype(np.float64), c.vel.astype(np.float64), n_steps=steps)
    np.testing.assert_array_equal(x, x2)
    np.testing.assert_array_equal(v, v2)
    assert 1 < builds < steps // 4 and when[0] == 0


def test_continuity_model_with_symmetric_faces():
    c = WL.mirror_box_case(2, (WL.SYMMETRIC, WL.SYMMETRIC, WL.PERIODIC), seed=2, n=300, ncell=(8, 7, 1),
                           model=WL.CONTINUITY)
    c = WL.scaled(c, skin=float(np.float32(min(c.cell_size[:2])) - 2.0 * c.h) * 0.9)
    dom, prm = domain_of(c), params_of(c)
    steps = 20
    fixed = c.fixed_mask()
    x, v, r, builds, _ = O.verlet_steps(dom, prm, c.pos, c.vel, c.skin, steps, fixed=fixed, rho=c.rho)
    x2, v2, r2, _, _, _ = O.step_ex1a(dom, prm, c.pos.astype(np.float64), c.vel.astype(np.float64),
                                      c.rho.astype(np.float64), fixed=fixed, n_steps=steps)
    np.testing.assert_array_equal(x, x2)
    np.testing.assert_array_equal(r, r2)
    assert 1 <= builds < steps


def _head_on():
    h, skin = 0.01, 0.004
    dom = O.Domain(dim=2, n=(10, 10, 1), cs=(0.025, 0.025, 1.0))
    prm = O.Params(h=h, mass=0.1, c0=10.0, nu=0.0, dt=1e-4)
    gap = 2.0 * h + skin + 1e-3
    x = np.array([[0.125 - gap / 2, 0.125], [0.125 + gap / 2, 0.125]])
    v = np.array([[0.5, 0.0], [-0.5, 0.0]])
    return dom, prm, x, v, skin


def test_half_skin_rule_keeps_an_approaching_pair_listed():
    dom, prm, x, v, skin = _head_on()
    x1, _, _, builds, _ = O.verlet_steps(dom, prm, x, v, skin, 90)
    assert x1[1, 0] - x1[0, 0] < 2.0 * prm.h  # the pair did enter the support
    assert builds >= 2


def test_full_skin_rule_misses_the_pair():
    dom, prm, x, v, skin = _head_on()
    with pytest.raises(AssertionError, match="not in the list"):
        O.verlet_steps(dom, prm, x, v, skin, 90, limit_fraction=1.0)


def test_skin_zero_builds_every_step_of_a_moving_system():
    c = _lively_2d(0.0)
    dom, prm = domain_of(c), params_of(c)
    _, _, _, builds, when = O.verlet_steps(dom, prm, c.pos, c.vel, 0.0, 6)
    assert builds == 6 and when == list(range(6))


def test_a_pair_law_steps_through_the_same_schedule():
    """Any stepper can run under the list: one DEM contact step at a time
    gives the plain DEM rollout, with the list complete at every step."""
    c = WL.dem_damper(spacing=2 * 0.004 * 0.985, jitter=0.05, v_sigma=1.0, seed=3, cf=0.0, skin=0.0008)
    dom, prm = domain_of(c), params_of(c)
    x0, v0 = c.pos.astype(np.float64), c.vel.astype(np.float64)
    fixed = c.fixed_mask()

    def one(x, v):
        x1, v1, _ = O.step_law("dem", dom, prm, x, v, c.radius, c.pmass, c.coef, fixed=fixed, n_steps=1)
        return x1, v1

    steps = 30
    x, v, _, builds, _ = O.verlet_steps(dom, prm, x0, v0, c.skin, steps, step_fn=one)
    x2, v2, _ = O.step_law("dem", dom, prm, x0, v0, c.radius, c.pmass, c.coef, fixed=fixed, n_steps=steps)
    np.testing.assert_array_equal(x, x2)
    np.testing.assert_array_equal(v, v2)
    assert 1 < builds < steps
