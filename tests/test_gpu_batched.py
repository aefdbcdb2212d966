"""Batched cases in one launch per phase: every launch shape the autotuner
may pick (work-item size, grid or persistent queue) gives bitwise the same
result, a batch of uneven cases equals the cases run one by one, and the
autotuner measures, picks and caches a shape."""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import case_absolute_from_state, f32, nauticle, norms, u32
from tests.oracle_helpers import domain_of, params_of, v64, x64

pytestmark = pytest.mark.gpu


def _run(N, cases, tuning, steps):
    prob = N.Problem(cases, tuning=tuning)
    st = prob.state_from_cases()
    prob.step(st, steps)
    torch.cuda.synchronize()
    prob.check()
    n = prob.n
    out = [u32(st.cell)[:n], u32(st.id)[:n], u32(prob.cells.nbr_count)[:n]]
    out += [f32(t)[:n].view(np.uint32) for t in st.off + st.vel]
    out += [f32(prob.fields.rho)[:n].view(np.uint32)]
    return out


def test_every_tuning_gives_bitwise_identical_steps():
    N = nauticle()
    from paper_1710_08259_amd.autotune import CANDIDATES

    cases = WL.batched_2d(n_cases=9, seed=11, max_side_exp=6.5)
    ref = _run(N, cases, N.Tuning(), 3)
    for cand in CANDIDATES:
        got = _run(N, cases, cand, 3)
        for a, b in zip(ref, got):
            np.testing.assert_array_equal(a, b, err_msg=str(cand))


def test_3d_persistent_launch_equals_grid_launch():
    N = nauticle()
    case = WL.lattice_case(3, (30, 27, 25), 0.01, 1.2, 0.05, 0.05, seed=13)
    ref = _run(N, [case], N.Tuning(), 3)
    got = _run(N, [case], N.Tuning(block=128, persistent=1, groups_per_cu=2), 3)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)


@pytest.fixture(scope="module")
def batched_oracle():
    """The oracle on every case of the batched workload (256 cases,
    1,024..65,536 particles, per-case nu and c0): the first step's rho, p
    and a, and positions and velocities after 20 steps."""
    cases = WL.batched_2d()
    one, twenty = [], []
    for c in cases:
        dom, prm = domain_of(c), params_of(c)
        _, _, rho, p, a = O.step(dom, prm, x64(c), v64(c), n_steps=1)
        one.append((rho, p, a))
        x, v, _, _, _ = O.step(dom, prm, x64(c), v64(c), n_steps=20)
        twenty.append((x, v))
    return cases, one, twenty


def _per_case(prob, st, cases):
    """The state and the last step's fields, per case, in id order."""
    offsets = np.cumsum([0] + [c.n for c in cases])
    ids = u32(st.id)
    cell = u32(st.cell)
    offs = [f32(t) for t in st.off]
    vels = [f32(t) for t in st.vel]
    rho, p = f32(prob.fields.rho), f32(prob.fields.p)
    acc = [f32(t) for t in prob.fields.acc]
    out = []
    for b, c in enumerate(cases):
        sl = slice(offsets[b], offsets[b + 1])
        i = ids[sl]
        x = np.empty((c.n, 2))
        x[i] = case_absolute_from_state(c, cell[sl], np.stack([o[sl] for o in offs], 1))
        v = np.empty((c.n, 2))
        v[i] = np.stack([t[sl] for t in vels], 1)
        r, pp, a = np.empty(c.n), np.empty(c.n), np.empty((c.n, 2))
        r[i], pp[i] = rho[sl], p[sl]
        a[i] = np.stack([t[sl] for t in acc], 1)
        out.append((x, v, r, pp, a))
    return out


def _tunings():
    """The persistent launch of the batched line, and the autotuner's pick
    for this table (measured now, cached in a temporary file)."""
    import tempfile

    from paper_1710_08259_amd import autotune
    from paper_1710_08259_amd import nauticle as N

    persistent = N.Tuning(block=128, persistent=1, groups_per_cu=4)
    with tempfile.TemporaryDirectory() as d:
        pick, _ = autotune.tune(WL.batched_2d(), steps=2, cache_path=os.path.join(d, "tune.json"))
    return {"persistent": persistent, "tuner": pick}


@pytest.mark.parametrize("which", ["persistent", "tuner"])
def test_256_uneven_cases_match_the_oracle_case_by_case(which, batched_oracle):
    """All 256 cases of the batched workload in one launch per phase: every
    case's first-step rho, p and a element by element (1e-5 of rho0,
    c0^2 rho0 and c0^2/h, each case's own constants, so a case that picked
    up another's nu or c0 fails), and every case's positions and velocities
    after 20 steps (5e-4 of the case's largest displacement over those steps
and of max |v|)."""
    N = nauticle()
    cases, one, twenty = batched_oracle
    tuning = _tunings()[which]
    prob = N.Problem(cases, tuning=tuning)
    st = prob.state_from_cases()
    prob.step(st, 1)
    torch.cuda.synchronize()
    prob.check()
    worst = dict(rho=0.0, p=0.0, a=0.0, a_own=0.0, x=0.0, v=0.0)
    for b, (c, got) in enumerate(zip(cases, _per_case(prob, st, cases))):
        rho, p, a = one[b]
        S = norms(c)
        e = dict(rho=np.abs(got[2] - rho).max() / S["rho"], p=np.abs(got[3] - p).max() / S["p"],
                 a=np.abs(got[4] - a).max() / S["a"], a_own=np.abs(got[4] - a).max() / np.abs(a).max())
        for k in e:
            worst[k] = max(worst[k], e[k])
        assert e["rho"] < 1e-5 and e["p"] < 1e-5 and e["a"] < 1e-5, (which, b, c.n, e)
    prob.step(st, 19)
    torch.cuda.synchronize()
    prob.check()
    worst["x_L"] = 0.0
    for b, (c, got) in enumerate(zip(cases, _per_case(prob, st, cases))):
        x, v = twenty[b]
        dom = domain_of(c)
        dx = np.abs(O.min_image(dom, got[0] - x)).max()
        moved = np.abs(O.min_image(dom, x - x64(c))).max()
        ex = dx / moved  # against the largest displacement over the 20 steps
        ev = np.abs(got[1] - v).max() / np.abs(v).max()
        worst["x"], worst["v"] = max(worst["x"], ex), max(worst["v"], ev)
        worst["x_L"] = max(worst["x_L"], dx / norms(c)["x"])
        assert ex < 5e-4 and ev < 5e-4, (which, b, c.n, ex, ev)
    print(f"256 cases, {which} {tuning}: worst step-1 rho {worst['rho']:.2e} p {worst['p']:.2e} "
          f"a {worst['a']:.2e} (of c0^2/h; {worst['a_own']:.2e} of the case's max |a|); "
          f"20 steps x {worst['x']:.2e} of the largest displacement ({worst['x_L']:.2e} of L), "
          f"v {worst['v']:.2e}")


def test_autotuner_measures_picks_and_caches(tmp_path):
    nauticle()
    from paper_1710_08259_amd import autotune
    from paper_1710_08259_amd import nauticle as N

    cases = WL.batched_2d(n_cases=16, seed=5, max_side_exp=7)
    path = str(tmp_path / "tune.json")
    cands = (N.Tuning(), N.Tuning(block=128, persistent=1, groups_per_cu=4))
    best, timings = autotune.tune(cases, steps=2, candidates=cands, cache_path=path)
    assert best in cands and set(timings) == set(cands) and all(t > 0 for t in timings.values())
    again, none = autotune.tune(cases, steps=2, candidates=cands, cache_path=path)
    assert again == best and none is None
