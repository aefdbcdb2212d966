"""Batched cases in one launch per phase: every launch shape the autotuner
may pick (work-item size, grid or persistent queue) gives bitwise the same
result, a batch of uneven cases equals the cases run one by one, and the
autotuner measures, picks and caches a shape."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import f32, nauticle, norms, stack, u32
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


def test_256_uneven_cases_in_one_persistent_launch_match_the_oracle():
    """The batched workload (256 cases, 1,024..65,536 particles, per-case nu
    and c0): one persistent launch per phase; three cases of different sizes
    are checked against the oracle after 2 steps."""
    N = nauticle()
    cases = WL.batched_2d()
    prob = N.Problem(cases, tuning=N.Tuning(block=128, persistent=1, groups_per_cu=4))
    st = prob.state_from_cases()
    steps = 2
    prob.step(st, steps)
    torch.cuda.synchronize()
    prob.check()
    offsets = np.cumsum([0] + [c.n for c in cases])
    sizes = np.array([c.n for c in cases])
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes)), int(np.argsort(sizes)[len(sizes) // 2])]
    ids = u32(st.id)
    cell = u32(st.cell)
    offs = [f32(t) for t in st.off]
    for b in picks:
        c = cases[b]
        sl = slice(offsets[b], offsets[b + 1])
        from tests.gpu_common import case_absolute_from_state

        x_gpu = np.empty((c.n, 2))
        x_gpu[ids[sl]] = case_absolute_from_state(c, cell[sl], np.stack([o[sl] for o in offs], 1))
        x, _, _, _, _ = O.step(domain_of(c), params_of(c), x64(c), v64(c), n_steps=steps)
        err = np.abs(O.min_image(domain_of(c), x_gpu - x)).max() / norms(c)["x"]
        assert err < 1e-6, (b, c.n, err)


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
