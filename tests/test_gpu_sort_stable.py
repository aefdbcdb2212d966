"""The build's sort gives the stable sort of this build's keys, bit for
bit, whatever the key and permutation arrays held before: checked against a
stable argsort after a first build, after few and many particles change cell
(a step's state, in the last build's order), when nothing changed, and with
the key array left out of order or all equal; for tables of one sort tile
and larger."""
import numpy as np
import pytest
import torch

from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import nauticle, u32

pytestmark = pytest.mark.gpu


def _keys(cases, cell):
    """Each particle's key: its cell plus its case's first cell."""
    keys = np.empty(len(cell), np.int64)
    at, base = 0, 0
    for c in cases:
        keys[at:at + c.n] = base + cell[at:at + c.n].astype(np.int64)
        at += c.n
        base += c.n_cells
    return keys


def _build_and_check(N, prob, cases, st, what):
    prob.build_cells(st)
    torch.cuda.synchronize()
    prob.check()
    n = prob.n
    keys = _keys(cases, u32(st.cell)[:n])
    ref = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(u32(prob.cells.perm)[:n].astype(np.int64), ref, err_msg=what)
    np.testing.assert_array_equal(u32(prob.cells.key)[:n].astype(np.int64), keys[ref], err_msg=what)
    # the cell table: each cell's sorted range, empty cells marked
    nc = sum(c.n_cells for c in cases)
    cells = np.arange(nc)
    lo = np.searchsorted(keys[ref], cells, side="left")
    hi = np.searchsorted(keys[ref], cells, side="right")
    empty = np.uint32(0xFFFFFFFF)
    np.testing.assert_array_equal(u32(prob.cells.cell_start)[:nc], np.where(hi > lo, lo, empty).astype(np.uint32),
                                  err_msg=what)
    np.testing.assert_array_equal(u32(prob.cells.cell_end)[:nc], np.where(hi > lo, hi, empty).astype(np.uint32),
                                  err_msg=what)
    # the reordered state
    np.testing.assert_array_equal(u32(prob.sorted.cell)[:n], u32(st.cell)[:n][ref], err_msg=what)
    np.testing.assert_array_equal(u32(prob.sorted.id)[:n], u32(st.id)[:n][ref], err_msg=what)
    for k in range(cases[0].dim):
        np.testing.assert_array_equal(u32(prob.sorted.off[k])[:n], u32(st.off[k])[:n][ref], err_msg=what)
        np.testing.assert_array_equal(u32(prob.sorted.vel[k])[:n], u32(st.vel[k])[:n][ref], err_msg=what)


def _moved(cases, st, frac, seed, far):
    """A copy of st with a fraction of each case's particles put in another
    cell of the same case: a neighbouring cell along x, or anywhere (far)."""
    out = st.clone()
    cell = out.cell
    rng = np.random.default_rng(seed)
    at = 0
    for c in cases:
        k = max(1, int(frac * c.n))
        idx = at + rng.choice(c.n, size=k, replace=False)
        cur = u32(cell)[idx].astype(np.int64)
        if far:
            new = rng.integers(0, c.n_cells, size=k)
        else:
            new = np.clip(cur + rng.choice([-1, 1], size=k), 0, c.n_cells - 1)
        cell[torch.from_numpy(idx).cuda()] = torch.from_numpy(new.astype(np.int32)).cuda()
        at += c.n
    return out


def _sparse_3d():
    """Fewer particles than cells (uniform random points, cells of 2h
    holding ~0.3 each): the sort orders each tile in LDS before storing."""
    base = WL.lattice_case(3, (28, 28, 26), 0.01, 0.3, 0.0, 0.05, seed=93, name="sparse_3d")
    rng = np.random.default_rng(93)
    pts = rng.uniform(0, 1, (base.n, 3)) * base.length()[:3]
    return [WL.scaled(base, pos=pts.astype(np.float32))]


def _sparse_small_3d():
    """Fewer particles than cells in a table of one sort tile."""
    base = WL.lattice_case(3, (10, 10, 9), 0.01, 0.3, 0.0, 0.05, seed=94, name="sparse_small_3d")
    rng = np.random.default_rng(94)
    pts = rng.uniform(0, 1, (base.n, 3)) * base.length()[:3]
    return [WL.scaled(base, pos=pts.astype(np.float32))]


def _sparse_many_cells_3d():
    """A table of one sort tile with more cells than the one-workgroup build
    takes: the general path, with the one-tile sort."""
    base = WL.lattice_case(3, (10, 10, 9), 0.01, 0.1, 0.0, 0.05, seed=99, name="sparse_many_cells_3d")
    rng = np.random.default_rng(99)
    pts = rng.uniform(0, 1, (base.n, 3)) * base.length()[:3]
    return [WL.scaled(base, pos=pts.astype(np.float32))]


def _sparse_8192_cells_2d():
    """2,048 random points in 128 x 64 = 8,192 cells: the most cells the
    one-workgroup build takes (nine cells per thread)."""
    base = WL.lattice_case(2, (64, 32), 0.01, 0.2499, 0.0, 0.05, seed=104, name="sparse_8192_cells_2d")
    rng = np.random.default_rng(104)
    pts = rng.uniform(0, 1, (base.n, 2)) * base.length()[:2]
    return [WL.scaled(base, pos=pts.astype(np.float32))]


# Tables of at most one sort tile (4096 keys) and 8192 cells are built by one
# workgroup; larger ones take the general path, whose sort runs one tile in
# one workgroup and more tiles pass by pass: all sides of those edges are
# here.
TABLES = {
    "lattice_3d": lambda: [WL.lattice_case(3, (40, 37, 33), 0.01, 1.2, 0.05, 0.05, seed=91)],
    "batched_2d": lambda: WL.batched_2d(n_cases=7, seed=92, max_side_exp=6.5),
    "sparse_3d": _sparse_3d,
    "tile_3d_2431": lambda: [WL.lattice_case(3, (11, 13, 17), 0.01, 1.2, 0.05, 0.05, seed=95)],
    "tile_2d_4096": lambda: [WL.lattice_case(2, (64, 64), 0.01, 1.3, 0.05, 0.05, seed=96)],
    "over_a_tile_2d_4097": lambda: [WL.lattice_case(2, (17, 241), 0.01, 1.3, 0.05, 0.05, seed=97)],
    "tile_batched_2d": lambda: WL.batched_2d(n_cases=3, seed=98, max_side_exp=5.0),
    "tile_sparse_3d": _sparse_small_3d,
    "tile_many_cells_3d": _sparse_many_cells_3d,
    "tile_8192_cells_2d": _sparse_8192_cells_2d,
    "tile_64_cases_2d": lambda: [WL.lattice_case(2, (8, 8), 0.01, 1.3, 0.05, 0.05, seed=200 + b) for b in range(64)],
}


@pytest.mark.parametrize("name", list(TABLES))
def test_sort_is_the_stable_sort_whatever_the_arrays_held(name):
    N = nauticle()
    cases = TABLES[name]()
    # room for the crowding that particles moved to random cells can make
    prob = N.Problem(cases, max_nbr=256)
    st = prob.state_from_cases()
    _build_and_check(N, prob, cases, st, "first build")
    # the next builds start from the sorted state, as a step leaves it
    base = prob.sorted.clone()
    _build_and_check(N, prob, cases, base.clone(), "nothing changed")
    for frac, far, seed in ((0.001, False, 1), (0.02, False, 2), (0.05, True, 3), (0.5, True, 4)):
        prob.build_cells(base)  # the last keys: those of the sorted state
        torch.cuda.synchronize()
        _build_and_check(N, prob, cases, _moved(cases, base, frac, seed, far), f"{frac} moved, far={far}")
    # last keys out of order, and all equal
    n = prob.n
    rng = np.random.default_rng(5)
    prob.cells.key[:n] = torch.from_numpy(rng.integers(0, 1 << 20, n).astype(np.int32)).cuda()
    _build_and_check(N, prob, cases, _moved(cases, base, 0.01, 6, False), "last keys out of order")
    prob.cells.key[:n] = 0
    _build_and_check(N, prob, cases, _moved(cases, base, 0.01, 7, False), "last keys all zero")
