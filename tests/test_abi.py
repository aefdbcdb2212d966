"""The C-ABI library loads, exports every entry point that include/nauticle.h
declares, and validates case tables on the host (no GPU needed: these calls
return before any HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1710_08259_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nauticle.h")


@pytest.fixture(scope="module")
def N():
    from paper_1710_08259_amd import nauticle as N

    if not os.path.exists(N.LIB_PATH):
        from paper_1710_08259_amd import build

        build.build()
    N.lib()
    return N


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nauticle_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ("nauticle_build_cells", "nauticle_sph_density", "nauticle_sph_forces", "nauticle_step",
                 "nauticle_sph_adjoint"):
        assert name in syms


def test_library_exports_every_declared_symbol(N):
    lib = ctypes.CDLL(N.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) == set(N.ENTRY_POINTS)


def _ws_bytes(N, cases):
    table = N.case_table(cases)
    out = ctypes.c_size_t(0)
    st = N.lib().nauticle_workspace_bytes(table, len(cases), ctypes.byref(out))
    return st, out.value


def test_workspace_bytes_for_valid_cases(N):
    st, nbytes = _ws_bytes(N, [WL.periodic_2d_4096()])
    assert st == N.OK and nbytes > 4096 * 4 * 8
    st, nbytes2 = _ws_bytes(N, WL.batched_2d(n_cases=5, seed=2, max_side_exp=6))
    assert st == N.OK and nbytes2 > 0
    assert N.lib().nauticle_cells_total(N.case_table([WL.periodic_2d_4096()]), 1) == 24 * 24


@pytest.mark.parametrize("mutate,status", [
    (lambda c: WL.scaled(c, cell_size=(0.02, 0.02, 1.0)), -2),                     # cell below 2h
    (lambda c: WL.scaled(c, ncell=(2, 24, 1)), -2),                                 # periodic axis < 3 cells
    (lambda c: WL.scaled(c, ncell=(24, 24, 2)), -2),                                # unused axis not 1
    (lambda c: WL.scaled(c, h=-1.0), -1),                                           # bad parameter
    (lambda c: WL.scaled(c, nu=float("nan")), -1),
    (lambda c: WL.scaled(c, dim=4), -2),
    (lambda c: WL.scaled(c, boundary=(7, 0, 0)), -2),
])
def test_invalid_cases_are_rejected_on_the_host(N, mutate, status):
    st, _ = _ws_bytes(N, [mutate(WL.periodic_2d_4096())])
    assert st == status
    assert len(N.lib().nauticle_last_error()) > 0


def test_mixed_dimensions_and_bad_offsets_are_rejected(N):
    a = WL.periodic_2d_4096()
    b = WL.lattice_case(3, (8, 8, 8), 0.01, 1.2, 0.0, 0.0, seed=0)
    st, _ = _ws_bytes(N, [a, b])
    assert st == N.ERR_DOMAIN
    table = N.case_table([a, a])
    table[1].offset = 5
    out = ctypes.c_size_t(0)
    assert N.lib().nauticle_workspace_bytes(table, 2, ctypes.byref(out)) == N.ERR_INVALID_ARG


def test_unprepared_workspace_is_rejected_without_touching_the_device(N):
    table = N.case_table([WL.periodic_2d_4096()])
    assert N.lib().nauticle_prepare(table, 1, None, None, 0, None) == N.ERR_WORKSPACE
    assert N.lib().nauticle_check(None, 0, None) == N.ERR_WORKSPACE
    fake = ctypes.c_void_p(0x1000)
    st = N.lib().nauticle_step(table, 1, None, 1, None, None, None, fake, 1 << 20, None)
    assert st == N.ERR_WORKSPACE


def test_the_oracle_is_not_reachable_from_the_package():
    """The product path never imports, loads or calls the oracle."""
    pat = re.compile(r"^\s*(from\s+oracle|import\s+oracle)|liboracle|\bor_[a-z_0-9]+\s*\(", re.M)
    pkg = os.path.join(ROOT, "paper_1710_08259_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not pat.search(text), f


def test_invalid_tuning_is_rejected_on_the_host(N):
    table = N.case_table([WL.periodic_2d_4096()])
    for bad in (N.Tuning(block=96), N.Tuning(persistent=2), N.Tuning(persistent=1, groups_per_cu=100)):
        assert N.lib().nauticle_prepare(table, 1, ctypes.byref(bad.c()), None, 0, None) == N.ERR_INVALID_ARG


@pytest.mark.parametrize("mutate,status", [
    (lambda c: WL.scaled(c, ncell=(1, c.ncell[1], 1)), -2),            # symmetric axis < 2 cells
    (lambda c: WL.scaled(c, model=7), -1),                            # unknown model
    (lambda c: WL.scaled(c, alpha_av=-0.1), -1),                      # negative artificial viscosity
    (lambda c: WL.scaled(c, alpha_av=float("inf")), -1),
])
def test_invalid_symmetric_and_continuity_cases_are_rejected(N, mutate, status):
    base = WL.ex1a_dam_break()
    assert _ws_bytes(N, [base])[0] == N.OK
    st, _ = _ws_bytes(N, [mutate(base)])
    assert st == status
    assert len(N.lib().nauticle_last_error()) > 0


def test_cases_of_one_table_share_one_model(N):
    a = WL.ex1a_dam_break()
    b = WL.scaled(a, model=WL.SUMMATION)
    assert _ws_bytes(N, [a, a])[0] == N.OK
    assert _ws_bytes(N, [a, b])[0] == N.ERR_INVALID_ARG


def test_continuity_model_workspace_holds_the_extra_arrays(N):
    a = WL.ex1a_dam_break()
    b = WL.scaled(a, model=WL.SUMMATION)
    # one float4 per particle more (the start-of-step velocity and density)
    assert _ws_bytes(N, [a])[1] >= _ws_bytes(N, [b])[1] + 16 * a.n


def test_pair_law_tables_are_validated(N):
    dem = WL.dem_damper()
    assert _ws_bytes(N, [dem])[0] == N.OK
    assert _ws_bytes(N, [WL.scaled(dem, law=(-0.1,))])[0] == N.ERR_INVALID_ARG   # negative friction
    soc = WL.social_room(width=6.0)
    assert _ws_bytes(N, [soc])[0] == N.OK
    assert _ws_bytes(N, [WL.scaled(soc, law=(2000.0, 0.0, 1.2e5, 0.5))])[0] == N.ERR_INVALID_ARG  # B = 0
    assert _ws_bytes(N, [WL.scaled(soc, law=(2000.0, 0.08, 1.2e5, float("nan")))])[0] == N.ERR_INVALID_ARG


def test_skin_tables_are_validated(N):
    """A skin needs cells of at least 2h + skin, must be finite and >= 0,
    and is refused by the social force (not compactly supported)."""
    base = WL.periodic_2d_4096()                       # h = 0.013, cells of 0.02667
    gap = float(np.float32(base.cell_size[0])) - 2.0 * base.h
    assert _ws_bytes(N, [WL.scaled(base, skin=0.99 * gap)])[0] == N.OK
    assert _ws_bytes(N, [WL.scaled(base, skin=1.01 * gap)])[0] == N.ERR_DOMAIN
    assert _ws_bytes(N, [WL.scaled(base, skin=-1e-4)])[0] == N.ERR_INVALID_ARG
    assert _ws_bytes(N, [WL.scaled(base, skin=float("nan"))])[0] == N.ERR_INVALID_ARG
    assert _ws_bytes(N, [WL.lattice_case(2, (64, 64), 0.01, 1.3, 0.01, 0.1, seed=1, skin=0.005)])[0] == N.OK
    soc = WL.social_room(width=6.0)
    assert _ws_bytes(N, [WL.scaled(soc, skin=1e-3)])[0] == N.ERR_INVALID_ARG


def test_skin_does_not_change_the_workspace(N):
    """Every summation or continuity table keeps room for the build-time
    offsets of the Verlet steps; the skin itself only changes the lists."""
    a = WL.periodic_2d_4096()
    gap = float(np.float32(a.cell_size[0])) - 2.0 * a.h
    assert _ws_bytes(N, [WL.scaled(a, skin=0.5 * gap)])[1] == _ws_bytes(N, [a])[1]


def test_particle_count_limit_of_the_list_index(N):
    """A list entry holds the neighbour's index in 26 bits: 2^26 - 1
    particles are accepted, 2^26 are rejected on the host.  (Case stand-ins:
    only the count matters here.)"""
    base = WL.periodic_2d_4096()

    class Counted:
        def __init__(self, n):
            self.__dict__.update(base.__dict__)
            self._n = n

        @property
        def n(self):
            return self._n

    limit = (1 << 26) - 1
    assert _ws_bytes(N, [Counted(limit)])[0] == N.OK
    assert _ws_bytes(N, [Counted(limit + 1)])[0] == N.ERR_INVALID_ARG
    assert "2^26" in N.lib().nauticle_last_error().decode()
