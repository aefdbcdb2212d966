"""nauticle_step_fixed_scratch (the entry point for callers that cannot
allocate: its scratch is a fixed array in the library's device code)
against nauticle_step on a caller-allocated workspace: two calls in a row,
the second on a smaller table, each bit for bit equal to nauticle_step
from the same state (the same kernels and launch shape run); a table too
large for the fixed scratch is refused on the host."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import f32, nauticle, u32

pytestmark = pytest.mark.gpu


def _snapshot(prob, st):
    n = prob.n
    out = [u32(st.cell)[:n], u32(st.id)[:n], u32(prob.cells.perm)[:n], u32(prob.cells.nbr_count)[:n]]
    out += [f32(t)[:n].view(np.uint32) for t in st.off + st.vel]
    out += [f32(prob.fields.rho)[:n].view(np.uint32), f32(prob.fields.p)[:n].view(np.uint32)]
    out += [f32(t)[:n].view(np.uint32) for t in prob.fields.acc]
    return out


def _compare(N, cases, steps):
    ref = N.Problem(cases)
    st_r = ref.state_from_cases()
    ref.step(st_r, steps)
    torch.cuda.synchronize()
    ref.check()
    fix = N.Problem(cases)
    st_f = fix.state_from_cases()
    # poison what the call must overwrite, so a stale result cannot pass
    for t in fix.fields.acc + [fix.fields.rho, fix.fields.p]:
        t.fill_(float("nan"))
    fix.step_fixed_scratch(st_f, steps)
    for a, b in zip(_snapshot(ref, st_r), _snapshot(fix, st_f)):
        np.testing.assert_array_equal(a, b)
    return ref.ws_bytes


def test_fixed_scratch_steps_equal_workspace_steps_on_two_calls():
    N = nauticle()
    big = [WL.lattice_case(3, (30, 28, 26), 0.01, 1.2, 0.05, 0.05, seed=71, name="first")]
    small = [WL.lattice_case(2, (40, 36), 0.01, 1.3, 0.05, 0.1, seed=72, name="second_smaller")]
    b1 = _compare(N, big, 4)
    b2 = _compare(N, small, 3)
    assert b2 < b1
    print(f"fixed scratch: {big[0].n} then {small[0].n} particles, bit-exact to nauticle_step "
          f"(workspaces {b1} and {b2} bytes)")


def test_fixed_scratch_refuses_tables_larger_than_it():
    N = nauticle()
    case = WL.periodic_3d_8m()
    table = N.case_table([case])
    nbytes = ctypes.c_size_t(0)
    assert N.lib().nauticle_workspace_bytes(table, 1, ctypes.byref(nbytes)) == N.OK
    assert nbytes.value > 64 << 20
    # no state is needed: the size is checked before anything else
    st = N.CState()
    cells = N.CCells()
    fields = N.CFields()
    status = N.lib().nauticle_step_fixed_scratch(table, 1, ctypes.byref(st), 1, ctypes.byref(cells),
                                                 ctypes.byref(fields), None)
    assert status == N.ERR_WORKSPACE
    assert b"fixed scratch" in N.lib().nauticle_last_error()
