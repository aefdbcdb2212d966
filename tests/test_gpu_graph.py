"""nauticle_step only launches kernels on the caller's stream (no
allocation, copy, memset or host synchronisation), so steps can be recorded
into a HIP graph under stream capture and replayed.  Each replay, with the
program's own work and synchronisations in between, must equal the same
steps run directly, bit for bit (the state and the last step's fields)."""
import numpy as np
import pytest
import torch

from paper_1710_08259_amd import workloads as WL
from tests.gpu_common import f32, nauticle, stack, u32

pytestmark = pytest.mark.gpu

TABLES = {
    "periodic_2d_4096": (lambda: [WL.periodic_2d_4096()], None, 1),
    "lattice_3d": (lambda: [WL.lattice_case(3, (30, 27, 25), 0.01, 1.2, 0.05, 0.05, seed=95)], None, 3),
    "batched_persistent": (lambda: WL.batched_2d(n_cases=9, seed=96, max_side_exp=6.5), "persistent", 2),
}


def _snapshot(prob, st):
    n = prob.n
    out = [u32(st.cell)[:n], u32(st.id)[:n], stack(st.off, n).view(np.uint32), stack(st.vel, n).view(np.uint32),
           f32(prob.fields.rho)[:n].view(np.uint32), f32(prob.fields.p)[:n].view(np.uint32)]
    out += [f32(t)[:n].view(np.uint32) for t in prob.fields.acc]
    return out


@pytest.mark.parametrize("name", list(TABLES))
def test_captured_steps_replay_as_direct_steps(name):
    N = nauticle()
    make, tuning, k = TABLES[name]
    cases = make()
    tn = N.Tuning(block=128, persistent=1, groups_per_cu=0) if tuning == "persistent" else N.Tuning()
    prob_g, prob_e = N.Problem(cases, tuning=tn), N.Problem(cases, tuning=tn)
    st_g, st_e = prob_g.state_from_cases(), prob_e.state_from_cases()
    # one direct step each first: every kernel module loaded and every
    # launch shape queried before the capture
    prob_g.step(st_g, 1)
    prob_e.step(st_e, 1)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        prob_g.step(st_g, k)
    for replay in range(4):
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda")  # the program's own work between replays
        junk.mul_(2.0).sum().item()
        prob_e.step(st_e, k)
        torch.cuda.synchronize()
        prob_g.check()
        prob_e.check()
        for a, b in zip(_snapshot(prob_g, st_g), _snapshot(prob_e, st_e)):
            np.testing.assert_array_equal(a, b, err_msg=f"{name}, replay {replay}")
