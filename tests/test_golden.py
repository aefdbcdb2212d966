"""Pins of the oracle and of the Example 1a inputs to numbers the paper
prints (fixtures under tests/golden/, each citing its passage)."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


@pytest.mark.parametrize("h", [0.004, 0.013, 0.25, 1.7])
def test_oracle_kernel_normalisation_is_the_printed_one(h):
    for dim, num, den, pi_pow in _rows("wendland_normalisation.txt"):
        d = int(dim)
        alpha = float(num) / (float(den) * math.pi ** int(pi_pow) * h ** d)
        assert O.alpha(d, h) == pytest.approx(alpha, rel=1e-15)
        assert O.W(d, h, 0.0) == pytest.approx(alpha, rel=1e-15)  # (1 - 0)^4 (0 + 1) = 1
        assert O.W(d, h, 2.0 * h) == 0.0


def test_example_1a_case_has_the_printed_constants():
    g = {k: v for k, v in _rows("example_1a_constants.txt")}
    case = WL.ex1a_dam_break(1.0)
    h = float(g["h"])
    dx = float(g["dx_over_h"]) * h
    assert case.h == pytest.approx(h, rel=1e-15)
    assert case.rho0 == float(g["rho0"])
    assert case.c0 == float(g["c"])
    assert case.mass == pytest.approx(float(g["mass_over_dx2_rho0"]) * dx * dx * float(g["rho0"]), rel=1e-12)
    assert tuple(case.g[:2]) == (float(g["g_x"]), float(g["g_y"]))
    assert case.dt == pytest.approx(float(g["dt"]), rel=1e-15)
    assert case.alpha_av == float(g["artificial_viscosity"])
    # cells of edge 2h (rounded up to the next float if FP32 would fall below 2h), 7/h x 10/h of them
    assert case.cell_size[0] >= float(g["cell_size_over_h"]) * h
    assert case.cell_size[0] == pytest.approx(float(g["cell_size_over_h"]) * h, rel=1e-7)
    assert case.ncell[:2] == (round(float(g["cells_x_times_h"]) / h), round(float(g["cells_y_times_h"]) / h))
    assert g["boundary"] == "symmetric" and case.boundary[:2] == (WL.SYMMETRIC, WL.SYMMETRIC)
    # the fluid block of the grid listing: 7 x 4 m at spacing dx, sites at half-spacing offsets
    pos = case.pos.astype(np.float64)
    assert pos[:, 0].max() < float(g["fluid_width"]) and pos[:, 1].max() < float(g["fluid_height"])
    assert pos[:, 0].min() == pytest.approx(0.5 * dx, rel=1e-6)
    assert len(np.unique(np.round(pos[:, 0] / dx, 3))) == int(math.ceil(float(g["fluid_width"]) / dx - 0.5))
