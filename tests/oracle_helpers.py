"""Helpers shared by tests: convert a workload Case into the oracle's
domain/parameter objects and FP64 inputs.  No method arithmetic here."""
import numpy as np

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL


def domain_of(case: WL.Case) -> O.Domain:
    return O.Domain(dim=case.dim, n=tuple(case.ncell), cs=tuple(case.cell_size),
                    origin=tuple(case.origin),
                    periodic=tuple(b == WL.PERIODIC for b in case.boundary),
                    symmetric=tuple(b == WL.SYMMETRIC for b in case.boundary))


def params_of(case: WL.Case) -> O.Params:
    return O.Params(h=case.h, mass=case.mass, rho0=case.rho0, c0=case.c0, gamma=case.gamma,
                    nu=case.nu, dt=case.dt, g=tuple(case.g), alpha_av=case.alpha_av,
                    law=tuple(case.law) + (0.0,) * (4 - len(case.law)))


def x64(case: WL.Case) -> np.ndarray:
    return case.pos.astype(np.float64)


def v64(case: WL.Case) -> np.ndarray:
    v = case.vel.astype(np.float64).copy()
    v[case.fixed_mask()] = 0.0
    return v
