"""Shared helpers of the GPU parity tests: run the HIP path through the
C-ABI binding and bring results back to the input order of the oracle.
No method arithmetic here (only index bookkeeping and tolerance norms)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1710_08259_amd import workloads as WL
from tests.oracle_helpers import domain_of, params_of, v64, x64


def nauticle():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1710_08259_amd import nauticle as N

    N.lib()  # raises if the library was not built: no fallback
    return N


def u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def f32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def stack(ts, n):
    return np.stack([f32(t)[:n] for t in ts], axis=1)


def decode_nbr(entries: np.ndarray):
    """List entries -> (sorted index, per-axis cell offset in {-1,0,1})."""
    j = entries & ((1 << 26) - 1)
    d = [((entries >> (26 + 2 * k)) & 3).astype(np.int64) - 1 for k in range(3)]
    return j, np.stack(d, axis=-1)


def case_absolute_from_state(case, cell, off):
    """FP64 absolute positions from a cell-relative FP32 state."""
    n = cell.shape[0]
    c = cell.astype(np.int64)
    coords = np.zeros((n, 3), np.int64)
    coords[:, 0] = c % case.ncell[0]
    coords[:, 1] = (c // case.ncell[0]) % case.ncell[1]
    coords[:, 2] = c // (case.ncell[0] * case.ncell[1])
    x = np.zeros((n, case.dim))
    for k in range(case.dim):
        x[:, k] = case.origin[k] + coords[:, k] * case.cell_size[k] + off[:, k].astype(np.float64)
    return x


def norms(case, rho=None, p=None, a=None):
    """Scale normalisers of the tolerance: rho0 for rho, c0^2 rho0 (the
    bulk modulus gamma B) for p, c0^2 / h for a, the box length for
    positions; each raised to the reference field's own magnitude when that
    is larger (strongly compressed states, where the Tait law amplifies)."""
    S = dict(rho=case.rho0, p=case.c0 ** 2 * case.rho0, a=case.c0 ** 2 / case.h,
             x=float(np.max(case.length()[: case.dim])))
    if rho is not None:
        S["rho"] = max(S["rho"], float(np.abs(rho).max()))
    if p is not None:
        S["p"] = max(S["p"], float(np.abs(p).max()))
    if a is not None:
        S["a"] = max(S["a"], float(np.abs(a).max()))
    return S
