"""ctypes binding of ``libnauticle.so`` (include/nauticle.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of the library.  PyTorch provides device memory (tensors) and the
stream (``torch.cuda.current_stream().cuda_stream``).  There is no CPU
fallback: if the library is missing, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnauticle.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_DOMAIN = -2
ERR_NONFINITE = -3
ERR_OUT_OF_DOMAIN = -4
ERR_WORKSPACE = -5
ERR_HIP = -6
ERR_NEIGHBOUR_OVERFLOW = -7
ERR_ATTRIBUTE = -8
PERIODIC = 0
CUTOFF = 1
SYMMETRIC = 2
MODEL_SUMMATION = 0
MODEL_CONTINUITY = 1
MODEL_DEM = 2
MODEL_SOCIAL = 3
MODEL_CAHN_HILLIARD = 4
MIRROR_CODE = 3
EMPTY = 0xFFFFFFFF
NBR_INDEX_BITS = 26

ENTRY_POINTS = (
    "nauticle_cells_total", "nauticle_workspace_bytes", "nauticle_prepare", "nauticle_bin",
    "nauticle_unbin", "nauticle_unbin_by_id", "nauticle_gather_by_id", "nauticle_build_cells", "nauticle_sph_density", "nauticle_sph_continuity",
    "nauticle_sph_forces",
    "nauticle_step", "nauticle_step_record", "nauticle_step_cfl", "nauticle_step_fixed_scratch", "nauticle_step_verlet", "nauticle_interact", "nauticle_step_law", "nauticle_ch_steps", "nauticle_sph_adjoint", "nauticle_position_loss", "nauticle_check",
    "nauticle_last_error",
)


class NauticleError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


# ----------------------------------------------------------------------------
# C structures (mirror include/nauticle.h)
# ----------------------------------------------------------------------------

class CDomain(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("ncell", ctypes.c_int32 * 3), ("boundary", ctypes.c_int32 * 3),
                ("origin", ctypes.c_double * 3), ("cell_size", ctypes.c_double * 3)]


class CParams(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("mass", ctypes.c_double), ("rho0", ctypes.c_double),
                ("c0", ctypes.c_double), ("gamma", ctypes.c_double), ("nu", ctypes.c_double),
                ("dt", ctypes.c_double), ("g", ctypes.c_double * 3), ("alpha_av", ctypes.c_double),
                ("law", ctypes.c_double * 4), ("skin", ctypes.c_double), ("model", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class CCase(ctypes.Structure):
    _fields_ = [("dom", CDomain), ("prm", CParams), ("offset", ctypes.c_int64), ("n", ctypes.c_int64),
                ("n_fixed", ctypes.c_int64)]


class CState(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_void_p), ("off", ctypes.c_void_p * 3), ("vel", ctypes.c_void_p * 3),
                ("id", ctypes.c_void_p), ("rho", ctypes.c_void_p)]


class CCells(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("perm", ctypes.c_void_p), ("cell_start", ctypes.c_void_p),
                ("cell_end", ctypes.c_void_p), ("nbr", ctypes.c_void_p), ("nbr_count", ctypes.c_void_p),
                ("max_nbr", ctypes.c_int32)]


class CLawAttrs(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_void_p), ("mass", ctypes.c_void_p), ("coef", ctypes.c_void_p),
                ("v0", ctypes.c_void_p), ("goal", ctypes.c_void_p * 3)]


class CTuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("persistent", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


@dataclass(frozen=True)
class Tuning:
    """Launch shape of the neighbour loops (results do not depend on it)."""

    block: int = 256
    persistent: int = 0
    groups_per_cu: int = 4

    def c(self) -> CTuning:
        t = CTuning()
        t.block, t.persistent, t.groups_per_cu, t.reserved = self.block, self.persistent, self.groups_per_cu, 0
        return t


class CFields(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_void_p), ("p", ctypes.c_void_p), ("s", ctypes.c_void_p),
                ("inv_rho", ctypes.c_void_p), ("acc", ctypes.c_void_p * 3), ("drho", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1710_08259_amd/build.py "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    ptr3 = ctypes.c_void_p * 3
    L.nauticle_cells_total.restype = ctypes.c_int64
    L.nauticle_cells_total.argtypes = [P(CCase), i32]
    L.nauticle_workspace_bytes.restype = st
    L.nauticle_workspace_bytes.argtypes = [P(CCase), i32, P(ctypes.c_size_t)]
    L.nauticle_prepare.restype = st
    L.nauticle_prepare.argtypes = [P(CCase), i32, P(CTuning), vp, ctypes.c_size_t, vp]
    L.nauticle_bin.restype = st
    L.nauticle_bin.argtypes = [P(CCase), i32, P(ptr3), P(CState), vp, ctypes.c_size_t, vp]
    L.nauticle_unbin.restype = st
    L.nauticle_unbin.argtypes = [P(CCase), i32, P(CState), P(ptr3), vp, ctypes.c_size_t, vp]
    L.nauticle_unbin_by_id.restype = st
    L.nauticle_unbin_by_id.argtypes = [P(CCase), i32, P(CState), P(ptr3), vp, ctypes.c_size_t, vp]
    L.nauticle_gather_by_id.restype = st
    L.nauticle_gather_by_id.argtypes = [P(CCase), i32, P(CState), P(ptr3), P(ptr3), vp, ctypes.c_size_t, vp]
    L.nauticle_build_cells.restype = st
    L.nauticle_build_cells.argtypes = [P(CCase), i32, P(CState), P(CState), P(CCells), vp, ctypes.c_size_t, vp]
    L.nauticle_sph_density.restype = st
    L.nauticle_sph_density.argtypes = [P(CCase), i32, P(CState), P(CCells), P(CFields), vp, ctypes.c_size_t, vp]
    L.nauticle_sph_continuity.restype = st
    L.nauticle_sph_continuity.argtypes = [P(CCase), i32, P(CState), P(CCells), P(CFields), vp, ctypes.c_size_t,
                                          vp]
    L.nauticle_sph_forces.restype = st
    L.nauticle_sph_forces.argtypes = [P(CCase), i32, P(CState), P(CCells), P(CFields), P(CState), vp,
                                      ctypes.c_size_t, vp]
    L.nauticle_step.restype = st
    L.nauticle_step.argtypes = [P(CCase), i32, P(CState), i32, P(CCells), P(CFields), P(vp), vp,
                                ctypes.c_size_t, vp]
    L.nauticle_step_cfl.restype = st
    L.nauticle_step_cfl.argtypes = [P(CCase), i32, P(CState), i32, P(CCells), P(CFields), ctypes.c_double, vp, vp,
                                    ctypes.c_size_t, vp]
    L.nauticle_step_record.restype = st
    L.nauticle_step_record.argtypes = [P(CCase), i32, P(CState), P(CState), P(CCells), P(CFields), vp,
                                       ctypes.c_size_t, vp]
    L.nauticle_step_fixed_scratch.restype = st
    L.nauticle_step_fixed_scratch.argtypes = [P(CCase), i32, P(CState), i32, P(CCells), P(CFields), vp]
    L.nauticle_step_verlet.restype = st
    L.nauticle_step_verlet.argtypes = [P(CCase), i32, P(CState), i32, P(CCells), P(CFields), P(CLawAttrs), P(i32),
                                       P(vp), vp, ctypes.c_size_t, vp]
    L.nauticle_interact.restype = st
    L.nauticle_interact.argtypes = [P(CCase), i32, P(CState), P(CCells), P(CLawAttrs), P(CFields), P(CState), vp,
                                    ctypes.c_size_t, vp]
    L.nauticle_step_law.restype = st
    L.nauticle_step_law.argtypes = [P(CCase), i32, P(CState), i32, P(CCells), P(CFields), P(CLawAttrs), P(vp), vp,
                                    ctypes.c_size_t, vp]
    L.nauticle_ch_steps.restype = st
    L.nauticle_ch_steps.argtypes = [P(CCase), i32, P(CState), P(CCells), vp, vp, vp, vp, i32, vp, ctypes.c_size_t,
                                    vp]
    L.nauticle_sph_adjoint.restype = st
    L.nauticle_sph_adjoint.argtypes = [P(CCase), i32, P(CState), P(CCells), P(CFields), P(ptr3), P(ptr3),
                                       P(ptr3), P(ptr3), vp, vp, vp, ctypes.c_size_t, vp]
    L.nauticle_position_loss.restype = st
    L.nauticle_position_loss.argtypes = [P(CCase), i32, P(CState), P(CState), vp, P(ptr3), vp,
                                         ctypes.c_size_t, vp]
    L.nauticle_check.restype = st
    L.nauticle_check.argtypes = [vp, ctypes.c_size_t, vp]
    L.nauticle_last_error.restype = ctypes.c_char_p
    L.nauticle_last_error.argtypes = []
    _lib = L
    return L


def _check(status: int, where: str):
    if status != OK:
        msg = lib().nauticle_last_error().decode(errors="replace")
        raise NauticleError(status, where, msg)


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _ptr3(ts: Sequence[Optional[torch.Tensor]]):
    arr = (ctypes.c_void_p * 3)()
    for k in range(3):
        arr[k] = ts[k].data_ptr() if k < len(ts) and ts[k] is not None else None
    return arr


# ----------------------------------------------------------------------------
# Python-side containers
# ----------------------------------------------------------------------------

@dataclass
class State:
    """Particle state in the cell-relative layout (device tensors)."""

    cell: torch.Tensor          # int32 (uint32 in C)
    off: list                   # dim x float32
    vel: list                   # dim x float32
    id: torch.Tensor            # int32
    rho: Optional[torch.Tensor] = None  # float32, the continuity model's evolved density

    def c(self) -> CState:
        s = CState()
        s.cell = self.cell.data_ptr()
        s.id = self.id.data_ptr()
        for k in range(3):
            s.off[k] = self.off[k].data_ptr() if k < len(self.off) else None
            s.vel[k] = self.vel[k].data_ptr() if k < len(self.vel) else None
        s.rho = self.rho.data_ptr() if self.rho is not None else None
        return s

    def clone(self) -> "State":
        return State(self.cell.clone(), [t.clone() for t in self.off], [t.clone() for t in self.vel],
                     self.id.clone(), None if self.rho is None else self.rho.clone())

    def copy_(self, other: "State") -> "State":
        self.cell.copy_(other.cell)
        self.id.copy_(other.id)
        if self.rho is not None and other.rho is not None:
            self.rho.copy_(other.rho)
        for a, b in zip(self.off, other.off):
            a.copy_(b)
        for a, b in zip(self.vel, other.vel):
            a.copy_(b)
        return self


@dataclass
class Cells:
    key: torch.Tensor
    perm: torch.Tensor
    cell_start: torch.Tensor
    cell_end: torch.Tensor
    nbr: torch.Tensor           # (max_nbr / 4, N, 4) int32: chunks of four entries
    nbr_count: torch.Tensor
    max_nbr: int

    def entries(self) -> torch.Tensor:
        """The lists as (max_nbr, N): entry k of sorted particle p at [k, p]."""
        n_chunks, N, w = self.nbr.shape
        return self.nbr.permute(0, 2, 1).reshape(n_chunks * w, N)

    def c(self) -> CCells:
        c = CCells()
        c.key, c.perm = self.key.data_ptr(), self.perm.data_ptr()
        c.cell_start, c.cell_end = self.cell_start.data_ptr(), self.cell_end.data_ptr()
        c.nbr, c.nbr_count = self.nbr.data_ptr(), self.nbr_count.data_ptr()
        c.max_nbr = self.max_nbr
        return c


@dataclass
class Fields:
    rho: torch.Tensor
    p: torch.Tensor
    s: torch.Tensor
    inv_rho: torch.Tensor
    acc: list
    drho: Optional[torch.Tensor] = None

    def c(self) -> CFields:
        f = CFields()
        f.rho, f.p, f.s, f.inv_rho = (self.rho.data_ptr(), self.p.data_ptr(), self.s.data_ptr(),
                                      self.inv_rho.data_ptr())
        for k in range(3):
            f.acc[k] = self.acc[k].data_ptr() if k < len(self.acc) else None
        f.drho = self.drho.data_ptr() if self.drho is not None else None
        return f


@dataclass
class LawAttrs:
    """Per-particle attributes of a pair law (device FP32 tensors in input
    order): radius, mass, coef (DEM: (1 - nu^2)/E; social force: attraction
    c), and for the social force v0 and goal (one tensor per axis)."""

    radius: torch.Tensor
    mass: torch.Tensor
    coef: torch.Tensor
    v0: Optional[torch.Tensor] = None
    goal: Optional[list] = None

    def c(self) -> CLawAttrs:
        a = CLawAttrs()
        a.radius, a.mass, a.coef = self.radius.data_ptr(), self.mass.data_ptr(), self.coef.data_ptr()
        a.v0 = self.v0.data_ptr() if self.v0 is not None else None
        for k in range(3):
            a.goal[k] = self.goal[k].data_ptr() if self.goal is not None and k < len(self.goal) else None
        return a


def case_table(cases) -> "ctypes.Array":
    """Case objects with the attributes of workloads.Case -> C case array."""
    arr = (CCase * len(cases))()
    offset = 0
    for b, c in enumerate(cases):
        d = arr[b].dom
        d.dim = c.dim
        for k in range(3):
            d.ncell[k] = int(c.ncell[k])
            d.boundary[k] = int(c.boundary[k])
            d.origin[k] = float(c.origin[k])
            d.cell_size[k] = float(c.cell_size[k])
        p = arr[b].prm
        p.h, p.mass, p.rho0, p.c0 = c.h, c.mass, c.rho0, c.c0
        p.gamma, p.nu, p.dt = c.gamma, c.nu, c.dt
        for k in range(3):
            p.g[k] = float(c.g[k])
        p.alpha_av = float(getattr(c, "alpha_av", 0.0))
        law = tuple(getattr(c, "law", ()) or ())
        for k in range(4):
            p.law[k] = float(law[k]) if k < len(law) else 0.0
        p.skin = float(getattr(c, "skin", 0.0))
        p.model = int(getattr(c, "model", MODEL_SUMMATION))
        p.reserved = 0
        arr[b].offset = offset
        arr[b].n = c.n
        arr[b].n_fixed = c.n_fixed
        offset += c.n
    return arr


def default_max_nbr(dim: int) -> int:
    return 64 if dim == 2 else 128


def _list_shape(max_nbr: int, n: int):
    """Storage of the neighbour lists: chunks of four entries, chunk-major.
    A max_nbr that is not a multiple of 4 is passed through for the library
    to reject."""
    return (max(max_nbr // 4, 1), n, 4) if max_nbr % 4 == 0 else (max_nbr, n)


class Problem:
    """A prepared set of independent cases on one device: owns the workspace,
    the neighbour structure and the field arrays."""

    def __init__(self, cases, device="cuda:0", max_nbr: Optional[int] = None, tuning: Optional[Tuning] = None):
        self.cases = list(cases)
        self.tuning = tuning or Tuning()
        self.device = torch.device(device)
        self.dim = self.cases[0].dim
        self.model = int(getattr(self.cases[0], "model", MODEL_SUMMATION))
        self.table = case_table(self.cases)
        self.n_cases = len(self.cases)
        self.n = int(sum(c.n for c in self.cases))
        self.n_cells = int(lib().nauticle_cells_total(self.table, self.n_cases))
        nbytes = ctypes.c_size_t(0)
        _check(lib().nauticle_workspace_bytes(self.table, self.n_cases, ctypes.byref(nbytes)),
               "nauticle_workspace_bytes")
        self.ws_bytes = int(nbytes.value)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        _check(lib().nauticle_prepare(self.table, self.n_cases, ctypes.byref(self.tuning.c()), _p(self.ws),
                                      self.ws_bytes, self.stream()), "nauticle_prepare")
        self.max_nbr = int(max_nbr or default_max_nbr(self.dim))
        i32 = dict(dtype=torch.int32, device=self.device)
        f32 = dict(dtype=torch.float32, device=self.device)
        N = max(self.n, 1)
        self.cells = Cells(torch.empty(N, **i32), torch.empty(N, **i32),
                           torch.empty(max(self.n_cells, 1), **i32), torch.empty(max(self.n_cells, 1), **i32),
                           torch.empty(_list_shape(self.max_nbr, N), **i32), torch.empty(N, **i32), self.max_nbr)
        self.fields = self.new_fields()
        self.sorted = self.new_state()

    # -- helpers ----------------------------------------------------------------
    def stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def new_state(self) -> State:
        N = max(self.n, 1)
        i32 = dict(dtype=torch.int32, device=self.device)
        f32 = dict(dtype=torch.float32, device=self.device)
        rho = torch.zeros(N, **f32) if self.model == MODEL_CONTINUITY else None
        return State(torch.zeros(N, **i32), [torch.zeros(N, **f32) for _ in range(self.dim)],
                     [torch.zeros(N, **f32) for _ in range(self.dim)], torch.zeros(N, **i32), rho)

    def _ws(self):
        return _p(self.ws), self.ws_bytes, self.stream()

    # -- entry points -------------------------------------------------------------
    def bin(self, pos: Sequence[torch.Tensor], vel: Optional[Sequence[torch.Tensor]] = None) -> State:
        """Absolute FP32 positions (per-axis device tensors) -> new state."""
        st = self.new_state()
        cs = st.c()
        _check(lib().nauticle_bin(self.table, self.n_cases, ctypes.byref(_ptr3(pos)), ctypes.byref(cs),
                                  *self._ws()), "nauticle_bin")
        if vel is not None:
            for k in range(self.dim):
                st.vel[k][: self.n].copy_(vel[k][: self.n])
        return st

    def state_from_cases(self) -> State:
        """Bins the cases' own positions and velocities (walls get v = 0);
        with the continuity model also their densities (rho0 if none)."""
        pos = np.concatenate([c.pos for c in self.cases], axis=0)
        vel = np.concatenate([np.where(c.fixed_mask()[:, None], 0.0, c.vel).astype(np.float32)
                              for c in self.cases], axis=0)
        pos_t = [torch.from_numpy(np.ascontiguousarray(pos[:, k])).to(self.device) for k in range(self.dim)]
        vel_t = [torch.from_numpy(np.ascontiguousarray(vel[:, k])).to(self.device) for k in range(self.dim)]
        st = self.bin(pos_t, vel_t)
        if st.rho is not None:
            rho = np.concatenate([c.rho if getattr(c, "rho", None) is not None
                                  else np.full(c.n, c.rho0, np.float32) for c in self.cases]).astype(np.float32)
            st.rho[: self.n].copy_(torch.from_numpy(rho))
        return st

    def unbin(self, st: State) -> list:
        pos = [torch.empty(max(self.n, 1), dtype=torch.float32, device=self.device) for _ in range(self.dim)]
        _check(lib().nauticle_unbin(self.table, self.n_cases, ctypes.byref(st.c()), ctypes.byref(_ptr3(pos)),
                                    *self._ws()), "nauticle_unbin")
        return pos

    def unbin_by_id(self, st: State) -> list:
        """Absolute FP32 positions in input (id) order, one tensor per axis."""
        pos = [torch.empty(max(self.n, 1), dtype=torch.float32, device=self.device) for _ in range(self.dim)]
        _check(lib().nauticle_unbin_by_id(self.table, self.n_cases, ctypes.byref(st.c()),
                                          ctypes.byref(_ptr3(pos)), *self._ws()), "nauticle_unbin_by_id")
        return pos

    def gather_by_id(self, st: State, g: Sequence[torch.Tensor]) -> list:
        """out[k][p] = g[k][id of p]: input-order vectors into st's order."""
        out = [torch.empty(max(self.n, 1), dtype=torch.float32, device=self.device) for _ in range(self.dim)]
        _check(lib().nauticle_gather_by_id(self.table, self.n_cases, ctypes.byref(st.c()), ctypes.byref(_ptr3(g)),
                                           ctypes.byref(_ptr3(out)), *self._ws()), "nauticle_gather_by_id")
        return out

    def build_cells(self, st: State, sorted_: Optional[State] = None, cells: Optional[Cells] = None) -> State:
        out = self.sorted if sorted_ is None else sorted_
        c = self.cells if cells is None else cells
        _check(lib().nauticle_build_cells(self.table, self.n_cases, ctypes.byref(st.c()), ctypes.byref(out.c()),
                                          ctypes.byref(c.c()), *self._ws()), "nauticle_build_cells")
        return out

    def density(self, sorted_: Optional[State] = None, cells: Optional[Cells] = None,
                fields: Optional[Fields] = None):
        s = self.sorted if sorted_ is None else sorted_
        c = self.cells if cells is None else cells
        f = self.fields if fields is None else fields
        _check(lib().nauticle_sph_density(self.table, self.n_cases, ctypes.byref(s.c()), ctypes.byref(c.c()),
                                          ctypes.byref(f.c()), *self._ws()), "nauticle_sph_density")
        return f

    def continuity(self, sorted_: Optional[State] = None, cells: Optional[Cells] = None,
                   fields: Optional[Fields] = None):
        s = self.sorted if sorted_ is None else sorted_
        c = self.cells if cells is None else cells
        f = self.fields if fields is None else fields
        _check(lib().nauticle_sph_continuity(self.table, self.n_cases, ctypes.byref(s.c()), ctypes.byref(c.c()),
                                             ctypes.byref(f.c()), *self._ws()), "nauticle_sph_continuity")
        return f

    def law_attrs(self) -> LawAttrs:
        """The cases' per-particle pair-law attributes as device tensors."""
        def cat(name):
            parts = [np.asarray(getattr(c, name), np.float32) for c in self.cases]
            return torch.from_numpy(np.ascontiguousarray(np.concatenate(parts))).to(self.device)

        v0 = goal = None
        if self.model == MODEL_SOCIAL:
            v0 = cat("v0")
            g = np.concatenate([np.asarray(c.goal, np.float32) for c in self.cases])
            goal = [torch.from_numpy(np.ascontiguousarray(g[:, k])).to(self.device) for k in range(self.dim)]
        return LawAttrs(cat("radius"), cat("pmass"), cat("coef"), v0, goal)

    def interact(self, attrs: LawAttrs, sorted_: Optional[State] = None, next_: Optional[State] = None,
                 cells: Optional[Cells] = None, fields: Optional[Fields] = None):
        s = self.sorted if sorted_ is None else sorted_
        c = self.cells if cells is None else cells
        f = self.fields if fields is None else fields
        nxt = ctypes.byref(next_.c()) if next_ is not None else None
        _check(lib().nauticle_interact(self.table, self.n_cases, ctypes.byref(s.c()), ctypes.byref(c.c()),
                                       ctypes.byref(attrs.c()), ctypes.byref(f.c()), nxt, *self._ws()),
               "nauticle_interact")
        return f

    def step_law(self, st: State, attrs: LawAttrs, n_steps: int = 1, events=None) -> State:
        ev = self._events(events, n_steps)
        _check(lib().nauticle_step_law(self.table, self.n_cases, ctypes.byref(st.c()), int(n_steps),
                                       ctypes.byref(self.cells.c()), ctypes.byref(self.fields.c()),
                                       ctypes.byref(attrs.c()), ev, *self._ws()), "nauticle_step_law")
        return st

    def ch_steps(self, c: torch.Tensor, clock: torch.Tensor, n_steps: int = 1, mu: Optional[torch.Tensor] = None,
                 cdot: Optional[torch.Tensor] = None, sorted_: Optional[State] = None, cells: Optional[Cells] = None):
        """Example 1b steps on the lists of the last build_cells: c (FP32,
        sorted order) in place; clock (FP64 device, {time, dt} per case)."""
        s = self.sorted if sorted_ is None else sorted_
        cl = self.cells if cells is None else cells
        _check(lib().nauticle_ch_steps(self.table, self.n_cases, ctypes.byref(s.c()), ctypes.byref(cl.c()), _p(c),
                                       _p(mu), _p(cdot), _p(clock), int(n_steps), *self._ws()), "nauticle_ch_steps")
        return c

    def _events(self, events, n_steps):
        if events is None:
            return None
        if len(events) != 5 * n_steps:
            raise ValueError("need 5 events per step")
        for e in events:  # torch creates the HIP event on first record
            if e.cuda_event == 0:
                e.record(torch.cuda.current_stream(self.device))
        return (ctypes.c_void_p * len(events))(*[e.cuda_event for e in events])

    def forces(self, sorted_: Optional[State] = None, next_: Optional[State] = None,
               cells: Optional[Cells] = None, fields: Optional[Fields] = None):
        s = self.sorted if sorted_ is None else sorted_
        c = self.cells if cells is None else cells
        f = self.fields if fields is None else fields
        nxt = ctypes.byref(next_.c()) if next_ is not None else None
        _check(lib().nauticle_sph_forces(self.table, self.n_cases, ctypes.byref(s.c()), ctypes.byref(c.c()),
                                         ctypes.byref(f.c()), nxt, *self._ws()), "nauticle_sph_forces")
        return f

    def step(self, st: State, n_steps: int = 1, events=None) -> State:
        """n_steps steps in place.  `events` (optional): 5 * n_steps
        torch.cuda.Event(enable_timing=True) recorded at each step's start,
        after its sort/reorder, its neighbour lists, density and forces."""
        ev = self._events(events, n_steps)
        _check(lib().nauticle_step(self.table, self.n_cases, ctypes.byref(st.c()), int(n_steps),
                                   ctypes.byref(self.cells.c()), ctypes.byref(self.fields.c()), ev, *self._ws()),
               "nauticle_step")
        return st

    def step_cfl(self, st: State, n_steps: int, cfl: float, clock: torch.Tensor) -> State:
        """n_steps steps in place, each case's dt = cfl h / (c0 + max |v|)
        before every step; clock: device float64 (n_cases, 2) = {time, dt},
        advanced on the device."""
        _check(lib().nauticle_step_cfl(self.table, self.n_cases, ctypes.byref(st.c()), int(n_steps),
                                       ctypes.byref(self.cells.c()), ctypes.byref(self.fields.c()), float(cfl),
                                       _p(clock), *self._ws()), "nauticle_step_cfl")
        return st

    def step_record(self, st: State, sorted_: State, cells: Cells, fields: Fields) -> State:
        """One step in place, as step() runs it, leaving the step's sorted
        input state in `sorted_`, its neighbour structure in `cells` and its
        fields in `fields` (what the step's adjoint needs)."""
        _check(lib().nauticle_step_record(self.table, self.n_cases, ctypes.byref(st.c()), ctypes.byref(sorted_.c()),
                                          ctypes.byref(cells.c()), ctypes.byref(fields.c()), *self._ws()),
               "nauticle_step_record")
        return st

    def step_fixed_scratch(self, st: State, n_steps: int = 1) -> State:
        """n_steps steps in place through nauticle_step_fixed_scratch: the
        library's fixed device scratch instead of this problem's workspace
        (no allocation in the call; it waits for the steps and raises on
        any condition the kernels flagged)."""
        _check(lib().nauticle_step_fixed_scratch(self.table, self.n_cases, ctypes.byref(st.c()), int(n_steps),
                                                 ctypes.byref(self.cells.c()), ctypes.byref(self.fields.c()),
                                                 self.stream()), "nauticle_step_fixed_scratch")
        return st

    def step_verlet(self, st: State, n_steps: int = 1, attrs: Optional["LawAttrs"] = None, events=None) -> int:
        """n_steps steps in place with the neighbour lists reused while no
        particle has moved beyond the table's skin allows; returns the
        number of neighbour builds.  `attrs`: the DEM attributes (DEM
        tables only).  `events` as in step()."""
        ev = self._events(events, n_steps)
        builds = ctypes.c_int32(0)
        a = ctypes.byref(attrs.c()) if attrs is not None else None
        _check(lib().nauticle_step_verlet(self.table, self.n_cases, ctypes.byref(st.c()), int(n_steps),
                                          ctypes.byref(self.cells.c()), ctypes.byref(self.fields.c()), a,
                                          ctypes.byref(builds), ev, *self._ws()), "nauticle_step_verlet")
        return int(builds.value)

    def adjoint(self, sorted_: State, cells: Cells, fields: Fields, lam_x_next, lam_v_next, lam_x, lam_v,
                dnu: torch.Tensor, dc0: torch.Tensor):
        _check(lib().nauticle_sph_adjoint(self.table, self.n_cases, ctypes.byref(sorted_.c()),
                                          ctypes.byref(cells.c()), ctypes.byref(fields.c()),
                                          ctypes.byref(_ptr3(lam_x_next)), ctypes.byref(_ptr3(lam_v_next)),
                                          ctypes.byref(_ptr3(lam_x)), ctypes.byref(_ptr3(lam_v)),
                                          _p(dnu), _p(dc0), *self._ws()), "nauticle_sph_adjoint")

    def position_loss(self, a: State, b: State, grad: bool = True):
        loss = torch.zeros(self.n_cases, dtype=torch.float64, device=self.device)
        g = [torch.empty(max(self.n, 1), dtype=torch.float32, device=self.device) for _ in range(self.dim)] \
            if grad else None
        _check(lib().nauticle_position_loss(self.table, self.n_cases, ctypes.byref(a.c()), ctypes.byref(b.c()),
                                            _p(loss), ctypes.byref(_ptr3(g)) if g else None, *self._ws()),
               "nauticle_position_loss")
        return loss, g

    def check(self):
        """Waits for the stream and raises on any condition the kernels flagged."""
        _check(lib().nauticle_check(*self._ws()), "nauticle_check")

    def new_cells(self) -> Cells:
        i32 = dict(dtype=torch.int32, device=self.device)
        N = max(self.n, 1)
        return Cells(torch.empty(N, **i32), torch.empty(N, **i32), torch.empty(max(self.n_cells, 1), **i32),
                     torch.empty(max(self.n_cells, 1), **i32), torch.empty(_list_shape(self.max_nbr, N), **i32),
                     torch.empty(N, **i32), self.max_nbr)

    def new_fields(self) -> Fields:
        f32 = dict(dtype=torch.float32, device=self.device)
        N = max(self.n, 1)
        drho = torch.empty(N, **f32) if self.model == MODEL_CONTINUITY else None
        return Fields(torch.empty(N, **f32), torch.empty(N, **f32), torch.empty(N, **f32), torch.empty(N, **f32),
                      [torch.empty(N, **f32) for _ in range(self.dim)], drho)


def to_numpy_u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)
