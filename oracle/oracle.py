"""FP64 CPU oracle for the WCSPH hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this module.  It loads ``oracle/liboracle.so`` (built from
``nauticle_oracle.c`` by ``oracle/build.py``) and shares no code with the HIP
library.

Every function follows the paper (arXiv:1710.08259):

* kernel, normalisation and derivative: Example 1a, Wendland kernel equation;
* density: SPH sampling expression with A = rho (Sec. 5.1);
* pressure gradient: eq. diffop1; viscosity: eq. diffop3 in Morris form;
* time step: semi-implicit Euler of Example 1a (velocity, then position);
* neighbour search: cell grid of Sec. 3.2.1 ("The computational domain");
* periodic shifting of leaving particles: Sec. 3.2.1;
* symmetric (mirror, free-slip) faces: Sec. 3.2.1 boundary kinds, used by
  the dam break of Example 1a;
* Example 1a's own operator set: continuity (eq. SPH_fluid_continuity),
  linear equation of state, momentum with the artificial viscosity Pi_ij
  (eq. SPH_fluid_momentum), stepped in the order of its equations eq1-eq7;
* two further pair laws on the same neighbour loop (Sec. 6, the interaction
  interface): the DEM contact law of Example 2 (eq. DEM_force) and the
  social force model (eq. social_force_model);
* Example 1b: Cahn-Hilliard with the SPH Laplacian sph_L0 (eq. diffop3 as
  Example 1b discretises it) and its adaptive time step;
* neighbour lists reused between builds (Sec. 4: the search reruns only when
  the layout has changed), with a skin beyond 2h and the displacement rule
  that keeps every pair inside the support listed (:func:`verlet_steps`).

The one-step adjoint (:func:`step_vjp`) is not in the paper; it is the exact
reverse-mode derivative of :func:`step` with one step, pinned against central
finite differences of :func:`step` in the tests.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# NAUTICLE_ORACLE_LIB selects another build of the same source (the
# sanitizer build of oracle/build.py)
_LIB_PATH = os.environ.get("NAUTICLE_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

EMPTY = 0xFFFFFFFF


class _Domain(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("periodic", ctypes.c_int32 * 3),
        ("mirror", ctypes.c_int32 * 3),
        ("origin", ctypes.c_double * 3),
        ("cs", ctypes.c_double * 3),
    ]


class _Params(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("c0", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("nu", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("alpha_av", ctypes.c_double),
        ("law", ctypes.c_double * 4),
    ]


@dataclass
class Domain:
    """Axis-aligned box of ``n[k]`` cells of edge ``cs[k]`` per axis."""

    dim: int
    n: tuple
    cs: tuple
    origin: tuple = (0.0, 0.0, 0.0)
    periodic: tuple = (True, True, True)
    # symmetric (mirror) faces; an axis that is neither periodic nor
    # symmetric is cut-off
    symmetric: tuple = (False, False, False)

    def length(self) -> np.ndarray:
        return np.array([self.n[k] * self.cs[k] for k in range(3)], dtype=np.float64)

    def n_cells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def _c(self) -> _Domain:
        d = _Domain()
        d.dim = self.dim
        for k in range(3):
            d.n[k] = int(self.n[k])
            d.periodic[k] = 1 if self.periodic[k] else 0
            d.mirror[k] = 1 if self.symmetric[k] else 0
            d.origin[k] = float(self.origin[k])
            d.cs[k] = float(self.cs[k])
        return d


@dataclass
class Params:
    h: float
    mass: float
    rho0: float = 1000.0
    c0: float = 10.0
    gamma: float = 7.0
    nu: float = 1e-3
    dt: float = 1e-4
    g: tuple = (0.0, 0.0, 0.0)
    alpha_av: float = 0.0   # artificial viscosity coefficient of Example 1a (0.1 there)
    law: tuple = (0.0, 0.0, 0.0, 0.0)  # DEM: (c_f,); social force: (A, B, k, tau)

    def _c(self) -> _Params:
        p = _Params()
        p.h, p.mass, p.rho0, p.c0 = self.h, self.mass, self.rho0, self.c0
        p.gamma, p.nu, p.dt = self.gamma, self.nu, self.dt
        for k in range(3):
            p.g[k] = float(self.g[k])
        p.alpha_av = float(self.alpha_av)
        for k in range(4):
            p.law[k] = float(self.law[k]) if k < len(self.law) else 0.0
        return p


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from oracle import build as _build  # noqa: WPS433 (build on first use)

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.or_alpha.restype = dbl
    lib.or_alpha.argtypes = [i32, dbl]
    for name in ("or_W", "or_F", "or_dF"):
        getattr(lib, name).restype = dbl
        getattr(lib, name).argtypes = [i32, dbl, dbl]
    lib.or_tait.restype = dbl
    lib.or_tait.argtypes = [P(_Params), dbl]
    lib.or_validate_domain.restype = ctypes.c_int
    lib.or_validate_domain.argtypes = [P(_Domain), dbl]
    lib.or_bin_f32.restype = None
    lib.or_bin_f32.argtypes = [P(_Domain), i64, vp, vp, vp, vp, vp, vp, vp]
    lib.or_sort_keys.restype = ctypes.c_int
    lib.or_sort_keys.argtypes = [i64, vp, ctypes.c_uint32, vp, vp, vp, vp]
    lib.or_neighbours_f32.restype = ctypes.c_int
    lib.or_neighbours_f32.argtypes = [P(_Domain), dbl, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, i32]
    lib.or_neighbours_f32_brute.restype = None
    lib.or_neighbours_f32_brute.argtypes = [P(_Domain), dbl, i64, vp, vp, vp, vp, vp]
    lib.or_density.restype = ctypes.c_int
    lib.or_density.argtypes = [P(_Domain), P(_Params), i64, vp, i64, vp, vp, vp, vp, ctypes.c_int]
    lib.or_forces.restype = ctypes.c_int
    lib.or_forces.argtypes = [P(_Domain), P(_Params), i64, vp, vp, vp, vp, vp, i64, vp, vp, ctypes.c_int]
    lib.or_step.restype = ctypes.c_int
    lib.or_step.argtypes = [P(_Domain), P(_Params), i64, vp, vp, vp, i32, vp, vp, vp, ctypes.c_int]
    lib.or_continuity.restype = ctypes.c_int
    lib.or_continuity.argtypes = [P(_Domain), P(_Params), i64, vp, vp, vp, i64, vp, vp, ctypes.c_int]
    lib.or_linear_eos.restype = dbl
    lib.or_linear_eos.argtypes = [P(_Params), dbl]
    lib.or_momentum.restype = ctypes.c_int
    lib.or_momentum.argtypes = [P(_Domain), P(_Params), i64, vp, vp, vp, vp, vp, i64, vp, vp,
                                ctypes.c_int]
    lib.or_step_ex1a.restype = ctypes.c_int
    lib.or_step_ex1a.argtypes = [P(_Domain), P(_Params), i64, vp, vp, vp, vp, i32, vp, vp, vp,
                                 ctypes.c_int]
    lib.or_dem.restype = ctypes.c_int
    lib.or_dem.argtypes = [P(_Domain), P(_Params), i64, vp, vp, vp, vp, vp, vp, i64, vp, vp, ctypes.c_int]
    lib.or_social.restype = ctypes.c_int
    lib.or_social.argtypes = [P(_Domain), P(_Params), i64, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp, vp,
                              ctypes.c_int]
    lib.or_law_diag.restype = ctypes.c_int
    lib.or_law_diag.argtypes = [ctypes.c_int, P(_Domain), P(_Params), i64, vp, vp, vp, vp, vp, vp, vp, vp, i64,
                                vp, vp, vp, ctypes.c_int]
    lib.or_step_law.restype = ctypes.c_int
    lib.or_step_law.argtypes = [ctypes.c_int, P(_Domain), P(_Params), i64, vp, vp, vp, vp, vp, vp, vp, vp,
                                i32, vp, ctypes.c_int]
    lib.or_laplacian.restype = ctypes.c_int
    lib.or_laplacian.argtypes = [P(_Domain), P(_Params), ctypes.c_int, i64, vp, vp, i64, vp, vp, ctypes.c_int]
    lib.or_ch_steps.restype = ctypes.c_int
    lib.or_ch_steps.argtypes = [P(_Domain), P(_Params), ctypes.c_int, i64, vp, vp, vp, i32, vp, vp,
                                ctypes.c_int]
    lib.or_step_vjp.restype = ctypes.c_int
    lib.or_step_vjp.argtypes = [P(_Domain), P(_Params), i64, vp, vp, vp, vp, vp, vp, vp,
                                P(dbl), P(dbl), ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


# --------------------------------------------------------------------------
# kernel and equation of state
# --------------------------------------------------------------------------

def alpha(dim: int, h: float) -> float:
    return _load().or_alpha(dim, h)


def W(dim: int, h: float, r: float) -> float:
    return _load().or_W(dim, h, r)


def F(dim: int, h: float, r: float) -> float:
    """(1/r) dW/dr, so that grad_i W_ij = F(r_ij) r_ij."""
    return _load().or_F(dim, h, r)


def dF(dim: int, h: float, r: float) -> float:
    return _load().or_dF(dim, h, r)


def tait(prm: Params, rho: float) -> float:
    return _load().or_tait(ctypes.byref(prm._c()), rho)


def validate_domain(dom: Domain, h: float) -> int:
    return _load().or_validate_domain(ctypes.byref(dom._c()), h)


# --------------------------------------------------------------------------
# FP32 binning, sort and neighbour counts (the bit-exact part)
# --------------------------------------------------------------------------

def bin_f32(dom: Domain, pos32: np.ndarray):
    """Absolute FP32 positions (n, dim) -> (cell u32[n], offsets f32[n, dim])."""
    pos32 = np.ascontiguousarray(pos32, dtype=np.float32)
    n = pos32.shape[0]
    cols = [np.ascontiguousarray(pos32[:, k]) for k in range(dom.dim)]
    offs = [np.zeros(n, np.float32) for _ in range(dom.dim)]
    cell = np.zeros(n, np.uint32)
    args = [_ptr(cols[k]) if k < dom.dim else None for k in range(3)]
    outs = [_ptr(offs[k]) if k < dom.dim else None for k in range(3)]
    _load().or_bin_f32(ctypes.byref(dom._c()), n, *args, _ptr(cell), *outs)
    return cell, np.stack(offs, axis=1)


def sort_keys(keys: np.ndarray, n_keys: int):
    """Stable counting sort: returns (key_sorted, perm, start, end)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    n = keys.shape[0]
    ks = np.zeros(n, np.uint32)
    perm = np.zeros(n, np.uint32)
    start = np.zeros(n_keys, np.uint32)
    end = np.zeros(n_keys, np.uint32)
    rc = _load().or_sort_keys(n, _ptr(keys), n_keys, _ptr(ks), _ptr(perm), _ptr(start), _ptr(end))
    if rc != 0:
        raise MemoryError("or_sort_keys failed")
    return ks, perm, start, end


def neighbours_f32(dom: Domain, h: float, cell: np.ndarray, off: np.ndarray,
                   max_nbr: int = 0, brute: bool = False, which=None, mirrors: bool = False):
    """FP32-predicate neighbour counts (and lists if max_nbr > 0), for all
    particles or for the subset ``which``.  With ``mirrors`` the lists come
    with a second array: per entry, the bit set of axes along which the
    neighbour is a mirror image."""
    cell = np.ascontiguousarray(cell, dtype=np.uint32)
    n = cell.shape[0]
    cols = [np.ascontiguousarray(off[:, k], dtype=np.float32) for k in range(dom.dim)]
    args = [_ptr(cols[k]) if k < dom.dim else None for k in range(3)]
    w = None if which is None else np.ascontiguousarray(which, dtype=np.int64)
    m = n if w is None else w.shape[0]
    count = np.zeros(m, np.int32)
    if brute:
        assert w is None
        _load().or_neighbours_f32_brute(ctypes.byref(dom._c()), h, n, _ptr(cell), *args, _ptr(count))
        return count
    lst = np.zeros((m, max_nbr), np.uint32) if max_nbr > 0 else None
    mir = np.zeros((m, max_nbr), np.uint8) if max_nbr > 0 else None
    rc = _load().or_neighbours_f32(ctypes.byref(dom._c()), h, n, _ptr(cell), *args, m, _ptr(w),
                                   _ptr(count), _ptr(lst), _ptr(mir), max_nbr)
    if rc != 0:
        raise MemoryError("or_neighbours_f32 failed")
    if max_nbr == 0:
        return count
    return (count, lst, mir) if mirrors else (count, lst)


# --------------------------------------------------------------------------
# FP64 physics
# --------------------------------------------------------------------------

def _x3(x: np.ndarray) -> np.ndarray:
    """(n, dim) -> contiguous (n, 3) FP64 with zero padding."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((x.shape[0], 3), np.float64)
    out[:, : x.shape[1]] = x
    return out


def density(dom: Domain, prm: Params, x, which=None, nthreads=None, counts=False):
    """rho, p for all particles (or for the subset ``which``)."""
    x3 = _x3(x)
    n = x3.shape[0]
    w = None if which is None else np.ascontiguousarray(which, dtype=np.int64)
    m = n if w is None else w.shape[0]
    rho = np.zeros(m)
    p = np.zeros(m)
    cnt = np.zeros(m, np.int32)
    rc = _load().or_density(ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3),
                            m, _ptr(w), _ptr(rho), _ptr(p), _ptr(cnt),
                            nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_density failed")
    return (rho, p, cnt) if counts else (rho, p)


def forces(dom: Domain, prm: Params, x, v, rho, p, fixed=None, which=None, nthreads=None):
    """Accelerations (n, dim); rho and p are given for all particles."""
    x3, v3 = _x3(x), _x3(v)
    n = x3.shape[0]
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    w = None if which is None else np.ascontiguousarray(which, dtype=np.int64)
    m = n if w is None else w.shape[0]
    a = np.zeros((m, 3))
    rc = _load().or_forces(ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3), _ptr(v3),
                           _ptr(rho), _ptr(p), _ptr(fx), m, _ptr(w), _ptr(a),
                           nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_forces failed")
    return a[:, : dom.dim]


def forces_at(dom: Domain, prm: Params, x, v, which, fixed=None, nthreads=None):
    """Accelerations of the particles ``which`` only, with the densities
    they need (theirs and their neighbours') computed by the oracle."""
    x3 = _x3(x)
    which = np.asarray(which, dtype=np.int64)
    # densities are needed at the sample and at every neighbour of it
    need = _neighbourhood(dom, prm, x3, which)
    rho_s, p_s = density(dom, prm, x3, which=need, nthreads=nthreads)
    rho = np.full(x3.shape[0], np.nan)
    p = np.full(x3.shape[0], np.nan)
    rho[need] = rho_s
    p[need] = p_s
    return forces(dom, prm, x3, v, rho, p, fixed=fixed, which=which, nthreads=nthreads)


def _neighbourhood(dom: Domain, prm: Params, x3, which):
    """which plus every particle within 2h of one of them (min image)."""
    L = dom.length()
    sel = set(int(i) for i in which)
    xs = x3[which]
    # cell grid lookup in numpy: bucket all particles by cell once
    cells = np.zeros((x3.shape[0], 3), np.int64)
    for k in range(dom.dim):
        cells[:, k] = np.clip(np.floor((x3[:, k] - dom.origin[k]) / dom.cs[k]), 0, dom.n[k] - 1)
    lin = cells[:, 0] + dom.n[0] * (cells[:, 1] + dom.n[1] * cells[:, 2])
    order = np.argsort(lin, kind="stable")
    lin_sorted = lin[order]
    r2max = 4.0 * prm.h * prm.h
    import itertools

    for s, i in enumerate(which):
        ci = cells[i]
        for d in itertools.product(*[(-1, 0, 1) if k < dom.dim else (0,) for k in range(3)]):
            c = ci + np.array(d)
            ok = True
            image = False
            for k in range(dom.dim):
                if dom.periodic[k]:
                    c[k] %= dom.n[k]
                elif c[k] < 0 or c[k] >= dom.n[k]:
                    if dom.symmetric[k]:
                        c[k] = ci[k]  # the boundary cell's mirror image
                        image = True
                    else:
                        ok = False
            if not ok:
                continue
            key = c[0] + dom.n[0] * (c[1] + dom.n[1] * c[2])
            lo = np.searchsorted(lin_sorted, key, "left")
            hi = np.searchsorted(lin_sorted, key, "right")
            js = order[lo:hi]
            if image:  # a superset is enough here: keep the whole cell
                sel.update(int(j) for j in js)
                continue
            r = x3[js] - xs[s]
            for k in range(dom.dim):
                if dom.periodic[k]:
                    r[:, k] -= L[k] * np.rint(r[:, k] / L[k])
            hit = js[(r * r).sum(axis=1) < r2max]
            sel.update(int(j) for j in hit)
    return np.array(sorted(sel), dtype=np.int64)


def step(dom: Domain, prm: Params, x, v, fixed=None, n_steps=1, nthreads=None):
    """Advance (x, v) by n_steps; returns (x, v, rho, p, a) of the last step."""
    x3, v3 = _x3(x), _x3(v)
    n = x3.shape[0]
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    rho = np.zeros(n)
    p = np.zeros(n)
    a = np.zeros((n, 3))
    rc = _load().or_step(ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3), _ptr(v3),
                         _ptr(fx), int(n_steps), _ptr(rho), _ptr(p), _ptr(a),
                         nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_step failed")
    d = dom.dim
    return x3[:, :d], v3[:, :d], rho, p, a[:, :d]


def step_cfl(dom: Domain, prm: Params, x, v, cfl: float, n_steps: int, fixed=None, time: float = 0.0,
             nthreads=None):
    """n_steps of :func:`step`, each with its own time step from a CFL
    condition on the sound speed and the flow speed: before every step
    dt = cfl h / (c0 + max |v_i|) over the fluid particles (FP64); returns
    (x, v, time + the sum of the dts, the last dt).  At rest this is the
    fixed dt = cfl h / c0.

    The paper keeps dt a variable that the scheduler may lower, and adapts it
    from a maximum over the particles in Example 1b; for SPH this reading
    takes the acoustic limit with the flow speed added."""
    import copy

    d = dom.dim
    x = np.asarray(x, np.float64)[:, :d].copy()
    v = np.asarray(v, np.float64)[:, :d].copy()
    fluid = np.ones(x.shape[0], bool) if fixed is None else ~np.asarray(fixed, bool)
    dt = 0.0
    for _ in range(n_steps):
        vmax = float(np.sqrt((v[fluid] ** 2).sum(axis=1)).max()) if fluid.any() else 0.0
        dt = cfl * prm.h / (prm.c0 + vmax)
        p = copy.copy(prm)
        p.dt = dt
        x, v, _, _, _ = step(dom, p, x, v, fixed=fixed, n_steps=1, nthreads=nthreads)
        time += dt
    return x, v, time, dt


# --------------------------------------------------------------------------
# Example 1a operator set
# --------------------------------------------------------------------------

def continuity(dom: Domain, prm: Params, x, v, rho, which=None, nthreads=None):
    """drho/dt = -rho_i sum_j (v_j - v_i) . grad_i W_ij m / rho_j for all
    particles (or the subset ``which``); rho is given for all particles."""
    x3, v3 = _x3(x), _x3(v)
    n = x3.shape[0]
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    w = None if which is None else np.ascontiguousarray(which, dtype=np.int64)
    m = n if w is None else w.shape[0]
    drho = np.zeros(m)
    rc = _load().or_continuity(ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3),
                               _ptr(v3), _ptr(rho), m, _ptr(w), _ptr(drho),
                               nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_continuity failed")
    return drho


def linear_eos(prm: Params, rho: float) -> float:
    """p = c^2 (rho - rho0) (Example 1a)."""
    return _load().or_linear_eos(ctypes.byref(prm._c()), rho)


def momentum(dom: Domain, prm: Params, x, v, rho, p, fixed=None, which=None, nthreads=None):
    """Example 1a accelerations: pressure gradient plus artificial viscosity
    plus g; rho and p are given for all particles."""
    x3, v3 = _x3(x), _x3(v)
    n = x3.shape[0]
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    w = None if which is None else np.ascontiguousarray(which, dtype=np.int64)
    m = n if w is None else w.shape[0]
    a = np.zeros((m, 3))
    rc = _load().or_momentum(ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3),
                             _ptr(v3), _ptr(rho), _ptr(p), _ptr(fx), m, _ptr(w), _ptr(a),
                             nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_momentum failed")
    return a[:, : dom.dim]


def step_ex1a(dom: Domain, prm: Params, x, v, rho, fixed=None, n_steps=1, nthreads=None):
    """Advance (x, v, rho) by n_steps of Example 1a; returns
    (x, v, rho, drho, p, a), the last three of the last step."""
    x3, v3 = _x3(x), _x3(v)
    n = x3.shape[0]
    r = np.array(rho, dtype=np.float64, copy=True)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    drho = np.zeros(n)
    p = np.zeros(n)
    a = np.zeros((n, 3))
    rc = _load().or_step_ex1a(ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3),
                              _ptr(v3), _ptr(r), _ptr(fx), int(n_steps), _ptr(drho), _ptr(p),
                              _ptr(a), nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_step_ex1a failed")
    d = dom.dim
    return x3[:, :d], v3[:, :d], r, drho, p, a[:, :d]


# --------------------------------------------------------------------------
# pair laws: DEM contact (Example 2) and social force (Sec. 6)
# --------------------------------------------------------------------------

def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def law_diag(law: str, dom: Domain, prm: Params, x, v, R, m, q, v0=None, goal=None, fixed=None, nthreads=None):
    """Accelerations of a pair law ("dem" or "social") and, per particle,
    how well its sum is conditioned (a test diagnostic): columns (sum_j
    |F_ij| / m_i + |own term| + |g|, the smallest overlap delta / (R_i +
    R_j) of its contacts, the smallest |v_t| / |v_j - v_i| of its sliding
    contacts; inf where there are none)."""
    x3, v3 = _x3(x), _x3(v)
    n = x3.shape[0]
    a = np.zeros((n, 3))
    diag = np.zeros((n, 3))
    lid = {"dem": 0, "social": 1}[law]
    g3 = None if goal is None else _x3(goal)
    rc = _load().or_law_diag(lid, ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3), _ptr(v3),
                             _ptr(_f64(R)), _ptr(_f64(m)), _ptr(_f64(q)),
                             _ptr(None if v0 is None else _f64(v0)), _ptr(g3), _ptr(_u8(fixed)), n, None,
                             _ptr(a), _ptr(diag), nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_law_diag failed")
    return a[:, : dom.dim], diag


def dem(dom: Domain, prm: Params, x, v, R, m, q, fixed=None, which=None, nthreads=None):
    """DEM accelerations; q = (1 - nu^2) / E per particle, c_f = prm.law[0]."""
    x3, v3 = _x3(x), _x3(v)
    n = x3.shape[0]
    w = None if which is None else np.ascontiguousarray(which, dtype=np.int64)
    mm = n if w is None else w.shape[0]
    a = np.zeros((mm, 3))
    rc = _load().or_dem(ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3), _ptr(v3),
                        _ptr(_f64(R)), _ptr(_f64(m)), _ptr(_f64(q)), _ptr(_u8(fixed)), mm, _ptr(w),
                        _ptr(a), nthreads or default_threads())
    if rc == -5:
        raise ValueError("dem: a radius exceeds h (contacts beyond the cell stencil)")
    if rc != 0:
        raise MemoryError("or_dem failed")
    return a[:, : dom.dim]


def social(dom: Domain, prm: Params, x, v, R, m, c, v0, goal, fixed=None, which=None, nthreads=None):
    """Social force accelerations; A, B, k, tau = prm.law."""
    x3, v3, g3 = _x3(x), _x3(v), _x3(goal)
    n = x3.shape[0]
    w = None if which is None else np.ascontiguousarray(which, dtype=np.int64)
    mm = n if w is None else w.shape[0]
    a = np.zeros((mm, 3))
    rc = _load().or_social(ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3), _ptr(v3),
                           _ptr(_f64(R)), _ptr(_f64(m)), _ptr(_f64(c)), _ptr(_f64(v0)), _ptr(g3),
                           _ptr(_u8(fixed)), mm, _ptr(w), _ptr(a), nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_social failed")
    return a[:, : dom.dim]


def step_law(law: str, dom: Domain, prm: Params, x, v, R, m, q, v0=None, goal=None, fixed=None,
             n_steps=1, nthreads=None):
    """n_steps semi-implicit Euler steps of a pair law ("dem" or "social");
    returns (x, v, a) with a of the last step."""
    x3, v3 = _x3(x), _x3(v)
    n = x3.shape[0]
    a = np.zeros((n, 3))
    lid = {"dem": 0, "social": 1}[law]
    g3 = None if goal is None else _x3(goal)
    rc = _load().or_step_law(lid, ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3), _ptr(v3),
                             _ptr(_f64(R)), _ptr(_f64(m)), _ptr(_f64(q)),
                             _ptr(None if v0 is None else _f64(v0)), _ptr(g3), _ptr(_u8(fixed)),
                             int(n_steps), _ptr(a), nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_step_law failed")
    d = dom.dim
    return x3[:, :d], v3[:, :d], a[:, :d]


# --------------------------------------------------------------------------
# Example 1b: Cahn-Hilliard with sph_L0
# --------------------------------------------------------------------------

def laplacian(dom: Domain, prm: Params, x, A, kdim=None, which=None, nthreads=None):
    """sph_L0: L(A)_i = 2 sum_j (A_i - A_j) F_ij m/rho0, kernel normalised in
    kdim dimensions (default: the domain's)."""
    x3 = _x3(x)
    n = x3.shape[0]
    w = None if which is None else np.ascontiguousarray(which, dtype=np.int64)
    m = n if w is None else w.shape[0]
    out = np.zeros(m)
    rc = _load().or_laplacian(ctypes.byref(dom._c()), ctypes.byref(prm._c()), int(kdim or dom.dim), n,
                              _ptr(x3), _ptr(_f64(A)), m, _ptr(w), _ptr(out), nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_laplacian failed")
    return out


def ch_steps(dom: Domain, prm: Params, x, c, time, dt, n_steps, kdim=2, nthreads=None):
    """n_steps of Example 1b (eq1-eq5); returns (c, time, dt, mu, cdot), the
    last two of the last step.  D, gamma, fac = prm.law[0..2]."""
    x3 = _x3(x)
    n = x3.shape[0]
    cc = np.array(c, dtype=np.float64, copy=True)
    clock = np.array([time, dt], dtype=np.float64)
    mu = np.zeros(n)
    cdot = np.zeros(n)
    rc = _load().or_ch_steps(ctypes.byref(dom._c()), ctypes.byref(prm._c()), int(kdim), n, _ptr(x3), _ptr(cc),
                             _ptr(clock), int(n_steps), _ptr(mu), _ptr(cdot), nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_ch_steps failed")
    return cc, float(clock[0]), float(clock[1]), mu, cdot


def step_vjp(dom: Domain, prm: Params, x, v, lam_x_next, lam_v_next, fixed=None, nthreads=None):
    """Reverse mode of one :func:`step`: returns (lam_x, lam_v, dL/dnu, dL/dc0)."""
    x3, v3 = _x3(x), _x3(v)
    lx, lv = _x3(lam_x_next), _x3(lam_v_next)
    n = x3.shape[0]
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    ox = np.zeros((n, 3))
    ov = np.zeros((n, 3))
    dnu = ctypes.c_double(0.0)
    dc0 = ctypes.c_double(0.0)
    rc = _load().or_step_vjp(ctypes.byref(dom._c()), ctypes.byref(prm._c()), n, _ptr(x3), _ptr(v3),
                             _ptr(fx), _ptr(lx), _ptr(lv), _ptr(ox), _ptr(ov),
                             ctypes.byref(dnu), ctypes.byref(dc0), nthreads or default_threads())
    if rc == -4:
        raise ValueError("step_vjp: domains with symmetric faces are not supported")
    if rc != 0:
        raise MemoryError("or_step_vjp failed")
    d = dom.dim
    return ox[:, :d], ov[:, :d], dnu.value, dc0.value


# --------------------------------------------------------------------------
# rollout loss and its gradient (checkpointed reverse sweep)
# --------------------------------------------------------------------------

def min_image(dom: Domain, d):
    """Displacements folded onto the nearest periodic image on periodic axes."""
    d = np.array(d, dtype=np.float64, copy=True)
    L = dom.length()
    for k in range(dom.dim):
        if dom.periodic[k]:
            d[:, k] -= L[k] * np.rint(d[:, k] / L[k])
    return d


def rollout_loss(dom: Domain, prm: Params, x0, v0, target, n_steps, fixed=None, nthreads=None):
    """L = (1/(N d)) sum_i |x_i^T - target_i|^2 (minimum image), over fluid."""
    x, _, _, _, _ = step(dom, prm, x0, v0, fixed=fixed, n_steps=n_steps, nthreads=nthreads)
    d = min_image(dom, x - np.asarray(target)[:, : dom.dim])
    mask = np.ones(d.shape[0], bool) if fixed is None else ~np.asarray(fixed, bool)
    return float((d[mask] ** 2).sum() / (mask.sum() * dom.dim))


def rollout_vjp(dom: Domain, prm: Params, x0, v0, n_steps, lam_x_T, lam_v_T, checkpoint_every=20,
                fixed=None, nthreads=None):
    """Reverse mode of ``n_steps`` of :func:`step` (the derivative the paper
    does not have): given cotangents lam_x_T, lam_v_T of the final positions
    and velocities (particle order of x0), returns (lam_x0, lam_v0, dL/dnu,
    dL/dc0), the cotangents of the initial state and of the two constants.
    The periodic shift of a leaving particle has derivative one, so the
    final position's cotangent is taken as that of the unshifted position.

    Forward: store (x, v) every ``checkpoint_every`` steps.  Backward: for
    each segment, recompute its states from the checkpoint, then apply the
    one-step VJPs in reverse order."""
    d = dom.dim
    x = np.asarray(x0, np.float64)[:, :d].copy()
    v = np.asarray(v0, np.float64)[:, :d].copy()
    ckpt = []
    for s in range(n_steps):
        if s % checkpoint_every == 0:
            ckpt.append((s, x.copy(), v.copy()))
        x, v, _, _, _ = step(dom, prm, x, v, fixed=fixed, n_steps=1, nthreads=nthreads)
    lam_x = np.array(lam_x_T, np.float64)[:, :d].copy()
    lam_v = np.array(lam_v_T, np.float64)[:, :d].copy()
    dnu = 0.0
    dc0 = 0.0
    for (s0, xc, vc) in reversed(ckpt):
        s1 = min(s0 + checkpoint_every, n_steps)
        states = [(xc.copy(), vc.copy())]
        for _ in range(s0, s1 - 1):
            xn, vn, _, _, _ = step(dom, prm, states[-1][0], states[-1][1], fixed=fixed,
                                   n_steps=1, nthreads=nthreads)
            states.append((xn, vn))
        for (xs, vs) in reversed(states):
            lam_x, lam_v, a, b = step_vjp(dom, prm, xs, vs, lam_x, lam_v, fixed=fixed,
                                          nthreads=nthreads)
            dnu += a
            dc0 += b
    return lam_x, lam_v, dnu, dc0


def rollout_grad(dom: Domain, prm: Params, x0, v0, target, n_steps, checkpoint_every=20,
                 fixed=None, nthreads=None):
    """(L, dL/dv0, dL/dnu, dL/dc0) of :func:`rollout_loss`: the loss's
    derivative in the final positions, lam_x = 2 delta / (N d) over fluid
    particles (delta the minimum-image displacement from the target), swept
    back by :func:`rollout_vjp`."""
    d = dom.dim
    x, _, _, _, _ = step(dom, prm, x0, v0, fixed=fixed, n_steps=n_steps, nthreads=nthreads)
    delta = min_image(dom, x - np.asarray(target)[:, :d])
    mask = np.ones(delta.shape[0], bool) if fixed is None else ~np.asarray(fixed, bool)
    nf = int(mask.sum())
    loss = float((delta[mask] ** 2).sum() / (nf * d))
    lam_x = np.where(mask[:, None], 2.0 * delta / (nf * d), 0.0)
    _, lam_v, dnu, dc0 = rollout_vjp(dom, prm, x0, v0, n_steps, lam_x, np.zeros_like(lam_x),
                                     checkpoint_every=checkpoint_every, fixed=fixed, nthreads=nthreads)
    return loss, lam_v, dnu, dc0


# --------------------------------------------------------------------------
# neighbour lists reused between builds (a Verlet list)
# --------------------------------------------------------------------------

def pair_keys(dom: Domain, x, radius: float) -> np.ndarray:
    """Every pair closer than ``radius`` (FP64, minimum image on periodic
    axes), as sorted keys (i n + j) 27 + image: image = sum_k 3^k c_k with
    c_k = 0 for j itself, 1 or 2 for j's reflection in the lower or upper
    symmetric face along axis k (a particle's own reflection included)."""
    x = np.asarray(x, dtype=np.float64)
    n, d = x.shape[0], dom.dim
    L = dom.length()
    lo = np.array(dom.origin[:3], dtype=np.float64)
    choices = [(0, 1, 2) if dom.symmetric[k] else (0,) for k in range(d)]
    out = []
    for combo in np.array(np.meshgrid(*choices, indexing="ij")).reshape(d, -1).T:
        xj = x.copy()
        code = 0
        for k in range(d):
            if combo[k] == 1:
                xj[:, k] = 2.0 * lo[k] - x[:, k]
            elif combo[k] == 2:
                xj[:, k] = 2.0 * (lo[k] + L[k]) - x[:, k]
            code += int(combo[k]) * 3 ** k
        for i0 in range(0, n, 256):
            diff = xj[None, :, :] - x[i0:i0 + 256, None, :]
            for k in range(d):
                if dom.periodic[k]:
                    diff[:, :, k] -= L[k] * np.rint(diff[:, :, k] / L[k])
            ii, jj = np.nonzero((diff * diff).sum(axis=2) < radius * radius)
            if code == 0:
                keep = ii + i0 != jj
                ii, jj = ii[keep], jj[keep]
            out.append(((ii + i0).astype(np.int64) * n + jj) * 27 + code)
    return np.unique(np.concatenate(out)) if out else np.zeros(0, np.int64)


def verlet_steps(dom: Domain, prm: Params, x, v, skin: float, n_steps: int, fixed=None, rho=None,
                 limit_fraction: float = 0.5, nthreads=None, step_fn=None, check: bool = True):
    """n_steps of :func:`step` (or of :func:`step_ex1a` when ``rho`` is
    given, or of ``step_fn(x, v) -> (x, v)``, e.g. one step of a pair law)
    with a Verlet neighbour list kept beside them: the pairs closer
    than 2h + skin at the last build, rebuilt before a step at whose start
    some particle lies farther than

        lim = limit_fraction * skin

    from its build-time position.  Before every step (unless ``check`` is
    false: then only the build schedule is kept) it checks that each pair
    closer than 2h is in the list, and raises AssertionError if not:
    with limit_fraction = 1/2 two particles close a gap of at most 2 lim =
    skin between builds, and a pair left out of the list was at least 2h +
    skin apart, so the check holds.  The steps themselves do not
    use the list (pairs beyond 2h add exact zeros), so x and v are those of
    the plain rollout.  A particle shifted across a face of a non-periodic
    axis has moved about a box length, which forces a build.  Returns
    (x, v, rho, builds, build_steps)."""
    d = dom.dim
    x = np.asarray(x, dtype=np.float64)[:, :d].copy()
    v = np.asarray(v, dtype=np.float64)[:, :d].copy()
    r = None if rho is None else np.array(rho, dtype=np.float64, copy=True)
    lim = limit_fraction * skin
    listed = None
    x_build = None
    build_steps = []
    for s in range(n_steps):
        if x_build is None or (min_image(dom, x - x_build) ** 2).sum(axis=1).max() > lim * lim:
            listed = pair_keys(dom, x, 2.0 * prm.h + skin) if check else None
            x_build = x.copy()
            build_steps.append(s)
        if check:
            missing = np.setdiff1d(pair_keys(dom, x, 2.0 * prm.h), listed, assume_unique=True)
            if missing.size:
                raise AssertionError(f"step {s}: {missing.size} pairs closer than 2h are not in the list")
        if step_fn is not None:
            x, v = step_fn(x, v)
        elif r is None:
            x, v, _, _, _ = step(dom, prm, x, v, fixed=fixed, n_steps=1, nthreads=nthreads)
        else:
            x, v, r, _, _, _ = step_ex1a(dom, prm, x, v, r, fixed=fixed, n_steps=1, nthreads=nthreads)
    return x, v, r, len(build_steps), build_steps
