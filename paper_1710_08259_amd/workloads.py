"""Seeded synthetic inputs for the WCSPH hot path.

This module only *generates* inputs: particle lattices with jitter, random
velocities, wall layers and the case constants.  It contains none of the
method's arithmetic (no kernel, no sums, no equation of state) and imports
neither the HIP binding nor the oracle, so both sides of every parity test
can take their inputs from here.

Conventions
-----------
* Everything is generated in FP64 with ``numpy.random.default_rng(seed)``
  and rounded once to FP32; the GPU receives the FP32 values and the oracle
  the same values widened to FP64.
* Lattice sites sit at ``(i + 1/2) dx``; jitter is uniform per component.
* The cell edge of every axis is rounded to FP32 first and the box length is
  then ``n_cells * cell_edge`` exactly, so a periodic box means the same
  thing in FP32 and FP64.  The lattice spacing is derived from that length.
* Cell edges are ``L / floor(L / 2h)`` (never below the support 2h).
* Fixed (wall) particles come last within a case.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

PERIODIC = 0
CUTOFF = 1
SYMMETRIC = 2

# Models of the interaction step: density summation + Tait + Morris
# viscosity, or Example 1a's continuity + linear EOS + artificial viscosity.
SUMMATION = 0
CONTINUITY = 1
DEM = 2         # Example 2's contact law
SOCIAL = 3      # the social force model
CAHN_HILLIARD = 4  # Example 1b


def _f32(x: float) -> float:
    return float(np.float32(x))


@dataclass
class Case:
    """One independent WCSPH problem."""

    dim: int
    ncell: tuple          # cells per axis, (nx, ny, nz); unused axes 1
    cell_size: tuple      # FP32-representable edge per axis
    origin: tuple         # FP32-representable lower corner
    boundary: tuple       # PERIODIC / CUTOFF / SYMMETRIC per axis
    h: float
    mass: float
    rho0: float
    c0: float
    gamma: float
    nu: float
    dt: float
    g: tuple
    pos: np.ndarray       # (n, dim) float32 absolute positions
    vel: np.ndarray       # (n, dim) float32
    n_fixed: int = 0
    name: str = ""
    model: int = SUMMATION
    alpha_av: float = 0.0                 # artificial viscosity coefficient (CONTINUITY)
    rho: Optional[np.ndarray] = None      # (n,) float32 initial density (CONTINUITY)
    law: tuple = ()                       # pair-law constants (DEM: (c_f,); SOCIAL: (A, B, k, tau))
    radius: Optional[np.ndarray] = None   # (n,) pair-law attributes, input order
    pmass: Optional[np.ndarray] = None
    coef: Optional[np.ndarray] = None     # DEM: (1 - nu^2)/E; SOCIAL: attraction c; CAHN_HILLIARD: c
    v0: Optional[np.ndarray] = None       # SOCIAL: desired speed
    goal: Optional[np.ndarray] = None     # SOCIAL: (n, dim) absolute target
    skin: float = 0.0                     # neighbour-list reach beyond 2h (Verlet steps)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.ncell[0]) * int(self.ncell[1]) * int(self.ncell[2])

    def length(self) -> np.ndarray:
        return np.array([self.ncell[k] * self.cell_size[k] for k in range(3)])

    def fixed_mask(self) -> np.ndarray:
        m = np.zeros(self.n, bool)
        if self.n_fixed:
            m[self.n - self.n_fixed:] = True
        return m


def _cells_for(length: float, h: float, skin: float = 0.0) -> tuple[int, float]:
    reach = 2.0 * h + skin
    n = int(math.floor(length / reach))
    n = max(n, 1)
    cs = _f32(length / n)
    if cs < reach:  # FP32 rounding went below the support: one cell fewer
        n -= 1
        cs = _f32(length / n)
    return n, cs


def lattice_case(dim, n_side, dx, h_over_dx, jitter, v_sigma, seed, *, c0=10.0, nu=1e-3,
                 dt=1e-4, rho0=1000.0, gamma=7.0, g=(0.0, 0.0, 0.0), skin=0.0, name="") -> Case:
    """Periodic box filled with a jittered square/cubic lattice.

    ``n_side`` lattice sites per axis at nominal spacing ``dx``; ``jitter``
    is the half-width of the uniform per-component perturbation in units of
    dx; velocities are N(0, v_sigma) per component.  ``skin``: the
    neighbour-list skin (cells no smaller than 2h + skin)."""
    rng = np.random.default_rng(seed)
    n_side = tuple(int(s) for s in n_side) + (1,) * (3 - dim)
    h = h_over_dx * dx
    ncell, cs, spacing = [1, 1, 1], [1.0, 1.0, 1.0], [dx, dx, dx]
    for k in range(dim):
        n, c = _cells_for(n_side[k] * dx, h, skin)
        ncell[k], cs[k] = n, c
        spacing[k] = n * c / n_side[k]
    grids = np.meshgrid(*[(np.arange(n_side[k]) + 0.5) * spacing[k] for k in range(dim)],
                        indexing="ij")
    pos = np.stack([g_.ravel(order="F") for g_ in grids], axis=1)  # x fastest
    pos += (rng.uniform(-1.0, 1.0, pos.shape) * jitter) * np.array(spacing[:dim])
    for k in range(dim):
        L = ncell[k] * cs[k]
        pos[:, k] = np.mod(pos[:, k], L)
    vel = rng.normal(0.0, v_sigma, pos.shape)
    mass = rho0 * float(np.prod(spacing[:dim]))
    return Case(dim=dim, ncell=tuple(ncell), cell_size=tuple(cs), origin=(0.0, 0.0, 0.0),
                boundary=(PERIODIC,) * 3, h=h, mass=mass, rho0=rho0, c0=c0, gamma=gamma,
                nu=nu, dt=dt, g=tuple(g), pos=pos.astype(np.float32),
                vel=vel.astype(np.float32), n_fixed=0, name=name, skin=float(skin))


def dam_break_case(dx=0.005, h_over_dx=1.2, c0=30.0, nu=1e-6, rho0=1000.0, gamma=7.0,
                   fluid=(0.4, 0.4, 0.8), tank=(1.6, 0.4, 1.0), layers=3, g=-9.81,
                   cfl=0.25, name="dam_break") -> Case:
    """3-D dam-break shape: a fluid column against the x = 0 wall of an
    open-top tank whose floor and four sides are ``layers`` layers of fixed
    particles on the same lattice.  Cut-off box, gravity along -z,
    dt = cfl * h / c0, fluid at rest."""
    h = h_over_dx * dx
    nf = [int(round(fluid[k] / dx)) for k in range(3)]
    nt = [int(round(tank[k] / dx)) for k in range(3)]
    fl = np.stack(np.meshgrid(*[np.arange(nf[k]) for k in range(3)], indexing="ij"), -1)
    fl = fl.reshape(-1, 3, order="F")
    ix = np.arange(-layers, nt[0] + layers)
    iy = np.arange(-layers, nt[1] + layers)
    iz = np.arange(-layers, nt[2])
    W = np.stack(np.meshgrid(ix, iy, iz, indexing="ij"), -1).reshape(-1, 3, order="F")
    inside = ((W[:, 0] >= 0) & (W[:, 0] < nt[0]) & (W[:, 1] >= 0) & (W[:, 1] < nt[1])
              & (W[:, 2] >= 0))
    W = W[~inside]
    idx = np.concatenate([fl, W], axis=0).astype(np.float64)
    pos = (idx + 0.5) * dx
    # cut-off box: one extra lattice spacing around the walls, 10 % headroom
    lo = np.array([-(layers + 1) * dx] * 3)
    hi = np.array([tank[0] + (layers + 1) * dx, tank[1] + (layers + 1) * dx, tank[2] * 1.1])
    origin = tuple(_f32(v) for v in lo)
    ncell, cs = [1, 1, 1], [1.0, 1.0, 1.0]
    for k in range(3):
        ncell[k], cs[k] = _cells_for(hi[k] - origin[k], h)
    vel = np.zeros_like(pos)
    return Case(dim=3, ncell=tuple(ncell), cell_size=tuple(cs), origin=origin,
                boundary=(CUTOFF,) * 3, h=h, mass=rho0 * dx ** 3, rho0=rho0, c0=c0,
                gamma=gamma, nu=nu, dt=cfl * h / c0, g=(0.0, 0.0, g),
                pos=pos.astype(np.float32), vel=vel.astype(np.float32),
                n_fixed=int(W.shape[0]), name=name)


def ex1a_dam_break(scale: float = 1.0, name: str = "") -> Case:
    """The 2-D dam break of Example 1a (its appendix configuration), with
    the resolution refined by ``scale``: h = 0.25 / scale, dx = h / 1.1,
    rho0 = 1000, c = 50 m/s, m = dx^2 rho0, g = (0, -9.81), alpha_av = 0.1,
    dt = 1e-3 / scale (the paper's dt at scale 1, kept at the same CFL
    number when refined).  Box: cells of edge 2h, round(7/h) x round(10/h) of
    them (the listing's integer extents read as cell counts), symmetric
    faces on both axes.  Fluid: the listing's 7 x 4 m grid of spacing dx,
    sites at (k + 1/2) dx inside it (31 x 18 at scale 1), at rest,
    rho = rho0.  The half-spacing keeps every particle off the faces: one on
    a symmetric face coincides with its own mirror image, feels nothing from
    it, and would fall through the floor in the first step."""
    h = 0.25 / scale
    dx = h / 1.1
    cs = _f32(2.0 * h)
    if cs < 2.0 * h:  # never below the support in FP32
        cs = float(np.nextafter(np.float32(cs), np.float32(np.inf)))
    ncell = (int(round(7.0 / h)), int(round(10.0 / h)), 1)
    nx = int(math.ceil(7.0 / dx - 0.5 - 1e-9))
    ny = int(math.ceil(4.0 / dx - 0.5 - 1e-9))
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    pos = (np.stack([ix.ravel(order="F"), iy.ravel(order="F")], axis=1).astype(np.float64) + 0.5) * dx
    rho0 = 1000.0
    n = pos.shape[0]
    return Case(dim=2, ncell=ncell, cell_size=(cs, cs, 1.0), origin=(0.0, 0.0, 0.0),
                boundary=(SYMMETRIC, SYMMETRIC, CUTOFF), h=h, mass=dx * dx * rho0, rho0=rho0,
                c0=50.0, gamma=1.0, nu=0.0, dt=1e-3 / scale, g=(0.0, -9.81, 0.0),
                pos=pos.astype(np.float32), vel=np.zeros((n, 2), np.float32), n_fixed=0,
                name=name or f"ex1a_dam_break_2d_{n}", model=CONTINUITY, alpha_av=0.1,
                rho=np.full(n, rho0, np.float32))


def mirror_box_case(dim, boundary, seed, n=2000, ncell=(12, 10, 8), h=0.02, model=SUMMATION,
                    v_sigma=0.5, rho_sigma=0.02, name="") -> Case:
    """Random particles in a box with (some) symmetric faces, crowded near
    the faces and corners: about a fifth of them within 2h of a face, a few
    exactly on the lower x face.  Cells of edge 2.14h; velocities N(0,
    v_sigma); with the continuity model, densities rho0 (1 + N(0, rho_sigma)).
    Particle volume (0.8 h)^dim."""
    rng = np.random.default_rng(seed)
    nc = tuple(int(c) for c in ncell[:dim]) + (1,) * (3 - dim)
    cs = tuple(_f32(2.0 * h * 1.07) for _ in range(dim)) + (1.0,) * (3 - dim)
    L = np.array([nc[k] * cs[k] for k in range(3)])
    x = rng.uniform(0, 1, (n, dim)) * L[:dim]
    near = rng.random(n) < 0.35
    for k in range(dim):
        side = rng.random(n) < 0.5
        d = rng.uniform(0, 2.0 * h, n)
        pick = near & (rng.random(n) < 0.6)
        x[pick & side, k] = d[pick & side]
        x[pick & ~side, k] = L[k] - d[pick & ~side]
    x[:3, 0] = 0.0
    x = np.minimum(x, np.nextafter(L[:dim].astype(np.float32), np.float32(0)))
    rho0 = 1000.0
    rho = (rho0 * (1.0 + rho_sigma * rng.standard_normal(n))).astype(np.float32) if model == CONTINUITY else None
    return Case(dim=dim, ncell=nc, cell_size=cs, origin=(0.0, 0.0, 0.0), boundary=tuple(boundary), h=h,
                mass=rho0 * (0.8 * h) ** dim, rho0=rho0, c0=20.0, gamma=7.0 if model == SUMMATION else 1.0,
                nu=1e-3 if model == SUMMATION else 0.0, dt=1e-4, g=(0.0, -9.81, 0.0),
                pos=x.astype(np.float32), vel=rng.normal(0.0, v_sigma, (n, dim)).astype(np.float32),
                n_fixed=0, name=name or f"mirror_box_{dim}d_{seed}", model=model,
                alpha_av=0.1 if model == CONTINUITY else 0.0, rho=rho)


def dem_damper(scale: int = 1, seed: int = 7, jitter: float = 0.3, cf: float = 0.3, dt: float = 2e-5,
               spacing: float = 0.1 / 9, v_sigma: float = 0.0, skin: float = 0.0, name: str = "") -> Case:
    """Example 2's particle damper without the tank's own motion: spheres of
    R = 4 mm, rho = 7850, E = 2.06e6 Pa (as the table prints it), nu = 0.33,
    g = -9.81 ez, in a cubic box of edge 0.1 scale m with symmetric faces.
    The table's 567 spheres are a 9 x 9 x 7 lattice; ``scale`` multiplies
    each lattice side (567 scale^3 spheres).  Sites (i + 1/2) spacing
    (0.1/9 m: the table's tank), jittered by U(+-jitter) of the gap between
    spheres (of the spacing when they overlap), velocities N(0, v_sigma).
    Cells of edge >= 2R + skin (h = R); c_f (not given) = 0.3."""
    rng = np.random.default_rng(seed)
    R, rho_s, E, nu = 0.004, 7850.0, 2.06e6, 0.33
    L = 0.1 * scale
    side = (9 * scale, 9 * scale, 7 * scale)
    sp = spacing
    grids = np.meshgrid(*[(np.arange(side[k]) + 0.5) * sp for k in range(3)], indexing="ij")
    pos = np.stack([g_.ravel(order="F") for g_ in grids], axis=1)
    gap = sp - 2 * R if sp > 2 * R else sp
    pos += rng.uniform(-1, 1, pos.shape) * jitter * gap / 2
    n = pos.shape[0]
    nc, cs = _cells_for(L, _f32(R), skin)  # h = R as stored (FP32): contacts reach 2h
    m = rho_s * 4.0 / 3.0 * math.pi * R ** 3
    return Case(dim=3, ncell=(nc, nc, nc), cell_size=(cs, cs, cs), origin=(0.0, 0.0, 0.0),
                boundary=(SYMMETRIC,) * 3, h=_f32(R), mass=m, rho0=rho_s, c0=1.0, gamma=1.0, nu=0.0, dt=dt,
                g=(0.0, 0.0, -9.81), pos=pos.astype(np.float32),
                vel=rng.normal(0.0, v_sigma, (n, 3)).astype(np.float32),
                n_fixed=0, name=name or f"dem_damper_{n}", model=DEM, law=(cf,),
                radius=np.full(n, R, np.float32), pmass=np.full(n, m, np.float32),
                coef=np.full(n, (1 - nu ** 2) / E, np.float32), skin=float(skin))


def social_room(width: float = 20.0, density: float = 1.0, seed: int = 11, c_max: float = 0.0,
                dt: float = 1e-3, name: str = "") -> Case:
    """A square room of side ``width`` for the social force model: walls of
    fixed people (R_w = 0.1 m, 0.2 m apart) with a 2 m exit in the right
    wall; people at ``density`` per m^2 inside (a square lattice jittered by
    U(+-0.1) of its spacing), masses U(50, 100) kg, radii
    0.002 m + 0.15 (the paper's rule), desired speeds U(0.8, 1.5) m/s, all
    heading for a point 3 m beyond the exit, at rest.  A, B, k, tau = 2000 N,
    0.08 m, 1.2e5 kg/s^2, 0.5 s; attraction c ~ U(0, c_max).  Cut-off box
    around the room, cells >= 1.2 m (interaction radius 2h = 1.2 m)."""
    rng = np.random.default_rng(seed)
    sp = 1.0 / math.sqrt(density)
    k = int((width - 1.0) / sp)
    ix, iy = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    people = 0.5 + (np.stack([ix.ravel(order="F"), iy.ravel(order="F")], axis=1) + 0.5) * sp
    people += rng.uniform(-0.1, 0.1, people.shape) * sp
    n = people.shape[0]
    wall = []
    ticks = np.arange(0.0, width + 1e-9, 0.2)
    for t in ticks:
        wall += [(t, 0.0), (t, width), (0.0, t)]
        if abs(t - width / 2) > 1.0:
            wall.append((width, t))
    wall = np.array(wall)
    pos = np.concatenate([people, wall])
    nw = wall.shape[0]
    mass = np.concatenate([rng.uniform(50, 100, n), np.full(nw, 80.0)])
    radius = np.concatenate([0.002 * mass[:n] + 0.15, np.full(nw, 0.1)])
    h = 0.6
    lo = np.array([-2.0, -2.0])
    hi = np.array([width + 5.0, width + 2.0])
    ncell, cs = [1, 1, 1], [1.0, 1.0, 1.0]
    for k in range(2):
        ncell[k], cs[k] = _cells_for(hi[k] - lo[k], h)
    goal = np.tile([width + 3.0, width / 2], (n + nw, 1))
    return Case(dim=2, ncell=tuple(ncell), cell_size=tuple(cs), origin=(float(lo[0]), float(lo[1]), 0.0),
                boundary=(CUTOFF,) * 3, h=h, mass=80.0, rho0=1.0, c0=1.0, gamma=1.0, nu=0.0, dt=dt,
                g=(0.0, 0.0, 0.0), pos=pos.astype(np.float32), vel=np.zeros((n + nw, 2), np.float32),
                n_fixed=nw, name=name or f"social_room_{n}", model=SOCIAL, law=(2000.0, 0.08, 1.2e5, 0.5),
                radius=radius.astype(np.float32), pmass=mass.astype(np.float32),
                coef=rng.uniform(0, c_max, n + nw).astype(np.float32),
                v0=np.concatenate([rng.uniform(0.8, 1.5, n), np.zeros(nw)]).astype(np.float32),
                goal=goal.astype(np.float32))


def ch_sphere(dx: float = 0.07, radius: float = 2.0, seed: int = 13, name: str = "") -> Case:
    """Example 1b: the Cahn-Hilliard equation on a sphere.  The paper reads
    its points from a file it does not include; here a Fibonacci lattice of
    round(4 pi R^2 / dx^2) points on a sphere of radius ``radius`` (2 m: inside
    the listing's box of +-15 cells of 2h) stands in for it.  dx = 0.07,
    h = 1.05 dx, m = dx^2 rho0, rho0 = 1000, D = 0.003, gamma = (2h/3)^2,
    dt = 0.003 to start, then 0.1 min(1/max|cdot|, gamma/(2h)^2);
    c ~ U(-1, 1).  Cells of 2h, +-15 of them (scaled with h) per axis,
    periodic (the listing's boundary 0)."""
    rng = np.random.default_rng(seed)
    n = int(round(4.0 * math.pi * radius * radius / dx ** 2))
    k = np.arange(n) + 0.5
    phi = np.arccos(1.0 - 2.0 * k / n)
    th = math.pi * (1.0 + 5.0 ** 0.5) * k
    pos = np.stack([radius * np.cos(th) * np.sin(phi), radius * np.sin(th) * np.sin(phi),
                    radius * np.cos(phi)], axis=1)
    h = 1.05 * dx
    cs = _f32(2.0 * h)
    if cs < 2.0 * h:
        cs = float(np.nextafter(np.float32(cs), np.float32(np.inf)))
    half = int(math.ceil(1.1 * radius / cs))
    nc = 2 * max(half, 15)
    o = _f32(-nc / 2 * cs)
    gamma = (2.0 * h / 3.0) ** 2
    return Case(dim=3, ncell=(nc, nc, nc), cell_size=(cs, cs, cs), origin=(o, o, o), boundary=(PERIODIC,) * 3,
                h=h, mass=dx * dx * 1000.0, rho0=1000.0, c0=1.0, gamma=1.0, nu=0.0, dt=0.003,
                g=(0.0, 0.0, 0.0), pos=pos.astype(np.float32), vel=np.zeros((n, 3), np.float32), n_fixed=0,
                name=name or f"ch_sphere_{n}", model=CAHN_HILLIARD, law=(0.003, gamma, 0.1),
                coef=rng.uniform(-1.0, 1.0, n).astype(np.float32))


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def periodic_2d_4096() -> Case:
    """2-D periodic, 64x64 lattice, dx 0.01 m, jitter U(+-0.01 dx), h 1.3 dx,
    c0 10 m/s, nu 1e-3, v ~ N(0, 0.1), dt 1e-4 (100-step parity case)."""
    return lattice_case(2, (64, 64), 0.01, 1.3, 0.01, 0.1, seed=1, c0=10.0, nu=1e-3,
                        dt=1e-4, name="periodic_2d_4096")


def dam_break_3d(dx=0.005) -> Case:
    """3-D dam-break shape: 0.4 x 0.4 x 0.8 m column, dx 0.005 m (1,024,000
    fluid + 571,308 wall particles), tank 1.6 x 0.4 x 1.0 m, c0 30 m/s."""
    return dam_break_case(dx=dx, name=f"dam_break_3d_dx{dx:g}")


def periodic_3d_8m() -> Case:
    """3-D periodic 256 x 256 x 128 jittered lattice = 8,388,608 particles,
    h 1.2 dx (56 lattice neighbours), jitter U(+-0.05 dx), v ~ N(0, 0.05)."""
    return lattice_case(3, (256, 256, 128), 0.01, 1.2, 0.05, 0.05, seed=3, c0=10.0,
                        nu=1e-3, dt=1e-4, name="periodic_3d_8388608")


def periodic_3d_262k() -> Case:
    """3-D periodic 64^3 = 262,144 (differentiation case)."""
    return lattice_case(3, (64, 64, 64), 0.01, 1.2, 0.05, 0.05, seed=5, c0=10.0, nu=1e-3,
                        dt=1e-4, name="periodic_3d_262144")


def batched_2d(n_cases=256, seed=4, max_side_exp=8.0) -> list[Case]:
    """Independent 2-D periodic cases: side round(2^U(5, max)), so particle
    counts are log-uniform in [1024, 65536]; nu ~ U(1e-6, 1e-3),
    c0 ~ U(5, 20) m/s; case b uses seed 1000 + b."""
    rng = np.random.default_rng(seed)
    sides = np.rint(2.0 ** rng.uniform(5.0, max_side_exp, n_cases)).astype(int)
    nus = rng.uniform(1e-6, 1e-3, n_cases)
    c0s = rng.uniform(5.0, 20.0, n_cases)
    return [lattice_case(2, (s, s), 0.01, 1.3, 0.01, 0.1, seed=1000 + b, c0=float(c0s[b]),
                         nu=float(nus[b]), dt=1e-4, name=f"batched_{b}")
            for b, s in enumerate(sides)]


def scaled(case: Case, **changes) -> Case:
    return replace(case, **changes)
