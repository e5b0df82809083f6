"""Seeded synthetic inputs for the stabilized implicit MPM (Zhao & Choo, arXiv 1905.00671).

This module builds problem *statements* only: background grids, material points, material
constants and the per-step boundary data (Dirichlet masks/values, nodal forces and fluxes) of
the strong form in Sec. 2.4.  It contains none of the method's arithmetic (no basis functions,
no constitutive law, no residuals).  Both the GPU library and the CPU oracle consume the arrays
produced here.

Workloads (sizes and physics follow the benchmark configurations of this repository):
  * ``terzaghi``      2D plane-strain consolidation column (Sec. 5.1 problem, re-parametrized).
  * ``footing2d``     2D displacement-controlled rigid strip footing on a half-model.
  * ``footing3d``     3D square footing on a quarter-model.
  * ``serving_trace`` a Poisson arrival stream of independent 2D problems.

Material points are placed 2 per axis per cell at (1/4, 3/4) h, with V0 = h^d / 2^d, GIMP
half-lengths lp0 = h/4, and mass m = rho0 V0 with the mixture density of Sec. 2.1,
rho0 = (1 - phi0) rho_s + phi0 rho_f.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

LINEAR, GIMP = 0, 1
HENCKY, NEO_HOOKEAN = 0, 1
TAU_OFF, TAU_WHITE, TAU_SUN, TAU_MONFORTE = 0, 1, 2, 3


@dataclass
class Grid:
    """Fixed structured background grid (Sec. 3.5: the mesh is never moved)."""
    dim: int
    ncell: Tuple[int, ...]
    h: float
    origin: Tuple[float, ...] = (0.0, 0.0, 0.0)

    @property
    def nnode_axis(self) -> Tuple[int, ...]:
        return tuple(n + 1 for n in self.ncell[: self.dim])

    @property
    def nnode(self) -> int:
        return int(np.prod(self.nnode_axis))

    @property
    def ncells(self) -> int:
        return int(np.prod(self.ncell[: self.dim]))

    def node_coords(self) -> np.ndarray:
        """Node coordinates, shape (nnode, dim); node id = ix + nx1*(iy + ny1*iz)."""
        axes = [self.origin[d] + self.h * np.arange(self.nnode_axis[d]) for d in range(self.dim)]
        mesh = np.meshgrid(*axes, indexing="ij")
        # natural order: x fastest
        return np.stack([m.transpose(*reversed(range(self.dim))).reshape(-1) for m in mesh], axis=1)

    def node_index(self, *idx) -> int:
        n = self.nnode_axis
        if self.dim == 2:
            return idx[0] + n[0] * idx[1]
        return idx[0] + n[0] * (idx[1] + n[1] * idx[2])


@dataclass
class Material:
    """Constants of Sec. 2: skeleton elasticity (E, nu), permeability k (the initial one when
    kozeny_carman is set), fluid viscosity mu_f, intrinsic densities, initial porosity and
    gravity."""
    model: int = NEO_HOOKEAN
    E: float = 10e6
    nu: float = 0.3
    k: float = 1e-12
    mu_f: float = 1e-3
    rho_s: float = 2500.0
    rho_f: float = 1000.0
    phi0: float = 0.33
    g: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    kozeny_carman: bool = False     # k(phi) from phi0 and the volume ratio (eq. kozeny-carman)
    alpha_vis: float = 0.0          # Kelvin-type damping parameter (s), dynamic problems only

    @property
    def rho0(self) -> float:
        return (1.0 - self.phi0) * self.rho_s + self.phi0 * self.rho_f


@dataclass
class Options:
    shape: int = LINEAR
    dynamic: int = 0
    beta: float = 0.25
    gamma: float = 0.5
    tau_kind: int = TAU_WHITE
    tau_scale: float = 1.0
    mixed: int = 0                 # 0: FP64 everywhere; 1: FP32 Jacobian/SpMV/preconditioner
    newton_rtol: float = 1e-8
    newton_atol_u: float = 0.0     # <= 0: 1e-12 E h^(dim-1)
    newton_atol_p: float = 0.0     # <= 0: 1e-12 h^dim / dt
    newton_max: int = 25
    krylov_rtol: float = 1e-8
    krylov_max: int = 4000
    drained_surface: int = 0       # 1: zero pore pressure on the current free surface of the material
    consistent_mass: int = 0       # 1: consistent-mass P2G mapping (solve with M_ij) instead of lumped
    negligible_mass: float = 0.0   # nodes below this fraction of the largest nodal mass are inactive (<= 0: 1e-15)
    schur: int = 0                 # Schur block of the preconditioner: 0 fixed-stress, 1 C - B2 diag(A)^-1 B1


@dataclass
class Particles:
    x: np.ndarray        # (np, dim)
    vol: np.ndarray      # (np,)
    mass: np.ndarray     # (np,)
    lp: np.ndarray       # (np, dim)   GIMP half-lengths (ignored by original MPM)
    v0: Optional[np.ndarray] = None   # (np, dim)
    p0: Optional[np.ndarray] = None   # (np,)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Workload:
    name: str
    grid: Grid
    material: Material
    options: Options
    particles: Particles
    dt: float
    nsteps: int
    bc: Callable[[int], Dict[str, np.ndarray]]   # step index (1-based) -> nodal BC arrays
    meta: Dict = field(default_factory=dict)


# ----------------------------------------------------------------------------------------------
# particles and boundary data
# ----------------------------------------------------------------------------------------------

def fill_particles(grid: Grid, cell_lo, cell_hi, rho0: float, ppa: int = 2,
                   jitter: float = 0.0, rng: Optional[np.random.Generator] = None) -> Particles:
    """Uniform filling of the cell box [cell_lo, cell_hi) with ppa material points per axis
    per cell at the centres of the ppa^d sub-cells ((1/4, 3/4) h for ppa = 2)."""
    d, h = grid.dim, grid.h
    sub = (np.arange(ppa) + 0.5) / ppa
    axes = []
    for a in range(d):
        cells = np.arange(cell_lo[a], cell_hi[a])
        axes.append(((cells[:, None] + sub[None, :]).reshape(-1)) * h + grid.origin[a])
    mesh = np.meshgrid(*axes, indexing="ij")
    x = np.stack([m.transpose(*reversed(range(d))).reshape(-1) for m in mesh], axis=1)
    if jitter > 0.0:
        rng = rng if rng is not None else np.random.default_rng(0)
        x = x + (rng.random(x.shape) - 0.5) * (jitter * h / ppa)
    n = x.shape[0]
    v0 = (h / ppa) ** d
    vol = np.full(n, v0)
    lp = np.full((n, d), 0.5 * h / ppa)
    return Particles(x=np.ascontiguousarray(x), vol=vol, mass=rho0 * vol, lp=lp)


def empty_bc(grid: Grid) -> Dict[str, np.ndarray]:
    n, d = grid.nnode, grid.dim
    return {
        "u_fixed": np.zeros((n, d), np.uint8),
        "u_inc": np.zeros((n, d), np.float64),
        "p_fixed": np.zeros(n, np.uint8),
        "p_val": np.zeros(n, np.float64),
        "f_ext": np.zeros((n, d), np.float64),
        "q_ext": np.zeros(n, np.float64),
    }


def _tol(grid: Grid) -> float:
    return 1e-9 * grid.h


def box_supports(grid: Grid, bc: Dict[str, np.ndarray], xlim: Tuple[float, ...]):
    """Rollers on every vertical face (normal displacement fixed on nodes at or beyond the face)
    and a fixed base (all displacement components fixed on nodes at or below the bottom)."""
    X = grid.node_coords()
    t = _tol(grid)
    d = grid.dim
    for a in range(d - 1):
        lo = X[:, a] <= grid.origin[a] + t
        hi = X[:, a] >= xlim[a] - t
        bc["u_fixed"][lo | hi, a] = 1
    base = X[:, d - 1] <= grid.origin[d - 1] + t
    bc["u_fixed"][base, :] = 1


# ----------------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------------

def terzaghi(ncell_x: int = 4, ncell_y: int = 40, h: float = 0.25, load: float = 10e3,
             k: float = 1e-10, dt: float = 0.1, nsteps: int = 10, tau_scale: float = 1.0,
             tau_kind: int = TAU_WHITE, model: int = HENCKY, E: float = 10e6, nu: float = 0.3,
             mu_f: float = 1e-3) -> Workload:
    """Plane-strain Terzaghi column (Sec. 5.1 set-up): rollers on both sides, fixed base,
    drained and loaded top, all other faces impermeable, no gravity.  The top edge load w is
    applied from the first step as consistent nodal forces of a linear edge (w h/2 at the two
    corners, w h at interior top nodes)."""
    grid = Grid(2, (ncell_x, ncell_y), h, (0.0, 0.0, 0.0))
    mat = Material(model=model, E=E, nu=nu, k=k, mu_f=mu_f)
    opt = Options(shape=LINEAR, dynamic=0, tau_kind=tau_kind, tau_scale=tau_scale)
    parts = fill_particles(grid, (0, 0), (ncell_x, ncell_y), mat.rho0)
    H = ncell_y * h
    W = ncell_x * h

    def bc(step: int):
        b = empty_bc(grid)
        box_supports(grid, b, (W,))
        X = grid.node_coords()
        top = np.abs(X[:, 1] - H) <= _tol(grid)
        b["p_fixed"][top] = 1
        for ix in range(ncell_x + 1):
            w = h if 0 < ix < ncell_x else 0.5 * h
            b["f_ext"][grid.node_index(ix, ncell_y), 1] = -load * w
        return b

    return Workload("terzaghi", grid, mat, opt, parts, dt, nsteps, bc,
                    meta=dict(H=H, W=W, load=load))


def footing2d(nx: int = 64, ny: int = 64, width: float = 10.0, empty_rows: int = 4,
              half_b: float = 1.0, delta: float = 5e-3, nsteps: int = 100, dt: float = 1e-3,
              k: float = 1e-16, dynamic: int = 1, shape: int = GIMP, tau_kind: int = TAU_WHITE,
              model: int = NEO_HOOKEAN, beta: float = 0.25, gamma: float = 0.5,
              seed: Optional[int] = None, k_range: Optional[Tuple[float, float]] = None,
              depth: Optional[float] = None, name: str = "footing2d") -> Workload:
    """Half-model of a rough rigid strip footing pushed down by delta per step.

    Footing reading: at step n the footing base is at y_f = H - (n-1) delta; every node with
    x <= B/2 and y >= y_f receives the Dirichlet increment (0, -delta).  Sides are rollers, the
    base is fixed, the top outside the footing (y >= H, x > B/2) is drained, the footing itself
    is impermeable.  When ``seed`` is given the permeability is drawn once per seed,
    k = 10^(lo + (hi-lo) u), u ~ U(0,1) from numpy's default_rng(seed)."""
    h = width / nx
    depth = depth if depth is not None else ny * h
    grid = Grid(2, (nx, ny + empty_rows), h, (0.0, 0.0, 0.0))
    if seed is not None:
        lo, hi = k_range if k_range is not None else (-14.0, -10.0)
        u = np.random.default_rng(seed).random()
        k = 10.0 ** (lo + (hi - lo) * u)
    mat = Material(model=model, k=k)
    opt = Options(shape=shape, dynamic=dynamic, beta=beta, gamma=gamma, tau_kind=tau_kind)
    parts = fill_particles(grid, (0, 0), (nx, ny), mat.rho0)
    H = ny * h
    W = nx * h
    X = grid.node_coords()
    t = _tol(grid)

    def bc(step: int):
        b = empty_bc(grid)
        box_supports(grid, b, (W,))
        yf = H - (step - 1) * delta
        foot = (X[:, 0] <= half_b + t) & (X[:, 1] >= yf - t)
        b["u_fixed"][foot, :] = 1
        b["u_inc"][foot, 0] = 0.0
        b["u_inc"][foot, 1] = -delta
        drained = (X[:, 1] >= H - t) & (X[:, 0] > half_b + t)
        b["p_fixed"][drained] = 1
        return b

    return Workload(name, grid, mat, opt, parts, dt, nsteps, bc,
                    meta=dict(H=H, W=W, half_b=half_b, delta=delta, k=k))


def footing3d(n: int = 96, size: float = 12.0, empty_layers: int = 2, half_b: float = 1.0,
              delta: float = 5e-3, nsteps: int = 20, dt: float = 0.1, k: float = 1e-12,
              tau_kind: int = TAU_WHITE) -> Workload:
    """Quarter-model of a rough rigid square footing (quarter 1 m x 1 m) on a cube of side
    ``size``; trilinear original MPM, quasi-static.  Same footing, drainage and support
    readings as ``footing2d`` with z vertical."""
    h = size / n
    grid = Grid(3, (n, n, n + empty_layers), h, (0.0, 0.0, 0.0))
    mat = Material(model=NEO_HOOKEAN, k=k)
    opt = Options(shape=LINEAR, dynamic=0, tau_kind=tau_kind)
    parts = fill_particles(grid, (0, 0, 0), (n, n, n), mat.rho0)
    H = n * h
    X = grid.node_coords()
    t = _tol(grid)

    def bc(step: int):
        b = empty_bc(grid)
        box_supports(grid, b, (size, size))
        zf = H - (step - 1) * delta
        foot = (X[:, 0] <= half_b + t) & (X[:, 1] <= half_b + t) & (X[:, 2] >= zf - t)
        b["u_fixed"][foot, :] = 1
        b["u_inc"][foot, 2] = -delta
        drained = (X[:, 2] >= H - t) & ~((X[:, 0] <= half_b + t) & (X[:, 1] <= half_b + t))
        b["p_fixed"][drained] = 1
        return b

    return Workload("footing3d", grid, mat, opt, parts, dt, nsteps, bc,
                    meta=dict(H=H, half_b=half_b, delta=delta, k=k))


def consolidation2d(n: int, k: float, width: float = 10.0, load: float = 10e3, nsteps: int = 20,
                    dt: float = 0.1) -> Workload:
    """Square n x n consolidation problem (serving stream): original MPM, rollers on the sides,
    fixed base, uniform top load w on the drained top."""
    h = width / n
    grid = Grid(2, (n, n), h, (0.0, 0.0, 0.0))
    mat = Material(model=NEO_HOOKEAN, k=k)
    opt = Options(shape=LINEAR, dynamic=0, tau_kind=TAU_WHITE)
    parts = fill_particles(grid, (0, 0), (n, n), mat.rho0)
    H = W = n * h

    def bc(step: int):
        b = empty_bc(grid)
        box_supports(grid, b, (W,))
        X = grid.node_coords()
        top = np.abs(X[:, 1] - H) <= _tol(grid)
        b["p_fixed"][top] = 1
        for ix in range(n + 1):
            w = h if 0 < ix < n else 0.5 * h
            b["f_ext"][grid.node_index(ix, n), 1] = -load * w
        return b

    return Workload("consolidation2d", grid, mat, opt, parts, dt, nsteps, bc,
                    meta=dict(H=H, W=W, load=load, k=k))


def self_weight(h: float = 0.125, ppa: int = 5, width: float = 2.0, height: float = 2.0, K: float = 15e3,
                nu: float = 0.3, k: float = 1e-14, phi0: float = 0.5, rho_s: float = 2600.0,
                rho_f: float = 1000.0, mu_f: float = 1e-3, dt0: float = 0.1, growth: float = 1.2,
                nsteps: int = 100, shape: int = GIMP, tau_kind: int = TAU_WHITE,
                right_drained: bool = True) -> Workload:
    """Consolidation under self weight (the paper's third example): the right half of a 4 m wide,
    2 m tall soft deposit, Hencky skeleton with bulk modulus K = 15 kPa, nu = 0.3, Kozeny-Carman
    permeability from k0 = 1e-14 m^2 and phi0 = 0.5, gravity applied at t = 0, quasi-static,
    dt = 0.1 s growing by 1.2 per step.  Readings: the left edge is the symmetry plane (roller,
    impermeable), the bottom is fixed and impermeable, the right edge is a drained roller
    (laterally confined deposit) and the top is a drained free surface, so that the zero pressure
    follows the settling surface (Options.drained_surface).  With gravity in the Darcy law a
    drained right edge is a seepage face (p = 0 at every depth); right_drained=False makes it
    impermeable, so that the column drains through its top to a hydrostatic end state.  h = 0.125 m with 5 x 5 points per cell
    (6,400 points) or h = 0.0625 m with 4 x 4 (16,384 points) as in the paper.
    Step n lasts dt0 growth^(n-1) (meta['dt_of'])."""
    nx, ny = int(round(width / h)), int(round(height / h))
    # two empty rows above the material: the drained surface is where active nodes meet inactive ones
    grid = Grid(2, (nx, ny + 2), h, (0.0, 0.0, 0.0))
    E = 3.0 * K * (1.0 - 2.0 * nu)
    mat = Material(model=HENCKY, E=E, nu=nu, k=k, mu_f=mu_f, rho_s=rho_s, rho_f=rho_f, phi0=phi0,
                   g=(0.0, -9.81, 0.0), kozeny_carman=True)
    opt = Options(shape=shape, dynamic=0, tau_kind=tau_kind, drained_surface=1)
    parts = fill_particles(grid, (0, 0), (nx, ny), mat.rho0, ppa=ppa)
    X = grid.node_coords()
    t = _tol(grid)

    def bc(step: int):
        b = empty_bc(grid)
        box_supports(grid, b, (width,))
        if right_drained:
            b["p_fixed"][X[:, 0] >= width - t] = 1
        return b

    def dt_of(step: int) -> float:
        return dt0 * growth ** (step - 1)

    return Workload("self_weight", grid, mat, opt, parts, dt0, nsteps, bc,
                    meta=dict(H=height, W=width, K=K, dt_of=dt_of, k=k))


def harmonic_footing(h: float = 0.25, ppa: int = 2, width: float = 10.0, depth: float = 10.0,
                     half_b: float = 1.0, empty_rows: int = 4, dt: float = 1e-3, nsteps: int = 400,
                     w0: float = 3e6, omega: float = 100.0, shape: int = GIMP, tau_kind: int = TAU_WHITE,
                     consistent_mass: int = 1) -> Workload:
    """Strip footing under harmonic loading (the paper's second example): right half of a 20 m
    wide, 10 m deep saturated ground, 40 x 40 cells of 0.25 m with 2 x 2 points per cell and 4
    empty rows (160 cells) above, Hencky skeleton with lambda = 8.4 MPa and G = 5.6 MPa,
    k = 1e-14 m^2, mu_f = 1e-3 Pa s, rho_s = 2.5 t/m^3, rho_f = 1 t/m^3, porosity 0.33, Kelvin
    damping alpha_vis = 0.04 s, Newmark with the paper's beta = 0.3025, gamma = 0.6, consistent
    mass mapping, dt = 1e-3 s for 400 steps.  The footing (half-width 1 m) pushes with
    w = w0 (1 - cos(omega t)), w0 = 3 MPa, omega = 100 rad/s, as a traction on the top faces of
    the points under it (point_force, outward normal +y, at the end of each step).
    Readings: the footing is impermeable and the rest of the top is drained (p = 0 on the grid
    nodes at and above the initial ground level beyond the footing, so that the drained
    boundary holds where the ground heaves); the base is fixed, the lateral faces are rollers,
    and both are impermeable.  meta['probes']: the points A, B, C (elevations 9.4375, 4.9375,
    0.0625 m on the symmetry line)."""
    nx, ny = int(round(width / h)), int(round(depth / h))
    grid = Grid(2, (nx, ny + empty_rows), h, (0.0, 0.0, 0.0))
    lam, G = 8.4e6, 5.6e6
    E = G * (3 * lam + 2 * G) / (lam + G)
    nu = lam / (2 * (lam + G))
    mat = Material(model=HENCKY, E=E, nu=nu, k=1e-14, mu_f=1e-3, rho_s=2500.0, rho_f=1000.0, phi0=0.33,
                   g=(0.0, 0.0, 0.0), alpha_vis=0.04)
    opt = Options(shape=shape, dynamic=1, beta=0.3025, gamma=0.6, tau_kind=tau_kind,
                  consistent_mass=consistent_mass, schur=1)
    parts = fill_particles(grid, (0, 0), (nx, ny), mat.rho0, ppa=ppa)
    X = grid.node_coords()
    t = _tol(grid)
    x = parts.x
    top = x[:, 1] > depth - h / ppa
    loaded = top & (x[:, 0] < half_b)
    seg = 2.0 * parts.lp[:, 0]                   # each loaded point's share of the footing width
    normal = np.zeros_like(x)
    normal[loaded, 1] = 1.0

    def load(step: int) -> float:
        return w0 * (1.0 - np.cos(omega * step * dt))

    def bc(step: int):
        b = empty_bc(grid)
        box_supports(grid, b, (width,))
        b["p_fixed"][(X[:, 1] >= depth - t) & (X[:, 0] > half_b + t)] = 1
        f = np.zeros_like(x)
        f[loaded, 1] = -load(step) * seg[loaded]
        b["point_force"] = f
        b["point_normal"] = normal
        return b

    probes = {name: int(np.argmin(np.hypot(x[:, 0] - h / (2 * ppa), x[:, 1] - y)))
              for name, y in (("A", 9.4375), ("B", 4.9375), ("C", 0.0625))}
    return Workload("harmonic_footing", grid, mat, opt, parts, dt, nsteps, bc,
                    meta=dict(load=load, probes=probes, loaded=np.flatnonzero(loaded), half_b=half_b))


def two_body_impact(h: float = 0.01, ppa: int = 4, radius: float = 0.2, v0: float = 0.1,
                    dt: float = 1e-3, nsteps: int = 3000, ghost: int = 2, n_drained: int = 18,
                    shape: int = GIMP, tau_kind: int = TAU_WHITE, centre: float = 0.2) -> Workload:
    """Impact of two poroelastic bodies (the paper's fourth example): discs of radius 0.2 m centred
    at (0.2, 0.2) and (0.8, 0.8) m in a 1 m square, moving towards each other at (0.1, 0.1) and
    (-0.1, -0.1) m/s, h = 0.01 m with 4 x 4 points per cell (the points at sub-cell centres inside
    a disc: 20,108 per body), ghost cells around the square, E = 1 kPa, nu = 0.3, Hencky,
    Kozeny-Carman permeability from k0 = 1e-14 m^2 and phi0 = 0.5, mu_f = 1e-3 Pa s,
    rho_s = rho_f = 1 t/m^3, no gravity, no damping, GIMP with tau_W, Newmark with the paper's
    beta = 0.3025, gamma = 0.6, dt = 1 ms.  Contact is the method's own: the bodies share the
    grid's single velocity field (no-slip), they touch at t ~ 1.6 s.  No grid boundary
    conditions; in each body the n_drained points nearest its top point hold zero pore pressure
    (point_p_fixed: the grid nodes those points reach hold p = 0).  `centre` moves the discs'
    centres to (c, c) and (1 - c, 1 - c) (shorter runs to contact for tests)."""
    n = int(round(1.0 / h))
    grid = Grid(2, (n + 2 * ghost, n + 2 * ghost), h, (-ghost * h, -ghost * h, 0.0))
    mat = Material(model=HENCKY, E=1000.0, nu=0.3, k=1e-14, mu_f=1e-3, rho_s=1000.0, rho_f=1000.0, phi0=0.5,
                   g=(0.0, 0.0, 0.0), kozeny_carman=True)
    # the bodies fly free before they meet, so the mass residual starts at ~0 and the default
    # absolute floor of a unit-rate nodal flux times 1e-12 would ask an iterative solve for 1e-16
    # of the momentum residual; 1e-6 of it is the floor here
    # where the bodies touch, point domains graze nodes with ~1e-7 of the largest nodal mass; their
    # displacement is then nearly undetermined (condition ~1e9) and their activation switches
    # from iteration to iteration, so nodes below 1e-5 of the largest mass are left out (1e-6
    # suffices on the coarse grid; the paper's grid needs 1e-5 through the whole compression).
    # The Schur block stays fixed-stress: the diagonal-inverse form divides by the displacement
    # blocks of the lightest nodes that remain at the contact, and Newton stopped converging there
    opt = Options(shape=shape, dynamic=1, beta=0.3025, gamma=0.6, tau_kind=tau_kind,
                  newton_atol_p=1e-6 * h * h / dt, negligible_mass=1e-5)
    box = fill_particles(grid, (ghost, ghost), (n + ghost, n + ghost), mat.rho0, ppa=ppa)
    centres = ((centre, centre), (1.0 - centre, 1.0 - centre))
    vels = ((v0, v0), (-v0, -v0))
    keep, vel, drained = [], [], []
    for (cx, cy), v in zip(centres, vels):
        inside = np.flatnonzero((box.x[:, 0] - cx) ** 2 + (box.x[:, 1] - cy) ** 2 <= radius ** 2)
        top = np.argsort(np.hypot(box.x[inside, 0] - cx, box.x[inside, 1] - (cy + radius)), kind="stable")
        drained.append(len(np.concatenate(keep)) + top[:n_drained] if keep else top[:n_drained])
        keep.append(inside)
        vel.append(np.tile(np.asarray(v, float), (inside.size, 1)))
    idx = np.concatenate(keep)
    parts = Particles(x=np.ascontiguousarray(box.x[idx]), vol=box.vol[idx].copy(), mass=box.mass[idx].copy(),
                      lp=np.ascontiguousarray(box.lp[idx]), v0=np.ascontiguousarray(np.concatenate(vel)))
    pfix = np.zeros(idx.size, np.uint8)
    pfix[np.concatenate(drained)] = 1

    def bc(step: int):
        b = empty_bc(grid)
        b["point_p_fixed"] = pfix
        b["point_p_val"] = np.zeros(idx.size)
        return b

    return Workload("two_body_impact", grid, mat, opt, parts, dt, nsteps, bc,
                    meta=dict(bodies=[k.size for k in keep], drained=np.flatnonzero(pfix), contact_time=1.59))


def jittered_box(nx: int = 8, ny: int = 8, h: float = 0.25, seed: int = 0, shape: int = LINEAR,
                 dynamic: int = 0, model: int = NEO_HOOKEAN, k: float = 1e-12,
                 jitter: float = 0.6, empty: int = 1) -> Workload:
    """Small test problem: a jittered particle block inside a grid with ``empty`` empty cells
    around it (so GIMP domains stay inside), rollers/base supports on the outer grid faces only
    where the material touches them (none here), and a downward edge load on the top nodes.
    Used for assembly and Jacobian checks on irregular particle layouts."""
    rng = np.random.default_rng(seed)
    grid = Grid(2, (nx + 2 * empty, ny + 2 * empty), h, (0.0, 0.0, 0.0))
    mat = Material(model=model, k=k)
    opt = Options(shape=shape, dynamic=dynamic)
    parts = fill_particles(grid, (empty, empty), (empty + nx, empty + ny), mat.rho0,
                           jitter=jitter, rng=rng)

    def bc(step: int):
        b = empty_bc(grid)
        X = grid.node_coords()
        t = _tol(grid)
        base = X[:, 1] <= empty * h + t
        b["u_fixed"][base, :] = 1
        top = np.abs(X[:, 1] - (empty + ny) * h) <= t
        b["p_fixed"][top] = 1
        b["f_ext"][top, 1] = -5e3 * h
        return b

    return Workload("jittered_box", grid, mat, opt, parts, 0.05, 3, bc, meta=dict(seed=seed))


# ----------------------------------------------------------------------------------------------
# the five benchmark configurations
# ----------------------------------------------------------------------------------------------

def config(idx: int, **kw) -> Workload:
    """Benchmark configuration by index (1-based, in the order they are listed for this
    repository's benchmark): 1 Terzaghi, 2 undrained dynamic GIMP footing, 3 large quasi-static
    GIMP footing, 4 3D footing.  The serving stream (5) is ``serving_trace``."""
    if idx == 1:
        return terzaghi(**kw)
    if idx == 2:
        args = dict(nx=64, ny=64, width=10.0, empty_rows=4, half_b=1.0, delta=5e-3, nsteps=100,
                    dt=1e-3, k=1e-16, dynamic=1, shape=GIMP, beta=0.25, gamma=0.5,
                    name="footing2d_undrained")
        args.update(kw)
        w = footing2d(**args)
        # undrained and inertia-dominated: the diagonal-inverse Schur block (the fixed-stress
        # diagonal leaves BiCGStab at 130-170 iterations per Newton iteration and stalls in FP32)
        w.options.schur = 1
        return w
    if idx == 3:
        args = dict(nx=512, ny=256, width=32.0, empty_rows=16, half_b=1.0, delta=5e-3,
                    nsteps=200, dt=0.1, dynamic=0, shape=GIMP, seed=0, k_range=(-14.0, -10.0),
                    name="footing2d_large")
        args.update(kw)
        return footing2d(**args)
    if idx == 4:
        return footing3d(**kw)
    raise ValueError(f"unknown configuration {idx}")


@dataclass
class Request:
    rid: int
    arrival: float
    kind: str          # "consolidation" or "footing"
    n: int
    k: float
    nsteps: int

    def workload(self) -> Workload:
        if self.kind == "consolidation":
            return consolidation2d(self.n, self.k, nsteps=self.nsteps)
        rows = max(2, int(np.ceil(0.05 * self.n)))
        return footing2d(nx=self.n, ny=self.n, width=10.0, empty_rows=rows, half_b=1.25,
                         delta=5e-3, nsteps=self.nsteps, dt=0.1, k=self.k, dynamic=0,
                         shape=GIMP, name="footing2d_serve")


def serving_trace(nreq: int = 256, rate: float = 20.0, n_range=(16, 256),
                  k_range=(1e-16, 1e-10), steps_range=(20, 50), seed: int = 0) -> List[Request]:
    """Poisson arrival stream of independent 2D problems: exponential inter-arrival gaps of
    mean 1/rate, grid n = round(exp(U(ln n_lo, ln n_hi))), k = exp(U(ln k_lo, ln k_hi)),
    steps ~ U{lo..hi}, kind 50/50 consolidation / footing."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(nreq):
        t += rng.exponential(1.0 / rate)
        n = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        k = float(np.exp(rng.uniform(np.log(k_range[0]), np.log(k_range[1]))))
        ns = int(rng.integers(steps_range[0], steps_range[1] + 1))
        kind = "consolidation" if rng.random() < 0.5 else "footing"
        out.append(Request(i, t, kind, n, k, ns))
    return out
