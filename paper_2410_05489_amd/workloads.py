"""Seeded synthetic workloads shaped like the paper's test problems.

Problem descriptions only: grids, parameters and exact cell averages of the
initial data.  Nothing here computes any part of the ASE-DF method; both the
CPU oracle and the GPU library consume what these generators return.

Arrays use the state layout U[v, J, I] (v = conserved variable, J = row with
ghosts, I = column with ghosts), float64, C-contiguous, with the row stride
``grid.ld`` equal to the padded row length.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

BC_PERIODIC = 0
BC_TRANSMISSIVE = 1
BC_INFLOW_SLOT = 2
BC_REFLECTIVE = 3   # slip wall: mirrored cells, normal momentum reversed
BC_WALL_INFLOW = 4  # y-lo: inflow state below wall_x0, slip wall beyond
BC_MOVING_SHOCK = 5 # y-hi: inflow state behind the moving shock, outer state ahead
BC_NOSLIP = 6       # no-slip adiabatic wall: mirrored cells, whole momentum reversed

# Interface states the DF strengths come from: the previous stage's
# Gauss-point states (lagged) or the current stage's cell averages.
DF_LAGGED = 0
DF_FIRST_ORDER = 1


@dataclasses.dataclass
class Grid:
    dim: int
    nx: int
    ny: int
    ng: int
    dx: float
    dy: float
    bc: Tuple[int, int, int, int] = (BC_TRANSMISSIVE,) * 4
    y0: float = 0.0
    inflow: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    slot_lo: float = 0.0
    slot_hi: float = 0.0
    ld: int = 0
    x0: float = 0.0
    wall_x0: float = 0.0
    shock_x0: float = 0.0
    shock_speed: float = 0.0
    outer: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)

    def __post_init__(self):
        if self.ld == 0:
            self.ld = self.nx + 2 * self.ng
        if self.dim == 1:
            self.ny = 1

    @property
    def nvar(self) -> int:
        return 3 if self.dim == 1 else 4

    @property
    def NX(self) -> int:
        return self.nx + 2 * self.ng

    @property
    def NY(self) -> int:
        return 1 if self.dim == 1 else self.ny + 2 * self.ng

    def shape(self) -> Tuple[int, int, int]:
        return (self.nvar, self.NY, self.ld)

    def interior(self, a: np.ndarray) -> np.ndarray:
        """View of the interior cells of a state-layout array."""
        g = self.ng
        if self.dim == 1:
            return a[..., 0:1, g:g + self.nx]
        return a[..., g:g + self.ny, g:g + self.nx]

    def ncells(self) -> int:
        return self.nx * (1 if self.dim == 1 else self.ny)


@dataclasses.dataclass
class Params:
    order: int
    gamma: float = 1.4
    cfl: float = 0.5
    sigma_thres: float = 2.0
    eps: float = 1e-6
    d_hi: float = 0.85
    d_lo: float = 0.85
    dt_cap: float = 0.0
    positivity_fallback: int = 0
    df_source: int = 1          # DF_FIRST_ORDER (the reading adopted) or DF_LAGGED
    fail_nonphysical: int = 0   # ase_step / ase_step_gks report a non-physical final state


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    params: Params
    U: np.ndarray
    nsteps: int
    t_end: float = 0.0


def ghosts_for(order: int) -> int:
    return (order + 1) // 2 if order > 1 else 1


def conservative(rho, u, v, p, gamma, dim):
    """Conservative state (rho, rho u, [rho v], E) of primitive data."""
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, u, v, p)))
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    if dim == 1:
        return np.stack([rho, rho * u, E])
    return np.stack([rho, rho * u, rho * v, E])


def empty_state(grid: Grid) -> np.ndarray:
    return np.zeros(grid.shape(), dtype=np.float64)


def empty_sigma(grid: Grid) -> np.ndarray:
    return np.zeros((grid.NY, grid.ld), dtype=np.float64)


def _fill_interior(grid: Grid, U: np.ndarray, W: np.ndarray) -> None:
    grid.interior(U)[...] = W.reshape(grid.interior(U).shape)


# --------------------------------------------------------------------------
# 1D problems
# --------------------------------------------------------------------------

def riemann_1d(n: int, left, right, order: int, x_split: float = 0.5, gamma: float = 1.4,
               cfl: float = 0.5, name: str = "riemann1d", nsteps: int = 0, t_end: float = 0.0,
               xlo: float = 0.0, xhi: float = 1.0) -> Workload:
    """Two-state Riemann data (rho, u, p) on [xlo, xhi]; exact averages."""
    dx = (xhi - xlo) / n
    g = Grid(dim=1, nx=n, ny=1, ng=ghosts_for(order), dx=dx, dy=dx, bc=(BC_TRANSMISSIVE,) * 4)
    xl = xlo + np.arange(n) * dx
    xr = xl + dx
    frac_left = np.clip((x_split - xl) / dx, 0.0, 1.0)
    WL = conservative(left[0], left[1], 0.0, left[2], gamma, 1)
    WR = conservative(right[0], right[1], 0.0, right[2], gamma, 1)
    W = frac_left[None, :] * WL[:, None] + (1.0 - frac_left[None, :]) * WR[:, None]
    U = empty_state(g)
    _fill_interior(g, U, W)
    return Workload(name, g, Params(order=order, gamma=gamma, cfl=cfl), U, nsteps, t_end)


def sod(n: int = 200, order: int = 5) -> Workload:
    """Sod shock tube: (1,0,1) | (0.125,0,0.1) at x=0.5, gamma 1.4, t=0.2."""
    return riemann_1d(n, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), order, 0.5, 1.4, 0.5, "sod", 100000, 0.2)


def blast_wave(n: int = 400, order: int = 9, t_end: float = 0.038) -> Workload:
    """Woodward-Colella blast wave on [0,1]: (1,0,1000) | (1,0,0.01) | (1,0,100)
    split at 0.1 and 0.9, reflective walls at both ends, gamma 1.4, CFL 0.5
    (exact cell averages)."""
    dx = 1.0 / n
    g = Grid(dim=1, nx=n, ny=1, ng=ghosts_for(order), dx=dx, dy=dx, bc=(BC_REFLECTIVE,) * 4)
    xl = np.arange(n) * dx
    xr = xl + dx
    fl = np.clip((0.1 - xl) / dx, 0.0, 1.0)             # fraction left of 0.1
    fr = np.clip((xr - 0.9) / dx, 0.0, 1.0)             # fraction right of 0.9
    fm = 1.0 - fl - fr
    gamma = 1.4
    E = (fl * 1000.0 + fm * 0.01 + fr * 100.0) / (gamma - 1.0)
    W = np.stack([np.ones(n), np.zeros(n), E])
    U = empty_state(g)
    _fill_interior(g, U, W)
    return Workload("blast_wave", g, Params(order=order, gamma=gamma, cfl=0.5), U, 100000, t_end)


def shu_osher(n: int = 200, order: int = 9, t_end: float = 1.8) -> Workload:
    """Shu-Osher shock / entropy-wave interaction on [0,10]: (3.857134,
    2.629369, 10.33333) for x < 1, (1 + 0.2 sin 5x, 0, 1) beyond, transmissive,
    gamma 1.4, CFL 0.5 (exact cell averages of the density)."""
    L = 10.0
    dx = L / n
    g = Grid(dim=1, nx=n, ny=1, ng=ghosts_for(order), dx=dx, dy=dx, bc=(BC_TRANSMISSIVE,) * 4)
    xl = np.arange(n) * dx
    xr = xl + dx
    fl = np.clip((1.0 - xl) / dx, 0.0, 1.0)
    # average of 1 + 0.2 sin(5x) over the part of the cell right of x = 1
    a = np.maximum(xl, 1.0)
    avg_r = np.where(xr > a, (xr - a) + 0.2 * (np.cos(5 * a) - np.cos(5 * xr)) / 5.0, 0.0) / dx
    gamma = 1.4
    WL_ = conservative(3.857134, 2.629369, 0.0, 10.33333, gamma, 1)
    # right state: u = 0, p = 1 -> momentum 0, energy p/(gamma-1) independent of rho
    rho = fl * WL_[0] + avg_r
    mom = fl * WL_[1]
    E = fl * WL_[2] + (1.0 - fl) * (1.0 / (gamma - 1.0))
    U = empty_state(g)
    _fill_interior(g, U, np.stack([rho, mom, E]))
    return Workload("shu_osher", g, Params(order=order, gamma=gamma, cfl=0.5), U, 100000, t_end)


def density_wave_1d(n: int, order: int, seed: int = -1, amp: float = 1e-3, cfl: float = 0.5,
                    t_end: float = 2.0) -> Workload:
    """rho = 1 + 0.2 sin(pi x), u = 1, p = 1, periodic on [0,2] (exact averages).

    seed >= 0 adds a seeded uniform perturbation of the density averages.
    """
    L = 2.0
    dx = L / n
    g = Grid(dim=1, nx=n, ny=1, ng=ghosts_for(order), dx=dx, dy=dx, bc=(BC_PERIODIC,) * 4)
    xl = np.arange(n) * dx
    xr = xl + dx
    rho = 1.0 + 0.2 * (np.cos(math.pi * xl) - np.cos(math.pi * xr)) / (math.pi * dx)
    if seed >= 0:
        rng = np.random.default_rng(seed)
        rho = rho + rng.uniform(-amp, amp, size=n)
    gamma = 1.4
    # u = 1 and p = 1 are constant, so rho u = rho and E = p/(gamma-1) + rho/2.
    W = np.stack([rho, rho * 1.0, 1.0 / (gamma - 1.0) + 0.5 * rho])
    U = empty_state(g)
    _fill_interior(g, U, W)
    return Workload("density_wave_1d", g, Params(order=order, gamma=gamma, cfl=cfl), U, 10 ** 9, t_end)


def density_wave_exact_1d(n: int, t: float) -> np.ndarray:
    """Exact cell averages of rho at time t for the 1D density wave."""
    dx = 2.0 / n
    xl = np.arange(n) * dx
    xr = xl + dx
    return 1.0 + 0.2 * (np.cos(math.pi * (xl - t)) - np.cos(math.pi * (xr - t))) / (math.pi * dx)


# --------------------------------------------------------------------------
# 2D problems
# --------------------------------------------------------------------------

def _avg_sin(lo, hi):
    return (np.cos(math.pi * lo) - np.cos(math.pi * hi)) / (math.pi * (hi - lo))


def density_wave_2d(n: int, order: int, seed: int = -1, amp: float = 1e-3, cfl: float = 0.5) -> Workload:
    """rho = 1 + 0.2 sin(pi x) sin(pi y), u = v = 1, p = 1 on [0,2]^2, periodic."""
    L = 2.0
    dx = L / n
    g = Grid(dim=2, nx=n, ny=n, ng=ghosts_for(order), dx=dx, dy=dx, bc=(BC_PERIODIC,) * 4)
    e = np.arange(n + 1) * dx
    sx = _avg_sin(e[:-1], e[1:])
    rho = 1.0 + 0.2 * np.outer(sx, sx)          # [j, i]
    if seed >= 0:
        rng = np.random.default_rng(seed)
        rho = rho + rng.uniform(-amp, amp, size=rho.shape)
    gamma = 1.4
    W = np.stack([rho, rho, rho, 1.0 / (gamma - 1.0) + rho])   # u = v = 1, p = 1
    U = empty_state(g)
    _fill_interior(g, U, W)
    return Workload("density_wave_2d", g, Params(order=order, gamma=gamma, cfl=cfl), U, 10 ** 9, 0.0)


def double_mach(nx: int = 960, ny: int = 240, order: int = 9, t_end: float = 0.2, cfl: float = 0.5,
                nsteps: int = 100000) -> Workload:
    """Double Mach reflection on [0,4] x [0,1]: a Mach 10 shock through
    (1/6, 0) at 60 degrees to the wall, post-shock (8, 7.145, -4.125,
    116.8333) above the line y = sqrt(3)(x - 1/6), (1.4, 0, 0, 1) below;
    gamma 1.4.  Left side inflow of the post-shock state, right side
    transmissive, bottom post-shock below x = 1/6 and slip wall beyond, top
    post-shock behind the shock's exact position 1/6 + (1 + 20 t)/sqrt(3).
    Cell averages from the exact post-shock area of each cell (x integral
    of the clipped line, 64 midpoints per cell).  First-order DF source and
    the positivity fallback, as for the other strong-shock problems."""
    gamma = 1.4
    post = (8.0, 7.145, -4.125, 116.8333)
    pre = (1.4, 0.0, 0.0, 1.0)
    s3 = math.sqrt(3.0)
    xw = 1.0 / 6.0
    dx, dy = 4.0 / nx, 1.0 / ny

    def cons(q):
        r, u, v, p = q
        return (r, r * u, r * v, p / (gamma - 1.0) + 0.5 * r * (u * u + v * v))
    g = Grid(dim=2, nx=nx, ny=ny, ng=ghosts_for(order), dx=dx, dy=dy,
             bc=(BC_INFLOW_SLOT, BC_TRANSMISSIVE, BC_WALL_INFLOW, BC_MOVING_SHOCK), y0=0.0, inflow=cons(post),
             slot_lo=-1e300, slot_hi=1e300, x0=0.0, wall_x0=xw, shock_x0=xw + 1.0 / s3, shock_speed=20.0 / s3,
             outer=cons(pre))
    m = 64
    xs = (np.arange(nx)[:, None] + (np.arange(m)[None, :] + 0.5) / m) * dx   # [i, sample]
    line = s3 * (xs - xw)
    ya = (np.arange(ny) * dy)[:, None, None]
    # post-shock height of each sub-column inside the cell, as a fraction of dy
    h = np.clip((ya + dy - np.maximum(ya, line[None, :, :])) / dy, 0.0, 1.0)
    frac = h.mean(axis=2)                      # [j, i]
    Wpost, Wpre = np.array(cons(post)), np.array(cons(pre))
    W = Wpre[:, None, None] + (Wpost - Wpre)[:, None, None] * frac[None]
    U = empty_state(g)
    _fill_interior(g, U, W)
    return Workload("double_mach", g, Params(order=order, gamma=gamma, cfl=cfl), U, nsteps, t_end)


def viscous_shock_tube(nx: int = 500, ny: int = 250, order: int = 5, re: float = 200.0, t_end: float = 1.0,
                       cfl: float = 0.5, nsteps: int = 100000) -> Workload:
    """Viscous shock tube on [0,1] x [0,0.5]: (120, 0, 0, 120/gamma) for
    x < 0.5, (1.2, 0, 0, 1.2/gamma) beyond, gamma 1.4, Pr = 1 (the BGK
    model's), mu = 1/Re; no-slip adiabatic walls left, right and below, a
    symmetry plane on top.  First-order DF source, positivity fallback.
    The workload carries mu (`w.mu`) for the gas-kinetic solver."""
    gamma = 1.4
    dx, dy = 1.0 / nx, 0.5 / ny
    g = Grid(dim=2, nx=nx, ny=ny, ng=ghosts_for(order), dx=dx, dy=dy,
             bc=(BC_NOSLIP, BC_NOSLIP, BC_NOSLIP, BC_REFLECTIVE))
    # the split x = 0.5 falls on a face for even nx; otherwise area fractions
    xl = np.arange(nx) * dx
    frac = np.clip((0.5 - xl) / dx, 0.0, 1.0)
    rho = 1.2 + (120.0 - 1.2) * frac
    p = rho / gamma
    W = np.stack([rho, 0 * rho, 0 * rho, p / (gamma - 1.0)])[:, None, :].repeat(ny, axis=1)
    U = empty_state(g)
    _fill_interior(g, U, W)
    w = Workload("viscous_shock_tube", g, Params(order=order, gamma=gamma, cfl=cfl, positivity_fallback=1,
                                                 df_source=DF_FIRST_ORDER), U, nsteps, t_end)
    w.mu = 1.0 / re
    return w


# Configuration 3 of the paper's 2D Riemann tests, quadrant order NE, NW, SW, SE.
CONFIG3_STATES = (
    (1.5, 0.0, 0.0, 1.5),          # NE: x >= 0.7, y >= 0.7
    (0.5323, 1.206, 0.0, 0.3),     # NW: x <  0.7, y >= 0.7
    (0.138, 1.206, 1.206, 0.129),  # SW: x <  0.7, y <  0.7
    (0.5323, 0.0, 1.206, 0.3),     # SE: x >= 0.7, y <  0.7
)


def quadrant_states(seed: int) -> Tuple[Tuple[float, float, float, float], ...]:
    """Per-seed quadrant states (NE, NW, SW, SE): rho in [0.1,1.5], |u|,|v| <= 1.2,
    p in [0.03,1.5]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        u = rng.uniform(-1.2, 1.2)
        v = rng.uniform(-1.2, 1.2)
        p = rng.uniform(0.03, 1.5)
        out.append((rho, u, v, p))
    return tuple(out)


def four_quadrant(n: int = 1024, order: int = 9, seed: int = 0, nsteps: int = 200, cfl: float = 0.4,
                  states=None, split=(0.7, 0.7), ny: int = 0) -> Workload:
    """2D four-quadrant Riemann problem on [0,1]^2 with area-fraction cut cells."""
    nyy = ny if ny else n
    dx = 1.0 / n
    dy = 1.0 / nyy
    gamma = 1.4
    g = Grid(dim=2, nx=n, ny=nyy, ng=ghosts_for(order), dx=dx, dy=dy, bc=(BC_TRANSMISSIVE,) * 4)
    if states is None:
        states = quadrant_states(seed)
    ex = np.arange(n) * dx
    ey = np.arange(nyy) * dy
    fx = np.clip((split[0] - ex) / dx, 0.0, 1.0)     # fraction left of the split
    fy = np.clip((split[1] - ey) / dy, 0.0, 1.0)     # fraction below the split
    Q = [conservative(s[0], s[1], s[2], s[3], gamma, 2) for s in states]
    NE, NW, SW, SE = Q
    FX = fx[None, None, :]
    FY = fy[None, :, None]
    W = (FX * FY * SW[:, None, None] + (1 - FX) * FY * SE[:, None, None]
         + FX * (1 - FY) * NW[:, None, None] + (1 - FX) * (1 - FY) * NE[:, None, None])
    U = empty_state(g)
    _fill_interior(g, U, W)
    return Workload(f"four_quadrant_{n}x{nyy}_r{order}_seed{seed}", g,
                    Params(order=order, gamma=gamma, cfl=cfl), U, nsteps, 0.0)


def jet(nx: int = 1600, ny: int = 800, order: int = 7, u_jet: float = 7400.0, nsteps: int = 500,
        cfl: float = 0.25, positivity_fallback: int = 1, df_source: int = DF_FIRST_ORDER) -> Workload:
    """High-Mach jet on [0,1] x [-0.25,0.25], gamma 5/3: ambient (0.5,0,0,0.4127),
    inflow (5, u_jet, 0, 0.4127) through |y| < 0.05 at x = 0, outflow elsewhere."""
    gamma = 5.0 / 3.0
    dx = 1.0 / nx
    dy = 0.5 / ny
    inflow = conservative(5.0, u_jet, 0.0, 0.4127, gamma, 2)
    g = Grid(dim=2, nx=nx, ny=ny, ng=ghosts_for(order), dx=dx, dy=dy,
             bc=(BC_INFLOW_SLOT, BC_TRANSMISSIVE, BC_TRANSMISSIVE, BC_TRANSMISSIVE), y0=-0.25,
             inflow=tuple(float(x) for x in inflow), slot_lo=-0.05, slot_hi=0.05)
    amb = conservative(0.5, 0.0, 0.0, 0.4127, gamma, 2)
    W = np.broadcast_to(amb[:, None, None], (4, ny, nx)).copy()
    U = empty_state(g)
    _fill_interior(g, U, W)
    return Workload(f"jet_{nx}x{ny}_r{order}", g,
                    Params(order=order, gamma=gamma, cfl=cfl, positivity_fallback=positivity_fallback,
                           df_source=df_source), U, nsteps, 0.0)


# --------------------------------------------------------------------------
# Batched 1D instances
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Batch:
    ncells: np.ndarray        # int32 [ninst]
    offsets: np.ndarray       # int64 [ninst]: first stored cell (ghosts incl.)
    dx: np.ndarray            # float64 [ninst]
    ng: int
    U: np.ndarray             # float64 [3, total]
    params: Params
    bc: int
    nsteps: int
    bc_inst: Optional[np.ndarray] = None   # int32 [ninst]: per-instance boundary code (else `bc`)

    @property
    def ninst(self) -> int:
        return int(self.ncells.shape[0])

    @property
    def total(self) -> int:
        return int(self.U.shape[1])

    def instance(self, k: int) -> np.ndarray:
        o = int(self.offsets[k])
        return self.U[:, o:o + int(self.ncells[k]) + 2 * self.ng]


def _pack(ncells: Sequence[int], ng: int) -> Tuple[np.ndarray, np.ndarray, int]:
    ncells = np.asarray(ncells, dtype=np.int32)
    sizes = ncells.astype(np.int64) + 2 * ng
    offsets = np.zeros(len(ncells), dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)[:-1]
    return ncells, offsets, int(sizes.sum())


def batched_riemann(ninst: int = 256, nmin: int = 64, nmax: int = 4096, order: int = 9, seed: int = 0,
                    nsteps: int = 100, cfl: float = 0.5, sizes: Optional[Sequence[int]] = None) -> Batch:
    """Independent 1D Riemann problems on [0,1] split at 0.5, transmissive:
    rho in [0.1,2], |u| <= 2, p in [0.05,2] per side; N uniform in [nmin, nmax]
    (or the given sizes, one instance each)."""
    rng = np.random.default_rng(seed)
    n = rng.integers(nmin, nmax + 1, size=ninst)
    if sizes is not None:
        n = np.asarray(sizes, dtype=np.int64)
        ninst = len(n)
    ng = ghosts_for(order)
    ncells, offsets, total = _pack(n, ng)
    gamma = 1.4
    U = np.zeros((3, total), dtype=np.float64)
    dx = 1.0 / ncells.astype(np.float64)
    for k in range(ninst):
        rl, rr = rng.uniform(0.1, 2.0, size=2)
        ul, ur = rng.uniform(-2.0, 2.0, size=2)
        pl, pr = rng.uniform(0.05, 2.0, size=2)
        N = int(ncells[k])
        xl = np.arange(N) * dx[k]
        frac = np.clip((0.5 - xl) / dx[k], 0.0, 1.0)
        WL = conservative(rl, ul, 0.0, pl, gamma, 1)
        WR = conservative(rr, ur, 0.0, pr, gamma, 1)
        W = frac[None, :] * WL[:, None] + (1 - frac[None, :]) * WR[:, None]
        o = int(offsets[k])
        U[:, o + ng:o + ng + N] = W
    return Batch(ncells, offsets, dx, ng, U, Params(order=order, gamma=gamma, cfl=cfl), BC_TRANSMISSIVE, nsteps)


def batched_smooth(ninst: int = 16, nmin: int = 64, nmax: int = 512, order: int = 9, seed: int = 1,
                   nsteps: int = 20, cfl: float = 0.5, sizes: Optional[Sequence[int]] = None) -> Batch:
    """Smooth periodic 1D instances: rho = 1 + 0.2 sin(2 pi x + phi),
    u = 0.5 + 0.1 cos(2 pi x), p = 1 + 0.1 sin(2 pi x + psi) (point values at
    five Gauss-Legendre nodes per cell averaged, i.e. 9th-order cell averages)."""
    rng = np.random.default_rng(seed)
    n = rng.integers(nmin, nmax + 1, size=ninst)
    if sizes is not None:
        n = np.asarray(sizes, dtype=np.int64)
        ninst = len(n)
    ng = ghosts_for(order)
    ncells, offsets, total = _pack(n, ng)
    gamma = 1.4
    U = np.zeros((3, total), dtype=np.float64)
    dx = 1.0 / ncells.astype(np.float64)
    xg, wg = np.polynomial.legendre.leggauss(5)
    for k in range(ninst):
        phi, psi = rng.uniform(0, 2 * math.pi, size=2)
        N = int(ncells[k])
        xc = (np.arange(N) + 0.5) * dx[k]
        acc = np.zeros((3, N))
        for xq, wq in zip(xg, wg):
            x = xc + 0.5 * dx[k] * xq
            rho = 1 + 0.2 * np.sin(2 * math.pi * x + phi)
            u = 0.5 + 0.1 * np.cos(2 * math.pi * x)
            p = 1 + 0.1 * np.sin(2 * math.pi * x + psi)
            acc += 0.5 * wq * conservative(rho, u, 0.0, p, gamma, 1)
        o = int(offsets[k])
        U[:, o + ng:o + ng + N] = acc
    return Batch(ncells, offsets, dx, ng, U, Params(order=order, gamma=gamma, cfl=cfl), BC_PERIODIC, nsteps)


def batch_subset(batch: Batch, keep) -> Batch:
    """The instances `keep` (indices, in order) of a batch, packed anew."""
    keep = [int(k) for k in keep]
    ncells, offsets, total = _pack([int(batch.ncells[k]) for k in keep], batch.ng)
    U = np.zeros((3, total), dtype=np.float64)
    for j, k in enumerate(keep):
        o = int(offsets[j])
        U[:, o:o + int(ncells[j]) + 2 * batch.ng] = batch.instance(k)
    bci = None if batch.bc_inst is None else np.asarray(batch.bc_inst)[keep].astype(np.int32)
    return Batch(ncells, offsets, np.asarray(batch.dx)[keep].copy(), batch.ng, U, dataclasses.replace(batch.params),
                 batch.bc, batch.nsteps, bci)


def instance_grid(batch: Batch, k: int) -> Grid:
    """The single-instance 1D grid of instance k of a batch."""
    N = int(batch.ncells[k])
    bc = int(batch.bc_inst[k]) if batch.bc_inst is not None else batch.bc
    return Grid(dim=1, nx=N, ny=1, ng=batch.ng, dx=float(batch.dx[k]), dy=float(batch.dx[k]), bc=(bc,) * 4)


def batched_mixed(ninst: int = 12, nmin: int = 16, nmax: int = 400, order: int = 9, seed: int = 5,
                  nsteps: int = 20, sizes: Optional[Sequence[int]] = None) -> Batch:
    """Instances with their own boundary conditions: instance k carries the
    smooth periodic data of batched_smooth (k % 3 == 0), the transmissive
    Riemann data of batched_riemann (k % 3 == 1) or that Riemann data between
    two reflective walls (k % 3 == 2); sizes: the cell counts, one instance
    each (else drawn from [nmin, nmax])."""
    if sizes is not None:
        ninst = len(sizes)
    sm = batched_smooth(ninst=ninst, nmin=nmin, nmax=nmax, order=order, seed=seed, nsteps=nsteps, sizes=sizes)
    rm = batched_riemann(ninst=ninst, nmin=nmin, nmax=nmax, order=order, seed=seed + 1, nsteps=nsteps,
                         sizes=sizes)
    pick = [sm if k % 3 == 0 else rm for k in range(ninst)]
    ncells, offsets, total = _pack([int(b.ncells[k]) for k, b in enumerate(pick)], sm.ng)
    U = np.zeros((3, total), dtype=np.float64)
    for k, b in enumerate(pick):
        o = int(offsets[k])
        U[:, o:o + int(ncells[k]) + 2 * sm.ng] = b.instance(k)
    dx = np.array([float(b.dx[k]) for k, b in enumerate(pick)])
    bc_inst = np.array([(BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE)[k % 3] for k in range(ninst)], dtype=np.int32)
    return Batch(ncells, offsets, dx, sm.ng, U, Params(order=order, gamma=1.4, cfl=0.5), BC_TRANSMISSIVE, nsteps,
                 bc_inst)
