"""Pins of the oracle's full solver: design order, conservation, the Sod
tube against the exact Riemann solution, uniform-state preservation,
mirror/transpose symmetry, boundary fills.
"""
import math
import os

import numpy as np
import pytest

import exact_riemann as ER
from paper_2410_05489_amd import workloads as WL
from paper_2410_05489_amd.workloads import Grid, Params

HERE = os.path.dirname(os.path.abspath(__file__))


def _orders(errs, ns):
    return [math.log(errs[k] / errs[k + 1]) / math.log(ns[k + 1] / ns[k]) for k in range(len(errs) - 1)]


# ---------------------------------------------------------------------------
# design order (semi-discrete residual on exact averages of a smooth wave)
# ---------------------------------------------------------------------------

def _exact_dWdt_1d(n):
    """Cell average of dW/dt for rho = 1 + 0.2 sin(pi (x - t)), u = 1, p = 1 at t = 0."""
    dx = 2.0 / n
    xl = np.arange(n) * dx
    drho = -0.2 * (np.sin(math.pi * (xl + dx)) - np.sin(math.pi * xl)) / dx
    return np.stack([drho, drho, 0.5 * drho])


@pytest.mark.parametrize("r,ns,lo", [(5, (20, 40, 80), 4.7), (7, (20, 40, 80), 6.7), (9, (10, 20, 40), 8.6)])
def test_design_order_1d_residual(oracle, r, ns, lo):
    errs = []
    for n in ns:
        w = WL.density_wave_1d(n, r)
        g, p = w.grid, w.params
        U = w.U.copy()
        sx, sy = oracle.sigma_init(g, p, U)
        L, _, _ = oracle.residual(g, p, U, sx, sy)
        err = np.abs(g.interior(L)[:, 0, :] - _exact_dWdt_1d(n))
        errs.append(err[0].mean() * 2.0)   # L1 over [0,2]
    od = _orders(errs, ns)
    assert min(od) > lo, (errs, od)


def _exact_dWdt_2d(n):
    """Cell average of dW/dt for rho = 1 + 0.2 sin(pi (x-t)) sin(pi (y-t)), u=v=1, p=1."""
    dx = 2.0 / n
    e = np.arange(n + 1) * dx
    S = (np.cos(math.pi * e[:-1]) - np.cos(math.pi * e[1:])) / (math.pi * dx)   # avg sin
    Cv = (np.sin(math.pi * e[1:]) - np.sin(math.pi * e[:-1])) / (math.pi * dx)  # avg cos
    # d/dt rho = -0.2 pi [cos(pi x) sin(pi y) + sin(pi x) cos(pi y)]
    drho = -0.2 * math.pi * (np.outer(S, Cv) + np.outer(Cv, S))   # [j, i]
    return np.stack([drho, drho, drho, drho])


@pytest.mark.parametrize("r,ns,lo", [(5, (10, 20, 40), 4.7), (7, (10, 20, 40), 6.7), (9, (10, 20, 40), 8.6)])
def test_design_order_2d_residual(oracle, r, ns, lo):
    """2D, with (r-1)/2 Gauss points per face: at these meshes the quadrature
    error is far below the reconstruction error and the order is r."""
    errs = []
    for n in ns:
        w = WL.density_wave_2d(n, r)
        g, p = w.grid, w.params
        U = w.U.copy()
        sx, sy = oracle.sigma_init(g, p, U)
        L, _, _ = oracle.residual(g, p, U, sx, sy)
        err = np.abs(g.interior(L)[0] - _exact_dWdt_2d(n)[0])
        errs.append(err.mean() * 4.0)
    od = _orders(errs, ns)
    assert min(od) > lo, (errs, od)


@pytest.mark.slow
def test_design_order_1d_time_marched(oracle):
    """r = 5 to t = 2 with dt = min(CFL dt, dx^{5/3}) (the paper's dt = dx^{r/s})."""
    errs = []
    ns = (20, 40, 80)
    for n in ns:
        w = WL.density_wave_1d(n, 5)
        p = w.params
        p.dt_cap = (2.0 / n) ** (5.0 / 3.0)
        U, sx, sy, t, dts = oracle.run(w.grid, p, w.U, 10 ** 7, 2.0)
        assert abs(t - 2.0) < 1e-12
        rho = w.grid.interior(U)[0, 0]
        errs.append(np.abs(rho - WL.density_wave_exact_1d(n, 2.0)).mean() * 2.0)
    od = _orders(errs, ns)
    assert min(od) > 4.5, (errs, od)


# ---------------------------------------------------------------------------
# Sod tube against the exact Riemann solution
# ---------------------------------------------------------------------------

def _golden_sod():
    out = {}
    with open(os.path.join(HERE, "golden", "sod_star.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


def test_exact_riemann_solver_matches_textbook():
    gold = _golden_sod()
    ps, us = ER.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert abs(ps - gold["p_star"]) < 1e-5 and abs(us - gold["u_star"]) < 1e-5
    rl = ER.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), us - 1e-9)[0]
    rr = ER.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), us + 1e-9)[0]
    assert abs(rl - gold["rho_star_left"]) < 1e-5 and abs(rr - gold["rho_star_right"]) < 1e-5


def _sod_l1(oracle, n, order):
    w = WL.sod(n, order)
    U, _, _, t, _ = oracle.run(w.grid, w.params, w.U, w.nsteps, w.t_end)
    assert abs(t - 0.2) < 1e-14
    rho = w.grid.interior(U)[0, 0]
    ex = ER.cell_average_density((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), n, 0.2, sub=16)
    return np.abs(rho - ex).mean()


def test_sod_against_exact(oracle):
    e5 = _sod_l1(oracle, 200, 5)
    e1 = _sod_l1(oracle, 200, 1)
    assert e5 < 0.5 * e1, (e5, e1)
    assert e5 < 6e-3
    e9 = _sod_l1(oracle, 200, 9)
    assert e9 < 0.5 * e1
    # convergence with the mesh
    e100 = _sod_l1(oracle, 100, 5)
    e400 = _sod_l1(oracle, 400, 5)
    assert e400 < e5 < e100


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def _random_periodic_2d(n, order, seed):
    w = WL.density_wave_2d(n, order, seed=seed, amp=0.05)
    rng = np.random.default_rng(seed + 100)
    g = w.grid
    inner = g.interior(w.U)
    # add a density jump and a pressure jump
    inner[0, :, : n // 3] *= 1.5
    inner[3, n // 2:, :] *= 2.0
    inner[1] += 0.1 * rng.normal(size=inner[1].shape)
    return w


@pytest.mark.parametrize("r", [3, 5, 7, 9])
def test_conservation_periodic_2d(oracle, r):
    w = _random_periodic_2d(24, r, r)
    g = w.grid
    before = g.interior(w.U).sum(axis=(1, 2))
    U, _, _, _, _ = oracle.run(g, w.params, w.U, 5)
    after = g.interior(U).sum(axis=(1, 2))
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())


@pytest.mark.parametrize("r", [5, 9])
def test_conservation_periodic_1d(oracle, r):
    w = WL.density_wave_1d(64, r, seed=1, amp=0.2)
    g = w.grid
    WL.Grid  # noqa
    g.interior(w.U)[0, 0, :20] *= 3.0
    before = g.interior(w.U).sum(axis=(1, 2))
    U, _, _, _, _ = oracle.run(g, w.params, w.U, 20)
    after = g.interior(U).sum(axis=(1, 2))
    assert np.all(np.abs(after - before) <= 1e-13 * np.abs(before).max())


@pytest.mark.parametrize("dim,r", [(1, 9), (2, 3), (2, 5), (2, 7), (2, 9)])
def test_uniform_state_is_preserved(oracle, dim, r):
    """Identical faces give exactly zero flux differences; the SSP-RK3 stage
    combinations then change a uniform state by rounding only."""
    if dim == 1:
        w = WL.riemann_1d(40, (0.7, 0.3, 1.3), (0.7, 0.3, 1.3), r)
    else:
        w = WL.four_quadrant(20, r, states=((0.7, 0.3, -0.2, 1.3),) * 4)
    # exactly uniform interior (cut-cell averaging of equal states rounds)
    inner = w.grid.interior(w.U)
    inner[...] = inner[:, :1, :1]
    U = w.U.copy()
    sx, sy = oracle.sigma_init(w.grid, w.params, U)
    L, _, _ = oracle.residual(w.grid, w.params, U, sx, sy)
    assert np.all(w.grid.interior(L) == 0.0)
    U, _, _, _, _ = oracle.run(w.grid, w.params, w.U, 3)
    a, b = w.grid.interior(U), w.grid.interior(w.U)
    assert np.all(np.abs(a - b) <= 4 * np.spacing(np.abs(b)))


def test_mirror_symmetry_1d(oracle):
    a = WL.riemann_1d(120, (1.0, 0.3, 1.0), (0.3, -0.2, 0.2), 9, x_split=0.4)
    b = WL.riemann_1d(120, (0.3, 0.2, 0.2), (1.0, -0.3, 1.0), 9, x_split=0.6)
    Ua, _, _, _, _ = oracle.run(a.grid, a.params, a.U, 30)
    Ub, _, _, _, _ = oracle.run(b.grid, b.params, b.U, 30)
    ia = a.grid.interior(Ua)[:, 0]
    ib = b.grid.interior(Ub)[:, 0, ::-1]
    ib = ib * np.array([1, -1, 1])[:, None]
    assert np.max(np.abs(ia - ib) / np.abs(ia).max(axis=1, keepdims=True)) < 1e-13


def test_transpose_symmetry_2d(oracle):
    """Swapping x and y (and u and v) commutes with the 2D step."""
    st = ((1.0, 0.2, -0.1, 1.0), (0.4, 0.5, 0.3, 0.5), (0.9, -0.3, 0.6, 0.8), (0.2, 0.1, 0.1, 0.3))
    st_t = (st[0], st[3], st[2], st[1])
    st_t = tuple((s[0], s[2], s[1], s[3]) for s in st_t)
    a = WL.four_quadrant(28, 9, states=st, split=(0.55, 0.55))
    b = WL.four_quadrant(28, 9, states=st_t, split=(0.55, 0.55))
    Ua, _, _, _, _ = oracle.run(a.grid, a.params, a.U, 6)
    Ub, _, _, _, _ = oracle.run(b.grid, b.params, b.U, 6)
    ia = a.grid.interior(Ua)
    ib = b.grid.interior(Ub).transpose(0, 2, 1)[[0, 2, 1, 3]]
    assert np.max(np.abs(ia - ib) / np.abs(ia).max(axis=(1, 2), keepdims=True)) < 1e-13


# ---------------------------------------------------------------------------
# boundary fills and the strength state
# ---------------------------------------------------------------------------

def test_ghost_cells(oracle):
    # periodic: ghosts are wrapped copies
    w = WL.density_wave_2d(12, 9, seed=3)
    g = w.grid
    U = w.U.copy()
    oracle.sigma_init(g, w.params, U)
    ng = g.ng
    assert np.array_equal(U[:, ng:ng + g.ny, :ng], U[:, ng:ng + g.ny, g.nx:g.nx + ng])
    assert np.array_equal(U[:, :ng, :], U[:, g.ny:g.ny + ng, :])
    # transmissive: zero-gradient copies, corners from the x fill
    w = WL.four_quadrant(16, 7, seed=2)
    g = w.grid
    U = w.U.copy()
    oracle.sigma_init(g, w.params, U)
    ng = g.ng
    for k in range(ng):
        assert np.array_equal(U[:, ng:ng + g.ny, k], U[:, ng:ng + g.ny, ng])
        assert np.array_equal(U[:, k, :], U[:, ng, :])
        assert np.array_equal(U[:, ng + g.ny + k, :], U[:, ng + g.ny - 1, :])
    # inflow slot: Dirichlet rows inside the slot only
    w = WL.jet(64, 32, 7)
    g = w.grid
    U = w.U.copy()
    oracle.sigma_init(g, w.params, U)
    yc = g.y0 + (np.arange(g.ny) + 0.5) * g.dy
    inside = np.abs(yc) < 0.05
    assert inside.sum() == 6
    for j in range(g.ny):
        col = U[:, g.ng + j, 0]
        if inside[j]:
            assert np.array_equal(col, np.array(g.inflow))
        else:
            assert np.array_equal(col, U[:, g.ng + j, g.ng])


def test_sigma_state_rules(oracle):
    """Lagged DF source: strengths of non-flux faces are the periodic wrap,
    or first order from the adjacent ghost-filled cells; the first-order
    source recomputes every face from the stage input."""
    w = WL.four_quadrant(16, 9, seed=4)
    g, p = w.grid, w.params
    p.df_source = WL.DF_LAGGED
    U = w.U.copy()
    sx, sy = oracle.sigma_init(g, p, U)
    # one step makes the flux-face strengths differ from first order
    oracle.step(g, p, U, sx, sy, 0.0, 1)
    sx2, sy2 = sx.copy(), sy.copy()
    oracle.bc_fill(g, p, U, sx2, sy2)
    ng = g.ng
    fo_x, fo_y = oracle.sigma_init(g, p, U.copy())
    # flux faces untouched
    assert np.array_equal(sx2[ng:ng + g.ny, ng - 1:ng + g.nx], sx[ng:ng + g.ny, ng - 1:ng + g.nx])
    # ghost-row x-faces take the first-order value (transmissive)
    assert np.array_equal(sx2[:ng, :-1], fo_x[:ng, :-1])
    assert np.array_equal(sy2[:, :ng], fo_y[:, :ng])
    # periodic: every face equals its wrapped flux face
    w = WL.density_wave_2d(12, 9, seed=5, amp=0.1)
    g, p = w.grid, w.params
    p.df_source = WL.DF_LAGGED
    U = w.U.copy()
    sx, sy = oracle.sigma_init(g, p, U)
    oracle.step(g, p, U, sx, sy, 0.0, 1)
    oracle.bc_fill(g, p, U, sx, sy)
    ng = g.ng
    for J in range(g.NY):
        for I in range(g.NX - 1):
            jw = (J - ng) % g.ny + ng
            iw = (I - ng) % g.nx + ng
            assert sx[J, I] == sx[jw, iw]
    # first-order source: the boundary step makes every stored strength the
    # first-order one of the (ghost-filled) stage input
    w = WL.four_quadrant(16, 9, seed=4)
    g, p = w.grid, w.params
    assert p.df_source == WL.DF_FIRST_ORDER
    U = w.U.copy()
    sx, sy = oracle.sigma_init(g, p, U)
    oracle.step(g, p, U, sx, sy, 0.0, 1)
    oracle.bc_fill(g, p, U, sx, sy)
    fo_x, fo_y = oracle.sigma_init(g, p, U.copy())
    assert np.array_equal(sx[:, :-1], fo_x[:, :-1]) and np.array_equal(sy[:-1], fo_y[:-1])


def test_levels_smooth_and_shocked(oracle):
    """Smooth data selects the top linear order; a shock forces lower levels."""
    w = WL.density_wave_2d(20, 9)
    g, p = w.grid, w.params
    U = w.U.copy()
    sx, sy = oracle.sigma_init(g, p, U)
    _, _, lev = oracle.reconstruct(g, p, 0, U, sx, sy, want_level=True)
    assert np.all(lev == 9)
    w = WL.four_quadrant(20, 9, states=WL.CONFIG3_STATES)
    g, p = w.grid, w.params
    U = w.U.copy()
    sx, sy = oracle.sigma_init(g, p, U)
    _, _, lev = oracle.reconstruct(g, p, 0, U, sx, sy, want_level=True)
    assert set(np.unique(lev)) >= {2, 9}


def test_oracle_threads_do_not_change_results(oracle):
    """The oracle's parallel loops write disjoint cells and faces: one
    thread and several give the same bits (2D and 1D, both DF sources)."""
    # (grids above 4096 cells: smaller ones run every loop serially)
    cases = [WL.four_quadrant(83, 9, seed=2, ny=61), WL.blast_wave(5003, 7)]
    lag = WL.four_quadrant(71, 7, seed=6)
    lag.params.df_source = WL.DF_LAGGED
    lag.params.positivity_fallback = 1
    cases.append(lag)
    before = oracle.set_threads(0)
    try:
        for w in cases:
            g, p = w.grid, w.params
            out = []
            for nt in (1, 3):
                assert oracle.set_threads(nt) == nt
                U = w.U.copy()
                sx, sy = oracle.sigma_init(g, p, U)
                oracle.step(g, p, U, sx, sy if g.dim == 2 else None, 0.0, 3)
                out.append((U, sx, sy))
            assert np.isfinite(out[0][0]).all()
            for a, b in zip(out[0], out[1]):
                if a is not None:
                    assert np.array_equal(a.view(np.int64), b.view(np.int64))
    finally:
        oracle.set_threads(before)
