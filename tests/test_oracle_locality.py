"""Locality of one oracle step, the property the sampled full-size GPU checks
rest on: a window of the input that reaches H cells beyond a cell, advanced
alone with the same time step, gives that cell exactly the full grid's
value once H covers the step's domain of dependence (two stages of R + 1
cell stencils and lagged strengths), and not before (1D, where the window
edges cut through structure)."""
import copy

import numpy as np

from oracle import oracle as O
from paper_2410_05489_amd import workloads as WL


def _capped(w, frac=0.5):
    g, p = w.grid, copy.copy(w.params)
    I = g.interior(w.U)
    rho = I[0]
    u = I[1] / rho
    if g.dim == 2:
        v = I[2] / rho
        pr = (p.gamma - 1.0) * (I[3] - 0.5 * rho * (u * u + v * v))
        c = np.sqrt(p.gamma * pr / rho)
        lam = (np.abs(u) + c) / g.dx + (np.abs(v) + c) / g.dy
    else:
        pr = (p.gamma - 1.0) * (I[2] - 0.5 * rho * u * u)
        c = np.sqrt(p.gamma * pr / rho)
        lam = (np.abs(u) + c) / g.dx
    p.dt_cap = frac * p.cfl / float(lam.max())
    return p


def _window(w, lo, hi):
    g = w.grid
    if g.dim == 2:
        sg = WL.Grid(dim=2, nx=hi[0] - lo[0], ny=hi[1] - lo[1], ng=g.ng, dx=g.dx, dy=g.dy, bc=g.bc)
        U = WL.empty_state(sg)
        sg.interior(U)[...] = g.interior(w.U)[:, lo[1]:hi[1], lo[0]:hi[0]]
    else:
        sg = WL.Grid(dim=1, nx=hi[0] - lo[0], ny=1, ng=g.ng, dx=g.dx, dy=g.dy, bc=g.bc)
        U = WL.empty_state(sg)
        sg.interior(U)[...] = g.interior(w.U)[:, :, lo[0]:hi[0]]
    return sg, U


def test_gks1d_step_is_local():
    n = 2048
    w = WL.shu_osher(n, 9)
    g = w.grid
    p = _capped(w)
    U = w.U.copy()
    sx, _ = O.sigma_init(g, p, U)
    O.step_gks(g, p, U, sx, 0.0, 1, c1=0.05, c2=1.0)
    shock = n // 10
    errs = {}
    for H in (4, 20):
        worst = 0.0
        for c in (0, 3, shock - 1, shock, shock + 2, n // 2, n - 1):
            lo, hi = max(0, c - H), min(n, c + H + 1)
            sg, Uw = _window(w, (lo,), (hi,))
            a, _ = O.sigma_init(sg, p, Uw)
            O.step_gks(sg, p, Uw, a, 0.0, 1, c1=0.05, c2=1.0)
            worst = max(worst, float(np.abs(sg.interior(Uw)[:, 0, c - lo] - g.interior(U)[:, 0, c]).max()))
        errs[H] = worst
    assert errs[20] == 0.0
    assert errs[4] > 1e-12   # the window edge does reach a cell 4 away


def test_gks2d_step_is_local():
    w = WL.four_quadrant(40, 9, states=WL.CONFIG3_STATES, split=(0.55, 0.45))
    g = w.grid
    p = _capped(w)
    U = w.U.copy()
    sx, sy = O.sigma_init(g, p, U)
    O.step_gks2d(g, p, U, sx, sy, 0.0, 1, c1=0.05, c2=1.0)
    H = 16
    for ci, cj in ((22, 18), (0, 0), (39, 17), (21, 39)):
        lo = (max(0, ci - H), max(0, cj - H))
        hi = (min(g.nx, ci + H + 1), min(g.ny, cj + H + 1))
        sg, Uw = _window(w, lo, hi)
        a, b = O.sigma_init(sg, p, Uw)
        O.step_gks2d(sg, p, Uw, a, b, 0.0, 1, c1=0.05, c2=1.0)
        assert np.array_equal(sg.interior(Uw)[:, cj - lo[1], ci - lo[0]], g.interior(U)[:, cj, ci]), (ci, cj)
