"""Pins of the reflective (slip-wall) boundary of the oracle: a wall is a
symmetry plane, so a mirror-symmetric periodic problem on [-1,1] restricted
to [0,1] must equal the same problem run on [0,1] between two walls; walls
conserve mass and energy; the blast wave and the Shu-Osher problem run to
their final times with physical states."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_05489_amd import workloads as WL


def _symmetric_pair(n, order):
    """(full periodic grid on [-1,1] with 2n cells, half grid on [0,1] with n
    cells between walls) and their initial states: rho, p even and u odd about
    x = 0 (and about x = +-1)."""
    gamma = 1.4

    def avg(f, xl, xr, q=8):
        xg, wg = np.polynomial.legendre.leggauss(q)
        acc = 0.0
        for a, b in zip(xg, wg):
            acc = acc + 0.5 * b * f(0.5 * (xl + xr) + 0.5 * (xr - xl) * a)
        return acc

    rho = lambda x: 1.0 + 0.2 * np.cos(math.pi * x)            # noqa: E731
    mom = lambda x: rho(x) * 0.3 * np.sin(math.pi * x)          # noqa: E731
    ene = lambda x: (1.0 + 0.1 * np.cos(math.pi * x)) / (gamma - 1) + 0.5 * mom(x) ** 2 / rho(x)   # noqa: E731
    out = []
    for lo, N, bc in ((-1.0, 2 * n, WL.BC_PERIODIC), (0.0, n, WL.BC_REFLECTIVE)):
        dx = 1.0 / n
        g = WL.Grid(dim=1, nx=N, ny=1, ng=WL.ghosts_for(order), dx=dx, dy=dx, bc=(bc,) * 4)
        xl = lo + np.arange(N) * dx
        W = np.stack([avg(f, xl, xl + dx) for f in (rho, mom, ene)])
        U = WL.empty_state(g)
        g.interior(U)[:, 0] = W
        out.append((g, U))
    return out, WL.Params(order=order, gamma=gamma, cfl=0.5)


@pytest.mark.parametrize("order", [9, 5, 3])
def test_wall_is_a_symmetry_plane(order):
    n = 32
    ((gf, Uf), (gh, Uh)), p = _symmetric_pair(n, order)
    Uf, _, _, tf, df = O.run(gf, p, Uf, 20)
    Uh, _, _, th, dh = O.run(gh, p, Uh, 20)
    assert np.allclose(df, dh, rtol=1e-14, atol=0)
    full = gf.interior(Uf)[:, 0, n:]            # the [0,1] half of the periodic run
    half = gh.interior(Uh)[:, 0]
    for v in range(3):
        assert np.max(np.abs(full[v] - half[v])) <= 1e-12 * np.max(np.abs(full[v])), v


def test_walls_conserve_mass_and_energy():
    w = WL.blast_wave(200, 9)
    g, p = w.grid, w.params
    m0 = g.interior(w.U)[:, 0].sum(axis=1)
    U, _, _, t, dts = O.run(g, p, w.U, 300)
    I = g.interior(U)[:, 0]
    m1 = I.sum(axis=1)
    assert abs(m1[0] - m0[0]) <= 1e-12 * m0[0]
    assert abs(m1[2] - m0[2]) <= 1e-12 * m0[2]


@pytest.mark.slow
@pytest.mark.parametrize("make", [lambda: WL.blast_wave(400, 9), lambda: WL.shu_osher(200, 9)])
def test_runs_to_final_time_with_physical_states(make):
    w = make()
    g, p = w.grid, w.params
    U, _, _, t, dts = O.run(g, p, w.U, w.nsteps, w.t_end)
    assert abs(t - w.t_end) < 1e-14
    I = g.interior(U)[:, 0]
    pr = (p.gamma - 1) * (I[2] - 0.5 * I[1] ** 2 / I[0])
    assert np.isfinite(I).all() and I[0].min() > 0 and pr.min() > 0


def test_box_walls_conserve_in_2d():
    """Four-quadrant data in a box of reflective walls (lagged DF source: the
    strengths of the ghost faces are the mirror images of the interior ones),
    60 steps: mass and energy totals to round-off."""
    w = WL.four_quadrant(45, 9, seed=7, ny=37)
    w.grid.bc = (WL.BC_REFLECTIVE,) * 4
    g, p = w.grid, w.params
    m0 = g.interior(w.U).sum(axis=(1, 2))
    U, _, _, _, _ = O.run(g, p, w.U, 60)
    m1 = g.interior(U).sum(axis=(1, 2))
    assert np.isfinite(m1).all()
    for v in (0, 3):
        assert abs(m1[v] - m0[v]) <= 1e-13 * m0[v], v
