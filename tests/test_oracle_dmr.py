"""The double Mach reflection set-up (Sec. 4, Example 4) in the oracle: its
boundary sides (post-shock inflow, slip wall from x = 1/6, the exact moving
shock on the top) and a coarse run that stays physical with the shock foot
and the top crossing where the exact shock is.
"""
import math

import numpy as np

from paper_2410_05489_amd import workloads as WL


def _prim(U):
    rho = U[0]
    u, v = U[1] / rho, U[2] / rho
    return rho, u, v, 0.4 * (U[3] - 0.5 * rho * (u * u + v * v))


def test_boundary_sides(oracle):
    w = WL.double_mach(48, 12, 5)
    g, p = w.grid, w.params
    U = w.U.copy()
    sx, sy = oracle.sigma_init(g, p, U)
    t = 0.013
    oracle.bc_fill_at(g, p, t, U, sx, sy)
    ng = g.ng
    post, pre = np.array(g.inflow), np.array(g.outer)
    xc = (np.arange(g.NX) - ng + 0.5) * g.dx
    xs = 1.0 / 6.0 + (1.0 + 20.0 * t) / math.sqrt(3.0)
    for k in range(ng):
        top = U[:, ng + g.ny + k, :]
        assert np.array_equal(top[:, xc < xs], np.repeat(post[:, None], int((xc < xs).sum()), 1))
        assert np.array_equal(top[:, xc >= xs], np.repeat(pre[:, None], int((xc >= xs).sum()), 1))
        bot = U[:, ng - 1 - k, :]
        inflow = xc < 1.0 / 6.0
        assert np.array_equal(bot[:, inflow], np.repeat(post[:, None], int(inflow.sum()), 1))
        mirror = U[:, ng + k, :].copy()
        mirror[2] = -mirror[2]
        assert np.array_equal(bot[:, ~inflow], mirror[:, ~inflow])
        # left side: post-shock inflow on every interior row
        assert np.array_equal(U[:, ng:ng + g.ny, ng - 1 - k], np.repeat(post[:, None], g.ny, 1))


def test_coarse_run_stays_physical_and_tracks_the_shock(oracle):
    w = WL.double_mach(96, 24, 5)
    g, p = w.grid, w.params
    U, _, _, t, h = oracle.run(g, p, w.U, w.nsteps, 0.2)
    assert abs(t - 0.2) < 1e-14
    rho, u, v, pr = _prim(g.interior(U))
    assert np.isfinite(rho).all() and rho.min() > 0 and pr.min() > 0
    # along the top row the density falls from the post-shock value to the
    # pre-shock one within a few cells of the exact shock position
    xs = 1.0 / 6.0 + (1.0 + 20.0 * t) / math.sqrt(3.0)
    xc = (np.arange(g.nx) + 0.5) * g.dx
    top = rho[-1]
    assert np.all(top[xc > xs + 4 * g.dx] < 1.5)
    assert np.all(top[(xc < xs - 4 * g.dx) & (xc > 1.0)] > 6.0)
