"""Symmetries of the GPU step, checked without the oracle: on a square grid
with the same boundary rule on all sides, the transposed problem (x and y
swapped, rho u and rho v swapped) advances to the transposed state -- the x
and y sweeps are different kernels with different tiles and lane
mappings, so this compares them with each other -- and the problem mirrored
in x or y (that momentum negated) to the mirrored state.  To rounding
(the mirrored stencils sum their taps in the other order): 1e-12 of each
conserved quantity's scale."""
import numpy as np
import pytest
import torch

from paper_2410_05489_amd import ase
from paper_2410_05489_amd import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _run(w, U, n):
    sim = ase.Simulation(w.grid, w.params, U, device=DEV)
    sim.run(n)
    torch.cuda.synchronize()
    return sim.U.cpu().numpy(), float(sim.t.cpu()[0])


def _close(a, b, g):
    I, J = g.interior(a).reshape(4, -1), g.interior(b).reshape(4, -1)
    scale = np.abs(J).max(axis=1)
    scale[1] = scale[2] = max(scale[1], scale[2])
    return float(np.max(np.abs(I - J).max(axis=1) / np.maximum(scale, 1e-300)))


@pytest.mark.parametrize("order,bc", [(9, WL.BC_TRANSMISSIVE), (7, WL.BC_REFLECTIVE), (5, WL.BC_PERIODIC)])
def test_transpose(order, bc):
    w = WL.four_quadrant(56, order, seed=12, split=(0.41, 0.63))
    w.grid.bc = (bc,) * 4
    g = w.grid
    assert g.ld == g.NX == g.NY
    UT = np.ascontiguousarray(w.U.transpose(0, 2, 1)[[0, 2, 1, 3]])
    a, ta = _run(w, w.U, 3)
    b, tb = _run(w, UT, 3)
    assert abs(ta - tb) <= 1e-14 * ta
    back = np.ascontiguousarray(b.transpose(0, 2, 1)[[0, 2, 1, 3]])
    assert _close(back, a, g) < 1e-12


@pytest.mark.parametrize("axis", [1, 2])
def test_mirror(axis):
    w = WL.four_quadrant(50, 9, seed=13, ny=38, split=(0.37, 0.58))
    g = w.grid
    assert g.ld == g.NX
    M = np.ascontiguousarray(np.flip(w.U, axis=axis))
    mom = 1 if axis == 2 else 2        # x mirror (columns) flips rho u, y mirror rho v
    M[mom] = -M[mom]
    a, ta = _run(w, w.U, 3)
    b, tb = _run(w, M, 3)
    assert abs(ta - tb) <= 1e-14 * ta
    back = np.ascontiguousarray(np.flip(b, axis=axis))
    back[mom] = -back[mom]
    assert _close(back, a, g) < 1e-12


def _run_gks(w, U, n, mu=0.0):
    sim = ase.GksSimulation(w.grid, w.params, U, c1=0.05, c2=1.0, mu=mu, device=DEV)
    sim.run(n)
    torch.cuda.synchronize()
    return sim.U.cpu().numpy(), float(sim.t.cpu()[0])


@pytest.mark.parametrize("order,mu", [(9, 0.0), (5, 0.0), (5, 2e-3)])
def test_gks_transpose(order, mu):
    """The gas-kinetic x and y flux kernels (local frames rotated by 90
    degrees) against each other, inviscid and viscous."""
    w = WL.four_quadrant(48, order, states=WL.CONFIG3_STATES, split=(0.57, 0.44))
    g = w.grid
    assert g.ld == g.NX == g.NY
    UT = np.ascontiguousarray(w.U.transpose(0, 2, 1)[[0, 2, 1, 3]])
    a, ta = _run_gks(w, w.U, 2, mu)
    b, tb = _run_gks(w, UT, 2, mu)
    assert abs(ta - tb) <= 1e-14 * ta
    back = np.ascontiguousarray(b.transpose(0, 2, 1)[[0, 2, 1, 3]])
    assert _close(back, a, g) < 1e-12
