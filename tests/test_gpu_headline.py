"""The headline workload at its benchmark size and launch configuration: the
four-quadrant Riemann problem on 1024 x 1024 cells at order 9 (CFL 0.4,
200 steps, first-order DF source, no positivity replacement), advanced by
ase_step exactly as bench.py times it.

- Per-step parity over the run: at steps 1, 10, 50 and 200 the oracle
  advances the GPU's own state of step s-1 by one step; every cell is
  compared (1e-12 per conserved quantity), and the stencil levels that
  both directions select from that state agree bit for bit.
- The full run: independent GPU and oracle runs of all 200 steps from the
  initial data agree to 1e-9.

The oracle runs its parallel loops on every host thread it is given
(results do not depend on the count: test_oracle_solver)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2410_05489_amd import ase
from paper_2410_05489_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda"
NSTEPS = 200
CHECK = (1, 10, 50, 200)


def _rel(a, b):
    """Max-norm error per conserved quantity (mass, momentum vector,
    energy) relative to that quantity's largest value."""
    a, b = np.asarray(a).reshape(4, -1), np.asarray(b).reshape(4, -1)
    den = np.abs(b).max(axis=1)
    den[1] = den[2] = float(np.sqrt(b[1] ** 2 + b[2] ** 2).max())
    return float(np.max(np.abs(a - b).max(axis=1) / den))


@pytest.fixture(scope="module")
def gpu_run():
    """The GPU's states (U, sx, sy, t) before each checked step and after
    the last one, from one ase_step call per step on the bench workload."""
    w = WL.four_quadrant(1024, 9, seed=0)
    g, p = w.grid, w.params
    assert p.df_source == WL.DF_FIRST_ORDER and not p.positivity_fallback and p.cfl == 0.4
    U0 = w.U.copy()
    sx0, sy0 = O.sigma_init(g, p, U0.copy())
    sim = ase.Simulation(g, p, U0, device=DEV, sx=sx0, sy=sy0)
    snaps = {}
    for s in range(1, NSTEPS + 1):
        if s in CHECK:
            torch.cuda.synchronize()
            snaps[s - 1] = (sim.U.cpu().numpy(), sim.sx.cpu().numpy(), sim.sy.cpu().numpy(),
                            float(sim.t.cpu()[0]))
        sim.run(1)
        if s in CHECK:
            torch.cuda.synchronize()
            snaps[s] = (sim.U.cpu().numpy(), sim.sx.cpu().numpy(), sim.sy.cpu().numpy(),
                        float(sim.t.cpu()[0]))
    print(f"headline: {NSTEPS} GPU steps of {w.name}, t = {snaps[NSTEPS][3]:.6g}", flush=True)
    return w, snaps


@pytest.mark.timeout(600)
@pytest.mark.parametrize("s", CHECK)
def test_headline_per_step_parity(gpu_run, s):
    w, snaps = gpu_run
    g, p = w.grid, w.params
    U, sx, sy, t = snaps[s - 1]
    Ug = snaps[s][0]
    print(f"headline step {s}: oracle step from the GPU state of step {s - 1}", flush=True)
    Uo, sxo, syo = U.copy(), sx.copy(), sy.copy()
    to, _ = O.step(g, p, Uo, sxo, syo, t, 1)
    assert abs(to - snaps[s][3]) <= 1e-15 * max(1.0, to)
    a, b = g.interior(Ug), g.interior(Uo)
    assert np.isfinite(a).all()
    assert _rel(a, b) < 1e-12
    # the levels both sweeps select from the state the step started from
    Uf, sxf, syf = U.copy(), sx.copy(), sy.copy()
    O.bc_fill(g, p, Uf, sxf, syf)
    for d in (0, 1):
        _, _, levo = O.reconstruct(g, p, d, Uf.copy(), sxf.copy(), syf.copy(), want_level=True)
        nf = ase.face_count(g, d)
        wl = torch.zeros((4, 4, nf), dtype=torch.float64, device=DEV)
        lev = torch.zeros((g.ny, g.nx), dtype=torch.int8, device=DEV)
        ase.reconstruct(g, p, d, torch.tensor(Uf, device=DEV), torch.tensor(sxf, device=DEV),
                        torch.tensor(syf, device=DEV), wl, torch.zeros_like(wl), lev)
        torch.cuda.synchronize()
        levg = lev.cpu().numpy()
        assert np.array_equal(levg, levo), (d, int((levg != levo).sum()))
        del wl


@pytest.mark.timeout(900)
def test_headline_full_run(gpu_run):
    w, snaps = gpu_run
    g, p = w.grid, w.params
    U = w.U.copy()
    sx, sy = O.sigma_init(g, p, U)
    print(f"headline full run: {NSTEPS} oracle steps on {O.set_threads(0)} host threads", flush=True)
    t, dts = O.step(g, p, U, sx, sy, 0.0, NSTEPS)
    assert len(dts) == NSTEPS
    assert abs(t - snaps[NSTEPS][3]) <= 1e-13 * t
    a, b = g.interior(snaps[NSTEPS][0]), g.interior(U)
    assert np.isfinite(b).all()
    assert _rel(a, b) < 1e-9
