"""Helpers shared by the adjoint tests: the torch adjoint oracle set up for a
1D grid, and one SSP-RK3 step of the C oracle with the three stage strengths
replayed (the frozen-decision map whose transposed Jacobian the adjoint is)."""
import dataclasses

import numpy as np
import torch

from oracle import oracle as O
from oracle.adjoint_torch import Step1D
from paper_2410_05489_amd import workloads as WL


def stepper(g, p):
    bc = {WL.BC_PERIODIC: "periodic", WL.BC_REFLECTIVE: "reflective"}.get(g.bc[0], "transmissive")
    return Step1D(g.nx, g.ng, g.dx, p.order, bc, p.gamma, p.sigma_thres, p.eps, p.d_hi, p.d_lo,
                  bool(p.positivity_fallback), p.df_source == WL.DF_FIRST_ORDER)


def _residual(g, p, U, s):
    """The C oracle's L(U) with the strengths s replayed: the boundary step
    runs with the lagged rule, which keeps the flux-face strengths as given
    (and for periodic, transmissive and reflective ends derives the other
    faces as the first-order rule does from first-order flux faces)."""
    q = dataclasses.replace(p, df_source=WL.DF_LAGGED)
    L, sn, _ = O.residual(g, q, U.copy(), s.copy(), np.zeros_like(s))
    return L, sn


def stage_sigmas(g, p, U, sx, dt):
    """Strength arrays read by the three stages of the C oracle's step from
    (U, sx) with time step dt: the previous stage's Gauss-point strengths
    (lagged source) or the first-order strengths of each stage input."""
    if p.df_source == WL.DF_FIRST_ORDER:
        s0 = O.sigma_init(g, p, U.copy())[0]
        L1, _ = _residual(g, p, U, s0)
        U1 = U + dt * L1
        s1 = O.sigma_init(g, p, U1.copy())[0]
        L2, _ = _residual(g, p, U1, s1)
        U2 = 0.75 * U + 0.25 * U1 + 0.25 * dt * L2
        s2 = O.sigma_init(g, p, U2.copy())[0]
        return [s0, s1, s2]
    L1, s1 = _residual(g, p, U, sx)
    U1 = U + dt * L1
    L2, s2 = _residual(g, p, U1, s1)
    return [sx.copy(), s1, s2]


def frozen_step(g, p, U, sigs, dt):
    """SSP-RK3 step of the C oracle's residual with the stage strengths
    given (stage k reads sigs[k]); returns the interior [3, nx]."""
    L1, _ = _residual(g, p, U, sigs[0])
    U1 = U + dt * L1
    L2, _ = _residual(g, p, U1, sigs[1])
    U2 = 0.75 * U + 0.25 * U1 + 0.25 * dt * L2
    L3, _ = _residual(g, p, U2, sigs[2])
    U3 = (1.0 / 3.0) * U + (2.0 / 3.0) * U2 + (2.0 / 3.0) * dt * L3
    return g.interior(U3)[:, 0]


def evolved(w, nsteps):
    """(U, sx) of a workload after nsteps oracle steps from its initial state."""
    g, p = w.grid, w.params
    U = w.U.copy()
    sx, _ = O.sigma_init(g, p, U)
    if nsteps:
        O.step(g, p, U, sx, None, 0.0, nsteps)
    return U, sx


def oracle_vjp(g, p, U, sx, dt, lam):
    """lam^T d(step)/dU from the torch adjoint oracle; lam, result [3, nx]."""
    st = stepper(g, p)
    Ui = torch.tensor(np.ascontiguousarray(g.interior(U)[:, 0]))
    return st.vjp(Ui, torch.tensor(sx[0]), float(dt), torch.tensor(lam)).numpy()
