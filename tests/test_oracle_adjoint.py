"""Pins of the reference discrete adjoint (oracle/adjoint_torch.py).

The torch restatement of the 1D step must equal the C oracle's step, and its
transposed Jacobian must match central finite differences of the C oracle's
step with the stage strengths (hence DF factors and levels) and the time step
replayed, on smooth data (every DF factor 1) and on shocked data (WENO-Z-AO
stencils and DF factors below 1 active)."""
import numpy as np
import pytest
import torch

from adjoint_ref import evolved, frozen_step, oracle_vjp, stage_sigmas, stepper
from oracle import oracle as O
from paper_2410_05489_amd import workloads as WL

CASES = [
    ("wave", 9), ("wave", 7), ("wave", 5), ("wave", 3),
    ("sod", 9), ("sod", 7), ("sod", 5), ("sod", 3), ("sodlag", 9), ("sodlag", 5), ("rarefaction", 9),
    ("wall", 9), ("wall", 5),
]


def _workload(kind, order, df_fo=False):
    if kind == "wave":
        w = WL.density_wave_1d(40, order, seed=1)
    elif kind == "sod":
        w = WL.sod(60, order)
    elif kind == "sodlag":
        # the lagged DF source: strengths from the previous stage's face states
        w = WL.sod(60, order)
        w.params.df_source = WL.DF_LAGGED
    elif kind == "wall":
        # smooth data between two reflective walls
        w = WL.shu_osher(40, order)
        g = w.grid
        g.bc = (WL.BC_REFLECTIVE,) * 4
        x = (np.arange(g.nx) + 0.5) / g.nx
        rho = 1.0 + 0.2 * np.cos(np.pi * x)
        g.interior(w.U)[:, 0] = WL.conservative(rho, 0.3 * np.sin(np.pi * x), 0.0,
                                                1.0 + 0.1 * np.cos(np.pi * x), 1.4, 1)
        w.params.positivity_fallback = 0
    elif kind == "rarefaction":
        # strong rarefaction: non-physical face states replaced by averages
        # (the lagged source lets the first stage reconstruct across the
        # jump; the first-order one damps it and leaves nothing to replace)
        w = WL.riemann_1d(60, (1.115, -4.992, 0.143), (0.884, 4.943, 0.137), order)
        w.params.positivity_fallback = 1
        w.params.df_source = WL.DF_LAGGED
    else:
        raise ValueError(kind)
    if df_fo:
        w.params.df_source = WL.DF_FIRST_ORDER
    return w


@pytest.mark.parametrize("kind,order", CASES)
def test_forward_equals_c_oracle(kind, order):
    w = _workload(kind, order)
    g, p = w.grid, w.params
    U, sx = evolved(w, 3)
    U0, s0 = U.copy(), sx.copy()
    _, dts = O.step(g, p, U, sx, None, 0.0, 1)
    st = stepper(g, p)
    Un, s3 = st.step(torch.tensor(np.ascontiguousarray(g.interior(U0)[:, 0])), torch.tensor(s0[0]), float(dts[0]))
    ref = g.interior(U)[:, 0]
    assert np.max(np.abs(Un.numpy() - ref)) <= 1e-14 * np.max(np.abs(ref))
    ng = g.ng
    # lagged source: the strengths the step hands on are its last stage's
    # Gauss-point ones, equal to rounding of the pressure difference they are
    # made of (the first-order source hands on those of the final state,
    # which the restatement does not form)
    if p.df_source == WL.DF_LAGGED:
        a, b = s3.numpy()[ng - 1:ng + g.nx], sx[0, ng - 1:ng + g.nx]
        assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b))


def test_forward_equals_c_oracle_first_order_df():
    w = _workload("sod", 9, df_fo=True)
    g, p = w.grid, w.params
    U, sx = evolved(w, 4)
    U0, s0 = U.copy(), sx.copy()
    _, dts = O.step(g, p, U, sx, None, 0.0, 1)
    Un, _ = stepper(g, p).step(torch.tensor(np.ascontiguousarray(g.interior(U0)[:, 0])), torch.tensor(s0[0]),
                               float(dts[0]))
    ref = g.interior(U)[:, 0]
    assert np.max(np.abs(Un.numpy() - ref)) <= 1e-14 * np.max(np.abs(ref))


def _levels(g, p, U, s):
    _, _, lev = O.reconstruct(g, p, 0, U.copy(), s.copy(), np.zeros_like(s), want_level=True)
    return lev


@pytest.mark.parametrize("kind,order", CASES)
def test_vjp_matches_finite_differences(kind, order):
    """Central differences (h = 1e-6 relative) of lam . step(U) with the stage
    strengths and dt replayed, on 24 random components and the cells next to
    the boundaries, within 1e-6 of the
    largest adjoint component."""
    w = _workload(kind, order)
    g, p = w.grid, w.params
    U, sx = evolved(w, {"wave": 6, "sod": 1, "sodlag": 1, "rarefaction": 1, "wall": 4}[kind])
    dt = O.cfl_dt(g, p, U)
    sigs = stage_sigmas(g, p, U, sx, dt)
    lev = _levels(g, p, U, sigs[0])
    if kind in ("wave", "wall"):
        assert np.all(lev == order)               # smooth: top level, DF factor 1
    elif kind == "wall":
        # smooth data between two reflective walls
        w = WL.shu_osher(40, order)
        g = w.grid
        g.bc = (WL.BC_REFLECTIVE,) * 4
        x = (np.arange(g.nx) + 0.5) / g.nx
        rho = 1.0 + 0.2 * np.cos(np.pi * x)
        g.interior(w.U)[:, 0] = WL.conservative(rho, 0.3 * np.sin(np.pi * x), 0.0,
                                                1.0 + 0.1 * np.cos(np.pi * x), 1.4, 1)
        w.params.positivity_fallback = 0
    elif kind == "rarefaction":
        wl, wr = O.reconstruct(g, p, 0, U.copy(), sigs[0].copy(), np.zeros_like(sigs[0]))
        W = np.concatenate([wl[:, 0], wr[:, 0]], axis=1)
        pr = (p.gamma - 1) * (W[2] - 0.5 * W[1] ** 2 / W[0])
        assert np.any((W[0] <= 0) | (pr <= 0))   # replacements present
    elif order > 3:
        assert np.any(lev == 2)                   # WENO-Z-AO cells present
    else:
        A = sigs[0][0, :-1] + sigs[0][0, 1:]
        assert np.any(A[g.ng - 1:g.ng + g.nx - 1] > p.sigma_thres)   # DF factor below 1
    rng = np.random.default_rng(order)
    lam = rng.standard_normal((3, g.nx))
    adj = oracle_vjp(g, p, U, sx, dt, lam)
    scale = np.max(np.abs(adj))
    ng = g.ng
    comps = [(int(rng.integers(0, 3)), int(rng.integers(0, g.nx))) for _ in range(24)]
    comps += [(v, i) for v in range(3) for i in (0, 1, g.nx - 2, g.nx - 1)]   # boundary cells (ghost folds)
    for v, i in comps:
        h = 1e-6 * max(1.0, abs(U[v, 0, ng + i]))
        Up, Um = U.copy(), U.copy()
        Up[v, 0, ng + i] += h
        Um[v, 0, ng + i] -= h
        fd = np.sum(lam * (frozen_step(g, p, Up, sigs, dt) - frozen_step(g, p, Um, sigs, dt))) / (2 * h)
        assert abs(fd - adj[v, i]) <= 1e-6 * scale, (v, i, fd, adj[v, i])


def test_vjp_first_order_df_smooth():
    """First-order DF source on smooth data (strengths far below the
    threshold): the frozen-strength VJP is the full derivative."""
    w = _workload("wave", 9, df_fo=True)
    g, p = w.grid, w.params
    U, sx = evolved(w, 2)
    dt = O.cfl_dt(g, p, U)
    rng = np.random.default_rng(5)
    lam = rng.standard_normal((3, g.nx))
    adj = oracle_vjp(g, p, U, sx, dt, lam)
    delta = rng.standard_normal((3, g.nx))
    h = 1e-6
    Up, Um = U.copy(), U.copy()
    g.interior(Up)[:, 0] += h * delta
    g.interior(Um)[:, 0] -= h * delta
    sp, sm = O.sigma_init(g, p, Up)[0], O.sigma_init(g, p, Um)[0]
    Op, Om = Up.copy(), Um.copy()
    O.step(g, p.__class__(**{**p.__dict__, "cfl": 1e6, "dt_cap": dt}), Op, sp, None, 0.0, 1)
    O.step(g, p.__class__(**{**p.__dict__, "cfl": 1e6, "dt_cap": dt}), Om, sm, None, 0.0, 1)
    fd = np.sum(lam * (g.interior(Op)[:, 0] - g.interior(Om)[:, 0])) / (2 * h)
    ad = np.sum(adj * delta)
    assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_vjp_is_linear_and_transposes_the_jvp():
    """Dot-product test on shocked data: <lam, J d> from central differences
    of the frozen C step equals <J^T lam, d>."""
    w = _workload("sod", 9)
    g, p = w.grid, w.params
    U, sx = evolved(w, 1)
    dt = O.cfl_dt(g, p, U)
    sigs = stage_sigmas(g, p, U, sx, dt)
    rng = np.random.default_rng(11)
    lam = rng.standard_normal((3, g.nx))
    delta = rng.standard_normal((3, g.nx)) * np.max(np.abs(g.interior(U)[:, 0]), axis=1, keepdims=True)
    adj = oracle_vjp(g, p, U, sx, dt, lam)
    adj2 = oracle_vjp(g, p, U, sx, dt, 2.0 * lam)
    assert np.allclose(adj2, 2.0 * adj, rtol=1e-14, atol=0.0)
    h = 1e-7
    Up, Um = U.copy(), U.copy()
    g.interior(Up)[:, 0] += h * delta
    g.interior(Um)[:, 0] -= h * delta
    jvp = (frozen_step(g, p, Up, sigs, dt) - frozen_step(g, p, Um, sigs, dt)) / (2 * h)
    lhs, rhs = np.sum(lam * jvp), np.sum(adj * delta)
    assert abs(lhs - rhs) <= 1e-6 * np.sum(np.abs(adj * delta))


@pytest.mark.parametrize("order", [9, 3])
def test_vjp_conservation_periodic(order):
    """With periodic boundaries the flux differences telescope, so each
    variable's total is conserved for any state: every column of the step
    Jacobian sums to one within its variable, i.e. J^T 1_v = 1_v."""
    w = WL.density_wave_1d(24, order, seed=3)
    g, p = w.grid, w.params
    U, sx = evolved(w, 2)
    dt = O.cfl_dt(g, p, U)
    for v in range(3):
        lam = np.zeros((3, g.nx))
        lam[v] = 1.0
        adj = oracle_vjp(g, p, U, sx, dt, lam)
        assert np.allclose(adj, lam, rtol=0, atol=1e-13)
