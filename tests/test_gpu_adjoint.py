"""Discrete adjoint on the GPU (ase_adjoint_step, ase_adjoint_batched and the
autograd wrappers) against the torch adjoint oracle, plus properties that
hold at any size: bit-equality across launch shapes and between the batched
and single-grid paths, and central differences of the GPU forward with the
time steps replayed on smooth data."""
import numpy as np
import pytest
import torch

from adjoint_ref import evolved, oracle_vjp
from oracle import oracle as O
from paper_2410_05489_amd import adjoint as A
from paper_2410_05489_amd import ase
from paper_2410_05489_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _rel(a, b):
    """Largest error per variable relative to that variable's largest value."""
    a, b = np.asarray(a).reshape(3, -1), np.asarray(b).reshape(3, -1)
    den = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return float(np.max(np.abs(a - b).max(axis=1) / den))


def _case(name):
    if name.startswith("wave"):
        n, order = {"wave9": (600, 9), "wave5": (300, 5), "wave3": (300, 3)}[name]
        return WL.density_wave_1d(n, order, seed=2), 4
    if name == "sodlag":
        # the lagged DF source: strengths from the previous stage's face states
        w = WL.sod(300, 9)
        w.params.df_source = WL.DF_LAGGED
        return w, 2
    if name.startswith("sod"):
        n, order = {"sod9": (600, 9), "sod7": (300, 7), "sod5": (300, 5), "sod3": (300, 3)}[name]
        return WL.sod(n, order), 1
    if name == "rarefaction":
        # lagged source: its first stage reconstructs across the jump, whose
        # non-physical face states the positivity replacement takes over
        w = WL.riemann_1d(300, (1.115, -4.992, 0.143), (0.884, 4.943, 0.137), 9)
        w.params.positivity_fallback = 1
        w.params.df_source = WL.DF_LAGGED
        return w, 1
    if name == "wall":
        # Sod data between two reflective walls, lagged DF source (mirrored
        # ghost-face strengths)
        w = WL.sod(300, 9)
        w.grid.bc = (WL.BC_REFLECTIVE,) * 4
        w.params.df_source = WL.DF_LAGGED
        return w, 40
    if name == "wallfo":
        w = WL.sod(300, 9)
        w.grid.bc = (WL.BC_REFLECTIVE,) * 4
        return w, 40
    if name == "blast":
        return WL.blast_wave(300, 9), 5
    raise ValueError(name)


CASES = ["wave9", "sod9", "sod7", "sod5", "sod3", "wave5", "wave3", "sodlag", "rarefaction", "wall", "wallfo",
         "blast"]


@pytest.mark.parametrize("name", CASES)
def test_adjoint_step_matches_oracle(name):
    """One step, several 256-cell tiles with a ragged tail, element-wise
    within 1e-12 of the oracle's transposed Jacobian."""
    w, nev = _case(name)
    g, p = w.grid, w.params
    U, sx = evolved(w, nev)
    dt = O.cfl_dt(g, p, U)
    if name == "rarefaction":
        # the case exercises the positivity replacement of face states
        wl, wr = O.reconstruct(g, p, 0, U.copy(), sx.copy(), np.zeros_like(sx))
        W = np.concatenate([wl[:, 0], wr[:, 0]], axis=1)
        pr = (p.gamma - 1) * (W[2] - 0.5 * W[1] ** 2 / W[0])
        assert np.any((W[0] <= 0) | (pr <= 0))
    rng = np.random.default_rng(7)
    lam = rng.standard_normal((3, g.nx))
    ref = oracle_vjp(g, p, U, sx, dt, lam)
    Ud = torch.tensor(U, device=DEV)
    sd = torch.tensor(sx, device=DEV)
    dtd = torch.tensor([dt], dtype=torch.float64, device=DEV)
    lam_full = np.zeros((3, 1, g.ld))
    g.interior(lam_full)[:, 0] = lam
    ld = torch.tensor(lam_full, device=DEV)
    out = torch.full_like(ld, np.nan)
    ws = ase.Workspace(ase.adjoint_workspace_bytes(g), DEV)
    ase.adjoint_step(g, p, Ud, sd, dtd, ld, out, ws)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert _rel(g.interior(o)[:, 0], ref) < 1e-12
    ng = g.ng
    assert np.all(o[:, 0, :ng] == 0.0) and np.all(o[:, 0, ng + g.nx:ng * 2 + g.nx] == 0.0)
    # inputs untouched, in place gives the same bits
    assert np.array_equal(Ud.cpu().numpy(), U) and np.array_equal(sd.cpu().numpy(), sx)
    ase.adjoint_step(g, p, Ud, sd, dtd, ld, ld, ws)
    torch.cuda.synchronize()
    assert torch.equal(ld, out)


def _oracle_gradient(g, p, U0, nsteps):
    """dJ/dU0 of J = dx sum p after nsteps oracle steps (frozen decisions),
    by the torch adjoint oracle stepped back over the C oracle's states."""
    U = U0.copy()
    sx, _ = O.sigma_init(g, p, U)
    tape = []
    for _ in range(nsteps):
        Us, ss = U.copy(), sx.copy()
        _, dts = O.step(g, p, U, sx, None, 0.0, 1)
        tape.append((Us, ss, float(dts[0])))
    Wn = g.interior(U)[:, 0]
    u = Wn[1] / Wn[0]
    lam = g.dx * (p.gamma - 1.0) * np.stack([0.5 * u * u, -u, np.ones_like(u)])
    J = g.dx * np.sum((p.gamma - 1.0) * (Wn[2] - 0.5 * Wn[1] * u))
    for Us, ss, dt in reversed(tape):
        lam = oracle_vjp(g, p, Us, ss, dt, lam)
    return J, lam


def test_adjoint1d_autograd_matches_oracle():
    """Twelve steps with checkpoints every five: dJ/dU0 through
    torch.autograd against the oracle chain."""
    w = WL.sod(150, 5)
    g, p = w.grid, w.params
    run = A.Adjoint1D(g, p, DEV, every=5)
    U0 = torch.tensor(w.U, device=DEV, requires_grad=True)
    J = run.pressure(run.run(U0, 12))
    J.sum().backward()
    Jo, go = _oracle_gradient(g, p, w.U, 12)
    assert abs(J.item() - Jo) <= 1e-11 * abs(Jo)
    gr = U0.grad.cpu().numpy()
    assert _rel(g.interior(gr)[:, 0], go) < 1e-10
    assert np.all(gr[:, 0, :g.ng] == 0.0)


def _inst(b, A_, k):
    o = int(b.offsets[k])
    N = int(b.ncells[k])
    return np.ascontiguousarray(A_[:, o:o + N + 2 * b.ng]).reshape(3, 1, N + 2 * b.ng)


def test_batched_adjoint_matches_oracle():
    b = WL.batched_riemann(ninst=4, nmin=10, nmax=120, order=9, seed=3, nsteps=8)
    run = A.BatchedAdjoint(b, DEV, nbins=3, every=3)
    U0 = torch.tensor(b.U, device=DEV, requires_grad=True)
    J = run.pressure(run.run(U0, 8))
    J.sum().backward()
    Jg = J.detach().cpu().numpy()
    G = U0.grad.cpu().numpy()
    checked = 0
    for k in range(b.ninst):
        g = WL.instance_grid(b, k)
        Jo, go = _oracle_gradient(g, b.params, _inst(b, b.U, k), 8)
        if not np.isfinite(Jo):
            continue
        checked += 1
        assert abs(Jg[k] - Jo) <= 1e-11 * abs(Jo), k
        assert _rel(g.interior(_inst(b, G, k))[:, 0], go) < 1e-10, k
    assert checked >= 3


def test_batched_adjoint_equals_single_grid_bitwise():
    """The batched adjoint of every instance has the bits of the single-grid
    path (per-step ase_adjoint_step with checkpoints) on that instance."""
    b = WL.batched_riemann(ninst=5, nmin=30, nmax=700, order=9, seed=5, nsteps=7)
    run = A.BatchedAdjoint(b, DEV, nbins=2, every=4)
    U0 = torch.tensor(b.U, device=DEV, requires_grad=True)
    run.pressure(run.run(U0, 7)).sum().backward()
    G = U0.grad.cpu().numpy()
    for k in range(b.ninst):
        g = WL.instance_grid(b, k)
        r1 = A.Adjoint1D(g, b.params, DEV, every=3)
        u = torch.tensor(_inst(b, b.U, k), device=DEV, requires_grad=True)
        r1.pressure(r1.run(u, 7)).sum().backward()
        assert np.array_equal(u.grad.cpu().numpy(), _inst(b, G, k), equal_nan=True), k


def test_batched_adjoint_launch_shapes_agree_bitwise():
    b = WL.batched_riemann(ninst=12, nmin=64, nmax=1500, order=9, seed=6, nsteps=6)
    grads = []
    for nbins, thr in ((1, 256), (5, 128), (12, 256)):
        run = A.BatchedAdjoint(b, DEV, nbins=nbins, adj_threads=thr, every=4)
        U0 = torch.tensor(b.U, device=DEV, requires_grad=True)
        run.pressure(run.run(U0, 6)).sum().backward()
        grads.append(U0.grad.cpu().numpy())
    for gr in grads[1:]:
        assert np.array_equal(gr, grads[0], equal_nan=True)


def test_batched_adjoint_fd_smooth():
    """Smooth periodic instances, 100 steps with checkpoints every 10 (the
    batched adjoint configuration): 32 components per instance, central
    differences (h = 1e-6 relative) of J_k through the GPU forward with the
    recorded time steps replayed, each component within 1e-6 of
    max(|fd|, |grad|) plus the rounding floor of the difference quotient,
    4 eps |J_k| / h.  Every stage of every step is checked smooth on the
    oracle (all stencil strength sums below the threshold, so every DF
    factor is 1 and the frozen-decision gradient is the full one)."""
    from adjoint_ref import stage_sigmas
    b = WL.batched_smooth(ninst=16, nmin=64, nmax=512, order=9, seed=1, nsteps=100)
    R = (b.params.order - 1) // 2
    for k in range(b.ninst):
        g = WL.instance_grid(b, k)
        U = _inst(b, b.U, k).copy()
        sx, _ = O.sigma_init(g, b.params, U)
        for _ in range(b.nsteps):
            dt = O.cfl_dt(g, b.params, U)
            for sg in stage_sigmas(g, b.params, U, sx, dt):
                assert 2 * R * float(sg.max()) < b.params.sigma_thres, k
            O.step(g, b.params, U, sx, None, 0.0, 1)
    run = A.BatchedAdjoint(b, DEV, nbins=16, every=10)
    U0 = torch.tensor(b.U, device=DEV, requires_grad=True)
    J = run.pressure(run.run(U0, b.nsteps))
    J.sum().backward()
    G = U0.grad.cpu().numpy()
    Jk = J.detach().cpu().numpy()
    hist = run.dt_hist.clone()
    fwd = ase.BatchedSimulation(b, DEV, nbins=16)
    rng = np.random.default_rng(4)
    comps = [[(int(rng.integers(0, 3)), int(rng.integers(0, int(b.ncells[k])))) for _ in range(32)]
             for k in range(b.ninst)]

    def J_of(Uh):
        fwd.U.copy_(torch.tensor(Uh, device=DEV))
        fwd.t.zero_()
        run.sim.U.copy_(fwd.U)
        run.init_sigma()
        fwd.sig.copy_(run.sim.sig)
        fwd.run(b.nsteps, dt_replay=hist)
        Jv = torch.zeros(b.ninst, dtype=torch.float64, device=DEV)
        ase.pressure_objective(fwd.p, fwd.offsets, fwd.ncells, fwd.dx, b.ng, b.total, fwd.U, J=Jv)
        return Jv.cpu().numpy()

    eps = np.finfo(np.float64).eps
    worst = 0.0
    for c in range(32):
        Up, Um = b.U.copy(), b.U.copy()
        hs = np.zeros(b.ninst)
        for k in range(b.ninst):
            v, i = comps[k][c]
            e = int(b.offsets[k]) + b.ng + i
            hs[k] = 1e-6 * max(1.0, abs(b.U[v, e]))
            Up[v, e] += hs[k]
            Um[v, e] -= hs[k]
        fd = (J_of(Up) - J_of(Um)) / (2 * hs)
        for k in range(b.ninst):
            v, i = comps[k][c]
            gk = _inst(b, G, k)[:, 0, b.ng:b.ng + int(b.ncells[k])]
            floor = 4 * eps * abs(Jk[k]) / hs[k]
            err = abs(fd[k] - gk[v, i])
            bound = 1e-6 * max(abs(fd[k]), abs(gk[v, i])) + floor
            worst = max(worst, err / bound)
            assert err <= bound, (k, v, i, fd[k], gk[v, i], floor)
    print(f"adjoint fd: worst error / bound {worst:.3f}", flush=True)


def test_batched_adjoint_full_size():
    """256 instances of 64..4096 cells, order 9, 20 steps with checkpoints
    every 10: finite wherever the forward is, and the two smallest instances
    against the oracle chain."""
    b = WL.batched_riemann(nsteps=20)
    run = A.BatchedAdjoint(b, DEV, nbins=256, every=10)
    U0 = torch.tensor(b.U, device=DEV, requires_grad=True)
    UN = run.run(U0, b.nsteps)
    J = run.pressure(UN)
    J.sum().backward()
    G = U0.grad.cpu().numpy()
    Jg = J.detach().cpu().numpy()
    for k in range(b.ninst):
        if np.isfinite(Jg[k]):
            assert np.isfinite(_inst(b, G, k)).all(), k
    for k in np.argsort(b.ncells)[:2]:
        k = int(k)
        g = WL.instance_grid(b, k)
        Jo, go = _oracle_gradient(g, b.params, _inst(b, b.U, k), b.nsteps)
        if not np.isfinite(Jo):
            continue
        assert abs(Jg[k] - Jo) <= 1e-11 * abs(Jo), k
        assert _rel(g.interior(_inst(b, G, k))[:, 0], go) < 1e-10, k


def test_batched_adjoint_mixed_boundaries():
    """Per-instance boundary codes (periodic, transmissive and reflective):
    each instance's gradient has the bits of the single-grid path."""
    b = WL.batched_mixed(ninst=9, nmin=20, nmax=300, order=9, seed=7, nsteps=6)
    run = A.BatchedAdjoint(b, DEV, nbins=2, every=4)
    U0 = torch.tensor(b.U, device=DEV, requires_grad=True)
    run.pressure(run.run(U0, 6)).sum().backward()
    G = U0.grad.cpu().numpy()
    for k in range(b.ninst):
        g = WL.instance_grid(b, k)
        r1 = A.Adjoint1D(g, b.params, DEV, every=3)
        u = torch.tensor(_inst(b, b.U, k), device=DEV, requires_grad=True)
        r1.pressure(r1.run(u, 6)).sum().backward()
        assert np.array_equal(u.grad.cpu().numpy(), _inst(b, G, k), equal_nan=True), k


def test_batched_adjoint_phases_and_overlap_bitwise():
    """The backward with the recomputation of each segment on a side stream
    (tape phase into a second workspace while the main stream runs the
    previous segment back) gives the bits of the one-launch-per-segment
    backward; so does a tape launch followed by a reverse launch."""
    b = WL.batched_riemann(ninst=14, nmin=40, nmax=2000, order=9, seed=21, nsteps=11)
    grads = []
    for overlap in (False, True):
        run = A.BatchedAdjoint(b, DEV, nbins=5, every=3, overlap=overlap)
        U0 = torch.tensor(b.U, device=DEV, requires_grad=True)
        run.pressure(run.run(U0, b.nsteps)).sum().backward()
        torch.cuda.synchronize()
        grads.append(U0.grad.cpu().numpy())
    assert np.array_equal(grads[0], grads[1], equal_nan=True)
    # one segment, split into its two phases
    run = A.BatchedAdjoint(b, DEV, nbins=5, every=4)
    U0 = torch.tensor(b.U, device=DEV)
    run.run(U0, 4)
    hist = run.dt_hist[:4].clone()
    sig0 = torch.zeros(b.total, dtype=torch.float64, device=DEV)
    run.sim.U.copy_(U0)
    run.init_sigma()
    sig0.copy_(run.sim.sig)
    rng = np.random.default_rng(3)
    lam0 = torch.tensor(rng.standard_normal((3, b.total)), device=DEV)
    outs = []
    for phases in ((ase.ADJ_TAPE | ase.ADJ_REVERSE,), (ase.ADJ_TAPE, ase.ADJ_REVERSE)):
        lam = lam0.clone()
        ws = ase.Workspace(ase.adjoint_batched_workspace_bytes(b.total, 4), DEV)
        for ph in phases:
            ase.adjoint_batched(run.sim, U0, sig0, hist, 4, lam, ws, 256, phase=ph)
        torch.cuda.synchronize()
        outs.append(lam.cpu().numpy())
    assert np.array_equal(outs[0], outs[1], equal_nan=True)
