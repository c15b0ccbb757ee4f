"""Wide batched form (ase_step_batched_wide): the large instances of a batch
run as one launch per RK stage over many tiles, beside the persistent
launch that keeps the rest.  Every output must equal the persistent form's
(ase_step_batched) bit for bit: the same cells, faces, time steps and
stopping decisions, only a different assignment of work to workgroups."""
import numpy as np
import pytest
import torch

from paper_2410_05489_amd import ase
from paper_2410_05489_amd import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda"
WS = ase.WIDE_STEP   # or'ed into wide_threads: one launch per step


def _tile(wide_threads, order):
    """Tile length of the wide form for these lanes (and form) and order."""
    halo = 3 if wide_threads & WS else 1
    return (wide_threads & ~WS) - halo * (order + 1)


def _outputs(sim, hist=None, status=None):
    torch.cuda.synchronize()
    out = {"U": sim.U.cpu().numpy(), "sig": sim.sig.cpu().numpy(), "t": sim.t.cpu().numpy()}
    if hist is not None:
        out["dt_hist"] = hist.cpu().numpy()
    if status is not None:
        out["status"] = status.cpu().numpy()
    return out


def _assert_same(a, b, what):
    for key in a:
        assert np.array_equal(a[key], b[key], equal_nan=True), (what, key)


def _pair(b, nsteps, min_cells, wide_threads=256, nbins=4, threads=256, t_end=0.0, dt_replay=None, status=False):
    """(persistent, wide) outputs of the same batch and arguments."""
    res = []
    for wide in (False, True):
        sim = ase.BatchedSimulation(b, DEV, nbins=nbins, threads=threads,
                                    wide_min_cells=min_cells if wide else 0, wide_threads=wide_threads)
        if wide:
            assert sim.wide is not None and sim.wide["nwide"] > 0
        hist = torch.full((nsteps, b.ninst), -1.0, dtype=torch.float64, device=DEV)
        st = torch.full((b.ninst,), -1, dtype=torch.int32, device=DEV) if status else None
        print(f"wide={wide} ninst={b.ninst} nsteps={nsteps} min_cells={min_cells} "
              f"wide_threads={wide_threads}", flush=True)
        sim.run(nsteps, t_end, hist, dt_replay=dt_replay, status=st)
        res.append(_outputs(sim, hist, st))
    return res


@pytest.mark.parametrize("order,wide_threads", [(9, 256), (9, 512), (5, 256), (3, 512), (7, 256),
                                                (9, 256 | WS), (9, 512 | WS), (5, 256 | WS), (3, 512 | WS),
                                                (7, 256 | WS)])
def test_wide_equals_persistent_mixed_boundaries(order, wide_threads):
    """Periodic, transmissive and reflective instances of 16..3000 cells:
    those of 600 cells and more take the wide form (several tiles each,
    ragged last tile)."""
    b = WL.batched_mixed(ninst=12, nmin=16, nmax=3000, order=order, seed=21, nsteps=12)
    assert b.params.df_source == WL.DF_FIRST_ORDER
    p, w = _pair(b, b.nsteps, 600, wide_threads)
    _assert_same(p, w, "mixed")
    assert np.all(p["dt_hist"] > 0.0)


@pytest.mark.parametrize("wide_threads", [256, 256 | WS])
def test_wide_equals_persistent_every_split(wide_threads):
    """No instance wide (no tile launches), some, and all of them: the same
    bits as the persistent launch."""
    b = WL.batched_riemann(ninst=10, nmin=250, nmax=2000, order=9, seed=8, nsteps=8)
    ref = None
    for min_cells in (10**6, 1200, 1):
        sim = ase.BatchedSimulation(b, DEV, nbins=3, wide_min_cells=min_cells, wide_threads=wide_threads)
        print(f"min_cells={min_cells} nwide={sim.wide['nwide']} ntiles={sim.wide['ntiles']}", flush=True)
        hist = torch.zeros((b.nsteps, b.ninst), dtype=torch.float64, device=DEV)
        sim.run(b.nsteps, 0.0, hist)
        out = _outputs(sim, hist)
        if ref is None:
            base = ase.BatchedSimulation(b, DEV, nbins=3)
            h0 = torch.zeros_like(hist)
            base.run(b.nsteps, 0.0, h0)
            ref = _outputs(base, h0)
        _assert_same(ref, out, min_cells)


@pytest.mark.parametrize("wide_threads,calls", [(256, (30, 30)), (256 | WS, (30, 30)), (256 | WS, (7, 4, 1, 48)),
                                                 (512 | WS, (1, 1, 13, 45))])
def test_wide_t_end_and_repeated_calls(wide_threads, calls):
    """Instances stop at t_end at different steps (dt_hist 0 from there on);
    each call continues from the previous call's state and time (odd and
    even step counts: the one-launch-per-step form alternates two buffers)."""
    b = WL.batched_riemann(ninst=8, nmin=300, nmax=1500, order=9, seed=13, nsteps=sum(calls))
    t_end = 0.002
    sims, hists = [], []
    for wide in (0, 500):
        sim = ase.BatchedSimulation(b, DEV, nbins=2, wide_min_cells=wide, wide_threads=wide_threads)
        hs = []
        for n in calls:
            h = torch.full((n, b.ninst), -1.0, dtype=torch.float64, device=DEV)
            sim.run(n, t_end, h)
            hs.append(h)
        sims.append(_outputs(sim))
        hists.append(np.concatenate([h.cpu().numpy() for h in hs]))
    _assert_same(sims[0], sims[1], "t_end")
    assert np.array_equal(hists[0], hists[1])
    assert np.all(sims[1]["t"] <= t_end + 1e-14) and np.any(np.abs(sims[1]["t"] - t_end) < 1e-14)
    assert np.any(hists[1] == 0.0) and np.all(hists[1] >= 0.0)


@pytest.mark.parametrize("wide_threads", [256, 256 | WS])
def test_wide_dt_replay_stops_where_the_replay_ends(wide_threads):
    """Replayed time steps, with a zero entry that stops one wide instance
    part-way: the same bits as the persistent launch."""
    b = WL.batched_riemann(ninst=6, nmin=400, nmax=1600, order=9, seed=17, nsteps=10)
    base = ase.BatchedSimulation(b, DEV, nbins=2)
    rec = torch.zeros((b.nsteps, b.ninst), dtype=torch.float64, device=DEV)
    base.run(b.nsteps, 0.0, rec)
    torch.cuda.synchronize()
    replay = rec.clone()
    k = int(np.argmax(b.ncells))
    replay[4:, k] = 0.0
    p, w = _pair(b, b.nsteps, 400, wide_threads, nbins=2, dt_replay=replay)
    _assert_same(p, w, "replay")
    assert np.all(w["dt_hist"][4:, k] == 0.0) and np.all(w["dt_hist"][:4, k] > 0.0)


@pytest.mark.parametrize("wide_threads", [256, 256 | WS])
def test_wide_status_on_the_full_batch(wide_threads):
    """The 256-instance batch (64..4096 cells, order 9, 100 steps) with a
    status array, instances of 2048 cells and more in the wide form: U,
    strengths, times, time steps and status flags all equal the persistent
    launch's, including those of the wide instances the method loses."""
    b = WL.batched_riemann(nsteps=100)
    p, w = _pair(b, b.nsteps, 2048, wide_threads, nbins=256, status=True)
    _assert_same(p, w, "status")
    st = w["status"]
    assert np.all(st >= 0)
    lost_wide = [k for k in np.flatnonzero(st) if b.ncells[k] >= 2048]
    print(f"lost: {np.flatnonzero(st).tolist()}, wide among them: {lost_wide}", flush=True)
    assert len(lost_wide) > 0


@pytest.mark.parametrize("order,wide_threads", [(9, 256), (5, 512), (9, 256 | WS), (5, 512 | WS), (3, 256 | WS)])
def test_wide_tile_edges(order, wide_threads):
    """Cell counts at the tile edges (one full tile, one cell more, one short
    of two tiles, two, two and one cell) under each boundary kind, beside
    small persistent instances: the persistent launch's bits."""
    T = _tile(wide_threads, order)
    sizes = [T, T + 1, 2 * T - 1, 2 * T, 2 * T + 1]
    sizes = [n for n in sizes for _ in range(3)] + [20, 100, 150]
    b = WL.batched_mixed(order=order, seed=41, nsteps=6, sizes=sizes)
    p, w = _pair(b, b.nsteps, T, wide_threads, nbins=2)
    _assert_same(p, w, "edges")


@pytest.mark.parametrize("order,wide_threads", [(9, 256 | WS), (5, 512 | WS), (3, 256 | WS)])
def test_wide_step_tiles_every_instance(order, wide_threads):
    """The per-step form with every instance tiled (min_cells 1): instances
    from ng cells (one tile whose window holds the whole instance and its
    ghost cells) to several tiles, under each boundary kind, over an odd
    step count: the persistent launch's bits."""
    ng = (order + 1) // 2
    T = _tile(wide_threads, order)
    sizes = [ng, ng + 1, 16, 40, T - 1, T, T + 1, 3 * T + 7]
    sizes = [n for n in sizes for _ in range(3)]
    b = WL.batched_mixed(order=order, seed=47, nsteps=7, sizes=sizes)
    p, w = _pair(b, b.nsteps, 1, wide_threads, nbins=3)
    _assert_same(p, w, "every instance tiled")


@pytest.mark.parametrize("wide_threads", [256, 256 | WS])
def test_wide_dt_cap(wide_threads):
    """A cap on the time step that binds for some instances and steps (the
    CFL step of the others is smaller): the persistent launch's bits."""
    b = WL.batched_mixed(ninst=9, nmin=300, nmax=2500, order=9, seed=59, nsteps=9)
    sim = ase.BatchedSimulation(b, DEV, nbins=2)
    h = torch.zeros((1, b.ninst), dtype=torch.float64, device=DEV)
    sim.run(1, dt_hist=h)
    torch.cuda.synchronize()
    b.params.dt_cap = float(np.median(h.cpu().numpy()))
    p, w = _pair(b, b.nsteps, 500, wide_threads, nbins=2)
    _assert_same(p, w, "dt_cap")
    capped = np.isclose(p["dt_hist"], b.params.dt_cap, rtol=0, atol=0)
    assert capped.any() and not capped.all()


@pytest.mark.parametrize("plan_threads,call_threads", [(256, 256 | WS), (256 | WS, 256), (512, 256)])
def test_wide_plan_for_another_tile_length_is_skipped(plan_threads, call_threads):
    """A step call whose tile length differs from the plan's leaves the
    tiled instances as they were (no partial updates), while the binned
    instances advance as in the persistent launch."""
    b = WL.batched_mixed(ninst=9, nmin=16, nmax=2500, order=9, seed=53, nsteps=5)
    sim = ase.BatchedSimulation(b, DEV, nbins=2, wide_min_cells=600, wide_threads=plan_threads)
    tiled = sim.wide["inst_ntiles"].cpu().numpy() > 0
    assert tiled.any() and not tiled.all()
    U0 = sim.U.cpu().numpy().copy()
    sim.wide = dict(sim.wide, threads=call_threads)
    print(f"plan {plan_threads} call {call_threads} tiled {np.flatnonzero(tiled).tolist()}", flush=True)
    sim.run(b.nsteps)
    ref = ase.BatchedSimulation(b, DEV, nbins=2)
    ref.run(b.nsteps)
    out, exp = _outputs(sim), _outputs(ref)
    for k in range(b.ninst):
        o, n = int(b.offsets[k]), int(b.ncells[k])
        cells = slice(o + b.ng, o + b.ng + n)
        if tiled[k]:
            assert np.array_equal(out["U"][:, cells], U0[:, cells]) and out["t"][k] == 0.0, k
        else:
            assert np.array_equal(out["U"][:, cells], exp["U"][:, cells]) and out["t"][k] == exp["t"][k], k


def test_wide_full_size_against_the_oracle():
    """The 256-instance batch, 100 steps, instances of 768 cells and more in
    the wide form: the six largest instances the method keeps against the
    oracle run of each alone (1e-9 relative after the full run), and one
    step of every instance (1e-12; an instance whose first step already
    leaves the physical states must do so on both sides)."""
    from oracle import oracle as O

    def oracle_run(b, k, nsteps):
        g = WL.instance_grid(b, k)
        o, n = int(b.offsets[k]), int(b.ncells[k])
        U = np.ascontiguousarray(b.U[:, o:o + n + 2 * b.ng]).reshape(3, 1, n + 2 * b.ng).copy()
        sx, _ = O.sigma_init(g, b.params, U)
        O.step(g, b.params, U, sx, None, 0.0, nsteps, 0.0)
        return g, U

    def rel(a, c):
        den = np.maximum(np.abs(c).max(axis=-1), 1e-300)
        return float(np.max(np.abs(a - c).max(axis=-1) / den))

    for nsteps, tol, picks in ((1, 1e-12, None), (100, 1e-9, 6)):
        b = WL.batched_riemann(nsteps=nsteps)
        sim = ase.BatchedSimulation(b, DEV, nbins=64, wide_min_cells=768)
        st = torch.zeros(b.ninst, dtype=torch.int32, device=DEV)
        print(f"wide full size: {nsteps} steps, {sim.wide['nwide']} wide instances", flush=True)
        sim.run(nsteps, status=st)
        torch.cuda.synchronize()
        Ug, status = sim.U.cpu().numpy(), st.cpu().numpy()
        ks = range(b.ninst) if picks is None else \
            [int(k) for k in np.argsort(b.ncells)[::-1] if status[k] == 0][:picks]
        for k in ks:
            if status[k] != 0:
                continue
            g, Uo = oracle_run(b, k, nsteps)
            o, n = int(b.offsets[k]), int(b.ncells[k])
            a = Ug[:, o + b.ng:o + b.ng + n]
            c = g.interior(Uo)[:, 0]
            assert np.isfinite(a).all() == np.isfinite(c).all(), k
            if np.isfinite(c).all():
                assert rel(a, c) < tol, (k, nsteps)
            else:
                print(f"instance {k} ({n} cells) leaves the physical states in step 1 on both sides", flush=True)


@pytest.mark.parametrize("wide_threads", [256, 256 | WS])
def test_wide_calls_on_two_streams_at_once(wide_threads):
    """Two batches stepped in the wide form on two streams at the same time
    (each caller stream gets its own second stream from the library): each
    ends with the bits of its run alone on the default stream."""
    b1 = WL.batched_mixed(ninst=10, nmin=20, nmax=2500, order=9, seed=51, nsteps=20)
    b2 = WL.batched_riemann(ninst=12, nmin=300, nmax=3000, order=9, seed=52, nsteps=20)
    alone = []
    for b in (b1, b2):
        sim = ase.BatchedSimulation(b, DEV, nbins=3, wide_min_cells=600, wide_threads=wide_threads)
        sim.run(b.nsteps)
        alone.append(_outputs(sim))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    sims = [ase.BatchedSimulation(b, DEV, nbins=3, wide_min_cells=600, wide_threads=wide_threads) for b in (b1, b2)]
    torch.cuda.synchronize()
    for _ in range(4):   # interleaved calls of 5 steps each
        for sim, st in zip(sims, (s1, s2)):
            with torch.cuda.stream(st):
                sim.run(5, stream=st)
    torch.cuda.synchronize()
    for sim, ref in zip(sims, alone):
        _assert_same(ref, _outputs(sim), "two streams")
