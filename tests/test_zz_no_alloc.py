"""The allocation-free batched entry point (ase_step_batched_noalloc, the
library's fixed device scratch) against ase_step_batched with a caller
workspace: two calls in a row on different batches, the second smaller,
must give the same states, strengths, times and time steps bit for bit."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2410_05489_amd import ase
from paper_2410_05489_amd import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda"
ERR_WORKSPACE = -6
SCRATCH_BYTES = 64 << 20


def _run(batch, noalloc, nsteps, nbins, threads, t_end=0.0):
    sim = ase.BatchedSimulation(batch, DEV, nbins=nbins, threads=threads)
    hist = torch.zeros((nsteps, batch.ninst), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    sim.run(nsteps, t_end, hist, noalloc=noalloc)
    torch.cuda.synchronize()
    return [sim.U.cpu().numpy(), sim.sig.cpu().numpy(), sim.t.cpu().numpy(), hist.cpu().numpy()]


def _same(a, b):
    # bit for bit, a NaN (an instance the method loses) equal to a NaN
    return a.shape == b.shape and np.array_equal(a.view(np.int64), b.view(np.int64))


def test_noalloc_equals_workspace_entry_point_two_calls():
    big = WL.batched_riemann(ninst=48, nmin=64, nmax=4096, order=9, seed=11, nsteps=12)
    small = WL.batched_riemann(ninst=7, nmin=10, nmax=300, order=5, seed=12, nsteps=9)
    assert small.total < big.total
    assert int(ase.lib().ase_batched_workspace_bytes(big.total)) <= SCRATCH_BYTES
    for batch, nbins, threads in ((big, 24, 512), (small, 3, 256)):
        print(f"noalloc: {batch.ninst} instances, {batch.total} stored cells, order {batch.params.order}", flush=True)
        ref = _run(batch, False, batch.nsteps, nbins, threads)
        got = _run(batch, True, batch.nsteps, nbins, threads)
        for name, a, b in zip(("U", "sigma", "t", "dt"), ref, got):
            assert _same(a, b), name
        # every instance advanced, or is one the method loses (NaN time)
        assert np.all((ref[2] > 0.0) | np.isnan(ref[2])) and np.mean(ref[2] > 0.0) > 0.5


def test_noalloc_stops_at_t_end_like_workspace_entry_point():
    b = WL.batched_smooth(ninst=9, nmin=12, nmax=200, order=7, seed=4, nsteps=40)
    print(f"noalloc t_end: {b.ninst} instances, {b.total} stored cells", flush=True)
    ref = _run(b, False, b.nsteps, 4, 256, t_end=0.05)
    got = _run(b, True, b.nsteps, 4, 256, t_end=0.05)
    for name, x, y in zip(("U", "sigma", "t", "dt"), ref, got):
        assert _same(x, y), name


def test_noalloc_refuses_batches_beyond_the_scratch():
    b = WL.batched_riemann(ninst=4, nmin=20, nmax=60, order=9, seed=1, nsteps=2)
    sim = ase.BatchedSimulation(b, DEV, nbins=2, threads=256)
    torch.cuda.synchronize()
    too_big = 1198369   # first stored-cell count whose workspace exceeds the scratch
    assert int(ase.lib().ase_batched_workspace_bytes(too_big)) > SCRATCH_BYTES
    assert int(ase.lib().ase_batched_workspace_bytes(too_big - 1)) <= SCRATCH_BYTES
    rc = ase.lib().ase_step_batched_noalloc(
        C.byref(ase.c_params(b.params)), b.bc, None, b.ninst, sim.offsets.data_ptr(), sim.ncells.data_ptr(),
        sim.dx.data_ptr(), b.ng, too_big, sim.U.data_ptr(), sim.sig.data_ptr(), sim.t.data_ptr(), None, None, None,
        2, 0.0,
        sim.bin_start.data_ptr(), sim.bin_list.data_ptr(), sim.nbins, sim.threads,
        torch.cuda.current_stream().cuda_stream)
    assert rc == ERR_WORKSPACE
    assert b"scratch" in ase.lib().ase_last_error()
    # nothing was launched: the state is untouched
    torch.cuda.synchronize()
    assert float(sim.t.abs().max()) == 0.0
