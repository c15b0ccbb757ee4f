"""Host-side logic without a GPU: the longest-first packing of batched
instances into bins (ase_batched_plan) and the launch-shape autotuner's
choice and cache (with the timing function replaced)."""
import ctypes as C
import json

import numpy as np
import pytest

from paper_2410_05489_amd import ase
from paper_2410_05489_amd import autotune
from paper_2410_05489_amd import workloads as WL


@pytest.mark.parametrize("ninst,nbins,seed", [(256, 256, 0), (256, 128, 1), (100, 7, 2), (5, 8, 3), (1, 1, 4)])
def test_batched_plan_is_a_longest_first_packing(ninst, nbins, seed):
    rng = np.random.default_rng(seed)
    nc = rng.integers(64, 4097, size=ninst).astype(np.int32)
    start, lst = ase.batched_plan(nc, nbins)
    # every instance exactly once, bins contiguous in the list
    assert start[0] == 0 and start[-1] == ninst and np.all(np.diff(start) >= 0)
    assert sorted(lst.tolist()) == list(range(ninst))
    loads = np.array([nc[lst[start[b]:start[b + 1]]].sum() for b in range(nbins)])
    # greedy longest-first onto the least-loaded bin: no bin exceeds the
    # lightest by more than its own smallest instance (else that instance
    # would have gone to the lightest bin), and the bound of the method
    for b in range(nbins):
        members = nc[lst[start[b]:start[b + 1]]]
        if len(members):
            assert loads[b] - members.min() <= loads.min()
    assert loads.max() <= max(nc.max(), 4.0 / 3.0 * nc.sum() / nbins + nc.max())
    # within a bin, instances are walked longest first
    for b in range(nbins):
        members = nc[lst[start[b]:start[b + 1]]]
        assert np.all(np.diff(members) <= 0)


def test_autotuner_picks_the_fastest_shape_and_caches_it(tmp_path, monkeypatch):
    monkeypatch.setenv("ASE_TUNE_CACHE", str(tmp_path / "tune.json"))
    b = WL.batched_riemann(ninst=12, nmin=16, nmax=200, nsteps=3)
    times = {(128, 512): 3.0, (256, 256): 2.5, (256, 512): 1.75, (512, 512): 2.0, (128, 1024): 9.0,
             (256, 1024): 1.9}
    calls = []

    def fake_time(batch, nbins, threads, nsteps, device="cuda", min_cells=0, wide_threads=256):
        calls.append((nbins, threads, min_cells))
        # the wide splits (bins capped at the instance count) are all slower here
        return times[(nbins, threads)] if min_cells == 0 else 5.0 + min_cells / 1e4

    monkeypatch.setattr(autotune, "time_batched", fake_time)
    best = autotune.tune_batched(b, nsteps=4)
    assert (best["nbins"], best["threads"], best["min_cells"]) == (256, 512, 0) and best["ms"] == 1.75
    assert sorted(c[:2] for c in calls if c[2] == 0) == sorted(times)
    # first-order DF source: the wide splits were timed as well, bins capped
    wide = [c for c in calls if c[2] > 0]
    assert len(wide) == len(autotune.WIDE_CANDIDATES) and all(c[0] <= b.ninst for c in wide)
    stored = json.load(open(tmp_path / "tune.json"))
    assert stored[autotune.batched_key(b)]["threads"] == 512

    def no_timing(*a, **k):
        raise AssertionError("a cached shape is not timed again")

    monkeypatch.setattr(autotune, "time_batched", no_timing)
    again = autotune.tune_batched(b, nsteps=4)
    assert (again["nbins"], again["threads"]) == (256, 512)
    # a wide split that wins is what the tuner hands back
    monkeypatch.setattr(autotune, "time_batched",
                        lambda batch, nbins, threads, nsteps, device="cuda", min_cells=0, wide_threads=256:
                        1.0 if (min_cells, wide_threads) == (1024, 512) else 2.0)
    w = autotune.tune_batched(b, nsteps=4, use_cache=False)
    assert (w["min_cells"], w["wide_threads"], w["ms"]) == (1024, 512, 1.0)
    # the Gauss-point DF source has no wide form
    b.params.df_source = 0
    g = autotune.tune_batched(b, nsteps=4, use_cache=False)
    assert all(t["min_cells"] == 0 for t in g["trials"])
    # a different batch shape is a different key
    b2 = WL.batched_riemann(ninst=13, nmin=16, nmax=200, nsteps=3)
    assert autotune.batched_key(b2) != autotune.batched_key(b)


def test_batched_plan_rejects_bad_arguments():
    L = ase.lib()
    nc = (C.c_int32 * 3)(10, 20, 30)
    start = (C.c_int32 * 4)()
    lst = (C.c_int32 * 3)()
    assert L.ase_batched_plan(3, None, 3, start, lst) == -1
    assert L.ase_batched_plan(3, nc, 3, None, lst) == -1
    assert L.ase_batched_plan(-1, nc, 3, start, lst) == -1


def test_traffic_fingerprint_follows_only_the_sweep_sources(tmp_path, monkeypatch):
    """bench.py reports the measured sweep traffic only while the sources the
    sweep kernel compiles from are unchanged: edits elsewhere in the kernel
    file leave the fingerprint alone, edits to the sweep or to the device
    helpers change it."""
    import os
    import shutil

    import bench

    src = os.path.join(bench.ROOT, "paper_2410_05489_amd", "csrc")
    csrc = tmp_path / "paper_2410_05489_amd" / "csrc"
    shutil.copytree(src, csrc)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    f0 = bench.kernel_fingerprint()
    k = csrc / "ase_kernels.hip"
    text = k.read_text()
    k.write_text(text.replace("k_fill_fo(BCInfo b,", "k_fill_fo(BCInfo  b,", 1))
    assert bench.kernel_fingerprint() == f0
    k.write_text(text.replace("k_sweep2d(SweepArgs a)\n{", "k_sweep2d(SweepArgs a)\n{ ", 1))
    assert bench.kernel_fingerprint() != f0
    k.write_text(text)
    d = csrc / "ase_device.h"
    d.write_text(d.read_text() + "\n")
    assert bench.kernel_fingerprint() != f0
