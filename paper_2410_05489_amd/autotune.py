"""Launch-shape autotuner for the batched kernels.

Times ase_step_batched (and ase_adjoint_batched) for a few (bins, threads)
shapes on the current GPU, and with the first-order DF source the wide form
(ase_step_batched_wide) for a few (bins, threads, min_cells, wide threads)
splits, and keeps the fastest in a JSON cache keyed by (arch, kernel, order,
instance-count, stored-cell total).  Results do not depend on the shape
(every instance is advanced by the same per-cell arithmetic), only the time
does.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional, Sequence, Tuple

import torch

from . import ase

DEFAULT_CANDIDATES: Sequence[Tuple[int, int]] = ((128, 512), (256, 256), (256, 512), (512, 512), (128, 1024),
                                                  (256, 1024))


# (bins, threads, min_cells, wide_threads) of the wide form
# (wide_threads with ase.WIDE_STEP: one launch per step)
WIDE_CANDIDATES: Sequence[Tuple[int, int, int, int]] = ((128, 256, 768, 256), (64, 256, 768, 256),
                                                        (128, 512, 1024, 256), (256, 512, 1024, 256),
                                                        (128, 512, 1536, 256), (128, 512, 1024, 512),
                                                        (64, 256, 768, 256 | ase.WIDE_STEP),
                                                        (64, 256, 896, 256 | ase.WIDE_STEP),
                                                        (128, 512, 1024, 256 | ase.WIDE_STEP))


def cache_path() -> str:
    return os.environ.get("ASE_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ase_mi355x",
                                                         "tune.json"))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # noqa: BLE001
        return "unknown"


def batched_key(batch) -> str:
    # the version field changes with the candidate forms (3: the per-step
    # wide form), so that a cache tuned without them is not reused
    return f"{_arch()}/batched3/r{batch.params.order}/n{batch.ninst}/c{batch.total}/s{batch.params.df_source}"


def _load() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: Dict[str, dict]) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_batched(batch, nbins: int, threads: int, nsteps: int, device="cuda", min_cells: int = 0,
                 wide_threads: int = 256) -> float:
    """Milliseconds for nsteps steps of the whole batch in one call
    (min_cells > 0: the wide form)."""
    sim = ase.BatchedSimulation(batch, device, nbins=nbins, threads=threads, wide_min_cells=min_cells,
                                wide_threads=wide_threads)
    sim.run(1)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    sim.run(nsteps)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop)


def tune_batched(batch, nsteps: int = 10, candidates: Optional[Sequence[Tuple[int, int]]] = None,
                 use_cache: bool = True, wide: Optional[bool] = None,
                 wide_candidates: Optional[Sequence[Tuple[int, int, int, int]]] = None) -> dict:
    """Best {'nbins', 'threads', 'min_cells', 'wide_threads', 'ms'} for this
    batch shape (cached); min_cells 0 is the persistent launch alone.  wide
    (default: with the first-order DF source) adds the wide-form splits."""
    key = batched_key(batch)
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        return cache[key]
    if wide is None:
        wide = batch.params.df_source == 1
    trials = []
    for nbins, threads in (candidates or DEFAULT_CANDIDATES):
        ms = time_batched(batch, nbins, threads, nsteps)
        trials.append({"nbins": nbins, "threads": threads, "min_cells": 0, "wide_threads": 0, "ms": ms})
    if wide:
        for nbins, threads, mc, wt in (wide_candidates or WIDE_CANDIDATES):
            nb = min(nbins, batch.ninst)
            ms = time_batched(batch, nb, threads, nsteps, min_cells=mc, wide_threads=wt)
            trials.append({"nbins": nb, "threads": threads, "min_cells": mc, "wide_threads": wt, "ms": ms})
    best = min(trials, key=lambda r: r["ms"])
    best = dict(best, steps=nsteps, trials=trials)
    if use_cache:
        cache[key] = best
        _store(cache)
    return best


ADJOINT_CANDIDATES: Sequence[Tuple[int, int]] = ((256, 256), (256, 512), (512, 256), (512, 512), (1024, 256))
# (min_cells, wide_threads) of the wide reverse sweep, beside the best
# persistent shape
ADJOINT_WIDE_CANDIDATES: Sequence[Tuple[int, int]] = ((400, 256), (768, 256), (1536, 256))


def tune_adjoint(batch, every: int = 10, candidates: Optional[Sequence[Tuple[int, int]]] = None,
                 use_cache: bool = True, fwd_shape: Tuple[int, int] = (256, 256),
                 wide_candidates: Optional[Sequence[Tuple[int, int]]] = None) -> dict:
    """Best {'nbins', 'threads', 'min_cells', 'wide_threads', 'ms'} for one
    adjoint segment of `every` steps of this batch (cached): the persistent
    shapes, then (first-order DF source) the wide reverse sweep beside the
    best of them; min_cells 0 is the persistent sweep alone.  The time is
    that of the reverse phase while the next tape phase runs on a second
    stream, as in the autograd backward, whose length the reverse phases
    set ('tape_ms': the tape phase alone)."""
    key = f"{_arch()}/adjoint2/r{batch.params.order}/n{batch.ninst}/c{batch.total}/s{every}"
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        return cache[key]
    sim = ase.BatchedSimulation(batch, "cuda", nbins=fwd_shape[0], threads=fwd_shape[1])
    U0, s0 = sim.U.clone(), sim.sig.clone()
    hist = torch.zeros((every, batch.ninst), dtype=torch.float64, device="cuda")
    sim.run(every, dt_hist=hist)
    ws = ase.Workspace(ase.adjoint_batched_workspace_bytes(batch.total, every))
    lam = torch.ones((3, batch.total), dtype=torch.float64, device="cuda")
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    mid = torch.cuda.Event(enable_timing=True)
    ws2 = ase.Workspace(ws.nbytes)
    side = torch.cuda.Stream()

    def timed(call):
        """(tape ms, reverse ms beside a tape into the other workspace) of
        the second of two rounds; call(ws, phase, stream)."""
        for rep in range(2):
            start.record()
            call(ws, ase.ADJ_TAPE, None)
            mid.record()
            side.wait_event(mid)
            with torch.cuda.stream(side):
                call(ws2, ase.ADJ_TAPE, side)
            call(ws, ase.ADJ_REVERSE, None)
            stop.record()
            torch.cuda.synchronize()
        return start.elapsed_time(mid), mid.elapsed_time(stop)

    trials = []
    for nbins, threads in (candidates or ADJOINT_CANDIDATES):
        plan = ase.device_plan(batch.ncells, nbins)
        tt, tr = timed(lambda w, ph, stm: ase.adjoint_batched(sim, U0, s0, hist, every, lam, w, threads, plan,
                                                              stream=stm, phase=ph))
        trials.append({"nbins": nbins, "threads": threads, "min_cells": 0, "wide_threads": 0, "ms": tr,
                       "tape_ms": tt})
    if batch.params.df_source == 1:
        pb = min(trials, key=lambda r: r["ms"])
        for mc, wt in (wide_candidates or ADJOINT_WIDE_CANDIDATES):
            wplan = ase.wide_plan_device(batch.ncells, mc, batch.params.order, wt, pb["nbins"])
            tt, tr = timed(lambda w, ph, stm: ase.adjoint_batched_wide(sim, U0, s0, hist, every, lam, w,
                                                                       pb["threads"], wplan, stream=stm, phase=ph))
            trials.append({"nbins": pb["nbins"], "threads": pb["threads"], "min_cells": mc, "wide_threads": wt,
                           "ms": tr, "tape_ms": tt})
    best = min(trials, key=lambda r: r["ms"])
    best = dict(best, steps=every, trials=trials)
    if use_cache:
        cache[key] = best
        _store(cache)
    return best
