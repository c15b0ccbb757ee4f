"""Reverse mode of the 1D ASE-DF step as torch.autograd.Functions.

Forward runs keep checkpoints (state and DF strengths) every `every` steps
and the device record of every time step; backward walks the segments last
to first and calls the adjoint entry points of libase, which recompute each
segment from its checkpoint.  The frozen decisions (time step, strengths,
LF side, positivity replacements) are those stated with ase_adjoint_step in
include/ase.h.  Objective: J = dx sum p over the interior of each grid.
"""
from __future__ import annotations

import math

import torch

from . import ase


class _BatchedRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, runner, nsteps):
        sim, b, every = runner.sim, runner.sim.b, runner.every
        sim.U.copy_(U0)
        sim.t.zero_()
        runner.init_sigma()
        nseg = max(1, math.ceil(nsteps / every))
        ckU = torch.empty((nseg, 3, b.total), dtype=torch.float64, device=sim.U.device)
        ckS = torch.empty((nseg, b.total), dtype=torch.float64, device=sim.U.device)
        hist = torch.zeros((max(nsteps, 1), b.ninst), dtype=torch.float64, device=sim.U.device)
        for s in range(nseg):
            n = min(every, nsteps - s * every)
            ckU[s].copy_(sim.U)
            ckS[s].copy_(sim.sig)
            if n > 0:
                sim.run(n, dt_hist=hist[s * every:s * every + n])
        ctx.runner, ctx.nsteps = runner, nsteps
        ctx.save_for_backward(ckU, ckS, hist)
        runner.dt_hist = hist
        return sim.U.clone()

    @staticmethod
    def backward(ctx, gU):
        runner, nsteps = ctx.runner, ctx.nsteps
        ckU, ckS, hist = ctx.saved_tensors
        every = runner.every
        lam = gU.contiguous().clone()
        segs = [s for s in reversed(range(ckU.shape[0])) if min(every, nsteps - s * every) > 0]

        def call(s, ws, phase, stream=None):
            n = min(every, nsteps - s * every)
            h = hist[s * every:s * every + n]
            if runner.wide_plan is None:
                ase.adjoint_batched(runner.sim, ckU[s], ckS[s], h, n, lam, ws, runner.adj_threads, runner.adj_plan,
                                    stream=stream, phase=phase)
                return
            ase.adjoint_batched_wide(runner.sim, ckU[s], ckS[s], h, n, lam, ws, runner.adj_threads,
                                     runner.wide_plan, stream=stream, phase=phase)

        if not runner.overlap or len(segs) < 2:
            for s in segs:
                call(s, runner.ws_adj, ase.ADJ_TAPE | ase.ADJ_REVERSE)
            return lam, None, None
        # The recomputation of a segment needs only its checkpoint, not the
        # adjoint: it runs on a side stream into the other workspace while
        # the main stream runs the previous segment back.
        main = torch.cuda.current_stream()
        side = runner.side_stream()
        ws = (runner.ws_adj, runner.ws_adj_other())
        side.wait_stream(main)
        call(segs[0], ws[0], ase.ADJ_TAPE)
        tape_done, rev_done = {}, {}
        for i, s in enumerate(segs):
            if i + 1 < len(segs):
                with torch.cuda.stream(side):
                    if i >= 1:
                        side.wait_event(rev_done[i - 1])   # its workspace held segment i-1's tape
                    call(segs[i + 1], ws[(i + 1) % 2], ase.ADJ_TAPE, stream=side)
                    tape_done[i + 1] = torch.cuda.Event()
                    tape_done[i + 1].record(side)
            if i >= 1:
                main.wait_event(tape_done[i])
            call(s, ws[i % 2], ase.ADJ_REVERSE, stream=main)
            rev_done[i] = torch.cuda.Event()
            rev_done[i].record(main)
        main.wait_stream(side)
        return lam, None, None


class _Pressure(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, tables):
        p, offsets, ncells, dx, ng, total = tables
        J = torch.zeros(ncells.numel(), dtype=torch.float64, device=U.device)
        ase.pressure_objective(p, offsets, ncells, dx, ng, total, U.contiguous(), J=J)
        ctx.tables = tables
        ctx.save_for_backward(U)
        return J

    @staticmethod
    def backward(ctx, gJ):
        (U,) = ctx.saved_tensors
        p, offsets, ncells, dx, ng, total = ctx.tables
        lam = torch.empty((3, total), dtype=torch.float64, device=U.device)
        ase.pressure_objective(p, offsets, ncells, dx, ng, total, U.contiguous(), lam=lam,
                               weights=gJ.contiguous())
        return lam.view_as(U), None


class BatchedAdjoint:
    """Differentiable runs of a batch of 1D instances (workloads.Batch):
    U_N = run(U0, nsteps) and J = pressure(U_N) are autograd-aware, so
    J.sum().backward() gives dJ/dU0 through the adjoint kernels."""

    def __init__(self, batch, device="cuda", nbins: int = 0, threads: int = 256, adj_threads: int = 256,
                 every: int = 10, adj_nbins: int = 0, overlap: bool = True, wide_min_cells: int = 0,
                 wide_threads: int = 256, adj_wide_min_cells: int = 0, adj_wide_threads: int = 256):
        """wide_min_cells / wide_threads: the forward's wide form (as
        BatchedSimulation); adj_wide_min_cells / adj_wide_threads: the reverse
        sweep's (ase_adjoint_batched_wide; 0: the persistent launch only)."""
        self.sim = ase.BatchedSimulation(batch, device, nbins=nbins, threads=threads, wide_min_cells=wide_min_cells,
                                         wide_threads=wide_threads)
        self.every = int(every)
        self.adj_threads = int(adj_threads)
        self.adj_plan = ase.device_plan(batch.ncells, adj_nbins, device) if adj_nbins else None
        self.wide_plan = None
        if adj_wide_min_cells > 0:
            self.wide_plan = ase.wide_plan_device(batch.ncells, adj_wide_min_cells, batch.params.order,
                                                  adj_wide_threads, adj_nbins or self.sim.nbins, device)
        self.ws_adj = ase.Workspace(ase.adjoint_batched_workspace_bytes(batch.total, self.every), device)
        self.device = device
        self.overlap = overlap          # recompute segment s-1 while running segment s back
        self._ws2 = None
        self._side = None
        self.dt_hist = None

    def ws_adj_other(self):
        """The second tape workspace of the overlapped backward."""
        if self._ws2 is None:
            self._ws2 = ase.Workspace(self.ws_adj.nbytes, self.device)
        return self._ws2

    def side_stream(self):
        """The stream the recomputations run on (default priority)."""
        if self._side is None:
            self._side = torch.cuda.Stream(device=self.device)
        return self._side

    def init_sigma(self):
        self.sim.sigma_init()

    def run(self, U0: torch.Tensor, nsteps: int) -> torch.Tensor:
        return _BatchedRun.apply(U0, self, int(nsteps))

    def pressure(self, U: torch.Tensor) -> torch.Tensor:
        b, s = self.sim.b, self.sim
        return _Pressure.apply(U, (s.p, s.offsets, s.ncells, s.dx, b.ng, b.total))


class _Run1D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, runner, nsteps):
        sim, every = runner.sim, runner.every
        sim.U.copy_(U0)
        sim.t.zero_()
        ase.sigma_init(sim.g, sim.p, sim.U, sim.sx, sim.sy)
        nseg = max(1, math.ceil(nsteps / every))
        cks = []
        hist = torch.zeros(max(nsteps, 1), dtype=torch.float64, device=sim.U.device)
        for s in range(nseg):
            n = min(every, nsteps - s * every)
            cks.append((sim.U.clone(), sim.sx.clone()))
            if n > 0:
                sim.run(n, dt_hist=hist[s * every:s * every + n])
        ctx.runner, ctx.nsteps, ctx.cks = runner, nsteps, cks
        ctx.save_for_backward(hist)
        return sim.U.clone()

    @staticmethod
    def backward(ctx, gU):
        runner, nsteps, cks = ctx.runner, ctx.nsteps, ctx.cks
        (hist,) = ctx.saved_tensors
        g, p, every = runner.sim.g, runner.sim.p, runner.every
        lam = gU.contiguous().clone()
        rs = runner.replay
        for s in reversed(range(len(cks))):
            n = min(every, nsteps - s * every)
            if n <= 0:
                continue
            # recompute the states the steps of this segment start from
            rs.U.copy_(cks[s][0])
            rs.sx.copy_(cks[s][1])
            tape = []
            for q in range(n):
                tape.append((rs.U.clone(), rs.sx.clone()))
                if q + 1 < n:
                    rs.run(1)
            for q in reversed(range(n)):
                Uq, sq = tape[q]
                i = s * every + q
                ase.adjoint_step(g, p, Uq, sq, hist[i:i + 1], lam, lam, runner.ws_adj)
        return lam, None, None


class Adjoint1D:
    """Differentiable runs of one 1D grid (ase_step forward, ase_adjoint_step
    backward, checkpoints every `every` steps)."""

    def __init__(self, g, p, device="cuda", every: int = 10):
        import numpy as np
        if g.dim != 1:
            raise ase.AseError("Adjoint1D: 1D grid expected")
        zero = np.zeros((3, 1, g.ld))
        self.sim = ase.Simulation(g, p, zero, device=device)
        self.replay = ase.Simulation(g, p, zero, device=device)
        self.every = int(every)
        self.ws_adj = ase.Workspace(ase.adjoint_workspace_bytes(g), device)
        self.tables = (p, torch.zeros(1, dtype=torch.int64, device=device),
                       torch.full((1,), g.nx, dtype=torch.int32, device=device),
                       torch.full((1,), g.dx, dtype=torch.float64, device=device), g.ng, g.ld)

    def run(self, U0: torch.Tensor, nsteps: int) -> torch.Tensor:
        return _Run1D.apply(U0, self, int(nsteps))

    def pressure(self, U: torch.Tensor) -> torch.Tensor:
        return _Pressure.apply(U, self.tables)
