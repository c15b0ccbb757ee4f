#!/usr/bin/env python3
"""Throughput of the 9th-order 2D ASE-DF step on one MI355X.

Workload (default): 2D four-quadrant Riemann problem, 1024 x 1024 cells on
[0,1]^2, order 9, gamma 1.4, CFL 0.4, transmissive boundaries, quadrant
states drawn with seed 0 (rho in [0.1,1.5], |u|,|v| <= 1.2, p in [0.03,1.5]).
A step is one full SSP-RK3 step of the whole grid (boundary fill, dt, three
stages of reconstruction, DF strengths, LF flux and update) with the state
resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 200] [--warmup 10] [--workload quad1024]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s, 9th-order 2D ASE step (FP64) + % HBM roofline; adjoint/fwd ratio"

# HBM bytes per launch of the two sweep kernels on the default workload, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB device copy (summary in
# profiles/k_sweep2d_quad1024_r9.md, 1024^2 and 4096^2).  Valid only for the sweep kernel sources
# with this fingerprint (kernel_fingerprint); once they change the bench reports traffic as null.
MEASURED_TRAFFIC = {"fingerprint": "5e5b813e0774b09c", "workloads": ("quad1024", "quad4096"),
                    "quad1024": {"sweep_x": 88022912, "sweep_y": 156486528},
                    "quad4096": {"sweep_x": 1751501024, "sweep_y": 2908951552}}
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz


def kernel_fingerprint() -> str:
    """Hash of what the two sweep kernels compile from: the device helpers,
    the sweep arguments, the text of the sweep kernel itself and the
    compiler flags (the other kernels of the library do not enter)."""
    from paper_2410_05489_amd import build as B
    csrc = os.path.join(ROOT, "paper_2410_05489_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "ase_device.h"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(csrc, "ase_host.h")) as fh:
        host = fh.read()
    i = host.index("enum SweepMode")
    h.update(host[i:host.index("};", host.index("struct SweepArgs")) + 2].encode())
    with open(os.path.join(csrc, "ase_kernels.hip")) as fh:
        k = fh.read()
    i = k.index("// 2D sweep: one tile of T0 x T1 cells")
    h.update(k[i:k.index("\n}\n", k.index("k_sweep2d(SweepArgs a)")) + 3].encode())
    h.update(" ".join(B.HIP_FLAGS).encode())
    return h.hexdigest()[:16]


def alg_flops_per_cell_sweep(order: int, dim: int, lagged: bool = False) -> float:
    """Algorithmic FP64 operations per interior cell for one direction of one
    stage on the top linear branch (every operation of the method counted once;
    an FMA counts 2, a divide or square root 1).

    2D, r = 2R+1, G = R Gauss points:
      normal reconstruction   : DF sums (r-2 + ... adds) + 2 points x 4 vars x (2r-1)
      tangential (two sides)  : 2 x (DF sums + G points x 4 vars x (2r-1))
      per Gauss point         : primitives 2 x 12, LF flux 33, quadrature 8 -> 65;
                                lagged DF source: + strength 14 and its sum 1
      face strength mean      : 1 (lagged DF source)
      flux difference         : 4 vars x 2
    With the first-order DF source the strengths are the cell-average ones,
    formed outside the sweeps (per cell one set of primitives and the
    strengths of its two faces).  The count is the method's direct form: the
    kernels evaluate the linear levels at three or four Gauss points in mirror
    pairs (r = 9: 44 instead of 68 operations per variable and side), so they
    execute fewer operations than counted here for the tangential part.
    """
    R = (order - 1) // 2
    sums = {1: 1, 2: 3, 3: 8, 4: 15}[R]
    if dim == 1:
        normal = sums + 2 * 3 * (2 * order - 1)
        point = 2 * 9 + 9 + 26
        return normal + point + 3 * 2
    G = R
    normal = sums + 2 * 4 * (2 * order - 1)
    tang = 2 * (sums + G * 4 * (2 * order - 1))
    return normal + tang + G * (80 if lagged else 65) + (1 if lagged else 0) + 8


def alg_bytes_per_cell(kernel: str, lagged: bool = False) -> float:
    """Algorithmic HBM bytes per interior cell of one launch (FP64 words):
    x sweep reads the stage state (4) and both strength planes (2), writes the
    x residual (4); y sweep reads the stage state (4), both strength planes
    (2), the x residual (4) and the step-start state (4, stages 2-3), writes
    the stage output (4).  Lagged DF source: each sweep also writes its new
    strengths (1)."""
    w = 1 if lagged else 0
    return {"sweep_x": (10 + w) * 8.0, "sweep_y": ((18 + w) * 8.0 * 2 + (14 + w) * 8.0) / 3.0}[kernel]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads the oracle may use: OMP_NUM_THREADS when set, else the CPUs
    this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def make_workload(name):
    from paper_2410_05489_amd import workloads as WL
    if name == "quad1024":
        return WL.four_quadrant(1024, 9, seed=0, nsteps=200)
    if name == "quad4096":
        return WL.four_quadrant(4096, 9, seed=0, nsteps=200)
    if name == "jet":
        return WL.jet(1600, 800, 7, nsteps=500)
    if name == "dmr":
        return WL.double_mach(960, 240, 9, nsteps=200)
    raise SystemExit(f"unknown workload {name}")


def bench_batched(args):
    """Batched 1D form: 256 instances (64..4096 cells), r = 9: the persistent
    launch, with the large instances in the wide form when that is faster
    (autotuned), against per-instance ase_step launches."""
    import torch
    from paper_2410_05489_amd import ase, autotune
    from paper_2410_05489_amd import workloads as WL

    b = WL.batched_riemann(nsteps=args.steps)
    if args.batched_shape:
        # a fixed launch shape (profiling runs): no autotuner trials
        nb, th, mc, wt = (int(x) for x in args.batched_shape.split(":"))
        best = {"nbins": nb, "threads": th, "min_cells": mc, "wide_threads": wt, "ms": None,
                "trials": [{"nbins": 256, "threads": 1024, "min_cells": 0, "wide_threads": 0, "ms": None}]}
    else:
        best = autotune.tune_batched(b, nsteps=10, use_cache=False)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    def timed(sim, prof):
        sim.run(args.warmup)
        torch.cuda.synchronize()
        ase.profile_enable(prof)
        start.record()
        sim.run(args.steps)
        stop.record()
        torch.cuda.synchronize()
        k = ase.profile_read("batched")
        ase.profile_enable(False)
        return start.elapsed_time(stop), k

    sim = ase.BatchedSimulation(b, "cuda", nbins=best["nbins"], threads=best["threads"],
                                wide_min_cells=best["min_cells"], wide_threads=best["wide_threads"] or 256)
    ms, (kms, kn) = timed(sim, True)
    cells = int(b.ncells.sum())
    value = cells * args.steps / (ms / 1e3) / 1e6
    # the fastest persistent launch alone, for comparison
    pbest = min((t for t in best["trials"] if t["min_cells"] == 0), key=lambda t: t["ms"] or 0.0)
    ms_p, _ = timed(ase.BatchedSimulation(b, "cuda", nbins=pbest["nbins"], threads=pbest["threads"]), False)
    value_p = cells * args.steps / (ms_p / 1e3) / 1e6
    # per-instance launches of the same 1D method (ase_step per instance)
    sims = []
    for k in range(b.ninst):
        g = WL.instance_grid(b, k)
        o = int(b.offsets[k])
        sims.append(ase.Simulation(g, b.params, b.U[:, o:o + g.NX].reshape(3, 1, g.NX), device="cuda"))
    pi_steps = max(1, args.steps // 10)
    for s1 in sims:
        s1.run(1)
    torch.cuda.synchronize()
    start.record()
    for s1 in sims:
        s1.run(pi_steps)
    stop.record()
    torch.cuda.synchronize()
    ms_pi = start.elapsed_time(stop)
    value_pi = cells * pi_steps / (ms_pi / 1e3) / 1e6
    flops = alg_flops_per_cell_sweep(b.params.order, 1) * 3 + 3 * 4
    achieved = flops * cells * args.steps / (kms / 1e3) / 1e12
    wide = best["min_cells"] > 0
    out = {"metric": "Mcell-updates/s, batched 1D order-9 instances", "value": round(value, 2),
           "unit": "Mcell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms / args.steps, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"batched_riemann_{b.ninst}x64..4096_r9_seed0", "ninst": b.ninst, "cells": cells,
                      "form": "persistent + wide" if wide else "persistent",
                      "nbins": best["nbins"], "threads": best["threads"], "wide_min_cells": best["min_cells"],
                      "wide_threads": best["wide_threads"],
                      "wide_instances": sim.wide["nwide"] if wide else 0,
                      "wide_tiles": sim.wide["ntiles"] if wide else 0},
           "persistent_only": {"value": round(value_p, 2), "ms": round(ms_p, 3), "nbins": pbest["nbins"],
                               "threads": pbest["threads"]},
           "per_instance_launches": {"value": round(value_pi, 2), "steps": pi_steps, "ms": round(ms_pi, 3)},
           "speedup_vs_per_instance": round(value / value_pi, 2),
           "autotune": best["trials"],
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VALU_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4), "traffic": None,
                        "kernel": "k_batched1d + k_batched_wide" if wide else "k_batched1d",
                        "avg_call_ms": round(kms / max(kn, 1), 4)}}
    print(json.dumps(out), flush=True)


def alg_flops_per_cell_gks_stage(order: int) -> float:
    """Algorithmic FP64 operations per cell of one S2O4 stage of the 1D
    gas-kinetic path (FMA = 2; divide, square root, exp and erfc = 1 each):
      reconstruction      : DF sums + 2 faces x 3 vars x (2r-1) for values
                            and again for slopes
      strength            : primitives of both sides 2 x 12, strength 14
      kinetic face flux   : three Maxwellians 21, whole-line moments to
                            <u^6> 3 x 21, half-line moments 2 x 37, xi
                            moments 18, micro slopes and time slopes 3 x 70,
                            kinetic averages W^c, W^c_x 138, nine moment
                            terms 9 x 30, tau_n 10, two time integrals
                            2 x 83, F and F_t 22                -> 992
      update              : L, L_t and the stage combination    -> 30
    """
    R = (order - 1) // 2
    sums = {1: 1, 2: 3, 3: 8, 4: 15}[R]
    recon = sums + 2 * 2 * 3 * (2 * order - 1)
    return recon + 2 * 12 + 14 + 992 + 30


def bench_gks(args):
    """1D gas-kinetic solver (S2O4 steps): Shu-Osher-type data on 2^20
    cells, order 9, one grid resident in HBM."""
    import torch
    from paper_2410_05489_amd import ase
    from paper_2410_05489_amd import workloads as WL

    n = 1 << 20
    w = WL.shu_osher(n, 9)
    g, p = w.grid, w.params
    c1, c2 = 0.05, 1.0
    sim = ase.GksSimulation(g, p, w.U, c1=c1, c2=c2, device="cuda")
    sim.run(args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    sim.run(args.steps)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    finite = bool(torch.isfinite(sim.U).all().item())
    prof_steps = max(1, min(args.steps, 50))
    ase.profile_enable(True)
    sim.run(prof_steps)
    torch.cuda.synchronize()
    kern = {k: ase.profile_read(k) for k in ("gks_1d", "bc", "cfl")}
    ase.profile_enable(False)
    value = n * args.steps / (ms / 1e3) / 1e6
    tot, nl = kern["gks_1d"]
    avg_s = tot / max(nl, 1) / 1e3
    flops = alg_flops_per_cell_gks_stage(p.order)
    achieved = flops * n / avg_s / 1e12
    bytes_cell = (14 + 17) / 2 * 8.0   # stage 1: 14 words per cell, stage 2: 17
    out = {"metric": "Mcell-updates/s, 1D gas-kinetic S2O4 step, order 9 (FP64)", "value": round(value, 3),
           "unit": "Mcell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms / args.steps, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"gks_shu_osher_{n}_r9", "order": 9, "nx": n, "c1": c1, "c2": c2,
                      "cfl": p.cfl},
           "finite": finite,
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VALU_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4), "traffic": None,
                        "kernel": "k_gks1d, order 9", "avg_launch_ms": round(avg_s * 1e3, 4), "launches": nl,
                        "alg_flops_per_launch": flops * n, "alg_bytes_per_launch": bytes_cell * n,
                        "hbm_frac_alg": round(bytes_cell * n / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                        "kernel_ms_per_step": {k: round(v[0] / prof_steps, 4) for k, v in kern.items() if v[1]}}}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        m = 1 << 18
        ws = WL.shu_osher(m, 9)
        U = ws.U.copy()
        sx, _ = O.sigma_init(ws.grid, ws.params, U)
        t0 = time.perf_counter()
        O.step_gks(ws.grid, ws.params, U, sx, 0.0, 1, c1=c1, c2=c2)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m / el / 1e6, "unit": "Mcell-updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"1 S2O4 step of the same problem on {m} cells, single-threaded C "
                                         f"oracle, {el:.1f} s"}
    print(json.dumps(out), flush=True)


def alg_flops_per_cell_gks2d_stage(order: int) -> float:
    """Algorithmic FP64 operations per cell of one S2O4 stage of the 2D
    gas-kinetic path, per direction (x and y alike; FMA = 2; divide, square
    root, exp and erfc = 1):
      normal reconstruction  : DF sums + 2 faces x 4 vars x (2r-1), values
                               and slopes
      tangential (two sides) : 2 x (DF sums + G points x 4 vars x (2r-1) x 3:
                               values, their slopes, the normal slopes)
      per Gauss point        : 24 moment sums <(c.psi) u^K v^Q psi_j>, 19
                               general ones of 36 products (137 operations:
                               c <u^n> <v^m> with the 1/2 of psi_3 and
                               <xi^(2l)> where they are not 1, plus the sum)
                               and 5 on c = (1,0,0,0) (16) -> 2683; nine
                               micro slopes 225 and their right-hand sides
                               39, Maxwellian moments 206, three
                               Maxwellians 30, time integrals and tau_n 48,
                               accumulation into F and the kinetic averages
                               240, F and F_t 29, strength 38, quadrature
                               16                                  -> 3554
      update                 : 2 x 4 vars x 4 (L, L_t) + stage combination 16
    """
    R = (order - 1) // 2
    G = R
    sums = {1: 1, 2: 3, 3: 8, 4: 15}[R]
    normal = sums + 2 * 2 * 4 * (2 * order - 1)
    tang = 2 * (sums + G * 4 * (2 * order - 1) * 3)
    return 2 * (normal + tang + G * 3554) + 48


def bench_gks2d(args):
    """2D gas-kinetic solver (S2O4 steps) on the paper's timing problem:
    the Configuration-3 Riemann problem (Table 4), order 9, with the mesh of
    its largest entry (400 x 400, 20 steps) and a 1024 x 1024 grid."""
    import torch
    from paper_2410_05489_amd import ase
    from paper_2410_05489_amd import workloads as WL

    c1, c2 = 0.05, 1.0
    res = {}
    for n, steps in ((400, 20), (1024, args.steps)):
        w = WL.four_quadrant(n, 9, states=WL.CONFIG3_STATES)
        g, p = w.grid, w.params
        sim = ase.GksSimulation(g, p, w.U, c1=c1, c2=c2, device="cuda")
        sim.run(args.warmup)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        sim.run(steps)
        stop.record()
        torch.cuda.synchronize()
        res[n] = (start.elapsed_time(stop), steps, sim, g, p)
    ms, steps, sim, g, p = res[1024]
    n = g.nx * g.ny
    finite = bool(torch.isfinite(sim.U).all().item())
    prof_steps = max(1, min(steps, 20))
    ase.profile_enable(True)
    sim.run(prof_steps)
    torch.cuda.synchronize()
    kern = {k: ase.profile_read(k) for k in ("gks_2d_recon", "gks_2d_flux", "gks_2d_update", "bc", "cfl")}
    ase.profile_enable(False)
    value = n * steps / (ms / 1e3) / 1e6
    step_flops = 2 * alg_flops_per_cell_gks2d_stage(9) * n
    kern_ms = sum(v[0] for v in kern.values()) / prof_steps
    tot, nl = kern["gks_2d_flux"]
    ms400 = res[400][0]
    # viscous shock tube (Navier-Stokes through the kinetic flux), the
    # paper's 500 x 250 mesh, order 9
    wv = WL.viscous_shock_tube(500, 250, 9)
    simv = ase.GksSimulation(wv.grid, wv.params, wv.U, c1=1.0, c2=10.0, mu=wv.mu, device="cuda")
    simv.run(args.warmup)
    torch.cuda.synchronize()
    start.record()
    simv.run(steps)
    stop.record()
    torch.cuda.synchronize()
    msv = start.elapsed_time(stop)
    vst = {"workload": "viscous_shock_tube_500x250_r9_re200", "steps": steps,
           "value": round(wv.grid.nx * wv.grid.ny * steps / (msv / 1e3) / 1e6, 3), "unit": "Mcell-updates/s",
           "ms_per_step": round(msv / steps, 5), "finite": bool(torch.isfinite(simv.U).all().item())}
    out = {"metric": "Mcell-updates/s, 2D gas-kinetic S2O4 step, order 9 (FP64)", "value": round(value, 3),
           "unit": "Mcell-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "ms_per_step": round(ms / steps, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "gks_config3_1024x1024_r9", "order": 9, "nx": g.nx, "ny": g.ny, "c1": c1,
                      "c2": c2, "cfl": p.cfl},
           "finite": finite,
           "viscous": vst,
           "table4_config": {"workload": "gks_config3_400x400_r9", "steps": 20, "seconds": round(ms400 / 1e3, 5),
                             "paper_seconds": 165.221,
                             "paper_hardware": "one core of an AMD EPYC 7401 (context, not a target)"},
           "roofline": {"bound": "alu", "achieved": round(step_flops / (kern_ms / 1e3) / 1e12, 3),
                        "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(step_flops / (kern_ms / 1e3) / 1e12 / FP64_VALU_PEAK_TFLOPS, 4),
                        "traffic": None, "kernel": "whole 2D GKS step (recon + flux + update kernels), order 9",
                        "alg_flops_per_step": step_flops,
                        "flux_avg_launch_ms": round(tot / max(nl, 1), 4),
                        "kernel_ms_per_step": {k: round(v[0] / prof_steps, 4) for k, v in kern.items() if v[1]}}}
    print(json.dumps(out), flush=True)


def measure_adjoint(nsteps=100, every=10, reps=3):
    """Adjoint/forward wall-time ratio on the batched workload: 256 Riemann
    instances of 64..4096 cells, order 9, `nsteps` steps; J = sum_k dx_k sum p
    at the final time; gradient with respect to the initial state through the
    autograd wrapper (checkpoints every `every` steps).  Forward = the plain
    batched run of nsteps steps; backward = J.sum().backward() (objective
    gradient + the tape and reverse launches of each segment).  Two pairs:
    the fastest forward and backward (each autotuned, the wide forms
    included), which gives the ratio, and the persistent launches alone."""
    import numpy as np
    import torch
    from paper_2410_05489_amd import adjoint as A
    from paper_2410_05489_amd import ase, autotune
    from paper_2410_05489_amd import workloads as WL

    b_all = WL.batched_riemann(nsteps=nsteps)
    # instances the method loses (status != 0 after nsteps) are left out of
    # the timing: NaN arithmetic is no work of the method
    probe = ase.BatchedSimulation(b_all, "cuda", nbins=min(b_all.ninst, 256))
    st = torch.zeros(b_all.ninst, dtype=torch.int32, device="cuda")
    probe.run(nsteps, status=st)
    torch.cuda.synchronize()
    keep = np.flatnonzero(st.cpu().numpy() == 0)
    del probe
    b = WL.batch_subset(b_all, keep)
    fwd = autotune.tune_batched(b, nsteps=10, use_cache=False)
    fwd_p = min((t for t in fwd["trials"] if t["min_cells"] == 0), key=lambda t: t["ms"])
    adj = autotune.tune_adjoint(b, every=every, use_cache=False, fwd_shape=(fwd_p["nbins"], fwd_p["threads"]))
    adj_p = min((t for t in adj["trials"] if t["min_cells"] == 0), key=lambda t: t["ms"])
    U0 = torch.tensor(b.U, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    med = lambda a: sorted(a)[len(a) // 2]   # noqa: E731

    def timed(f, a, profile):
        """Median (plain forward, forward with checkpoints, backward) ms of
        forward shape f and adjoint shape a; the gradient and objective of
        the last repetition."""
        run = A.BatchedAdjoint(b, "cuda", nbins=f["nbins"], threads=f["threads"], adj_threads=a["threads"],
                               every=every, adj_nbins=a["nbins"], wide_min_cells=f["min_cells"],
                               wide_threads=f["wide_threads"] or 256, adj_wide_min_cells=a["min_cells"],
                               adj_wide_threads=a["wide_threads"] or 256)
        plain = ase.BatchedSimulation(b, "cuda", nbins=f["nbins"], threads=f["threads"],
                                      wide_min_cells=f["min_cells"], wide_threads=f["wide_threads"] or 256)
        t_plain, t_fwd, t_bwd = [], [], []
        for rep in range(reps + 1):
            plain.U.copy_(U0)
            plain.t.zero_()
            torch.cuda.synchronize()
            ev[0].record()
            plain.run(nsteps)
            ev[1].record()
            x = U0.clone().requires_grad_(True)
            torch.cuda.synchronize()
            ev[2].record()
            J = run.pressure(run.run(x, nsteps))
            ev[3].record()
            if profile and rep == reps:
                ase.profile_enable(True)
            ev[4].record()
            J.sum().backward()
            ev[5].record()
            torch.cuda.synchronize()
            if rep > 0:
                t_plain.append(ev[0].elapsed_time(ev[1]))
                t_fwd.append(ev[2].elapsed_time(ev[3]))
                t_bwd.append(ev[4].elapsed_time(ev[5]))
        return med(t_plain), med(t_fwd), med(t_bwd), J.detach().cpu().numpy(), x.grad.cpu().numpy()

    tp, tf, tb, Jh, gh = timed(fwd, adj, True)
    kms, kn = ase.profile_read("adjoint")
    ase.profile_enable(False)
    pp, pf, pb, _, _ = timed(fwd_p, adj_p, False)
    ok = 0
    for k in range(b.ninst):
        o, n = int(b.offsets[k]), int(b.ncells[k])
        ok += int(bool(np.isfinite(Jh[k])) and bool(np.isfinite(gh[:, o:o + n + 2 * b.ng]).all()))
    form = lambda t: "persistent + wide" if t["min_cells"] else "persistent"   # noqa: E731
    return {"workload": f"batched_riemann_{b_all.ninst}x64..4096_r9_seed0", "instances_timed": b.ninst,
            "instances_lost": [int(k) for k in np.flatnonzero(st.cpu().numpy() != 0)],
            "steps": nsteps, "checkpoint_every": every,
            "cells": int(b.ncells.sum()), "forward_ms": round(tp, 3), "forward_with_checkpoints_ms": round(tf, 3),
            "backward_ms": round(tb, 3), "adjoint_fwd_ratio": round(tb / tp, 3),
            "forward_form": form(fwd), "adjoint_form": form(adj),
            "forward_shape": [fwd["nbins"], fwd["threads"], fwd["min_cells"], fwd["wide_threads"]],
            "adjoint_shape": [adj["nbins"], adj["threads"], adj["min_cells"], adj["wide_threads"]],
            "adjoint_ms_per_segment_call": round(kms / max(kn, 1), 3),
            "persistent_only": {"forward_ms": round(pp, 3), "forward_with_checkpoints_ms": round(pf, 3),
                                "backward_ms": round(pb, 3), "adjoint_fwd_ratio": round(pb / pp, 3),
                                "forward_shape": [fwd_p["nbins"], fwd_p["threads"]],
                                "adjoint_shape": [adj_p["nbins"], adj_p["threads"]]},
            "instances_finite": ok, "adjoint_trials": adj["trials"]}


def cpu_baseline(w):
    """The oracle as it stands (OpenMP over grid lines) on the host's
    threads: eight steps of the same grid from its initial state (about 3 s
    on 16 threads); and two steps on a single thread (about 9 s)."""
    from oracle import oracle as O
    n = w.grid.ncells()
    nt = host_threads()
    rates = {}
    for threads, k in ((nt, 8), (1, 2)):
        used = O.set_threads(threads)
        U = w.U.copy()
        sx, sy = O.sigma_init(w.grid, w.params, U)
        t0 = time.perf_counter()
        O.step(w.grid, w.params, U, sx, sy, 0.0, k)
        el = time.perf_counter() - t0
        rates[threads] = (n * k / el / 1e6, used, k, el)
    v, used, k, el = rates[nt]
    v1, _, k1, el1 = rates[1]
    return {"value": v, "unit": "Mcell-updates/s", "cores": used, "kind": "oracle",
            "sample": f"{k} steps of {w.name} ({n} cells) from its initial state, C oracle on {used} threads, "
                      f"{el:.1f} s; {k1} steps on 1 thread, {el1:.1f} s",
            "single_thread": v1, "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def progress(msg: str) -> None:
    """A progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="quad1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratio measurement")
    ap.add_argument("--batched-shape", default="", metavar="BINS:THREADS:MIN_CELLS:WIDE_THREADS",
                    help="--workload batched: this launch shape instead of the autotuner's (MIN_CELLS 0: "
                         "the persistent launch alone; the persistent comparison then uses 256 bins of 1024 lanes)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this program runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU domain decomposition is a design note, not implemented)"}))
        sys.exit(2)

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "gks1d":
        return bench_gks(args)
    if args.workload == "gks2d":
        return bench_gks2d(args)
    if args.workload == "adjoint":
        print(json.dumps({"metric": "adjoint/forward wall-time ratio, batched 1D order 9", **measure_adjoint()}),
              flush=True)
        return

    import torch
    from paper_2410_05489_amd import ase

    ase.lib()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    w = make_workload(args.workload)
    g, p = w.grid, w.params
    sim = ase.Simulation(g, p, w.U, device="cuda")
    torch.cuda.synchronize()
    if args.warmup:
        sim.run(args.warmup)
    torch.cuda.synchronize()

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    sim.run(args.steps)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    finite = bool(torch.isfinite(sim.U).all().item())
    progress(f"{args.workload}: {args.steps} steps in {ms:.1f} ms")
    # per-kernel durations from a separate run with event timing around every
    # launch (the events themselves slow the step, so the timed run above has
    # none)
    prof_steps = max(1, min(args.steps, 50))
    ase.profile_enable(True)
    sim.run(prof_steps)
    torch.cuda.synchronize()
    kern = {k: ase.profile_read(k) for k in ("sweep_x", "sweep_y", "stage_1d", "bc", "cfl")}
    ase.profile_enable(False)

    ncell = g.ncells()
    value = ncell * args.steps / (ms / 1e3) / 1e6
    dom = max(("sweep_x", "sweep_y"), key=lambda k: kern[k][0])
    tot, nl = kern[dom]
    avg_s = tot / max(nl, 1) / 1e3
    lagged = p.df_source == 0
    flops = alg_flops_per_cell_sweep(p.order, g.dim, lagged) + (4 + 56.0 / 3.0 if dom == "sweep_y" else 0.0)
    achieved_tf = flops * ncell / avg_s / 1e12
    bytes_launch = alg_bytes_per_cell(dom, lagged) * ncell
    # minimal HBM traffic of a step: read U^n (3 stages), U^(s-1) (stages 2,
    # 3), write U^(s) (3 stages) = 8 nvar words per cell-update; the lagged
    # DF source adds a read and a write of each face strength per stage
    step_bytes = 8 * 4 * 8 + (12 * 8 if lagged else 0)
    traffic = None
    if args.workload in MEASURED_TRAFFIC["workloads"] and kernel_fingerprint() == MEASURED_TRAFFIC["fingerprint"]:
        traffic = MEASURED_TRAFFIC[args.workload][dom]
    roof = {"bound": "alu", "achieved": round(achieved_tf, 3), "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved_tf / FP64_VALU_PEAK_TFLOPS, 4), "traffic": traffic, "traffic_unit": "bytes/launch",
            "kernel": f"k_sweep2d ({dom}), order {p.order}",
            "avg_launch_ms": round(avg_s * 1e3, 4), "launches": nl,
            "alg_flops_per_launch": flops * ncell, "alg_bytes_per_launch": bytes_launch,
            "hbm_frac_alg": round(bytes_launch / avg_s / 1e9 / HBM_PEAK_GBS, 4),
            "step_alg_bytes_per_cell": step_bytes,
            "step_hbm_frac_alg": round(value * 1e6 * step_bytes / 1e9 / HBM_PEAK_GBS, 4),
            "kernel_ms_per_step": {k: round(v[0] / prof_steps, 4) for k, v in kern.items() if v[1]},
            "profiled_steps": prof_steps}
    out = {"metric": METRIC, "value": round(value, 3), "unit": "Mcell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {"workload": w.name, "order": p.order, "nx": g.nx, "ny": g.ny,
                                           "gamma": p.gamma, "cfl": p.cfl, "sigma_thres": p.sigma_thres,
                                           "df_source": "lagged" if lagged else "first_order",
                                           "positivity_fallback": bool(p.positivity_fallback)},
           "finite": finite, "roofline": roof}
    if args.workload == "jet":
        # the method as read does not carry this case through its 500 steps
        out["config"]["full_run"] = ("fails: a cell-average pressure turns negative before step 500 "
                                     "(step 298 with these kernels, 279 for the oracle: the method as read, "
                                     "not the kernels); "
                                     "timed over the first steps only")
    if not args.no_adjoint:
        progress("adjoint/forward ratio on the batched workload")
        out["adjoint"] = measure_adjoint()
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
