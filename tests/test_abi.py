"""The C-ABI library loads, exports every symbol the header declares, and
rejects bad arguments before touching the GPU (CPU-only checks)."""
import ctypes as C
import os
import re

import pytest

from paper_2410_05489_amd import ase
from paper_2410_05489_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(ase_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = ase.lib()
    names = _declared()
    assert "ase_step" in names and "ase_reconstruct" in names
    for n in names:
        assert hasattr(L, n), n
    assert L.ase_version() == 4


def _args(order=9, **kw):
    w = WL.four_quadrant(16, 9, seed=0)
    g, p = w.grid, w.params
    p.order = order
    for k, v in kw.items():
        setattr(g, k, v)
    return C.byref(ase.c_grid(g)), C.byref(ase.c_params(p))


@pytest.mark.parametrize("kw,code", [({"order": 4}, -2), ({"order": 11}, -2), ({"ng": 4}, -3),
                                     ({"ld": 20}, -1), ({"dim": 3}, -1), ({"nx": 0}, -1), ({"ny": 0}, -1),
                                     ({"nx": -5}, -1)])
def test_argument_errors(kw, code):
    L = ase.lib()
    order = kw.pop("order", 9)
    G, P = _args(order, **kw)
    rc = L.ase_step(G, P, None, None, None, None, None, 1, 0.0, None, 0, None)
    assert rc == code
    assert len(L.ase_last_error()) > 0
    assert L.ase_workspace_bytes(G, P) == 0


def test_periodic_must_pair():
    L = ase.lib()
    G, P = _args(bc=(0, 1, 1, 1))
    assert L.ase_bc_fill(G, P, None, None, None, None) == -1
    assert b"periodic" in L.ase_last_error()


def test_adjoint_argument_errors():
    """The adjoint entry points reject 2D grids, unsupported boundaries and
    launch shapes before any device work."""
    L = ase.lib()
    G, P = _args()                                # 2D grid
    rc = L.ase_adjoint_step(G, P, None, None, None, None, None, None, 0, None)
    assert rc == -1 and b"1D" in L.ase_last_error()
    assert L.ase_adjoint_workspace_bytes(G) == 0
    w = WL.sod(50, 9)
    g = w.grid
    g.bc = (WL.BC_INFLOW_SLOT, WL.BC_TRANSMISSIVE, 1, 1)
    G1, P1 = C.byref(ase.c_grid(g)), C.byref(ase.c_params(w.params))
    rc = L.ase_adjoint_step(G1, P1, None, None, None, None, None, None, 0, None)
    assert rc == -1 and b"transmissive" in L.ase_last_error()
    g.bc = (WL.BC_TRANSMISSIVE,) * 4
    assert L.ase_adjoint_workspace_bytes(C.byref(ase.c_grid(g))) > 0
    rc = L.ase_adjoint_batched(P1, 1, None, 4, None, None, None, 5, 100, None, None, None, 3, None, None, None, 2,
                               1024, 3, None, 0, None)
    assert rc == -1
    assert L.ase_adjoint_batched_workspace_bytes(1000, 10) >= 1000 * 8 * (12 * 10 + 6)


def test_gks_argument_errors():
    """The gas-kinetic entry points reject missing arrays and bad collision
    parameters before any device work."""
    L = ase.lib()
    G, P = _args()                                # 2D grid
    gk = ase.c_gks(0.05, 1.0)
    assert L.ase_gks_workspace_bytes(G, P) > L.ase_workspace_bytes(G, P)
    rc = L.ase_step_gks(G, P, C.byref(gk), None, None, None, None, None, 1, 0.0, None, 0, None)
    assert rc == -1 and b"null" in L.ase_last_error()
    w = WL.sod(50, 5)
    G1, P1 = C.byref(ase.c_grid(w.grid)), C.byref(ase.c_params(w.params))
    assert L.ase_gks_workspace_bytes(G1, P1) == L.ase_workspace_bytes(G1, P1)
    bad = ase.c_gks(-1.0, 1.0)
    rc = L.ase_step_gks(G1, P1, C.byref(bad), None, None, None, None, None, 1, 0.0, None, 0, None)
    assert rc == -1 and b"c1" in L.ase_last_error()
    rc = L.ase_gks_flux(P1, C.byref(gk), 4, None, None, None, None, 0.0, None, None, None)
    assert rc == -1 and b"dt" in L.ase_last_error()
    assert L.ase_gks_flux(P1, C.byref(gk), 0, None, None, None, None, 0.1, None, None, None) == 0


def test_python_constants_match_header():
    """Flag and status values the binding uses are the header's."""
    text = open(os.path.join(ROOT, "include", "ase.h")).read()

    def val(name):
        return int(re.search(rf"\b{name}\s*=\s*(-?\d+)", text).group(1))

    assert val("ASE_FLAG_POSITIVITY_FALLBACK") == ase.FLAG_POSITIVITY_FALLBACK
    assert val("ASE_FLAG_DF_FIRST_ORDER") == ase.FLAG_DF_FIRST_ORDER
    assert val("ASE_FLAG_FAIL_NONPHYSICAL") == ase.FLAG_FAIL_NONPHYSICAL
    assert val("ASE_ERR_NONPHYSICAL") == ase.ERR_NONPHYSICAL
    p = WL.sod(20, 5).params
    p.fail_nonphysical = 1
    assert ase.c_params(p).flags & ase.FLAG_FAIL_NONPHYSICAL


def test_empty_batches_are_rejected():
    """A batch of no instances, an empty plan or a batch of no cells is an
    argument error (host checks, nothing launched)."""
    L = ase.lib()
    nc = (C.c_int32 * 2)(5, 7)
    start = (C.c_int32 * 3)()
    lst = (C.c_int32 * 2)()
    assert L.ase_batched_plan(0, nc, 2, start, lst) == -1
    assert L.ase_batched_plan(2, nc, 0, start, lst) == -1
    assert L.ase_batched_plan(2, nc, 2, start, lst) == 0
    assert sorted(lst) == [0, 1] and start[2] == 2
    P = C.byref(ase.c_params(WL.sod(20, 9).params))
    rc = L.ase_step_batched(P, 1, None, 0, None, None, None, 5, 0, None, None, None, None, None, None, 1, 0.0,
                            None, None, 1, 256, None, 0, None)
    assert rc == -1 and len(L.ase_last_error()) > 0


@pytest.mark.parametrize("order,threads", [(9, 256), (5, 512), (3, 256), (9, 256 | ase.WIDE_STEP),
                                          (7, 512 | ase.WIDE_STEP)])
def test_wide_plan_covers_each_large_instance_once(order, threads):
    """The wide plan cuts every instance of at least min_cells cells (and one
    full tile) into consecutive tiles of threads - order - 1 cells (one
    launch per step: threads - 3 (order + 1)) that cover it exactly once;
    every other instance lands in exactly one bin."""
    import numpy as np
    rng = np.random.default_rng(3)
    nc = rng.integers(1, 5000, size=40).astype(np.int32)
    lanes = threads & ~ase.WIDE_STEP
    T = lanes - (3 if threads & ase.WIDE_STEP else 1) * (order + 1)
    nc[0], nc[1] = 4096, T   # one tile exactly
    start, lst, ti, t0, it0, itn = ase.batched_plan_wide(nc, 1500, order, threads, 7)
    wide = (nc >= 1500) & (nc >= T)
    if threads & ase.WIDE_STEP:
        # the per-step form tiles an instance of any length
        _, lst1, ti1, _, it01, itn1 = ase.batched_plan_wide(nc, 1, order, threads, 7)
        assert len(lst1) == 0 and np.all(it01 >= 0) and np.all(itn1 == -(-nc // T))
    assert sorted(lst.tolist()) == sorted(np.flatnonzero(~wide).tolist())
    assert start[0] == 0 and np.all(np.diff(start) >= 0) and start[-1] == len(lst)
    assert len(ti) == int(sum(-(-int(n) // T) for n in nc[wide]))
    for k in range(len(nc)):
        if not wide[k]:
            assert it0[k] == -1 and itn[k] == 0
            continue
        js = np.arange(it0[k], it0[k] + itn[k])
        assert np.all(ti[js] == k)
        assert np.array_equal(t0[js], np.arange(itn[k]) * T)
        assert t0[js[-1]] < nc[k] <= t0[js[-1]] + T
    # no minimum: the plain plan's bins, no tiles
    start0, lst0, ti0, _, it00, _ = ase.batched_plan_wide(nc, 0, order, threads, 7)
    s1, l1 = ase.batched_plan(nc, 7)
    assert len(ti0) == 0 and np.all(it00 == -1)
    assert np.array_equal(start0, s1) and np.array_equal(lst0, l1)


def test_wide_form_argument_errors():
    """The wide form refuses the Gauss-point source, other tile widths and a
    missing or short workspace before launching anything."""
    L = ase.lib()
    w = WL.sod(20, 9)
    one = (C.c_int32 * 1)(20)
    off = (C.c_int64 * 1)(0)
    buf = (C.c_double * 128)()
    nb = L.ase_batched_wide_workspace_bytes(30, 1, 1)
    assert nb > L.ase_batched_workspace_bytes(30)
    wsbuf = C.create_string_buffer(nb + 512)
    ws = (C.addressof(wsbuf) + 255) // 256 * 256

    def call(params, thr, wsp, nbytes):
        return L.ase_step_batched_wide(C.byref(ase.c_params(params)), 1, None, 1, off, one, buf, 5, 30, buf, buf,
                                       buf, None, None, None, 1, 0.0, one, one, 1, 256, one, one, one, one, 1, thr,
                                       wsp, nbytes, None)

    w.params.df_source = 0
    assert call(w.params, 256, ws, nb) == -1 and b"FIRST_ORDER" in L.ase_last_error()
    w.params.df_source = 1
    assert call(w.params, 384, ws, nb) == -1 and b"threads_wide" in L.ase_last_error()
    assert call(w.params, 1024 | ase.WIDE_STEP, ws, nb) == -1 and b"threads_wide" in L.ase_last_error()
    assert call(w.params, 256 | (ase.WIDE_STEP << 1), ws, nb) == -1 and b"threads_wide" in L.ase_last_error()
    assert call(w.params, 256, None, nb) == -6
    assert call(w.params, 256, ws, nb - 8) == -6
