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
    assert L.ase_version() == 1


def _args(order=9, **kw):
    w = WL.four_quadrant(16, 9, seed=0)
    g, p = w.grid, w.params
    p.order = order
    for k, v in kw.items():
        setattr(g, k, v)
    return C.byref(ase.c_grid(g)), C.byref(ase.c_params(p))


@pytest.mark.parametrize("kw,code", [({"order": 4}, -2), ({"order": 11}, -2), ({"ng": 4}, -3),
                                     ({"ld": 20}, -1), ({"dim": 3}, -1)])
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
