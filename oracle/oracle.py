"""ctypes front end of the C oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It loads ``liboracle.so`` (built from ase_oracle.c by
``build_oracle.build()``) and never touches the GPU library.

Arrays follow the state layout of ``paper_2410_05489_amd.workloads``:
U[v, J, I] and strengths s[J, I], float64, C-contiguous.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = C.POINTER(C.c_double)


class OrcGrid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("ng", C.c_int32),
                ("ld", C.c_int32), ("bc", C.c_int32 * 4), ("dx", C.c_double), ("dy", C.c_double),
                ("y0", C.c_double), ("inflow", C.c_double * 4), ("slot_lo", C.c_double),
                ("slot_hi", C.c_double), ("x0", C.c_double), ("wall_x0", C.c_double), ("shock_x0", C.c_double),
                ("shock_speed", C.c_double), ("outer", C.c_double * 4)]


class OrcParams(C.Structure):
    _fields_ = [("order", C.c_int32), ("positivity_fallback", C.c_int32), ("df_source", C.c_int32),
                ("pad_", C.c_int32), ("gamma", C.c_double),
                ("cfl", C.c_double), ("sigma_thres", C.c_double), ("eps", C.c_double),
                ("d_hi", C.c_double), ("d_lo", C.c_double), ("dt_cap", C.c_double)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build_oracle  # noqa: F401  (package-relative when imported as oracle.oracle)
            build_oracle.build()
        _LIB = C.CDLL(path)
        L = _LIB
        vp = C.c_void_p
        L.orc_bc_fill.argtypes = [vp, vp, _dp, _dp, _dp]
        L.orc_sigma_init.argtypes = [vp, vp, _dp, _dp, _dp]
        L.orc_reconstruct.argtypes = [vp, vp, C.c_int, _dp, _dp, _dp, _dp, _dp, C.POINTER(C.c_int8)]
        L.orc_df_compute.argtypes = [vp, vp, C.c_int, _dp, _dp, _dp]
        L.orc_flux.argtypes = [vp, vp, C.c_int, _dp, _dp, _dp]
        L.orc_stage_update.argtypes = [vp, vp, C.c_int, C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.orc_residual.argtypes = [vp, vp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_cfl_dt.argtypes = [vp, vp, _dp, C.c_double, C.c_double, _dp]
        L.orc_step.argtypes = [vp, vp, _dp, _dp, _dp, _dp, C.c_int, C.c_double, _dp]
        L.orc_poly.argtypes = [vp, _dp, _dp, C.c_int, _dp, _dp]
        L.orc_weno_ao53.argtypes = [vp, _dp, _dp, C.c_int, _dp, _dp]
        L.orc_weno_ao53.restype = None
        L.orc_coeffs.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.orc_beta3.argtypes = [_dp]
        L.orc_beta3.restype = C.c_double
        L.orc_zk.argtypes = [C.c_int, C.c_double]
        L.orc_zk.restype = C.c_double
        L.orc_alpha.argtypes = [C.c_double, C.c_double]
        L.orc_alpha.restype = C.c_double
        L.orc_gauss.argtypes = [C.c_int, _dp, _dp]
        L.orc_gauss.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        L.orc_sigma_point.argtypes = [vp, vp, _dp, _dp, C.c_int]
        L.orc_sigma_point.restype = C.c_double
        L.orc_lf_point.argtypes = [vp, vp, _dp, _dp, C.c_int, _dp]
        L.orc_lf_point.restype = None
        L.orc_bc_fill_at.argtypes = [vp, vp, C.c_double, _dp, _dp, _dp]
        L.orc_step_gks.argtypes = [vp, vp, vp, _dp, _dp, _dp, C.c_int, C.c_double, _dp]
        L.orc_residual_gks.argtypes = [vp, vp, vp, _dp, _dp, C.c_double, _dp, _dp, _dp]
        L.orc_gks_moments.argtypes = [C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.orc_gks_slopes.argtypes = [C.c_double, _dp, _dp, _dp, _dp]
        L.orc_gks_flux.argtypes = [C.c_double, _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
        L.orc_gks_point.argtypes = [C.c_double, vp, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_poly_d.argtypes = [vp, _dp, _dp, C.c_int, _dp, _dp, _dp]
        L.orc_step_gks2d.argtypes = [vp, vp, vp, _dp, _dp, _dp, _dp, C.c_int, C.c_double, _dp]
        L.orc_gks2_slopes.argtypes = [C.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_gks2_point.argtypes = [C.c_double, vp, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    return _LIB


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def c_grid(g) -> OrcGrid:
    s = OrcGrid()
    s.dim, s.nx, s.ny, s.ng, s.ld = g.dim, g.nx, g.ny, g.ng, g.ld
    for k in range(4):
        s.bc[k] = int(g.bc[k])
        s.inflow[k] = float(g.inflow[k])
    s.dx, s.dy, s.y0 = g.dx, g.dy, g.y0
    s.slot_lo, s.slot_hi = g.slot_lo, g.slot_hi
    s.x0, s.wall_x0, s.shock_x0, s.shock_speed = g.x0, g.wall_x0, g.shock_x0, g.shock_speed
    for k in range(4):
        s.outer[k] = float(g.outer[k])
    return s


def c_params(p) -> OrcParams:
    s = OrcParams()
    s.order, s.positivity_fallback = int(p.order), int(p.positivity_fallback)
    s.df_source = int(p.df_source)
    s.gamma, s.cfl, s.sigma_thres, s.eps = p.gamma, p.cfl, p.sigma_thres, p.eps
    s.d_hi, s.d_lo, s.dt_cap = p.d_hi, p.d_lo, p.dt_cap
    return s


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


def _gp(g, p):
    return C.byref(c_grid(g)), C.byref(c_params(p))


def ngauss(g, order):
    return 1 if g.dim == 1 else max(1, (order - 1) // 2)


def face_count(g, d):
    if g.dim == 1:
        return g.nx + 1
    return (g.nx + 1) * g.ny if d == 0 else g.nx * (g.ny + 1)


def sigma_init(g, p, U):
    """First-order strengths on every stored face; fills the ghosts of U."""
    sx = np.zeros((g.NY, g.ld))
    sy = np.zeros((g.NY, g.ld))
    G, P = _gp(g, p)
    _check(lib().orc_sigma_init(G, P, _ptr(U), _ptr(sx), _ptr(sy)), "sigma_init")
    return sx, sy


def bc_fill(g, p, U, sx, sy):
    G, P = _gp(g, p)
    _check(lib().orc_bc_fill(G, P, _ptr(U), _ptr(sx), _ptr(sy)), "bc_fill")


def bc_fill_at(g, p, t, U, sx, sy):
    """Ghost cells (moving-shock side at time t) and non-flux strengths."""
    G, P = _gp(g, p)
    _check(lib().orc_bc_fill_at(G, P, float(t), _ptr(U), _ptr(sx), _ptr(sy)), "bc_fill_at")


def reconstruct(g, p, d, U, sx, sy, want_level=False):
    Gq = ngauss(g, p.order)
    nf = face_count(g, d)
    wl = np.zeros((g.nvar, Gq, nf))
    wr = np.zeros((g.nvar, Gq, nf))
    lev = np.zeros((g.ny, g.nx), dtype=np.int8) if want_level else None
    G, P = _gp(g, p)
    _check(lib().orc_reconstruct(G, P, d, _ptr(U), _ptr(sx), _ptr(sy), _ptr(wl), _ptr(wr),
                                 lev.ctypes.data_as(C.POINTER(C.c_int8)) if lev is not None else None),
           "reconstruct")
    return (wl, wr, lev) if want_level else (wl, wr)


def df_compute(g, p, d, wl, wr, sig):
    G, P = _gp(g, p)
    _check(lib().orc_df_compute(G, P, d, _ptr(wl), _ptr(wr), _ptr(sig)), "df_compute")


def flux(g, p, d, wl, wr):
    F = np.zeros((g.nvar, face_count(g, d)))
    G, P = _gp(g, p)
    _check(lib().orc_flux(G, P, d, _ptr(wl), _ptr(wr), _ptr(F)), "flux")
    return F


def stage_update(g, p, stage, dt, Un, Us, F, Gf, Uo):
    G, P = _gp(g, p)
    _check(lib().orc_stage_update(G, P, stage, dt, _ptr(Un), _ptr(Us), _ptr(F), _ptr(Gf), _ptr(Uo)),
           "stage_update")


def residual(g, p, U, sx, sy):
    """L(W) at interior cells plus the strengths it produces on flux faces."""
    L = np.zeros(g.shape())
    sxn = sx.copy()
    syn = sy.copy()
    G, P = _gp(g, p)
    _check(lib().orc_residual(G, P, _ptr(U), _ptr(sx), _ptr(sy), _ptr(L), _ptr(sxn),
                              _ptr(syn) if g.dim == 2 else None), "residual")
    return L, sxn, syn


def cfl_dt(g, p, U, t=0.0, t_end=0.0):
    out = C.c_double(0.0)
    G, P = _gp(g, p)
    _check(lib().orc_cfl_dt(G, P, _ptr(U), t, t_end, C.byref(out)), "cfl_dt")
    return out.value


def step(g, p, U, sx, sy, t, nsteps, t_end=0.0):
    """Advance in place; returns (t, dt history)."""
    tt = C.c_double(t)
    hist = np.zeros(max(nsteps, 1))
    G, P = _gp(g, p)
    n = _check(lib().orc_step(G, P, _ptr(U), _ptr(sx), _ptr(sy) if sy is not None else None,
                              C.byref(tt), nsteps, t_end, _ptr(hist)), "step")
    return tt.value, hist[:n]


def run(g, p, U, nsteps, t_end=0.0):
    """Initialise strengths and march; returns (U, sx, sy, t, dts)."""
    U = U.copy()
    sx, sy = sigma_init(g, p, U)
    t, dts = step(g, p, U, sx, sy, 0.0, nsteps, t_end)
    return U, sx, sy, t, dts


# ---- single-cell hooks ------------------------------------------------------

def poly(p, W, s, xi):
    W = np.ascontiguousarray(W, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.zeros(len(xi))
    lvl = lib().orc_poly(C.byref(c_params(p)), _ptr(W), _ptr(s), len(xi), _ptr(xi), _ptr(out))
    return out, lvl


def weno_ao53(p, W, alpha, xi):
    W = np.ascontiguousarray(W, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.zeros(len(xi))
    lib().orc_weno_ao53(C.byref(c_params(p)), _ptr(W), _ptr(alpha), len(xi), _ptr(xi), _ptr(out))
    return out


def coeffs(kind, sub, W):
    W = np.ascontiguousarray(W, dtype=np.float64)
    a = np.zeros(8)
    n = lib().orc_coeffs(kind, sub, _ptr(W), _ptr(a))
    return a[:n]


def beta3(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return lib().orc_beta3(_ptr(a))


def zk(k, xi):
    return lib().orc_zk(k, xi)


def alpha(A, thres):
    return lib().orc_alpha(A, thres)


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops; returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


def gauss(G):
    node = np.zeros(4)
    eta = np.zeros(4)
    lib().orc_gauss(G, _ptr(node), _ptr(eta))
    return node[:G], eta[:G]


def sigma_point(g, p, Wl, Wr, d):
    Wl = np.ascontiguousarray(Wl, dtype=np.float64)
    Wr = np.ascontiguousarray(Wr, dtype=np.float64)
    G, P = _gp(g, p)
    return lib().orc_sigma_point(G, P, _ptr(Wl), _ptr(Wr), d)


def lf_point(g, p, Wl, Wr, d):
    Wl = np.ascontiguousarray(Wl, dtype=np.float64)
    Wr = np.ascontiguousarray(Wr, dtype=np.float64)
    F = np.zeros(g.nvar)
    G, P = _gp(g, p)
    lib().orc_lf_point(G, P, _ptr(Wl), _ptr(Wr), d, _ptr(F))
    return F


# ---- gas-kinetic solver (1D) -------------------------------------------------

class OrcGks(C.Structure):
    _fields_ = [("c1", C.c_double), ("c2", C.c_double), ("tau", C.c_double), ("mu", C.c_double)]


def c_gks(c1, c2, tau=0.0, mu=0.0) -> OrcGks:
    return OrcGks(float(c1), float(c2), float(tau), float(mu))


def _vec(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def step_gks(g, p, U, sx, t, nsteps, t_end=0.0, c1=0.05, c2=1.0, tau=0.0):
    """S2O4 GKS steps in place (1D); returns (t, dt history)."""
    tt = C.c_double(t)
    hist = np.zeros(max(nsteps, 1))
    G, P = _gp(g, p)
    K = c_gks(c1, c2, tau)
    n = _check(lib().orc_step_gks(G, P, C.byref(K), _ptr(U), _ptr(sx), C.byref(tt), nsteps, t_end,
                                  _ptr(hist)), "step_gks")
    return tt.value, hist[:n]


def run_gks(g, p, U, nsteps, t_end=0.0, c1=0.05, c2=1.0, tau=0.0):
    U = U.copy()
    sx, _ = sigma_init(g, p, U)
    t, dts = step_gks(g, p, U, sx, 0.0, nsteps, t_end, c1, c2, tau)
    return U, sx, t, dts


def residual_gks(g, p, U, sx, dt, c1=0.05, c2=1.0, tau=0.0):
    """L, L_t at interior cells and the face strengths of one GKS stage."""
    L = np.zeros(g.shape())
    Lt = np.zeros(g.shape())
    sxn = sx.copy()
    G, P = _gp(g, p)
    K = c_gks(c1, c2, tau)
    _check(lib().orc_residual_gks(G, P, C.byref(K), _ptr(U), _ptr(sx), dt, _ptr(L), _ptr(Lt), _ptr(sxn)),
           "residual_gks")
    return L, Lt, sxn


def gks_moments(gamma, W):
    um, up, un, xm = np.zeros(8), np.zeros(8), np.zeros(8), np.zeros(3)
    _check(lib().orc_gks_moments(gamma, _ptr(_vec(W)), _ptr(um), _ptr(up), _ptr(un), _ptr(xm)), "gks_moments")
    return um, up, un, xm


def gks_slopes(gamma, W, Wx):
    a, A = np.zeros(3), np.zeros(3)
    _check(lib().orc_gks_slopes(gamma, _ptr(_vec(W)), _ptr(_vec(Wx)), _ptr(a), _ptr(A)), "gks_slopes")
    return a, A


def gks_flux(gamma, Wl, Wlx, Wr, Wrx, tau, taun, delta):
    F = np.zeros(3)
    _check(lib().orc_gks_flux(gamma, _ptr(_vec(Wl)), _ptr(_vec(Wlx)), _ptr(_vec(Wr)), _ptr(_vec(Wrx)),
                              tau, taun, delta, _ptr(F)), "gks_flux")
    return F


def gks_point(gamma, dt, Wl, Wlx, Wr, Wrx, c1=0.05, c2=1.0, tau=0.0):
    Fn, Ft = np.zeros(3), np.zeros(3)
    K = c_gks(c1, c2, tau)
    _check(lib().orc_gks_point(gamma, C.byref(K), dt, _ptr(_vec(Wl)), _ptr(_vec(Wlx)), _ptr(_vec(Wr)),
                               _ptr(_vec(Wrx)), _ptr(Fn), _ptr(Ft)), "gks_point")
    return Fn, Ft


def poly_d(p, W, s, xi):
    W, s, xi = _vec(W), _vec(s), _vec(xi)
    out, dout = np.zeros(len(xi)), np.zeros(len(xi))
    lvl = lib().orc_poly_d(C.byref(c_params(p)), _ptr(W), _ptr(s), len(xi), _ptr(xi), _ptr(out), _ptr(dout))
    return out, dout, lvl


# ---- gas-kinetic solver (2D) -------------------------------------------------

def step_gks2d(g, p, U, sx, sy, t, nsteps, t_end=0.0, c1=0.05, c2=1.0, tau=0.0, mu=0.0):
    """S2O4 GKS steps in place (2D; mu > 0: viscous); returns (t, dt history)."""
    tt = C.c_double(t)
    hist = np.zeros(max(nsteps, 1))
    G, P = _gp(g, p)
    K = c_gks(c1, c2, tau, mu)
    n = _check(lib().orc_step_gks2d(G, P, C.byref(K), _ptr(U), _ptr(sx), _ptr(sy), C.byref(tt), nsteps, t_end,
                                    _ptr(hist)), "step_gks2d")
    return tt.value, hist[:n]


def run_gks2d(g, p, U, nsteps, t_end=0.0, c1=0.05, c2=1.0, tau=0.0, mu=0.0):
    U = U.copy()
    sx, sy = sigma_init(g, p, U)
    t, dts = step_gks2d(g, p, U, sx, sy, 0.0, nsteps, t_end, c1, c2, tau, mu)
    return U, sx, sy, t, dts


def gks2_slopes(gamma, W, Wn, Wt):
    an, at, A = np.zeros(4), np.zeros(4), np.zeros(4)
    _check(lib().orc_gks2_slopes(gamma, _ptr(_vec(W)), _ptr(_vec(Wn)), _ptr(_vec(Wt)), _ptr(an), _ptr(at),
                                 _ptr(A)), "gks2_slopes")
    return an, at, A


def gks2_point(gamma, dt, Wl, Wln, Wlt, Wr, Wrn, Wrt, c1=0.05, c2=1.0, tau=0.0, mu=0.0):
    Fn, Ft = np.zeros(4), np.zeros(4)
    K = c_gks(c1, c2, tau, mu)
    _check(lib().orc_gks2_point(gamma, C.byref(K), dt, _ptr(_vec(Wl)), _ptr(_vec(Wln)), _ptr(_vec(Wlt)),
                                _ptr(_vec(Wr)), _ptr(_vec(Wrn)), _ptr(_vec(Wrt)), _ptr(Fn), _ptr(Ft)), "gks2_point")
    return Fn, Ft
