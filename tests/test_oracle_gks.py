"""Pins of the oracle's gas-kinetic solver (Sec. 2.2, App. A): the Maxwellian
moments against quadrature, the micro slopes against the closed form of
App. A, the flux of a uniform state, the equilibrium (Lax-Wendroff) limit
against the Euler Jacobian, conservation, the Sod tube, and Table 1's printed
L1 errors of the sine wave.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import exact_riemann as ER
from paper_2410_05489_amd import workloads as WL

HERE = os.path.dirname(os.path.abspath(__file__))
GAMMA = 1.4


def _prim(W, gamma=GAMMA):
    rho = W[0]
    u = W[1] / rho
    p = (gamma - 1.0) * (W[2] - 0.5 * rho * u * u)
    return rho, u, p


def _euler_flux(W, gamma=GAMMA):
    rho, u, p = _prim(W, gamma)
    return np.array([rho * u, rho * u * u + p, u * (W[2] + p)])


def _jacobian(W, h=1e-6):
    J = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h * max(1.0, abs(W[k]))
        J[:, k] = (_euler_flux(W + e) - _euler_flux(W - e)) / (2 * e[k])
    return J


STATES = [np.array([1.0, 0.3, 2.5]), np.array([0.125, -0.2, 0.3]), np.array([2.0, 3.0, 9.0]),
          np.array([0.7, -1.5, 4.0])]


@pytest.mark.parametrize("W", STATES)
def test_moments_against_quadrature(oracle, W):
    rho, U, p = _prim(W)
    lam = rho / (2 * p)
    um, up, un, xm = oracle.gks_moments(GAMMA, W)
    f = lambda u: math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2)
    for n in range(8):
        full = integrate.quad(lambda u: u ** n * f(u), -np.inf, np.inf, epsabs=1e-13, epsrel=1e-12)[0]
        pos = integrate.quad(lambda u: u ** n * f(u), 0.0, np.inf, epsabs=1e-13, epsrel=1e-12)[0]
        neg = integrate.quad(lambda u: u ** n * f(u), -np.inf, 0.0, epsabs=1e-13, epsrel=1e-12)[0]
        scale = max(1.0, abs(full))
        assert abs(um[n] - full) < 1e-10 * scale
        assert abs(up[n] - pos) < 1e-10 * scale
        assert abs(un[n] - neg) < 1e-10 * scale
    # K internal Gaussian degrees of freedom of variance 1/(2 lambda):
    # E[xi^2] = K s, E[xi^4] = K (K + 2) s^2 with s = 1/(2 lambda)
    K = (3 - GAMMA) / (GAMMA - 1)
    s = 1 / (2 * lam)
    assert abs(xm[1] - K * s) < 1e-14 * K * s
    assert abs(xm[2] - K * (K + 2) * s * s) < 1e-13 * K * (K + 2) * s * s
    # rho <psi> = W: the Maxwellian carries the state
    psi = np.array([um[0], um[1], 0.5 * (um[2] + xm[1])])
    assert np.allclose(rho * psi, W, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("W", STATES)
def test_micro_slopes_match_appendix_closed_form(oracle, W):
    """The oracle solves M a = b by elimination on the moment matrix; App. A
    prints the closed-form solution (2D; the 1D state is V = 0 with one
    internal degree of freedom fewer: K_2D + 2 = K_1D + 1)."""
    rng = np.random.default_rng(3)
    Wx = rng.normal(size=3)
    a, A = oracle.gks_slopes(GAMMA, W, Wx)
    rho, U, p = _prim(W)
    lam = rho / (2 * p)
    K2 = (3 - GAMMA) / (GAMMA - 1) - 1
    b1, b2, b4 = Wx / rho
    R4 = 2 * b4 - (U * U + (K2 + 2) / (2 * lam)) * b1
    R2 = b2 - U * b1
    a4 = 4 * lam * lam / (K2 + 2) * (R4 - 2 * U * R2)
    a2 = 2 * lam * R2 - U * a4
    a1 = b1 - U * a2 - 0.5 * a4 * (U * U + (K2 + 2) / (2 * lam))
    ref = np.array([a1, a2, a4])
    assert np.allclose(a, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    # compatibility: <A + a u> = 0 moment by moment, i.e. rho <A psi> is
    # minus the x-derivative of the Euler flux: -J W_x
    um, _, _, xm = oracle.gks_moments(GAMMA, W)
    def avg_lin(c, k):   # <(c . psi) u^k psi_j>, j = 0..2
        out = np.zeros(3)
        for j in range(3):
            # polynomial in u and xi^2, coefficients per (power of u, power of xi^2)
            terms = {}
            lin = {(0, 0): c[0], (1, 0): c[1], (2, 0): 0.5 * c[2], (0, 1): 0.5 * c[2]}
            psi = [{(0, 0): 1.0}, {(1, 0): 1.0}, {(2, 0): 0.5, (0, 1): 0.5}][j]
            for (n1, l1), v1 in lin.items():
                for (n2, l2), v2 in psi.items():
                    key = (n1 + n2 + k, l1 + l2)
                    terms[key] = terms.get(key, 0.0) + v1 * v2
            out[j] = sum(v * um[n] * xm[l] for (n, l), v in terms.items())
        return out
    assert np.allclose(rho * avg_lin(a, 0), Wx, rtol=1e-11, atol=1e-11)
    assert np.allclose(rho * avg_lin(A, 0), -_jacobian(W) @ Wx, rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("tau,taun,delta", [(0.0, 0.0, 0.1), (0.0, 0.02, 0.1), (0.01, 0.03, 0.05),
                                            (0.0, 10.0, 0.1)])
def test_uniform_state_flux_is_euler_flux(oracle, tau, taun, delta):
    for W in STATES:
        F = oracle.gks_flux(GAMMA, W, np.zeros(3), W, np.zeros(3), tau, taun, delta)
        assert np.allclose(F, delta * _euler_flux(W), rtol=1e-13, atol=1e-13 * delta)


def test_equilibrium_limit_is_lax_wendroff(oracle):
    """Collision times zero, equal smooth sides: F = F_E(W) and
    F_t = J W_t = -J^2 W_x."""
    rng = np.random.default_rng(7)
    for W in STATES:
        Wx = rng.normal(size=3)
        Fn, Ft = oracle.gks_point(GAMMA, 0.01, W, Wx, W, Wx, c1=0.0, c2=0.0)
        J = _jacobian(W)
        assert np.allclose(Fn, _euler_flux(W), rtol=1e-12, atol=1e-12)
        assert np.allclose(Ft, -J @ J @ Wx, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("order", [3, 5, 7, 9])
def test_reconstruction_slope_is_the_polynomial_derivative(oracle, order):
    """The slope the kinetic flux takes is dP/dxi of the same ASE-DF
    polynomial, on every level (linear, WENO-Z-AO fallback)."""
    R = (order - 1) // 2
    rng = np.random.default_rng(order)
    p = WL.Params(order=order)
    for trial in range(12):
        W = rng.normal(size=2 * R + 1)
        s = rng.uniform(0, 1.5, size=2 * R) if trial % 3 else rng.uniform(0, 0.1, size=2 * R)
        if trial % 4 == 1:
            s[R] = 5.0      # a jump inside the 5-cell stencil: WENO fallback
        xi = np.array([0.0, -1.0, -0.3])
        h = 1e-5
        out, dout, lvl = oracle.poly_d(p, W, s, xi)
        up, _ = oracle.poly(p, W, s, xi + h)
        dn, _ = oracle.poly(p, W, s, xi - h)
        assert np.allclose(out, oracle.poly(p, W, s, xi)[0], rtol=0, atol=0)
        assert np.allclose(dout, (up - dn) / (2 * h), rtol=1e-7, atol=1e-7)


def _table1():
    out = {}
    with open(os.path.join(HERE, "golden", "sine_wave_gks_1d.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, *errs = line.split()
            out[int(n)] = dict(zip((5, 7, 9), map(float, errs)))
    return out


def _sine_l1(oracle, n, order):
    w = WL.density_wave_1d(n, order, t_end=2.0)
    g, p = w.grid, w.params
    p.dt_cap = g.dx ** (order / 4.0)   # dt = dx^(r/4): fourth order in time
    p.cfl = 1e3                        # (the cap governs)
    U, _, t, _ = oracle.run_gks(g, p, w.U, 10 ** 7, 2.0, c1=0.0, c2=0.0)
    assert abs(t - 2.0) < 1e-14
    return np.abs(g.interior(U)[0] - WL.density_wave_exact_1d(n, 2.0)).mean()


@pytest.mark.parametrize("order,n", [(5, 20), (5, 40), (5, 80), (7, 20), (7, 40), (9, 20), (9, 40)])
def test_sine_wave_errors_match_table1(oracle, order, n):
    """The printed L1 errors of Table 1, reproduced to the printed digits
    away from the round-off floor (an absolute 1e-15 allows for the rounding
    accumulated over the 1692 steps of r = 9 at N = 40)."""
    ref = _table1()[n][order]
    err = _sine_l1(oracle, n, order)
    assert abs(err - ref) < max(1e-6 * ref, 1e-15), (err, ref)


def test_gks_conserves_and_keeps_uniform_flow(oracle):
    n, order = 64, 9
    w = WL.density_wave_1d(n, order, seed=3, amp=0.05)
    g, p = w.grid, w.params
    U, _, _, _ = oracle.run_gks(g, p, w.U, 30, c1=0.05, c2=1.0)
    s0 = g.interior(w.U).sum(axis=-1)
    s1 = g.interior(U).sum(axis=-1)
    assert np.allclose(s1, s0, rtol=1e-13, atol=0)
    # uniform flow stays uniform (to round-off)
    U0 = w.U.copy()
    g.interior(U0)[...] = np.array([1.0, 0.5, 2.7])[:, None, None] if g.interior(U0).ndim == 3 else \
        np.array([1.0, 0.5, 2.7])[:, None]
    U1, _, _, _ = oracle.run_gks(g, p, U0, 10, c1=0.05, c2=1.0)
    assert np.abs(g.interior(U1) - g.interior(U0)).max() < 1e-13


def test_gks_sod_against_exact(oracle):
    n = 200
    errs = {}
    for order in (1, 5):
        w = WL.sod(n, order)
        w.params.positivity_fallback = 1
        U, _, t, _ = oracle.run_gks(w.grid, w.params, w.U, w.nsteps, w.t_end, c1=0.05, c2=1.0)
        assert abs(t - 0.2) < 1e-14
        rho = w.grid.interior(U)[0].ravel()
        ex = ER.cell_average_density((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), n, 0.2, sub=16)
        errs[order] = np.abs(rho - ex).mean()
    assert errs[5] < 0.5 * errs[1], errs
    assert errs[5] < 4e-3, errs
