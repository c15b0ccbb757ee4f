"""Pins of the oracle's reconstruction formulas against independent facts.

Each test compares the oracle with something other than itself: exact
rational cell-average fits computed here from the definition of the zero-mean
basis, textbook linear weights and smoothness indicators, Taylor series,
numpy's Gauss-Legendre rule, and invariants of the DF/level rule.
"""
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_2410_05489_amd.workloads import Params

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# exact cell-average fits (definition: P in span{1, xi^k}, mean of P over
# each stencil cell = that cell's average; cell m occupies [m-1, m])
# ---------------------------------------------------------------------------

def _mean_pow(k, a, b):
    return Fr(b ** (k + 1) - a ** (k + 1), (k + 1) * (b - a))


def _solve(M, rhs):
    n = len(M)
    A = [row[:] + [rhs[i]] for i, row in enumerate(M)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        p = A[c][c]
        A[c] = [x / p for x in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [A[i][n] for i in range(n)]


def exact_fit_coeffs(cells, W):
    """Coefficients a_1..a_{n-1} of P = W_0 + sum a_k (xi^k - mean_{[-1,0]} xi^k)."""
    others = [c for c in cells if c != 0]
    n = len(cells)
    M = [[_mean_pow(k, c - 1, c) - _mean_pow(k, -1, 0) for k in range(1, n)] for c in others]
    rhs = [W[c] - W[0] for c in others]
    return _solve(M, rhs)


STENCILS = [(3, -1, [-2, -1, 0]), (3, 0, [-1, 0, 1]), (3, 1, [0, 1, 2]),
            (5, 0, list(range(-2, 3))), (7, 0, list(range(-3, 4))), (9, 0, list(range(-4, 5)))]


@pytest.mark.parametrize("kind,sub,cells", STENCILS)
def test_printed_coefficients_are_the_exact_fit(oracle, kind, sub, cells):
    rng = np.random.default_rng(kind * 10 + sub)
    R = {3: 2, 5: 2, 7: 3, 9: 4}[kind]
    for trial in range(5):
        vals = rng.integers(-50, 50, size=2 * R + 1)
        Wd = {m: Fr(int(vals[m + R])) for m in range(-R, R + 1)}
        exact = exact_fit_coeffs(cells, Wd)
        got = oracle.coeffs(kind, sub, vals.astype(np.float64))
        assert len(got) == len(exact)
        for g, e in zip(got, exact):
            assert abs(g - float(e)) <= 1e-12 * max(1.0, abs(float(e)))


def _golden_face_weights():
    out = {}
    with open(os.path.join(HERE, "golden", "face_weights.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = [int(x) for x in line.split()]
            out[parts[0]] = np.array(parts[2:], dtype=np.float64) / parts[1]
    return out


@pytest.mark.parametrize("r", [5, 7, 9])
def test_linear_face_weights_match_textbook(oracle, r):
    w = _golden_face_weights()[r]
    p = Params(order=r)
    n = r
    for m in range(n):
        e = np.zeros(n)
        e[m] = 1.0
        # all-zero strengths: the linear r-th order polynomial
        out, lvl = oracle.poly(p, e, np.zeros(n - 1), [0.0, -1.0])
        assert lvl == r
        assert abs(out[0] - w[m]) < 1e-14
        # left face value is the mirror image
        assert abs(out[1] - w[n - 1 - m]) < 1e-14


def test_zero_mean_basis(oracle):
    x, wq = np.polynomial.legendre.leggauss(10)
    xi = -0.5 + 0.5 * x
    for k in range(1, 9):
        vals = np.array([oracle.zk(k, t) for t in xi])
        assert abs(np.sum(0.5 * wq * vals)) < 1e-15
        # Z_k - xi^k is a constant
        d = vals - xi ** k
        assert np.ptp(d) < 1e-15


def _poly_cell_avg(coef, a, b):
    """Average of sum c_k x^k over [a, b]."""
    P = np.polynomial.polynomial.Polynomial(coef).integ()
    return (P(b) - P(a)) / (b - a)


@pytest.mark.parametrize("r", [3, 5, 7, 9])
def test_polynomial_exactness(oracle, r):
    """Cell averages of a degree <= r-1 polynomial give exact point values."""
    rng = np.random.default_rng(r)
    R = (r - 1) // 2
    p = Params(order=r)
    G = max(1, (r - 1) // 2)
    node = np.polynomial.legendre.leggauss(G)[0] / 2
    xi = np.concatenate([[0.0, -1.0], -0.5 + node])
    for deg in range(0, r):
        coef = rng.normal(size=deg + 1)
        W = np.array([_poly_cell_avg(coef, m - 1, m) for m in range(-R, R + 1)])
        out, lvl = oracle.poly(p, W, np.zeros(2 * R), xi)
        exact = np.polynomial.polynomial.polyval(xi, coef)
        assert np.max(np.abs(out - exact)) < 1e-12, (deg, out - exact)
    coef = np.zeros(r + 1)
    coef[r] = 1.0
    W = np.array([_poly_cell_avg(coef, m - 1, m) for m in range(-R, R + 1)])
    out, _ = oracle.poly(p, W, np.zeros(2 * R), xi)
    assert np.max(np.abs(out - np.polynomial.polynomial.polyval(xi, coef))) > 1e-6


def test_beta3_equals_jiang_shu(oracle):
    rng = np.random.default_rng(3)
    for _ in range(20):
        W = rng.normal(size=5)  # W[-2..2] at W[0..4]
        Wm2, Wm1, W0, W1, W2 = W
        js = [13 / 12 * (Wm2 - 2 * Wm1 + W0) ** 2 + 0.25 * (Wm2 - 4 * Wm1 + 3 * W0) ** 2,
              13 / 12 * (Wm1 - 2 * W0 + W1) ** 2 + 0.25 * (Wm1 - W1) ** 2,
              13 / 12 * (W0 - 2 * W1 + W2) ** 2 + 0.25 * (3 * W0 - 4 * W1 + W2) ** 2]
        for k, sub in enumerate((-1, 0, 1)):
            a = oracle.coeffs(3, sub, W)
            b = oracle.beta3(a)
            assert abs(b - js[k]) <= 1e-13 * max(1.0, js[k])


def test_remark3_taylor_series(oracle):
    """beta3_k = W'^2 h^2 + (13/12 W''^2 + c_k W' W''') h^4 + O(h^5), c = -2/3, 1/3, -2/3,
    for point samples W_j = W(x_i + j h) (Remark 3)."""
    f = lambda x: np.sin(1.3 * x) + 0.4 * np.exp(0.7 * x)
    d1 = lambda x: 1.3 * np.cos(1.3 * x) + 0.28 * np.exp(0.7 * x)
    d2 = lambda x: -1.69 * np.sin(1.3 * x) + 0.196 * np.exp(0.7 * x)
    d3 = lambda x: -2.197 * np.cos(1.3 * x) + 0.1372 * np.exp(0.7 * x)
    x0 = 0.37
    cs = (-2 / 3, 1 / 3, -2 / 3)
    for k, sub in enumerate((-1, 0, 1)):
        res = []
        for h in (0.04, 0.02, 0.01):
            W = f(x0 + h * np.arange(-2, 3))
            b = oracle.beta3(oracle.coeffs(3, sub, W))
            series = d1(x0) ** 2 * h ** 2 + (13 / 12 * d2(x0) ** 2 + cs[k] * d1(x0) * d3(x0)) * h ** 4
            res.append(abs(b - series))
        # remainder is O(h^5): halving h divides it by ~32
        assert res[1] / res[2] > 20 and res[0] / res[1] > 20, res


def test_weno_ao_special_cases(oracle):
    p = Params(order=5)
    xi = np.array([0.0, -1.0, -0.3])
    # constant data: W0 for any DF factors (exact in exact arithmetic; the
    # omega-weighted combination rounds at the last place)
    for al in ([1, 1, 1, 1], [0.3, 0.2, 0.9, 0.1], [0, 0, 0, 0]):
        out = oracle.weno_ao53(p, np.full(5, 1.7), np.array(al, float), xi)
        assert np.max(np.abs(out - 1.7)) <= 4 * np.spacing(1.7)
    # all DF factors 0: first order
    W = np.array([1.0, 3.0, 2.0, 7.0, 5.0])
    out = oracle.weno_ao53(p, W, np.zeros(4), xi)
    assert np.max(np.abs(out - 2.0)) < 1e-14
    # linear data, alpha = 1: tau_Z = 0, omega = d, result = P5 = exact line
    W = 0.5 + 2.0 * (np.arange(-2, 3) - 0.5)        # averages of 0.5 + 2 x on [m-1, m]
    out = oracle.weno_ao53(p, W, np.ones(4), xi)
    assert np.max(np.abs(out - (0.5 + 2.0 * xi))) < 1e-14
    # the linear weights sum to one
    d5 = p.d_hi
    d3m = (1 - p.d_hi) * (1 - p.d_lo) / 2
    assert abs(d5 + 2 * d3m + (1 - p.d_hi) * p.d_lo - 1.0) < 1e-15


def test_df_alpha(oracle):
    assert oracle.alpha(0.0, 2.0) == 1.0
    assert oracle.alpha(1.999999, 2.0) == 1.0
    assert oracle.alpha(2.0, 2.0) == 1.0
    assert oracle.alpha(4.0, 2.0) == 0.5
    assert oracle.alpha(math.inf, 2.0) == 0.0
    prev = 1.0
    for A in np.linspace(2.0, 50.0, 100):
        a = oracle.alpha(A, 2.0)
        assert 0 < a <= prev
        prev = a


_RANK = {2: 0, 5: 1, 7: 2, 9: 3}


def test_df_level_rule_brute_force(oracle):
    """Exhaustive small patterns of face strengths around a 9-cell stencil."""
    p = Params(order=9)
    rng = np.random.default_rng(9)
    W = rng.normal(size=9)
    levels = (0.0, 0.4, 1.5)
    import itertools
    seen = set()
    for pat in itertools.product(levels, repeat=8):
        s = np.array(pat)
        out, lvl = oracle.poly(p, W, s, [0.0, -1.0])
        seen.add(lvl)
        # the level depends only on the strengths inside the chosen stencil:
        # the linear L-stencil spans faces 4-(L-1)/2 .. 3+(L-1)/2
        if lvl in (5, 7, 9):
            h = (lvl - 1) // 2
            inner = s[4 - h:4 + h]
            assert inner.sum() <= p.sigma_thres
        # mirror symmetry: reversed data gives the mirrored values
        out_m, lvl_m = oracle.poly(p, W[::-1].copy(), s[::-1].copy(), [0.0, -1.0])
        assert lvl_m == lvl
        assert abs(out_m[0] - out[1]) < 1e-12 and abs(out_m[1] - out[0]) < 1e-12
    assert seen == {2, 5, 7, 9}
    # monotone: raising any strength never raises the level
    for _ in range(300):
        s = rng.choice(levels, size=8)
        _, l0 = oracle.poly(p, W, s, [0.0])
        k = rng.integers(8)
        s2 = s.copy()
        s2[k] += rng.uniform(0, 2)
        _, l1 = oracle.poly(p, W, s2, [0.0])
        assert _RANK[l1] <= _RANK[l0]


def test_df_strong_discontinuity_gives_first_order(oracle):
    """Remark 4: alpha -> 0 reduces the reconstruction to W_0."""
    for r in (3, 5, 7, 9):
        p = Params(order=r)
        R = (r - 1) // 2
        W = np.arange(2 * R + 1, dtype=float) ** 2
        s = np.full(2 * R, 1e300)
        out, _ = oracle.poly(p, W, s, [0.0, -1.0, -0.5])
        assert np.max(np.abs(out - W[R])) < 1e-12


def test_gauss_legendre(oracle):
    for G in (1, 2, 3, 4):
        node, eta = oracle.gauss(G)
        x, w = np.polynomial.legendre.leggauss(G)
        assert np.max(np.abs(node - x / 2)) < 1e-15
        assert np.max(np.abs(eta - w / 2)) < 1e-15


def test_sigma_point_values(oracle):
    from paper_2410_05489_amd.workloads import Grid, conservative
    g2 = Grid(dim=2, nx=4, ny=4, ng=5, dx=1, dy=1)
    p = Params(order=9)
    W = conservative(1.2, 0.3, -0.4, 0.9, 1.4, 2)
    assert oracle.sigma_point(g2, p, W, W, 0) == 0.0
    # pressure jump only, at rest: |dp|/pl + |dp|/pr
    Wl = conservative(1.0, 0.0, 0.0, 1.0, 1.4, 2)
    Wr = conservative(1.0, 0.0, 0.0, 2.0, 1.4, 2)
    assert abs(oracle.sigma_point(g2, p, Wl, Wr, 0) - 1.5) < 1e-15
    # normal velocity jump at equal p, rho: (du/c)^2 with c = sqrt(1.4)
    Wl = conservative(1.0, 0.5, 0.0, 1.0, 1.4, 2)
    Wr = conservative(1.0, -0.5, 0.0, 1.0, 1.4, 2)
    assert abs(oracle.sigma_point(g2, p, Wl, Wr, 0) - 1.0 / 1.4) < 1e-15
    # the same jump is tangential on a y-face
    assert abs(oracle.sigma_point(g2, p, Wl, Wr, 1) - 1.0 / 1.4) < 1e-15
    # non-physical side
    Wbad = np.array([1.0, 0.0, 0.0, -1.0])
    assert oracle.sigma_point(g2, p, Wl, Wbad, 0) == math.inf


def test_lf_flux_consistency(oracle):
    from paper_2410_05489_amd.workloads import Grid, conservative
    g2 = Grid(dim=2, nx=4, ny=4, ng=5, dx=1, dy=1)
    p = Params(order=9)
    rho, u, v, pr = 0.8, 0.3, -0.7, 1.1
    W = conservative(rho, u, v, pr, 1.4, 2)
    E = W[3]
    Fx = np.array([rho * u, rho * u * u + pr, rho * u * v, u * (E + pr)])
    Fy = np.array([rho * v, rho * u * v, rho * v * v + pr, v * (E + pr)])
    assert np.allclose(oracle.lf_point(g2, p, W, W, 0), Fx, rtol=1e-15, atol=1e-15)
    assert np.allclose(oracle.lf_point(g2, p, W, W, 1), Fy, rtol=1e-15, atol=1e-15)
    # rotational symmetry: an x-face problem with u, v swapped is the y-face problem
    Wl = conservative(1.0, 0.2, 0.5, 1.0, 1.4, 2)
    Wr = conservative(0.4, -0.1, 0.3, 0.6, 1.4, 2)
    sw = lambda w: np.array([w[0], w[2], w[1], w[3]])
    Fxs = oracle.lf_point(g2, p, Wl, Wr, 0)
    Fys = oracle.lf_point(g2, p, sw(Wl), sw(Wr), 1)
    assert np.allclose(sw(Fys), Fxs, rtol=1e-14, atol=1e-15)
    # dissipation term: max signal speed times the jump
    g1 = Grid(dim=1, nx=4, ny=1, ng=5, dx=1, dy=1)
    Wl1 = conservative(1.0, 0.0, 0.0, 1.0, 1.4, 1)
    Wr1 = conservative(0.5, 0.0, 0.0, 1.0, 1.4, 1)
    F = oracle.lf_point(g1, p, Wl1, Wr1, 0)
    smax = math.sqrt(1.4 / 0.5)
    assert abs(F[0] - (-0.5 * smax * (0.5 - 1.0))) < 1e-15
