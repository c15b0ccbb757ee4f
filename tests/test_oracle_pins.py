"""Independent pins of two parts of the oracle that the other formula and
solver tests cannot tell apart from plausible mistakes:

1. The nonlinear weight law of the WENO-Z-AO(5,3) fallback (Sec. 3.2,
   omega_k = d_k (1 + tau_Z^2 / (beta_k + eps)^2)).  The weights are read
   back from the oracle's reconstructed polynomial itself: it must be a
   combination of the four candidate polynomials (fitted here from their
   cell averages), and the combination coefficients give the normalised
   weights.  When one sub-stencil holds a jump, tau_Z dwarfs the indicators
   of the two smooth sub-stencils and the ratio of their weights tends to
   (d_j / d_k) ((beta_k + eps) / (beta_j + eps))^2, with beta_k the
   smoothness indicator of Eq. (LocalSmoothnessIndicator) computed here by
   quadrature of the fitted polynomials.  The exponent, the epsilon and
   the linear weights are all visible in that limit.

2. The DF strengths of the tangential reconstruction (Sec. 3.1, Remark 2):
   each side of a face uses the strengths of its own cell's column (row).
   Mirroring the problem in x (or in y), with the normal velocity negated,
   must mirror the solution; a rule that takes one fixed side's column for
   both sides breaks that symmetry where the two columns see different
   discontinuities, which four-quadrant data provide at the quadrant
   corner.  (x <-> y transposition cannot see such a mistake: it maps the
   left side onto the lower one.)
"""
import numpy as np
import pytest

from paper_2410_05489_amd import workloads as WL
from paper_2410_05489_amd.workloads import Params

# ---------------------------------------------------------------------------
# 1. WENO-Z weights
# ---------------------------------------------------------------------------

D_HI = D_LO = 0.85                      # Sec. 3.2
D5 = D_HI
D3 = {-1: (1 - D_HI) * (1 - D_LO) / 2, 0: (1 - D_HI) * D_LO, 1: (1 - D_HI) * (1 - D_LO) / 2}


def _fit(cells, W):
    """Coefficients (ascending powers of xi) of the polynomial of degree
    len(cells)-1 whose average over cell m, xi in [m-1, m], is W[m]."""
    n = len(cells)
    A = np.array([[(m ** (k + 1) - (m - 1) ** (k + 1)) / (k + 1) for k in range(n)] for m in cells], float)
    return np.linalg.solve(A, np.array([W[m] for m in cells], float))


def _ev(c, xi):
    return np.polynomial.polynomial.polyval(xi, c)


def _beta(c):
    """Eq. (LocalSmoothnessIndicator) over the cell xi in [-1, 0]: the sum
    over derivative orders q = 1..deg of the integral of (d^q P / dxi^q)^2
    (the powers of dx cancel in xi), by Gauss-Legendre quadrature."""
    x, w = np.polynomial.legendre.leggauss(8)
    x, w = 0.5 * (x - 1.0), 0.5 * w
    b = 0.0
    d = np.array(c, float)
    for _ in range(len(c) - 1):
        d = np.polynomial.polynomial.polyder(d)
        b += float(np.sum(w * _ev(d, x) ** 2))
    return b


def _weights_from_output(W, P, xi, alpha=(1.0, 1.0, 1.0, 1.0)):
    """Normalised weights (w5, w3[-1], w3[0], w3[1]) of the WENO-AO
    combination P = w5 (P5/d5 - sum d3_k/d5 P3_k) + sum w3_k P3_k of the
    (DF-damped) candidates, solved from the output values P(xi)."""
    W0 = W[0]
    cand = []
    for k in (-1, 0, 1):
        c = _fit([k - 1, k, k + 1], W)
        cand.append(W0 + alpha[k + 1] * (_ev(c, xi) - W0))
    c5 = _fit([-2, -1, 0, 1, 2], W)
    p5 = W0 + alpha[3] * (_ev(c5, xi) - W0)
    A = np.stack([p5] + cand, axis=1)
    coef, res, rank, _ = np.linalg.lstsq(A, P, rcond=None)
    assert rank == 4
    fit_err = float(np.max(np.abs(A @ coef - P)))
    w5 = coef[0] * D5
    w3 = [coef[1 + i] + w5 * D3[k] / D5 for i, k in enumerate((-1, 0, 1))]
    return w5, w3, fit_err


def _stencil(vals):
    return {m: v for m, v in zip(range(-2, 3), vals)}


XI = np.linspace(-1.0, 0.0, 11)


@pytest.mark.parametrize("vals,smooth", [
    ((0.0, 0.1, 0.3, 0.2, 100.0), (-1, 0)),      # jump between cells 1 and 2
    ((100.0, 0.2, 0.3, 0.1, 0.0), (0, 1)),       # its mirror image
    ((1.0, 1.4, 1.3, 1.9, -4000.0), (-1, 0)),
    ((-2500.0, 2.0, 2.5, 2.25, 2.0), (0, 1)),
])
def test_weno_z_weight_ratio_tends_to_the_squared_indicator_ratio(oracle, vals, smooth):
    W = _stencil(vals)
    p = Params(order=5)
    P = oracle.weno_ao53(p, np.array(vals, float), np.ones(4), XI)
    w5, w3, fit_err = _weights_from_output(W, P, XI)
    # the output is exactly a combination of the four candidates ...
    assert fit_err < 1e-12 * max(1.0, np.max(np.abs(P)))
    # ... with normalised, non-negative weights
    assert abs(w5 + sum(w3) - 1.0) < 1e-12
    assert w5 >= -1e-14 and min(w3) >= -1e-14
    j, k = smooth
    bj = _beta(_fit([j - 1, j, j + 1], W))
    bk = _beta(_fit([k - 1, k, k + 1], W))
    assert abs(bj / bk - 1.0) > 0.2            # the two smooth indicators differ
    eps = p.eps
    expect = (D3[j] / D3[k]) * ((bk + eps) / (bj + eps)) ** 2
    got = w3[j + 1] / w3[k + 1]
    assert abs(got / expect - 1.0) < 1e-7, (got, expect)


def test_weno_z_weights_scale_with_epsilon(oracle):
    """Two smooth sub-stencils whose indicators are of the size of eps: the
    ratio of their weights follows ((beta_k + eps) / (beta_j + eps))^2 with
    eps where the weight law puts it, for two values of eps."""
    dl = 1e-3
    vals = (0.0, dl, 2 * dl, 4 * dl, 60.0)     # linear, then bending, then a jump
    W = _stencil(vals)
    bm = _beta(_fit([-2, -1, 0], W))
    b0 = _beta(_fit([-1, 0, 1], W))
    assert 0.5e-6 < bm < 2e-6 and b0 > 2 * bm
    ratios = []
    for eps in (1e-6, 4e-6):
        p = Params(order=5, eps=eps)
        P = oracle.weno_ao53(p, np.array(vals, float), np.ones(4), XI)
        w5, w3, _ = _weights_from_output(W, P, XI)
        r = w3[0] / w3[1]
        assert abs(r / ((D3[-1] / D3[0]) * ((b0 + eps) / (bm + eps)) ** 2) - 1.0) < 1e-7
        ratios.append(r)
    assert abs(ratios[0] / ratios[1] - 1.0) > 0.05   # eps is visible in the ratio


def test_weno_z_weights_through_the_stencil_selection(oracle):
    """The fallback as the reconstruction selects it: face strengths whose
    sub-stencil sums stay below the threshold but whose 5-cell sum does not
    give alpha(S^{r3}) = 1 and alpha(S^{r5}) = thres / A5 (Sec. 3.1); the
    weights read back from the output obey the same limit."""
    vals = (0.0, 0.1, 0.3, 0.2, 100.0)
    W = _stencil(vals)
    p = Params(order=5)
    s = np.full(4, 0.6)                        # A3 = 1.2 < 2, A5 = 2.4 >= 2
    P, lvl = oracle.poly(p, np.array(vals, float), s, XI)
    assert lvl == 2
    a5 = p.sigma_thres / 2.4
    w5, w3, fit_err = _weights_from_output(W, P, XI, alpha=(1.0, 1.0, 1.0, a5))
    assert fit_err < 1e-12 * np.max(np.abs(P))
    b_m, b_0 = _beta(_fit([-2, -1, 0], W)), _beta(_fit([-1, 0, 1], W))
    expect = (D3[-1] / D3[0]) * ((b_0 + p.eps) / (b_m + p.eps)) ** 2
    assert abs(w3[0] / w3[1] / expect - 1.0) < 1e-7


# ---------------------------------------------------------------------------
# 2. Tangential DF column (Remark 2): mirror symmetry in x and in y
# ---------------------------------------------------------------------------

QUAD = ((1.5, 0.0, 0.0, 1.5), (0.5323, 1.206, 0.0, 0.3), (0.138, 1.206, 1.206, 0.129), (0.5323, 0.0, 1.206, 0.3))


def _mirror(U, axis, g):
    """Interior of U mirrored along axis (1 = y rows, 2 = x columns), the
    momentum normal to the mirror negated."""
    a = g.interior(U)
    a = np.flip(a, axis=axis).copy()
    a[1 if axis == 2 else 2] *= -1.0
    return a


@pytest.mark.parametrize("axis", [2, 1])
@pytest.mark.parametrize("order,n,split", [(9, 36, (0.6, 0.45)), (5, 30, (0.55, 0.4)), (7, 33, (0.5, 0.62))])
def test_mirror_symmetry_2d(oracle, axis, order, n, split):
    """One problem and its mirror image (four-quadrant data with the
    quadrant lines off the centre, so the mirror is a different problem)
    give mirrored states over several steps, to round-off, with
    WENO-Z-AO cells present in both directions' tangential reconstruction."""
    a = WL.four_quadrant(n, order, states=QUAD, split=split)
    a.params.positivity_fallback = 1
    g = a.grid
    # the mirrored initial state, in the same grid layout
    Ub = a.U.copy()
    Ub[:, g.ng:g.ng + g.ny, g.ng:g.ng + g.nx] = _mirror(a.U, axis, g)
    # the fallback is used where the tangential stencils cross the corner
    sx, sy = oracle.sigma_init(g, a.params, a.U.copy())
    for d in (0, 1):
        _, _, lvl = oracle.reconstruct(g, a.params, d, a.U.copy(), sx, sy, want_level=True)
        assert np.any(lvl == 2) and np.any(lvl == order)
    Ua, _, _, _, _ = oracle.run(g, a.params, a.U, 8)
    Ubr, _, _, _, _ = oracle.run(g, a.params, Ub, 8)
    ia = g.interior(Ua)
    ib = _mirror(Ubr, axis, g)
    scale = np.abs(ia).max(axis=(1, 2), keepdims=True)
    assert np.isfinite(ia).all()
    assert np.max(np.abs(ia - ib) / scale) < 1e-12
