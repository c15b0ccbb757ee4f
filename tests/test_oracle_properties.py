"""Property tests of the oracle's reconstruction and strength on generated
stencils and states (hypothesis): invariants the method has for any data,
whatever level the DF rule picks.
  - a constant stencil reconstructs to that constant at every point (to
    rounding);
  - adding a constant to the data adds it to every reconstructed value
    (all candidate polynomials and smoothness indicators depend on
    differences only);
  - mirrored data and strengths give the mirrored face values and the same
    level;
  - raising face strengths never raises the level;
  - the strength of a face is symmetric in its two states, zero for equal
    states, non-negative, and +inf for a non-physical side.
"""
import math

import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import oracle as O
from paper_2410_05489_amd.workloads import Grid, Params, conservative

ORDERS = st.sampled_from([3, 5, 7, 9])
VALUE = st.floats(min_value=-50.0, max_value=50.0, allow_nan=False, allow_infinity=False)
STRENGTH = st.one_of(st.floats(min_value=0.0, max_value=10.0, allow_nan=False),
                     st.sampled_from([0.0, 2.0, 1e300]))
_RANK = {3: 0, 2: 0, 5: 1, 7: 2, 9: 3}


def _stencil(draw, r):
    R = (r - 1) // 2
    W = np.array(draw(st.lists(VALUE, min_size=2 * R + 1, max_size=2 * R + 1)))
    s = np.array(draw(st.lists(STRENGTH, min_size=2 * R, max_size=2 * R)))
    return W, s


@st.composite
def stencils(draw):
    r = draw(ORDERS)
    W, s = _stencil(draw, r)
    return r, W, s


XI = [0.0, -1.0, -0.5, -0.5 - 0.4305681557970263, -0.5 + 0.1699905217924281]


@settings(max_examples=150, deadline=None)
@given(stencils(), VALUE)
def test_constant_data_is_reproduced(case, c):
    """To rounding: the polynomial coefficients are weighted sums of the data
    whose weights sum to zero (and the WENO-AO recombination to one) only in
    exact arithmetic."""
    r, W, s = case
    out, _ = O.poly(Params(order=r), np.full_like(W, c), s, XI)
    assert np.max(np.abs(out - c)) <= 1e-14 * max(1.0, abs(c))


@settings(max_examples=150, deadline=None)
@given(stencils(), st.floats(min_value=-20.0, max_value=20.0, allow_nan=False))
def test_shift_invariance(case, b):
    r, W, s = case
    p = Params(order=r)
    out, lvl = O.poly(p, W, s, XI)
    out_b, lvl_b = O.poly(p, W + b, s, XI)
    assert lvl_b == lvl
    scale = max(1.0, float(np.abs(W).max()) + abs(b))
    assert np.max(np.abs(out_b - (out + b))) <= 1e-12 * scale


@settings(max_examples=150, deadline=None)
@given(stencils())
def test_mirror_symmetry(case):
    r, W, s = case
    p = Params(order=r)
    out, lvl = O.poly(p, W, s, [0.0, -1.0])
    out_m, lvl_m = O.poly(p, W[::-1].copy(), s[::-1].copy(), [0.0, -1.0])
    assert lvl_m == lvl
    scale = max(1.0, float(np.abs(W).max()))
    assert abs(out_m[0] - out[1]) <= 1e-12 * scale and abs(out_m[1] - out[0]) <= 1e-12 * scale


@settings(max_examples=150, deadline=None)
@given(stencils(), st.integers(min_value=0, max_value=7), st.floats(min_value=0.0, max_value=5.0))
def test_stronger_faces_never_raise_the_level(case, k, extra):
    r, W, s = case
    p = Params(order=r)
    _, l0 = O.poly(p, W, s, [0.0])
    s2 = s.copy()
    s2[k % len(s2)] += extra
    _, l1 = O.poly(p, W, s2, [0.0])
    assert _RANK[l1] <= _RANK[l0]


STATE = st.tuples(st.floats(min_value=0.05, max_value=5.0), st.floats(min_value=-3.0, max_value=3.0),
                  st.floats(min_value=-3.0, max_value=3.0), st.floats(min_value=0.05, max_value=5.0))
G2 = Grid(dim=2, nx=4, ny=4, ng=5, dx=1, dy=1)


@settings(max_examples=200, deadline=None)
@given(STATE, STATE, st.sampled_from([0, 1]))
def test_strength_is_symmetric_nonnegative_and_zero_on_equal_states(a, b, d):
    p = Params(order=9)
    Wa = conservative(*a, 1.4, 2)
    Wb = conservative(*b, 1.4, 2)
    s_ab = O.sigma_point(G2, p, Wa, Wb, d)
    s_ba = O.sigma_point(G2, p, Wb, Wa, d)
    assert s_ab >= 0.0 and math.isfinite(s_ab)
    assert abs(s_ab - s_ba) <= 1e-14 * max(1.0, s_ab)
    assert O.sigma_point(G2, p, Wa, Wa, d) == 0.0


@settings(max_examples=100, deadline=None)
@given(STATE, st.floats(min_value=-5.0, max_value=-1e-3), st.sampled_from([0, 1]))
def test_strength_of_a_non_physical_side_is_infinite(a, p_bad, d):
    """(p is recomputed from the conservative state: a pressure of exactly 0
    can come back as a rounding-size positive one, a physical state.)"""
    p = Params(order=9)
    Wa = conservative(*a, 1.4, 2)
    Wbad = conservative(a[0], a[1], a[2], p_bad, 1.4, 2)   # p < 0
    assert O.sigma_point(G2, p, Wa, Wbad, d) == math.inf
    assert O.sigma_point(G2, p, Wbad, Wa, d) == math.inf
