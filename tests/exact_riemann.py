"""Exact solution of the 1D Euler Riemann problem for an ideal gas.

Textbook construction (Toro, "Riemann Solvers and Numerical Methods for
Fluid Dynamics", ch. 4): the star pressure is the root of
f_L(p) + f_R(p) + (u_R - u_L) = 0, with the shock (Rankine-Hugoniot) or
rarefaction (isentropic) branch on each side, solved here by bisection;
the self-similar solution is then sampled at x/t.  Independent of the
oracle; used only to pin it.
"""
import math

import numpy as np


def _f(p, rho, pk, gamma):
    a = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * a / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(left, right, gamma=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    g = lambda p: _f(p, rl, pl, gamma) + _f(p, rr, pr, gamma) + (ur - ul)
    lo, hi = 1e-14, 10.0 * max(pl, pr) + 10.0
    while g(hi) < 0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (_f(ps, rr, pr, gamma) - _f(ps, rl, pl, gamma))
    return ps, us


def sample(left, right, xi, gamma=1.4):
    """(rho, u, p) at similarity coordinate xi = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    gm1, gp1 = gamma - 1.0, gamma + 1.0
    if xi <= us:  # left of contact
        al = math.sqrt(gamma * pl / rl)
        if ps > pl:  # left shock
            S = ul - al * math.sqrt(gp1 / (2 * gamma) * ps / pl + gm1 / (2 * gamma))
            if xi < S:
                return rl, ul, pl
            r = rl * (ps / pl + gm1 / gp1) / (gm1 / gp1 * ps / pl + 1.0)
            return r, us, ps
        ast = al * (ps / pl) ** (gm1 / (2 * gamma))
        if xi < ul - al:
            return rl, ul, pl
        if xi > us - ast:
            return rl * (ps / pl) ** (1.0 / gamma), us, ps
        c = 2.0 / gp1 + gm1 / (gp1 * al) * (ul - xi)
        return rl * c ** (2.0 / gm1), 2.0 / gp1 * (al + gm1 / 2.0 * ul + xi), pl * c ** (2.0 * gamma / gm1)
    ar = math.sqrt(gamma * pr / rr)
    if ps > pr:  # right shock
        S = ur + ar * math.sqrt(gp1 / (2 * gamma) * ps / pr + gm1 / (2 * gamma))
        if xi > S:
            return rr, ur, pr
        r = rr * (ps / pr + gm1 / gp1) / (gm1 / gp1 * ps / pr + 1.0)
        return r, us, ps
    ast = ar * (ps / pr) ** (gm1 / (2 * gamma))
    if xi > ur + ar:
        return rr, ur, pr
    if xi < us + ast:
        return rr * (ps / pr) ** (1.0 / gamma), us, ps
    c = 2.0 / gp1 - gm1 / (gp1 * ar) * (ur - xi)
    return rr * c ** (2.0 / gm1), 2.0 / gp1 * (-ar + gm1 / 2.0 * ur + xi), pr * c ** (2.0 * gamma / gm1)


def cell_average_density(left, right, n, t, x0=0.5, gamma=1.4, sub=64):
    """Cell averages of rho on [0,1] with n cells (midpoint rule, sub points)."""
    dx = 1.0 / n
    out = np.zeros(n)
    for i in range(n):
        xs = (i + (np.arange(sub) + 0.5) / sub) * dx
        out[i] = np.mean([sample(left, right, (x - x0) / t, gamma)[0] for x in xs])
    return out
