"""Reference discrete adjoint of the 1D ASE-DF step -- TEST INFRASTRUCTURE ONLY.

A second, independent statement of the 1D method (Sec. 2.1, 2.3, 3.1-3.4
and Algorithm 1 of the paper) written with plain PyTorch CPU ops in float64,
so that torch.autograd yields the exact transposed Jacobian of one SSP-RK3
step.  The adjoint convention: the time step, the DF strengths (hence every
DF factor and stencil level), the side that gives the LF signal speed and
the positivity replacements are frozen at their forward values; everything
else -- reconstruction (including the WENO-Z-AO weights), fluxes, the
stage combinations and the boundary copies -- is differentiated.

Readings are the oracle's (design notes R1-R18).  Pinned against the C
oracle's forward step (same states to rounding) and against central finite
differences of the C oracle with the time step and strengths replayed.
"""
from __future__ import annotations

import math

import torch

TD = torch.float64


def _zk(k: int, xi: float) -> float:
    return xi ** k - ((-1) ** k) / (k + 1)


# Zero-mean polynomial coefficients of each stencil (Sec. 3.2-3.4), as
# functions of the shifted cell averages W(m) (m = offset from the cell).
def _coef5(W):
    return [(-15 * W(0) + W(-1) + 15 * W(1) - W(2)) / 12,
            (-8 * W(0) + 6 * W(-1) - W(-2) + 2 * W(1) + W(2)) / 8,
            (3 * W(0) - W(-1) - 3 * W(1) + W(2)) / 6,
            (6 * W(0) - 4 * W(-1) + W(-2) - 4 * W(1) + W(2)) / 24]


def _coef7(W):
    return [(-245 * W(0) + 25 * W(-1) - 2 * W(-2) + 245 * W(1) - 25 * W(2) + 2 * W(3)) / 180,
            (-230 * W(0) + 210 * W(-1) - 57 * W(-2) + 7 * W(-3) + 15 * W(1) + 63 * W(2) - 8 * W(3)) / 240,
            (28 * W(0) - 11 * W(-1) + W(-2) - 28 * W(1) + 11 * W(2) - W(3)) / 36,
            (46 * W(0) - 39 * W(-1) + 15 * W(-2) - 2 * W(-3) - 24 * W(1) + 3 * W(2) + W(3)) / 144,
            (-10 * W(0) + 5 * W(-1) - W(-2) + 10 * W(1) - 5 * W(2) + W(3)) / 120,
            (-20 * W(0) + 15 * W(-1) - 6 * W(-2) + W(-3) + 15 * W(1) - 6 * W(2) + W(3)) / 720]


def _coef9(W):
    return [(-7175 * W(0) + 889 * W(-1) - 119 * W(-2) + 9 * W(-3) + 7175 * W(1) - 889 * W(2) + 119 * W(3)
             - 9 * W(4)) / 5040,
            (-27895 * W(0) + 28679 * W(-1) - 9835 * W(-2) + 2081 * W(-3) - 205 * W(-4) - 2065 * W(1)
             + 11459 * W(2) - 2455 * W(3) + 236 * W(4)) / 30240,
            (1365 * W(0) - 587 * W(-1) + 89 * W(-2) - 7 * W(-3) - 1365 * W(1) + 587 * W(2) - 89 * W(3)
             + 7 * W(4)) / 1440,
            (1174 * W(0) - 1160 * W(-1) + 556 * W(-2) - 128 * W(-3) + 13 * W(-4) - 464 * W(1) - 68 * W(2)
             + 88 * W(3) - 11 * W(4)) / 3456,
            (-75 * W(0) + 41 * W(-1) - 11 * W(-2) + W(-3) + 75 * W(1) - 41 * W(2) + 11 * W(3) - W(4)) / 480,
            (-380 * W(0) + 334 * W(-1) - 170 * W(-2) + 46 * W(-3) - 5 * W(-4) + 250 * W(1) - 86 * W(2)
             + 10 * W(3) + W(4)) / 8640,
            (35 * W(0) - 21 * W(-1) + 7 * W(-2) - W(-3) - 35 * W(1) + 21 * W(2) - 7 * W(3) + W(4)) / 5040,
            (70 * W(0) - 56 * W(-1) + 28 * W(-2) - 8 * W(-3) + W(-4) - 56 * W(1) + 28 * W(2) - 8 * W(3)
             + W(4)) / 40320]


def _sub3(W, k):
    if k == -1:
        return 2 * W(0) - 3 * W(-1) + W(-2), 0.5 * (W(-2) - 2 * W(-1) + W(0))
    if k == 0:
        return W(1) - W(0), 0.5 * (W(-1) - 2 * W(0) + W(1))
    return W(1) - W(0), 0.5 * (W(0) - 2 * W(1) + W(2))


def _poly(W0, coefs, xi):
    P = W0
    for k, a in enumerate(coefs, start=1):
        P = P + a * _zk(k, xi)
    return P


def _alpha(A, thr):
    # DF factor; the strengths are frozen, so this is a constant tensor
    return torch.where(A < thr, torch.ones_like(A), thr / A)


class Step1D:
    """One SSP-RK3 step of a 1D grid with frozen decisions.

    ncell, ng, dx, order, bc ('periodic' | 'transmissive' | 'reflective'), gamma,
    sigma_thres, eps, d_hi, d_lo, positivity (bool), df_first_order (bool).
    """

    def __init__(self, ncell, ng, dx, order, bc, gamma=1.4, sigma_thres=2.0, eps=1e-6, d_hi=0.85, d_lo=0.85,
                 positivity=False, df_first_order=False):
        self.N, self.ng, self.dx, self.r = ncell, ng, dx, order
        self.R = (order - 1) // 2
        self.bc = bc
        self.gamma, self.thr, self.eps = gamma, sigma_thres, eps
        self.d5 = d_hi
        self.d3 = [(1 - d_hi) * (1 - d_lo) / 2, (1 - d_hi) * d_lo, (1 - d_hi) * (1 - d_lo) / 2]
        self.positivity = positivity
        self.fo = df_first_order

    # -- pieces -------------------------------------------------------------
    def ghost(self, U):
        """U: [3, N] interior -> [3, N + 2 ng] with ghost copies (differentiable)."""
        N, ng = self.N, self.ng
        if self.bc == "periodic":
            left, right = U[:, N - ng:], U[:, :ng]
        elif self.bc == "reflective":
            # slip wall: mirrored cells, momentum reversed
            sign = torch.tensor([1.0, -1.0, 1.0], dtype=TD)[:, None]
            left = sign * torch.flip(U[:, :ng], dims=[1])
            right = sign * torch.flip(U[:, N - ng:], dims=[1])
        else:
            left, right = U[:, :1].expand(3, ng), U[:, N - 1:].expand(3, ng)
        return torch.cat([left, U, right], dim=1)

    def prim(self, W):
        rho, m, E = W[0], W[1], W[2]
        u = m / rho
        p = (self.gamma - 1) * (E - 0.5 * rho * (u * u))
        c = torch.sqrt(self.gamma * p / rho)
        return rho, u, p, c

    def sigma(self, Wl, Wr):
        """Strength of the faces from left/right states (no gradient)."""
        with torch.no_grad():
            rl, ul, pl, cl = self.prim(Wl)
            rr, ur, pr, cr = self.prim(Wr)
            dp = (pl - pr).abs()
            s = dp / pl + dp / pr + (ul / cl - ur / cr) ** 2 + (0.0 / cl - 0.0 / cr) ** 2
            bad = ~((rl > 0) & (pl > 0) & (rr > 0) & (pr > 0))
            return torch.where(bad, torch.full_like(s, math.inf), s)

    def sigma_fill(self, Ug, sig):
        """Strengths of every stored face: flux faces from `sig`, the others
        by periodic wrap or wall mirror (face f -> -f-2 at the left wall,
        2N-f-2 at the right one) or from the first-order states (no
        gradient)."""
        N, ng = self.N, self.ng
        NX = N + 2 * ng
        with torch.no_grad():
            out = sig.clone()
            fo = self.sigma(Ug[:, :-1].detach(), Ug[:, 1:].detach())   # face I between I, I+1
            for I in range(NX - 1):
                f = I - ng
                if self.fo:
                    out[I] = fo[I]
                elif -1 <= f <= N - 1:
                    continue
                elif self.bc == "periodic":
                    out[I] = sig[(f % N) + ng]
                elif self.bc == "reflective":
                    out[I] = sig[(-f - 2 if f < -1 else 2 * N - f - 2) + ng]
                else:
                    out[I] = fo[I]
            return out

    def cell_poly(self, Ug, sg, i):
        """Face values (xi = 0, xi = -1) of cell i (interior index, -1..N) for
        the three variables, as differentiable tensors."""
        ng, R, thr = self.ng, self.R, self.thr
        I = i + ng
        W = lambda m: Ug[:, I + m]                                       # noqa: E731
        s = lambda m: sg[I + m]                                          # face between m and m+1 # noqa: E731

        def A(lo, hi):
            a = torch.zeros((), dtype=TD)
            for m in range(lo, hi):
                a = a + s(m)
            return a

        if self.r == 3:
            al = _alpha(A(-1, 1), thr)
            a1, a2 = _sub3(W, 0)
            return [W(0) + al * (a1 * _zk(1, xi) + a2 * _zk(2, xi)) for xi in (0.0, -1.0)]
        if not (A(-2, 2) < thr or A(-2, 2) == thr):
            return self.weno_ao(W, [_alpha(A(-2, 0), thr), _alpha(A(-1, 1), thr), _alpha(A(0, 2), thr),
                                    _alpha(A(-2, 2), thr)])
        level = 5
        if self.r >= 7 and (A(-3, 3) < thr or A(-3, 3) == thr):
            level = 7
            if self.r >= 9 and (A(-4, 4) < thr or A(-4, 4) == thr):
                level = 9
        coefs = {5: _coef5, 7: _coef7, 9: _coef9}[level](W)
        return [_poly(W(0), coefs, xi) for xi in (0.0, -1.0)]

    def weno_ao(self, W, al):
        """WENO-Z-AO(5,3) with DF factors (Sec. 3.2), both face values."""
        a3 = [_sub3(W, k) for k in (-1, 0, 1)]
        b3 = [a1 * a1 - 2 * a1 * a2 + (4 / 3) * a2 * a2 + 4 * a2 * a2 for a1, a2 in a3]
        b5 = (b3[0] + 4 * b3[1] + b3[2]) / 6 + (b3[0] - b3[2]).abs()
        tz = ((b5 - b3[0]).abs() + (b5 - b3[1]).abs() + (b5 - b3[2]).abs()) / 3
        w5 = self.d5 * (1 + tz * tz / ((b5 + self.eps) ** 2))
        w3 = [self.d3[k] * (1 + tz * tz / ((b3[k] + self.eps) ** 2)) for k in range(3)]
        ws = w5 + w3[0] + w3[1] + w3[2]
        c5 = _coef5(W)
        out = []
        for xi in (0.0, -1.0):
            P3 = [W(0) + al[k] * (a3[k][0] * _zk(1, xi) + a3[k][1] * _zk(2, xi)) for k in range(3)]
            P5 = W(0) + al[3] * (c5[0] * _zk(1, xi) + c5[1] * _zk(2, xi) + c5[2] * _zk(3, xi) + c5[3] * _zk(4, xi))
            inner = P5 / self.d5
            for k in range(3):
                inner = inner - self.d3[k] / self.d5 * P3[k]
            P = w5 / ws * inner
            for k in range(3):
                P = P + w3[k] / ws * P3[k]
            out.append(P)
        return out

    def flux(self, Wl, Wr, Cl, Cr):
        """LF flux with frozen signal-speed side and positivity replacement."""
        g = self.gamma
        with torch.no_grad():
            rl, _, pl, _ = self.prim(Wl)
            rr, _, pr, _ = self.prim(Wr)
            badl = ~((rl > 0) & (pl > 0))
            badr = ~((rr > 0) & (pr > 0))
        if self.positivity:
            Wl = torch.where(badl, Cl, Wl)
            Wr = torch.where(badr, Cr, Wr)

        def F(W):
            rho, u, p, c = self.prim(W)
            return torch.stack([W[1], W[1] * u + p, u * (W[2] + p)]), u.abs() + c

        Fl, sl = F(Wl)
        Fr, sr = F(Wr)
        with torch.no_grad():
            take_l = sl > sr
        s = torch.where(take_l, sl, sr)
        return 0.5 * (Fl + Fr) - 0.5 * s * (Wr - Wl), Wl, Wr

    def residual(self, U, sig):
        """L(U) on the interior and the new flux-face strengths."""
        N, ng = self.N, self.ng
        Ug = self.ghost(U)
        sg = self.sigma_fill(Ug, sig)
        traces = [self.cell_poly(Ug, sg, i) for i in range(-1, N + 1)]   # cells -1..N
        Pr = torch.stack([t[0] for t in traces], dim=1)   # value at right face, [3, N+2]
        Pl = torch.stack([t[1] for t in traces], dim=1)   # value at left face
        Wl = Pr[:, :-1]            # faces -1/2 .. N-1/2: left state = right value of cell i
        Wr = Pl[:, 1:]
        Cl, Cr = Ug[:, ng - 1:ng + N], Ug[:, ng:ng + N + 1]
        F, Wlu, Wru = self.flux(Wl, Wr, Cl, Cr)
        L = -(F[:, 1:] - F[:, :-1]) / self.dx
        new = sig.clone()
        new[ng - 1:ng + N] = self.sigma(Wl.detach(), Wr.detach())
        return L, new

    def step(self, U, sig, dt):
        """One SSP-RK3 step; U interior [3, N] (may require grad), sig the
        state strengths [N + 2 ng]; returns (U_next, sig_next)."""
        L1, s1 = self.residual(U, sig)
        U1 = U + dt * L1
        L2, s2 = self.residual(U1, s1)
        U2 = 0.75 * U + 0.25 * U1 + 0.25 * dt * L2
        L3, s3 = self.residual(U2, s2)
        Un = (1.0 / 3.0) * U + (2.0 / 3.0) * U2 + (2.0 / 3.0) * dt * L3
        return Un, s3

    def vjp(self, U, sig, dt, lam):
        """lam^T d(step)/dU at U (frozen decisions)."""
        Ut = U.detach().clone().requires_grad_(True)
        Un, _ = self.step(Ut, sig, dt)
        (g,) = torch.autograd.grad(Un, Ut, grad_outputs=lam)
        return g
