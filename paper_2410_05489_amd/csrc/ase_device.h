// Device-side building blocks of the ASE-DF path for gfx950: the constant
// tables, the discontinuity-feedback level rule, the per-cell reconstruction
// (linear stencils and the WENO-Z-AO(5,3) fallback), Euler primitives, the
// discontinuity strength and the Lax-Friedrichs flux.
//
// Everything is FP64.  Linear reconstructions are applied as point-evaluation
// weights (the paper's zero-mean stencil coefficients contracted with the
// basis at the evaluation point, tabulated at compile time); the DF sums are
// formed left to right across the stencil.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace ase {

// Evaluation-point sets, per nominal order r in {3,5,7,9} (index r/2-1):
// point 0 is the right face (xi = 0), point 1 the left face (xi = -1) and
// points 2..2+G-1 the Gauss points xi = -1/2 + g_k of the face quadrature.
constexpr int kMaxPts = 6;
constexpr int kTaps = 9;  // stencil taps, centred on index 4

struct Tables {
    // lin[oi][li][q][t]: weight of tap t-4 for the linear stencil of level
    // li (0: 3-cell S^{r3}_0, 1: 5, 2: 7, 3: 9 cells) at point q of order oi.
    double lin[4][4][kMaxPts][kTaps];
    // z[oi][q][k-1] = Z_k(xi_q), k = 1..4 (zero-mean basis on [-1,0]).
    double z[4][kMaxPts][4];
    // Gauss weights eta_k per order (normalised to 1).
    double eta[4][4];
    // Slopes dP/dxi at the same points: dlin[oi][li][q][t] weights of the
    // linear levels, dz[oi][q][k-1] = dZ_k/dxi = k xi^(k-1).  Used by the
    // gas-kinetic flux.
    double dlin[4][4][kMaxPts][kTaps];
    double dz[4][kMaxPts][4];
    // The Gauss points are symmetric about the cell centre, and so are the
    // centred linear stencils: at the p-th point from the left and its
    // mirror image the weights of taps m and -m trade places.  sym[oi][li][p]
    // holds the even parts a_0..a_4 (a_m = (c_m + c_-m)/2) and, from index 5,
    // the odd parts b_1..b_4 (b_m = (c_m - c_-m)/2) of the weights c of the
    // p-th Gauss point; the point and its mirror are E + O and E - O with
    // E = a_0 W_0 + sum a_m (W_m + W_-m), O = sum b_m (W_m - W_-m).
    double sym[4][4][2][kTaps];
};

// ---------------------------------------------------------------------------
// Compile-time construction of the tables.  The kernels index them with
// compile-time constants, so every weight becomes an instruction literal.
//
// Stencil coefficients: the zero-mean polynomial coefficients W_xk of the 3-,
// 5-, 7- and 9-cell stencils printed in Sec. 3.2-3.4 (with W_3 for the
// misprinted f_3 of the 7-cell W_x1), as integer numerators over a common
// denominator, taps W_{-h}..W_{h}.  Zero-mean basis on the cell [-1,0]:
// Z_k(xi) = xi^k - (-1)^k/(k+1), under which those coefficients are the exact
// cell-average fit.  P(xi) = W_0 + sum_k W_xk Z_k(xi) is linear in the taps;
// its weights at each evaluation point are tabulated.
// ---------------------------------------------------------------------------
namespace tables {

struct Stencil {
    int h;           // half width
    int ncoef;       // coefficients W_x1..W_xn
    double den[8];
    double num[8][9];  // num[k][m+h]
};

constexpr Stencil kS3 = {1, 2, {1, 2}, {{0, -1, 1}, {1, -2, 1}}};
constexpr Stencil kS5 = {2, 4, {12, 8, 6, 24},
                         {{0, 1, -15, 15, -1}, {-1, 6, -8, 2, 1}, {0, -1, 3, -3, 1}, {1, -4, 6, -4, 1}}};
constexpr Stencil kS7 = {3, 6, {180, 240, 36, 144, 120, 720},
                         {{0, -2, 25, -245, 245, -25, 2},
                          {7, -57, 210, -230, 15, 63, -8},
                          {0, 1, -11, 28, -28, 11, -1},
                          {-2, 15, -39, 46, -24, 3, 1},
                          {0, -1, 5, -10, 10, -5, 1},
                          {1, -6, 15, -20, 15, -6, 1}}};
constexpr Stencil kS9 = {4, 8, {5040, 30240, 1440, 3456, 480, 8640, 5040, 40320},
                         {{0, 9, -119, 889, -7175, 7175, -889, 119, -9},
                          {-205, 2081, -9835, 28679, -27895, -2065, 11459, -2455, 236},
                          {0, -7, 89, -587, 1365, -1365, 587, -89, 7},
                          {13, -128, 556, -1160, 1174, -464, -68, 88, -11},
                          {0, 1, -11, 41, -75, 75, -41, 11, -1},
                          {-5, 46, -170, 334, -380, 250, -86, 10, 1},
                          {0, -1, 7, -21, 35, -35, 21, -7, 1},
                          {1, -8, 28, -56, 70, -56, 28, -8, 1}}};

// Newton iteration from above: monotone, converges to the root within an ulp.
constexpr double csqrt(double x)
{
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 200; ++i) r = 0.5 * (r + x / r);
    return r;
}

constexpr double zk(int k, double xi)
{
    double p = 1.0;
    for (int i = 0; i < k; ++i) p *= xi;
    return p - ((k % 2 == 0) ? 1.0 : -1.0) / double(k + 1);
}

constexpr double dzk(int k, double xi)
{
    double p = double(k);
    for (int i = 1; i < k; ++i) p *= xi;
    return p;
}

// Gauss-Legendre nodes on [-1/2, 1/2] and weights normalised to 1.
constexpr void gauss_nodes(int G, double *x, double *w)
{
    if (G == 1) {
        x[0] = 0.0;
        w[0] = 1.0;
    } else if (G == 2) {
        const double a = 1.0 / (2.0 * csqrt(3.0));
        x[0] = -a;
        x[1] = a;
        w[0] = w[1] = 0.5;
    } else if (G == 3) {
        const double a = csqrt(0.15);   // sqrt(3/5)/2
        x[0] = -a;
        x[1] = 0.0;
        x[2] = a;
        w[0] = w[2] = 5.0 / 18.0;
        w[1] = 4.0 / 9.0;
    } else {
        const double t = 2.0 * csqrt(1.2) / 7.0;
        const double in = 0.5 * csqrt(3.0 / 7.0 - t), out = 0.5 * csqrt(3.0 / 7.0 + t);
        const double r30 = csqrt(30.0) / 72.0;
        x[0] = -out;
        x[1] = -in;
        x[2] = in;
        x[3] = out;
        w[0] = w[3] = 0.25 - r30;
        w[1] = w[2] = 0.25 + r30;
    }
}

constexpr Tables make_tables()
{
    Tables t{};
    const Stencil *st[4] = {&kS3, &kS5, &kS7, &kS9};
    for (int oi = 0; oi < 4; ++oi) {
        const int r = 2 * oi + 3;
        const int G = (r - 1) / 2;
        double pts[kMaxPts] = {0.0, -1.0, 0.0, 0.0, 0.0, 0.0};
        double gx[4] = {0, 0, 0, 0}, gw[4] = {0, 0, 0, 0};
        gauss_nodes(G, gx, gw);
        for (int k = 0; k < G; ++k) {
            pts[2 + k] = -0.5 + gx[k];
            t.eta[oi][k] = gw[k];
        }
        for (int q = 0; q < 2 + G; ++q) {
            for (int k = 1; k <= 4; ++k) t.z[oi][q][k - 1] = zk(k, pts[q]);
            for (int li = 0; li < 4; ++li) {
                const Stencil &S = *st[li];
                t.lin[oi][li][q][4] = 1.0;  // W_0
                for (int k = 1; k <= S.ncoef; ++k) {
                    const double zq = zk(k, pts[q]);
                    for (int m = -S.h; m <= S.h; ++m)
                        t.lin[oi][li][q][4 + m] += S.num[k - 1][m + S.h] / S.den[k - 1] * zq;
                }
            }
        }
    }
    for (int oi = 0; oi < 4; ++oi) {
        const int G = oi + 1;
        double pts[kMaxPts] = {0.0, -1.0, 0.0, 0.0, 0.0, 0.0};
        double gx[4] = {0, 0, 0, 0}, gw[4] = {0, 0, 0, 0};
        gauss_nodes(G, gx, gw);
        for (int k = 0; k < G; ++k) pts[2 + k] = -0.5 + gx[k];
        for (int q = 0; q < 2 + G; ++q) {
            for (int k = 1; k <= 4; ++k) t.dz[oi][q][k - 1] = dzk(k, pts[q]);
            for (int li = 0; li < 4; ++li) {
                const Stencil &S = *st[li];
                for (int k = 1; k <= S.ncoef; ++k)
                    for (int m = -S.h; m <= S.h; ++m)
                        t.dlin[oi][li][q][4 + m] += S.num[k - 1][m + S.h] / S.den[k - 1] * dzk(k, pts[q]);
            }
        }
    }
    for (int oi = 0; oi < 4; ++oi) {
        const int G = oi + 1;
        for (int p = 0; p < (G + 1) / 2 && p < 2; ++p)
            for (int li = 0; li < 4; ++li) {
                const double *c = t.lin[oi][li][2 + p];
                t.sym[oi][li][p][0] = c[4];
                for (int m = 1; m <= 4; ++m) {
                    t.sym[oi][li][p][m] = 0.5 * (c[4 + m] + c[4 - m]);
                    t.sym[oi][li][p][4 + m] = 0.5 * (c[4 + m] - c[4 - m]);
                }
            }
    }
    return t;
}

}  // namespace tables

// Extents of a 2D sweep tile of T0 x T1 cells with faces of direction DIR:
// staged cells (UX x UY), cells whose face traces phase 1 forms (TX x TY),
// flux faces (FX x FY).
template <int DIR, int R, int T0, int T1>
struct SweepShape {
    static constexpr int UX = (DIR == 0) ? T0 + 2 + 2 * R : T0 + 2 * R;
    static constexpr int UY = (DIR == 0) ? T1 + 2 * R : T1 + 2 + 2 * R;
    static constexpr int TX = (DIR == 0) ? T0 + 2 : T0 + 2 * R;
    static constexpr int TY = (DIR == 0) ? T1 + 2 * R : T1 + 2;
    static constexpr int FX = (DIR == 0) ? T0 + 1 : T0;
    static constexpr int FY = (DIR == 0) ? T1 : T1 + 1;
};

struct MethodConst {
    double gamma, gm1;          // gamma, gamma - 1
    double thr;                 // sigma_thres
    double eps;
    double d5, d3m, d30;        // linear weights d^5_0, d^3_{-1} (= d^3_1), d^3_0
    double inv_d5, r3m, r30;    // 1/d5, d3m/d5, d30/d5
    int order;
    int flags;
};

#if defined(ASE_KERNEL_TU)
// Device code below is compiled only into the kernel translation unit.
__device__ constexpr Tables kTab = tables::make_tables();

// ---------------------------------------------------------------------------
// DF factor and level (Sec. 3.1 Eq. discontinuity strength; Algorithm 1 with
// the text's rule at the nominal order).
// ---------------------------------------------------------------------------
constexpr int LVL_WENOAO = 2;
constexpr int LVL_R3 = 3;

__device__ __forceinline__ double rcp_nr(double x);
// thr / A by a refined reciprocal; an infinite strength (a non-physical
// state beside a face) gives 0 as the quotient does
__device__ __forceinline__ double df_alpha(double A, double thr)
{
    return A < thr ? 1.0 : (__builtin_isinf(A) ? 0.0 : thr * rcp_nr(A));
}

// Sum of face strengths s[lo..hi-1] in left-to-right order.
template <int R>
__device__ __forceinline__ double ssum(const double (&s)[2 * R], int lo, int hi)
{
    double A = 0.0;
#pragma unroll
    for (int m = -R; m < R; ++m)
        if (m >= lo && m < hi) A += s[m + R];
    return A;
}

// Level of the cell whose stencil face strengths are s[m+R], m = -R..R-1
// (s[m+R] between cells m and m+1).  alpha(S) < 1  <=>  A(S) > thr.
template <int R>
__device__ __forceinline__ int select_level(const double (&s)[2 * R], double thr)
{
    if constexpr (R == 1) {
        return LVL_R3;
    } else {
        if (ssum<R>(s, -2, 2) > thr) return LVL_WENOAO;
        if constexpr (R == 2) {
            return 5;
        } else {
            if (ssum<R>(s, -3, 3) > thr) return 5;
            if constexpr (R == 3) {
                return 7;
            } else {
                if (ssum<R>(s, -4, 4) > thr) return 7;
                return 9;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Per-cell reconstruction of NV variables at NP points.
//   ld(v, m), m = -R..R  : cell average of variable v at stencil offset m
//                          (read on demand, one variable at a time)
//   s[m+R], m = -R..R-1  : strength of the face between cells m and m+1
//   q0                   : first evaluation point of the table (0 for the
//                          two faces, 2 for the Gauss points)
// ---------------------------------------------------------------------------
template <int NV, int NP, int H, class LD>
__device__ __forceinline__ void eval_linear(LD ld, int oi, int li, int q0, double (&out)[NV][NP])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double w[2 * H + 1];
#pragma unroll
        for (int m = -H; m <= H; ++m) w[m + H] = ld(v, m);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const double *c = kTab.lin[oi][li][q0 + q];
            double acc = c[4 - H] * w[0];
#pragma unroll
            for (int m = -H + 1; m <= H; ++m) acc = fma(c[4 + m], w[m + H], acc);
            out[v][q] = acc;
        }
    }
}

// eval_linear at the NP (3 or 4) Gauss points from the even and odd parts
// of the weights (table sym): the tap sums and differences are formed once
// and each mirror pair of points costs one dot product of H + 1 and one of
// H terms (r = 9: 30 operations per variable instead of 36).
template <int H>
__device__ __forceinline__ double sym_even(const double *c, double w0, const double (&sm)[H])
{
    double E = c[0] * w0;
#pragma unroll
    for (int m = 1; m <= H; ++m) E = fma(c[m], sm[m - 1], E);
    return E;
}

template <int H>
__device__ __forceinline__ double sym_odd(const double *c, const double (&dm)[H])
{
    double O = c[5] * dm[0];
#pragma unroll
    for (int m = 2; m <= H; ++m) O = fma(c[4 + m], dm[m - 1], O);
    return O;
}

template <int NV, int NP, int H, class LD>
__device__ __forceinline__ void eval_linear_gauss(LD ld, int oi, int li, double (&out)[NV][NP])
{
    static_assert(NP <= 4, "at most two mirror pairs");
    if constexpr (NP >= 3) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double w0 = ld(v, 0);
            double sm[H], dm[H];
#pragma unroll
            for (int m = 1; m <= H; ++m) {
                const double wp = ld(v, m), wm = ld(v, -m);
                sm[m - 1] = wp + wm;
                dm[m - 1] = wp - wm;
            }
            const double *c0 = kTab.sym[oi][li][0], *c1 = kTab.sym[oi][li][1];
            const double E0 = sym_even<H>(c0, w0, sm), O0 = sym_odd<H>(c0, dm);
            const double E1 = sym_even<H>(c1, w0, sm);
            if constexpr (NP == 4) {
                const double O1 = sym_odd<H>(c1, dm);
                out[v][0] = E0 + O0;
                out[v][1] = E1 + O1;
                out[v][2] = E1 - O1;
                out[v][3] = E0 - O0;
            } else {
                out[v][0] = E0 + O0;
                out[v][1] = E1;   // the centre point: no odd part
                out[v][2] = E0 - O0;
            }
        }
    }
}

// WENO-Z-AO(5,3) with DF factors (Sec. 3.2); one variable, W[0..4] = W_{-2..2}.
// The candidate coefficients and the normalised nonlinear weights do not
// depend on the evaluation point.
struct WenoAO53 {
    double am1, am2, a01, a02, ap1, ap2;   // 3-cell sub-stencils (W_x1, W_x2)
    double b1, b2, b3, b4;                 // 5-cell stencil
    double o5, om, o0, op;                 // normalised weights
};

__device__ __forceinline__ WenoAO53 weno_ao53_setup(const double (&W)[5], const MethodConst &mc)
{
    WenoAO53 c;
    const double Wm2 = W[0], Wm1 = W[1], W0 = W[2], W1 = W[3], W2 = W[4];
    // sub-stencil coefficients (W_x1, W_x2)
    c.am1 = 2.0 * W0 - 3.0 * Wm1 + Wm2;
    c.am2 = 0.5 * (Wm2 - 2.0 * Wm1 + W0);
    c.a01 = W1 - W0;
    c.a02 = 0.5 * (Wm1 - 2.0 * W0 + W1);
    c.ap1 = W1 - W0;
    c.ap2 = 0.5 * (W0 - 2.0 * W1 + W2);
    // 5-cell coefficients
    c.b1 = (-15.0 * W0 + Wm1 + 15.0 * W1 - W2) * (1.0 / 12.0);
    c.b2 = (-8.0 * W0 + 6.0 * Wm1 - Wm2 + 2.0 * W1 + W2) * 0.125;
    c.b3 = (3.0 * W0 - Wm1 - 3.0 * W1 + W2) * (1.0 / 6.0);
    c.b4 = (6.0 * W0 - 4.0 * Wm1 + Wm2 - 4.0 * W1 + W2) * (1.0 / 24.0);
    // smoothness indicators of the 3-cell polynomials on [-1,0]:
    // int (P')^2 + int (P'')^2 = a1^2 - 2 a1 a2 + 16/3 a2^2
    const double sm = c.am1 * c.am1 - 2.0 * c.am1 * c.am2 + (16.0 / 3.0) * c.am2 * c.am2;
    const double s0 = c.a01 * c.a01 - 2.0 * c.a01 * c.a02 + (16.0 / 3.0) * c.a02 * c.a02;
    const double sp = c.ap1 * c.ap1 - 2.0 * c.ap1 * c.ap2 + (16.0 / 3.0) * c.ap2 * c.ap2;
    const double s5 = (sm + 4.0 * s0 + sp) * (1.0 / 6.0) + fabs(sm - sp);
    const double tz = (fabs(s5 - sm) + fabs(s5 - s0) + fabs(s5 - sp)) * (1.0 / 3.0);
    const double tz2 = tz * tz;
    const double e5 = s5 + mc.eps, em = sm + mc.eps, e0 = s0 + mc.eps, ep = sp + mc.eps;
    // reciprocals as the hardware estimate refined (rcp_nr, within an ulp or
    // two): the weights are continuous in them and decide nothing discrete
    const double w5 = mc.d5 * (1.0 + tz2 * rcp_nr(e5 * e5));
    const double wm = mc.d3m * (1.0 + tz2 * rcp_nr(em * em));
    const double w0 = mc.d30 * (1.0 + tz2 * rcp_nr(e0 * e0));
    const double wp = mc.d3m * (1.0 + tz2 * rcp_nr(ep * ep));
    const double inv = rcp_nr(w5 + wm + w0 + wp);
    c.o5 = w5 * inv;
    c.om = wm * inv;
    c.o0 = w0 * inv;
    c.op = wp * inv;
    return c;
}

template <int NP>
__device__ __forceinline__ void weno_ao53(const double (&W)[5], const double al[4], const MethodConst &mc, int oi,
                                          int q0, double (&out)[NP])
{
    const WenoAO53 c = weno_ao53_setup(W, mc);
    const double W0 = W[2];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const double *z = kTab.z[oi][q0 + q];
        const double Pm = W0 + al[0] * (c.am1 * z[0] + c.am2 * z[1]);
        const double P0 = W0 + al[1] * (c.a01 * z[0] + c.a02 * z[1]);
        const double Pp = W0 + al[2] * (c.ap1 * z[0] + c.ap2 * z[1]);
        const double P5 = W0 + al[3] * (c.b1 * z[0] + c.b2 * z[1] + c.b3 * z[2] + c.b4 * z[3]);
        const double inner = P5 * mc.inv_d5 - mc.r3m * Pm - mc.r30 * P0 - mc.r3m * Pp;
        out[q] = c.o5 * inner + c.om * Pm + c.o0 * P0 + c.op * Pp;
    }
}

// Reconstruction of all NV variables of a cell at NP points of order r (oi).
// Returns the level used.
template <int R, int NV, int NP, class LD>
__device__ __forceinline__ int reconstruct_cell(LD ld, const double (&s)[2 * R], const MethodConst &mc, int oi,
                                                int q0, double (&out)[NV][NP])
{
    const int lvl = select_level<R>(s, mc.thr);
    if constexpr (R == 1) {
        // DF-damped centred 3-cell polynomial.
        const double al = df_alpha(s[0] + s[1], mc.thr);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double Wm = ld(v, -1), W0 = ld(v, 0), Wp = ld(v, 1);
            const double a1 = Wp - W0;
            const double a2 = 0.5 * (Wm - 2.0 * W0 + Wp);
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const double *z = kTab.z[oi][q0 + q];
                out[v][q] = W0 + al * (a1 * z[0] + a2 * z[1]);
            }
        }
        return lvl;
    } else {
        // the linear levels: at three or four Gauss points (q0 = 2) in the
        // mirror-pair form
        constexpr bool kPairs = NP >= 3;
        if (lvl == 9) {
            if constexpr (R >= 4) {
                if (kPairs && q0 == 2) eval_linear_gauss<NV, NP, 4>(ld, oi, 3, out);
                else eval_linear<NV, NP, 4>(ld, oi, 3, q0, out);
            }
        } else if (lvl == 7) {
            if constexpr (R >= 3) {
                if (kPairs && q0 == 2) eval_linear_gauss<NV, NP, 3>(ld, oi, 2, out);
                else eval_linear<NV, NP, 3>(ld, oi, 2, q0, out);
            }
        } else if (lvl == 5) {
            if (kPairs && q0 == 2) eval_linear_gauss<NV, NP, 2>(ld, oi, 1, out);
            else eval_linear<NV, NP, 2>(ld, oi, 1, q0, out);
        } else {
            double al[4];
            al[0] = df_alpha(ssum<R>(s, -2, 0), mc.thr);
            al[1] = df_alpha(ssum<R>(s, -1, 1), mc.thr);
            al[2] = df_alpha(ssum<R>(s, 0, 2), mc.thr);
            al[3] = df_alpha(ssum<R>(s, -2, 2), mc.thr);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double W[5], o[NP];
#pragma unroll
                for (int m = -2; m <= 2; ++m) W[m + 2] = ld(v, m);
                weno_ao53<NP>(W, al, mc, oi, q0, o);
#pragma unroll
                for (int q = 0; q < NP; ++q) out[v][q] = o[q];
            }
        }
        return lvl;
    }
}

// ---------------------------------------------------------------------------
// Euler equations (Sec. 2.3).
// ---------------------------------------------------------------------------

// Reciprocal and reciprocal square root: the hardware estimate (relative
// error about 2^-24 on gfx950) refined by one third-order step.  With
// e = 1 - x r0, 1/x = r0 / (1 - e) = r0 (1 + e + e^2 + ...); with
// e = 1 - x y0^2, 1/sqrt(x) = y0 (1 - e)^(-1/2) = y0 (1 + e/2 + 3 e^2/8 + ...).
// The dropped terms are O(e^3) ~ 2^-72: the results are within a few ulp,
// far below the 1e-12 parity bound.
__device__ __forceinline__ double rcp_nr(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
}

__device__ __forceinline__ double rsq_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

struct Prim {
    double un, ut, p, c, ic;  // normal/tangential velocity, pressure, sound speed, 1/c
    bool ok;
};

// dir 0: x-normal, 1: y-normal.  NV = 3 (1D) or 4 (2D).
template <int NV>
__device__ __forceinline__ Prim primitives(const double (&W)[NV], int dir, const MethodConst &mc)
{
    Prim q;
    const double rho = W[0];
    const double ir = rcp_nr(rho);
    const double u = W[1] * ir;
    double v = 0.0, ke;
    if constexpr (NV == 4) {
        v = W[2] * ir;
        ke = W[1] * u + W[2] * v;   // rho (u^2 + v^2)
    } else {
        ke = W[1] * u;
    }
    const double p = mc.gm1 * (W[NV - 1] - 0.5 * ke);
    q.un = dir == 0 ? u : v;
    q.ut = dir == 0 ? v : u;
    q.p = p;
    q.ok = (rho > 0.0) && (p > 0.0);
    const double c2 = mc.gamma * p * ir;
    q.ic = rsq_nr(c2);
    q.c = c2 * q.ic;
    return q;
}

// Discontinuity strength of one Gauss point (Sec. 3.1); +inf if a side is
// non-physical.  |pl-pr|/pl + |pl-pr|/pr is formed as |pl-pr| (pl+pr)/(pl pr).
__device__ __forceinline__ double sigma_point(const Prim &l, const Prim &r)
{
    // No contraction: equal states must give exactly zero.
#pragma clang fp contract(off)
    if (!(l.ok && r.ok)) return __builtin_huge_val();
    const double dp = fabs(l.p - r.p);
    const double dn = l.un * l.ic - r.un * r.ic;
    const double dt = l.ut * l.ic - r.ut * r.ic;
    return dp * (l.p + r.p) * rcp_nr(l.p * r.p) + dn * dn + dt * dt;
}

// Physical flux along dir.
template <int NV>
__device__ __forceinline__ void euler_flux(const double (&W)[NV], const Prim &q, int dir, double (&F)[NV])
{
    if constexpr (NV == 3) {
        F[0] = W[1];
        F[1] = W[1] * q.un + q.p;
        F[2] = q.un * (W[2] + q.p);
    } else {
        F[0] = dir == 0 ? W[1] : W[2];
        F[1] = W[1] * q.un + (dir == 0 ? q.p : 0.0);
        F[2] = W[2] * q.un + (dir == 0 ? 0.0 : q.p);
        F[3] = q.un * (W[3] + q.p);
    }
}

// Lax-Friedrichs flux with the local maximal signal speed (Sec. 2.3).
template <int NV>
__device__ __forceinline__ void lf_flux(const double (&Wl)[NV], const Prim &ql, const double (&Wr)[NV],
                                        const Prim &qr, int dir, double (&F)[NV])
{
    double Fl[NV], Fr[NV];
    euler_flux<NV>(Wl, ql, dir, Fl);
    euler_flux<NV>(Wr, qr, dir, Fr);
    const double sl = fabs(ql.un) + ql.c, sr = fabs(qr.un) + qr.c;
    const double hs = 0.5 * (sl > sr ? sl : sr);
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = 0.5 * (Fl[v] + Fr[v]) - hs * (Wr[v] - Wl[v]);
}

// Strength and LF flux at one Gauss point, with the optional positivity
// replacement of a non-physical side by its cell average (fetched lazily:
// cl(v) / cr(v) return variable v of the left / right cell average).
// With want_sigma false (first-order DF source) the strength is not
// evaluated and 0 returned.
template <int NV, class CL, class CR>
__device__ __forceinline__ double gauss_point(double (&Wl)[NV], double (&Wr)[NV], CL cl, CR cr, int dir,
                                              const MethodConst &mc, double (&F)[NV], bool want_sigma = true)
{
    Prim ql = primitives<NV>(Wl, dir, mc);
    Prim qr = primitives<NV>(Wr, dir, mc);
    const double sg = want_sigma ? sigma_point(ql, qr) : 0.0;
    if (mc.flags & 1) {
        if (!ql.ok) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Wl[v] = cl(v);
            ql = primitives<NV>(Wl, dir, mc);
        }
        if (!qr.ok) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Wr[v] = cr(v);
            qr = primitives<NV>(Wr, dir, mc);
        }
    }
    lf_flux<NV>(Wl, ql, Wr, qr, dir, F);
    return sg;
}

// Strength and LF flux at one Gauss point seen from one side of the face:
// Wo is this lane's own state, Wt the state across the face, sgn = +1 when
// the own side is the left (lower) one and -1 otherwise.  Equal to
// gauss_point with (Wl, Wr) = (Wo, Wt) or (Wt, Wo): the flux average, the
// signal speed and the strength are symmetric in the two states.
// With want_sigma false (first-order DF source: the strengths come from the
// cell averages) the Gauss-point strength is not evaluated and 0 returned.
template <int NV, class CO, class CT>
__device__ __forceinline__ double gauss_point_sided(double (&Wo)[NV], double (&Wt)[NV], double sgn, CO co, CT ct,
                                                    int dir, const MethodConst &mc, double (&F)[NV],
                                                    bool want_sigma = true)
{
    Prim qo = primitives<NV>(Wo, dir, mc);
    Prim qt = primitives<NV>(Wt, dir, mc);
    const double sg = want_sigma ? sigma_point(qo, qt) : 0.0;
    if (mc.flags & 1) {
        if (!qo.ok) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Wo[v] = co(v);
            qo = primitives<NV>(Wo, dir, mc);
        }
        if (!qt.ok) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Wt[v] = ct(v);
            qt = primitives<NV>(Wt, dir, mc);
        }
    }
    double Fo[NV], Ft[NV];
    euler_flux<NV>(Wo, qo, dir, Fo);
    euler_flux<NV>(Wt, qt, dir, Ft);
    const double so = fabs(qo.un) + qo.c, st = fabs(qt.un) + qt.c;
    const double hs = sgn * 0.5 * (so > st ? so : st);
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = 0.5 * (Fo[v] + Ft[v]) - hs * (Wt[v] - Wo[v]);
    return sg;
}

// Tile of this workgroup.  Workgroups are dispatched round-robin over the
// 8 XCDs (each with its own L2); remapping the linear block index so that
// every XCD receives one contiguous band of tiles keeps the halos that
// neighbouring tiles share inside one L2.
__device__ __forceinline__ void xcd_tile(int &tx, int &ty)
{
    constexpr int kXCD = 8;
    const int gx = gridDim.x, n = gridDim.x * gridDim.y;
    const int b = blockIdx.y * gx + blockIdx.x;
    const int per = n / kXCD;
    int t = b;
    if (b < per * kXCD) t = (b % kXCD) * per + b / kXCD;
    tx = t % gx;
    ty = t / gx;
}

// Exchange a double with the neighbouring lane (lane ^ 1) of a pair.  Both
// lanes of the pair must be active.
__device__ __forceinline__ double swap_pair(double x)
{
    const int lo = __double2loint(x), hi = __double2hiint(x);
    const int lo2 = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
    const int hi2 = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
    return __hiloint2double(hi2, lo2);
}

// ---------------------------------------------------------------------------
// Adjoint building blocks (1D): Jacobians of the reconstruction with the DF
// factors and the stencil level frozen, and the transposed LF flux with the
// signal-speed side and positivity replacements frozen.
// ---------------------------------------------------------------------------

// Reverse mode of WENO-Z-AO(5,3)+DF for one variable (DF factors frozen):
// with Y = g[0] P(xi=0) + g[1] P(xi=-1), returns gW[m+2] = dY/dW_m,
// m = -2..2.  Every intermediate of weno_ao53 is recomputed, then the
// adjoints flow back through the nonlinear weights, tau_Z, the smoothness
// indicators and the sub-stencil coefficients.  |x| has derivative sign(x)
// (0 at 0).
__device__ __forceinline__ void weno_ao53_vjp(const double (&W)[5], const double al[4], const MethodConst &mc, int oi,
                                              const double (&g)[2], double (&gW)[5])
{
    const double Wm2 = W[0], Wm1 = W[1], W0 = W[2], W1 = W[3], W2 = W[4];
    const double am1 = 2.0 * W0 - 3.0 * Wm1 + Wm2, am2 = 0.5 * (Wm2 - 2.0 * Wm1 + W0);
    const double a01 = W1 - W0, a02 = 0.5 * (Wm1 - 2.0 * W0 + W1);
    const double ap1 = W1 - W0, ap2 = 0.5 * (W0 - 2.0 * W1 + W2);
    const double b1 = (-15.0 * W0 + Wm1 + 15.0 * W1 - W2) * (1.0 / 12.0);
    const double b2 = (-8.0 * W0 + 6.0 * Wm1 - Wm2 + 2.0 * W1 + W2) * 0.125;
    const double b3 = (3.0 * W0 - Wm1 - 3.0 * W1 + W2) * (1.0 / 6.0);
    const double b4 = (6.0 * W0 - 4.0 * Wm1 + Wm2 - 4.0 * W1 + W2) * (1.0 / 24.0);
    const double sm = am1 * am1 - 2.0 * am1 * am2 + (16.0 / 3.0) * am2 * am2;
    const double s0 = a01 * a01 - 2.0 * a01 * a02 + (16.0 / 3.0) * a02 * a02;
    const double sp = ap1 * ap1 - 2.0 * ap1 * ap2 + (16.0 / 3.0) * ap2 * ap2;
    const double sgd = sm > sp ? 1.0 : (sm < sp ? -1.0 : 0.0);
    const double s5 = (sm + 4.0 * s0 + sp) * (1.0 / 6.0) + fabs(sm - sp);
    const double sgm = s5 > sm ? 1.0 : (s5 < sm ? -1.0 : 0.0);
    const double sg0 = s5 > s0 ? 1.0 : (s5 < s0 ? -1.0 : 0.0);
    const double sgp = s5 > sp ? 1.0 : (s5 < sp ? -1.0 : 0.0);
    const double tz = (fabs(s5 - sm) + fabs(s5 - s0) + fabs(s5 - sp)) * (1.0 / 3.0);
    const double tz2 = tz * tz;
    const double e5 = s5 + mc.eps, em = sm + mc.eps, e0 = s0 + mc.eps, ep = sp + mc.eps;
    const double i5 = 1.0 / (e5 * e5), im = 1.0 / (em * em), i0 = 1.0 / (e0 * e0), ip = 1.0 / (ep * ep);
    const double w5 = mc.d5 * (1.0 + tz2 * i5);
    const double wm = mc.d3m * (1.0 + tz2 * im);
    const double w0 = mc.d30 * (1.0 + tz2 * i0);
    const double wp = mc.d3m * (1.0 + tz2 * ip);
    const double iws = 1.0 / (w5 + wm + w0 + wp);
    const double o5 = w5 * iws, om = wm * iws, o0 = w0 * iws, op = wp * iws;

    // adjoints of the weights and of the candidate polynomials
    double I5 = 0.0, Im = 0.0, I0 = 0.0, Ip = 0.0;
    double gam1 = 0.0, gam2 = 0.0, ga01 = 0.0, ga02 = 0.0, gap1 = 0.0, gap2 = 0.0;
    double gb1 = 0.0, gb2 = 0.0, gb3 = 0.0, gb4 = 0.0, gW0 = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double *z = kTab.z[oi][q];
        const double Pm = W0 + al[0] * (am1 * z[0] + am2 * z[1]);
        const double P0 = W0 + al[1] * (a01 * z[0] + a02 * z[1]);
        const double Pp = W0 + al[2] * (ap1 * z[0] + ap2 * z[1]);
        const double P5 = W0 + al[3] * (b1 * z[0] + b2 * z[1] + b3 * z[2] + b4 * z[3]);
        const double inner = P5 * mc.inv_d5 - mc.r3m * Pm - mc.r30 * P0 - mc.r3m * Pp;
        I5 += g[q] * inner;
        Im += g[q] * Pm;
        I0 += g[q] * P0;
        Ip += g[q] * Pp;
        const double gPm = g[q] * (om - o5 * mc.r3m);
        const double gP0 = g[q] * (o0 - o5 * mc.r30);
        const double gPp = g[q] * (op - o5 * mc.r3m);
        const double gP5 = g[q] * o5 * mc.inv_d5;
        gW0 += gPm + gP0 + gPp + gP5;
        gam1 += gPm * al[0] * z[0];
        gam2 += gPm * al[0] * z[1];
        ga01 += gP0 * al[1] * z[0];
        ga02 += gP0 * al[1] * z[1];
        gap1 += gPp * al[2] * z[0];
        gap2 += gPp * al[2] * z[1];
        gb1 += gP5 * al[3] * z[0];
        gb2 += gP5 * al[3] * z[1];
        gb3 += gP5 * al[3] * z[2];
        gb4 += gP5 * al[3] * z[3];
    }
    // o_k = w_k / sum w  ->  dY/dw_k = (I_k - sum_j o_j I_j) / sum w
    const double Ibar = o5 * I5 + om * Im + o0 * I0 + op * Ip;
    const double gw5 = (I5 - Ibar) * iws, gwm = (Im - Ibar) * iws, gw0 = (I0 - Ibar) * iws, gwp = (Ip - Ibar) * iws;
    // w_k = d_k (1 + tz^2 / e_k^2)
    const double gtz2 = gw5 * mc.d5 * i5 + gwm * mc.d3m * im + gw0 * mc.d30 * i0 + gwp * mc.d3m * ip;
    double gs5 = -2.0 * gw5 * mc.d5 * tz2 * i5 / e5;
    double gsm = -2.0 * gwm * mc.d3m * tz2 * im / em;
    double gs0 = -2.0 * gw0 * mc.d30 * tz2 * i0 / e0;
    double gsp = -2.0 * gwp * mc.d3m * tz2 * ip / ep;
    // tau_Z
    const double gtz = 2.0 * tz * gtz2 * (1.0 / 3.0);
    gs5 += gtz * (sgm + sg0 + sgp);
    gsm -= gtz * sgm;
    gs0 -= gtz * sg0;
    gsp -= gtz * sgp;
    // beta_5 = (beta_m + 4 beta_0 + beta_p) / 6 + |beta_m - beta_p|
    gsm += gs5 * ((1.0 / 6.0) + sgd);
    gs0 += gs5 * (4.0 / 6.0);
    gsp += gs5 * ((1.0 / 6.0) - sgd);
    // beta_k = a1^2 - 2 a1 a2 + 16/3 a2^2
    gam1 += gsm * (2.0 * am1 - 2.0 * am2);
    gam2 += gsm * (-2.0 * am1 + (32.0 / 3.0) * am2);
    ga01 += gs0 * (2.0 * a01 - 2.0 * a02);
    ga02 += gs0 * (-2.0 * a01 + (32.0 / 3.0) * a02);
    gap1 += gsp * (2.0 * ap1 - 2.0 * ap2);
    gap2 += gsp * (-2.0 * ap1 + (32.0 / 3.0) * ap2);
    // coefficients -> cell averages
    gW[0] = gam1 + 0.5 * gam2 - gb2 * 0.125 + gb4 * (1.0 / 24.0);
    gW[1] = -3.0 * gam1 - gam2 + 0.5 * ga02 + gb1 * (1.0 / 12.0) + gb2 * 0.75 - gb3 * (1.0 / 6.0) -
            gb4 * (4.0 / 24.0);
    gW[2] = gW0 + 2.0 * gam1 + 0.5 * gam2 - ga01 - ga02 - gap1 + 0.5 * gap2 - gb1 * (15.0 / 12.0) - gb2 +
            gb3 * 0.5 + gb4 * 0.25;
    gW[3] = ga01 + 0.5 * ga02 + gap1 - gap2 + gb1 * (15.0 / 12.0) + gb2 * 0.25 - gb3 * 0.5 - gb4 * (4.0 / 24.0);
    gW[4] = 0.5 * gap2 - gb1 * (1.0 / 12.0) + gb2 * 0.125 + gb3 * (1.0 / 6.0) + gb4 * (1.0 / 24.0);
}

// Frozen decisions of one cell's reconstruction: its level and DF factors
// (R = 1: al[0] of the 3-cell stencil; WENO-Z-AO: al[0..3] of S^3_{-1},
// S^3_0, S^3_1 and S^5; linear levels: unused).
template <int R>
__device__ __forceinline__ int cell_decisions(const double (&s)[2 * R], const MethodConst &mc, double (&al)[4])
{
    al[0] = al[1] = al[2] = al[3] = 1.0;
    if constexpr (R == 1) {
        al[0] = df_alpha(s[0] + s[1], mc.thr);
        return LVL_R3;
    } else {
        const int lvl = select_level<R>(s, mc.thr);
        if (lvl == LVL_WENOAO) {
            al[0] = df_alpha(ssum<R>(s, -2, 0), mc.thr);
            al[1] = df_alpha(ssum<R>(s, -1, 1), mc.thr);
            al[2] = df_alpha(ssum<R>(s, 0, 2), mc.thr);
            al[3] = df_alpha(ssum<R>(s, -2, 2), mc.thr);
        }
        return lvl;
    }
}

// Transposed reconstruction of one cell for one variable: with gR, gL the
// adjoints of the cell's right (xi = 0) and left (xi = -1) face values,
// cc[m + R] = gR dP(0)/dW_m + gL dP(-1)/dW_m, m = -R..R, for the level and
// DF factors of cell_decisions; ldv(m) reads the variable at offset m.
template <int R, class LDV>
__device__ __forceinline__ void recon_vjp_var(LDV ldv, int lvl, const double (&al)[4], const MethodConst &mc,
                                              double gR, double gL, double (&cc)[2 * R + 1])
{
    constexpr int OI = R - 1;
#pragma unroll
    for (int m = 0; m < 2 * R + 1; ++m) cc[m] = 0.0;
    if constexpr (R == 1) {
        // P = W0 + al ((W1 - W0) Z1 + (W-1 - 2 W0 + W1) Z2 / 2)
        const double a = al[0];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double *z = kTab.z[OI][q];
            const double gq = q == 0 ? gR : gL;
            cc[0] += gq * (a * 0.5 * z[1]);
            cc[1] += gq * (1.0 + a * (-z[0] - z[1]));
            cc[2] += gq * (a * (z[0] + 0.5 * z[1]));
        }
    } else {
        if (lvl == LVL_WENOAO) {
            double W[5], gW[5];
            const double g2[2] = {gR, gL};
#pragma unroll
            for (int m = -2; m <= 2; ++m) W[m + 2] = ldv(m);
            weno_ao53_vjp(W, al, mc, OI, g2, gW);
#pragma unroll
            for (int m = -2; m <= 2; ++m) cc[m + R] = gW[m + 2];
        } else {
            // linear levels: the tap weights themselves, one branch per level
            // so that they stay compile-time constants
            auto taps = [&](auto LI) {
                constexpr int li = decltype(LI)::value, h = li + 1;
#pragma unroll
                for (int m = -R; m <= R; ++m)
                    if (m >= -h && m <= h)
                        cc[m + R] = gR * kTab.lin[OI][li][0][4 + m] + gL * kTab.lin[OI][li][1][4 + m];
            };
            if (lvl == 9) {
                if constexpr (R >= 4) taps(std::integral_constant<int, 3>{});
            } else if (lvl == 7) {
                if constexpr (R >= 3) taps(std::integral_constant<int, 2>{});
            } else {
                taps(std::integral_constant<int, 1>{});
            }
        }
    }
}

// Transposed 1D Euler flux Jacobian and signal-speed gradient of a state:
// gW += (dF/dW)^T gF ; ds/dW written to ds.
__device__ __forceinline__ void euler1d_vjp(const double (&W)[3], const Prim &q, const MethodConst &mc,
                                            const double (&gF)[3], double scale, double (&gW)[3], double (&ds)[3])
{
    const double rho = W[0], u = q.un, p = q.p, E = W[2];
    const double gm = mc.gm1;
    const double pr = gm * 0.5 * u * u, pm = -gm * u, pE = gm;   // dp/d(rho, m, E)
    const double H = (E + p) / rho;
    // rows of A = dF/dW
    const double A[3][3] = {{0.0, 1.0, 0.0},
                            {-u * u + pr, 2.0 * u + pm, pE},
                            {u * pr - u * H, H + u * pm, u * (1.0 + pE)}};
#pragma unroll
    for (int c = 0; c < 3; ++c) gW[c] += scale * (A[0][c] * gF[0] + A[1][c] * gF[1] + A[2][c] * gF[2]);
    // s = |u| + c, c = sqrt(gamma p / rho)
    const double su = u > 0.0 ? 1.0 : (u < 0.0 ? -1.0 : 0.0);
    const double dc = 0.5 * mc.gamma / (q.c * rho);
    ds[0] = su * (-u / rho) + dc * (pr - p / rho);
    ds[1] = su * (1.0 / rho) + dc * pm;
    ds[2] = dc * pE;
}

#endif  // ASE_KERNEL_TU

}  // namespace ase
