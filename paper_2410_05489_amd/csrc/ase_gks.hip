// Gas-kinetic interface flux (Sec. 2.2, App. A) and the two stages of the
// S2O4 time step (Eq. S2O4 temporal) on 1D grids, for gfx950.
//
// Per face the reconstruction gives the two interface states and their
// x-slopes; the flux is the moment of the second-order BGK distribution
// (Eq. GKS flux) integrated over [0, dt] and [0, dt/2], from which the face
// flux and its time derivative at t_n follow (Eq. time advance).  Moments
// of the Maxwellians are written out explicitly: with
// psi = (1, u, (u^2 + xi^2)/2) every quantity is a short combination of
// <u^n> (whole or half line, n <= 6) and <xi^2>, <xi^4>.
#include <hip/hip_runtime.h>

#include "ase_device.h"
#include "ase_host.h"

namespace ase {
namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Reconstruction slopes at the faces.
// ---------------------------------------------------------------------------

// dP/dxi of the WENO-Z-AO(5,3) polynomial at NP points from q0 of order oi:
// the point-independent weights applied to the candidates' slopes.
template <int NP>
__device__ __forceinline__ void weno_ao53_slopes(const double (&W)[5], const double al[4], const MethodConst &mc,
                                                 int oi, int q0, double (&d)[NP])
{
    const WenoAO53 c = weno_ao53_setup(W, mc);
#pragma unroll
    for (int f = 0; f < NP; ++f) {
        const double *z = kTab.dz[oi][q0 + f];
        const double Dm = al[0] * (c.am1 * z[0] + c.am2 * z[1]);
        const double D0 = al[1] * (c.a01 * z[0] + c.a02 * z[1]);
        const double Dp = al[2] * (c.ap1 * z[0] + c.ap2 * z[1]);
        const double D5 = al[3] * (c.b1 * z[0] + c.b2 * z[1] + c.b3 * z[2] + c.b4 * z[3]);
        const double inner = D5 * mc.inv_d5 - mc.r3m * Dm - mc.r30 * D0 - mc.r3m * Dp;
        d[f] = c.o5 * inner + c.om * Dm + c.o0 * D0 + c.op * Dp;
    }
}

// Slopes of the linear (2H+1)-cell polynomial at NP points from q0 (weights
// tabulated at compile time).
template <int NV, int NP, int H, class LD>
__device__ __forceinline__ void slopes_linear(LD ld, int oi, int q0, double (&der)[NV][NP])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double w[2 * H + 1];
#pragma unroll
        for (int m = -H; m <= H; ++m) w[m + H] = ld(v, m);
#pragma unroll
        for (int f = 0; f < NP; ++f) {
            const double *c = kTab.dlin[oi][H - 1][q0 + f];
            double acc = c[4 - H] * w[0];
#pragma unroll
            for (int m = -H + 1; m <= H; ++m) acc = fma(c[4 + m], w[m + H], acc);
            der[v][f] = acc;
        }
    }
}

// Values and xi-slopes of the ASE-DF polynomial of a cell at NP points from
// q0 (0: the right face xi = 0, then the left face; 2: the Gauss points):
// the level rule and values of the LF path, then the slopes of the same
// polynomial.
template <int R, int NV, int NP, class LD>
__device__ __forceinline__ void reconstruct_with_slopes(LD ld, const double (&s)[2 * R], const MethodConst &mc,
                                                        int q0, double (&val)[NV][NP], double (&der)[NV][NP])
{
    constexpr int OI = R - 1;
    const int lvl = reconstruct_cell<R, NV, NP>(ld, s, mc, OI, q0, val);
    if constexpr (R == 1) {
        const double al = df_alpha(s[0] + s[1], mc.thr);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double Wm = ld(v, -1), W0 = ld(v, 0), Wp = ld(v, 1);
            const double a1 = Wp - W0, a2 = 0.5 * (Wm - 2.0 * W0 + Wp);
#pragma unroll
            for (int f = 0; f < NP; ++f)
                der[v][f] = al * (a1 * kTab.dz[OI][q0 + f][0] + a2 * kTab.dz[OI][q0 + f][1]);
        }
    } else if (lvl == 9) {
        if constexpr (R >= 4) slopes_linear<NV, NP, 4>(ld, OI, q0, der);
    } else if (lvl == 7) {
        if constexpr (R >= 3) slopes_linear<NV, NP, 3>(ld, OI, q0, der);
    } else if (lvl == 5) {
        slopes_linear<NV, NP, 2>(ld, OI, q0, der);
    } else {
        double al[4];
        al[0] = df_alpha(ssum<R>(s, -2, 0), mc.thr);
        al[1] = df_alpha(ssum<R>(s, -1, 1), mc.thr);
        al[2] = df_alpha(ssum<R>(s, 0, 2), mc.thr);
        al[3] = df_alpha(ssum<R>(s, -2, 2), mc.thr);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double W[5], d[NP];
#pragma unroll
            for (int m = -2; m <= 2; ++m) W[m + 2] = ld(v, m);
            weno_ao53_slopes<NP>(W, al, mc, OI, q0, d);
#pragma unroll
            for (int f = 0; f < NP; ++f) der[v][f] = d[f];
        }
    }
}

// ---------------------------------------------------------------------------
// Maxwellian moments (App. A).
// ---------------------------------------------------------------------------
constexpr int kNM = 7;   // <u^0> .. <u^6>

struct Maxw {
    double rho, U, lam;
    bool ok;
};

__device__ __forceinline__ Maxw maxwellian(const double (&W)[3], double gm1)
{
    Maxw m;
    m.rho = W[0];
    m.U = W[1] / W[0];
    const double p = gm1 * (W[2] - 0.5 * W[1] * m.U);
    m.ok = m.rho > 0.0 && p > 0.0;
    m.lam = m.rho / (2.0 * p);
    return m;
}

// <u^n> over the whole line: <u^{n+2}> = U <u^{n+1}> + (n+1)/(2 lam) <u^n>.
__device__ __forceinline__ void moments_full(const Maxw &m, double (&M)[kNM])
{
    const double h = 0.5 / m.lam;
    M[0] = 1.0;
    M[1] = m.U;
#pragma unroll
    for (int n = 0; n + 2 < kNM; ++n) M[n + 2] = fma(m.U, M[n + 1], (n + 1) * h * M[n]);
}

// <u^n> over u > 0 (sgn = 1) or u < 0 (sgn = -1): the same recursion from
// <u^0> = erfc(-sgn sqrt(lam) U)/2 and <u^1> = U <u^0> + sgn exp(-lam U^2)/(2 sqrt(pi lam)).
__device__ __forceinline__ void moments_half(const Maxw &m, double sgn, double (&M)[kNM])
{
    const double h = 0.5 / m.lam;
    const double sl = sqrt(m.lam);
    M[0] = 0.5 * erfc(-sgn * sl * m.U);
    M[1] = fma(m.U, M[0], sgn * 0.5 * exp(-m.lam * m.U * m.U) / sqrt(kPi * m.lam));
#pragma unroll
    for (int n = 0; n + 2 < kNM; ++n) M[n + 2] = fma(m.U, M[n + 1], (n + 1) * h * M[n]);
}

// <(c . psi) u^k psi_j>, j = 0..2, with <u^n psi_0> = M_n, <u^n psi_1> =
// M_{n+1}, <u^n psi_2> = (M_{n+2} + M_n X2)/2 and (u^2 + xi^2) u^n psi_j
// expanded the same way.
template <int K>
__device__ __forceinline__ void lin_moment(const double (&c)[3], const double (&M)[kNM], double X2, double X4,
                                           double (&out)[3])
{
    const double t0 = M[K], t1 = M[K + 1], t2 = 0.5 * (M[K + 2] + M[K] * X2);
    const double u0 = M[K + 1], u1 = M[K + 2], u2 = 0.5 * (M[K + 3] + M[K + 1] * X2);
    const double s0 = M[K + 2] + M[K] * X2;
    const double s1 = M[K + 3] + M[K + 1] * X2;
    const double s2 = 0.5 * (M[K + 4] + 2.0 * M[K + 2] * X2 + M[K] * X4);
    out[0] = c[0] * t0 + c[1] * u0 + 0.5 * c[2] * s0;
    out[1] = c[0] * t1 + c[1] * u1 + 0.5 * c[2] * s1;
    out[2] = c[0] * t2 + c[1] * u2 + 0.5 * c[2] * s2;
}

// Micro slope a of <(a . psi) psi_j> = b_j: App. A's closed-form solution of
// M a = b for one velocity direction (K internal degrees of freedom).
__device__ __forceinline__ void micro_slope(const Maxw &m, double K, const double (&b)[3], double (&a)[3])
{
    const double c = m.U * m.U + (K + 1.0) / (2.0 * m.lam);
    const double R3 = 2.0 * b[2] - c * b[0];
    const double R2 = b[1] - m.U * b[0];
    a[2] = 4.0 * m.lam * m.lam / (K + 1.0) * (R3 - 2.0 * m.U * R2);
    a[1] = 2.0 * m.lam * R2 - m.U * a[2];
    a[0] = b[0] - m.U * a[1] - 0.5 * a[2] * c;
}

// Spatial slope a from W_x and the time slope A from <A + a u> = 0.
__device__ __forceinline__ void slopes(const Maxw &m, double K, const double (&Mf)[kNM], double X2, double X4,
                                       const double (&Wx)[3], double (&a)[3], double (&A)[3])
{
    const double ir = 1.0 / m.rho;
    const double b[3] = {Wx[0] * ir, Wx[1] * ir, Wx[2] * ir};
    micro_slope(m, K, b, a);
    double t[3];
    lin_moment<1>(a, Mf, X2, X4, t);
    const double bt[3] = {-t[0], -t[1], -t[2]};
    micro_slope(m, K, bt, A);
}

// Face flux F and its time derivative F_t at t_n (Eq. time advance) from the
// interface states and x-slopes.  Collision time tau outside the
// exponentials, tau_n = C1 dt + C2 |p_l - p_r|/(p_l + p_r) dt inside.
// Returns false (and NaN) when a state is not physical.
__device__ __forceinline__ bool gks_face(const double (&Wl)[3], const double (&Wlx)[3], const double (&Wr)[3],
                                         const double (&Wrx)[3], double dt, double gm1, const GksConst &gk,
                                         double (&Fn)[3], double (&Ft)[3])
{
    const Maxw ml = maxwellian(Wl, gm1), mr = maxwellian(Wr, gm1);
    const double K = gk.K;
    bool ok = ml.ok && mr.ok;
    double Mlf[kNM], Mlp[kNM], Mrf[kNM], Mrn[kNM];
    moments_full(ml, Mlf);
    moments_half(ml, 1.0, Mlp);
    moments_full(mr, Mrf);
    moments_half(mr, -1.0, Mrn);
    const double Xl2 = K * 0.5 / ml.lam, Xl4 = (K + 2.0) * 0.5 / ml.lam * Xl2;
    const double Xr2 = K * 0.5 / mr.lam, Xr4 = (K + 2.0) * 0.5 / mr.lam * Xr2;
    double al[3], Al[3], ar[3], Ar[3];
    slopes(ml, K, Mlf, Xl2, Xl4, Wlx, al, Al);
    slopes(mr, K, Mrf, Xr2, Xr4, Wrx, ar, Ar);

    // equilibrium state at the interface and its slope (kinetic weighting)
    const double one[3] = {1.0, 0.0, 0.0};
    double tl[3], tr[3], Wc[3], Wcx[3];
    lin_moment<0>(one, Mlp, Xl2, Xl4, tl);
    lin_moment<0>(one, Mrn, Xr2, Xr4, tr);
#pragma unroll
    for (int j = 0; j < 3; ++j) Wc[j] = ml.rho * tl[j] + mr.rho * tr[j];
    lin_moment<0>(al, Mlp, Xl2, Xl4, tl);
    lin_moment<0>(ar, Mrn, Xr2, Xr4, tr);
#pragma unroll
    for (int j = 0; j < 3; ++j) Wcx[j] = ml.rho * tl[j] + mr.rho * tr[j];
    const Maxw mc = maxwellian(Wc, gm1);
    ok = ok && mc.ok;
    double Mcf[kNM];
    moments_full(mc, Mcf);
    const double Xc2 = K * 0.5 / mc.lam, Xc4 = (K + 2.0) * 0.5 / mc.lam * Xc2;
    double ac[3], Ac[3];
    slopes(mc, K, Mcf, Xc2, Xc4, Wcx, ac, Ac);

    // moment terms of the distribution, independent of the time interval
    double e0[3], e1[3], e2[3], l0[3], l1[3], l2[3], r0[3], r1[3], r2[3];
    lin_moment<1>(one, Mcf, Xc2, Xc4, e0);
    lin_moment<2>(ac, Mcf, Xc2, Xc4, e1);
    lin_moment<1>(Ac, Mcf, Xc2, Xc4, e2);
    lin_moment<1>(one, Mlp, Xl2, Xl4, l0);
    lin_moment<2>(al, Mlp, Xl2, Xl4, l1);
    lin_moment<1>(Al, Mlp, Xl2, Xl4, l2);
    lin_moment<1>(one, Mrn, Xr2, Xr4, r0);
    lin_moment<2>(ar, Mrn, Xr2, Xr4, r1);
    lin_moment<1>(Ar, Mrn, Xr2, Xr4, r2);

    const double pl = 0.5 * ml.rho / ml.lam, pr = 0.5 * mr.rho / mr.lam;
    const double taun = gk.c1 * dt + gk.c2 * fabs(pl - pr) / (pl + pr) * dt;
    const double tau = gk.tau;
    double F[2][3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double d = h == 0 ? dt : 0.5 * dt;
        // time integrals of the coefficients over [0, d]
        const double E = exp(-d / taun);
        const double i0 = taun * (1.0 - E);
        const double i1 = taun * taun * (1.0 - E) - taun * d * E;
        const double q0 = d - i0;
        const double q1 = i1 + tau * i0 - tau * d;
        const double q2 = 0.5 * d * d - tau * d + tau * i0;
        const double q3 = i0;
        const double q4 = tau * i0 + i1;
        const double q5 = tau * i0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double fc = mc.rho * (q0 * e0[j] + q1 * e1[j] + q2 * e2[j]);
            const double fl = ml.rho * (q3 * l0[j] - q4 * l1[j] - q5 * l2[j]);
            const double fr = mr.rho * (q3 * r0[j] - q4 * r1[j] - q5 * r2[j]);
            F[h][j] = fc + fl + fr;
        }
    }
    const double idt = 1.0 / dt;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Fn[j] = ok ? (4.0 * F[1][j] - F[0][j]) * idt : __builtin_nan("");
        Ft[j] = ok ? 4.0 * (F[0][j] - 2.0 * F[1][j]) * idt * idt : __builtin_nan("");
    }
    return ok;
}

// ---------------------------------------------------------------------------
// 2D (Sec. 2.1): the flux at a Gauss point is evaluated in the local frame
// of its face -- u along the normal, v along the face,
// psi = (1, u, v, (u^2 + v^2 + xi^2)/2), K = (4 - 2 gamma)/(gamma - 1) --
// with the tangential slopes entering through a_t v in a . u = a_n u + a_t v.
// ---------------------------------------------------------------------------
constexpr int kNV2 = 6;   // <v^0> .. <v^5>

struct Maxw2 {
    double rho, U, V, lam;
    bool ok;
};

__device__ __forceinline__ Maxw2 maxwellian2(const double (&W)[4], double gm1)
{
    Maxw2 m;
    m.rho = W[0];
    const double ir = 1.0 / W[0];
    m.U = W[1] * ir;
    m.V = W[2] * ir;
    const double p = gm1 * (W[3] - 0.5 * (W[1] * m.U + W[2] * m.V));
    m.ok = m.rho > 0.0 && p > 0.0;
    m.lam = m.rho / (2.0 * p);
    return m;
}

template <int N>
__device__ __forceinline__ void moments_line(double U, double lam, double (&M)[N])
{
    const double h = 0.5 / lam;
    M[0] = 1.0;
    M[1] = U;
#pragma unroll
    for (int n = 0; n + 2 < N; ++n) M[n + 2] = fma(U, M[n + 1], (n + 1) * h * M[n]);
}

__device__ __forceinline__ void moments_half_line(double U, double lam, double sgn, double (&M)[kNM])
{
    const double h = 0.5 / lam;
    M[0] = 0.5 * erfc(-sgn * sqrt(lam) * U);
    M[1] = fma(U, M[0], sgn * 0.5 * exp(-lam * U * U) / sqrt(kPi * lam));
#pragma unroll
    for (int n = 0; n + 2 < kNM; ++n) M[n + 2] = fma(U, M[n + 1], (n + 1) * h * M[n]);
}

// <(c . psi) u^K v^Q psi_j>, j = 0..3: the six terms of c . psi times the
// terms of psi_j, each a product <u^n> <v^m> <xi^(2l)>.
template <int K, int Q>
__device__ __forceinline__ void lin_moment2(const double (&c)[4], const double (&Mu)[kNM], const double (&Mv)[kNV2],
                                            double X2, double X4, double (&out)[4])
{
    const double X[3] = {1.0, X2, X4};
    const double ca[6] = {c[0], c[1], c[2], 0.5 * c[3], 0.5 * c[3], 0.5 * c[3]};
    constexpr int na[6] = {0, 1, 0, 2, 0, 0}, ma[6] = {0, 0, 1, 0, 2, 0}, la[6] = {0, 0, 0, 0, 0, 1};
    constexpr double cb[6] = {1.0, 1.0, 1.0, 0.5, 0.5, 0.5};
    constexpr int jb[6] = {0, 1, 2, 3, 3, 3};
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b < 6; ++b)
            out[jb[b]] += ca[a] * cb[b] * Mu[K + na[a] + na[b]] * Mv[Q + ma[a] + ma[b]] * X[la[a] + la[b]];
}

// App. A's closed-form solution of M a = b in 2D.
__device__ __forceinline__ void micro_slope2(const Maxw2 &m, double K, const double (&b)[4], double (&a)[4])
{
    const double c = m.U * m.U + m.V * m.V + (K + 2.0) / (2.0 * m.lam);
    const double R4 = 2.0 * b[3] - c * b[0];
    const double R3 = b[2] - m.V * b[0];
    const double R2 = b[1] - m.U * b[0];
    a[3] = 4.0 * m.lam * m.lam / (K + 2.0) * (R4 - 2.0 * m.U * R2 - 2.0 * m.V * R3);
    a[2] = 2.0 * m.lam * R3 - m.V * a[3];
    a[1] = 2.0 * m.lam * R2 - m.U * a[3];
    a[0] = b[0] - m.U * a[1] - m.V * a[2] - 0.5 * a[3] * c;
}

// Normal and tangential slopes from W_n, W_t; time slope A from
// <A + a_n u + a_t v> = 0.
__device__ __forceinline__ void slopes2(const Maxw2 &m, double K, const double (&Muf)[kNM], const double (&Mv)[kNV2],
                                        double X2, double X4, const double (&Wn)[4], const double (&Wt)[4],
                                        double (&an)[4], double (&at)[4], double (&A)[4])
{
    const double ir = 1.0 / m.rho;
    const double bn[4] = {Wn[0] * ir, Wn[1] * ir, Wn[2] * ir, Wn[3] * ir};
    const double bt[4] = {Wt[0] * ir, Wt[1] * ir, Wt[2] * ir, Wt[3] * ir};
    micro_slope2(m, K, bn, an);
    micro_slope2(m, K, bt, at);
    double t1[4], t2[4];
    lin_moment2<1, 0>(an, Muf, Mv, X2, X4, t1);
    lin_moment2<0, 1>(at, Muf, Mv, X2, X4, t2);
    const double bA[4] = {-(t1[0] + t2[0]), -(t1[1] + t2[1]), -(t1[2] + t2[2]), -(t1[3] + t2[3])};
    micro_slope2(m, K, bA, A);
}

// Time integrals over [0, d] of the coefficients of the distribution
// (Eq. GKS flux), d = dt (h = 0) and dt/2 (h = 1).
__device__ __forceinline__ void time_coefs(double dt, double tau, double taun, double (&q)[2][6])
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double d = h == 0 ? dt : 0.5 * dt;
        const double E = exp(-d / taun);
        const double i0 = taun * (1.0 - E);
        const double i1 = taun * taun * (1.0 - E) - taun * d * E;
        q[h][0] = d - i0;
        q[h][1] = i1 + tau * i0 - tau * d;
        q[h][2] = 0.5 * d * d - tau * d + tau * i0;
        q[h][3] = i0;
        q[h][4] = tau * i0 + i1;
        q[h][5] = tau * i0;
    }
}

// Contribution of one side's half-line Maxwellian (sgn = 1: left, u > 0;
// -1: right, u < 0) to the transported fluxes F[h] and to the kinetic
// averages W^c, W^c_n, W^c_t.
__device__ __forceinline__ void side_terms2(const Maxw2 &m, double sgn, const double (&Wn)[4], const double (&Wt)[4],
                                            double K, const double (&q)[2][6], double (&F)[2][4], double (&Wc)[4],
                                            double (&Wcn)[4], double (&Wct)[4])
{
    double Mf[kNM], Mh[kNM], Mv[kNV2];
    moments_line<kNM>(m.U, m.lam, Mf);
    moments_half_line(m.U, m.lam, sgn, Mh);
    moments_line<kNV2>(m.V, m.lam, Mv);
    const double X2 = K * 0.5 / m.lam, X4 = (K + 2.0) * 0.5 / m.lam * X2;
    double an[4], at[4], A[4];
    slopes2(m, K, Mf, Mv, X2, X4, Wn, Wt, an, at, A);
    const double one[4] = {1.0, 0.0, 0.0, 0.0};
    double t[4], x[4];
    lin_moment2<0, 0>(one, Mh, Mv, X2, X4, t);
#pragma unroll
    for (int j = 0; j < 4; ++j) Wc[j] = fma(m.rho, t[j], Wc[j]);
    lin_moment2<0, 0>(an, Mh, Mv, X2, X4, t);
#pragma unroll
    for (int j = 0; j < 4; ++j) Wcn[j] = fma(m.rho, t[j], Wcn[j]);
    lin_moment2<0, 0>(at, Mh, Mv, X2, X4, t);
#pragma unroll
    for (int j = 0; j < 4; ++j) Wct[j] = fma(m.rho, t[j], Wct[j]);
    // rho [q3 <u psi> - q4 (<(a_n.psi) u^2 psi> + <(a_t.psi) u v psi>) - q5 <(A.psi) u psi>]
    lin_moment2<1, 0>(one, Mh, Mv, X2, X4, t);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 4; ++j) F[h][j] = fma(m.rho * q[h][3], t[j], F[h][j]);
    lin_moment2<2, 0>(an, Mh, Mv, X2, X4, t);
    lin_moment2<1, 1>(at, Mh, Mv, X2, X4, x);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 4; ++j) F[h][j] = fma(-m.rho * q[h][4], t[j] + x[j], F[h][j]);
    lin_moment2<1, 0>(A, Mh, Mv, X2, X4, t);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 4; ++j) F[h][j] = fma(-m.rho * q[h][5], t[j], F[h][j]);
}

// Flux and time derivative at t_n at one Gauss point, local frame.  The
// sides are taken one after the other (their terms accumulate into the
// transported fluxes and the kinetic averages), then the equilibrium part.
__device__ __forceinline__ bool gks2_point(const double (&Wl)[4], const double (&Wln)[4], const double (&Wlt)[4],
                                           const double (&Wr)[4], const double (&Wrn)[4], const double (&Wrt)[4],
                                           double dt, double gm1, const GksConst &gk, double (&Fn)[4],
                                           double (&Ft)[4])
{
    const double K = gk.K;
    const Maxw2 ml = maxwellian2(Wl, gm1), mr = maxwellian2(Wr, gm1);
    const double pl = 0.5 * ml.rho / ml.lam, pr = 0.5 * mr.rho / mr.lam;
    const double jump = gk.c2 * fabs(pl - pr) / (pl + pr) * dt;
    double tau = gk.tau, taun = gk.c1 * dt + jump;
    if (gk.mu > 0.0) {
        // viscous: tau = mu / p of the equilibrium state W^c (the kinetic
        // average of the two half Maxwellians), tau_n = tau + the jump term
        const double one[4] = {1.0, 0.0, 0.0, 0.0};
        double Mh[kNM], Mv[kNV2], t[4], Wc0[4];
        moments_half_line(ml.U, ml.lam, 1.0, Mh);
        moments_line<kNV2>(ml.V, ml.lam, Mv);
        const double Xl2 = K * 0.5 / ml.lam;
        lin_moment2<0, 0>(one, Mh, Mv, Xl2, 0.0, t);
#pragma unroll
        for (int j = 0; j < 4; ++j) Wc0[j] = ml.rho * t[j];
        moments_half_line(mr.U, mr.lam, -1.0, Mh);
        moments_line<kNV2>(mr.V, mr.lam, Mv);
        const double Xr2 = K * 0.5 / mr.lam;
        lin_moment2<0, 0>(one, Mh, Mv, Xr2, 0.0, t);
#pragma unroll
        for (int j = 0; j < 4; ++j) Wc0[j] = fma(mr.rho, t[j], Wc0[j]);
        const Maxw2 m0 = maxwellian2(Wc0, gm1);
        tau = gk.mu / (0.5 * m0.rho / m0.lam);
        taun = tau + jump;
    }
    double q[2][6];
    time_coefs(dt, tau, taun, q);
    double F[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    double Wc[4] = {0, 0, 0, 0}, Wcn[4] = {0, 0, 0, 0}, Wct[4] = {0, 0, 0, 0};
    side_terms2(ml, 1.0, Wln, Wlt, K, q, F, Wc, Wcn, Wct);
    side_terms2(mr, -1.0, Wrn, Wrt, K, q, F, Wc, Wcn, Wct);
    const Maxw2 mc = maxwellian2(Wc, gm1);
    const bool ok = ml.ok && mr.ok && mc.ok;
    {
        double Mf[kNM], Mv[kNV2];
        moments_line<kNM>(mc.U, mc.lam, Mf);
        moments_line<kNV2>(mc.V, mc.lam, Mv);
        const double X2 = K * 0.5 / mc.lam, X4 = (K + 2.0) * 0.5 / mc.lam * X2;
        double an[4], at[4], A[4];
        slopes2(mc, K, Mf, Mv, X2, X4, Wcn, Wct, an, at, A);
        const double one[4] = {1.0, 0.0, 0.0, 0.0};
        double t[4], x[4];
        // rho_c [q0 <u psi> + q1 (<(a_n.psi) u^2 psi> + <(a_t.psi) u v psi>) + q2 <(A.psi) u psi>]
        lin_moment2<1, 0>(one, Mf, Mv, X2, X4, t);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int j = 0; j < 4; ++j) F[h][j] = fma(mc.rho * q[h][0], t[j], F[h][j]);
        lin_moment2<2, 0>(an, Mf, Mv, X2, X4, t);
        lin_moment2<1, 1>(at, Mf, Mv, X2, X4, x);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int j = 0; j < 4; ++j) F[h][j] = fma(mc.rho * q[h][1], t[j] + x[j], F[h][j]);
        lin_moment2<1, 0>(A, Mf, Mv, X2, X4, t);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int j = 0; j < 4; ++j) F[h][j] = fma(mc.rho * q[h][2], t[j], F[h][j]);
    }
    const double idt = 1.0 / dt;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        Fn[j] = ok ? (4.0 * F[1][j] - F[0][j]) * idt : __builtin_nan("");
        Ft[j] = ok ? 4.0 * (F[0][j] - 2.0 * F[1][j]) * idt * idt : __builtin_nan("");
    }
    return ok;
}

// Reconstruction of one direction: per flux face and Gauss point, both
// sides' values, normal slopes and tangential slopes, into rec[c][face] with
// c = (side G + k) 12 + (0..3 value, 4..7 normal slope, 8..11 tangential
// slope).  Tiles as the LF sweep: phase 1 reconstructs every cell the
// tangential stencils need along DIR (values and normal slopes at both
// faces), phase 2 one lane per (face, side) reconstructs along the face.
template <int DIR, int R, int T0, int T1, int NT>
__global__ void __launch_bounds__(NT) k_gks2d_recon(Gks2DArgs a)
{
    constexpr int NV = 4, G = R, OI = R - 1;
    using S = SweepShape<DIR, R, T0, T1>;
    constexpr int UX = S::UX, UY = S::UY, TX = S::TX, TY = S::TY, FX = S::FX, FY = S::FY;
    constexpr int SY = (DIR == 0) ? UY : TY, SX = (DIR == 0) ? TX : UX;
    __shared__ double sU[NV][UY][UX];
    __shared__ double sSN[UY][UX];
    __shared__ double sST[SY][SX];
    // face traces and their normal slopes, right- and left-face values of
    // each cell: four segments of one array, placed so that the two lanes of
    // a face pair (8 faces per 16 lanes) read addresses 8 doubles apart
    // modulo 16 (the LDS serves a 64-bit read to 16 lanes per cycle, double
    // d in bank pair d mod 16); the upper side reads the next column (x
    // faces, +1) or the next row (y faces, +TX)
    constexpr int NT1 = NV * TY * TX;
    constexpr int SEG = (NT1 + 15) / 16 * 16;
    constexpr int TSTEP = (DIR == 0) ? 1 : TX;
    constexpr int PAIR = SEG + ((8 - TSTEP) % 16 + 16) % 16;
    constexpr int OTL = PAIR, ODR = (OTL + NT1 + 15) / 16 * 16, ODL = ODR + PAIR;
    __shared__ double sT[ODL + NT1];
    double(*sTR)[TY][TX] = reinterpret_cast<double(*)[TY][TX]>(&sT[0]);
    double(*sTL)[TY][TX] = reinterpret_cast<double(*)[TY][TX]>(&sT[OTL]);
    double(*sDR)[TY][TX] = reinterpret_cast<double(*)[TY][TX]>(&sT[ODR]);
    double(*sDL)[TY][TX] = reinterpret_cast<double(*)[TY][TX]>(&sT[ODL]);
    if (a.skip != nullptr && *a.skip != 0.0) return;
    const int tid = threadIdx.x;
    int btx, bty;
    xcd_tile(btx, bty);
    const int i0 = btx * T0, j0 = bty * T1;
    const int ox = (DIR == 0) ? i0 - 1 - R : i0 - R;
    const int oy = (DIR == 0) ? j0 - R : j0 - 1 - R;
    const MethodConst &mc = a.mc;
    const double inv_hn = DIR == 0 ? a.inv_dx : a.inv_dy, inv_ht = DIR == 0 ? a.inv_dy : a.inv_dx;

    for (int it = tid; it < UX * UY; it += NT) {
        const int lx = it % UX, ly = it / UX;
        const int I = ox + lx + a.ng, J = oy + ly + a.ng;
        const bool in = I < a.NX && J < a.NY;
        const long long pos = (long long)J * a.ld + I;
#pragma unroll
        for (int v = 0; v < NV; ++v) sU[v][ly][lx] = in ? a.U[v * a.plane + pos] : 0.0;
        sSN[ly][lx] = in ? (DIR == 0 ? a.sx[pos] : a.sy[pos]) : 0.0;
        const int sty = (DIR == 0) ? ly : ly - R, stx = (DIR == 0) ? lx - R : lx;
        if (sty >= 0 && sty < SY && stx >= 0 && stx < SX) sST[sty][stx] = in ? (DIR == 0 ? a.sy[pos] : a.sx[pos]) : 0.0;
    }
    __syncthreads();

    for (int it = tid; it < TX * TY; it += NT) {
        // x faces (TX = 17): groups of 16 lanes take 16 columns of one row,
        // the last column is walked down its rows (distinct bank pairs)
        int tx, ty;
        if constexpr (DIR == 0 && TX > 16) {
            constexpr int MAIN = 16 * TY;
            if (it < MAIN) {
                tx = it % 16;
                ty = it / 16;
            } else {
                tx = 16 + (it - MAIN) / TY;
                ty = (it - MAIN) % TY;
            }
        } else {
            tx = it % TX;
            ty = it / TX;
        }
        const int lx = (DIR == 0) ? tx + R : tx;
        const int ly = (DIR == 0) ? ty : ty + R;
        const int x = ox + lx, y = oy + ly;
        const bool need = (DIR == 0) ? (x <= a.nx && y < a.ny + R) : (x < a.nx + R && y <= a.ny);
        if (!need) continue;
        double s[2 * R];
#pragma unroll
        for (int m = -R; m < R; ++m) s[m + R] = (DIR == 0) ? sSN[ly][lx + m] : sSN[ly + m][lx];
        auto ld = [&](int v, int m) { return (DIR == 0) ? sU[v][ly][lx + m] : sU[v][ly + m][lx]; };
        double val[NV][2], der[NV][2];
        reconstruct_with_slopes<R, NV, 2>(ld, s, mc, 0, val, der);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            sTR[v][ty][tx] = val[v][0];
            sTL[v][ty][tx] = val[v][1];
            sDR[v][ty][tx] = der[v][0] * inv_hn;
            sDL[v][ty][tx] = der[v][1] * inv_hn;
        }
    }
    __syncthreads();

    for (int it = tid; it < 2 * FX * FY; it += NT) {
        const int side = it & 1, f = it >> 1;
        const int fx = f % FX, fy = f / FX;
        const int x = DIR == 0 ? i0 - 1 + fx : i0 + fx;
        const int y = DIR == 0 ? j0 + fy : j0 - 1 + fy;
        if (DIR == 0 ? (x > a.nx - 1 || y >= a.ny) : (x >= a.nx || y > a.ny - 1)) continue;
        const double *tr = side == 0 ? &sTR[0][0][0] : &sTL[0][0][0];
        const double *dr = side == 0 ? &sDR[0][0][0] : &sDL[0][0][0];
        double s[2 * R], val[NV][G], der[NV][G], nrm[NV][G];
        if (DIR == 0) {
            const int tx = fx + side;
#pragma unroll
            for (int m = -R; m < R; ++m) s[m + R] = sST[fy + R + m][tx];
            auto ldv = [&](int v, int m) { return tr[(v * TY + fy + R + m) * TX + tx]; };
            auto ldd = [&](int v, int m) { return dr[(v * TY + fy + R + m) * TX + tx]; };
            reconstruct_with_slopes<R, NV, G>(ldv, s, mc, 2, val, der);
            reconstruct_cell<R, NV, G>(ldd, s, mc, OI, 2, nrm);
        } else {
            const int ty = fy + side;
#pragma unroll
            for (int m = -R; m < R; ++m) s[m + R] = sST[ty][fx + R + m];
            auto ldv = [&](int v, int m) { return tr[(v * TY + ty) * TX + fx + R + m]; };
            auto ldd = [&](int v, int m) { return dr[(v * TY + ty) * TX + fx + R + m]; };
            reconstruct_with_slopes<R, NV, G>(ldv, s, mc, 2, val, der);
            reconstruct_cell<R, NV, G>(ldd, s, mc, OI, 2, nrm);
        }
        const long long fid = DIR == 0 ? (long long)y * (a.nx + 1) + (x + 1) : (long long)(y + 1) * a.nx + x;
        const long long nf = a.nfaces;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            double *dst = a.rec + (long long)((side * G + k) * 12) * nf + fid;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                dst[(long long)v * nf] = val[v][k];
                dst[(long long)(4 + v) * nf] = nrm[v][k];
                dst[(long long)(8 + v) * nf] = der[v][k] * inv_ht;
            }
        }
    }
}

// Face fluxes of one direction: one thread per flux face, G Gauss points:
// strength, positivity fallback, local frame (normal (1,0) for x faces,
// (0,1) for y faces, tangent (-sin, cos)), flux, back to the global frame,
// quadrature.
template <int DIR, int R>
__global__ void __launch_bounds__(kGksPointThreads) k_gks2d_flux(Gks2DArgs a)
{
    constexpr int G = R, OI = R - 1;
    if (a.skip != nullptr && *a.skip != 0.0) return;
    const long long fid = (long long)blockIdx.x * kGksPointThreads + threadIdx.x;
    if (fid >= a.nfaces) return;
    int i, j;   // left/lower cell; the other is (i+1, j) or (i, j+1)
    if (DIR == 0) {
        j = (int)(fid / (a.nx + 1));
        i = (int)(fid % (a.nx + 1)) - 1;
    } else {
        j = (int)(fid / a.nx) - 1;
        i = (int)(fid % a.nx);
    }
    const long long pl = (long long)(j + a.ng) * a.ld + i + a.ng;
    const long long pr = DIR == 0 ? pl + 1 : pl + a.ld;
    const long long nf = a.nfaces;
    const double dt = *a.dt;
    double Fs[4] = {0, 0, 0, 0}, Fts[4] = {0, 0, 0, 0}, ssum = 0.0;
#pragma unroll 1
    for (int k = 0; k < G; ++k) {
        double W[2][4], Wn[2][4], Wt[2][4];
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const double *src = a.rec + (long long)((sd * G + k) * 12) * nf + fid;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                W[sd][v] = src[(long long)v * nf];
                Wn[sd][v] = src[(long long)(4 + v) * nf];
                Wt[sd][v] = src[(long long)(8 + v) * nf];
            }
        }
        const Prim ql = primitives<4>(W[0], DIR, a.mc), qr = primitives<4>(W[1], DIR, a.mc);
        ssum += sigma_point(ql, qr);
        if (a.mc.flags & 1) {
            const bool okd[2] = {ql.ok, qr.ok};
#pragma unroll
            for (int sd = 0; sd < 2; ++sd)
                if (!okd[sd]) {
                    const long long pc = sd == 0 ? pl : pr;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        W[sd][v] = a.U[v * a.plane + pc];
                        Wn[sd][v] = 0.0;
                        Wt[sd][v] = 0.0;
                    }
                }
        }
        // local frame: x faces as they are; y faces (rho, rho v, -rho u, E),
        // tangential derivative along -x
        double lW[2][4], lWn[2][4], lWt[2][4];
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            if (DIR == 0) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    lW[sd][v] = W[sd][v];
                    lWn[sd][v] = Wn[sd][v];
                    lWt[sd][v] = Wt[sd][v];
                }
            } else {
                lW[sd][0] = W[sd][0];
                lW[sd][1] = W[sd][2];
                lW[sd][2] = -W[sd][1];
                lW[sd][3] = W[sd][3];
                lWn[sd][0] = Wn[sd][0];
                lWn[sd][1] = Wn[sd][2];
                lWn[sd][2] = -Wn[sd][1];
                lWn[sd][3] = Wn[sd][3];
                lWt[sd][0] = -Wt[sd][0];
                lWt[sd][1] = -Wt[sd][2];
                lWt[sd][2] = Wt[sd][1];
                lWt[sd][3] = -Wt[sd][3];
            }
        }
        double fn[4], ft[4];
        gks2_point(lW[0], lWn[0], lWt[0], lW[1], lWn[1], lWt[1], dt, a.mc.gm1, a.gk, fn, ft);
        double Fg[4], Ftg[4];
        if (DIR == 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                Fg[v] = fn[v];
                Ftg[v] = ft[v];
            }
        } else {
            Fg[0] = fn[0];
            Fg[1] = -fn[2];
            Fg[2] = fn[1];
            Fg[3] = fn[3];
            Ftg[0] = ft[0];
            Ftg[1] = -ft[2];
            Ftg[2] = ft[1];
            Ftg[3] = ft[3];
        }
        const double eta = kTab.eta[OI][k];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            Fs[v] = fma(eta, Fg[v], Fs[v]);
            Fts[v] = fma(eta, Ftg[v], Fts[v]);
        }
    }
    // no-slip adiabatic wall: no mass or energy crosses it (the mirrored
    // ghost cells reverse the tangential velocity too, which the
    // tangential-slope terms do not see as a symmetry)
    const int lo = DIR == 0 ? a.bc[0] : a.bc[2], hi = DIR == 0 ? a.bc[1] : a.bc[3];
    const int k1 = DIR == 0 ? i : j, n1 = DIR == 0 ? a.nx : a.ny;
    if ((k1 == -1 && lo == ASE_BC_NOSLIP) || (k1 == n1 - 1 && hi == ASE_BC_NOSLIP)) {
        Fs[0] = Fs[3] = 0.0;
        Fts[0] = Fts[3] = 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        a.F[(long long)v * nf + fid] = Fs[v];
        a.Ft[(long long)v * nf + fid] = Fts[v];
    }
    a.sig_out[pl] = ssum / (double)G;
}

// Divergences of F and F_t and the S2O4 stage combination on interior cells.
__global__ void __launch_bounds__(kGksPointThreads) k_gks2d_update(Gks2DUpdate a)
{
    if (a.skip != nullptr && *a.skip != 0.0) return;
    const long long c = (long long)blockIdx.x * kGksPointThreads + threadIdx.x;
    if (c >= (long long)a.nx * a.ny) return;
    const int i = (int)(c % a.nx), j = (int)(c / a.nx);
    const long long fxp = (long long)j * (a.nx + 1) + i + 1, fxm = fxp - 1;
    const long long fyp = (long long)(j + 1) * a.nx + i, fym = fyp - a.nx;
    const long long pos = (long long)(j + a.ng) * a.ld + i + a.ng;
    const double dt = *a.dt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long long e = v * a.plane + pos;
        const double L = -(a.Fx[v * a.nfx + fxp] - a.Fx[v * a.nfx + fxm]) * a.inv_dx -
                         (a.Fy[v * a.nfy + fyp] - a.Fy[v * a.nfy + fym]) * a.inv_dy;
        const double Lt = -(a.Ftx[v * a.nfx + fxp] - a.Ftx[v * a.nfx + fxm]) * a.inv_dx -
                          (a.Fty[v * a.nfy + fyp] - a.Fty[v * a.nfy + fym]) * a.inv_dy;
        if (a.stage == 1) {
            a.Uout[e] = a.U[e] + 0.5 * dt * L + 0.125 * dt * dt * Lt;
            a.L0[e] = L;
            a.Lt0[e] = Lt;
        } else {
            a.Uout[e] = a.Un[e] + dt * a.L0[e] + dt * dt / 6.0 * (a.Lt0[e] + 2.0 * Lt);
        }
    }
}

// ---------------------------------------------------------------------------
// One S2O4 stage on one tile of T cells (one workgroup of NT lanes, each
// per-item loop one pass).
// ---------------------------------------------------------------------------
template <int R, int T>
struct LdsGks {
    static constexpr int UX = T + 2 + 2 * R;
    double sU[3][UX];
    double sS[UX];
    double sTR[3][T + 2], sTL[3][T + 2];   // values at the right / left face
    double sDR[3][T + 2], sDL[3][T + 2];   // x-slopes there
    double sF[3][T + 1], sFt[3][T + 1];
};

template <int R, int T, int NT>
__global__ void __launch_bounds__(NT) k_gks1d(Gks1DArgs a)
{
    constexpr int NV = 3;
    constexpr int UX = LdsGks<R, T>::UX;
    __shared__ LdsGks<R, T> L;
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * T;
    const int ox = i0 - 1 - R;
    // a finished run: nothing changes (state and strengths stay)
    if (a.skip != nullptr && *a.skip != 0.0) return;
    const MethodConst &mc = a.mc;

    for (int lx = tid; lx < UX; lx += NT) {
        const int I = ox + lx + a.ng;
        const bool in = I < a.NX;
#pragma unroll
        for (int v = 0; v < NV; ++v) L.sU[v][lx] = in ? a.U[v * a.plane + I] : 0.0;
        L.sS[lx] = in ? a.sx[I] : 0.0;
    }
    __syncthreads();

    for (int tx = tid; tx < T + 2; tx += NT) {
        const int lx = tx + R;
        const int x = ox + lx;
        if (x > a.nx) continue;
        double s[2 * R];
#pragma unroll
        for (int m = -R; m < R; ++m) s[m + R] = L.sS[lx + m];
        auto ld = [&](int v, int m) { return L.sU[v][lx + m]; };
        double val[NV][2], der[NV][2];
        reconstruct_with_slopes<R, NV, 2>(ld, s, mc, 0, val, der);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            L.sTR[v][tx] = val[v][0];
            L.sTL[v][tx] = val[v][1];
            L.sDR[v][tx] = der[v][0] * a.inv_dx;
            L.sDL[v][tx] = der[v][1] * a.inv_dx;
        }
    }
    __syncthreads();

    const double dt = *a.dt;
    for (int fx = tid; fx < T + 1; fx += NT) {
        const int x = i0 - 1 + fx;   // face x + 1/2
        if (x > a.nx - 1) continue;
        double Wl[NV], Wr[NV], Wlx[NV], Wrx[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Wl[v] = L.sTR[v][fx];
            Wr[v] = L.sTL[v][fx + 1];
            Wlx[v] = L.sDR[v][fx];
            Wrx[v] = L.sDL[v][fx + 1];
        }
        const Prim ql = primitives<NV>(Wl, 0, mc), qr = primitives<NV>(Wr, 0, mc);
        const double sg = sigma_point(ql, qr);
        if (mc.flags & 1) {
            // positivity fallback: a non-physical side becomes its cell average, flat
            if (!ql.ok) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Wl[v] = L.sU[v][fx + R];
                    Wlx[v] = 0.0;
                }
            }
            if (!qr.ok) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Wr[v] = L.sU[v][fx + R + 1];
                    Wrx[v] = 0.0;
                }
            }
        }
        double Fn[NV], Ft[NV];
        gks_face(Wl, Wlx, Wr, Wrx, dt, mc.gm1, a.gk, Fn, Ft);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            L.sF[v][fx] = Fn[v];
            L.sFt[v][fx] = Ft[v];
        }
        if (fx > 0 || i0 == 0) a.sig_out[x + a.ng] = sg;
    }
    __syncthreads();

    for (int cx = tid; cx < T; cx += NT) {
        const int x = i0 + cx;
        if (x >= a.nx) continue;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const long long e = v * a.plane + x + a.ng;
            const double Lx = -(L.sF[v][cx + 1] - L.sF[v][cx]) * a.inv_dx;
            const double Lt = -(L.sFt[v][cx + 1] - L.sFt[v][cx]) * a.inv_dx;
            if (a.stage == 1) {
                // W* = W^n + dt/2 L(W^n) + dt^2/8 L_t(W^n)
                a.Uout[e] = a.U[e] + 0.5 * dt * Lx + 0.125 * dt * dt * Lt;
                a.L0[e] = Lx;
                a.Lt0[e] = Lt;
            } else {
                // W^{n+1} = W^n + dt L(W^n) + dt^2/6 (L_t(W^n) + 2 L_t(W*))
                a.Uout[e] = a.Un[e] + dt * a.L0[e] + dt * dt / 6.0 * (a.Lt0[e] + 2.0 * Lt);
            }
        }
    }
}

// Flux and time derivative of independent faces ([3][n] arrays).
__global__ void __launch_bounds__(kGksPointThreads) k_gks_points(GksPointArgs a)
{
    const int f = blockIdx.x * kGksPointThreads + threadIdx.x;
    if (f >= a.n) return;
    double Wl[3], Wr[3], Wlx[3], Wrx[3], Fn[3], Ft[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        Wl[v] = a.Wl[(long long)v * a.n + f];
        Wr[v] = a.Wr[(long long)v * a.n + f];
        Wlx[v] = a.Wlx[(long long)v * a.n + f];
        Wrx[v] = a.Wrx[(long long)v * a.n + f];
    }
    gks_face(Wl, Wlx, Wr, Wrx, a.dt, a.gm1, a.gk, Fn, Ft);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        a.Fn[(long long)v * a.n + f] = Fn[v];
        a.Ft[(long long)v * a.n + f] = Ft[v];
    }
}

constexpr int kGksNT = 256;
// 2D reconstruction tiles: x faces 15 x 7 cells, y faces 16 x 7 cells, 256
// lanes each (phase 1 in one pass of 255 / 216 cells, phase 2 one (face,
// side) item per lane).  At 147 registers three 4-wave workgroups fit a CU.
constexpr int kGX_T0 = 15, kGX_T1 = 7, kGX_NT = 256, kGY_T0 = 16, kGY_T1 = 7, kGY_NT = 256;

template <int R>
void gks1d_r(int nx, const Gks1DArgs &a, hipStream_t st)
{
    constexpr int T = kGksNT - 2 * R - 2;
    dim3 grid((nx + T - 1) / T);
    k_gks1d<R, T, kGksNT><<<grid, kGksNT, 0, st>>>(a);
}
}  // namespace

void launch_gks1d(int R, int nx, const Gks1DArgs &a, hipStream_t st)
{
    switch (R) {
    case 1: gks1d_r<1>(nx, a, st); break;
    case 2: gks1d_r<2>(nx, a, st); break;
    case 3: gks1d_r<3>(nx, a, st); break;
    default: gks1d_r<4>(nx, a, st); break;
    }
}

template <int R>
void gks2d_r(int dir, bool recon, const Gks2DArgs &a, hipStream_t st)
{
    const unsigned fb = (unsigned)((a.nfaces + kGksPointThreads - 1) / kGksPointThreads);
    if (dir == 0) {
        dim3 grid((a.nx + kGX_T0 - 1) / kGX_T0, (a.ny + kGX_T1 - 1) / kGX_T1);
        if (recon) k_gks2d_recon<0, R, kGX_T0, kGX_T1, kGX_NT><<<grid, kGX_NT, 0, st>>>(a);
        else k_gks2d_flux<0, R><<<fb, kGksPointThreads, 0, st>>>(a);
    } else {
        dim3 grid((a.nx + kGY_T0 - 1) / kGY_T0, (a.ny + kGY_T1 - 1) / kGY_T1);
        if (recon) k_gks2d_recon<1, R, kGY_T0, kGY_T1, kGY_NT><<<grid, kGY_NT, 0, st>>>(a);
        else k_gks2d_flux<1, R><<<fb, kGksPointThreads, 0, st>>>(a);
    }
}

void launch_gks2d(int R, int dir, bool recon, const Gks2DArgs &a, hipStream_t st)
{
    switch (R) {
    case 1: gks2d_r<1>(dir, recon, a, st); break;
    case 2: gks2d_r<2>(dir, recon, a, st); break;
    case 3: gks2d_r<3>(dir, recon, a, st); break;
    default: gks2d_r<4>(dir, recon, a, st); break;
    }
}

void launch_gks2d_update(const Gks2DUpdate &u, hipStream_t st)
{
    const long long n = (long long)u.nx * u.ny;
    dim3 grid((unsigned)((n + kGksPointThreads - 1) / kGksPointThreads));
    k_gks2d_update<<<grid, kGksPointThreads, 0, st>>>(u);
}

void launch_gks_points(const GksPointArgs &a, hipStream_t st)
{
    dim3 grid((a.n + kGksPointThreads - 1) / kGksPointThreads);
    k_gks_points<<<grid, kGksPointThreads, 0, st>>>(a);
}

}  // namespace ase
