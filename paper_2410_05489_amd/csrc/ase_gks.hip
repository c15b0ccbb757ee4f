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

// dP/dxi of the WENO-Z-AO(5,3) polynomial at the right (f = 0) and left
// (f = 1) faces: the point-independent weights applied to the candidates'
// slopes.
__device__ __forceinline__ void weno_ao53_slopes(const double (&W)[5], const double al[4], const MethodConst &mc,
                                                 double (&d)[2])
{
    const WenoAO53 c = weno_ao53_setup(W, mc);
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const double *z = kTab.dz[f];
        const double Dm = al[0] * (c.am1 * z[0] + c.am2 * z[1]);
        const double D0 = al[1] * (c.a01 * z[0] + c.a02 * z[1]);
        const double Dp = al[2] * (c.ap1 * z[0] + c.ap2 * z[1]);
        const double D5 = al[3] * (c.b1 * z[0] + c.b2 * z[1] + c.b3 * z[2] + c.b4 * z[3]);
        const double inner = D5 * mc.inv_d5 - mc.r3m * Dm - mc.r30 * D0 - mc.r3m * Dp;
        d[f] = c.o5 * inner + c.om * Dm + c.o0 * D0 + c.op * Dp;
    }
}

// Slopes of the linear (2H+1)-cell polynomial at both faces (weights
// tabulated at compile time).
template <int NV, int H, class LD>
__device__ __forceinline__ void slopes_linear(LD ld, double (&der)[NV][2])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double w[2 * H + 1];
#pragma unroll
        for (int m = -H; m <= H; ++m) w[m + H] = ld(v, m);
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const double *c = kTab.dlin[H - 1][f];
            double acc = c[4 - H] * w[0];
#pragma unroll
            for (int m = -H + 1; m <= H; ++m) acc = fma(c[4 + m], w[m + H], acc);
            der[v][f] = acc;
        }
    }
}

// Values (val[v][0] right face, [1] left face) and xi-slopes of the ASE-DF
// polynomial of a cell: the level rule and values of the LF path, then the
// slopes of the same polynomial.
template <int R, int NV, class LD>
__device__ __forceinline__ void reconstruct_with_slopes(LD ld, const double (&s)[2 * R], const MethodConst &mc,
                                                        double (&val)[NV][2], double (&der)[NV][2])
{
    constexpr int OI = R - 1;
    const int lvl = reconstruct_cell<R, NV, 2>(ld, s, mc, OI, 0, val);
    if constexpr (R == 1) {
        const double al = df_alpha(s[0] + s[1], mc.thr);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double Wm = ld(v, -1), W0 = ld(v, 0), Wp = ld(v, 1);
            const double a1 = Wp - W0, a2 = 0.5 * (Wm - 2.0 * W0 + Wp);
#pragma unroll
            for (int f = 0; f < 2; ++f) der[v][f] = al * (a1 * kTab.dz[f][0] + a2 * kTab.dz[f][1]);
        }
    } else if (lvl == 9) {
        if constexpr (R >= 4) slopes_linear<NV, 4>(ld, der);
    } else if (lvl == 7) {
        if constexpr (R >= 3) slopes_linear<NV, 3>(ld, der);
    } else if (lvl == 5) {
        slopes_linear<NV, 2>(ld, der);
    } else {
        double al[4];
        al[0] = df_alpha(ssum<R>(s, -2, 0), mc.thr);
        al[1] = df_alpha(ssum<R>(s, -1, 1), mc.thr);
        al[2] = df_alpha(ssum<R>(s, 0, 2), mc.thr);
        al[3] = df_alpha(ssum<R>(s, -2, 2), mc.thr);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double W[5], d[2];
#pragma unroll
            for (int m = -2; m <= 2; ++m) W[m + 2] = ld(v, m);
            weno_ao53_slopes(W, al, mc, d);
            der[v][0] = d[0];
            der[v][1] = d[1];
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
        reconstruct_with_slopes<R, NV>(ld, s, mc, val, der);
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

void launch_gks_points(const GksPointArgs &a, hipStream_t st)
{
    dim3 grid((a.n + kGksPointThreads - 1) / kGksPointThreads);
    k_gks_points<<<grid, kGksPointThreads, 0, st>>>(a);
}

}  // namespace ase
