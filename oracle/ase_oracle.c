/*
 * ASE-DF oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the method of
 * Zhang, Zhao, Ji & Xu, "An Adaptive Reconstruction Method for Arbitrary
 * High-Order Accuracy Using Discontinuity Feedback" (arXiv 2410.05489):
 * adaptive-stencil-extension reconstruction driven by the discontinuity
 * feedback factor (ASE-DF), Lax-Friedrichs interface flux with Gauss
 * quadrature on faces, and the SSP-RK3 conservative update, for the 1D and
 * 2D compressible Euler equations.
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library; the GPU product path never calls it.
 *
 * Every step follows the paper in its own order and notation.  Where the
 * paper is garbled or silent, the reading taken is stated at the spot
 * (readings R1..R16 are listed in the design notes of the repository).
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC -lm
 *
 * Threads: the loops over grid lines (rows or columns) of the sweeps, the
 * residual, the first-order strengths and the stage combination run under
 * OpenMP.  Every iteration writes its own cells and faces and no parallel
 * loop reduces, so results are bitwise the same for any thread count
 * (orc_set_threads); the time-step maximum stays a serial loop.  Grids of
 * at most 4096 cells run every loop serially.
 *
 * Array layout (shared with callers, not with any GPU source):
 *   U[v*NY*ld + J*ld + I], I in [0,NX), J in [0,NY), NX = nx+2ng,
 *   NY = ny+2ng in 2D and 1 in 1D; interior cell (i,j) sits at
 *   I = i+ng, J = j+ng.  nvar = 3 in 1D (rho, rho u, E) and 4 in 2D
 *   (rho, rho u, rho v, rho E).
 *   sx[J*ld+I]: discontinuity strength of the x-face between (I,J), (I+1,J).
 *   sy[J*ld+I]: same for the y-face between (I,J) and (I,J+1).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Problem statement                                                          */
/* ------------------------------------------------------------------------ */

enum { ORC_BC_PERIODIC = 0, ORC_BC_TRANSMISSIVE = 1, ORC_BC_INFLOW_SLOT = 2, ORC_BC_REFLECTIVE = 3,
       ORC_BC_WALL_INFLOW = 4, ORC_BC_MOVING_SHOCK = 5, ORC_BC_NOSLIP = 6 };

/* Mirror sides: the slip wall and the no-slip adiabatic wall (Sec. 4,
   Example 5) both mirror the cells; the slip wall reverses the momentum
   normal to it, the no-slip wall the whole momentum. */
static int is_wall(int bc) { return bc == ORC_BC_REFLECTIVE || bc == ORC_BC_NOSLIP; }

typedef struct {
    int32_t dim;        /* 1 or 2 */
    int32_t nx, ny;     /* interior cells (ny = 1 in 1D) */
    int32_t ng;         /* ghost layers per side */
    int32_t ld;         /* row stride (>= nx + 2 ng) */
    int32_t bc[4];      /* x-lo, x-hi, y-lo, y-hi */
    double dx, dy;
    double y0;          /* lower edge of the domain in y (slot test) */
    double inflow[4];   /* conservative state of inflow ghost cells */
    double slot_lo, slot_hi;
    /* double Mach reflection (Sec. 4, Example 4): the y-lo side is inflow
       below wall_x0 and a slip wall beyond; the y-hi side is inflow below
       the shock position shock_x0 + shock_speed t and the outer state
       beyond (column centres, x0 the domain's left edge) */
    double x0, wall_x0, shock_x0, shock_speed;
    double outer[4];
} orc_grid;

/* Source of the interface states the DF strengths are computed from        */
/* (reading R9): LAGGED -- the Gauss-point states of the previous stage's   */
/* reconstruction; FIRST_ORDER -- the first-order (cell-average) states of  */
/* the current stage input.                                                  */
enum { ORC_DF_LAGGED = 0, ORC_DF_FIRST_ORDER = 1 };

typedef struct {
    int32_t order;      /* 1 (first order, test aid), 3, 5, 7, 9 */
    int32_t positivity_fallback;
    int32_t df_source;  /* ORC_DF_* */
    int32_t pad_;
    double gamma, cfl, sigma_thres, eps, d_hi, d_lo;
    double dt_cap;      /* > 0: dt = min(dt_cfl, dt_cap) */
} orc_params;

static int nvar_of(const orc_grid *g) { return g->dim == 1 ? 3 : 4; }
static int NXof(const orc_grid *g) { return g->nx + 2 * g->ng; }
static int NYof(const orc_grid *g) { return g->dim == 1 ? 1 : g->ny + 2 * g->ng; }
static size_t plane(const orc_grid *g) { return (size_t)NYof(g) * (size_t)g->ld; }
static int halfwidth(int r) { return r <= 1 ? 0 : (r - 1) / 2; }

/* Number of Gauss points per face: (r-1)/2 for order r (Sec. 2.1); in 1D the
 * face is a point.  Reading R13: fixed by the nominal order. */
static int ngauss(const orc_grid *g, int r)
{
    if (g->dim == 1) return 1;
    int G = (r - 1) / 2;
    return G < 1 ? 1 : G;
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre quadrature on the face, nodes on [-1/2, 1/2] and weights    */
/* normalised to sum 1 (Sec. 2.1, face integral = |l| sum eta_k F(x_k)).      */
/* ------------------------------------------------------------------------ */
static void gauss_legendre(int G, double *node, double *eta)
{
    if (G == 1) {
        node[0] = 0.0; eta[0] = 1.0;
    } else if (G == 2) {
        double a = 0.5 / sqrt(3.0);
        node[0] = -a; node[1] = a; eta[0] = 0.5; eta[1] = 0.5;
    } else if (G == 3) {
        double a = 0.5 * sqrt(3.0 / 5.0);
        node[0] = -a; node[1] = 0.0; node[2] = a;
        eta[0] = 5.0 / 18.0; eta[1] = 8.0 / 18.0; eta[2] = 5.0 / 18.0;
    } else { /* G == 4 */
        double s = 2.0 / 7.0 * sqrt(6.0 / 5.0);
        double a = 0.5 * sqrt(3.0 / 7.0 - s);   /* inner pair */
        double b = 0.5 * sqrt(3.0 / 7.0 + s);   /* outer pair */
        double wa = (18.0 + sqrt(30.0)) / 72.0; /* Legendre weights / 2 */
        double wb = (18.0 - sqrt(30.0)) / 72.0;
        node[0] = -b; node[1] = -a; node[2] = a; node[3] = b;
        eta[0] = wb; eta[1] = wa; eta[2] = wa; eta[3] = wb;
    }
}

/* ------------------------------------------------------------------------ */
/* Zero-mean basis on the cell [-1, 0] (Sec. 3, opening).  Reading R1: the    */
/* printed constants make Z_k zero-mean only with                            */
/*     Z_k(xi) = xi^k - (-1)^k / (k+1),   xi = x / dx,                        */
/* which is the basis in which every printed stencil coefficient is the      */
/* exact cell-average fit.                                                   */
/* ------------------------------------------------------------------------ */
static double Zk(int k, double xi)
{
    double p = 1.0;
    for (int m = 0; m < k; ++m) p *= xi;
    double mean = ((k % 2) == 0 ? 1.0 : -1.0) / (double)(k + 1);
    return p - mean;
}

/* dZ_k/dxi = k xi^(k-1): slopes of the reconstruction, which the gas-kinetic */
/* flux takes at the interface (Sec. 2.2; the derivative in x is this / dx).  */
static double dZk(int k, double xi)
{
    double p = (double)k;
    for (int m = 1; m < k; ++m) p *= xi;
    return p;
}

/* ------------------------------------------------------------------------ */
/* Stencil coefficients W_xk of the zero-mean polynomial on each stencil.    */
/* W points at W_0; W[m] is the cell average of the m-th neighbour.           */
/* ------------------------------------------------------------------------ */

/* S^{r3}_{-1}, S^{r3}_{0}, S^{r3}_{1} (Sec. 3.2). */
static void coef_r3(int k, const double *W, double a[2])
{
    if (k == -1) {
        a[0] = 2.0 * W[0] - 3.0 * W[-1] + W[-2];
        a[1] = 0.5 * (W[-2] - 2.0 * W[-1] + W[0]);
    } else if (k == 0) {
        a[0] = W[1] - W[0];
        a[1] = 0.5 * (W[-1] - 2.0 * W[0] + W[1]);
    } else {
        a[0] = W[1] - W[0];
        a[1] = 0.5 * (W[0] - 2.0 * W[1] + W[2]);
    }
}

/* S^{r5} (Sec. 3.2). */
static void coef_r5(const double *W, double a[4])
{
    a[0] = (-15.0 * W[0] + W[-1] + 15.0 * W[1] - W[2]) / 12.0;
    a[1] = (-8.0 * W[0] + 6.0 * W[-1] - W[-2] + 2.0 * W[1] + W[2]) / 8.0;
    a[2] = (3.0 * W[0] - W[-1] - 3.0 * W[1] + W[2]) / 6.0;
    a[3] = (6.0 * W[0] - 4.0 * W[-1] + W[-2] - 4.0 * W[1] + W[2]) / 24.0;
}

/* S^{r7} (Sec. 3.3).  Reading R2: the printed "2 f_3" in W_x1 is 2 W_3. */
static void coef_r7(const double *W, double a[6])
{
    a[0] = (-245.0 * W[0] + 25.0 * W[-1] - 2.0 * W[-2] + 245.0 * W[1] - 25.0 * W[2] + 2.0 * W[3]) / 180.0;
    a[1] = (-230.0 * W[0] + 210.0 * W[-1] - 57.0 * W[-2] + 7.0 * W[-3] + 15.0 * W[1] + 63.0 * W[2] - 8.0 * W[3]) / 240.0;
    a[2] = (28.0 * W[0] - 11.0 * W[-1] + W[-2] - 28.0 * W[1] + 11.0 * W[2] - W[3]) / 36.0;
    a[3] = (46.0 * W[0] - 39.0 * W[-1] + 15.0 * W[-2] - 2.0 * W[-3] - 24.0 * W[1] + 3.0 * W[2] + W[3]) / 144.0;
    a[4] = (-10.0 * W[0] + 5.0 * W[-1] - W[-2] + 10.0 * W[1] - 5.0 * W[2] + W[3]) / 120.0;
    a[5] = (-20.0 * W[0] + 15.0 * W[-1] - 6.0 * W[-2] + W[-3] + 15.0 * W[1] - 6.0 * W[2] + W[3]) / 720.0;
}

/* S^{r9} (Sec. 3.4). */
static void coef_r9(const double *W, double a[8])
{
    a[0] = (-7175.0 * W[0] + 889.0 * W[-1] - 119.0 * W[-2] + 9.0 * W[-3] + 7175.0 * W[1] - 889.0 * W[2] + 119.0 * W[3] - 9.0 * W[4]) / 5040.0;
    a[1] = (-27895.0 * W[0] + 28679.0 * W[-1] - 9835.0 * W[-2] + 2081.0 * W[-3] - 205.0 * W[-4] - 2065.0 * W[1]
            + 11459.0 * W[2] - 2455.0 * W[3] + 236.0 * W[4]) / 30240.0;
    a[2] = (1365.0 * W[0] - 587.0 * W[-1] + 89.0 * W[-2] - 7.0 * W[-3] - 1365.0 * W[1] + 587.0 * W[2] - 89.0 * W[3] + 7.0 * W[4]) / 1440.0;
    a[3] = (1174.0 * W[0] - 1160.0 * W[-1] + 556.0 * W[-2] - 128.0 * W[-3] + 13.0 * W[-4] - 464.0 * W[1] - 68.0 * W[2]
            + 88.0 * W[3] - 11.0 * W[4]) / 3456.0;
    a[4] = (-75.0 * W[0] + 41.0 * W[-1] - 11.0 * W[-2] + W[-3] + 75.0 * W[1] - 41.0 * W[2] + 11.0 * W[3] - W[4]) / 480.0;
    a[5] = (-380.0 * W[0] + 334.0 * W[-1] - 170.0 * W[-2] + 46.0 * W[-3] - 5.0 * W[-4] + 250.0 * W[1] - 86.0 * W[2]
            + 10.0 * W[3] + W[4]) / 8640.0;
    a[6] = (35.0 * W[0] - 21.0 * W[-1] + 7.0 * W[-2] - W[-3] - 35.0 * W[1] + 21.0 * W[2] - 7.0 * W[3] + W[4]) / 5040.0;
    a[7] = (70.0 * W[0] - 56.0 * W[-1] + 28.0 * W[-2] - 8.0 * W[-3] + W[-4] - 56.0 * W[1] + 28.0 * W[2] - 8.0 * W[3] + W[4]) / 40320.0;
}

/* P(xi) = W_0 + sum_{k=1}^{n} a_k Z_k(xi). */
static double poly_eval(double W0, const double *a, int n, double xi)
{
    double P = W0;
    for (int k = 1; k <= n; ++k) P += a[k - 1] * Zk(k, xi);
    return P;
}

/* dP/dxi = sum_{k=1}^{n} a_k dZ_k/dxi. */
static double poly_deriv(const double *a, int n, double xi)
{
    double D = 0.0;
    for (int k = 1; k <= n; ++k) D += a[k - 1] * dZk(k, xi);
    return D;
}

/* ------------------------------------------------------------------------ */
/* Discontinuity feedback (Sec. 3.1).                                         */
/* ------------------------------------------------------------------------ */

/* DF factor of a stencil, Eq. (discontinuity strength): alpha = 1 when the   */
/* summed strength A of the stencil's interfaces is below sigma_thres, else   */
/* sigma_thres / A.  (A = sigma_thres gives exactly 1.0 either way.)          */
static double df_alpha(double A, double thres)
{
    if (A < thres) return 1.0;
    return thres / A;
}

/* Summed strength of the faces interior to the stencil of cells [lo, hi]:   */
/* reading R8 -- the hi-lo faces separating consecutive stencil cells.       */
/* s[m] is the strength of the face between cells m and m+1.               */
static double stencil_sum(const double *s, int lo, int hi)
{
    double A = 0.0;
    for (int m = lo; m < hi; ++m) A += s[m];
    return A;
}

/* Local smoothness indicator of a 3-cell polynomial, Eq.                    */
/* (LocalSmoothnessIndicator):  beta = sum_q dx^{2q-1} int (d^q P/dx^q)^2 dx  */
/* over the cell.  In xi = x/dx on [-1,0] with P = W0 + a1 Z1 + a2 Z2:         */
/*   P' = a1 + 2 a2 xi,  P'' = 2 a2,                                          */
/*   int_{-1}^{0} (a1 + 2 a2 xi)^2 dxi = a1^2 - 2 a1 a2 + (4/3) a2^2,         */
/*   int_{-1}^{0} (2 a2)^2 dxi         = 4 a2^2.                              */
static double beta3(const double a[2])
{
    double first = a[0] * a[0] - 2.0 * a[0] * a[1] + (4.0 / 3.0) * a[1] * a[1];
    double second = 4.0 * a[1] * a[1];
    return first + second;
}

/* WENO-Z-AO(5,3) with DF (Sec. 3.2).  Wc points at W_0 (needs W_{-2..2});    */
/* alpha[0..2] are the DF factors of S^{r3}_{-1,0,1}, alpha[3] of S^{r5}.     */
/* dout (may be NULL) receives dP/dxi of the same combined polynomial.         */
static void weno_ao53_df(const orc_params *p, const double *Wc, const double alpha[4],
                         int npts, const double *xi, double *out, double *dout)
{
    double a3[3][2], a5[4], b3[3];
    for (int k = -1; k <= 1; ++k) {
        coef_r3(k, Wc, a3[k + 1]);
        b3[k + 1] = beta3(a3[k + 1]);           /* reading R10: raw polynomials */
    }
    coef_r5(Wc, a5);

    /* Simplified indicator for P^{r5} and the modified global indicator.     */
    double b5 = (b3[0] + 4.0 * b3[1] + b3[2]) / 6.0 + fabs(b3[0] - b3[2]);
    /* Reading R5: the printed tau_Z repeats |b5 - b3_1|; the mirror-symmetric */
    /* form over the three sub-stencils is taken.                              */
    double tauZ = (fabs(b5 - b3[0]) + fabs(b5 - b3[1]) + fabs(b5 - b3[2])) / 3.0;

    /* Linear weights d. */
    double d5 = p->d_hi;
    double d3[3];
    d3[0] = (1.0 - p->d_hi) * (1.0 - p->d_lo) / 2.0;
    d3[1] = (1.0 - p->d_hi) * p->d_lo;
    d3[2] = d3[0];

    /* WENO-Z weights omega_k = d_k (1 + tau_Z^2 / (beta_k + eps)^2). */
    double w5 = d5 * (1.0 + tauZ * tauZ / ((b5 + p->eps) * (b5 + p->eps)));
    double w3[3];
    for (int k = 0; k < 3; ++k) w3[k] = d3[k] * (1.0 + tauZ * tauZ / ((b3[k] + p->eps) * (b3[k] + p->eps)));
    double wsum = w5 + w3[0] + w3[1] + w3[2];
    double wb5 = w5 / wsum;
    double wb3[3];
    for (int k = 0; k < 3; ++k) wb3[k] = w3[k] / wsum;

    for (int q = 0; q < npts; ++q) {
        /* DF-damped candidate polynomials.  Reading R3: the printed P^{r5}    */
        /* lacks W_x4 in front of Z_4; it is W_x4 Z_4.                         */
        double P3[3];
        for (int k = 0; k < 3; ++k)
            P3[k] = Wc[0] + alpha[k] * (a3[k][0] * Zk(1, xi[q]) + a3[k][1] * Zk(2, xi[q]));
        double P5 = Wc[0] + alpha[3] * (a5[0] * Zk(1, xi[q]) + a5[1] * Zk(2, xi[q]) + a5[2] * Zk(3, xi[q])
                                       + a5[3] * Zk(4, xi[q]));
        double inner = P5 / d5;
        for (int k = 0; k < 3; ++k) inner -= d3[k] / d5 * P3[k];
        double P = wb5 * inner;
        for (int k = 0; k < 3; ++k) P += wb3[k] * P3[k];
        out[q] = P;
        if (dout) {
            /* the weights do not depend on xi: the same combination of slopes */
            double D3[3];
            for (int k = 0; k < 3; ++k) D3[k] = alpha[k] * (a3[k][0] * dZk(1, xi[q]) + a3[k][1] * dZk(2, xi[q]));
            double D5 = alpha[3] * poly_deriv(a5, 4, xi[q]);
            double dinner = D5 / d5;
            for (int k = 0; k < 3; ++k) dinner -= d3[k] / d5 * D3[k];
            double D = wb5 * dinner;
            for (int k = 0; k < 3; ++k) D += wb3[k] * D3[k];
            dout[q] = D;
        }
    }
}

/* Level codes reported for the reconstruction of a cell. */
enum { ORC_LVL_FIRST = 1, ORC_LVL_WENOAO = 2, ORC_LVL_R3 = 3, ORC_LVL_5 = 5, ORC_LVL_7 = 7, ORC_LVL_9 = 9 };

/* ASE-DF reconstruction polynomial of one cell, evaluated at npts points     */
/* xi in the cell [-1,0] (Sec. 3.2-3.4 and Algorithm 1).                      */
/*   Wc[m], m = -R..R  : cell averages around the cell (Wc points at W_0),    */
/*   sc[m], m = -R..R-1: strength of the face between cells m and m+1.        */
/* Reading R7: the text governs at the nominal order r -- the largest linear  */
/* stencil L <= r whose DF factor is 1 is used; alpha(S^{r5}) < 1 selects the */
/* WENO-Z-AO(5,3) with DF.  Reading R12: r = 3 is the centred S^{r3}_0       */
/* polynomial damped by its own DF factor.                                  */
/* dout (may be NULL) receives dP/dxi at the same points.                    */
static int ase_poly(const orc_params *p, int r, const double *Wc, const double *sc,
                    int npts, const double *xi, double *out, double *dout)
{
    double thr = p->sigma_thres;
    if (r == 1) {
        for (int q = 0; q < npts; ++q) out[q] = Wc[0];
        if (dout) for (int q = 0; q < npts; ++q) dout[q] = 0.0;
        return ORC_LVL_FIRST;
    }
    if (r == 3) {
        double a[2];
        coef_r3(0, Wc, a);
        double al = df_alpha(stencil_sum(sc, -1, 1), thr);
        for (int q = 0; q < npts; ++q) out[q] = Wc[0] + al * (a[0] * Zk(1, xi[q]) + a[1] * Zk(2, xi[q]));
        if (dout)
            for (int q = 0; q < npts; ++q) dout[q] = al * (a[0] * dZk(1, xi[q]) + a[1] * dZk(2, xi[q]));
        return ORC_LVL_R3;
    }
    /* Start from the 5-cell stencil and extend while the DF factor is 1. */
    double alpha5 = df_alpha(stencil_sum(sc, -2, 2), thr);
    int level;
    if (alpha5 < 1.0) {
        level = ORC_LVL_WENOAO;
    } else if (r == 5) {
        level = 5;
    } else {
        double alpha7 = df_alpha(stencil_sum(sc, -3, 3), thr);
        if (alpha7 < 1.0) {
            level = 5;
        } else if (r == 7) {
            level = 7;
        } else {
            double alpha9 = df_alpha(stencil_sum(sc, -4, 4), thr);
            level = (alpha9 < 1.0) ? 7 : 9;
        }
    }

    if (level == ORC_LVL_WENOAO) {
        double al[4];
        al[0] = df_alpha(stencil_sum(sc, -2, 0), thr);   /* S^{r3}_{-1}: cells -2..0 */
        al[1] = df_alpha(stencil_sum(sc, -1, 1), thr);   /* S^{r3}_{0} : cells -1..1 */
        al[2] = df_alpha(stencil_sum(sc, 0, 2), thr);    /* S^{r3}_{1} : cells  0..2 */
        al[3] = alpha5;                                  /* S^{r5}     : cells -2..2 */
        weno_ao53_df(p, Wc, al, npts, xi, out, dout);
        return level;
    }
    double a[8];
    int n;
    if (level == 5) { coef_r5(Wc, a); n = 4; }
    else if (level == 7) { coef_r7(Wc, a); n = 6; }
    else { coef_r9(Wc, a); n = 8; }
    for (int q = 0; q < npts; ++q) out[q] = poly_eval(Wc[0], a, n, xi[q]);
    if (dout) for (int q = 0; q < npts; ++q) dout[q] = poly_deriv(a, n, xi[q]);
    return level;
}

/* ------------------------------------------------------------------------ */
/* Euler equations (Sec. 2.3).                                                */
/* ------------------------------------------------------------------------ */

/* Primitive variables of a conservative state; dir 0 = x-normal, 1 = y.    */
/* Returns 0 when rho > 0 and p > 0, else -1.                                 */
typedef struct { double rho, un, ut, p, c; } prim_t;

static int primitives(const orc_grid *g, const orc_params *p, const double *W, int dir, prim_t *q)
{
    double rho = W[0];
    double u = W[1] / rho;
    double v = (g->dim == 2) ? W[2] / rho : 0.0;
    double E = W[nvar_of(g) - 1];
    double pr = (p->gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v));
    q->rho = rho;
    q->un = (dir == 0) ? u : v;
    q->ut = (dir == 0) ? v : u;
    q->p = pr;
    if (!(rho > 0.0) || !(pr > 0.0)) { q->c = NAN; return -1; }
    q->c = sqrt(p->gamma * pr / rho);
    return 0;
}

/* Physical flux F(W) (dir 0) or G(W) (dir 1). */
static void euler_flux(const orc_grid *g, const double *W, const prim_t *q, int dir, double *F)
{
    if (g->dim == 1) {
        F[0] = W[1];
        F[1] = W[1] * q->un + q->p;
        F[2] = q->un * (W[2] + q->p);
        return;
    }
    F[0] = (dir == 0) ? W[1] : W[2];     /* normal mass flux */
    if (dir == 0) {
        F[1] = W[1] * q->un + q->p;      /* rho u u + p */
        F[2] = W[2] * q->un;             /* rho v u     */
    } else {
        F[1] = W[1] * q->un;             /* rho u v     */
        F[2] = W[2] * q->un + q->p;      /* rho v v + p */
    }
    F[3] = q->un * (W[3] + q->p);
}

/* Discontinuity strength at one Gauss point (Sec. 3.1):                      */
/*   |pl-pr|/pl + |pl-pr|/pr + (Ma_n^l - Ma_n^r)^2 + (Ma_t^l - Ma_t^r)^2.     */
/* Reading R15: a non-physical side (rho <= 0 or p <= 0) gives +inf, which    */
/* drives every DF factor touching the face to 0.                             */
static double sigma_point(const prim_t *l, int okl, const prim_t *r, int okr)
{
    if (okl != 0 || okr != 0) return INFINITY;
    double dp = fabs(l->p - r->p);
    double dman = l->un / l->c - r->un / r->c;
    double dmat = l->ut / l->c - r->ut / r->c;
    return dp / l->p + dp / r->p + dman * dman + dmat * dmat;
}

/* Lax-Friedrichs flux with the local maximal signal speed (Sec. 2.3). */
static void lf_flux(const orc_grid *g, const double *Wl, const prim_t *ql, const double *Wr,
                    const prim_t *qr, int dir, double *F)
{
    int nv = nvar_of(g);
    double Fl[4], Fr[4];
    euler_flux(g, Wl, ql, dir, Fl);
    euler_flux(g, Wr, qr, dir, Fr);
    double sl = fabs(ql->un) + ql->c;
    double sr = fabs(qr->un) + qr->c;
    double smax = sl > sr ? sl : sr;
    for (int v = 0; v < nv; ++v) F[v] = 0.5 * (Fl[v] + Fr[v]) - 0.5 * smax * (Wr[v] - Wl[v]);
}

/* One Gauss point: sigma_m and the LF flux.  With positivity_fallback, a     */
/* non-physical state is replaced by the average of its own cell (R15).       */
static double gauss_point_flux(const orc_grid *g, const orc_params *p, const double *Wl_in,
                               const double *Wr_in, const double *Wl_cell, const double *Wr_cell,
                               int dir, double *F)
{
    prim_t ql, qr;
    int okl = primitives(g, p, Wl_in, dir, &ql);
    int okr = primitives(g, p, Wr_in, dir, &qr);
    double sig = sigma_point(&ql, okl, &qr, okr);
    const double *Wl = Wl_in, *Wr = Wr_in;
    if (p->positivity_fallback) {
        if (okl != 0) { Wl = Wl_cell; primitives(g, p, Wl, dir, &ql); }
        if (okr != 0) { Wr = Wr_cell; primitives(g, p, Wr, dir, &qr); }
    }
    lf_flux(g, Wl, &ql, Wr, &qr, dir, F);
    return sig;
}

/* ------------------------------------------------------------------------ */
/* Boundary conditions (reading R16).                                         */
/* ------------------------------------------------------------------------ */

static int in_slot(const orc_grid *g, int J)
{
    if (g->dim == 1) return 1;
    double y = g->y0 + ((double)(J - g->ng) + 0.5) * g->dy;
    return y > g->slot_lo && y < g->slot_hi;
}

/* Ghost cells: x first on interior rows, then y on every column. */
static void bc_fill_cells(const orc_grid *g, double *U, double t)
{
    int nv = nvar_of(g), ng = g->ng, NX = NXof(g), NY = NYof(g);
    size_t P = plane(g);
    int j0 = (g->dim == 1) ? 0 : ng, j1 = (g->dim == 1) ? 1 : ng + g->ny;
    for (int J = j0; J < j1; ++J) {
        double *row = U + (size_t)J * g->ld;
        for (int k = 0; k < ng; ++k) {
            int Il = ng - 1 - k, Ir = ng + g->nx + k;
            for (int v = 0; v < nv; ++v) {
                double *rv = row + v * P;
                /* a reflective (slip) wall mirrors the cells and reverses the
                   momentum normal to it (x momentum is variable 1); a no-slip
                   wall reverses both momenta */
                int mom = v == 1 || (g->dim == 2 && v == 2);
                double flo = (v == 1 || (g->bc[0] == ORC_BC_NOSLIP && mom)) ? -1.0 : 1.0;
                double fhi = (v == 1 || (g->bc[1] == ORC_BC_NOSLIP && mom)) ? -1.0 : 1.0;
                /* low side */
                if (g->bc[0] == ORC_BC_PERIODIC) rv[Il] = rv[Il + g->nx];
                else if (g->bc[0] == ORC_BC_INFLOW_SLOT && in_slot(g, J)) rv[Il] = g->inflow[v];
                else if (is_wall(g->bc[0])) rv[Il] = flo * rv[ng + k];
                else rv[Il] = rv[ng];
                /* high side */
                if (g->bc[1] == ORC_BC_PERIODIC) rv[Ir] = rv[Ir - g->nx];
                else if (g->bc[1] == ORC_BC_INFLOW_SLOT && in_slot(g, J)) rv[Ir] = g->inflow[v];
                else if (is_wall(g->bc[1])) rv[Ir] = fhi * rv[ng + g->nx - 1 - k];
                else rv[Ir] = rv[ng + g->nx - 1];
            }
        }
    }
    if (g->dim == 1) return;
    for (int k = 0; k < ng; ++k) {
        int Jl = ng - 1 - k, Jh = ng + g->ny + k;
        for (int v = 0; v < nv; ++v) {
            double *Uv = U + v * P;
            double flip = (v == 2) ? -1.0 : 1.0;   /* y momentum */
            double flo = (v == 2 || (g->bc[2] == ORC_BC_NOSLIP && v == 1)) ? -1.0 : 1.0;
            double fhi = (v == 2 || (g->bc[3] == ORC_BC_NOSLIP && v == 1)) ? -1.0 : 1.0;
            for (int I = 0; I < NX; ++I) {
                /* centre of the column (double Mach reflection sides) */
                double xc = g->x0 + ((double)(I - ng) + 0.5) * g->dx;
                if (g->bc[2] == ORC_BC_PERIODIC) Uv[(size_t)Jl * g->ld + I] = Uv[(size_t)(Jl + g->ny) * g->ld + I];
                else if (is_wall(g->bc[2]) || (g->bc[2] == ORC_BC_WALL_INFLOW && !(xc < g->wall_x0)))
                    Uv[(size_t)Jl * g->ld + I] = (g->bc[2] == ORC_BC_NOSLIP ? flo : flip) * Uv[(size_t)(ng + k) * g->ld + I];
                else if (g->bc[2] == ORC_BC_WALL_INFLOW) Uv[(size_t)Jl * g->ld + I] = g->inflow[v];
                else Uv[(size_t)Jl * g->ld + I] = Uv[(size_t)ng * g->ld + I];
                if (g->bc[3] == ORC_BC_PERIODIC) Uv[(size_t)Jh * g->ld + I] = Uv[(size_t)(Jh - g->ny) * g->ld + I];
                else if (is_wall(g->bc[3]))
                    Uv[(size_t)Jh * g->ld + I] = fhi * Uv[(size_t)(ng + g->ny - 1 - k) * g->ld + I];
                else if (g->bc[3] == ORC_BC_MOVING_SHOCK)
                    Uv[(size_t)Jh * g->ld + I] = (xc < g->shock_x0 + g->shock_speed * t) ? g->inflow[v] : g->outer[v];
                else Uv[(size_t)Jh * g->ld + I] = Uv[(size_t)(ng + g->ny - 1) * g->ld + I];
            }
        }
    }
    (void)NY;
}

static void cell_state(const orc_grid *g, const double *U, int I, int J, double *W)
{
    size_t P = plane(g);
    for (int v = 0; v < nvar_of(g); ++v) W[v] = U[v * P + (size_t)J * g->ld + I];
}

/* First-order strength of a face: the Gauss-point formula applied to the     */
/* two adjacent cell averages (one point; the states are constant on it).     */
static double sigma_first_order(const orc_grid *g, const orc_params *p, const double *U,
                                int I0, int J0, int I1, int J1, int dir)
{
    double Wa[4], Wb[4];
    prim_t qa, qb;
    cell_state(g, U, I0, J0, Wa);
    cell_state(g, U, I1, J1, Wb);
    int oka = primitives(g, p, Wa, dir, &qa);
    int okb = primitives(g, p, Wb, dir, &qb);
    return sigma_point(&qa, oka, &qb, okb);
}

/* First-order strength on every stored face (ghost cells already filled). */
static void sigma_all_first_order(const orc_grid *g, const orc_params *p, const double *U, double *sx, double *sy)
{
    int NX = NXof(g), NY = NYof(g);
#pragma omp parallel for schedule(static) if ((long)NY * NX > 4096)
    for (int J = 0; J < NY; ++J)
        for (int I = 0; I + 1 < NX; ++I)
            sx[(size_t)J * g->ld + I] = sigma_first_order(g, p, U, I, J, I + 1, J, 0);
    if (g->dim == 2)
#pragma omp parallel for schedule(static) if ((long)NY * NX > 4096)
        for (int J = 0; J < NY - 1; ++J)
            for (int I = 0; I < NX; ++I)
                sy[(size_t)J * g->ld + I] = sigma_first_order(g, p, U, I, J, I, J + 1, 1);
}

/* Boundary step of a stage: ghost cells, then the strengths the stage's    */
/* DF factors read -- derived non-flux faces (lagged source) or first-order */
/* strengths of the stage input on every face (first-order source).        */
static void stage_bc(const orc_grid *g, const orc_params *p, double *U, double *sx, double *sy, double t);

static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Strength on faces the previous stage did not produce.  Flux faces are     */
/* x-faces i+1/2, i in [-1, nx-1], on interior rows (y-faces likewise).  A     */
/* face that periodic wrapping or reflective mirroring maps onto a flux face  */
/* takes that face's value (a wall is a symmetry plane of the lagged DF       */
/* state too); any other face takes the first-order strength of its two       */
/* ghost-filled cells.                                                        */

/* Cell index mapped by the boundary rule of one axis (periodic wrap or wall   */
/* mirror); other codes leave it.                                             */
static int map_cell(int i, int n, int bc_lo, int bc_hi)
{
    if (i < 0) {
        if (bc_lo == ORC_BC_PERIODIC) return wrap(i, n);
        if (is_wall(bc_lo)) return -1 - i;
    } else if (i >= n) {
        if (bc_hi == ORC_BC_PERIODIC) return wrap(i, n);
        if (is_wall(bc_hi)) return 2 * n - 1 - i;
    }
    return i;
}

/* Face index f (face f + 1/2) mapped likewise: a wall at -1/2 maps f to      */
/* -f-2, a wall at n-1/2 maps f to 2n-f-2.                                    */
static int map_face(int f, int n, int bc_lo, int bc_hi)
{
    if (f < -1) {
        if (bc_lo == ORC_BC_PERIODIC) return wrap(f, n);
        if (is_wall(bc_lo)) return -f - 2;
    } else if (f > n - 1) {
        if (bc_hi == ORC_BC_PERIODIC) return wrap(f, n);
        if (is_wall(bc_hi)) return 2 * n - f - 2;
    }
    return f;
}

static void bc_fill_sigma(const orc_grid *g, const orc_params *p, const double *U, double *sx, double *sy)
{
    int ng = g->ng, NX = NXof(g), NY = NYof(g);
    for (int J = 0; J < NY; ++J) {
        int j = J - ng;
        int jrow_ok = (g->dim == 1) || (j >= 0 && j < g->ny);
        for (int I = 0; I + 1 < NX; ++I) {
            int f = I - ng;                     /* face f + 1/2 */
            if (jrow_ok && f >= -1 && f <= g->nx - 1) continue;   /* produced */
            int fw = map_face(f, g->nx, g->bc[0], g->bc[1]);
            int jw = (g->dim == 2) ? map_cell(j, g->ny, g->bc[2], g->bc[3]) : j;
            int jw_ok = (g->dim == 1) || (jw >= 0 && jw < g->ny);
            if (jw_ok && fw >= -1 && fw <= g->nx - 1) {
                int Jw = (g->dim == 1) ? 0 : jw + ng;
                sx[(size_t)J * g->ld + I] = sx[(size_t)Jw * g->ld + fw + ng];
            } else {
                sx[(size_t)J * g->ld + I] = sigma_first_order(g, p, U, I, J, I + 1, J, 0);
            }
        }
    }
    if (g->dim == 1) return;
    for (int J = 0; J + 1 < NY; ++J) {
        int f = J - ng;
        for (int I = 0; I < NX; ++I) {
            int i = I - ng;
            if (i >= 0 && i < g->nx && f >= -1 && f <= g->ny - 1) continue;
            int fw = map_face(f, g->ny, g->bc[2], g->bc[3]);
            int iw = map_cell(i, g->nx, g->bc[0], g->bc[1]);
            if (iw >= 0 && iw < g->nx && fw >= -1 && fw <= g->ny - 1) {
                sy[(size_t)J * g->ld + I] = sy[(size_t)(fw + ng) * g->ld + iw + ng];
            } else {
                sy[(size_t)J * g->ld + I] = sigma_first_order(g, p, U, I, J, I, J + 1, 1);
            }
        }
    }
}

/* Ghost cells at time t (the time of the stage input; only the moving    */
/* shock side depends on it), then the strengths a stage reads.            */
static void stage_bc(const orc_grid *g, const orc_params *p, double *U, double *sx, double *sy, double t)
{
    bc_fill_cells(g, U, t);
    if (p->df_source == ORC_DF_FIRST_ORDER) sigma_all_first_order(g, p, U, sx, sy);
    else bc_fill_sigma(g, p, U, sx, sy);
}

/* ------------------------------------------------------------------------ */
/* Spatial operator L(W) of the semi-discrete form (Sec. 2.1).               */
/* ------------------------------------------------------------------------ */

/* Reconstruct along one direction and build the interface fluxes.          */
/* For dir = 0 (x-faces):                                                    */
/*  1. normal reconstruction: every cell I in [ng-1, ng+nx] of every row     */
/*     J the tangential stencils reach gives its face-averaged values at     */
/*     its right face (xi = 0) and left face (xi = -1); DF from sx of row J. */
/*  2. tangential reconstruction (2D, Remark 2): the face values of rows     */
/*     J-R..J+R are treated as averages along y and reconstructed with the   */
/*     y-face strengths of the side cell's own column (reading R14), then    */
/*     evaluated at the Gauss points.                                       */
/*  3. per Gauss point: strength sigma_m and the LF flux; the face flux is   */
/*     sum eta_k F_k and the face strength is the mean of sigma_m (R6).      */
/* Outputs per flux face (compact numbering, see face_index): wl, wr         */
/* [v][k][face] (optional), flux [v][face] (optional) and the strength       */
/* written into sig_out at the face's place in the strength layout.          */
static int face_count(const orc_grid *g, int dir)
{
    if (g->dim == 1) return g->nx + 1;
    return dir == 0 ? (g->nx + 1) * g->ny : g->nx * (g->ny + 1);
}
/* x-face i+1/2 of row j -> j*(nx+1) + (i+1); y-face j+1/2 of column i ->    */
/* (j+1)*nx + i.                                                             */
static size_t face_index(const orc_grid *g, int dir, int i, int j)
{
    if (g->dim == 1) return (size_t)(i + 1);
    if (dir == 0) return (size_t)j * (g->nx + 1) + (i + 1);
    return (size_t)(j + 1) * g->nx + i;
}

static int sweep(const orc_grid *g, const orc_params *p, int dir, const double *U,
                 const double *sx, const double *sy, double *wl, double *wr, double *flux,
                 double *sig_out, int8_t *level)
{
    int r = p->order, R = halfwidth(r), ng = g->ng, nv = nvar_of(g);
    int G = ngauss(g, r);
    size_t P = plane(g);
    int ld = g->ld;
    double node[4], eta[4], xi_g[4];
    gauss_legendre(G, node, eta);
    for (int k = 0; k < G; ++k) xi_g[k] = -0.5 + node[k];
    const double xi_n[2] = {0.0, -1.0};

    /* Extent along the sweep (n_along) and across it (n_across). */
    int n_along = dir == 0 ? g->nx : g->ny;
    int n_across = g->dim == 1 ? 1 : (dir == 0 ? g->ny : g->nx);
    int Rt = g->dim == 1 ? 0 : R;                 /* tangential half width */
    int nrow = n_across + 2 * Rt;                 /* lines reconstructed    */
    int ncell = n_along + 2;                      /* cells -1 .. n_along    */
    size_t tsz = (size_t)nv * nrow * ncell;
    double *tR = malloc(tsz * sizeof(double));    /* value at xi = 0  */
    double *tL = malloc(tsz * sizeof(double));    /* value at xi = -1 */
    if (!tR || !tL) { free(tR); free(tL); return -1; }

    /* Address of cell (a along, c across) in interior indexing. */
#define CELL(a, c) ((dir == 0) ? ((size_t)((g->dim == 1 ? 0 : (c) + ng)) * ld + (size_t)((a) + ng)) \
                               : ((size_t)((a) + ng) * ld + (size_t)((c) + ng)))
    const double *snorm = dir == 0 ? sx : sy;     /* faces along the sweep  */
    const double *stang = dir == 0 ? sy : sx;     /* faces across the sweep */
    /* Stride between neighbouring cells along / across the sweep. */
    ptrdiff_t s_along = dir == 0 ? 1 : ld;
    ptrdiff_t s_across = dir == 0 ? ld : 1;

    /* 1. normal reconstruction */
#pragma omp parallel for schedule(static) if ((long)n_across * n_along > 4096)
    for (int c = -Rt; c < n_across + Rt; ++c) {
        for (int a = -1; a <= n_along; ++a) {
            size_t base = CELL(a, c);
            double Wline[9], sline[8], out[2];
            for (int v = 0; v < nv; ++v) {
                for (int m = -R; m <= R; ++m) Wline[m + R] = U[v * P + base + m * s_along];
                for (int m = -R; m < R; ++m) sline[m + R] = snorm[base + m * s_along];
                int lv = ase_poly(p, r, Wline + R, sline + R, 2, xi_n, out, NULL);
                size_t t = ((size_t)v * nrow + (c + Rt)) * ncell + (a + 1);
                tR[t] = out[0];
                tL[t] = out[1];
                if (level && v == 0 && c >= 0 && c < n_across && a >= 0 && a < n_along)
                    level[(size_t)(dir == 0 ? c : a) * g->nx + (dir == 0 ? a : c)] = (int8_t)lv;
            }
        }
    }

    /* 2.-3. tangential reconstruction and fluxes */
#pragma omp parallel for schedule(static) if ((long)n_across * n_along > 4096)
    for (int c = 0; c < n_across; ++c) {
        for (int a = -1; a < n_along; ++a) {          /* face a + 1/2 */
            double WL[4][4], WR[4][4];                  /* [gauss][var] */
            for (int v = 0; v < nv; ++v) {
                double outl[4], outr[4];
                if (g->dim == 1) {
                    outl[0] = tR[((size_t)v * nrow) * ncell + (a + 1)];
                    outr[0] = tL[((size_t)v * nrow) * ncell + (a + 2)];
                } else {
                    double Wl_line[9], Wr_line[9], sl_line[8], sr_line[8];
                    size_t bl = CELL(a, c), br = CELL(a + 1, c);
                    for (int m = -R; m <= R; ++m) {
                        Wl_line[m + R] = tR[((size_t)v * nrow + (c + m + Rt)) * ncell + (a + 1)];
                        Wr_line[m + R] = tL[((size_t)v * nrow + (c + m + Rt)) * ncell + (a + 2)];
                    }
                    for (int m = -R; m < R; ++m) {
                        sl_line[m + R] = stang[bl + m * s_across];
                        sr_line[m + R] = stang[br + m * s_across];
                    }
                    ase_poly(p, r, Wl_line + R, sl_line + R, G, xi_g, outl, NULL);
                    ase_poly(p, r, Wr_line + R, sr_line + R, G, xi_g, outr, NULL);
                }
                for (int k = 0; k < G; ++k) { WL[k][v] = outl[k]; WR[k][v] = outr[k]; }
            }
            double Wlc[4], Wrc[4];
            {
                size_t bl = CELL(a, c), br = CELL(a + 1, c);
                for (int v = 0; v < nv; ++v) { Wlc[v] = U[v * P + bl]; Wrc[v] = U[v * P + br]; }
            }
            double Fsum[4] = {0, 0, 0, 0}, ssum = 0.0;
            int fi = dir == 0 ? a : c, fj = dir == 0 ? c : a;
            size_t fid = face_index(g, dir, fi, fj);
            size_t nf = (size_t)face_count(g, dir);
            for (int k = 0; k < G; ++k) {
                double Fk[4];
                double sk = gauss_point_flux(g, p, WL[k], WR[k], Wlc, Wrc, dir, Fk);
                ssum += sk;
                for (int v = 0; v < nv; ++v) Fsum[v] += eta[k] * Fk[v];
                if (wl) for (int v = 0; v < nv; ++v) wl[((size_t)v * G + k) * nf + fid] = WL[k][v];
                if (wr) for (int v = 0; v < nv; ++v) wr[((size_t)v * G + k) * nf + fid] = WR[k][v];
            }
            if (flux) for (int v = 0; v < nv; ++v) flux[(size_t)v * nf + fid] = Fsum[v];
            if (sig_out) sig_out[CELL(a, c)] = ssum / (double)G;
        }
    }
#undef CELL
    free(tR);
    free(tL);
    return 0;
}

/* L(W) on interior cells:                                                   */
/*   L = -(F_{i+1/2} - F_{i-1/2})/dx - (G_{j+1/2} - G_{j-1/2})/dy.           */
static int residual(const orc_grid *g, const orc_params *p, const double *U, const double *sx,
                    const double *sy, double *L, double *sx_new, double *sy_new)
{
    int nv = nvar_of(g), ng = g->ng;
    size_t P = plane(g);
    size_t nfx = (size_t)face_count(g, 0);
    double *Fx = malloc((size_t)nv * nfx * sizeof(double));
    if (!Fx) return -1;
    if (sweep(g, p, 0, U, sx, sy, NULL, NULL, Fx, sx_new, NULL)) { free(Fx); return -1; }
    double *Fy = NULL;
    size_t nfy = 0;
    if (g->dim == 2) {
        nfy = (size_t)face_count(g, 1);
        Fy = malloc((size_t)nv * nfy * sizeof(double));
        if (!Fy) { free(Fx); return -1; }
        if (sweep(g, p, 1, U, sx, sy, NULL, NULL, Fy, sy_new, NULL)) { free(Fx); free(Fy); return -1; }
    }
    int nyl = g->dim == 1 ? 1 : g->ny;
#pragma omp parallel for schedule(static) if ((long)nyl * g->nx > 4096)
    for (int j = 0; j < nyl; ++j) {
        for (int i = 0; i < g->nx; ++i) {
            size_t c = (size_t)(g->dim == 1 ? 0 : j + ng) * g->ld + (size_t)(i + ng);
            for (int v = 0; v < nv; ++v) {
                double dFx = Fx[v * nfx + face_index(g, 0, i, j)] - Fx[v * nfx + face_index(g, 0, i - 1, j)];
                double val = -dFx / g->dx;
                if (g->dim == 2) {
                    double dFy = Fy[v * nfy + face_index(g, 1, i, j)] - Fy[v * nfy + face_index(g, 1, i, j - 1)];
                    val = val - dFy / g->dy;
                }
                L[v * P + c] = val;
            }
        }
    }
    free(Fx);
    free(Fy);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Time step (reading R9): dt = CFL / max over interior cells (and the       */
/* inflow state, when a boundary has one) of (|u|+c)/dx [+ (|v|+c)/dy],      */
/* optionally capped, then clipped to t_end.                                 */
/* ------------------------------------------------------------------------ */
static double cfl_dt(const orc_grid *g, const orc_params *p, const double *U, double t, double t_end)
{
    int ng = g->ng;
    int nyl = g->dim == 1 ? 1 : g->ny;
    double lam = 0.0;
    for (int j = 0; j < nyl; ++j) {
        for (int i = 0; i < g->nx; ++i) {
            double W[4];
            prim_t qx, qy;
            cell_state(g, U, i + ng, g->dim == 1 ? 0 : j + ng, W);
            primitives(g, p, W, 0, &qx);
            double l = (fabs(qx.un) + qx.c) / g->dx;
            if (g->dim == 2) {
                primitives(g, p, W, 1, &qy);
                l = l + (fabs(qy.un) + qy.c) / g->dy;
            }
            if (l > lam || l != l) lam = l;
        }
    }
    /* Inflow ghost states enter the domain: their signal speed counts too. */
    if (g->bc[0] == ORC_BC_INFLOW_SLOT || g->bc[1] == ORC_BC_INFLOW_SLOT) {
        prim_t qx, qy;
        primitives(g, p, g->inflow, 0, &qx);
        double l = (fabs(qx.un) + qx.c) / g->dx;
        if (g->dim == 2) {
            primitives(g, p, g->inflow, 1, &qy);
            l = l + (fabs(qy.un) + qy.c) / g->dy;
        }
        if (l > lam || l != l) lam = l;
    }
    double dt = p->cfl / lam;
    if (p->dt_cap > 0.0 && dt > p->dt_cap) dt = p->dt_cap;
    if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
    return dt;
}

/* ------------------------------------------------------------------------ */
/* SSP-RK3 step (Eq. SSP-RK3) with lagged discontinuity feedback (reading    */
/* R9 of the DF source): the strength a stage computes at its Gauss points   */
/* feeds the next stage's DF factors, so (U, sx, sy) is the state.           */
/* ------------------------------------------------------------------------ */

/* Stage combination on interior cells.                                     */
/*   s=1: U1 = Un + dt L(Un)                                                 */
/*   s=2: U2 = 3/4 Un + 1/4 U1 + 1/4 dt L(U1)                                */
/*   s=3: Un+1 = 1/3 Un + 2/3 U2 + 2/3 dt L(U2)                              */
static void stage_combine(const orc_grid *g, int stage, double dt, const double *Un, const double *Us,
                          const double *L, double *Uo)
{
    int nv = nvar_of(g), ng = g->ng;
    size_t P = plane(g);
    int nyl = g->dim == 1 ? 1 : g->ny;
#pragma omp parallel for collapse(2) schedule(static) if ((long)nyl * g->nx > 4096)
    for (int v = 0; v < nv; ++v)
        for (int j = 0; j < nyl; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = v * P + (size_t)(g->dim == 1 ? 0 : j + ng) * g->ld + (size_t)(i + ng);
                if (stage == 1) Uo[c] = Un[c] + dt * L[c];
                else if (stage == 2) Uo[c] = 0.75 * Un[c] + 0.25 * Us[c] + 0.25 * dt * L[c];
                else Uo[c] = (1.0 / 3.0) * Un[c] + (2.0 / 3.0) * Us[c] + (2.0 / 3.0) * dt * L[c];
            }
}

static int check_args(const orc_grid *g, const orc_params *p)
{
    int r = p->order;
    if (r != 1 && r != 3 && r != 5 && r != 7 && r != 9) return -2;
    if (g->dim != 1 && g->dim != 2) return -1;
    if (g->ng < halfwidth(r) + 1) return -3;
    if (g->nx < 1 || (g->dim == 2 && g->ny < 1)) return -1;
    if (g->ld < NXof(g)) return -1;
    if (g->dim == 1 && g->ny != 1) return -1;
    if (g->bc[0] == ORC_BC_PERIODIC && g->bc[1] != ORC_BC_PERIODIC) return -1;
    if (g->bc[1] == ORC_BC_PERIODIC && g->bc[0] != ORC_BC_PERIODIC) return -1;
    if (g->dim == 2 && (g->bc[2] == ORC_BC_PERIODIC) != (g->bc[3] == ORC_BC_PERIODIC)) return -1;
    if (g->dim == 2 && (g->bc[2] == ORC_BC_INFLOW_SLOT || g->bc[3] == ORC_BC_INFLOW_SLOT)) return -1;
    for (int k = 0; k < (g->dim == 2 ? 4 : 2); ++k)
        if (g->bc[k] < ORC_BC_PERIODIC || g->bc[k] > ORC_BC_NOSLIP) return -1;
    /* the double Mach reflection sides: wall/inflow on y-lo, moving shock on y-hi */
    for (int k = 0; k < 4; ++k) {
        if (g->bc[k] == ORC_BC_WALL_INFLOW && !(k == 2 && g->dim == 2)) return -1;
        if (g->bc[k] == ORC_BC_MOVING_SHOCK && !(k == 3 && g->dim == 2)) return -1;
    }
    if (g->dim == 2 && g->bc[2] == ORC_BC_WALL_INFLOW && g->ny < g->ng) return -1;
    /* a mirror or a wrap reads ng interior cells */
    if ((is_wall(g->bc[0]) || is_wall(g->bc[1])) && g->nx < g->ng) return -1;
    if (g->dim == 2 && (is_wall(g->bc[2]) || is_wall(g->bc[3])) && g->ny < g->ng) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (ctypes).                                           */
/* ------------------------------------------------------------------------ */

/* Ghost cells of U, then the strengths a stage reads: all non-flux faces   */
/* (lagged source) or every face at first order (first-order source).      */
int orc_bc_fill(const orc_grid *g, const orc_params *p, double *U, double *sx, double *sy)
{
    int e = check_args(g, p);
    if (e) return e;
    stage_bc(g, p, U, sx, sy, 0.0);
    return 0;
}

/* As orc_bc_fill with the ghost cells at time t (the moving-shock side).   */
int orc_bc_fill_at(const orc_grid *g, const orc_params *p, double t, double *U, double *sx, double *sy)
{
    int e = check_args(g, p);
    if (e) return e;
    stage_bc(g, p, U, sx, sy, t);
    return 0;
}

/* Initial strengths: first-order states on every stored face (after the    */
/* ghost cells of U are filled).                                             */
int orc_sigma_init(const orc_grid *g, const orc_params *p, double *U, double *sx, double *sy)
{
    int e = check_args(g, p);
    if (e) return e;
    bc_fill_cells(g, U, 0.0);
    sigma_all_first_order(g, p, U, sx, sy);
    return 0;
}

/* Reconstruction of one direction: Gauss-point states of every flux face.  */
/* U and the strengths must already carry their ghosts (orc_bc_fill).        */
int orc_reconstruct(const orc_grid *g, const orc_params *p, int dir, const double *U, const double *sx,
                    const double *sy, double *wl, double *wr, int8_t *level)
{
    int e = check_args(g, p);
    if (e) return e;
    if (dir != 0 && !(dir == 1 && g->dim == 2)) return -1;
    return sweep(g, p, dir, U, sx, sy, wl, wr, NULL, NULL, level);
}

/* Face strengths from Gauss-point states ([v][k][face] layout), written     */
/* into the strength layout at the flux faces.                               */
int orc_df_compute(const orc_grid *g, const orc_params *p, int dir, const double *wl, const double *wr,
                   double *sig)
{
    int e = check_args(g, p);
    if (e) return e;
    int nv = nvar_of(g), G = ngauss(g, p->order), ng = g->ng;
    size_t nf = (size_t)face_count(g, dir);
    int n_along = dir == 0 ? g->nx : g->ny;
    int n_across = g->dim == 1 ? 1 : (dir == 0 ? g->ny : g->nx);
    for (int c = 0; c < n_across; ++c)
        for (int a = -1; a < n_along; ++a) {
            int fi = dir == 0 ? a : c, fj = dir == 0 ? c : a;
            size_t fid = face_index(g, dir, fi, fj);
            double ssum = 0.0;
            for (int k = 0; k < G; ++k) {
                double Wl[4], Wr[4];
                prim_t ql, qr;
                for (int v = 0; v < nv; ++v) {
                    Wl[v] = wl[((size_t)v * G + k) * nf + fid];
                    Wr[v] = wr[((size_t)v * G + k) * nf + fid];
                }
                int okl = primitives(g, p, Wl, dir, &ql);
                int okr = primitives(g, p, Wr, dir, &qr);
                ssum += sigma_point(&ql, okl, &qr, okr);
            }
            size_t pos = dir == 0 ? (size_t)(g->dim == 1 ? 0 : c + ng) * g->ld + (size_t)(a + ng)
                                  : (size_t)(a + ng) * g->ld + (size_t)(c + ng);
            sig[pos] = ssum / (double)G;
        }
    return 0;
}

/* Interface fluxes (sum over Gauss points of eta_k F_LF) from Gauss-point   */
/* states.  No positivity replacement here (it needs the cell averages).     */
int orc_flux(const orc_grid *g, const orc_params *p, int dir, const double *wl, const double *wr, double *F)
{
    int e = check_args(g, p);
    if (e) return e;
    int nv = nvar_of(g), G = ngauss(g, p->order);
    size_t nf = (size_t)face_count(g, dir);
    double node[4], eta[4];
    gauss_legendre(G, node, eta);
    for (size_t f = 0; f < nf; ++f) {
        double Fs[4] = {0, 0, 0, 0};
        for (int k = 0; k < G; ++k) {
            double Wl[4], Wr[4], Fk[4];
            prim_t ql, qr;
            for (int v = 0; v < nv; ++v) {
                Wl[v] = wl[((size_t)v * G + k) * nf + f];
                Wr[v] = wr[((size_t)v * G + k) * nf + f];
            }
            primitives(g, p, Wl, dir, &ql);
            primitives(g, p, Wr, dir, &qr);
            lf_flux(g, Wl, &ql, Wr, &qr, dir, Fk);
            for (int v = 0; v < nv; ++v) Fs[v] += eta[k] * Fk[v];
        }
        for (int v = 0; v < nv; ++v) F[(size_t)v * nf + f] = Fs[v];
    }
    return 0;
}

/* Conservative update of one SSP-RK3 stage from face fluxes F (x) and G (y, */
/* 2D only), compact face numbering.                                         */
int orc_stage_update(const orc_grid *g, const orc_params *p, int stage, double dt, const double *Un,
                     const double *Us, const double *F, const double *Gf, double *Uo)
{
    int e = check_args(g, p);
    if (e) return e;
    if (stage < 1 || stage > 3) return -1;
    int nv = nvar_of(g), ng = g->ng;
    size_t P = plane(g);
    size_t nfx = (size_t)face_count(g, 0), nfy = g->dim == 2 ? (size_t)face_count(g, 1) : 0;
    double *L = calloc((size_t)nv * P, sizeof(double));
    if (!L) return -1;
    int nyl = g->dim == 1 ? 1 : g->ny;
    for (int j = 0; j < nyl; ++j)
        for (int i = 0; i < g->nx; ++i) {
            size_t c = (size_t)(g->dim == 1 ? 0 : j + ng) * g->ld + (size_t)(i + ng);
            for (int v = 0; v < nv; ++v) {
                double val = -(F[v * nfx + face_index(g, 0, i, j)] - F[v * nfx + face_index(g, 0, i - 1, j)]) / g->dx;
                if (g->dim == 2)
                    val = val - (Gf[v * nfy + face_index(g, 1, i, j)] - Gf[v * nfy + face_index(g, 1, i, j - 1)]) / g->dy;
                L[v * P + c] = val;
            }
        }
    stage_combine(g, stage, dt, Un, Us, L, Uo);
    free(L);
    return 0;
}

/* Semi-discrete operator L(W) on interior cells (ghosts filled inside);     */
/* sx_new / sy_new receive the strengths at the flux faces (may be NULL).    */
int orc_residual(const orc_grid *g, const orc_params *p, double *U, double *sx, double *sy, double *L,
                 double *sx_new, double *sy_new)
{
    int e = check_args(g, p);
    if (e) return e;
    stage_bc(g, p, U, sx, sy, 0.0);
    size_t n = plane(g);
    double *tx = sx_new ? sx_new : malloc(n * sizeof(double));
    double *ty = (g->dim == 2) ? (sy_new ? sy_new : malloc(n * sizeof(double))) : NULL;
    int rc = residual(g, p, U, sx, sy, L, tx, ty);
    if (!sx_new) free(tx);
    if (g->dim == 2 && !sy_new) free(ty);
    return rc;
}

int orc_cfl_dt(const orc_grid *g, const orc_params *p, const double *U, double t, double t_end, double *dt)
{
    int e = check_args(g, p);
    if (e) return e;
    *dt = cfl_dt(g, p, U, t, t_end);
    return 0;
}

/* nsteps SSP-RK3 steps (fewer when t reaches t_end > 0).  U, sx, sy hold the */
/* state on entry and exit; *t is advanced; dt_hist[s] receives each step's  */
/* dt (may be NULL).  Returns the number of steps taken, or < 0 on error.    */
int orc_step(const orc_grid *g, const orc_params *p, double *U, double *sx, double *sy, double *t,
             int nsteps, double t_end, double *dt_hist)
{
    int e = check_args(g, p);
    if (e) return e;
    int nv = nvar_of(g);
    size_t P = plane(g);
    size_t n = (size_t)nv * P;
    double *U1 = malloc(n * sizeof(double)), *U2 = malloc(n * sizeof(double));
    double *L = malloc(n * sizeof(double));
    double *sxa = malloc(P * sizeof(double)), *sya = malloc(P * sizeof(double));
    if (!U1 || !U2 || !L || !sxa || !sya) { free(U1); free(U2); free(L); free(sxa); free(sya); return -1; }
    int taken = 0;
    for (int s = 0; s < nsteps; ++s) {
        if (t_end > 0.0 && *t >= t_end) break;
        /* Stage inputs carry their ghosts; non-interior parts of U1, U2 are    */
        /* filled by the boundary step before they are read.                    */
        memcpy(U1, U, n * sizeof(double));
        memcpy(U2, U, n * sizeof(double));
        stage_bc(g, p, U, sx, sy, *t);
        double dt = cfl_dt(g, p, U, *t, t_end);
        /* stage 1 (stage inputs at t, t + dt, t + dt/2) */
        memcpy(sxa, sx, P * sizeof(double));
        memcpy(sya, sy ? sy : sx, P * sizeof(double));
        if (residual(g, p, U, sx, sy, L, sxa, g->dim == 2 ? sya : NULL)) goto fail;
        stage_combine(g, 1, dt, U, U, L, U1);
        stage_bc(g, p, U1, sxa, g->dim == 2 ? sya : NULL, *t + dt);
        /* stage 2 */
        if (residual(g, p, U1, sxa, sya, L, sx, g->dim == 2 ? sy : NULL)) goto fail;
        stage_combine(g, 2, dt, U, U1, L, U2);
        stage_bc(g, p, U2, sx, g->dim == 2 ? sy : NULL, *t + 0.5 * dt);
        /* stage 3 */
        if (residual(g, p, U2, sx, sy, L, sxa, g->dim == 2 ? sya : NULL)) goto fail;
        stage_combine(g, 3, dt, U, U2, L, U);
        memcpy(sx, sxa, P * sizeof(double));
        if (g->dim == 2) memcpy(sy, sya, P * sizeof(double));
        *t += dt;
        if (dt_hist) dt_hist[s] = dt;
        ++taken;
    }
    /* First-order source: the strengths handed back are those the next     */
    /* stage would read, the first-order strengths of the final state.       */
    if (p->df_source == ORC_DF_FIRST_ORDER && nsteps > 0) stage_bc(g, p, U, sx, sy, *t);
    free(U1); free(U2); free(L); free(sxa); free(sya);
    return taken;
fail:
    free(U1); free(U2); free(L); free(sxa); free(sya);
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Test hooks: single-cell pieces of the reconstruction.                     */
/* ------------------------------------------------------------------------ */

/* ASE-DF polynomial of one cell: W[0..2R], s[0..2R-1] (cell R is W_0).      */
int orc_poly(const orc_params *p, const double *W, const double *s, int npts, const double *xi, double *out)
{
    int R = halfwidth(p->order);
    return ase_poly(p, p->order, W + R, s + R, npts, xi, out, NULL);
}

/* WENO-Z-AO(5,3) with given DF factors: W[0..4] (W_0 = W[2]).               */
void orc_weno_ao53(const orc_params *p, const double *W, const double *alpha, int npts, const double *xi,
                   double *out)
{
    weno_ao53_df(p, W + 2, alpha, npts, xi, out, NULL);
}

/* Stencil coefficients W_xk of stencil kind (3 with sub = -1,0,1; 5; 7; 9)   */
/* applied to W (centred at W[R]).                                            */
int orc_coeffs(int kind, int sub, const double *W, double *a)
{
    if (kind == 3) { coef_r3(sub, W + 2, a); return 2; }
    if (kind == 5) { coef_r5(W + 2, a); return 4; }
    if (kind == 7) { coef_r7(W + 3, a); return 6; }
    if (kind == 9) { coef_r9(W + 4, a); return 8; }
    return -1;
}

double orc_beta3(const double *a) { return beta3(a); }
double orc_zk(int k, double xi) { return Zk(k, xi); }
double orc_alpha(double A, double thres) { return df_alpha(A, thres); }
void orc_gauss(int G, double *node, double *eta) { gauss_legendre(G, node, eta); }

/* Threads of the parallel loops (n >= 1); returns the count now in effect
   (1 when built without OpenMP). */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Discontinuity strength and LF flux of one Gauss point (dir 0 / 1). */
double orc_sigma_point(const orc_grid *g, const orc_params *p, const double *Wl, const double *Wr, int dir)
{
    prim_t ql, qr;
    int okl = primitives(g, p, Wl, dir, &ql);
    int okr = primitives(g, p, Wr, dir, &qr);
    return sigma_point(&ql, okl, &qr, okr);
}

void orc_lf_point(const orc_grid *g, const orc_params *p, const double *Wl, const double *Wr, int dir, double *F)
{
    prim_t ql, qr;
    primitives(g, p, Wl, dir, &ql);
    primitives(g, p, Wr, dir, &qr);
    lf_flux(g, Wl, &ql, Wr, &qr, dir, F);
}

/* ======================================================================== */
/* Gas-kinetic flux and two-stage fourth-order time stepping, 1D            */
/* (Sec. 2.2 and App. A).                                                    */
/*                                                                          */
/* Velocity space of the 1D BGK model: particle velocity u and K internal   */
/* degrees of freedom xi; psi = (1, u, (u^2 + xi^2)/2).  The paper writes   */
/* the 2D form, K = (4 - 2 gamma)/(gamma - 1); with no v-direction the v    */
/* degree of freedom joins the internal ones, K = (3 - gamma)/(gamma - 1)   */
/* (reading: the 1D form of the same model).  A Maxwellian is              */
/* g = rho (lambda/pi)^((K+1)/2) exp(-lambda((u-U)^2 + xi^2)) with          */
/* lambda = rho / (2 p).                                                    */
/*                                                                          */
/* Moments are taken of polynomials in (u, xi^2), stored as coefficient     */
/* tables c[n][l] of u^n xi^(2l): <c> = sum c[n][l] <u^n> <xi^(2l)>, the    */
/* factorisation of App. A.                                                  */
/* ======================================================================== */

enum { GKS_NU = 8, GKS_NL = 3 };
typedef struct { double c[GKS_NU][GKS_NL]; } upoly;

typedef struct {
    double rho, U, lam, K;
    double um[GKS_NU];   /* <u^n>, whole line        */
    double up[GKS_NU];   /* <u^n>_{>0}, half line    */
    double un[GKS_NU];   /* <u^n>_{<0}, half line    */
    double xm[GKS_NL];   /* <xi^(2l)>                */
} gks_maxw;

/* c1, c2: numerical collision time; tau: collision time outside the
   exponentials (inviscid); mu > 0: viscous flow, tau = mu/p (Sec. 2.2) */
typedef struct { double c1, c2, tau, mu; } orc_gks;

/* Maxwellian of the state W = (rho, rho U, E) and its moments (App. A):     */
/*   <u^0> = 1, <u^1> = U, <u^(n+2)> = U <u^(n+1)> + (n+1)/(2 lambda) <u^n>; */
/*   half lines start from erfc(-+sqrt(lambda) U)/2 and                      */
/*   +-exp(-lambda U^2) / (2 sqrt(pi lambda)), same recursion;              */
/*   <xi^0> = 1, <xi^2> = K/(2 lambda), <xi^(2l)> = (K + 2(l-1))/(2 lambda)  */
/*   <xi^(2(l-1))>.                                                          */
/* Returns -1 when rho <= 0 or p <= 0.                                       */
static int gks_maxwellian(double gamma, const double *W, gks_maxw *m)
{
    double rho = W[0];
    double U = W[1] / rho;
    double p = (gamma - 1.0) * (W[2] - 0.5 * rho * U * U);
    if (!(rho > 0.0) || !(p > 0.0)) return -1;
    m->rho = rho;
    m->U = U;
    m->lam = rho / (2.0 * p);
    m->K = (3.0 - gamma) / (gamma - 1.0);
    double lam = m->lam;
    m->um[0] = 1.0;
    m->um[1] = U;
    m->up[0] = 0.5 * erfc(-sqrt(lam) * U);
    m->un[0] = 0.5 * erfc(sqrt(lam) * U);
    const double pi = 3.14159265358979323846;
    double e = exp(-lam * U * U) / (2.0 * sqrt(pi * lam));
    m->up[1] = U * m->up[0] + e;
    m->un[1] = U * m->un[0] - e;
    for (int n = 0; n + 2 < GKS_NU; ++n) {
        double h = (double)(n + 1) / (2.0 * lam);
        m->um[n + 2] = U * m->um[n + 1] + h * m->um[n];
        m->up[n + 2] = U * m->up[n + 1] + h * m->up[n];
        m->un[n + 2] = U * m->un[n + 1] + h * m->un[n];
    }
    m->xm[0] = 1.0;
    for (int l = 1; l < GKS_NL; ++l) m->xm[l] = (m->K + 2.0 * (l - 1)) / (2.0 * lam) * m->xm[l - 1];
    return 0;
}

/* psi_j as a polynomial (j = 0, 1, 2). */
static upoly gks_psi(int j)
{
    upoly q;
    memset(&q, 0, sizeof q);
    if (j == 0) q.c[0][0] = 1.0;
    else if (j == 1) q.c[1][0] = 1.0;
    else { q.c[2][0] = 0.5; q.c[0][1] = 0.5; }
    return q;
}

/* a . psi = a_1 + a_2 u + a_3 (u^2 + xi^2)/2 (the form of every micro slope). */
static upoly gks_lin(const double a[3])
{
    upoly q;
    memset(&q, 0, sizeof q);
    for (int j = 0; j < 3; ++j) {
        upoly s = gks_psi(j);
        for (int n = 0; n < GKS_NU; ++n)
            for (int l = 0; l < GKS_NL; ++l) q.c[n][l] += a[j] * s.c[n][l];
    }
    return q;
}

static upoly gks_mul(const upoly *x, const upoly *y)
{
    upoly q;
    memset(&q, 0, sizeof q);
    for (int n = 0; n < GKS_NU; ++n)
        for (int l = 0; l < GKS_NL; ++l) {
            if (x->c[n][l] == 0.0) continue;
            for (int n2 = 0; n + n2 < GKS_NU; ++n2)
                for (int l2 = 0; l + l2 < GKS_NL; ++l2) q.c[n + n2][l + l2] += x->c[n][l] * y->c[n2][l2];
        }
    return q;
}

/* u^k as a polynomial. */
static upoly gks_upow(int k)
{
    upoly q;
    memset(&q, 0, sizeof q);
    q.c[k][0] = 1.0;
    return q;
}

/* <q> with the u-moments um (whole or half line) and the xi-moments xm. */
static double gks_avg(const upoly *q, const double *um, const double *xm)
{
    double s = 0.0;
    for (int n = 0; n < GKS_NU; ++n)
        for (int l = 0; l < GKS_NL; ++l) s += q->c[n][l] * um[n] * xm[l];
    return s;
}

/* <q psi_j>, j = 0..2. */
static void gks_avg_psi(const upoly *q, const double *um, const double *xm, double out[3])
{
    for (int j = 0; j < 3; ++j) {
        upoly s = gks_psi(j);
        upoly t = gks_mul(q, &s);
        out[j] = gks_avg(&t, um, xm);
    }
}

/* Micro slope a from <a . psi psi_j> = b_j (App. A, M a = b with           */
/* M_ij = <psi_i psi_j>), solved by Gaussian elimination with partial        */
/* pivoting on the moment matrix built from its definition.                  */
static void gks_solve(const gks_maxw *m, const double b[3], double a[3])
{
    double M[3][4];
    for (int i = 0; i < 3; ++i) {
        upoly pi = gks_psi(i);
        for (int j = 0; j < 3; ++j) {
            upoly pj = gks_psi(j);
            upoly t = gks_mul(&pi, &pj);
            M[i][j] = gks_avg(&t, m->um, m->xm);
        }
        M[i][3] = b[i];
    }
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (piv != c)
            for (int k = 0; k < 4; ++k) { double t = M[c][k]; M[c][k] = M[piv][k]; M[piv][k] = t; }
        for (int r = c + 1; r < 3; ++r) {
            double f = M[r][c] / M[c][c];
            for (int k = c; k < 4; ++k) M[r][k] -= f * M[c][k];
        }
    }
    for (int c = 2; c >= 0; --c) {
        double s = M[c][3];
        for (int k = c + 1; k < 3; ++k) s -= M[c][k] * a[k];
        a[c] = s / M[c][c];
    }
}

/* Spatial slope a (b = W_x / rho) and the time slope A from the            */
/* compatibility condition <A + a u> = 0 moment by moment:                  */
/* M A = -<(a . psi) u psi>.                                                 */
static void gks_slopes(const gks_maxw *m, const double *Wx, double a[3], double A[3])
{
    double b[3];
    for (int j = 0; j < 3; ++j) b[j] = Wx[j] / m->rho;
    gks_solve(m, b, a);
    upoly la = gks_lin(a), u1 = gks_upow(1);
    upoly t = gks_mul(&la, &u1);
    double bt[3];
    gks_avg_psi(&t, m->um, m->xm, bt);
    for (int j = 0; j < 3; ++j) bt[j] = -bt[j];
    gks_solve(m, bt, A);
}

/* Time integrals over [0, delta] of the coefficients of the distribution    */
/* at the interface (Eq. GKS flux), collision time tau outside and tau_n in  */
/* the exponentials, E = exp(-delta/tau_n):                                  */
/*   q0 = int (1 - e^{-t/tau_n})                                             */
/*   q1 = int ((t + tau) e^{-t/tau_n} - tau)                                 */
/*   q2 = int (t - tau + tau e^{-t/tau_n})                                   */
/*   q3 = int e^{-t/tau_n}                                                   */
/*   q4 = int (tau + t) e^{-t/tau_n}                                         */
/*   q5 = int tau e^{-t/tau_n}                                               */
/* with int e^{-t/tau_n} = tau_n (1 - E) and                                */
/* int t e^{-t/tau_n} = tau_n^2 (1 - E) - tau_n delta E.                      */
/* tau_n = 0 is the limit E = 0 (exp(-inf)).                                 */
static void gks_time_coef(double tau, double taun, double delta, double q[6])
{
    double E = exp(-delta / taun);
    double i0 = taun * (1.0 - E);
    double i1 = taun * taun * (1.0 - E) - taun * delta * E;
    q[0] = delta - i0;
    q[1] = i1 + tau * i0 - tau * delta;
    q[2] = 0.5 * delta * delta - tau * delta + tau * i0;
    q[3] = i0;
    q[4] = tau * i0 + i1;
    q[5] = tau * i0;
}

/* Flux transported through the interface over [0, delta] (Eq. total flux)   */
/* from the two interface states W^l, W^r and their x-slopes:               */
/*   W^c   = int_{u>0} psi g^l + int_{u<0} psi g^r      (Sec. 3.5)           */
/*   W^c_x = int_{u>0} psi g^l_x + int_{u<0} psi g^r_x, g_x = (a . psi) g     */
/*   F = rho_c [q0 <u psi> + q1 <(a^c.psi) u^2 psi> + q2 <(A^c.psi) u psi>]_c */
/*     + rho_l [q3 <u psi> - q4 <(a^l.psi) u^2 psi> - q5 <(A^l.psi) u psi>]_{l,u>0} */
/*     + rho_r [same]_{r,u<0}.                                               */
/* Returns -1 when a state (or W^c) is not physical.                         */
static int gks_flux_int(double gamma, const double *Wl, const double *Wlx, const double *Wr, const double *Wrx,
                        double tau, double taun, double delta, double *F)
{
    gks_maxw ml, mr, mc;
    if (gks_maxwellian(gamma, Wl, &ml) || gks_maxwellian(gamma, Wr, &mr)) return -1;
    double al[3], Al[3], ar[3], Ar[3];
    gks_slopes(&ml, Wlx, al, Al);
    gks_slopes(&mr, Wrx, ar, Ar);
    upoly one = gks_upow(0), u1 = gks_upow(1), u2 = gks_upow(2);
    upoly pal = gks_lin(al), par = gks_lin(ar);
    double Wc[3], Wcx[3], t1[3], t2[3];
    gks_avg_psi(&one, ml.up, ml.xm, t1);
    gks_avg_psi(&one, mr.un, mr.xm, t2);
    for (int j = 0; j < 3; ++j) Wc[j] = ml.rho * t1[j] + mr.rho * t2[j];
    gks_avg_psi(&pal, ml.up, ml.xm, t1);
    gks_avg_psi(&par, mr.un, mr.xm, t2);
    for (int j = 0; j < 3; ++j) Wcx[j] = ml.rho * t1[j] + mr.rho * t2[j];
    if (gks_maxwellian(gamma, Wc, &mc)) return -1;
    double ac[3], Ac[3];
    gks_slopes(&mc, Wcx, ac, Ac);
    double q[6];
    gks_time_coef(tau, taun, delta, q);

    upoly pac = gks_lin(ac), pAc = gks_lin(Ac), pAl = gks_lin(Al), pAr = gks_lin(Ar);
    upoly c_a = gks_mul(&pac, &u2), c_A = gks_mul(&pAc, &u1);
    upoly l_a = gks_mul(&pal, &u2), l_A = gks_mul(&pAl, &u1);
    upoly r_a = gks_mul(&par, &u2), r_A = gks_mul(&pAr, &u1);
    double e0[3], e1[3], e2[3], l0[3], l1[3], l2[3], r0[3], r1[3], r2[3];
    gks_avg_psi(&u1, mc.um, mc.xm, e0);
    gks_avg_psi(&c_a, mc.um, mc.xm, e1);
    gks_avg_psi(&c_A, mc.um, mc.xm, e2);
    gks_avg_psi(&u1, ml.up, ml.xm, l0);
    gks_avg_psi(&l_a, ml.up, ml.xm, l1);
    gks_avg_psi(&l_A, ml.up, ml.xm, l2);
    gks_avg_psi(&u1, mr.un, mr.xm, r0);
    gks_avg_psi(&r_a, mr.un, mr.xm, r1);
    gks_avg_psi(&r_A, mr.un, mr.xm, r2);
    for (int j = 0; j < 3; ++j) {
        double fc = mc.rho * (q[0] * e0[j] + q[1] * e1[j] + q[2] * e2[j]);
        double fl = ml.rho * (q[3] * l0[j] - q[4] * l1[j] - q[5] * l2[j]);
        double fr = mr.rho * (q[3] * r0[j] - q[4] * r1[j] - q[5] * r2[j]);
        F[j] = fc + fl + fr;
    }
    return 0;
}

/* Numerical collision time of inviscid flow (Sec. 2.2):                     */
/*   tau_n = C1 dt + C2 |p_l - p_r| / (p_l + p_r) dt.                         */
/* Reading: the collision time outside the exponentials is the physical one, */
/* 0 for the Euler equations (gk->tau).                                     */
static double gks_taun(double gamma, const orc_gks *gk, const double *Wl, const double *Wr, double dt)
{
    double pl = (gamma - 1.0) * (Wl[2] - 0.5 * Wl[1] * Wl[1] / Wl[0]);
    double pr = (gamma - 1.0) * (Wr[2] - 0.5 * Wr[1] * Wr[1] / Wr[0]);
    return gk->c1 * dt + gk->c2 * fabs(pl - pr) / (pl + pr) * dt;
}

/* Flux and its time derivative at t_n from the two transported fluxes     */
/* (Eq. time advance): F = (4 F(dt/2) - F(dt))/dt,                          */
/* F_t = 4 (F(dt) - 2 F(dt/2)) / dt^2.                                       */
static int gks_point(double gamma, const orc_gks *gk, double dt, const double *Wl, const double *Wlx,
                     const double *Wr, const double *Wrx, double *Fn, double *Ft)
{
    double taun = gks_taun(gamma, gk, Wl, Wr, dt);
    double F1[3], F2[3];
    if (gks_flux_int(gamma, Wl, Wlx, Wr, Wrx, gk->tau, taun, dt, F1)) return -1;
    if (gks_flux_int(gamma, Wl, Wlx, Wr, Wrx, gk->tau, taun, 0.5 * dt, F2)) return -1;
    for (int j = 0; j < 3; ++j) {
        Fn[j] = (4.0 * F2[j] - F1[j]) / dt;
        Ft[j] = 4.0 * (F1[j] - 2.0 * F2[j]) / (dt * dt);
    }
    return 0;
}

/* L(W) and dL/dt on the interior cells of a 1D grid (Sec. 2.2):            */
/*   per face i+1/2: the ASE-DF polynomial of cell i at xi = 0 and of cell   */
/*   i+1 at xi = -1 give W^l, W^r and their slopes (d/dxi / dx); the face    */
/*   strength is the DF strength of (W^l, W^r) (as on the LF path); with    */
/*   positivity_fallback a non-physical side becomes its cell average with  */
/*   zero slope (reading, as R15); then F, F_t (gks_point) and               */
/*   L = -(F_{i+1/2} - F_{i-1/2})/dx, L_t likewise.                          */
static int residual_gks1d(const orc_grid *g, const orc_params *p, const orc_gks *gk, const double *U,
                          const double *sx, double dt, double *L, double *Lt, double *sx_new)
{
    int r = p->order, R = halfwidth(r), ng = g->ng, nx = g->nx;
    size_t P = plane(g);
    double *F = malloc((size_t)3 * (nx + 1) * sizeof(double));
    double *FT = malloc((size_t)3 * (nx + 1) * sizeof(double));
    if (!F || !FT) { free(F); free(FT); return -1; }
    int rc = 0;
    for (int a = -1; a < nx; ++a) {
        int Il = a + ng, Ir = a + 1 + ng;
        double Wl[3], Wr[3], Wlx[3], Wrx[3], Wlc[3], Wrc[3];
        for (int v = 0; v < 3; ++v) {
            double Wline[9], sline[8], out, dout;
            const double xr = 0.0, xl = -1.0;
            for (int m = -R; m <= R; ++m) Wline[m + R] = U[v * P + Il + m];
            for (int m = -R; m < R; ++m) sline[m + R] = sx[Il + m];
            ase_poly(p, r, Wline + R, sline + R, 1, &xr, &out, &dout);
            Wl[v] = out;
            Wlx[v] = dout / g->dx;
            for (int m = -R; m <= R; ++m) Wline[m + R] = U[v * P + Ir + m];
            for (int m = -R; m < R; ++m) sline[m + R] = sx[Ir + m];
            ase_poly(p, r, Wline + R, sline + R, 1, &xl, &out, &dout);
            Wr[v] = out;
            Wrx[v] = dout / g->dx;
            Wlc[v] = U[v * P + Il];
            Wrc[v] = U[v * P + Ir];
        }
        prim_t ql, qr;
        int okl = primitives(g, p, Wl, 0, &ql);
        int okr = primitives(g, p, Wr, 0, &qr);
        if (sx_new) sx_new[Il] = sigma_point(&ql, okl, &qr, okr);
        if (p->positivity_fallback) {
            if (okl != 0) for (int v = 0; v < 3; ++v) { Wl[v] = Wlc[v]; Wlx[v] = 0.0; }
            if (okr != 0) for (int v = 0; v < 3; ++v) { Wr[v] = Wrc[v]; Wrx[v] = 0.0; }
        }
        double Fn[3], Ft[3];
        if (gks_point(p->gamma, gk, dt, Wl, Wlx, Wr, Wrx, Fn, Ft)) {
            for (int v = 0; v < 3; ++v) Fn[v] = Ft[v] = NAN;
            rc = 1;
        }
        for (int v = 0; v < 3; ++v) {
            F[(size_t)v * (nx + 1) + (a + 1)] = Fn[v];
            FT[(size_t)v * (nx + 1) + (a + 1)] = Ft[v];
        }
    }
    for (int i = 0; i < nx; ++i)
        for (int v = 0; v < 3; ++v) {
            size_t c = (size_t)v * P + (size_t)(i + ng);
            L[c] = -(F[(size_t)v * (nx + 1) + (i + 1)] - F[(size_t)v * (nx + 1) + i]) / g->dx;
            Lt[c] = -(FT[(size_t)v * (nx + 1) + (i + 1)] - FT[(size_t)v * (nx + 1) + i]) / g->dx;
        }
    free(F);
    free(FT);
    (void)rc;   /* non-physical states propagate as NaN */
    return 0;
}

/* nsteps S2O4 steps (Eq. S2O4 temporal) of the 1D GKS solver:               */
/*   W*      = W^n + dt/2 L(W^n) + dt^2/8 L_t(W^n)                           */
/*   W^{n+1} = W^n + dt L(W^n) + dt^2/6 (L_t(W^n) + 2 L_t(W*)).              */
/* The DF state is lagged across the two stages as on the LF path (R9).     */
/* Returns the number of steps taken, or < 0 on error.                       */
int orc_step_gks(const orc_grid *g, const orc_params *p, const orc_gks *gk, double *U, double *sx, double *t,
                 int nsteps, double t_end, double *dt_hist)
{
    int e = check_args(g, p);
    if (e) return e;
    if (g->dim != 1 || gk->mu > 0.0) return -1;   /* viscous flow: 2D only */
    size_t P = plane(g), n = 3 * P;
    double *Ws = malloc(n * sizeof(double)), *L0 = calloc(n, sizeof(double)), *T0 = calloc(n, sizeof(double));
    double *L1 = calloc(n, sizeof(double)), *T1 = calloc(n, sizeof(double)), *sxa = malloc(P * sizeof(double));
    if (!Ws || !L0 || !T0 || !L1 || !T1 || !sxa) {
        free(Ws); free(L0); free(T0); free(L1); free(T1); free(sxa);
        return -1;
    }
    int taken = 0;
    for (int s = 0; s < nsteps; ++s) {
        if (t_end > 0.0 && *t >= t_end) break;
        stage_bc(g, p, U, sx, NULL, *t);
        double dt = cfl_dt(g, p, U, *t, t_end);
        memcpy(Ws, U, n * sizeof(double));
        memcpy(sxa, sx, P * sizeof(double));
        residual_gks1d(g, p, gk, U, sx, dt, L0, T0, sxa);
        for (int v = 0; v < 3; ++v)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = (size_t)v * P + (size_t)(i + g->ng);
                Ws[c] = U[c] + 0.5 * dt * L0[c] + 0.125 * dt * dt * T0[c];
            }
        stage_bc(g, p, Ws, sxa, NULL, *t + 0.5 * dt);
        residual_gks1d(g, p, gk, Ws, sxa, dt, L1, T1, sx);
        for (int v = 0; v < 3; ++v)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = (size_t)v * P + (size_t)(i + g->ng);
                U[c] = U[c] + dt * L0[c] + dt * dt / 6.0 * (T0[c] + 2.0 * T1[c]);
            }
        *t += dt;
        if (dt_hist) dt_hist[s] = dt;
        ++taken;
    }
    free(Ws); free(L0); free(T0); free(L1); free(T1); free(sxa);
    return taken;
}

/* L and L_t of one stage (ghosts and strengths filled inside, as            */
/* orc_residual); sx_new receives the face strengths (may be NULL).          */
int orc_residual_gks(const orc_grid *g, const orc_params *p, const orc_gks *gk, double *U, double *sx,
                     double dt, double *L, double *Lt, double *sx_new)
{
    int e = check_args(g, p);
    if (e) return e;
    if (g->dim != 1) return -1;
    stage_bc(g, p, U, sx, NULL, 0.0);
    return residual_gks1d(g, p, gk, U, sx, dt, L, Lt, sx_new);
}

/* Test hooks of the kinetic pieces. */
int orc_gks_moments(double gamma, const double *W, double *um, double *up, double *un, double *xm)
{
    gks_maxw m;
    if (gks_maxwellian(gamma, W, &m)) return -1;
    memcpy(um, m.um, sizeof m.um);
    memcpy(up, m.up, sizeof m.up);
    memcpy(un, m.un, sizeof m.un);
    memcpy(xm, m.xm, sizeof m.xm);
    return GKS_NU;
}

int orc_gks_slopes(double gamma, const double *W, const double *Wx, double *a, double *A)
{
    gks_maxw m;
    if (gks_maxwellian(gamma, W, &m)) return -1;
    gks_slopes(&m, Wx, a, A);
    return 0;
}

int orc_gks_flux(double gamma, const double *Wl, const double *Wlx, const double *Wr, const double *Wrx,
                 double tau, double taun, double delta, double *F)
{
    return gks_flux_int(gamma, Wl, Wlx, Wr, Wrx, tau, taun, delta, F);
}

int orc_gks_point(double gamma, const orc_gks *gk, double dt, const double *Wl, const double *Wlx,
                  const double *Wr, const double *Wrx, double *Fn, double *Ft)
{
    return gks_point(gamma, gk, dt, Wl, Wlx, Wr, Wrx, Fn, Ft);
}

/* ASE-DF polynomial and its xi-derivative at npts points. */
int orc_poly_d(const orc_params *p, const double *W, const double *s, int npts, const double *xi, double *out,
               double *dout)
{
    int R = halfwidth(p->order);
    return ase_poly(p, p->order, W + R, s + R, npts, xi, out, dout);
}

/* ======================================================================== */
/* Gas-kinetic flux and S2O4 stepping, 2D (Sec. 2.1-2.2, App. A).           */
/*                                                                          */
/* Local frame of a face: u along the normal, v along the face;             */
/* psi = (1, u, v, (u^2 + v^2 + xi^2)/2), K = (4 - 2 gamma)/(gamma - 1).     */
/* Polynomials in (u, v, xi^2) are coefficient tables c[n][m][l] of         */
/* u^n v^m xi^(2l); <c> = sum c <u^n> <v^m> <xi^(2l)> (App. A), the half    */
/* lines taken in u only.                                                   */
/* ======================================================================== */

enum { G2_N = 8, G2_L = 3 };
typedef struct { double c[G2_N][G2_N][G2_L]; } vpoly;

typedef struct {
    double rho, U, V, lam, K;
    double um[G2_N], up[G2_N], un[G2_N];
    double vm[G2_N];
    double xm[G2_L];
    double M[4][4];      /* <psi_i psi_j>, filled by g2_maxwellian */
} g2_maxw;

static vpoly g2_psi(int j);
static vpoly g2_mul(const vpoly *x, const vpoly *y);
static double g2_avg(const vpoly *q, const double *um, const g2_maxw *mw);

/* Maxwellian of the local-frame state W = (rho, rho U, rho V, E). */
static int g2_maxwellian(double gamma, const double *W, g2_maxw *m)
{
    double rho = W[0];
    double U = W[1] / rho, V = W[2] / rho;
    double p = (gamma - 1.0) * (W[3] - 0.5 * rho * (U * U + V * V));
    if (!(rho > 0.0) || !(p > 0.0)) return -1;
    m->rho = rho;
    m->U = U;
    m->V = V;
    m->lam = rho / (2.0 * p);
    m->K = (4.0 - 2.0 * gamma) / (gamma - 1.0);
    double lam = m->lam;
    const double pi = 3.14159265358979323846;
    m->um[0] = 1.0;
    m->um[1] = U;
    m->vm[0] = 1.0;
    m->vm[1] = V;
    m->up[0] = 0.5 * erfc(-sqrt(lam) * U);
    m->un[0] = 0.5 * erfc(sqrt(lam) * U);
    double e = exp(-lam * U * U) / (2.0 * sqrt(pi * lam));
    m->up[1] = U * m->up[0] + e;
    m->un[1] = U * m->un[0] - e;
    for (int n = 0; n + 2 < G2_N; ++n) {
        double h = (double)(n + 1) / (2.0 * lam);
        m->um[n + 2] = U * m->um[n + 1] + h * m->um[n];
        m->up[n + 2] = U * m->up[n + 1] + h * m->up[n];
        m->un[n + 2] = U * m->un[n + 1] + h * m->un[n];
        m->vm[n + 2] = V * m->vm[n + 1] + h * m->vm[n];
    }
    m->xm[0] = 1.0;
    for (int l = 1; l < G2_L; ++l) m->xm[l] = (m->K + 2.0 * (l - 1)) / (2.0 * lam) * m->xm[l - 1];
    for (int i = 0; i < 4; ++i) {
        vpoly pi = g2_psi(i);
        for (int j = 0; j < 4; ++j) {
            vpoly pj = g2_psi(j);
            vpoly t = g2_mul(&pi, &pj);
            m->M[i][j] = g2_avg(&t, m->um, m);
        }
    }
    return 0;
}

static vpoly g2_zero(void)
{
    vpoly q;
    memset(&q, 0, sizeof q);
    return q;
}

static vpoly g2_psi(int j)
{
    vpoly q = g2_zero();
    if (j == 0) q.c[0][0][0] = 1.0;
    else if (j == 1) q.c[1][0][0] = 1.0;
    else if (j == 2) q.c[0][1][0] = 1.0;
    else { q.c[2][0][0] = 0.5; q.c[0][2][0] = 0.5; q.c[0][0][1] = 0.5; }
    return q;
}

static vpoly g2_lin(const double a[4])
{
    vpoly q = g2_zero();
    for (int j = 0; j < 4; ++j) {
        vpoly s = g2_psi(j);
        for (int n = 0; n < G2_N; ++n)
            for (int m = 0; m < G2_N; ++m)
                for (int l = 0; l < G2_L; ++l) q.c[n][m][l] += a[j] * s.c[n][m][l];
    }
    return q;
}

/* Product of two polynomials (terms beyond the table's degrees must not   */
/* arise: the callers stay within u^7, v^7, xi^4).                          */
static vpoly g2_mul(const vpoly *x, const vpoly *y)
{
    int yi[G2_N * G2_N * G2_L][3], ny = 0;
    for (int n = 0; n < G2_N; ++n)
        for (int m = 0; m < G2_N; ++m)
            for (int l = 0; l < G2_L; ++l)
                if (y->c[n][m][l] != 0.0) { yi[ny][0] = n; yi[ny][1] = m; yi[ny][2] = l; ++ny; }
    vpoly q = g2_zero();
    for (int n = 0; n < G2_N; ++n)
        for (int m = 0; m < G2_N; ++m)
            for (int l = 0; l < G2_L; ++l) {
                double xv = x->c[n][m][l];
                if (xv == 0.0) continue;
                for (int k = 0; k < ny; ++k) {
                    int n2 = yi[k][0], m2 = yi[k][1], l2 = yi[k][2];
                    if (n + n2 < G2_N && m + m2 < G2_N && l + l2 < G2_L)
                        q.c[n + n2][m + m2][l + l2] += xv * y->c[n2][m2][l2];
                }
            }
    return q;
}

static vpoly g2_add(const vpoly *x, const vpoly *y)
{
    vpoly q = *x;
    for (int n = 0; n < G2_N; ++n)
        for (int m = 0; m < G2_N; ++m)
            for (int l = 0; l < G2_L; ++l) q.c[n][m][l] += y->c[n][m][l];
    return q;
}

/* u^a v^b */
static vpoly g2_mono(int a, int b)
{
    vpoly q = g2_zero();
    q.c[a][b][0] = 1.0;
    return q;
}

static double g2_avg(const vpoly *q, const double *um, const g2_maxw *mw)
{
    double s = 0.0;
    for (int n = 0; n < G2_N; ++n)
        for (int m = 0; m < G2_N; ++m)
            for (int l = 0; l < G2_L; ++l) s += q->c[n][m][l] * um[n] * mw->vm[m] * mw->xm[l];
    return s;
}

/* <q psi_j>, j = 0..3: each term c u^n v^m xi^(2l) of q times each term of */
/* psi_j, averaged (the product written out term by term).                  */
static void g2_avg_psi(const vpoly *q, const double *um, const g2_maxw *mw, double out[4])
{
    /* terms of psi_j: (coefficient, du, dv, dl) */
    static const double pc[4][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}, {0.5, 0.5, 0.5}};
    static const int pt[4][3][3] = {{{0, 0, 0}}, {{1, 0, 0}}, {{0, 1, 0}}, {{2, 0, 0}, {0, 2, 0}, {0, 0, 1}}};
    static const int pn[4] = {1, 1, 1, 3};
    for (int j = 0; j < 4; ++j) out[j] = 0.0;
    for (int n = 0; n < G2_N; ++n)
        for (int m = 0; m < G2_N; ++m)
            for (int l = 0; l < G2_L; ++l) {
                double c = q->c[n][m][l];
                if (c == 0.0) continue;
                for (int j = 0; j < 4; ++j)
                    for (int k = 0; k < pn[j]; ++k) {
                        int n2 = n + pt[j][k][0], m2 = m + pt[j][k][1], l2 = l + pt[j][k][2];
                        if (n2 >= G2_N || m2 >= G2_N || l2 >= G2_L) continue;   /* never reached */
                        out[j] += c * pc[j][k] * um[n2] * mw->vm[m2] * mw->xm[l2];
                    }
            }
}

/* M a = b with M_ij = <psi_i psi_j> (App. A), Gaussian elimination. */
static void g2_solve(const g2_maxw *mw, const double b[4], double a[4])
{
    double M[4][5];
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) M[i][j] = mw->M[i][j];
        M[i][4] = b[i];
    }
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (piv != c)
            for (int k = 0; k < 5; ++k) { double t = M[c][k]; M[c][k] = M[piv][k]; M[piv][k] = t; }
        for (int r = c + 1; r < 4; ++r) {
            double f = M[r][c] / M[c][c];
            for (int k = c; k < 5; ++k) M[r][k] -= f * M[c][k];
        }
    }
    for (int c = 3; c >= 0; --c) {
        double s = M[c][4];
        for (int k = c + 1; k < 4; ++k) s -= M[c][k] * a[k];
        a[c] = s / M[c][c];
    }
}

/* Normal and tangential slopes an, at from W_n, W_t and the time slope A  */
/* from <A + an u + at v> = 0.                                              */
static void g2_slopes(const g2_maxw *mw, const double *Wn, const double *Wt, double an[4], double at[4],
                      double A[4])
{
    double b[4];
    for (int j = 0; j < 4; ++j) b[j] = Wn[j] / mw->rho;
    g2_solve(mw, b, an);
    for (int j = 0; j < 4; ++j) b[j] = Wt[j] / mw->rho;
    g2_solve(mw, b, at);
    vpoly pn = g2_lin(an), pt = g2_lin(at), u1 = g2_mono(1, 0), v1 = g2_mono(0, 1);
    vpoly x = g2_mul(&pn, &u1), y = g2_mul(&pt, &v1);
    vpoly s = g2_add(&x, &y);
    double bt[4];
    g2_avg_psi(&s, mw->um, mw, bt);
    for (int j = 0; j < 4; ++j) bt[j] = -bt[j];
    g2_solve(mw, bt, A);
}

/* Transported flux over [0, delta] at one Gauss point in the local frame   */
/* (Eq. GKS flux with a . u = a_n u + a_t v).                                */
static int g2_flux_int(double gamma, const double *Wl, const double *Wln, const double *Wlt, const double *Wr,
                       const double *Wrn, const double *Wrt, double tau, double taun, double delta, double *F)
{
    g2_maxw ml, mr, mc;
    if (g2_maxwellian(gamma, Wl, &ml) || g2_maxwellian(gamma, Wr, &mr)) return -1;
    double lan[4], lat[4], lA[4], ran[4], rat[4], rA[4];
    g2_slopes(&ml, Wln, Wlt, lan, lat, lA);
    g2_slopes(&mr, Wrn, Wrt, ran, rat, rA);
    vpoly one = g2_mono(0, 0), u1 = g2_mono(1, 0), v1 = g2_mono(0, 1);
    double Wc[4], Wcn[4], Wct[4], t1[4], t2[4];
    g2_avg_psi(&one, ml.up, &ml, t1);
    g2_avg_psi(&one, mr.un, &mr, t2);
    for (int j = 0; j < 4; ++j) Wc[j] = ml.rho * t1[j] + mr.rho * t2[j];
    vpoly p1 = g2_lin(lan), p2 = g2_lin(ran);
    g2_avg_psi(&p1, ml.up, &ml, t1);
    g2_avg_psi(&p2, mr.un, &mr, t2);
    for (int j = 0; j < 4; ++j) Wcn[j] = ml.rho * t1[j] + mr.rho * t2[j];
    p1 = g2_lin(lat);
    p2 = g2_lin(rat);
    g2_avg_psi(&p1, ml.up, &ml, t1);
    g2_avg_psi(&p2, mr.un, &mr, t2);
    for (int j = 0; j < 4; ++j) Wct[j] = ml.rho * t1[j] + mr.rho * t2[j];
    if (g2_maxwellian(gamma, Wc, &mc)) return -1;
    double can[4], cat[4], cA[4];
    g2_slopes(&mc, Wcn, Wct, can, cat, cA);
    double q[6];
    gks_time_coef(tau, taun, delta, q);

    /* (a_n . psi) u + (a_t . psi) v, times u; and (A . psi) u */
    const double *an[3] = {can, lan, ran}, *at[3] = {cat, lat, rat}, *AA[3] = {cA, lA, rA};
    const g2_maxw *mm[3] = {&mc, &ml, &mr};
    const double *um[3] = {mc.um, ml.up, mr.un};
    double T0[3][4], T1[3][4], T2[3][4];
    for (int s = 0; s < 3; ++s) {
        vpoly pn = g2_lin(an[s]), pt = g2_lin(at[s]), pA = g2_lin(AA[s]);
        vpoly x = g2_mul(&pn, &u1), y = g2_mul(&pt, &v1);
        vpoly av = g2_add(&x, &y);
        vpoly avu = g2_mul(&av, &u1), Au = g2_mul(&pA, &u1);
        g2_avg_psi(&u1, um[s], mm[s], T0[s]);
        g2_avg_psi(&avu, um[s], mm[s], T1[s]);
        g2_avg_psi(&Au, um[s], mm[s], T2[s]);
    }
    for (int j = 0; j < 4; ++j) {
        double fc = mc.rho * (q[0] * T0[0][j] + q[1] * T1[0][j] + q[2] * T2[0][j]);
        double fl = ml.rho * (q[3] * T0[1][j] - q[4] * T1[1][j] - q[5] * T2[1][j]);
        double fr = mr.rho * (q[3] * T0[2][j] - q[4] * T1[2][j] - q[5] * T2[2][j]);
        F[j] = fc + fl + fr;
    }
    return 0;
}

/* F and F_t at t_n at one Gauss point (local frame), Eq. time advance.     */
/* Collision times (Sec. 2.2).  Inviscid: tau as given, tau_n = C1 dt +    */
/* C2 |p_l - p_r|/(p_l + p_r) dt.  Viscous (mu > 0): tau = mu/p with p the  */
/* pressure of the equilibrium state W^c at the interface (reading), and    */
/* tau_n = tau + C2 |p_l - p_r|/(p_l + p_r) dt.                              */
static int g2_times(double gamma, const orc_gks *gk, double dt, const double *Wl, const double *Wr, double *tau,
                    double *taun)
{
    double pl = (gamma - 1.0) * (Wl[3] - 0.5 * (Wl[1] * Wl[1] + Wl[2] * Wl[2]) / Wl[0]);
    double pr = (gamma - 1.0) * (Wr[3] - 0.5 * (Wr[1] * Wr[1] + Wr[2] * Wr[2]) / Wr[0]);
    double jump = gk->c2 * fabs(pl - pr) / (pl + pr) * dt;
    if (!(gk->mu > 0.0)) {
        *tau = gk->tau;
        *taun = gk->c1 * dt + jump;
        return 0;
    }
    g2_maxw ml, mr, mc;
    if (g2_maxwellian(gamma, Wl, &ml) || g2_maxwellian(gamma, Wr, &mr)) return -1;
    vpoly one = g2_mono(0, 0);
    double t1[4], t2[4], Wc[4];
    g2_avg_psi(&one, ml.up, &ml, t1);
    g2_avg_psi(&one, mr.un, &mr, t2);
    for (int j = 0; j < 4; ++j) Wc[j] = ml.rho * t1[j] + mr.rho * t2[j];
    if (g2_maxwellian(gamma, Wc, &mc)) return -1;
    *tau = gk->mu / (mc.rho / (2.0 * mc.lam));
    *taun = *tau + jump;
    return 0;
}

static int g2_point(double gamma, const orc_gks *gk, double dt, const double *Wl, const double *Wln,
                    const double *Wlt, const double *Wr, const double *Wrn, const double *Wrt, double *Fn,
                    double *Ft)
{
    double tau, taun;
    if (g2_times(gamma, gk, dt, Wl, Wr, &tau, &taun)) return -1;
    double F1[4], F2[4];
    if (g2_flux_int(gamma, Wl, Wln, Wlt, Wr, Wrn, Wrt, tau, taun, dt, F1)) return -1;
    if (g2_flux_int(gamma, Wl, Wln, Wlt, Wr, Wrn, Wrt, tau, taun, 0.5 * dt, F2)) return -1;
    for (int j = 0; j < 4; ++j) {
        Fn[j] = (4.0 * F2[j] - F1[j]) / dt;
        Ft[j] = 4.0 * (F1[j] - 2.0 * F2[j]) / (dt * dt);
    }
    return 0;
}

/* Rotation into the local frame of a face with normal (c, s) (Sec. 2.1):   */
/* (rho, rho(u c + v s), rho(-u s + v c), E); back with the transpose.       */
static void rot_in(int c, int s, const double *W, double *Wt)
{
    Wt[0] = W[0];
    Wt[1] = c * W[1] + s * W[2];
    Wt[2] = -s * W[1] + c * W[2];
    Wt[3] = W[3];
}

static void rot_out(int c, int s, const double *Ft, double *F)
{
    F[0] = Ft[0];
    F[1] = c * Ft[1] - s * Ft[2];
    F[2] = s * Ft[1] + c * Ft[2];
    F[3] = Ft[3];
}

/* One direction of the 2D GKS operator: face fluxes F and F_t (compact     */
/* face numbering) and the face strengths.                                   */
/*  1. normal reconstruction of the side cells on every row the tangential   */
/*     stencils reach: values and normal slopes (d/dxi / h_n) at the face;   */
/*  2. tangential reconstruction (reading R14 for the strengths) of the      */
/*     values -- at the Gauss points, with the tangential slope d/deta/h_t   */
/*     -- and of the normal slopes, as line averages with the same           */
/*     polynomial rule (reading R28);                                        */
/*  3. per Gauss point: strength, positivity fallback (value to the cell     */
/*     average, slopes to zero), the flux in the local frame of normal       */
/*     (cos, sin) = (1, 0) for x-faces, (0, 1) for y-faces, rotated back;    */
/*     quadrature with the Gauss weights.                                    */
static int sweep_gks2d(const orc_grid *g, const orc_params *p, const orc_gks *gk, int dir, const double *U,
                       const double *sx, const double *sy, double dt, double *Fx, double *Ftx, double *sig_out)
{
    int r = p->order, R = halfwidth(r), ng = g->ng, nv = 4;
    int G = ngauss(g, r);
    size_t P = plane(g);
    int ld = g->ld;
    double node[4], eta[4], xi_g[4];
    gauss_legendre(G, node, eta);
    for (int k = 0; k < G; ++k) xi_g[k] = -0.5 + node[k];
    const double hn = dir == 0 ? g->dx : g->dy, ht = dir == 0 ? g->dy : g->dx;
    const int cs = dir == 0 ? 1 : 0, sn = dir == 0 ? 0 : 1;
    int n_along = dir == 0 ? g->nx : g->ny;
    int n_across = dir == 0 ? g->ny : g->nx;
    size_t nf = (size_t)face_count(g, dir);
#define CELL2(a, c) ((dir == 0) ? ((size_t)((c) + ng) * ld + (size_t)((a) + ng)) \
                                : ((size_t)((a) + ng) * ld + (size_t)((c) + ng)))
    const double *snorm = dir == 0 ? sx : sy;
    const double *stang = dir == 0 ? sy : sx;
    ptrdiff_t s_along = dir == 0 ? 1 : ld;
    ptrdiff_t s_across = dir == 0 ? ld : 1;
    for (int c = 0; c < n_across; ++c) {
        for (int a = -1; a < n_along; ++a) {
            /* per side: line values / normal slopes of rows c-R..c+R */
            double V[2][4][9], S[2][4][9];
            for (int side = 0; side < 2; ++side) {
                int ac = a + side;
                const double xq = side == 0 ? 0.0 : -1.0;
                for (int m = -R; m <= R; ++m) {
                    size_t base = CELL2(ac, c + m);
                    for (int v = 0; v < nv; ++v) {
                        double Wline[9], sline[8], out, dout;
                        for (int k = -R; k <= R; ++k) Wline[k + R] = U[v * P + base + k * s_along];
                        for (int k = -R; k < R; ++k) sline[k + R] = snorm[base + k * s_along];
                        ase_poly(p, r, Wline + R, sline + R, 1, &xq, &out, &dout);
                        V[side][v][m + R] = out;
                        S[side][v][m + R] = dout / hn;
                    }
                }
            }
            double Wg[2][4][4], Wgn[2][4][4], Wgt[2][4][4];   /* [side][gauss][var] */
            for (int side = 0; side < 2; ++side) {
                size_t bc = CELL2(a + side, c);
                double st[8];
                for (int k = -R; k < R; ++k) st[k + R] = stang[bc + k * s_across];
                for (int v = 0; v < nv; ++v) {
                    double o[4], d[4], on[4];
                    ase_poly(p, r, V[side][v] + R, st + R, G, xi_g, o, d);
                    ase_poly(p, r, S[side][v] + R, st + R, G, xi_g, on, NULL);
                    for (int k = 0; k < G; ++k) {
                        Wg[side][k][v] = o[k];
                        Wgt[side][k][v] = d[k] / ht;
                        Wgn[side][k][v] = on[k];
                    }
                }
            }
            double Wcell[2][4];
            for (int side = 0; side < 2; ++side)
                for (int v = 0; v < nv; ++v) Wcell[side][v] = U[v * P + CELL2(a + side, c)];
            double Fs[4] = {0, 0, 0, 0}, Fts[4] = {0, 0, 0, 0}, ssum = 0.0;
            for (int k = 0; k < G; ++k) {
                prim_t ql, qr;
                int okl = primitives(g, p, Wg[0][k], dir, &ql);
                int okr = primitives(g, p, Wg[1][k], dir, &qr);
                ssum += sigma_point(&ql, okl, &qr, okr);
                double *Wl = Wg[0][k], *Wr = Wg[1][k];
                double *Wln = Wgn[0][k], *Wlt = Wgt[0][k], *Wrn = Wgn[1][k], *Wrt = Wgt[1][k];
                double z[4] = {0, 0, 0, 0};
                if (p->positivity_fallback) {
                    if (okl != 0) { Wl = Wcell[0]; Wln = z; Wlt = z; }
                    if (okr != 0) { Wr = Wcell[1]; Wrn = z; Wrt = z; }
                }
                /* local frame; the tangential direction is (-sin, cos) */
                double lW[4], lWn[4], lWt[4], rW[4], rWn[4], rWt[4];
                rot_in(cs, sn, Wl, lW);
                rot_in(cs, sn, Wln, lWn);
                rot_in(cs, sn, Wr, rW);
                rot_in(cs, sn, Wrn, rWn);
                double mt[4];
                for (int v = 0; v < 4; ++v) mt[v] = (dir == 0 ? 1.0 : -1.0) * Wlt[v];
                rot_in(cs, sn, mt, lWt);
                for (int v = 0; v < 4; ++v) mt[v] = (dir == 0 ? 1.0 : -1.0) * Wrt[v];
                rot_in(cs, sn, mt, rWt);
                double fl[4], ftl[4], F[4], Ftk[4];
                if (g2_point(p->gamma, gk, dt, lW, lWn, lWt, rW, rWn, rWt, fl, ftl)) {
                    for (int v = 0; v < 4; ++v) fl[v] = ftl[v] = NAN;
                }
                rot_out(cs, sn, fl, F);
                rot_out(cs, sn, ftl, Ftk);
                for (int v = 0; v < 4; ++v) {
                    Fs[v] += eta[k] * F[v];
                    Fts[v] += eta[k] * Ftk[v];
                }
            }
            int fi = dir == 0 ? a : c, fj = dir == 0 ? c : a;
            size_t fid = face_index(g, dir, fi, fj);
            /* no-slip adiabatic wall (reading): nothing crosses it, the mass
               and energy fluxes are zero; the momentum flux (pressure and
               viscous stress) is the kinetic one.  The mirrored ghost
               cells reverse the tangential velocity too, which the
               tangential-slope terms of the distribution do not see as a
               symmetry, so the kinetic mass flux would not vanish. */
            int lo = dir == 0 ? g->bc[0] : g->bc[2], hi = dir == 0 ? g->bc[1] : g->bc[3];
            if ((a == -1 && lo == ORC_BC_NOSLIP) || (a == n_along - 1 && hi == ORC_BC_NOSLIP)) {
                Fs[0] = Fs[3] = 0.0;
                Fts[0] = Fts[3] = 0.0;
            }
            for (int v = 0; v < nv; ++v) {
                Fx[(size_t)v * nf + fid] = Fs[v];
                Ftx[(size_t)v * nf + fid] = Fts[v];
            }
            if (sig_out) sig_out[CELL2(a, c)] = ssum / (double)G;
        }
    }
#undef CELL2
    return 0;
}

/* L and L_t of the 2D GKS operator on interior cells. */
static int residual_gks2d(const orc_grid *g, const orc_params *p, const orc_gks *gk, const double *U,
                          const double *sx, const double *sy, double dt, double *L, double *Lt, double *sx_new,
                          double *sy_new)
{
    int ng = g->ng;
    size_t P = plane(g);
    size_t nfx = (size_t)face_count(g, 0), nfy = (size_t)face_count(g, 1);
    double *Fx = malloc(4 * nfx * sizeof(double)), *Ftx = malloc(4 * nfx * sizeof(double));
    double *Fy = malloc(4 * nfy * sizeof(double)), *Fty = malloc(4 * nfy * sizeof(double));
    if (!Fx || !Ftx || !Fy || !Fty) { free(Fx); free(Ftx); free(Fy); free(Fty); return -1; }
    sweep_gks2d(g, p, gk, 0, U, sx, sy, dt, Fx, Ftx, sx_new);
    sweep_gks2d(g, p, gk, 1, U, sx, sy, dt, Fy, Fty, sy_new);
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            size_t c = (size_t)(j + ng) * g->ld + (size_t)(i + ng);
            for (int v = 0; v < 4; ++v) {
                size_t e = v * P + c;
                size_t fxp = face_index(g, 0, i, j), fxm = face_index(g, 0, i - 1, j);
                size_t fyp = face_index(g, 1, i, j), fym = face_index(g, 1, i, j - 1);
                L[e] = -(Fx[v * nfx + fxp] - Fx[v * nfx + fxm]) / g->dx - (Fy[v * nfy + fyp] - Fy[v * nfy + fym]) / g->dy;
                Lt[e] = -(Ftx[v * nfx + fxp] - Ftx[v * nfx + fxm]) / g->dx
                        - (Fty[v * nfy + fyp] - Fty[v * nfy + fym]) / g->dy;
            }
        }
    free(Fx); free(Ftx); free(Fy); free(Fty);
    return 0;
}

/* nsteps S2O4 steps of the 2D GKS solver (as orc_step_gks). */
int orc_step_gks2d(const orc_grid *g, const orc_params *p, const orc_gks *gk, double *U, double *sx, double *sy,
                   double *t, int nsteps, double t_end, double *dt_hist)
{
    int e = check_args(g, p);
    if (e) return e;
    if (g->dim != 2) return -1;
    size_t P = plane(g), n = 4 * P;
    double *Ws = malloc(n * sizeof(double)), *L0 = calloc(n, sizeof(double)), *T0 = calloc(n, sizeof(double));
    double *L1 = calloc(n, sizeof(double)), *T1 = calloc(n, sizeof(double));
    double *sxa = malloc(P * sizeof(double)), *sya = malloc(P * sizeof(double));
    if (!Ws || !L0 || !T0 || !L1 || !T1 || !sxa || !sya) {
        free(Ws); free(L0); free(T0); free(L1); free(T1); free(sxa); free(sya);
        return -1;
    }
    int taken = 0;
    for (int s = 0; s < nsteps; ++s) {
        if (t_end > 0.0 && *t >= t_end) break;
        stage_bc(g, p, U, sx, sy, *t);
        double dt = cfl_dt(g, p, U, *t, t_end);
        memcpy(Ws, U, n * sizeof(double));
        memcpy(sxa, sx, P * sizeof(double));
        memcpy(sya, sy, P * sizeof(double));
        residual_gks2d(g, p, gk, U, sx, sy, dt, L0, T0, sxa, sya);
        for (int v = 0; v < 4; ++v)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    size_t c = (size_t)v * P + (size_t)(j + g->ng) * g->ld + (size_t)(i + g->ng);
                    Ws[c] = U[c] + 0.5 * dt * L0[c] + 0.125 * dt * dt * T0[c];
                }
        stage_bc(g, p, Ws, sxa, sya, *t + 0.5 * dt);
        residual_gks2d(g, p, gk, Ws, sxa, sya, dt, L1, T1, sx, sy);
        for (int v = 0; v < 4; ++v)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    size_t c = (size_t)v * P + (size_t)(j + g->ng) * g->ld + (size_t)(i + g->ng);
                    U[c] = U[c] + dt * L0[c] + dt * dt / 6.0 * (T0[c] + 2.0 * T1[c]);
                }
        *t += dt;
        if (dt_hist) dt_hist[s] = dt;
        ++taken;
    }
    free(Ws); free(L0); free(T0); free(L1); free(T1); free(sxa); free(sya);
    return taken;
}

/* Test hooks of the 2D kinetic pieces (local frame). */
int orc_gks2_slopes(double gamma, const double *W, const double *Wn, const double *Wt, double *an, double *at,
                    double *A)
{
    g2_maxw m;
    if (g2_maxwellian(gamma, W, &m)) return -1;
    g2_slopes(&m, Wn, Wt, an, at, A);
    return 0;
}

int orc_gks2_point(double gamma, const orc_gks *gk, double dt, const double *Wl, const double *Wln,
                   const double *Wlt, const double *Wr, const double *Wrn, const double *Wrt, double *Fn, double *Ft)
{
    return g2_point(gamma, gk, dt, Wl, Wln, Wlt, Wr, Wrn, Wrt, Fn, Ft);
}
