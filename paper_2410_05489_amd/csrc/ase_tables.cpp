// Host construction of the constant tables used by the reconstruction
// kernels: point-evaluation weights of the linear stencils and the values of
// the zero-mean basis at every evaluation point.
//
// Stencil coefficients: the zero-mean polynomial coefficients W_xk of the
// 3-, 5-, 7- and 9-cell stencils printed in Sec. 3.2-3.4 (with W_3 for the
// misprinted f_3 of the 7-cell W_x1), as integer numerators over a common
// denominator, taps ordered W_{-R}..W_{R}.  The zero-mean basis on the cell
// [-1,0] is Z_k(xi) = xi^k - (-1)^k/(k+1), the form under which those
// coefficients are the exact cell-average fit.
#include <cmath>
#include <cstring>

#include "ase_device.h"
#include "ase_host.h"

namespace ase {

namespace {

struct Stencil {
    int h;                  // half width
    int ncoef;              // number of coefficients W_x1..W_xn
    double den[8];
    double num[8][9];       // num[k][m+h], m = -h..h
};

// S^{r3}_0
const Stencil kS3 = {1, 2, {1, 2}, {{0, -1, 1}, {1, -2, 1}}};

// S^{r5}
const Stencil kS5 = {2, 4, {12, 8, 6, 24},
                     {{0, 1, -15, 15, -1}, {-1, 6, -8, 2, 1}, {0, -1, 3, -3, 1}, {1, -4, 6, -4, 1}}};

// S^{r7}
const Stencil kS7 = {3, 6, {180, 240, 36, 144, 120, 720},
                     {{0, -2, 25, -245, 245, -25, 2},
                      {7, -57, 210, -230, 15, 63, -8},
                      {0, 1, -11, 28, -28, 11, -1},
                      {-2, 15, -39, 46, -24, 3, 1},
                      {0, -1, 5, -10, 10, -5, 1},
                      {1, -6, 15, -20, 15, -6, 1}}};

// S^{r9}
const Stencil kS9 = {4, 8, {5040, 30240, 1440, 3456, 480, 8640, 5040, 40320},
                     {{0, 9, -119, 889, -7175, 7175, -889, 119, -9},
                      {-205, 2081, -9835, 28679, -27895, -2065, 11459, -2455, 236},
                      {0, -7, 89, -587, 1365, -1365, 587, -89, 7},
                      {13, -128, 556, -1160, 1174, -464, -68, 88, -11},
                      {0, 1, -11, 41, -75, 75, -41, 11, -1},
                      {-5, 46, -170, 334, -380, 250, -86, 10, 1},
                      {0, -1, 7, -21, 35, -35, 21, -7, 1},
                      {1, -8, 28, -56, 70, -56, 28, -8, 1}}};

double zk(int k, double xi)
{
    double p = 1.0;
    for (int i = 0; i < k; ++i) p *= xi;
    return p - ((k % 2 == 0) ? 1.0 : -1.0) / double(k + 1);
}

void gauss_nodes(int G, double *x, double *w)
{
    if (G == 1) {
        x[0] = 0.0;
        w[0] = 1.0;
    } else if (G == 2) {
        const double a = 1.0 / (2.0 * std::sqrt(3.0));
        x[0] = -a; x[1] = a;
        w[0] = w[1] = 0.5;
    } else if (G == 3) {
        const double a = std::sqrt(0.15);   // sqrt(3/5)/2
        x[0] = -a; x[1] = 0.0; x[2] = a;
        w[0] = w[2] = 5.0 / 18.0;
        w[1] = 4.0 / 9.0;
    } else {
        const double t = 2.0 * std::sqrt(1.2) / 7.0;
        const double in = 0.5 * std::sqrt(3.0 / 7.0 - t), out = 0.5 * std::sqrt(3.0 / 7.0 + t);
        const double wi = 0.25 + std::sqrt(30.0) / 72.0, wo = 0.25 - std::sqrt(30.0) / 72.0;
        x[0] = -out; x[1] = -in; x[2] = in; x[3] = out;
        w[0] = w[3] = wo;
        w[1] = w[2] = wi;
    }
}

}  // namespace

void build_tables(Tables *t)
{
    std::memset(t, 0, sizeof(*t));
    const Stencil *st[4] = {&kS3, &kS5, &kS7, &kS9};
    for (int oi = 0; oi < 4; ++oi) {
        const int r = 2 * oi + 3;
        const int G = (r - 1) / 2;
        double pts[kMaxPts] = {0.0, -1.0, 0, 0, 0, 0};
        double gx[4], gw[4];
        gauss_nodes(G, gx, gw);
        for (int k = 0; k < G; ++k) {
            pts[2 + k] = -0.5 + gx[k];
            t->eta[oi][k] = gw[k];
        }
        const int np = 2 + G;
        for (int q = 0; q < np; ++q) {
            for (int k = 1; k <= 4; ++k) t->z[oi][q][k - 1] = zk(k, pts[q]);
            for (int li = 0; li < 4; ++li) {
                const Stencil &S = *st[li];
                double *w = t->lin[oi][li][q];
                w[4] = 1.0;  // W_0
                for (int k = 1; k <= S.ncoef; ++k) {
                    const double zq = zk(k, pts[q]);
                    for (int m = -S.h; m <= S.h; ++m) w[4 + m] += S.num[k - 1][m + S.h] / S.den[k - 1] * zq;
                }
            }
        }
    }
}

}  // namespace ase
