/* Address/undefined-behaviour sanitizer run of the CPU oracle (test
 * infrastructure): the oracle's own source compiled into this driver with
 * -fsanitize=address,undefined, then every entry point exercised on small
 * grids of each kind -- 1D and 2D, every order, periodic, transmissive,
 * reflective, no-slip, inflow-slot and double-Mach sides, both DF sources,
 * the positivity replacement, the gas-kinetic solver in 1D and 2D, and the
 * argument checks.  Any out-of-bounds access, use after free, leak or
 * undefined operation aborts with a report; the exit status is 0 otherwise. */
#include "../../oracle/ase_oracle.c"

#include <stdio.h>

static void fill_quadrants(const orc_grid *g, double *U, double gamma)
{
    const double st[4][4] = {{1.5, 0.0, 0.0, 1.5}, {0.5323, 1.206, 0.0, 0.3}, {0.138, 1.206, 1.206, 0.129},
                             {0.5323, 0.0, 1.206, 0.3}};
    size_t P = plane(g);
    for (int j = 0; j < (g->dim == 1 ? 1 : g->ny); ++j)
        for (int i = 0; i < g->nx; ++i) {
            int q = (i * 10 >= 6 * g->nx) ? ((g->dim == 1 || j * 10 >= 6 * g->ny) ? 0 : 3)
                                          : ((g->dim == 1 || j * 10 >= 6 * g->ny) ? 1 : 2);
            const double *s = st[q];
            size_t c = (size_t)(g->dim == 1 ? 0 : j + g->ng) * g->ld + (size_t)(i + g->ng);
            double rho = s[0], u = s[1], v = s[2], p = s[3];
            U[c] = rho;
            U[P + c] = rho * u;
            if (g->dim == 2) {
                U[2 * P + c] = rho * v;
                U[3 * P + c] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v);
            } else {
                U[2 * P + c] = p / (gamma - 1.0) + 0.5 * rho * u * u;
            }
        }
}

static int run_case(int dim, int nx, int ny, int order, int bc, int df, int fb)
{
    orc_grid g;
    memset(&g, 0, sizeof(g));
    g.dim = dim;
    g.nx = nx;
    g.ny = dim == 1 ? 1 : ny;
    g.ng = (order + 1) / 2;
    g.ld = nx + 2 * g.ng + 3;
    for (int k = 0; k < 4; ++k) g.bc[k] = bc;
    if (bc == ORC_BC_INFLOW_SLOT) {
        g.bc[1] = g.bc[2] = g.bc[3] = ORC_BC_TRANSMISSIVE;
        g.inflow[0] = 5.0; g.inflow[1] = 5.0 * 30.0; g.inflow[2] = 0.0;
        g.inflow[3] = 0.4127 / (5.0 / 3.0 - 1.0) + 0.5 * 5.0 * 900.0;
        g.slot_lo = -0.05; g.slot_hi = 0.05; g.y0 = -0.25;
    }
    if (bc == ORC_BC_WALL_INFLOW) {
        g.bc[0] = g.bc[1] = ORC_BC_TRANSMISSIVE;
        g.bc[2] = ORC_BC_WALL_INFLOW;
        g.bc[3] = ORC_BC_MOVING_SHOCK;
        g.wall_x0 = 1.0 / 6.0; g.shock_x0 = 0.3; g.shock_speed = 10.0;
        g.inflow[0] = 8.0; g.inflow[1] = 8.0 * 7.145; g.inflow[2] = -8.0 * 4.125; g.inflow[3] = 563.5;
        g.outer[0] = 1.4; g.outer[3] = 2.5;
    }
    g.dx = 1.0 / nx;
    g.dy = dim == 1 ? g.dx : 1.0 / ny;
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.order = order;
    p.df_source = df;
    p.positivity_fallback = fb;
    p.gamma = bc == ORC_BC_INFLOW_SLOT ? 5.0 / 3.0 : 1.4;
    p.cfl = 0.4;
    p.sigma_thres = 2.0;
    p.eps = 1e-6;
    p.d_hi = p.d_lo = 0.85;
    int nv = dim == 1 ? 3 : 4;
    size_t P = plane(&g);
    double *U = calloc((size_t)nv * P, sizeof(double));
    double *sx = calloc(P, sizeof(double)), *sy = calloc(P, sizeof(double));
    fill_quadrants(&g, U, p.gamma);
    double t = 0.0, dt_hist[3];
    int rc = orc_sigma_init(&g, &p, U, sx, sy);
    if (rc == 0) rc = orc_step(&g, &p, U, sx, sy, &t, 3, 0.0, dt_hist) == 3 ? 0 : -99;
    if (rc == 0 && order > 1) {
        int G = dim == 1 ? 1 : (order - 1) / 2;
        for (int d = 0; d < dim; ++d) {
            size_t nf = (size_t)face_count(&g, d);
            double *wl = calloc((size_t)nv * G * nf, sizeof(double)), *wr = calloc((size_t)nv * G * nf, sizeof(double));
            double *F = calloc((size_t)nv * nf, sizeof(double)), *sg = calloc(P, sizeof(double));
            int8_t *lev = calloc((size_t)g.nx * g.ny, 1);
            rc |= orc_reconstruct(&g, &p, d, U, sx, sy, wl, wr, lev);
            rc |= orc_df_compute(&g, &p, d, wl, wr, sg);
            rc |= orc_flux(&g, &p, d, wl, wr, F);
            free(wl); free(wr); free(F); free(sg); free(lev);
        }
    }
    /* the gas-kinetic solver: 1D on every case it accepts, 2D at order 5 */
    if (rc == 0 && order > 1 && (dim == 1 || order == 5) &&
        (bc == ORC_BC_TRANSMISSIVE || bc == ORC_BC_PERIODIC || bc == ORC_BC_REFLECTIVE)) {
        orc_gks gk;
        memset(&gk, 0, sizeof(gk));
        gk.c1 = 0.05;
        gk.c2 = 1.0;
        double t2 = 0.0;
        if (dim == 1) rc = orc_step_gks(&g, &p, &gk, U, sx, &t2, 2, 0.0, NULL) == 2 ? 0 : -98;
        else rc = orc_step_gks2d(&g, &p, &gk, U, sx, sy, &t2, 2, 0.0, NULL) == 2 ? 0 : -97;
    }
    free(U); free(sx); free(sy);
    return rc;
}

int main(void)
{
    int fails = 0, n = 0;
    const int orders[] = {3, 5, 7, 9};
    const int bcs[] = {ORC_BC_PERIODIC, ORC_BC_TRANSMISSIVE, ORC_BC_REFLECTIVE, ORC_BC_NOSLIP};
    for (int oi = 0; oi < 4; ++oi)
        for (int b = 0; b < 4; ++b)
            for (int df = 0; df < 2; ++df) {
                int r = orders[oi];
                if (bcs[b] != ORC_BC_NOSLIP) {
                    fails += run_case(1, 23 + r, 1, r, bcs[b], df, 1) != 0;
                    ++n;
                }
                fails += run_case(2, 11 + r, 9 + r, r, bcs[b], df, df) != 0;
                ++n;
            }
    fails += run_case(2, 24, 16, 7, ORC_BC_INFLOW_SLOT, 1, 1) != 0;
    fails += run_case(2, 28, 14, 9, ORC_BC_WALL_INFLOW, 1, 0) != 0;
    n += 2;
    /* argument checks return errors, touch nothing */
    orc_grid g;
    memset(&g, 0, sizeof(g));
    orc_params p;
    memset(&p, 0, sizeof(p));
    p.order = 4;
    g.dim = 2; g.nx = 8; g.ny = 8; g.ng = 5; g.ld = 18;
    fails += orc_step(&g, &p, NULL, NULL, NULL, NULL, 1, 0.0, NULL) >= 0;
    p.order = 9; g.ng = 2;
    fails += orc_step(&g, &p, NULL, NULL, NULL, NULL, 1, 0.0, NULL) >= 0;
    n += 2;
    printf("oracle sanitizer run: %d cases, %d failed\n", n, fails);
    return fails ? 1 : 0;
}
