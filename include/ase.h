/*
 * ase.h -- C ABI of the MI355X (gfx950) ASE-DF library (libase.so).
 *
 * Adaptive-stencil-extension reconstruction driven by the discontinuity
 * feedback factor (ASE-DF), Lax-Friedrichs interface flux and SSP-RK3
 * update for the compressible Euler equations on uniform 1D/2D grids, after
 * Zhang, Zhao, Ji & Xu, "An Adaptive Reconstruction Method for Arbitrary
 * High-Order Accuracy Using Discontinuity Feedback" (arXiv 2410.05489).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers to float64 (int8 for levels)
 *    owned by the caller; the library never allocates, frees or keeps them.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *    asynchronous on that stream; results are ready once the caller
 *    synchronises the stream.  Scalars such as dt and t live in device
 *    memory so whole steps can run without a host round trip.  (Only
 *    ASE_FLAG_FAIL_NONPHYSICAL makes ase_step / ase_step_gks synchronise,
 *    to read back the count they report.)
 *  - Return value: ASE_OK (0) or a negative ASE_ERR_* code; the message of
 *    the last failure on the calling host thread is ase_last_error().
 *    Argument errors are detected before anything is launched.
 *  - State layout (structure of arrays with ghost cells):
 *      U[v*NY*ld + J*ld + I]   v = conserved variable, J row, I column
 *    NX = nx + 2 ng columns, NY = ny + 2 ng rows (NY = 1 in 1D), row stride
 *    ld >= NX; interior cell (i,j) is at I = i+ng, J = j+ng.  Variables are
 *    (rho, rho u, E) in 1D and (rho, rho u, rho v, rho E) in 2D.
 *  - Discontinuity strengths (the DF state) use one plane of the same shape:
 *      sx[J*ld + I]  strength of the x-face between cells (I,J), (I+1,J)
 *      sy[J*ld + I]  strength of the y-face between cells (I,J), (I,J+1)
 *    The "flux faces" are x-faces i+1/2, i in [-1, nx-1], of interior rows
 *    and y-faces j+1/2, j in [-1, ny-1], of interior columns.  A stage
 *    writes the strengths of the flux faces; ase_bc_fill derives all other
 *    stored faces from them (periodic wrap) or from the two adjacent
 *    ghost-filled cell averages (first-order strength).
 *  - Face arrays (compact numbering): x-face i+1/2 of row j has index
 *    j*(nx+1) + (i+1); y-face j+1/2 of column i has index (j+1)*nx + i;
 *    in 1D face i+1/2 has index i+1.  nfaces = (nx+1)*ny resp. nx*(ny+1).
 *    Gauss-point states wl/wr are [v][k][face] with k over the G Gauss
 *    points of the face (G = (order-1)/2 in 2D, 1 in 1D), ordered by
 *    increasing coordinate; face fluxes F are [v][face] and already hold
 *    the quadrature sum  sum_k eta_k F_k  (weights normalised to 1).
 */
#ifndef ASE_H
#define ASE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ASE_OK = 0,
    ASE_ERR_ARG = -1,       /* bad pointer, size, direction or stage     */
    ASE_ERR_ORDER = -2,     /* order not in {3,5,7,9}                    */
    ASE_ERR_GHOST = -3,     /* ng < (order+1)/2                          */
    ASE_ERR_ALIGN = -4,     /* device pointer not 8-byte aligned         */
    ASE_ERR_HIP = -5,       /* a HIP runtime call failed                 */
    ASE_ERR_WORKSPACE = -6, /* workspace missing or too small            */
    ASE_ERR_NONPHYSICAL = -7 /* ASE_FLAG_FAIL_NONPHYSICAL: the final state
                                holds a cell with rho <= 0, p <= 0 or NaN */
};

/* Boundary codes.  TRANSMISSIVE: zero-gradient copy of the boundary cell;
 * INFLOW_SLOT: Dirichlet inflow state in the ghost cells of the slot rows
 * (x sides only); REFLECTIVE: slip wall, the ghost cells mirror the interior
 * cells with the momentum normal to the wall reversed (needs n >= ng). */
enum { ASE_BC_PERIODIC = 0, ASE_BC_TRANSMISSIVE = 1, ASE_BC_INFLOW_SLOT = 2, ASE_BC_REFLECTIVE = 3,
       ASE_BC_WALL_INFLOW = 4, ASE_BC_MOVING_SHOCK = 5, ASE_BC_NOSLIP = 6 };
/* ASE_BC_NOSLIP: no-slip adiabatic wall (Sec. 4, Example 5), any side:
 * ghost cells mirror the interior with the whole momentum reversed; lagged
 * strengths mirror as at a slip wall; on the gas-kinetic path the mass and
 * energy fluxes through it are zero. */

/* Flags of ase_params_t. */
enum {
    /* A Gauss-point state with rho <= 0 or p <= 0 is replaced by the
     * average of its own cell for the flux (its strength is +inf anyway). */
    ASE_FLAG_POSITIVITY_FALLBACK = 1,
    /* Source of the interface states the DF strengths (Sec. 3.1) are
     * computed from.  Set ("first order", the reading this library's
     * workloads use): the first-order states of the current stage input,
     * i.e. the two cell averages beside each face; ase_bc_fill then
     * recomputes every stored strength from the ghost-filled state, and
     * the 2D sweeps evaluate no Gauss-point strengths.  Clear ("lagged"):
     * the Gauss-point states of the previous stage's reconstruction, so the
     * strengths are part of the state and ase_bc_fill derives the non-flux
     * faces. */
    ASE_FLAG_DF_FIRST_ORDER = 2,
    /* ase_step, ase_step_gks: after the last step count the interior cells
     * whose average has rho <= 0, p <= 0 or a NaN component and return
     * ASE_ERR_NONPHYSICAL if there is one (U, the strengths and t are
     * written all the same).  The count is read back to the host, so the
     * call synchronises its stream; it cannot be captured in a graph
     * (ASE_ERR_ARG while the stream is capturing). */
    ASE_FLAG_FAIL_NONPHYSICAL = 4
};

/* Grid and boundary description (the problem statement of Sec. 2.1 and
 * the test set-ups of Sec. 4). */
typedef struct {
    int32_t dim;        /* 1 or 2                                           */
    int32_t nx, ny;     /* interior cells; ny = 1 in 1D                     */
    int32_t ng;         /* ghost layers per side, >= (order+1)/2            */
    int32_t ld;         /* row stride in elements, >= nx + 2 ng             */
    int32_t bc[4];      /* x-lo, x-hi, y-lo, y-hi: ASE_BC_*.  Periodic must
                           pair on both sides; INFLOW_SLOT only in x.       */
    double dx, dy;      /* cell sizes                                        */
    double y0;          /* lower edge of the domain (slot test)              */
    double inflow[4];   /* conservative state of INFLOW_SLOT ghost cells     */
    double slot_lo, slot_hi;  /* INFLOW_SLOT applies to ghost cells of rows
                           whose centre y lies in (slot_lo, slot_hi); other
                           rows of that side are transmissive.              */
    /* Boundaries of the double Mach reflection (Sec. 4, Example 4), y sides
     * only.  WALL_INFLOW (y-lo): ghost cells of columns whose centre x lies
     * below wall_x0 take the inflow state, the others mirror the wall (as
     * REFLECTIVE).  MOVING_SHOCK (y-hi): ghost cells of columns whose centre
     * x lies below shock_x0 + shock_speed t take the inflow state, the
     * others the outer state; t is the time of the stage being filled
     * (ase_step, ase_step_gks; the granular ase_bc_fill / ase_sigma_init
     * use t = 0).  Lagged strengths of their ghost faces are first-order
     * ones. */
    double x0;                /* left edge of the domain (column centres)    */
    double wall_x0;
    double shock_x0, shock_speed;
    double outer[4];          /* conservative state beyond the moving shock  */
} ase_grid_t;

/* Method parameters. */
typedef struct {
    int32_t order;      /* nominal order r: 3, 5, 7 or 9 (Sec. 3.2-3.4)     */
    int32_t flags;      /* ASE_FLAG_*                                        */
    double gamma;       /* ratio of specific heats                           */
    double cfl;         /* CFL number                                        */
    double sigma_thres; /* DF threshold (Remark 1; 2.0 in the paper)         */
    double eps;         /* WENO-Z epsilon (1e-6)                             */
    double d_hi, d_lo;  /* WENO-AO linear-weight parameters (0.85, 0.85)     */
    double dt_cap;      /* > 0: dt = min(CFL dt, dt_cap)                     */
} ase_params_t;

/* Message of the last failed call on this host thread ("" if none). */
const char *ase_last_error(void);

/* Library ABI version (increments on any signature change). */
int ase_version(void);

/* Ghost cells and derived strengths (boundary conditions of Sec. 4).
 * Fills every ghost cell of U (x first on interior rows, then y on every
 * column, so corners take the y rule applied to x-filled values; a moving
 * shock side at t = 0), then the
 * strengths a stage reads.  Lagged DF source: every stored strength that is
 * not a flux-face strength -- periodic faces take the wrapped flux-face
 * value, the others the first-order strength of their two cells.
 * First-order DF source: every stored strength becomes the first-order
 * strength of its two cells.  U: state layout, in/out.  sx, sy: in/out (sy
 * unused in 1D, may be NULL). */
int ase_bc_fill(const ase_grid_t *g, const ase_params_t *p, double *U, double *sx, double *sy,
                void *stream);

/* Initial DF state: fills the ghosts of U, then sets every stored strength
 * to the first-order strength of its two adjacent cell averages (the DF of
 * Sec. 3.1 applied to piecewise-constant states).  U in/out, sx/sy out. */
int ase_sigma_init(const ase_grid_t *g, const ase_params_t *p, double *U, double *sx, double *sy,
                   void *stream);

/* Time step: dt = CFL / max over interior cells of (|u|+c)/dx [+ (|v|+c)/dy]
 * (CFL number of Sec. 4), capped by dt_cap, clipped so that t + dt <= t_end
 * when t_end > 0, and 0 once t >= t_end.  U: state (interior read).
 * t: device scalar (in).  dt: device scalar (out).  ws: device workspace of
 * at least ase_workspace_bytes() bytes. */
int ase_cfl_dt(const ase_grid_t *g, const ase_params_t *p, const double *U, const double *t,
               double t_end, double *dt, void *ws, size_t ws_bytes, void *stream);

/* ASE-DF reconstruction along direction dir (0 = x-faces, 1 = y-faces):
 * normal reconstruction of every cell with the DF factors of the faces in
 * its stencil, then (2D) tangential reconstruction of the face values to
 * the Gauss points with the strengths of the perpendicular faces of the
 * side cell's column (Sec. 3.1 Remark 2, Sec. 3.2-3.4, Algorithm 1).
 * U, sx, sy: state with ghosts already filled (ase_bc_fill).
 * wl, wr: out, [v][k][face], left/right (lower/upper) states.
 * level: optional out, [ny][nx] int8 level of the normal reconstruction of
 * each interior cell: 9/7/5 linear order used, 2 = WENO-Z-AO(5,3) with DF,
 * 3 = DF-damped centred polynomial (order 3).  May be NULL. */
int ase_reconstruct(const ase_grid_t *g, const ase_params_t *p, int dir, const double *U,
                    const double *sx, const double *sy, double *wl, double *wr, int8_t *level,
                    void *stream);

/* Discontinuity strength of every flux face of direction dir (Sec. 3.1):
 * per Gauss point |pl-pr|/pl + |pl-pr|/pr + (Ma_n^l-Ma_n^r)^2 +
 * (Ma_t^l-Ma_t^r)^2 (+inf if a side has rho <= 0 or p <= 0), averaged over
 * the face's Gauss points.  wl, wr: in, [v][k][face].  sigma: out, the
 * strength plane (sx for dir 0, sy for dir 1); only flux faces written. */
int ase_df_compute(const ase_grid_t *g, const ase_params_t *p, int dir, const double *wl,
                   const double *wr, double *sigma, void *stream);

/* Lax-Friedrichs flux with local maximal signal speed at every Gauss point
 * (Sec. 2.3), summed with the Gauss weights (Sec. 2.1).  wl, wr: in.
 * F: out, [v][face]. */
int ase_flux(const ase_grid_t *g, const ase_params_t *p, int dir, const double *wl, const double *wr,
             double *F, void *stream);

/* One SSP-RK3 stage (Eq. SSP-RK3) on interior cells with
 * L = -(F_{i+1/2}-F_{i-1/2})/dx - (G_{j+1/2}-G_{j-1/2})/dy:
 *   stage 1: Uout = Un + dt L;  stage 2: Uout = 3/4 Un + 1/4 Us + 1/4 dt L;
 *   stage 3: Uout = 1/3 Un + 2/3 Us + 2/3 dt L.
 * dt: device scalar.  F, G: face fluxes [v][face] (G ignored in 1D).
 * Un, Us: state layout, in.  Uout: interior written (may alias Un). */
int ase_stage_update(const ase_grid_t *g, const ase_params_t *p, int stage, const double *dt,
                     const double *Un, const double *Us, const double *F, const double *G,
                     double *Uout, void *stream);

/* Bytes of device workspace that ase_step / ase_cfl_dt need for grid g. */
size_t ase_workspace_bytes(const ase_grid_t *g, const ase_params_t *p);

/* nsteps SSP-RK3 steps (Eq. SSP-RK3) of the whole method: the ASE-DF
 * reconstruction of Sec. 3 with Gauss points on the faces (Sec. 2.1), the
 * Lax-Friedrichs flux of Sec. 2.3 and the conservative update of the
 * semi-discrete form (Sec. 2.1).  The DF strengths a stage reads come from
 * its own cell averages (ASE_FLAG_DF_FIRST_ORDER; the strengths handed back
 * are those of the final state) or, lagged, from the previous stage's
 * Gauss-point states (each stage writes the strengths of its flux faces).
 * Per step: boundary fill, dt, then three stages of reconstruction, flux,
 * quadrature and update, all on device; the ghost cells of the stage
 * inputs are filled at their times t_n, t_n + dt, t_n + dt/2 (a moving
 * shock side reads it).  Steps stop advancing once t >=
 * t_end (t_end > 0); remaining launches are no-ops.
 * U, sx, sy: the state (U interior + flux-face strengths), in/out; the DF
 * state must come from ase_sigma_init or a previous ase_step.
 * t: device scalar, in/out.  dt_hist: optional device array [nsteps] of
 * the dt of each step (0 for skipped steps).  ws: device workspace of
 * ws_bytes >= ase_workspace_bytes(g, p). */
int ase_step(const ase_grid_t *g, const ase_params_t *p, double *U, double *sx, double *sy, double *t,
             double *dt_hist, int32_t nsteps, double t_end, void *ws, size_t ws_bytes, void *stream);

/* ---- Gas-kinetic solver, 1D (Sec. 2.2, App. A) -----------------------------
 * The paper's primary flux: the moments of the second-order BGK distribution
 * at the interface (Eq. GKS flux) integrated over the time step, with the
 * two-stage fourth-order time stepping (Eq. S2O4 temporal).  The
 * reconstruction (values and x-slopes of the ASE-DF polynomials at the
 * faces) and the DF state are those of the Lax-Friedrichs path. */
typedef struct {
    double c1, c2;  /* numerical collision time tau_n = c1 dt + c2 |p_l - p_r| / (p_l + p_r) dt */
    double tau;     /* collision time outside the exponentials: 0 for the Euler equations */
    double mu;      /* > 0: Navier-Stokes (2D only): tau = mu / p with p the pressure of the
                       equilibrium state at the Gauss point, tau_n = tau + c2 |p_l - p_r| /
                       (p_l + p_r) dt (c1 unused); Pr = 1, the BGK model's */
} ase_gks_t;

/* Flux F and its time derivative F_t at t_n of n independent faces
 * (Eq. time advance): from the transported fluxes over [0, dt] and
 * [0, dt/2] of the BGK distribution built on the interface states Wl, Wr
 * (1D conservative (rho, rho u, E)) and their x-slopes Wlx, Wrx.  All
 * arrays are device [3][n] (variable-major); p supplies gamma.  A face with
 * a non-physical state (rho <= 0 or p <= 0, also of the kinetic average)
 * gets NaN. */
int ase_gks_flux(const ase_params_t *p, const ase_gks_t *gk, int32_t n, const double *Wl, const double *Wlx,
                 const double *Wr, const double *Wrx, double dt, double *Fn, double *Ft, void *stream);

/* Bytes of device workspace ase_step_gks needs for grid g (1D: as
 * ase_workspace_bytes; 2D adds the face-point states and the face fluxes
 * of both directions).  0 on invalid arguments. */
size_t ase_gks_workspace_bytes(const ase_grid_t *g, const ase_params_t *p);

/* nsteps S2O4 steps of the gas-kinetic solver (Eq. S2O4 temporal):
 * W* = W^n + dt/2 L(W^n) + dt^2/8 L_t(W^n),
 * W^{n+1} = W^n + dt L(W^n) + dt^2/6 (L_t(W^n) + 2 L_t(W*)),
 * L and L_t the divergences of F and F_t.  Per step: boundary fill, dt
 * (CFL rule of ase_cfl_dt), two stages with a boundary fill between.  1D:
 * one fused launch per stage.  2D (Sec. 2.1): per direction a
 * reconstruction launch (values, normal slopes and tangential slopes of
 * both sides at every Gauss point: the normal ASE-DF reconstruction, then
 * the tangential one of the face values and of the normal slopes) and a
 * flux launch (the BGK flux in the local frame of each Gauss point,
 * rotated back, Gauss quadrature), then one update launch.  The DF state
 * is lagged across the stages as in ase_step (or first order with
 * ASE_FLAG_DF_FIRST_ORDER); with ASE_FLAG_POSITIVITY_FALLBACK a
 * non-physical interface state becomes its cell average with zero slopes.
 * Arguments as ase_step (sy: y-face strengths, 2D only, may be NULL in 1D;
 * ws_bytes >= ase_gks_workspace_bytes(g, p)). */
int ase_step_gks(const ase_grid_t *g, const ase_params_t *p, const ase_gks_t *gk, double *U, double *sx,
                 double *sy, double *t, double *dt_hist, int32_t nsteps, double t_end, void *ws,
                 size_t ws_bytes, void *stream);

/* ---- Batched 1D instances (one persistent launch) -------------------------
 * Many independent 1D problems of uneven size stored back to back:
 * instance k occupies stored cells [offsets[k], offsets[k] + ncells[k] +
 * 2 ng) of a concatenated state U[v * total + c] (v = rho, rho u, E) and of
 * a strength array sigma[c] (strength of the face between stored cells c and
 * c+1 of the same instance; the DF state as in the 1D grid form).  Every
 * instance has its own dx and its own time t[k] and dt (CFL of its own
 * cells); all share the method parameters and ng >= (order+1)/2; the
 * boundary kind is `bc` or, per instance, bc_inst (below).  The
 * caller guarantees disjoint, in-range instances (the kernel skips an
 * instance whose range leaves [0, total)); periodic instances need
 * ncells >= ng. */

/* Host-side packing of instances into nbins work bins (longest processing
 * time first on ncells): bin b holds bin_list[bin_start[b] ..
 * bin_start[b+1]).  HOST arrays: ncells[ninst] in, bin_start[nbins+1] and
 * bin_list[ninst] out.  Upload both to the device for ase_step_batched. */
int ase_batched_plan(int32_t ninst, const int32_t *ncells, int32_t nbins, int32_t *bin_start, int32_t *bin_list);

/* Device workspace of ase_step_batched for `total` stored cells. */
size_t ase_batched_workspace_bytes(int64_t total);

/* Boundary codes of a batch: `bc` (ASE_BC_PERIODIC, ASE_BC_TRANSMISSIVE or
 * ASE_BC_REFLECTIVE, both ends alike) applies to every instance unless
 * `bc_inst` (device [ninst], may be NULL) gives one code per instance; there
 * any other code means transmissive.  A periodic or reflective instance
 * needs ncells >= ng. */

/* First-order DF strengths of every instance (the 1D ase_sigma_init per
 * instance); fills the ghost cells of U.  Device arrays. */
int ase_batched_sigma_init(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                           const int64_t *offsets, const int32_t *ncells, int32_t ng, int64_t total, double *U,
                           double *sigma, void *stream);

/* nsteps SSP-RK3 steps of every instance in ONE persistent launch: nbins
 * workgroups of `threads` (256, 512 or 1024) lanes, each walking the instances of
 * its bin through all steps (ghost cells, DF state, per-instance dt and
 * boundary code, three stages of the 1D method of ase_step, Sec. 2.1-3.4)
 * without returning to the host.
 * Results equal ase_step on each instance alone.  t: device [ninst], in/out.
 * dt_hist: optional device [nsteps][ninst].  dt_replay: optional device
 * [nsteps][ninst] of time steps to take instead of the CFL rule (an entry
 * <= 0 stops that instance; dt_cap and the clipping at t_end are then not
 * applied) -- for replaying a recorded run.  t_end > 0 stops each instance at t_end.
 * status: optional device int32 [ninst], out.  When given, an instance whose
 * CFL time step is not a positive number at the start of step s (some cell
 * has rho <= 0, p <= 0 or a NaN: the method has lost the state) stops there
 * and gets status s+1; the others get 0.  A stopped instance keeps the
 * state and time it had (dt_hist 0 from step s on).  Without status such an
 * instance runs on with NaN values, as ase_step does.
 * With ASE_FLAG_DF_FIRST_ORDER the strengths handed back in sigma are the
 * first-order ones of each final state (ase_step likewise).
 * bin_start/bin_list: device copies of an ase_batched_plan. */
int ase_step_batched(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                     const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng, int64_t total,
                     double *U, double *sigma, double *t, double *dt_hist, const double *dt_replay,
                     int32_t *status, int32_t nsteps, double t_end, const int32_t *bin_start,
                     const int32_t *bin_list, int32_t nbins, int32_t threads, void *ws, size_t ws_bytes,
                     void *stream);

/* ---- Wide batched form (first-order DF source) -----------------------------
 * The persistent launch above walks every instance with one workgroup, so
 * the batch lasts as long as its longest instance.  The wide form gives each
 * instance of at least min_cells cells many workgroups instead: one launch
 * per RK stage (Sec. 2.1) over all tiles of these instances, on a second
 * stream of the library's beside the persistent launch, which keeps the
 * rest.  Results equal ase_step_batched's bit for bit (U including its
 * ghost cells, sigma, t, dt_hist, status).  Needs ASE_FLAG_DF_FIRST_ORDER
 * (strengths from the two cell averages beside each face, Sec. 3.1).
 *
 * threads_wide is 256 or 512 lanes per tile, optionally or'ed with
 * ASE_WIDE_STEP: then one launch per step instead of per stage, each tile
 * running the three stages of the step in on-chip memory over a window that
 * reaches three stages' stencils beyond its cells; tiles are then
 * threads_wide - 3 (order + 1) cells long instead of threads_wide - order - 1.
 * Plan and step call take the same value: the step's kernels skip an
 * instance whose tiles do not fit their tile length (it does not advance).
 *
 * ase_batched_plan_wide: HOST arrays.  Instances with ncells >= min_cells
 * (min_cells <= 0: none) and, in the per-stage form, at least one full tile
 * are cut into tiles of that length (the last one ragged; in the per-step
 * form an instance shorter than a tile is one tile): tile j of instance k starts at
 * interior cell tile_i0[j]; tile_inst[j] = k; the tiles of k are
 * inst_tile0[k] .. inst_tile0[k] + inst_ntiles[k] - 1 (inst_tile0 -1 and
 * inst_ntiles 0 for the others).  The others are packed into nbins bins as
 * ase_batched_plan does (a bin may be empty).  *ntiles gets the tile count;
 * tile_inst and tile_i0 hold cap entries (ASE_ERR_ARG, with *ntiles set,
 * when cap < *ntiles; call with cap 0 and NULL arrays to count).
 * ase_batched_wide_workspace_bytes: device workspace for the call below.
 * ase_step_batched_wide: the arguments of ase_step_batched (bin_start and
 * bin_list: the wide plan's, which hold only the untiled instances) plus
 * device copies of the tile arrays, ntiles and threads_wide (as planned).  The call returns once both streams' work is queued; the
 * caller's stream waits for the second stream's before the final launch,
 * so work queued behind the call on `stream` sees every result.  The
 * library keeps one second stream (and two events) per device and caller
 * stream, created on first use and held until the process ends; calls on
 * different caller streams run concurrently. */
#define ASE_WIDE_STEP 0x10000

int ase_batched_plan_wide(int32_t ninst, const int32_t *ncells, int32_t min_cells, int32_t order,
                          int32_t threads_wide, int32_t nbins, int32_t *bin_start, int32_t *bin_list,
                          int32_t *tile_inst, int32_t *tile_i0, int32_t *inst_tile0, int32_t *inst_ntiles,
                          int32_t cap, int32_t *ntiles);

size_t ase_batched_wide_workspace_bytes(int64_t total, int32_t ninst, int32_t ntiles);

int ase_step_batched_wide(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                          const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng,
                          int64_t total, double *U, double *sigma, double *t, double *dt_hist,
                          const double *dt_replay, int32_t *status, int32_t nsteps, double t_end,
                          const int32_t *bin_start, const int32_t *bin_list, int32_t nbins, int32_t threads,
                          const int32_t *tile_inst, const int32_t *tile_i0, const int32_t *inst_tile0,
                          const int32_t *inst_ntiles, int32_t ntiles, int32_t threads_wide, void *ws,
                          size_t ws_bytes, void *stream);

/* ---- Allocation-free batched stepping --------------------------------------
 * For callers that cannot allocate device memory or hand in a workspace:
 * code under HIP graph capture, tight serving loops, hosts that forbid
 * hipMalloc.  ase_step_batched_noalloc is ase_step_batched with the same
 * arguments (minus ws, ws_bytes), the same kernels and the same results;
 * its workspace is a fixed device array of ASE_NOALLOC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends (located
 * on the first call on each device).  The call allocates and frees nothing.
 * A batch whose workspace, ase_batched_workspace_bytes(total), exceeds
 * ASE_NOALLOC_SCRATCH_BYTES (total > 1198368 stored cells) is refused with
 * ASE_ERR_WORKSPACE before anything is launched.  All calls on one GPU share
 * the array, which keeps the last call's contents (no call depends on
 * them: every scratch word is written before it is read): calls that can
 * overlap on the same GPU (other streams, other host threads) race, and
 * the caller must serialise them. */
#define ASE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

int ase_step_batched_noalloc(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                             const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng,
                             int64_t total, double *U, double *sigma, double *t, double *dt_hist,
                             const double *dt_replay, int32_t *status, int32_t nsteps, double t_end,
                             const int32_t *bin_start, const int32_t *bin_list, int32_t nbins, int32_t threads,
                             void *stream);

/* ---- Discrete adjoint of the 1D step ---------------------------------------
 * The paper defines the forward method only.  The adjoint here is the exact
 * transposed Jacobian of the discrete SSP-RK3 step (Sec. 2.1) with these
 * decisions frozen at their forward values: the time step, the DF strengths
 * every stage reads (hence each DF factor of Sec. 3.1 and each stencil level
 * of Algorithm 1), the side that gives the LF signal speed (Sec. 2.3) and the
 * positivity replacements.  Differentiated exactly: the reconstructions of
 * Sec. 3.2-3.4 (including the nonlinear WENO-Z-AO weights), the Euler and LF
 * fluxes, the stage combinations and the ghost copies of the boundary
 * conditions.  Boundaries: transmissive, periodic or reflective (both sides
 * alike; per instance in the batched form).  1D grids only. */

/* Device workspace of ase_adjoint_step on the 1D grid g. */
size_t ase_adjoint_workspace_bytes(const ase_grid_t *g);

/* lam_n = (dU_{n+1}/dU_n)^T lam_np1 for one step of a 1D grid.  U_n, sigma_n:
 * the state and DF strengths the step starts from (what ase_step holds before
 * it; layouts as ase_step, U [3][ld], sigma [ld]); dt: device scalar, the
 * step's time step (ase_step's dt_hist entry).  Only interior entries of
 * lam_np1 are read; ghost entries of lam_n are set to 0; lam_n may equal
 * lam_np1.  U_n and sigma_n are not modified.  The step is recomputed from
 * (U_n, sigma_n, dt) bit for bit as ase_step takes it.  One workgroup walks
 * the grid (batches of 1D grids go through ase_adjoint_batched).  Device
 * pointers; asynchronous on `stream`. */
int ase_adjoint_step(const ase_grid_t *g, const ase_params_t *p, const double *U_n, const double *sigma_n,
                     const double *dt, const double *lam_np1, double *lam_n, void *ws, size_t ws_bytes,
                     void *stream);

/* Device workspace of ase_adjoint_batched for `total` stored cells and a
 * segment of nsteps steps (a tape of 3 nsteps stage inputs). */
size_t ase_adjoint_batched_workspace_bytes(int64_t total, int32_t nsteps);

/* Phases of ase_adjoint_batched. */
enum { ASE_ADJ_TAPE = 1, ASE_ADJ_REVERSE = 2 };

/* Adjoint of nsteps batched steps (instance table, bc and bins as in
 * ase_step_batched; threads 128, 256 or 512).  U_ck, sigma_ck: state and DF
 * strengths at the segment start (a checkpoint of the forward run);
 * dt_hist: device [nsteps][ninst], the segment's recorded time steps (0 =
 * step not taken).  lam [3][total]: in, the adjoint at the segment end; out,
 * the adjoint at its start (ghost entries 0).  One persistent launch per
 * phase: with ASE_ADJ_TAPE each workgroup re-runs the segment forward for
 * its instances and keeps every stage input in the workspace (lam is not
 * touched); with ASE_ADJ_REVERSE it runs the steps back over the tape a
 * tape phase left in the same workspace for the same segment and
 * arguments; both bits do both in one launch.  A tape phase of one segment
 * (its own workspace) may run concurrently with the reverse phase of
 * another on a second stream.  Device pointers; asynchronous on `stream`. */
int ase_adjoint_batched(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                        const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng, int64_t total,
                        const double *U_ck,
                        const double *sigma_ck, const double *dt_hist, int32_t nsteps, double *lam,
                        const int32_t *bin_start, const int32_t *bin_list, int32_t nbins, int32_t threads,
                        int32_t phase, void *ws, size_t ws_bytes, void *stream);

/* ase_adjoint_batched with the instances of a wide plan
 * (ase_batched_plan_wide) split (first-order DF source): the binned
 * instances run in the persistent launch, each tiled instance as one launch
 * per step and forward stage over its tiles (tape phase) and one per step
 * and transposed stage (reverse phase; plus, for periodic and reflective
 * instances, a launch that adds the ghost gradients onto the cells the
 * ghosts copy), on the library's second stream for `stream` (as in
 * ase_step_batched_wide) beside the persistent launch.  Arguments as ase_adjoint_batched (bins: the wide plan's, which
 * hold only the untiled instances) plus device copies of tile_inst, tile_i0
 * and inst_ntiles, ntiles and threads_wide (256 or 512; it sets the tile
 * length threads_wide - order - 1 the plan was made for).  A reverse phase
 * needs the tape of a tape phase of this call with the same plan and
 * segment in the same workspace.  lam equals ase_adjoint_batched's bit for
 * bit.  Work queued behind the call on `stream` sees every result. */
int ase_adjoint_batched_wide(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                             const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng,
                             int64_t total, const double *U_ck, const double *sigma_ck, const double *dt_hist,
                             int32_t nsteps, double *lam, const int32_t *bin_start, const int32_t *bin_list,
                             int32_t nbins, int32_t threads, const int32_t *tile_inst, const int32_t *tile_i0,
                             const int32_t *inst_ntiles, int32_t ntiles, int32_t threads_wide, int32_t phase,
                             void *ws, size_t ws_bytes, void *stream);

/* Objective of the adjoint runs: J_k = dx_k sum_i p_i over the interior cells
 * of each instance (p from the Euler equation of state, Sec. 2.3), and the
 * weighted gradient lam = w_k dJ_k/dU = w_k dx_k (gamma-1) (u^2/2, -u, 1)
 * (ghost entries 0).  weights [ninst] may be NULL (all 1); J [ninst] and
 * lam [3][total] may each be NULL.  A single 1D grid is the table
 * {offset 0, nx, dx} with total = ld.  Device pointers; asynchronous. */
int ase_pressure_objective(const ase_params_t *p, int32_t ninst, const int64_t *offsets, const int32_t *ncells,
                           const double *dx, int32_t ng, int64_t total, const double *U, const double *weights,
                           double *J, double *lam, void *stream);

/* Per-kernel timing of ase_step, for benchmarks and profiling (not for
 * production runs).  While enabled, ase_step brackets every launch of its
 * reconstruction/flux/update kernels with HIP events on the call's stream
 * and of the persistent kernels of ase_step_batched and the adjoint entry
 * points (pool of 8192 launches;
 * further launches go unrecorded).
 * ase_profile_enable(1) clears and enables recording, (0) disables it.
 * ase_profile_read waits for the recorded events, then returns the summed
 * duration in milliseconds and the number of launches of one kernel class
 * (ASE_KCLASS_*); it does not clear the record. */
enum { ASE_KCLASS_SWEEP_X = 0, ASE_KCLASS_SWEEP_Y = 1, ASE_KCLASS_STAGE_1D = 2, ASE_KCLASS_BC = 3,
       ASE_KCLASS_CFL = 4, ASE_KCLASS_BATCHED = 5, ASE_KCLASS_ADJOINT = 6, ASE_KCLASS_GKS_1D = 7,
       ASE_KCLASS_GKS_2D_RECON = 8, ASE_KCLASS_GKS_2D_FLUX = 9, ASE_KCLASS_GKS_2D_UPDATE = 10,
       ASE_KCLASS_COUNT = 11 };
int ase_profile_enable(int on);
int ase_profile_read(int kernel_class, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* ASE_H */
