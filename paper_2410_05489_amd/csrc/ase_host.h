// Host-side internals of libase: argument validation, error reporting,
// workspace layout and the kernel launchers shared by the entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/ase.h"
#include "ase_device.h"

namespace ase {


// Thread-local error message; returns code.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);


struct Geo {
    int dim, nx, ny, ng, ld, NX, NY, nv;
    long long plane;   // NY * ld
    int R, G, oi;      // stencil half width, Gauss points, order index
};

int validate(const ase_grid_t *g, const ase_params_t *p, Geo *geo);
MethodConst method_const(const ase_params_t *p);

// Workspace layout for ase_step / ase_cfl_dt.
struct Workspace {
    double *U1, *U2, *Res;     // stage states and x-sweep residual
    double *sxa, *sya;         // ping-pong strengths
    double *scal;              // [0] dt, [1] skip flag
    double *part;              // per-block partial maxima
    int nparts;
};
size_t workspace_bytes(const Geo &geo);
int carve_workspace(const Geo &geo, void *ws, size_t bytes, Workspace *w);

// Launchers (asynchronous on `st`).
// Ghost cells at the stage time *t + ct * *dt (device scalars; t null: time
// 0, dt null: *t), which only the moving-shock side reads.
void launch_bc_fill(const ase_grid_t &g, const Geo &geo, const MethodConst &mc, double *U, double *sx, double *sy,
                    hipStream_t st, const double *t = nullptr, const double *dt = nullptr, double ct = 0.0);
// First-order DF source: ghost cells and every stored strength from the filled
// state in one launch; with `part`, also the signal-speed maxima of the
// time step, sigma_init_parts(geo) of them (for launch_cfl_final).
void launch_sigma_init(const ase_grid_t &g, const Geo &geo, const MethodConst &mc, double *U, double *sx,
                       double *sy, hipStream_t st, const double *t = nullptr, const double *dt = nullptr,
                       double ct = 0.0, double *part = nullptr);
// its tiles: 256 cells of the row in 1D, 32 x 8 stored cells in 2D
constexpr int kFoTX1 = 256, kFoTX2 = 32, kFoTY2 = 8;
inline int sigma_init_parts(const Geo &geo)
{
    if (geo.dim == 1) return (geo.NX + kFoTX1 - 1) / kFoTX1;
    return ((geo.NX + kFoTX2 - 1) / kFoTX2) * ((geo.NY + kFoTY2 - 1) / kFoTY2);
}
// per-block counts of non-physical interior cells into part[0..nparts)
void launch_nonphysical(const ase_grid_t &g, const Geo &geo, const MethodConst &mc, const double *U, double *part,
                        int nparts, hipStream_t st);
void launch_cfl(const ase_grid_t &g, const Geo &geo, const ase_params_t &p, const MethodConst &mc, const double *U,
                const double *t_in, double *t_out, double t_end, double *dt, double *skip, double *dt_hist,
                double *part, int nparts, hipStream_t st);
// the time step from nparts signal-speed maxima already in part
void launch_cfl_final(const ase_grid_t &g, const Geo &geo, const ase_params_t &p, const MethodConst &mc,
                      const double *t_in, double *t_out, double t_end, double *dt, double *skip, double *dt_hist,
                      const double *part, int nparts, hipStream_t st);

enum SweepMode { MODE_RECON = 0, MODE_FUSED_X = 1, MODE_FUSED_Y = 2, MODE_FUSED_1D = 3 };

struct SweepArgs {
    const double *U;       // stage input (ghosts filled)
    const double *sx, *sy; // strengths read by this stage
    double *sig_out;       // strengths written (flux faces of this direction)
    double *wl, *wr;       // MODE_RECON outputs
    int8_t *level;         // MODE_RECON optional output
    double *Res;           // x residual (FUSED_X writes, FUSED_Y reads)
    const double *Un;      // step start state (FUSED_Y / 1D)
    double *Uout;          // stage output (FUSED_Y / 1D)
    const double *dt;      // device dt
    const double *skip;    // device skip flag (nullptr: never skip)
    int stage;
    int nx, ny, ng, ld, NX, NY;
    long long plane;
    int nfaces;
    double inv_dx, inv_dy;
    MethodConst mc;
};

void launch_sweep(const Geo &geo, int dir, int mode, const SweepArgs &a, hipStream_t st);

void launch_df(const Geo &geo, const MethodConst &mc, int dir, const double *wl, const double *wr, double *sig,
               hipStream_t st);
void launch_flux(const Geo &geo, const MethodConst &mc, int dir, const double *wl, const double *wr, double *F,
                 hipStream_t st);
void launch_stage_update(const ase_grid_t &g, const Geo &geo, int stage, const double *dt, const double *Un,
                         const double *Us, const double *F, const double *Gf, double *Uout, hipStream_t st);

struct BatchLaunch {
    const long long *offsets;
    const int *ncells;
    const double *dx;
    double *U, *sig, *t, *dt_hist, *U1, *U2, *sig2;
    const double *dt_in;
    int *status;
    const int *bin_start, *bin_list;
    const int *bc_inst;
    const int *only;   // init: optional [ninst], only the instances with only[k] > 0
    long long total;
    int ninst, nbins, threads, R, ng, nsteps, bc, fo, init;
    double t_end, cfl, dt_cap;
    MethodConst mc;
};
void launch_batched(const BatchLaunch &bl, hipStream_t st);

// Wide form of the batched step (first-order DF source): stage 0 is the
// prep launch, stages 1-3 the stages of step `step`.
struct WideLaunch {
    const long long *offsets;
    const int *ncells;
    const double *dx;
    double *U, *U1, *U2, *t, *dt_hist;
    const double *dt_in;
    int *status;
    const int *bc_inst;
    const int *tile_inst, *tile_i0, *inst_tile0, *inst_ntiles;
    double *lam, *dt_cur;
    int *done;
    long long total;
    int ninst, ntiles, threads, R, ng, bc, step, stage, nsteps;
    int per_step;   // one launch per step (k_batched_wide_step) instead of per stage
    double t_end, cfl, dt_cap;
    MethodConst mc;
};
void launch_batched_wide(const WideLaunch &wl, hipStream_t st);
// Tile length of the wide form for `threads` lanes and half width R (one
// launch per stage: the window reaches R + 1 cells beyond the tile on each
// side; one launch per step: three times that).
inline int wide_tile_cells(int threads, int R) { return threads - 2 * R - 2; }
inline int wide_step_tile_cells(int threads, int R) { return threads - 6 * R - 6; }
// Address of this device's fixed scratch array (ASE_NOALLOC_SCRATCH_BYTES).
int noalloc_scratch(void **ptr);

struct AdjLaunch {
    const long long *offsets;   // nullptr: single instance (n1, dx1) at offset 0
    const int *ncells;
    const double *dx;
    int n1;
    double dx1;
    const double *ck_U, *ck_sig, *dt_hist;
    double *lam, *mu1, *mu2, *tapeU, *tapeS;
    const int *bin_start, *bin_list;   // nullptr: one workgroup per instance
    const int *bc_inst;
    long long total;
    int ninst, nbins, threads, R, ng, nsteps, bc, fo;
    int phase;   // ASE_ADJ_TAPE, ASE_ADJ_REVERSE or both
    MethodConst mc;
};
void launch_adjoint(const AdjLaunch &al, hipStream_t st);

// Reverse sweep of the wide instances (tiles of threads - 2R - 2 cells) over
// the tape the persistent tape phase left in the workspace.
struct AdjWideLaunch {
    const long long *offsets;
    const int *ncells;
    const double *dx, *dt_hist, *ck_U;
    double *lam, *mu1, *mu2, *tapeU, *tapeS;
    const int *bc_inst, *tile_inst, *tile_i0, *inst_ntiles;
    long long total;
    int ninst, ntiles, threads, R, ng, nsteps, bc;
    MethodConst mc;
};
void launch_adjoint_wide(const AdjWideLaunch &wl, hipStream_t st);
// Tape phase of the wide instances (forward stages into the tape slots).
void launch_tape_wide(const AdjWideLaunch &wl, hipStream_t st);

struct ObjLaunch {
    const long long *offsets;
    const int *ncells;
    const double *dx;
    int n1;
    double dx1;
    const double *U;
    const double *w;
    double *J, *lam;
    long long total;
    int ninst, ng;
    double gm1;
};
void launch_objective(const ObjLaunch &ol, hipStream_t st);

// Gas-kinetic solver (1D).
struct GksConst {
    double K;          // internal degrees of freedom, (3 - gamma)/(gamma - 1)
    double c1, c2;     // numerical collision time tau_n = c1 dt + c2 |dp|/(p_l + p_r) dt
    double tau;        // collision time outside the exponentials (0: Euler)
    double mu;         // > 0: viscous, tau = mu / p of the equilibrium state
};

struct Gks1DArgs {
    const double *U;       // stage input (ghosts filled)
    const double *sx;      // strengths read by this stage
    double *sig_out;       // strengths written at the flux faces
    const double *Un;      // step-start state (stage 2)
    double *Uout;          // stage output
    double *L0, *Lt0;      // L and L_t of the first stage (written by stage 1, read by stage 2)
    const double *dt, *skip;
    long long plane;
    int nx, ng, NX, stage;
    double inv_dx;
    MethodConst mc;
    GksConst gk;
};
void launch_gks1d(int R, int nx, const Gks1DArgs &a, hipStream_t st);

struct Gks2DArgs {
    const double *U;       // stage input (ghosts filled)
    const double *sx, *sy; // strengths read by this stage
    double *sig_out;       // strengths written at this direction's flux faces
    double *rec;           // [2 G 12][nfaces] face-point states and slopes
    double *F, *Ft;        // [4][nfaces] face flux and its time derivative
    const double *dt, *skip;
    long long plane, nfaces;
    int nx, ny, ng, ld, NX, NY;
    int bc[4];             // boundary codes (no-slip wall faces carry no mass or energy)
    double inv_dx, inv_dy;
    MethodConst mc;
    GksConst gk;
};
// recon: the face-point reconstruction of direction dir into rec; else the
// face fluxes from rec
void launch_gks2d(int R, int dir, bool recon, const Gks2DArgs &a, hipStream_t st);

struct Gks2DUpdate {
    const double *Fx, *Ftx, *Fy, *Fty;   // [4][nfx], [4][nfy]
    const double *U, *Un;
    double *Uout, *L0, *Lt0;
    const double *dt, *skip;
    long long plane, nfx, nfy;
    int nx, ny, ng, ld, stage;
    double inv_dx, inv_dy;
};
void launch_gks2d_update(const Gks2DUpdate &u, hipStream_t st);

constexpr int kGksPointThreads = 256;
struct GksPointArgs {
    const double *Wl, *Wlx, *Wr, *Wrx;   // [3][n]
    double *Fn, *Ft;                     // [3][n]
    int n;
    double dt, gm1;
    GksConst gk;
};
void launch_gks_points(const GksPointArgs &a, hipStream_t st);

}  // namespace ase
