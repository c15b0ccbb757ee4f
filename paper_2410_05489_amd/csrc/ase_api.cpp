// C ABI of libase: validation, error reporting, workspace layout and the
// orchestration of whole SSP-RK3 steps on device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ase.h"
#include "ase_device.h"
#include "ase_host.h"

namespace ase {

namespace {
thread_local std::string g_err;
constexpr size_t kAlign = 256;
constexpr int kMaxParts = 1024;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool misaligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) != 0; }
}  // namespace

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(ASE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int validate(const ase_grid_t *g, const ase_params_t *p, Geo *geo)
{
    if (!g || !p) return fail(ASE_ERR_ARG, "null grid or params");
    const int r = p->order;
    if (r != 3 && r != 5 && r != 7 && r != 9) return fail(ASE_ERR_ORDER, "order must be 3, 5, 7 or 9");
    if (g->dim != 1 && g->dim != 2) return fail(ASE_ERR_ARG, "dim must be 1 or 2");
    if (g->nx < 1 || g->ny < 1) return fail(ASE_ERR_ARG, "nx, ny must be >= 1");
    if (g->dim == 1 && g->ny != 1) return fail(ASE_ERR_ARG, "ny must be 1 in 1D");
    if (g->ng < (r + 1) / 2) return fail(ASE_ERR_GHOST, "ng must be >= (order+1)/2");
    if (g->ld < g->nx + 2 * g->ng) return fail(ASE_ERR_ARG, "ld must be >= nx + 2 ng");
    if (!(g->dx > 0.0) || (g->dim == 2 && !(g->dy > 0.0))) return fail(ASE_ERR_ARG, "dx, dy must be > 0");
    for (int k = 0; k < 4; ++k)
        if (g->bc[k] < 0 || g->bc[k] > ASE_BC_NOSLIP) return fail(ASE_ERR_ARG, "unknown boundary code");
    for (int k = 0; k < 4; ++k) {
        if (g->bc[k] == ASE_BC_WALL_INFLOW && !(k == 2 && g->dim == 2))
            return fail(ASE_ERR_ARG, "WALL_INFLOW is a 2D y-lo boundary only");
        if (g->bc[k] == ASE_BC_MOVING_SHOCK && !(k == 3 && g->dim == 2))
            return fail(ASE_ERR_ARG, "MOVING_SHOCK is a 2D y-hi boundary only");
    }
    if (g->dim == 2 && g->bc[2] == ASE_BC_WALL_INFLOW && g->ny < g->ng)
        return fail(ASE_ERR_ARG, "a y wall needs ny >= ng");
    if ((g->bc[0] == ASE_BC_PERIODIC) != (g->bc[1] == ASE_BC_PERIODIC))
        return fail(ASE_ERR_ARG, "periodic x boundaries must pair");
    if (g->dim == 2 && (g->bc[2] == ASE_BC_PERIODIC) != (g->bc[3] == ASE_BC_PERIODIC))
        return fail(ASE_ERR_ARG, "periodic y boundaries must pair");
    if (g->dim == 2 && (g->bc[2] == ASE_BC_INFLOW_SLOT || g->bc[3] == ASE_BC_INFLOW_SLOT))
        return fail(ASE_ERR_ARG, "inflow slot is an x boundary only");
    if ((g->bc[0] == ASE_BC_PERIODIC || g->bc[0] == ASE_BC_REFLECTIVE || g->bc[1] == ASE_BC_REFLECTIVE ||
         g->bc[0] == ASE_BC_NOSLIP || g->bc[1] == ASE_BC_NOSLIP) &&
        g->nx < g->ng)
        return fail(ASE_ERR_ARG, "periodic or reflective x needs nx >= ng");
    if (g->dim == 2 && (g->bc[2] == ASE_BC_REFLECTIVE || g->bc[3] == ASE_BC_REFLECTIVE ||
                        g->bc[2] == ASE_BC_NOSLIP || g->bc[3] == ASE_BC_NOSLIP) && g->ny < g->ng)
        return fail(ASE_ERR_ARG, "reflective y needs ny >= ng");
    if (g->dim == 2 && g->bc[2] == ASE_BC_PERIODIC && g->ny < g->ng)
        return fail(ASE_ERR_ARG, "periodic y needs ny >= ng");
    const long long NX = g->nx + 2LL * g->ng, NY = g->dim == 1 ? 1 : g->ny + 2LL * g->ng;
    if (NY * (long long)g->ld > (1LL << 31) - 1 || (long long)(g->nx + 1) * (g->ny + 1) > (1LL << 31) - 1)
        return fail(ASE_ERR_ARG, "grid too large");
    if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || !(p->sigma_thres > 0.0) || !(p->eps > 0.0) ||
        !(p->d_hi > 0.0 && p->d_hi < 1.0) || !(p->d_lo >= 0.0 && p->d_lo <= 1.0))
        return fail(ASE_ERR_ARG, "invalid method parameters");
    geo->dim = g->dim;
    geo->nx = g->nx;
    geo->ny = g->ny;
    geo->ng = g->ng;
    geo->ld = g->ld;
    geo->NX = (int)NX;
    geo->NY = (int)NY;
    geo->nv = g->dim == 1 ? 3 : 4;
    geo->plane = NY * g->ld;
    geo->R = (r - 1) / 2;
    geo->G = g->dim == 1 ? 1 : (r - 1) / 2;
    geo->oi = (r - 3) / 2;
    return ASE_OK;
}

MethodConst method_const(const ase_params_t *p)
{
    MethodConst m;
    m.gamma = p->gamma;
    m.gm1 = p->gamma - 1.0;
    m.thr = p->sigma_thres;
    m.eps = p->eps;
    m.d5 = p->d_hi;
    m.d3m = (1.0 - p->d_hi) * (1.0 - p->d_lo) / 2.0;
    m.d30 = (1.0 - p->d_hi) * p->d_lo;
    m.inv_d5 = 1.0 / m.d5;
    m.r3m = m.d3m / m.d5;
    m.r30 = m.d30 / m.d5;
    m.order = p->order;
    m.flags = p->flags;
    return m;
}

static int nparts_for(const Geo &geo)
{
    const long long n = (long long)geo.nx * (geo.dim == 1 ? 1 : geo.ny);
    long long b = (n + 255) / 256;
    if (b > kMaxParts) b = kMaxParts;
    return (int)(b < 1 ? 1 : b);
}

// signal-speed partials: those of k_cfl_partial or one per first-order fill tile
static size_t parts_capacity(const Geo &geo)
{
    const int n = sigma_init_parts(geo);
    return (size_t)(n > kMaxParts ? n : kMaxParts);
}

size_t workspace_bytes(const Geo &geo)
{
    const size_t state = align_up((size_t)geo.nv * (size_t)geo.plane * sizeof(double));
    const size_t plane = align_up((size_t)geo.plane * sizeof(double));
    return 3 * state + 2 * plane + align_up(4 * sizeof(double)) + align_up(parts_capacity(geo) * sizeof(double));
}

int carve_workspace(const Geo &geo, void *ws, size_t bytes, Workspace *w)
{
    if (!ws) return fail(ASE_ERR_WORKSPACE, "workspace is required");
    if (bytes < workspace_bytes(geo)) return fail(ASE_ERR_WORKSPACE, "workspace too small");
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(ASE_ERR_ALIGN, "workspace must be 256-byte aligned");
    char *c = static_cast<char *>(ws);
    const size_t state = align_up((size_t)geo.nv * (size_t)geo.plane * sizeof(double));
    const size_t plane = align_up((size_t)geo.plane * sizeof(double));
    w->U1 = reinterpret_cast<double *>(c); c += state;
    w->U2 = reinterpret_cast<double *>(c); c += state;
    w->Res = reinterpret_cast<double *>(c); c += state;
    w->sxa = reinterpret_cast<double *>(c); c += plane;
    w->sya = reinterpret_cast<double *>(c); c += plane;
    w->scal = reinterpret_cast<double *>(c); c += align_up(4 * sizeof(double));
    w->part = reinterpret_cast<double *>(c);
    w->nparts = nparts_for(geo);
    return ASE_OK;
}

static SweepArgs base_args(const ase_grid_t *g, const Geo &geo, const MethodConst &mc)
{
    SweepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = geo.nx; a.ny = geo.ny; a.ng = geo.ng; a.ld = geo.ld; a.NX = geo.NX; a.NY = geo.NY;
    a.plane = geo.plane;
    a.inv_dx = 1.0 / g->dx;
    a.inv_dy = geo.dim == 2 ? 1.0 / g->dy : 0.0;
    a.mc = mc;
    return a;
}

// ---- per-kernel event timing (benchmarks) ---------------------------------
namespace {
struct ProfRec {
    int cls;
    hipEvent_t a, b;
};
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<ProfRec> recs;
    size_t next = 0;
} g_prof;
constexpr size_t kProfPool = 16384;
}  // namespace

struct ProfScope {
    hipStream_t st;
    ProfRec rec;
    bool active = false;
    ProfScope(int cls, hipStream_t s) : st(s)
    {
        if (!g_prof.on) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (g_prof.next + 2 > g_prof.pool.size()) return;
        rec.cls = cls;
        rec.a = g_prof.pool[g_prof.next++];
        rec.b = g_prof.pool[g_prof.next++];
        active = hipEventRecord(rec.a, st) == hipSuccess;
    }
    ~ProfScope()
    {
        if (!active) return;
        if (hipEventRecord(rec.b, st) == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_prof.mu);
            g_prof.recs.push_back(rec);
        }
    }
};

static int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return ASE_OK;
}

}  // namespace ase

using namespace ase;

#define ASE_PTR(p, name)                                                        \
    do {                                                                        \
        if (!(p)) return fail(ASE_ERR_ARG, std::string("null pointer: ") + name); \
        if (misaligned(p)) return fail(ASE_ERR_ALIGN, std::string("misaligned: ") + name); \
    } while (0)

extern "C" {

const char *ase_last_error(void) { return g_err.c_str(); }

int ase_version(void) { return 4; }

int ase_bc_fill(const ase_grid_t *g, const ase_params_t *p, double *U, double *sx, double *sy, void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    ASE_PTR(U, "U");
    ASE_PTR(sx, "sx");
    if (geo.dim == 2) ASE_PTR(sy, "sy");
    if (p->flags & ASE_FLAG_DF_FIRST_ORDER)
        launch_sigma_init(*g, geo, method_const(p), U, sx, geo.dim == 2 ? sy : sx, (hipStream_t)stream);
    else
        launch_bc_fill(*g, geo, method_const(p), U, sx, geo.dim == 2 ? sy : sx, (hipStream_t)stream);
    return check_launch("ase_bc_fill");
}

int ase_sigma_init(const ase_grid_t *g, const ase_params_t *p, double *U, double *sx, double *sy, void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    ASE_PTR(U, "U");
    ASE_PTR(sx, "sx");
    if (geo.dim == 2) ASE_PTR(sy, "sy");
    launch_sigma_init(*g, geo, method_const(p), U, sx, geo.dim == 2 ? sy : sx, (hipStream_t)stream);
    return check_launch("ase_sigma_init");
}

size_t ase_workspace_bytes(const ase_grid_t *g, const ase_params_t *p)
{
    Geo geo;
    if (validate(g, p, &geo)) return 0;
    return workspace_bytes(geo);
}

int ase_cfl_dt(const ase_grid_t *g, const ase_params_t *p, const double *U, const double *t, double t_end,
               double *dt, void *ws, size_t ws_bytes, void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    ASE_PTR(U, "U");
    ASE_PTR(t, "t");
    ASE_PTR(dt, "dt");
    Workspace w;
    rc = carve_workspace(geo, ws, ws_bytes, &w);
    if (rc) return rc;
    launch_cfl(*g, geo, *p, method_const(p), U, t, nullptr, t_end, dt, nullptr, nullptr, w.part, w.nparts,
               (hipStream_t)stream);
    return check_launch("ase_cfl_dt");
}

int ase_reconstruct(const ase_grid_t *g, const ase_params_t *p, int dir, const double *U, const double *sx,
                    const double *sy, double *wl, double *wr, int8_t *level, void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    if (dir != 0 && !(dir == 1 && geo.dim == 2)) return fail(ASE_ERR_ARG, "dir must be 0 (or 1 in 2D)");
    ASE_PTR(U, "U");
    ASE_PTR(sx, "sx");
    if (geo.dim == 2) ASE_PTR(sy, "sy");
    ASE_PTR(wl, "wl");
    ASE_PTR(wr, "wr");
    SweepArgs a = base_args(g, geo, method_const(p));
    a.U = U;
    a.sx = sx;
    a.sy = geo.dim == 2 ? sy : sx;
    a.wl = wl;
    a.wr = wr;
    a.level = level;
    a.nfaces = geo.dim == 1 ? geo.nx + 1 : (dir == 0 ? (geo.nx + 1) * geo.ny : geo.nx * (geo.ny + 1));
    launch_sweep(geo, dir, MODE_RECON, a, (hipStream_t)stream);
    return check_launch("ase_reconstruct");
}

int ase_df_compute(const ase_grid_t *g, const ase_params_t *p, int dir, const double *wl, const double *wr,
                   double *sigma, void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    if (dir != 0 && !(dir == 1 && geo.dim == 2)) return fail(ASE_ERR_ARG, "dir must be 0 (or 1 in 2D)");
    ASE_PTR(wl, "wl");
    ASE_PTR(wr, "wr");
    ASE_PTR(sigma, "sigma");
    launch_df(geo, method_const(p), dir, wl, wr, sigma, (hipStream_t)stream);
    return check_launch("ase_df_compute");
}

int ase_flux(const ase_grid_t *g, const ase_params_t *p, int dir, const double *wl, const double *wr, double *F,
             void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    if (dir != 0 && !(dir == 1 && geo.dim == 2)) return fail(ASE_ERR_ARG, "dir must be 0 (or 1 in 2D)");
    ASE_PTR(wl, "wl");
    ASE_PTR(wr, "wr");
    ASE_PTR(F, "F");
    launch_flux(geo, method_const(p), dir, wl, wr, F, (hipStream_t)stream);
    return check_launch("ase_flux");
}

int ase_stage_update(const ase_grid_t *g, const ase_params_t *p, int stage, const double *dt, const double *Un,
                     const double *Us, const double *F, const double *G, double *Uout, void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    if (stage < 1 || stage > 3) return fail(ASE_ERR_ARG, "stage must be 1, 2 or 3");
    ASE_PTR(dt, "dt");
    ASE_PTR(Un, "Un");
    ASE_PTR(Us, "Us");
    ASE_PTR(F, "F");
    if (geo.dim == 2) ASE_PTR(G, "G");
    ASE_PTR(Uout, "Uout");
    launch_stage_update(*g, geo, stage, dt, Un, Us, F, geo.dim == 2 ? G : F, Uout, (hipStream_t)stream);
    return check_launch("ase_stage_update");
}

// ASE_FLAG_FAIL_NONPHYSICAL: refuse graph capture before any launch ...
static int nonphysical_capturable(const ase_params_t *p, hipStream_t st)
{
    if (!(p->flags & ASE_FLAG_FAIL_NONPHYSICAL)) return ASE_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(ASE_ERR_ARG, "ASE_FLAG_FAIL_NONPHYSICAL synchronises the stream and cannot be captured");
    return ASE_OK;
}

// ... and after the last step count the non-physical interior cells.
static int nonphysical_check(const ase_grid_t *g, const Geo &geo, const ase_params_t *p, const double *U,
                             const Workspace &w, hipStream_t st, const char *who)
{
    if (!(p->flags & ASE_FLAG_FAIL_NONPHYSICAL)) return ASE_OK;
    launch_nonphysical(*g, geo, method_const(p), U, w.part, w.nparts, st);
    int rc = check_launch(who);
    if (rc) return rc;
    std::vector<double> part((size_t)w.nparts);
    hipError_t e = hipMemcpyAsync(part.data(), w.part, part.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(non-physical count)");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    double n = 0.0;
    for (double c : part) n += c;
    if (n > 0.0)
        return fail(ASE_ERR_NONPHYSICAL, std::string(who) + ": " + std::to_string((long long)n) +
                                             " interior cells with rho <= 0, p <= 0 or NaN");
    return ASE_OK;
}

int ase_step(const ase_grid_t *g, const ase_params_t *p, double *U, double *sx, double *sy, double *t,
             double *dt_hist, int32_t nsteps, double t_end, void *ws, size_t ws_bytes, void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    if (nsteps < 0) return fail(ASE_ERR_ARG, "nsteps must be >= 0");
    ASE_PTR(U, "U");
    ASE_PTR(sx, "sx");
    if (geo.dim == 2) ASE_PTR(sy, "sy");
    ASE_PTR(t, "t");
    if (dt_hist && misaligned(dt_hist)) return fail(ASE_ERR_ALIGN, "misaligned: dt_hist");
    Workspace w;
    rc = carve_workspace(geo, ws, ws_bytes, &w);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    rc = nonphysical_capturable(p, st);
    if (rc) return rc;
    const MethodConst mc = method_const(p);
    SweepArgs a = base_args(g, geo, mc);
    a.dt = w.scal;
    a.skip = w.scal + 1;
    a.Res = w.Res;
    a.Un = U;

    // Ghost cells and the strengths the stage reads (lagged or first order).
    const bool fo = (p->flags & ASE_FLAG_DF_FIRST_ORDER) != 0;
    // stage inputs at t_n, t_n + dt, t_n + dt/2; after the dt kernel *t
    // holds t_n + dt, so the times are *t (first fill: before it), *t and
    // *t - dt/2
    // With the first-order source the fill of a step's first stage input also
    // leaves the signal-speed maxima of the time step in w.part.
    auto stage_bc = [&](double *Us, double *sxs_, double *sys_, double ct, double *part = nullptr) {
        // (dt is read only with a nonzero ct: before the first dt kernel it is unset)
        const double *dtp = ct != 0.0 ? w.scal : nullptr;
        if (fo) launch_sigma_init(*g, geo, mc, Us, sxs_, sys_, st, t, dtp, ct, part);
        else launch_bc_fill(*g, geo, mc, Us, sxs_, sys_, st, t, dtp, ct);
    };
    auto step_dt = [&](int s) {
        double *dth = dt_hist ? dt_hist + s : nullptr;
        if (fo)
            launch_cfl_final(*g, geo, *p, mc, t, t, t_end, w.scal, w.scal + 1, dth, w.part, sigma_init_parts(geo), st);
        else
            launch_cfl(*g, geo, *p, mc, U, t, t, t_end, w.scal, w.scal + 1, dth, w.part, w.nparts, st);
    };
    double *sxs[2] = {sx, w.sxa};
    double *sys[2] = {geo.dim == 2 ? sy : sx, w.sya};
    int cur = 0;
    for (int s = 0; s < nsteps; ++s) {
        double *sxc = sxs[cur], *syc = sys[cur], *sxn = sxs[cur ^ 1], *syn = sys[cur ^ 1];
        {
            ProfScope ps(ASE_KCLASS_BC, st);
            stage_bc(U, sxc, syc, 0.0, w.part);
        }
        {
            ProfScope ps(ASE_KCLASS_CFL, st);
            step_dt(s);
        }
        double *in_st[3] = {U, w.U1, w.U2};
        double *out_st[3] = {w.U1, w.U2, U};
        double *sx_in[3] = {sxc, sxn, sxc}, *sy_in[3] = {syc, syn, syc};
        double *sx_out[3] = {sxn, sxc, sxn}, *sy_out[3] = {syn, syc, syn};
        for (int k = 0; k < 3; ++k) {
            if (k > 0) {
                ProfScope ps(ASE_KCLASS_BC, st);
                stage_bc(in_st[k], sx_in[k], sy_in[k], k == 1 ? 0.0 : -0.5);
            }
            a.U = in_st[k];
            a.sx = sx_in[k];
            a.sy = sy_in[k];
            a.stage = k + 1;
            a.Uout = out_st[k];
            if (geo.dim == 1) {
                a.sig_out = sx_out[k];
                ProfScope ps(ASE_KCLASS_STAGE_1D, st);
                launch_sweep(geo, 0, MODE_FUSED_1D, a, st);
            } else {
                a.sig_out = sx_out[k];
                {
                    ProfScope ps(ASE_KCLASS_SWEEP_X, st);
                    launch_sweep(geo, 0, MODE_FUSED_X, a, st);
                }
                a.sig_out = sy_out[k];
                {
                    ProfScope ps(ASE_KCLASS_SWEEP_Y, st);
                    launch_sweep(geo, 1, MODE_FUSED_Y, a, st);
                }
            }
        }
        cur ^= 1;
    }
    if (fo) {
        // first-order source: hand back the strengths of the final state
        // (the sweeps write none in this mode)
        if (nsteps > 0) {
            ProfScope ps(ASE_KCLASS_BC, st);
            stage_bc(U, sx, geo.dim == 2 ? sy : sx, 0.0);
        }
    } else if (cur == 1) {
        hipError_t e = hipMemcpyAsync(sx, w.sxa, (size_t)geo.plane * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(sx)");
        if (geo.dim == 2) {
            e = hipMemcpyAsync(sy, w.sya, (size_t)geo.plane * sizeof(double), hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(sy)");
        }
    }
    rc = check_launch("ase_step");
    if (rc) return rc;
    return nonphysical_check(g, geo, p, U, w, st, "ase_step");
}

static GksConst gks_const(const ase_params_t *p, const ase_gks_t *gk, int dim)
{
    GksConst c;
    // internal degrees of freedom: 1D (3 - gamma)/(gamma - 1), 2D (4 - 2 gamma)/(gamma - 1)
    c.K = dim == 1 ? (3.0 - p->gamma) / (p->gamma - 1.0) : (4.0 - 2.0 * p->gamma) / (p->gamma - 1.0);
    c.c1 = gk->c1;
    c.c2 = gk->c2;
    c.tau = gk->tau;
    c.mu = gk->mu;
    return c;
}

static int check_gks(const ase_gks_t *gk)
{
    if (!gk) return fail(ASE_ERR_ARG, "null gks parameters");
    if (!(gk->c1 >= 0.0) || !(gk->c2 >= 0.0) || !(gk->tau >= 0.0) || !(gk->mu >= 0.0))
        return fail(ASE_ERR_ARG, "gks c1, c2, tau, mu must be >= 0");
    return ASE_OK;
}

// 2D extras behind the LF workspace: face-point states [2 G 12][nf_max],
// fluxes Fx, Ftx [4][nfx], Fy, Fty [4][nfy].
struct GksWs2D {
    double *rec, *Fx, *Ftx, *Fy, *Fty;
    long long nfx, nfy;
};

static size_t gks_extra_bytes(const Geo &geo)
{
    if (geo.dim == 1) return 0;
    const long long nfx = (long long)(geo.nx + 1) * geo.ny, nfy = (long long)geo.nx * (geo.ny + 1);
    const long long nfm = nfx > nfy ? nfx : nfy;
    return align_up((size_t)(2 * geo.G * 12) * nfm * sizeof(double)) + 2 * align_up((size_t)4 * nfx * sizeof(double)) +
           2 * align_up((size_t)4 * nfy * sizeof(double));
}

static void carve_gks2d(const Geo &geo, void *ws, GksWs2D *w)
{
    char *c = static_cast<char *>(ws) + workspace_bytes(geo);
    w->nfx = (long long)(geo.nx + 1) * geo.ny;
    w->nfy = (long long)geo.nx * (geo.ny + 1);
    const long long nfm = w->nfx > w->nfy ? w->nfx : w->nfy;
    w->rec = reinterpret_cast<double *>(c); c += align_up((size_t)(2 * geo.G * 12) * nfm * sizeof(double));
    w->Fx = reinterpret_cast<double *>(c); c += align_up((size_t)4 * w->nfx * sizeof(double));
    w->Ftx = reinterpret_cast<double *>(c); c += align_up((size_t)4 * w->nfx * sizeof(double));
    w->Fy = reinterpret_cast<double *>(c); c += align_up((size_t)4 * w->nfy * sizeof(double));
    w->Fty = reinterpret_cast<double *>(c);
}

size_t ase_gks_workspace_bytes(const ase_grid_t *g, const ase_params_t *p)
{
    Geo geo;
    if (validate(g, p, &geo)) return 0;
    return workspace_bytes(geo) + gks_extra_bytes(geo);
}

int ase_gks_flux(const ase_params_t *p, const ase_gks_t *gk, int32_t n, const double *Wl, const double *Wlx,
                 const double *Wr, const double *Wrx, double dt, double *Fn, double *Ft, void *stream)
{
    if (!p) return fail(ASE_ERR_ARG, "null params");
    int rc = check_gks(gk);
    if (rc) return rc;
    if (gk->mu > 0.0) return fail(ASE_ERR_ARG, "viscous flow (mu > 0) needs a 2D grid");
    if (!(p->gamma > 1.0)) return fail(ASE_ERR_ARG, "gamma must be > 1");
    if (n < 0) return fail(ASE_ERR_ARG, "n must be >= 0");
    if (!(dt > 0.0)) return fail(ASE_ERR_ARG, "dt must be > 0");
    if (n == 0) return ASE_OK;
    ASE_PTR(Wl, "Wl");
    ASE_PTR(Wlx, "Wlx");
    ASE_PTR(Wr, "Wr");
    ASE_PTR(Wrx, "Wrx");
    ASE_PTR(Fn, "Fn");
    ASE_PTR(Ft, "Ft");
    GksPointArgs a;
    a.Wl = Wl;
    a.Wlx = Wlx;
    a.Wr = Wr;
    a.Wrx = Wrx;
    a.Fn = Fn;
    a.Ft = Ft;
    a.n = n;
    a.dt = dt;
    a.gm1 = p->gamma - 1.0;
    a.gk = gks_const(p, gk, 1);
    launch_gks_points(a, (hipStream_t)stream);
    return check_launch("ase_gks_flux");
}

int ase_step_gks(const ase_grid_t *g, const ase_params_t *p, const ase_gks_t *gk, double *U, double *sx,
                 double *sy, double *t, double *dt_hist, int32_t nsteps, double t_end, void *ws, size_t ws_bytes,
                 void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    rc = check_gks(gk);
    if (rc) return rc;
    if (geo.dim == 1 && gk->mu > 0.0) return fail(ASE_ERR_ARG, "viscous flow (mu > 0) needs a 2D grid");
    if (nsteps < 0) return fail(ASE_ERR_ARG, "nsteps must be >= 0");
    ASE_PTR(U, "U");
    ASE_PTR(sx, "sx");
    if (geo.dim == 2) ASE_PTR(sy, "sy");
    ASE_PTR(t, "t");
    if (dt_hist && misaligned(dt_hist)) return fail(ASE_ERR_ALIGN, "misaligned: dt_hist");
    if (ws_bytes < workspace_bytes(geo) + gks_extra_bytes(geo))
        return fail(ASE_ERR_WORKSPACE, "workspace too small (ase_gks_workspace_bytes)");
    Workspace w;
    rc = carve_workspace(geo, ws, ws_bytes, &w);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    rc = nonphysical_capturable(p, st);
    if (rc) return rc;
    const MethodConst mc = method_const(p);
    const GksConst gc = gks_const(p, gk, geo.dim);
    const bool fo = (p->flags & ASE_FLAG_DF_FIRST_ORDER) != 0;
    double *syv = geo.dim == 2 ? sy : sx;    // 1D: the y-strength argument is unused
    double *syav = geo.dim == 2 ? w.sya : w.sxa;
    // stage inputs at t_n (before the dt kernel) and t_n + dt/2 = *t - dt/2
    auto stage_bc = [&](double *Us, double *sxs, double *sys, double ct, double *part = nullptr) {
        // (dt is read only with a nonzero ct: before the first dt kernel it is unset)
        const double *dtp = ct != 0.0 ? w.scal : nullptr;
        if (fo) launch_sigma_init(*g, geo, mc, Us, sxs, sys, st, t, dtp, ct, part);
        else launch_bc_fill(*g, geo, mc, Us, sxs, sys, st, t, dtp, ct);
    };
    // workspace: W* in U1, L(W^n) in U2, L_t(W^n) in Res, stage-1 strengths in sxa / sya
    Gks1DArgs a1;
    Gks2DArgs a2;
    Gks2DUpdate up;
    GksWs2D w2;
    if (geo.dim == 1) {
        a1.dt = w.scal;
        a1.skip = w.scal + 1;
        a1.plane = geo.plane;
        a1.nx = geo.nx;
        a1.ng = geo.ng;
        a1.NX = geo.NX;
        a1.inv_dx = 1.0 / g->dx;
        a1.mc = mc;
        a1.gk = gc;
        a1.L0 = w.U2;
        a1.Lt0 = w.Res;
    } else {
        carve_gks2d(geo, ws, &w2);
        a2.dt = w.scal;
        a2.skip = w.scal + 1;
        a2.plane = geo.plane;
        a2.nx = geo.nx;
        a2.ny = geo.ny;
        a2.ng = geo.ng;
        a2.ld = geo.ld;
        a2.NX = geo.NX;
        a2.NY = geo.NY;
        a2.inv_dx = 1.0 / g->dx;
        a2.inv_dy = 1.0 / g->dy;
        for (int k = 0; k < 4; ++k) a2.bc[k] = g->bc[k];
        a2.mc = mc;
        a2.gk = gc;
        a2.rec = w2.rec;
        up.Fx = w2.Fx;
        up.Ftx = w2.Ftx;
        up.Fy = w2.Fy;
        up.Fty = w2.Fty;
        up.dt = w.scal;
        up.skip = w.scal + 1;
        up.plane = geo.plane;
        up.nfx = w2.nfx;
        up.nfy = w2.nfy;
        up.nx = geo.nx;
        up.ny = geo.ny;
        up.ng = geo.ng;
        up.ld = geo.ld;
        up.inv_dx = 1.0 / g->dx;
        up.inv_dy = 1.0 / g->dy;
        up.L0 = w.U2;
        up.Lt0 = w.Res;
    }
    // one stage: stage 1 from U (strengths sx, sy) into W*, stage 2 from W*
    // (strengths sxa, sya) into U
    auto stage = [&](int k) {
        double *Uin = k == 1 ? U : w.U1;
        double *sxi = k == 1 ? sx : w.sxa, *syi = k == 1 ? syv : syav;
        double *sxo = k == 1 ? w.sxa : sx, *syo = k == 1 ? syav : syv;
        double *Uo = k == 1 ? w.U1 : U;
        if (geo.dim == 1) {
            a1.stage = k;
            a1.U = Uin;
            a1.sx = sxi;
            a1.sig_out = sxo;
            a1.Un = U;
            a1.Uout = Uo;
            ProfScope ps(ASE_KCLASS_GKS_1D, st);
            launch_gks1d(geo.R, geo.nx, a1, st);
            return;
        }
        a2.U = Uin;
        a2.sx = sxi;
        a2.sy = syi;
        for (int dir = 0; dir < 2; ++dir) {
            a2.sig_out = dir == 0 ? sxo : syo;
            a2.F = dir == 0 ? w2.Fx : w2.Fy;
            a2.Ft = dir == 0 ? w2.Ftx : w2.Fty;
            a2.nfaces = dir == 0 ? w2.nfx : w2.nfy;
            {
                ProfScope ps(ASE_KCLASS_GKS_2D_RECON, st);
                launch_gks2d(geo.R, dir, true, a2, st);
            }
            {
                ProfScope ps(ASE_KCLASS_GKS_2D_FLUX, st);
                launch_gks2d(geo.R, dir, false, a2, st);
            }
        }
        up.stage = k;
        up.U = Uin;
        up.Un = U;
        up.Uout = Uo;
        ProfScope ps(ASE_KCLASS_GKS_2D_UPDATE, st);
        launch_gks2d_update(up, st);
    };
    for (int s = 0; s < nsteps; ++s) {
        {
            ProfScope ps(ASE_KCLASS_BC, st);
            stage_bc(U, sx, syv, 0.0, w.part);
        }
        {
            ProfScope ps(ASE_KCLASS_CFL, st);
            double *dth = dt_hist ? dt_hist + s : nullptr;
            if (fo)
                launch_cfl_final(*g, geo, *p, mc, t, t, t_end, w.scal, w.scal + 1, dth, w.part,
                                 sigma_init_parts(geo), st);
            else
                launch_cfl(*g, geo, *p, mc, U, t, t, t_end, w.scal, w.scal + 1, dth, w.part, w.nparts, st);
        }
        stage(1);
        {
            ProfScope ps(ASE_KCLASS_BC, st);
            stage_bc(w.U1, w.sxa, syav, -0.5);
        }
        stage(2);
    }
    rc = check_launch("ase_step_gks");
    if (rc) return rc;
    return nonphysical_check(g, geo, p, U, w, st, "ase_step_gks");
}

// Longest processing time first: the instances `ks`, longest first, each onto
// the least-loaded of nbins bins.
static void lpt_bins(const std::vector<int> &ks, const int32_t *ncells, int32_t nbins, int32_t *bin_start,
                     int32_t *bin_list)
{
    std::vector<int> order(ks);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ncells[a] > ncells[b]; });
    std::vector<long long> load(nbins, 0);
    std::vector<std::vector<int>> bins(nbins);
    for (int k : order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        bins[b].push_back(k);
        load[b] += ncells[k] > 0 ? ncells[k] : 0;
    }
    int pos = 0;
    for (int b = 0; b < nbins; ++b) {
        bin_start[b] = pos;
        for (int k : bins[b]) bin_list[pos++] = k;
    }
    bin_start[nbins] = pos;
}

int ase_batched_plan(int32_t ninst, const int32_t *ncells, int32_t nbins, int32_t *bin_start, int32_t *bin_list)
{
    if (ninst < 1 || nbins < 1 || !ncells || !bin_start || !bin_list)
        return fail(ASE_ERR_ARG, "ase_batched_plan: bad arguments");
    std::vector<int> all(ninst);
    std::iota(all.begin(), all.end(), 0);
    lpt_bins(all, ncells, nbins, bin_start, bin_list);
    return ASE_OK;
}

int ase_batched_plan_wide(int32_t ninst, const int32_t *ncells, int32_t min_cells, int32_t order,
                          int32_t threads_wide, int32_t nbins, int32_t *bin_start, int32_t *bin_list,
                          int32_t *tile_inst, int32_t *tile_i0, int32_t *inst_tile0, int32_t *inst_ntiles,
                          int32_t cap, int32_t *ntiles)
{
    if (ninst < 1 || nbins < 1 || !ncells || !bin_start || !bin_list || !inst_tile0 || !inst_ntiles || !ntiles ||
        cap < 0 || (cap > 0 && (!tile_inst || !tile_i0)))
        return fail(ASE_ERR_ARG, "ase_batched_plan_wide: bad arguments");
    if (order != 3 && order != 5 && order != 7 && order != 9) return fail(ASE_ERR_ORDER, "order must be 3, 5, 7 or 9");
    const int nt_lanes = threads_wide & ~ASE_WIDE_STEP;
    if ((nt_lanes != 256 && nt_lanes != 512) || (threads_wide & ~(ASE_WIDE_STEP | 0x3ff)))
        return fail(ASE_ERR_ARG, "threads_wide must be 256 or 512, optionally with ASE_WIDE_STEP");
    const int T = (threads_wide & ASE_WIDE_STEP) ? wide_step_tile_cells(nt_lanes, (order - 1) / 2)
                                                 : wide_tile_cells(nt_lanes, (order - 1) / 2);
    // an instance takes the per-stage wide form from one full tile up, the
    // per-step form at any length
    const int tmin = (threads_wide & ASE_WIDE_STEP) ? 1 : T;
    auto wide = [&](int k) { return min_cells > 0 && ncells[k] >= min_cells && ncells[k] >= tmin; };
    std::vector<int> small;
    long long nt = 0;
    for (int k = 0; k < ninst; ++k) {
        if (wide(k)) nt += (ncells[k] + T - 1) / T;
        else small.push_back(k);
    }
    if (nt > INT32_MAX) return fail(ASE_ERR_ARG, "ase_batched_plan_wide: too many tiles");
    *ntiles = (int32_t)nt;
    if (nt > cap) return fail(ASE_ERR_ARG, "ase_batched_plan_wide: tile arrays smaller than *ntiles");
    int pos = 0;
    for (int k = 0; k < ninst; ++k) {
        if (wide(k)) {
            const int n = (ncells[k] + T - 1) / T;
            inst_tile0[k] = pos;
            inst_ntiles[k] = n;
            for (int j = 0; j < n; ++j) {
                tile_inst[pos] = k;
                tile_i0[pos] = j * T;
                ++pos;
            }
        } else {
            inst_tile0[k] = -1;
            inst_ntiles[k] = 0;
        }
    }
    lpt_bins(small, ncells, nbins, bin_start, bin_list);
    return ASE_OK;
}

size_t ase_batched_wide_workspace_bytes(int64_t total, int32_t ninst, int32_t ntiles)
{
    if (total < 1 || ninst < 1 || ntiles < 0) return 0;
    return ase_batched_workspace_bytes(total) + align_up((size_t)(ntiles > 0 ? ntiles : 1) * 2 * sizeof(double)) +
           align_up((size_t)ninst * sizeof(double)) + align_up((size_t)ninst * sizeof(int));
}

size_t ase_batched_workspace_bytes(int64_t total)
{
    if (total < 1) return 0;
    return 7 * align_up((size_t)total * sizeof(double));
}

static int batched_common(const ase_params_t *p, int32_t bc, int32_t ninst, const int64_t *offsets,
                          const int32_t *ncells, int32_t ng, int64_t total, double *U, double *sigma)
{
    if (!p) return fail(ASE_ERR_ARG, "null params");
    const int r = p->order;
    if (r != 3 && r != 5 && r != 7 && r != 9) return fail(ASE_ERR_ORDER, "order must be 3, 5, 7 or 9");
    if (ng < (r + 1) / 2) return fail(ASE_ERR_GHOST, "ng must be >= (order+1)/2");
    if (bc != ASE_BC_PERIODIC && bc != ASE_BC_TRANSMISSIVE && bc != ASE_BC_REFLECTIVE)
        return fail(ASE_ERR_ARG, "bc must be periodic, transmissive or reflective");
    if (ninst < 1 || total < 1) return fail(ASE_ERR_ARG, "ninst and total must be >= 1");
    if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || !(p->sigma_thres > 0.0) || !(p->eps > 0.0) ||
        !(p->d_hi > 0.0 && p->d_hi < 1.0) || !(p->d_lo >= 0.0 && p->d_lo <= 1.0))
        return fail(ASE_ERR_ARG, "invalid method parameters");
    ASE_PTR(offsets, "offsets");
    ASE_PTR(ncells, "ncells");
    ASE_PTR(U, "U");
    ASE_PTR(sigma, "sigma");
    return ASE_OK;
}

int ase_batched_sigma_init(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                           const int64_t *offsets, const int32_t *ncells, int32_t ng, int64_t total, double *U,
                           double *sigma, void *stream)
{
    int rc = batched_common(p, bc, ninst, offsets, ncells, ng, total, U, sigma);
    if (rc) return rc;
    BatchLaunch bl;
    std::memset(&bl, 0, sizeof(bl));
    bl.offsets = reinterpret_cast<const long long *>(offsets);
    bl.ncells = ncells;
    bl.U = U;
    bl.sig = sigma;
    bl.total = total;
    bl.ninst = ninst;
    bl.ng = ng;
    bl.bc = bc;
    bl.bc_inst = bc_inst;
    bl.init = 1;
    bl.mc = method_const(p);
    launch_batched(bl, (hipStream_t)stream);
    return check_launch("ase_batched_sigma_init");
}

// Validation of ase_step_batched's arguments and its persistent launch.
static int batched_setup(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                         const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng, int64_t total,
                         double *U, double *sigma, double *t, double *dt_hist, const double *dt_replay,
                         int32_t *status, int32_t nsteps, double t_end, const int32_t *bin_start,
                         const int32_t *bin_list, int32_t nbins, int32_t threads, void *ws, size_t ws_bytes,
                         size_t ws_need, BatchLaunch *bl)
{
    int rc = batched_common(p, bc, ninst, offsets, ncells, ng, total, U, sigma);
    if (rc) return rc;
    if (nsteps < 0) return fail(ASE_ERR_ARG, "nsteps must be >= 0");
    if (nbins < 1) return fail(ASE_ERR_ARG, "nbins must be >= 1");
    if (threads != 256 && threads != 512 && threads != 1024)
        return fail(ASE_ERR_ARG, "threads must be 256, 512 or 1024");
    ASE_PTR(dx, "dx");
    ASE_PTR(t, "t");
    if (dt_hist && misaligned(dt_hist)) return fail(ASE_ERR_ALIGN, "misaligned: dt_hist");
    if (dt_replay && misaligned(dt_replay)) return fail(ASE_ERR_ALIGN, "misaligned: dt_replay");
    if (status && (reinterpret_cast<uintptr_t>(status) & 3u) != 0) return fail(ASE_ERR_ALIGN, "misaligned: status");
    if (!bin_start || !bin_list) return fail(ASE_ERR_ARG, "null bin arrays");
    if (!ws) return fail(ASE_ERR_WORKSPACE, "workspace is required");
    if (ws_bytes < ws_need) return fail(ASE_ERR_WORKSPACE, "workspace too small");
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(ASE_ERR_ALIGN, "workspace must be 256-byte aligned");
    char *c = static_cast<char *>(ws);
    const size_t arr = align_up((size_t)total * sizeof(double));
    std::memset(bl, 0, sizeof(*bl));
    bl->offsets = reinterpret_cast<const long long *>(offsets);
    bl->ncells = ncells;
    bl->dx = dx;
    bl->U = U;
    bl->sig = sigma;
    bl->t = t;
    bl->dt_hist = dt_hist;
    bl->dt_in = dt_replay;
    bl->status = status;
    bl->U1 = reinterpret_cast<double *>(c);
    bl->U2 = reinterpret_cast<double *>(c + 3 * arr);
    bl->sig2 = reinterpret_cast<double *>(c + 6 * arr);
    bl->bin_start = bin_start;
    bl->bin_list = bin_list;
    bl->bc_inst = bc_inst;
    bl->total = total;
    bl->ninst = ninst;
    bl->nbins = nbins;
    bl->threads = threads;
    bl->R = (p->order - 1) / 2;
    bl->ng = ng;
    bl->nsteps = nsteps;
    bl->bc = bc;
    bl->fo = (p->flags & ASE_FLAG_DF_FIRST_ORDER) ? 1 : 0;
    bl->t_end = t_end;
    bl->cfl = p->cfl;
    bl->dt_cap = p->dt_cap;
    bl->mc = method_const(p);
    return ASE_OK;
}

int ase_step_batched(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                     const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng, int64_t total,
                     double *U, double *sigma, double *t, double *dt_hist, const double *dt_replay,
                     int32_t *status, int32_t nsteps, double t_end, const int32_t *bin_start,
                     const int32_t *bin_list, int32_t nbins, int32_t threads, void *ws, size_t ws_bytes,
                     void *stream)
{
    BatchLaunch bl;
    int rc = batched_setup(p, bc, bc_inst, ninst, offsets, ncells, dx, ng, total, U, sigma, t, dt_hist, dt_replay,
                           status, nsteps, t_end, bin_start, bin_list, nbins, threads, ws, ws_bytes,
                           ase_batched_workspace_bytes(total), &bl);
    if (rc) return rc;
    if (nsteps == 0) return ASE_OK;
    {
        ProfScope ps(ASE_KCLASS_BATCHED, (hipStream_t)stream);
        launch_batched(bl, (hipStream_t)stream);
    }
    return check_launch("ase_step_batched");
}

// The library's second stream for a caller's stream on the current device
// (the wide part of a batched call runs there) and the events that fork it
// from and join it back into the caller's stream.  One per (device, caller
// stream), so calls on different streams stay concurrent; default priority;
// created on first use and kept until the process ends.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
static std::mutex g_side_mu;
static std::map<std::pair<int, hipStream_t>, SideStream> g_side;

static int side_stream(hipStream_t caller, SideStream **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    SideStream &ss = g_side[std::make_pair(dev, caller)];
    if (ss.s == nullptr) {
        e = hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
        e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
        e = hipEventCreateWithFlags(&ss.join, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
    }
    *out = &ss;
    return ASE_OK;
}

int ase_step_batched_wide(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                          const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng,
                          int64_t total, double *U, double *sigma, double *t, double *dt_hist,
                          const double *dt_replay, int32_t *status, int32_t nsteps, double t_end,
                          const int32_t *bin_start, const int32_t *bin_list, int32_t nbins, int32_t threads,
                          const int32_t *tile_inst, const int32_t *tile_i0, const int32_t *inst_tile0,
                          const int32_t *inst_ntiles, int32_t ntiles, int32_t threads_wide, void *ws,
                          size_t ws_bytes, void *stream)
{
    BatchLaunch bl;
    int rc = batched_setup(p, bc, bc_inst, ninst, offsets, ncells, dx, ng, total, U, sigma, t, dt_hist, dt_replay,
                           status, nsteps, t_end, bin_start, bin_list, nbins, threads, ws, ws_bytes,
                           ase_batched_wide_workspace_bytes(total, ninst, ntiles), &bl);
    if (rc) return rc;
    if (!(p->flags & ASE_FLAG_DF_FIRST_ORDER))
        return fail(ASE_ERR_ARG, "the wide batched form needs the first-order DF source (ASE_FLAG_DF_FIRST_ORDER)");
    if (ntiles < 0) return fail(ASE_ERR_ARG, "ntiles must be >= 0");
    const int nt_lanes = threads_wide & ~ASE_WIDE_STEP;
    if ((nt_lanes != 256 && nt_lanes != 512) || (threads_wide & ~(ASE_WIDE_STEP | 0x3ff)))
        return fail(ASE_ERR_ARG, "threads_wide must be 256 or 512, optionally with ASE_WIDE_STEP");
    if (!inst_tile0 || !inst_ntiles || (ntiles > 0 && (!tile_inst || !tile_i0)))
        return fail(ASE_ERR_ARG, "null tile arrays");
    if (nsteps == 0) return ASE_OK;
    hipStream_t st = (hipStream_t)stream;
    char *c = static_cast<char *>(ws) + ase_batched_workspace_bytes(total);
    WideLaunch wl;
    std::memset(&wl, 0, sizeof(wl));
    wl.offsets = bl.offsets; wl.ncells = ncells; wl.dx = dx;
    wl.U = U; wl.U1 = bl.U1; wl.U2 = bl.U2; wl.t = t; wl.dt_hist = dt_hist; wl.dt_in = dt_replay;
    wl.status = status; wl.bc_inst = bc_inst;
    wl.tile_inst = tile_inst; wl.tile_i0 = tile_i0; wl.inst_tile0 = inst_tile0; wl.inst_ntiles = inst_ntiles;
    wl.lam = reinterpret_cast<double *>(c);
    c += align_up((size_t)(ntiles > 0 ? ntiles : 1) * 2 * sizeof(double));
    wl.dt_cur = reinterpret_cast<double *>(c);
    c += align_up((size_t)ninst * sizeof(double));
    wl.done = reinterpret_cast<int *>(c);
    wl.total = total; wl.ninst = ninst; wl.ntiles = ntiles; wl.threads = nt_lanes; wl.R = bl.R; wl.ng = ng;
    wl.per_step = (threads_wide & ASE_WIDE_STEP) ? 1 : 0;
    wl.nsteps = nsteps;
    wl.bc = bc; wl.t_end = t_end; wl.cfl = p->cfl; wl.dt_cap = p->dt_cap; wl.mc = bl.mc;
    {
        ProfScope ps(ASE_KCLASS_BATCHED, st);
        if (ntiles == 0) {
            launch_batched(bl, st);
        } else {
            // the wide instances on the second stream, forked from the
            // caller's stream before the persistent launch (so the two run
            // side by side) and joined back into it
            std::lock_guard<std::mutex> lk(g_side_mu);
            SideStream *ss = nullptr;
            rc = side_stream(st, &ss);
            if (rc) return rc;
            hipError_t e = hipEventRecord(ss->fork, st);
            if (e == hipSuccess) e = hipStreamWaitEvent(ss->s, ss->fork, 0);
            if (e != hipSuccess) return hip_fail(e, "ase_step_batched_wide: fork");
            // the persistent launch carries the instances of the bins
            launch_batched(bl, st);
            wl.stage = 0;
            launch_batched_wide(wl, ss->s);
            for (int sidx = 0; sidx < nsteps; ++sidx)
                for (int stg = 1; stg <= (wl.per_step ? 1 : 3); ++stg) {
                    wl.step = sidx;
                    wl.stage = stg;
                    launch_batched_wide(wl, ss->s);
                }
            e = hipEventRecord(ss->join, ss->s);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, ss->join, 0);
            if (e != hipSuccess) return hip_fail(e, "ase_step_batched_wide: join");
            // the first-order strengths and ghost cells of the final states
            // of the tiled instances (the persistent launch wrote those of
            // its own)
            BatchLaunch ib = bl;
            ib.init = 1;
            ib.only = inst_ntiles;
            launch_batched(ib, st);
        }
    }
    return check_launch("ase_step_batched_wide");
}

int ase_step_batched_noalloc(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                             const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng,
                             int64_t total, double *U, double *sigma, double *t, double *dt_hist,
                             const double *dt_replay, int32_t *status, int32_t nsteps, double t_end,
                             const int32_t *bin_start, const int32_t *bin_list, int32_t nbins, int32_t threads,
                             void *stream)
{
    int rc = batched_common(p, bc, ninst, offsets, ncells, ng, total, U, sigma);
    if (rc) return rc;
    const size_t need = ase_batched_workspace_bytes(total);
    if (need > ASE_NOALLOC_SCRATCH_BYTES)
        return fail(ASE_ERR_WORKSPACE, "batch too large for the fixed scratch: ase_batched_workspace_bytes(total) = " +
                                           std::to_string(need) + " > ASE_NOALLOC_SCRATCH_BYTES = " +
                                           std::to_string((size_t)ASE_NOALLOC_SCRATCH_BYTES));
    void *scr = nullptr;
    rc = noalloc_scratch(&scr);
    if (rc) return rc;
    return ase_step_batched(p, bc, bc_inst, ninst, offsets, ncells, dx, ng, total, U, sigma, t, dt_hist, dt_replay,
                            status, nsteps, t_end, bin_start, bin_list, nbins, threads, scr,
                            ASE_NOALLOC_SCRATCH_BYTES, stream);
}

// ---- adjoint ----------------------------------------------------------------

static size_t adjoint_bytes(long long total, int nsteps)
{
    const size_t n = (size_t)total * sizeof(double);
    return align_up(9 * (size_t)nsteps * n) + align_up(3 * (size_t)nsteps * n) + 2 * align_up(3 * n);
}

static void carve_adjoint(void *ws, long long total, int nsteps, AdjLaunch *al)
{
    const size_t n = (size_t)total * sizeof(double);
    char *c = static_cast<char *>(ws);
    al->tapeU = reinterpret_cast<double *>(c);
    c += align_up(9 * (size_t)nsteps * n);
    al->tapeS = reinterpret_cast<double *>(c);
    c += align_up(3 * (size_t)nsteps * n);
    al->mu1 = reinterpret_cast<double *>(c);
    c += align_up(3 * n);
    al->mu2 = reinterpret_cast<double *>(c);
}

static int check_ws(void *ws, size_t ws_bytes, size_t need)
{
    if (!ws) return fail(ASE_ERR_WORKSPACE, "workspace is required");
    if (ws_bytes < need) return fail(ASE_ERR_WORKSPACE, "workspace too small");
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(ASE_ERR_ALIGN, "workspace must be 256-byte aligned");
    return ASE_OK;
}

size_t ase_adjoint_workspace_bytes(const ase_grid_t *g)
{
    if (!g || g->dim != 1 || g->ld < 1) return 0;
    return adjoint_bytes(g->ld, 1);
}

int ase_adjoint_step(const ase_grid_t *g, const ase_params_t *p, const double *U_n, const double *sigma_n,
                     const double *dt, const double *lam_np1, double *lam_n, void *ws, size_t ws_bytes,
                     void *stream)
{
    Geo geo;
    int rc = validate(g, p, &geo);
    if (rc) return rc;
    if (geo.dim != 1) return fail(ASE_ERR_ARG, "ase_adjoint_step: 1D grids only");
    if (g->bc[0] != g->bc[1] || (g->bc[0] != ASE_BC_TRANSMISSIVE && g->bc[0] != ASE_BC_PERIODIC &&
                                 g->bc[0] != ASE_BC_REFLECTIVE))
        return fail(ASE_ERR_ARG,
                    "ase_adjoint_step: boundaries must be both transmissive, both periodic or both reflective");
    ASE_PTR(U_n, "U_n");
    ASE_PTR(sigma_n, "sigma_n");
    ASE_PTR(dt, "dt");
    ASE_PTR(lam_np1, "lam_np1");
    ASE_PTR(lam_n, "lam_n");
    rc = check_ws(ws, ws_bytes, adjoint_bytes(geo.ld, 1));
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (lam_n != lam_np1) {
        hipError_t e = hipMemcpyAsync(lam_n, lam_np1, 3 * (size_t)geo.ld * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(lam)");
    }
    AdjLaunch al;
    std::memset(&al, 0, sizeof(al));
    carve_adjoint(ws, geo.ld, 1, &al);
    al.n1 = geo.nx;
    al.dx1 = g->dx;
    al.ck_U = U_n;
    al.ck_sig = sigma_n;
    al.dt_hist = dt;
    al.lam = lam_n;
    al.total = geo.ld;
    al.ninst = 1;
    al.threads = 256;
    al.R = geo.R;
    al.ng = geo.ng;
    al.nsteps = 1;
    al.bc = g->bc[0];
    al.fo = (p->flags & ASE_FLAG_DF_FIRST_ORDER) ? 1 : 0;
    al.phase = ASE_ADJ_TAPE | ASE_ADJ_REVERSE;
    al.mc = method_const(p);
    {
        ProfScope ps(ASE_KCLASS_ADJOINT, st);
        launch_adjoint(al, st);
    }
    return check_launch("ase_adjoint_step");
}

size_t ase_adjoint_batched_workspace_bytes(int64_t total, int32_t nsteps)
{
    if (total < 1 || nsteps < 1) return 0;
    return adjoint_bytes(total, nsteps);
}

// Validation of ase_adjoint_batched's arguments and its launch description.
static int adjoint_setup(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                         const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng, int64_t total,
                         const double *U_ck, const double *sigma_ck, const double *dt_hist, int32_t nsteps,
                         double *lam, const int32_t *bin_start, const int32_t *bin_list, int32_t nbins,
                         int32_t threads, int32_t phase, void *ws, size_t ws_bytes, AdjLaunch *al)
{
    int rc = batched_common(p, bc, ninst, offsets, ncells, ng, total, const_cast<double *>(U_ck),
                            const_cast<double *>(sigma_ck));
    if (rc) return rc;
    if (nsteps < 0) return fail(ASE_ERR_ARG, "nsteps must be >= 0");
    if (nbins < 1) return fail(ASE_ERR_ARG, "nbins must be >= 1");
    if (threads != 128 && threads != 256 && threads != 512)
        return fail(ASE_ERR_ARG, "threads must be 128, 256 or 512");
    if (phase < ASE_ADJ_TAPE || phase > (ASE_ADJ_TAPE | ASE_ADJ_REVERSE))
        return fail(ASE_ERR_ARG, "phase must be ASE_ADJ_TAPE, ASE_ADJ_REVERSE or both");
    ASE_PTR(dx, "dx");
    ASE_PTR(dt_hist, "dt_hist");
    ASE_PTR(lam, "lam");
    if (!bin_start || !bin_list) return fail(ASE_ERR_ARG, "null bin arrays");
    if (nsteps == 0) return ASE_OK;
    rc = check_ws(ws, ws_bytes, adjoint_bytes(total, nsteps));
    if (rc) return rc;
    std::memset(al, 0, sizeof(*al));
    carve_adjoint(ws, total, nsteps, al);
    al->offsets = reinterpret_cast<const long long *>(offsets);
    al->ncells = ncells;
    al->dx = dx;
    al->ck_U = U_ck;
    al->ck_sig = sigma_ck;
    al->dt_hist = dt_hist;
    al->lam = lam;
    al->bin_start = bin_start;
    al->bin_list = bin_list;
    al->bc_inst = bc_inst;
    al->total = total;
    al->ninst = ninst;
    al->nbins = nbins;
    al->threads = threads;
    al->R = (p->order - 1) / 2;
    al->ng = ng;
    al->nsteps = nsteps;
    al->bc = bc;
    al->fo = (p->flags & ASE_FLAG_DF_FIRST_ORDER) ? 1 : 0;
    al->phase = phase;
    al->mc = method_const(p);
    return ASE_OK;
}

int ase_adjoint_batched(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                        const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng, int64_t total,
                        const double *U_ck,
                        const double *sigma_ck, const double *dt_hist, int32_t nsteps, double *lam,
                        const int32_t *bin_start, const int32_t *bin_list, int32_t nbins, int32_t threads,
                        int32_t phase, void *ws, size_t ws_bytes, void *stream)
{
    AdjLaunch al;
    int rc = adjoint_setup(p, bc, bc_inst, ninst, offsets, ncells, dx, ng, total, U_ck, sigma_ck, dt_hist, nsteps,
                           lam, bin_start, bin_list, nbins, threads, phase, ws, ws_bytes, &al);
    if (rc || nsteps == 0) return rc;
    {
        ProfScope ps(ASE_KCLASS_ADJOINT, (hipStream_t)stream);
        launch_adjoint(al, (hipStream_t)stream);
    }
    return check_launch("ase_adjoint_batched");
}

int ase_adjoint_batched_wide(const ase_params_t *p, int32_t bc, const int32_t *bc_inst, int32_t ninst,
                             const int64_t *offsets, const int32_t *ncells, const double *dx, int32_t ng,
                             int64_t total, const double *U_ck, const double *sigma_ck, const double *dt_hist,
                             int32_t nsteps, double *lam, const int32_t *bin_start, const int32_t *bin_list,
                             int32_t nbins, int32_t threads, const int32_t *tile_inst, const int32_t *tile_i0,
                             const int32_t *inst_ntiles, int32_t ntiles, int32_t threads_wide, int32_t phase,
                             void *ws, size_t ws_bytes, void *stream)
{
    AdjLaunch al;
    int rc = adjoint_setup(p, bc, bc_inst, ninst, offsets, ncells, dx, ng, total, U_ck, sigma_ck, dt_hist, nsteps,
                           lam, bin_start, bin_list, nbins, threads, phase, ws, ws_bytes, &al);
    if (rc) return rc;
    if (!(p->flags & ASE_FLAG_DF_FIRST_ORDER))
        return fail(ASE_ERR_ARG, "the wide batched form needs the first-order DF source (ASE_FLAG_DF_FIRST_ORDER)");
    if (ntiles < 0) return fail(ASE_ERR_ARG, "ntiles must be >= 0");
    if (threads_wide != 256 && threads_wide != 512) return fail(ASE_ERR_ARG, "threads_wide must be 256 or 512");
    if (!inst_ntiles || (ntiles > 0 && (!tile_inst || !tile_i0))) return fail(ASE_ERR_ARG, "null tile arrays");
    if (nsteps == 0) return ASE_OK;
    hipStream_t st = (hipStream_t)stream;
    AdjWideLaunch wl;
    std::memset(&wl, 0, sizeof(wl));
    wl.offsets = al.offsets; wl.ncells = ncells; wl.dx = dx; wl.dt_hist = dt_hist; wl.ck_U = U_ck;
    wl.lam = lam; wl.mu1 = al.mu1; wl.mu2 = al.mu2; wl.tapeU = al.tapeU; wl.tapeS = al.tapeS;
    wl.bc_inst = bc_inst; wl.tile_inst = tile_inst; wl.tile_i0 = tile_i0; wl.inst_ntiles = inst_ntiles;
    wl.total = total; wl.ninst = ninst; wl.ntiles = ntiles; wl.threads = threads_wide; wl.R = al.R; wl.ng = ng;
    wl.nsteps = nsteps; wl.bc = bc; wl.mc = al.mc;
    {
        ProfScope ps(ASE_KCLASS_ADJOINT, st);
        if (ntiles == 0) {
            launch_adjoint(al, st);
        } else {
            // the wide instances on the library's second stream, forked before
            // the persistent launch and joined back after the last fold
            std::lock_guard<std::mutex> lk(g_side_mu);
            SideStream *ss = nullptr;
            rc = side_stream(st, &ss);
            if (rc) return rc;
            hipError_t e = hipEventRecord(ss->fork, st);
            if (e == hipSuccess) e = hipStreamWaitEvent(ss->s, ss->fork, 0);
            if (e != hipSuccess) return hip_fail(e, "ase_adjoint_batched_wide: fork");
            launch_adjoint(al, st);
            if (phase & ASE_ADJ_TAPE) launch_tape_wide(wl, ss->s);
            if (phase & ASE_ADJ_REVERSE) launch_adjoint_wide(wl, ss->s);
            e = hipEventRecord(ss->join, ss->s);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, ss->join, 0);
            if (e != hipSuccess) return hip_fail(e, "ase_adjoint_batched_wide: join");
        }
    }
    return check_launch("ase_adjoint_batched_wide");
}

int ase_pressure_objective(const ase_params_t *p, int32_t ninst, const int64_t *offsets, const int32_t *ncells,
                           const double *dx, int32_t ng, int64_t total, const double *U, const double *weights,
                           double *J, double *lam, void *stream)
{
    if (!p) return fail(ASE_ERR_ARG, "null params");
    if (!(p->gamma > 1.0)) return fail(ASE_ERR_ARG, "gamma must be > 1");
    if (ninst < 1 || total < 1 || ng < 0) return fail(ASE_ERR_ARG, "ninst, total must be >= 1 and ng >= 0");
    ASE_PTR(offsets, "offsets");
    ASE_PTR(ncells, "ncells");
    ASE_PTR(dx, "dx");
    ASE_PTR(U, "U");
    if (weights && misaligned(weights)) return fail(ASE_ERR_ALIGN, "misaligned: weights");
    if (J && misaligned(J)) return fail(ASE_ERR_ALIGN, "misaligned: J");
    if (lam && misaligned(lam)) return fail(ASE_ERR_ALIGN, "misaligned: lam");
    ObjLaunch ol;
    std::memset(&ol, 0, sizeof(ol));
    ol.offsets = reinterpret_cast<const long long *>(offsets);
    ol.ncells = ncells;
    ol.dx = dx;
    ol.U = U;
    ol.w = weights;
    ol.J = J;
    ol.lam = lam;
    ol.total = total;
    ol.ninst = ninst;
    ol.ng = ng;
    ol.gm1 = p->gamma - 1.0;
    launch_objective(ol, (hipStream_t)stream);
    return check_launch("ase_pressure_objective");
}

int ase_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (on && g_prof.pool.empty()) {
        g_prof.pool.resize(kProfPool);
        for (auto &e : g_prof.pool) {
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) {
                g_prof.pool.clear();
                return hip_fail(err, "hipEventCreate");
            }
        }
    }
    g_prof.recs.clear();
    g_prof.next = 0;
    g_prof.on = on != 0;
    return ASE_OK;
}

int ase_profile_read(int kernel_class, double *total_ms, int64_t *launches)
{
    if (!total_ms || !launches) return fail(ASE_ERR_ARG, "null output");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    double tot = 0.0;
    int64_t n = 0;
    for (const ProfRec &r : g_prof.recs) {
        if (r.cls != kernel_class) continue;
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return ASE_OK;
}

}  // extern "C"
