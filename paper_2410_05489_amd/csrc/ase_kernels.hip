// HIP kernels of the ASE-DF path for gfx950 (MI355X) and their launchers.
//
// Data layout: structure of arrays with ghost cells, U[v][J][I] (row stride
// ld), one strength plane per face direction of the same shape.  One thread
// per cell or face; reconstruction kernels stage a halo tile of the state and
// of both strength planes in LDS, reconstruct every cell of the tile (and of
// the halo rows the tangential stencils reach) once, keep the face traces in
// LDS, and evaluate Gauss points, strengths and fluxes from there.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>

#include "ase_device.h"
#include "ase_host.h"

namespace ase {


namespace {

constexpr int kThreads = 256;

struct BCInfo {
    int dim, nx, ny, ng, ld, NX, NY;
    int bc[4];
    long long plane;
    double y0, dy, slot_lo, slot_hi;
    double inflow[4];
    // double Mach reflection sides
    double x0, dx, wall_x0, shock_x0, shock_speed;
    double outer[4];
    // time of the stage being filled: *t + ct * *dt (t, dt device scalars;
    // null t: time 0)
    const double *t, *dt;
    double ct;
};

BCInfo make_bc(const ase_grid_t &g, const Geo &geo)
{
    BCInfo b;
    b.dim = geo.dim; b.nx = geo.nx; b.ny = geo.ny; b.ng = geo.ng; b.ld = geo.ld; b.NX = geo.NX; b.NY = geo.NY;
    for (int k = 0; k < 4; ++k) { b.bc[k] = g.bc[k]; b.inflow[k] = g.inflow[k]; }
    b.plane = geo.plane;
    b.y0 = g.y0; b.dy = g.dy; b.slot_lo = g.slot_lo; b.slot_hi = g.slot_hi;
    b.x0 = g.x0; b.dx = g.dx; b.wall_x0 = g.wall_x0; b.shock_x0 = g.shock_x0; b.shock_speed = g.shock_speed;
    for (int k = 0; k < 4; ++k) b.outer[k] = g.outer[k];
    b.t = nullptr;
    b.dt = nullptr;
    b.ct = 0.0;
    return b;
}

__device__ __forceinline__ double bc_time(const BCInfo &b)
{
    if (b.t == nullptr) return 0.0;
    return b.dt == nullptr ? *b.t : *b.t + b.ct * *b.dt;
}

__device__ __forceinline__ bool in_slot(const BCInfo &b, int J)
{
    if (b.dim == 1) return true;
    const double y = b.y0 + ((double)(J - b.ng) + 0.5) * b.dy;
    return y > b.slot_lo && y < b.slot_hi;
}

// Source of stored cell (I, J) under the boundary conditions: the row is
// mapped by the y rule, then the column by the x rule within that row (so
// corners are the y rule applied to x-filled values).  A reflective (slip)
// side mirrors the cells and reverses the momentum normal to it: flipx /
// flipy tell the caller to negate the x / y momentum.  Returns SRC_CELL, or
// SRC_INFLOW / SRC_OUTER when the cell takes that fixed state (a fixed
// y-side state covers the corner columns too).
enum { SRC_CELL = 0, SRC_INFLOW = 1, SRC_OUTER = 2 };

__device__ __forceinline__ int src_cell(const BCInfo &b, int I, int J, int &Is, int &Js, bool &flipx, bool &flipy)
{
    Js = J;
    flipx = flipy = false;
    if (b.dim == 2) {
        const int j = J - b.ng;
        const double xc = b.x0 + ((double)(I - b.ng) + 0.5) * b.dx;
        if (j < 0) {
            if (b.bc[2] == ASE_BC_PERIODIC) Js = J + b.ny;
            else if (b.bc[2] == ASE_BC_REFLECTIVE || b.bc[2] == ASE_BC_NOSLIP ||
                     (b.bc[2] == ASE_BC_WALL_INFLOW && !(xc < b.wall_x0))) {
                Js = 2 * b.ng - 1 - J;
                flipy = true;
                flipx = b.bc[2] == ASE_BC_NOSLIP;
            } else if (b.bc[2] == ASE_BC_WALL_INFLOW) return SRC_INFLOW;
            else Js = b.ng;
        } else if (j >= b.ny) {
            if (b.bc[3] == ASE_BC_PERIODIC) Js = J - b.ny;
            else if (b.bc[3] == ASE_BC_REFLECTIVE || b.bc[3] == ASE_BC_NOSLIP) {
                Js = 2 * (b.ny + b.ng) - 1 - J;
                flipy = true;
                flipx = b.bc[3] == ASE_BC_NOSLIP;
            } else if (b.bc[3] == ASE_BC_MOVING_SHOCK)
                return xc < b.shock_x0 + b.shock_speed * bc_time(b) ? SRC_INFLOW : SRC_OUTER;
            else Js = b.ng + b.ny - 1;
        }
    }
    // the x rule toggles the flips of the y rule (a no-slip corner reverses
    // the momentum twice)
    Is = I;
    const int i = I - b.ng;
    if (i < 0) {
        if (b.bc[0] == ASE_BC_PERIODIC) Is = I + b.nx;
        else if (b.bc[0] == ASE_BC_INFLOW_SLOT && in_slot(b, Js)) return SRC_INFLOW;
        else if (b.bc[0] == ASE_BC_REFLECTIVE || b.bc[0] == ASE_BC_NOSLIP) {
            Is = 2 * b.ng - 1 - I;
            flipx = !flipx;
            if (b.bc[0] == ASE_BC_NOSLIP) flipy = !flipy;
        } else Is = b.ng;
    } else if (i >= b.nx) {
        if (b.bc[1] == ASE_BC_PERIODIC) Is = I - b.nx;
        else if (b.bc[1] == ASE_BC_INFLOW_SLOT && in_slot(b, Js)) return SRC_INFLOW;
        else if (b.bc[1] == ASE_BC_REFLECTIVE || b.bc[1] == ASE_BC_NOSLIP) {
            Is = 2 * (b.nx + b.ng) - 1 - I;
            flipx = !flipx;
            if (b.bc[1] == ASE_BC_NOSLIP) flipy = !flipy;
        } else Is = b.ng + b.nx - 1;
    }
    return SRC_CELL;
}

// Ghost frame: full ghost rows (2D) followed by the ghost columns of the
// interior rows.  frame_size() cells, enumerated by frame_cell().
__host__ __device__ __forceinline__ long long frame_size(const BCInfo &b)
{
    const long long side = (long long)(b.dim == 1 ? 1 : b.ny) * 2 * b.ng;
    return (b.dim == 1 ? 0 : 2LL * b.ng * b.NX) + side;
}

__device__ __forceinline__ void frame_cell(const BCInfo &b, long long idx, int &I, int &J)
{
    const long long rows = b.dim == 1 ? 0 : 2LL * b.ng * b.NX;
    if (idx < rows) {
        const int r = (int)(idx / b.NX);
        J = r < b.ng ? r : r + b.ny;
        I = (int)(idx % b.NX);
    } else {
        const long long q = idx - rows;
        const int c = (int)(q % (2 * b.ng));
        J = b.dim == 1 ? 0 : b.ng + (int)(q / (2 * b.ng));
        I = c < b.ng ? c : c + b.nx;
    }
}

// Value of stored cell (I, J) under the boundary conditions: the interior
// cell it copies, or the inflow state.  Sources are always interior cells,
// so this never reads a ghost cell and may run while ghosts are written.
template <int NV>
__device__ __forceinline__ void cell_value(const BCInfo &b, const double *U, int I, int J, double (&W)[NV])
{
    int Is, Js;
    bool fx, fy;
    const int src = src_cell(b, I, J, Is, Js, fx, fy);
    if (src == SRC_CELL) {
        const long long pos = (long long)Js * b.ld + Is;
#pragma unroll
        for (int v = 0; v < NV; ++v) W[v] = U[v * b.plane + pos];
        if (fx) W[1] = -W[1];
        if (NV == 4 && fy) W[2] = -W[2];
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) W[v] = src == SRC_INFLOW ? b.inflow[v] : b.outer[v];
    }
}

template <int NV>
__device__ __forceinline__ double sigma_first_order(const BCInfo &b, const double *U, int Ia, int Ja, int Ib, int Jb,
                                                    int dir, const MethodConst &mc)
{
    double Wa[NV], Wb[NV];
    cell_value<NV>(b, U, Ia, Ja, Wa);
    cell_value<NV>(b, U, Ib, Jb, Wb);
    const Prim qa = primitives<NV>(Wa, dir, mc);
    const Prim qb = primitives<NV>(Wb, dir, mc);
    return sigma_point(qa, qb);
}

__device__ __forceinline__ int wrapi(int i, int n) { return ((i % n) + n) % n; }

__device__ __forceinline__ bool is_wall(int bc) { return bc == ASE_BC_REFLECTIVE || bc == ASE_BC_NOSLIP; }

// Cell index mapped by the boundary rule of one axis: periodic wrap or wall
// mirror; other codes leave it.
__device__ __forceinline__ int map_cell(int i, int n, int lo, int hi)
{
    if (i < 0) {
        if (lo == ASE_BC_PERIODIC) return wrapi(i, n);
        if (is_wall(lo)) return -1 - i;
    } else if (i >= n) {
        if (hi == ASE_BC_PERIODIC) return wrapi(i, n);
        if (is_wall(hi)) return 2 * n - 1 - i;
    }
    return i;
}

// Face index f (face f + 1/2) mapped likewise: a wall at -1/2 maps f to
// -f-2, a wall at n-1/2 maps f to 2n-f-2 (a wall is a symmetry plane of the
// lagged strengths as well as of the cells).
__device__ __forceinline__ int map_face(int f, int n, int lo, int hi)
{
    if (f < -1) {
        if (lo == ASE_BC_PERIODIC) return wrapi(f, n);
        if (is_wall(lo)) return -f - 2;
    } else if (f > n - 1) {
        if (hi == ASE_BC_PERIODIC) return wrapi(f, n);
        if (is_wall(hi)) return 2 * n - f - 2;
    }
    return f;
}

// The ghost frame: ghost cells and the strengths of the stored faces that
// are not flux faces; each non-flux face takes its periodic image or its
// mirror image at a wall if that is a flux face, else the first-order
// strength of its two (boundary-mapped) cells.  The three jobs of a frame
// cell -- its ghost value, the strength of its x-face, that of its y-face --
// are independent (strengths read boundary-mapped interior values, never
// the ghosts being written, and non-flux faces only the flux faces) and run
// in separate workgroups (blockIdx.y): the frame is too small to fill the
// chip, and three short chains per cell finish sooner than one.  (With the
// first-order DF source k_fill_fo does the ghosts and every strength.)
template <int NV>
__global__ void __launch_bounds__(kThreads) k_bc_fill(BCInfo b, MethodConst mc, double *U, double *sx, double *sy)
{
    const int job = (int)blockIdx.y;
    const long long n = frame_size(b);
    for (long long idx = (long long)blockIdx.x * kThreads + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * kThreads) {
        int I, J;
        frame_cell(b, idx, I, J);
        const long long pos = (long long)J * b.ld + I;
        const int i = I - b.ng, j = J - b.ng;
        const bool ghost = i < 0 || i >= b.nx || (b.dim == 2 && (j < 0 || j >= b.ny));
        if (job == 0 && ghost) {
            double W[NV];
            cell_value<NV>(b, U, I, J, W);
#pragma unroll
            for (int v = 0; v < NV; ++v) U[v * b.plane + pos] = W[v];
        }
        // x-face between (I,J) and (I+1,J)
        if (job == 1 && I + 1 < b.NX) {
            const int f = i;
            const bool row_ok = b.dim == 1 || (j >= 0 && j < b.ny);
            const bool produced = row_ok && f >= -1 && f <= b.nx - 1;
            if (!produced) {
                const int fw = map_face(f, b.nx, b.bc[0], b.bc[1]);
                const int jw = b.dim == 2 ? map_cell(j, b.ny, b.bc[2], b.bc[3]) : j;
                const bool jw_ok = b.dim == 1 || (jw >= 0 && jw < b.ny);
                if (jw_ok && fw >= -1 && fw <= b.nx - 1) {
                    const int Jw = b.dim == 1 ? 0 : jw + b.ng;
                    sx[pos] = sx[(long long)Jw * b.ld + fw + b.ng];
                } else {
                    sx[pos] = sigma_first_order<NV>(b, U, I, J, I + 1, J, 0, mc);
                }
            }
        }
        if (job == 2 && b.dim == 2 && J + 1 < b.NY) {
            const int f = j;
            const bool produced = i >= 0 && i < b.nx && f >= -1 && f <= b.ny - 1;
            if (!produced) {
                const int fw = map_face(f, b.ny, b.bc[2], b.bc[3]);
                const int iw = map_cell(i, b.nx, b.bc[0], b.bc[1]);
                if (iw >= 0 && iw < b.nx && fw >= -1 && fw <= b.ny - 1) {
                    sy[pos] = sy[(long long)(fw + b.ng) * b.ld + iw + b.ng];
                } else {
                    sy[pos] = sigma_first_order<NV>(b, U, I, J, I, J + 1, 1, mc);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Time step: per-block maxima of the signal-speed sum, then one block that
// reduces them, clips against t_end and advances t.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double max_nan(double a, double b) { return (b > a || b != b) ? b : a; }

// First-order DF source of a stage input in one pass: the ghost cells, every
// stored strength from the two cell averages beside its face, and, when
// `part` is given, the largest signal-speed sum of the tile's interior cells
// for the time step (the per-cell value of k_cfl_partial).  Tiles of TX x TY
// stored cells plus the next column and row; the primitive variables of each
// cell are formed once, in LDS, and each cell's x-face and y-face take the
// argument order and normal/tangential roles of sigma_first_order.  A ghost
// cell gets the value of the interior cell it copies (cell_value never reads
// a ghost, so tiles may write ghosts while others read), which is what
// k_bc_fill writes there; the strengths are those of the filled state.
template <int NV, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) k_fill_fo(BCInfo b, MethodConst mc, double *U, double *sx, double *sy,
                                                     double inv_dx, double inv_dy, double *part)
{
    constexpr int NT = TX * TY;
    constexpr int NI = ((TY + 1) * (TX + 1) + NT - 1) / NT;   // items per lane
    __shared__ double sp[TY + 1][TX + 1], su[TY + 1][TX + 1], sv[TY + 1][TX + 1], sic[TY + 1][TX + 1];
    __shared__ bool sok[TY + 1][TX + 1];
    __shared__ double red[NT / 64];
    const int NYs = b.dim == 1 ? 1 : b.NY;
    // tiles in contiguous bands per XCD: the extra column and row a tile
    // reads are then mostly in its own L2
    int btx, bty;
    xcd_tile(btx, bty);
    const int I0 = btx * TX, J0 = bty * TY;
    double lam = 0.0;
    // all loads of a lane first, then the primitive variables
    double W[NI][NV];
    bool valid[NI], ghost[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int it = threadIdx.x + k * NT;
        const int lx = it % (TX + 1), ly = it / (TX + 1);
        const int I = I0 + lx, J = J0 + ly;
        valid[k] = it < (TY + 1) * (TX + 1) && I < b.NX && J < NYs;
        const int i = I - b.ng, j = J - b.ng;
        ghost[k] = i < 0 || i >= b.nx || (b.dim == 2 && (j < 0 || j >= b.ny));
        if (!valid[k]) {
#pragma unroll
            for (int v = 0; v < NV; ++v) W[k][v] = 0.0;
        } else if (ghost[k]) {
            cell_value<NV>(b, U, I, J, W[k]);
        } else {
            const long long pos = (long long)J * b.ld + I;
#pragma unroll
            for (int v = 0; v < NV; ++v) W[k][v] = U[v * b.plane + pos];
        }
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        if (!valid[k]) continue;
        const int it = threadIdx.x + k * NT;
        const int lx = it % (TX + 1), ly = it / (TX + 1);
        const bool own = lx < TX && ly < TY;
        if (ghost[k] && own) {
            const long long pos = (long long)(J0 + ly) * b.ld + I0 + lx;
#pragma unroll
            for (int v = 0; v < NV; ++v) U[v * b.plane + pos] = W[k][v];
        }
        const Prim q = primitives<NV>(W[k], 0, mc);
        sp[ly][lx] = q.p;
        su[ly][lx] = q.un;
        sv[ly][lx] = q.ut;
        sic[ly][lx] = q.ic;
        sok[ly][lx] = q.ok;
        if (part != nullptr && own && !ghost[k]) {
            double l = (fabs(q.un) + q.c) * inv_dx;
            if constexpr (NV == 4) l = l + (fabs(q.ut) + q.c) * inv_dy;
            lam = max_nan(lam, l);
        }
    }
    if (part != nullptr) {
        // the maximum is exact and NaN-sticky in any order
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lam = max_nan(lam, __shfl_xor(lam, o));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lam;
    }
    __syncthreads();
    if (part != nullptr && threadIdx.x == 0) {
        double m = red[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) m = max_nan(m, red[w]);
        part[(long long)blockIdx.y * gridDim.x + blockIdx.x] = m;
    }
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int I = I0 + lx, J = J0 + ly;
    if (I >= b.NX || J >= NYs) return;
    const long long pos = (long long)J * b.ld + I;
    auto prim = [&](int y, int x, bool xface) {
        Prim q;
        q.p = sp[y][x];
        q.un = xface ? su[y][x] : sv[y][x];
        q.ut = xface ? sv[y][x] : su[y][x];
        q.ic = sic[y][x];
        q.c = 0.0;
        q.ok = sok[y][x];
        return q;
    };
    if (I + 1 < b.NX) sx[pos] = sigma_point(prim(ly, lx, true), prim(ly, lx + 1, true));
    if (b.dim == 2 && J + 1 < b.NY) sy[pos] = sigma_point(prim(ly, lx, false), prim(ly + 1, lx, false));
}

template <int NV>
__global__ void __launch_bounds__(kThreads) k_cfl_partial(BCInfo b, MethodConst mc, const double *U, double inv_dx,
                                                          double inv_dy, double *part)
{
    __shared__ double red[kThreads];
    const int ny = b.dim == 1 ? 1 : b.ny;
    const long long n = (long long)ny * b.nx;
    double lam = 0.0;
    for (long long idx = (long long)blockIdx.x * kThreads + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * kThreads) {
        const int j = (int)(idx / b.nx), i = (int)(idx % b.nx);
        const long long pos = (long long)(b.dim == 1 ? 0 : j + b.ng) * b.ld + i + b.ng;
        double W[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) W[v] = U[v * b.plane + pos];
        const Prim q = primitives<NV>(W, 0, mc);
        double l = (fabs(q.un) + q.c) * inv_dx;
        if constexpr (NV == 4) l = l + (fabs(q.ut) + q.c) * inv_dy;
        lam = max_nan(lam, l);
    }
    red[threadIdx.x] = lam;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = max_nan(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Number of interior cells with rho <= 0, p <= 0 or a NaN among them, per
// block (an exact integer in a double); the host adds the blocks up.
template <int NV>
__global__ void __launch_bounds__(kThreads) k_nonphysical_partial(BCInfo b, MethodConst mc, const double *U,
                                                                  double *part)
{
    __shared__ double red[kThreads];
    const int ny = b.dim == 1 ? 1 : b.ny;
    const long long n = (long long)ny * b.nx;
    double cnt = 0.0;
    for (long long idx = (long long)blockIdx.x * kThreads + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * kThreads) {
        const int j = (int)(idx / b.nx), i = (int)(idx % b.nx);
        const long long pos = (long long)(b.dim == 1 ? 0 : j + b.ng) * b.ld + i + b.ng;
        double W[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) W[v] = U[v * b.plane + pos];
        double ke = W[1] * W[1];
        if constexpr (NV == 4) ke += W[2] * W[2];
        const double p = mc.gm1 * (W[NV - 1] - 0.5 * ke / W[0]);
        bool bad = !(W[0] > 0.0) || !(p > 0.0);
#pragma unroll
        for (int v = 0; v < NV; ++v) bad = bad || W[v] != W[v];
        cnt += bad ? 1.0 : 0.0;
    }
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

struct InflowSpeed {
    int on, dim;
    double W[4];
    double inv_dx, inv_dy;
};

// One workgroup of kFinalThreads lanes (a lane's loads in flight cover the
// partials of a 1024^2 grid's fill tiles in one round).
constexpr int kFinalThreads = 1024;

__global__ void __launch_bounds__(kFinalThreads) k_cfl_final(const double *part, int nparts, double cfl,
                                                             double dt_cap, const double *t_in, double *t_out,
                                                             double t_end, double *dt_out, double *skip_out,
                                                             double *dt_hist, InflowSpeed inf, MethodConst mc)
{
    __shared__ double red[kFinalThreads / 64];
    double lam = 0.0;
    if (threadIdx.x == 0 && inf.on) {
        // inflow ghost states enter the domain: their signal speed counts too
        double l;
        if (inf.dim == 2) {
            const double W[4] = {inf.W[0], inf.W[1], inf.W[2], inf.W[3]};
            const Prim q = primitives<4>(W, 0, mc);
            l = (fabs(q.un) + q.c) * inf.inv_dx + (fabs(q.ut) + q.c) * inf.inv_dy;
        } else {
            const double W[3] = {inf.W[0], inf.W[1], inf.W[2]};
            const Prim q = primitives<3>(W, 0, mc);
            l = (fabs(q.un) + q.c) * inf.inv_dx;
        }
        lam = max_nan(lam, l);
    }
    // eight loads in flight per lane (the partials are >= 0, so a padding 0
    // leaves the maximum as it is)
    for (int k0 = threadIdx.x; k0 < nparts; k0 += 8 * kFinalThreads) {
        double pv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u * kFinalThreads;
            pv[u] = k < nparts ? part[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) lam = max_nan(lam, pv[u]);
    }
    // the maximum is exact and NaN-sticky in any order: lanes, then waves
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lam = max_nan(lam, __shfl_xor(lam, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lam;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
#pragma unroll
        for (int w = 1; w < kFinalThreads / 64; ++w) m = max_nan(m, red[w]);
        const double t = *t_in;
        const bool skip = t_end > 0.0 && t >= t_end;
        double dt = 0.0;
        if (!skip) {
            dt = cfl / m;
            if (dt_cap > 0.0 && dt > dt_cap) dt = dt_cap;
            if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
        }
        *dt_out = dt;
        if (skip_out) *skip_out = skip ? 1.0 : 0.0;
        if (t_out) *t_out = t + dt;
        if (dt_hist) *dt_hist = dt;
    }
}

// ---------------------------------------------------------------------------
// 2D sweep: one tile of T0 x T1 cells, faces of direction DIR, NT threads.
//
// Phase 1 reconstructs, along DIR, every cell whose face values the tile's
// tangential stencils need (normal reconstruction; one cell per thread).
// Phase 2 gives each face two adjacent lanes, one per side: each lane runs
// the tangential reconstruction of its side to the G Gauss points, the pair
// swaps half of the Gauss states (lane ^ 1) so that each lane evaluates
// strengths and LF fluxes at half of the points, and a second swap sums the
// quadrature.  Phase 3 forms flux differences and, in the second sweep, the
// SSP-RK3 stage combination.
// ---------------------------------------------------------------------------

// Occupancy: the bound of six 256-lane waves per SIMD (80 registers) gives
// the x sweep (512 lanes, 52 KB of LDS) three workgroups per CU and the y
// sweep (256 lanes, 19 KB with its traces over the staged state) six.
template <int DIR, int R, int T0, int T1, int NT, int MODE>
__global__ void __launch_bounds__(NT, 6) k_sweep2d(SweepArgs a)
{
    constexpr int NV = 4, G = R, OI = R - 1;
    using S = SweepShape<DIR, R, T0, T1>;
    constexpr int UX = S::UX, UY = S::UY, TX = S::TX, TY = S::TY, FX = S::FX, FY = S::FY;
    constexpr int GA = (G + 1) / 2;   // Gauss points evaluated by the lower/left lane of a pair
    constexpr int NU = NV * UY * UX;
    constexpr int NF = (MODE == MODE_RECON) ? 0 : NV * FY * FX;
    static_assert(NF <= NU, "flux tile must fit in the state tile");
    // y faces: the face traces overwrite the staged state once phase 1 has
    // read it, so a workgroup needs 19 instead of 32 KB of LDS and six fit on
    // a CU (the register bound of 80 then decides).  x faces keep separate
    // arrays: their 512-lane workgroups are register-bound at three per CU.
    constexpr bool SHARE = (DIR == 1);
    // strengths: the normal plane over the whole staged tile, the tangential
    // plane only where the side cells' columns (rows) read it
    constexpr int SY = (DIR == 0) ? UY : TY, SX = (DIR == 0) ? TX : UX;
    __shared__ double sSN[UY][UX];
    __shared__ double sST[SY][SX];
    // right-face traces, then left-face traces.  The LDS serves a 64-bit
    // read to 16 lanes per cycle, double d in bank pair d mod 16.  A group of
    // 16 lanes in phase 2 holds 8 faces, both sides; the offset of the
    // second array puts the two sides of a face 8 doubles apart modulo 16
    // (x faces: the upper side reads the next column, +1; y faces: the next
    // row, +TX), so the 16 reads hit 16 different bank pairs.
    constexpr int NT1 = NV * TY * TX;
    constexpr int TSTEP = (DIR == 0) ? 1 : TX;
    constexpr int TOFF = (NT1 + 15) / 16 * 16 + ((8 - TSTEP) % 16 + 16) % 16;
    constexpr int NTT = TOFF + NT1;
    // staged state; the face traces (SHARE); the face fluxes
    __shared__ double sUF[SHARE ? (NU > NTT ? NU : NTT) : NU];
    __shared__ double sTown[SHARE ? 1 : NTT];
    double *sT = SHARE ? sUF : sTown;
    double(*sTR)[TY][TX] = reinterpret_cast<double(*)[TY][TX]>(&sT[0]);
    double(*sTL)[TY][TX] = reinterpret_cast<double(*)[TY][TX]>(&sT[TOFF]);
    auto sU = [&](int v, int y, int x) -> double & { return sUF[(v * UY + y) * UX + x]; };
    auto sF = [&](int v, int y, int x) -> double & { return sUF[(v * FY + y) * FX + x]; };

    const int tid = threadIdx.x;
    int btx, bty;
    xcd_tile(btx, bty);
    const int i0 = btx * T0, j0 = bty * T1;
    const int ox = (DIR == 0) ? i0 - 1 - R : i0 - R;
    const int oy = (DIR == 0) ? j0 - R : j0 - 1 - R;
    const MethodConst &mc = a.mc;

    // first-order DF source: the stage's strengths come from its cell
    // averages (boundary step), so the sweep evaluates and writes none
    const bool want_sigma = (a.mc.flags & ASE_FLAG_DF_FIRST_ORDER) == 0;
    if (MODE != MODE_RECON && a.skip != nullptr && *a.skip != 0.0) {
        if (!want_sigma) return;
        // finished run: carry the strengths of the owned flux faces over
        const double *sin = DIR == 0 ? a.sx : a.sy;
        for (int it = tid; it < FX * FY; it += NT) {
            const int fx = it % FX, fy = it / FX;
            const int x = DIR == 0 ? i0 - 1 + fx : i0 + fx;
            const int y = DIR == 0 ? j0 + fy : j0 - 1 + fy;
            if (DIR == 0 ? (x > a.nx - 1 || y >= a.ny) : (x >= a.nx || y > a.ny - 1)) continue;
            const bool own = DIR == 0 ? (fx > 0 || i0 == 0) : (fy > 0 || j0 == 0);
            if (own) {
                const long long pos = (long long)(y + a.ng) * a.ld + x + a.ng;
                a.sig_out[pos] = sin[pos];
            }
        }
        return;
    }

    // stage the halo tile
    for (int it = tid; it < UX * UY; it += NT) {
        const int lx = it % UX, ly = it / UX;
        const int I = ox + lx + a.ng, J = oy + ly + a.ng;
        const bool in = I < a.NX && J < a.NY;
        const long long pos = (long long)J * a.ld + I;
#pragma unroll
        for (int v = 0; v < NV; ++v) sU(v, ly, lx) = in ? a.U[v * a.plane + pos] : 0.0;
        sSN[ly][lx] = in ? (DIR == 0 ? a.sx[pos] : a.sy[pos]) : 0.0;
        const int sty = (DIR == 0) ? ly : ly - R, stx = (DIR == 0) ? lx - R : lx;
        if (sty >= 0 && sty < SY && stx >= 0 && stx < SX) sST[sty][stx] = in ? (DIR == 0 ? a.sy[pos] : a.sx[pos]) : 0.0;
    }
    __syncthreads();

    if constexpr (SHARE) {
        // phase 1 in one pass, the traces held in registers until every lane
        // has read its stencil from the staged state they replace
        static_assert(DIR == 1 && TX * TY <= NT, "one phase-1 pass");
        const int tx = tid % TX, ty = tid / TX;
        const int lx = tx, ly = ty + R;
        const int x = ox + lx, y = oy + ly;
        const bool need = tid < TX * TY && x < a.nx + R && y <= a.ny;
        double out[NV][2];
        int lvl = 0;
        if (need) {
            double s[2 * R];
#pragma unroll
            for (int m = -R; m < R; ++m) s[m + R] = sSN[ly + m][lx];
            auto ld = [&](int v, int m) { return sU(v, ly + m, lx); };
            lvl = reconstruct_cell<R, NV, 2>(ld, s, mc, OI, 0, out);
        }
        __syncthreads();
        if (need) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                sTR[v][ty][tx] = out[v][0];
                sTL[v][ty][tx] = out[v][1];
            }
            if (MODE == MODE_RECON && a.level != nullptr && x >= 0 && x < a.nx && y >= 0 && y < a.ny)
                a.level[(long long)y * a.nx + x] = (int8_t)lvl;
        }
    } else {
    // phase 1: normal reconstruction, face traces of every cell the tile needs.
    // x faces (TX = 17 trace columns): each group of 16 lanes takes 16
    // columns of one row, the last column is walked down its rows; both
    // orders keep the 16 reads of a group in distinct bank pairs.
    for (int it = tid; it < TX * TY; it += NT) {
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
        auto ld = [&](int v, int m) { return (DIR == 0) ? sU(v, ly, lx + m) : sU(v, ly + m, lx); };
        double out[NV][2];
        const int lvl = reconstruct_cell<R, NV, 2>(ld, s, mc, OI, 0, out);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            sTR[v][ty][tx] = out[v][0];
            sTL[v][ty][tx] = out[v][1];
        }
        if (MODE == MODE_RECON && a.level != nullptr && x >= 0 && x < a.nx && y >= 0 && y < a.ny)
            a.level[(long long)y * a.nx + x] = (int8_t)lvl;
    }
    }
    __syncthreads();

    // phase 2: two lanes per face (side = lane & 1)
    constexpr int NITEMS = 2 * FX * FY;
    static_assert(!SHARE || NITEMS <= NT, "one phase-2 pass");
    double Fkeep[NV];        // SHARE: this face's flux, stored after the traces are read
    bool keep = false;
    int kfx = 0, kfy = 0;
    for (int base = 0; base < NITEMS; base += NT) {   // uniform trip count: lane pairs swap together
        const int it = base + tid;
        const int side = it & 1, f = it >> 1;
        const int fx = f % FX, fy = f / FX;
        const int x = DIR == 0 ? i0 - 1 + fx : i0 + fx;
        const int y = DIR == 0 ? j0 + fy : j0 - 1 + fy;
        const bool valid = it < NITEMS && (DIR == 0 ? (x <= a.nx - 1 && y < a.ny) : (x < a.nx && y <= a.ny - 1));
        double Ws[NV][G];
        if (valid) {
            double s[2 * R];
            // this side's face traces: right-face values of the left (lower)
            // cell, left-face values of the right (upper) cell
            const double *tr = side == 0 ? &sTR[0][0][0] : &sTL[0][0][0];
            if (DIR == 0) {
                const int tx = fx + side;
#pragma unroll
                for (int m = -R; m < R; ++m) s[m + R] = sST[fy + R + m][tx];
                auto ld = [&](int v, int m) { return tr[(v * TY + fy + R + m) * TX + tx]; };
                reconstruct_cell<R, NV, G>(ld, s, mc, OI, 2, Ws);
            } else {
                const int ty = fy + side;
#pragma unroll
                for (int m = -R; m < R; ++m) s[m + R] = sST[ty][fx + R + m];
                auto ld = [&](int v, int m) { return tr[(v * TY + ty) * TX + fx + R + m]; };
                reconstruct_cell<R, NV, G>(ld, s, mc, OI, 2, Ws);
            }
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int k = 0; k < G; ++k) Ws[v][k] = 1.0;
        }
        if constexpr (MODE == MODE_RECON) {
            if (valid) {
                const long long fid =
                    DIR == 0 ? (long long)y * (a.nx + 1) + (x + 1) : (long long)(y + 1) * a.nx + x;
                double *dst = side == 0 ? a.wl : a.wr;
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int k = 0; k < G; ++k) dst[(long long)(v * G + k) * a.nfaces + fid] = Ws[v][k];
            }
        } else {
            // lane 0 of the pair evaluates points [0, GA), lane 1 points [GA, G)
            constexpr int GB = G - GA;
            double lo[NV][GA], hi[NV][GA];
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int j = 0; j < GA; ++j) {
                    lo[v][j] = Ws[v][j];
                    hi[v][j] = 0.0;
                }
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int j = 0; j < GB; ++j) hi[v][j] = Ws[v][GA + j];
            double Fs[NV], ssum = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) Fs[v] = 0.0;
            // cell averages of this lane's side and of the other side (read
            // only for the positivity replacement)
            // (positions within a plane fit in 32 bits: the host checks it)
            // The face position is formed again from the lane index (behind
            // an empty asm, so that x and y need not stay live across the
            // reconstruction: they were spilled there).
            int tid2 = tid;
            asm volatile("" : "+v"(tid2));
            const int f2 = (base + tid2) >> 1;
            const int x2 = DIR == 0 ? i0 - 1 + f2 % FX : i0 + f2 % FX;
            const int y2 = DIR == 0 ? j0 + f2 / FX : j0 - 1 + f2 / FX;
            const int pl = (y2 + a.ng) * a.ld + x2 + a.ng;
            const int pr = DIR == 0 ? pl + 1 : pl + a.ld;
            const int po = side == 0 ? pl : pr, pt = side == 0 ? pr : pl;
            const double *U = a.U;
            const long long P = a.plane;
            // the replacement is rare: an empty asm on the position keeps
            // its address arithmetic from being hoisted into registers that
            // stay live across the Gauss points (4 spilled registers)
            auto co = [=](int v) {
                int q = po;
                asm volatile("" : "+v"(q));
                return U[v * P + q];
            };
            auto ct = [=](int v) {
                int q = pt;
                asm volatile("" : "+v"(q));
                return U[v * P + q];
            };
            const double sgn = side == 0 ? 1.0 : -1.0;
#pragma unroll
            for (int j = 0; j < GA; ++j) {
                double Wown[NV], Woth[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Wown[v] = side == 0 ? lo[v][j] : hi[v][j];
                    Woth[v] = swap_pair(side == 0 ? hi[v][j] : lo[v][j]);
                }
                const bool has = valid && (side == 0 || j < GB);
                if (has) {
                    double Fk[NV];
                    // one call for both sides: a select on `side` around the
                    // call would run the whole point evaluation twice per wave
                    ssum += gauss_point_sided<NV>(Wown, Woth, sgn, co, ct, DIR, mc, Fk, want_sigma);
                    const double eta = kTab.eta[OI][side == 0 ? j : GA + j];
#pragma unroll
                    for (int v = 0; v < NV; ++v) Fs[v] = fma(eta, Fk[v], Fs[v]);
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) Fs[v] += swap_pair(Fs[v]);
            ssum += swap_pair(ssum);
            if (want_sigma && valid && side == 0) {
                const bool own = DIR == 0 ? (fx > 0 || i0 == 0) : (fy > 0 || j0 == 0);
                if (own) a.sig_out[pl] = ssum / (double)G;
            }
            // the flux tile reuses the state tile (x faces: phase 2 reads no
            // staged state; y faces: stored once every lane has read its traces)
            if (valid && side == 0) {
                if constexpr (SHARE) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) Fkeep[v] = Fs[v];
                    keep = true;
                    kfx = fx;
                    kfy = fy;
                } else {
#pragma unroll
                    for (int v = 0; v < NV; ++v) sF(v, fy, fx) = Fs[v];
                }
            }
        }
    }
    if constexpr (MODE == MODE_RECON) return;
    if constexpr (SHARE) {
        __syncthreads();   // the traces are read; the flux tile overwrites them
        if (keep) {
#pragma unroll
            for (int v = 0; v < NV; ++v) sF(v, kfy, kfx) = Fkeep[v];
        }
    }
    __syncthreads();

    // phase 3: flux differences and (second sweep) the stage update
    const double dt = (MODE == MODE_FUSED_Y) ? *a.dt : 0.0;
    for (int it = tid; it < T0 * T1; it += NT) {
        const int cx = it % T0, cy = it / T0;
        const int x = i0 + cx, y = j0 + cy;
        if (x >= a.nx || y >= a.ny) continue;
        const long long pos = (long long)(y + a.ng) * a.ld + x + a.ng;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const long long e = v * a.plane + pos;
            if constexpr (DIR == 0) {
                const double d = -(sF(v, cy, cx + 1) - sF(v, cy, cx)) * a.inv_dx;
                a.Res[e] = d;
            } else {
                const double d = -(sF(v, cy + 1, cx) - sF(v, cy, cx)) * a.inv_dy;
                const double L = a.Res[e] + d;
                const double Un = a.Un[e];
                double o;
                if (a.stage == 1) o = Un + dt * L;
                else if (a.stage == 2) o = 0.75 * Un + 0.25 * a.U[e] + 0.25 * dt * L;
                else o = (1.0 / 3.0) * Un + (2.0 / 3.0) * a.U[e] + (2.0 / 3.0) * dt * L;
                a.Uout[e] = o;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 1D stage on one tile of T cells: reconstruction, strengths, LF flux and
// update in one pass (MODE_FUSED_1D), or the face states only (MODE_RECON).
// The same device routine serves the grid kernel (one tile per workgroup) and
// the batched persistent kernel (a workgroup walks the tiles of its
// instances).
// ---------------------------------------------------------------------------
struct Tile1D {
    const double *U;       // stage input (ghosts filled), variable stride `plane`
    const double *sx;      // strengths read by this stage
    double *sig_out;       // strengths written at the flux faces
    const double *Un;      // step-start state
    double *Uout;          // stage output
    double *wl, *wr;       // MODE_RECON outputs (may be null)
    int8_t *level;
    long long plane;
    int nx, ng, NX, nfaces, stage;
    double inv_dx, dt;
};

template <int R, int T>
struct Lds1D {
    static constexpr int UX = T + 2 + 2 * R;
    double sU[3][UX];
    double sS[UX];
    double sTR[3][T + 2];
    double sTL[3][T + 2];
    double sF[3][T + 1];
};

// The step-start state of this lane's cell, for the stage combination
// (loaded before the tile's window, used after the flux phase).
template <int T, int NT, int MODE>
__device__ __forceinline__ void stage1d_prefetch(const Tile1D &a, int i0, double (&un)[3])
{
    static_assert(T <= NT, "one cell of the tile per lane");
    const int tid = threadIdx.x;
#pragma unroll
    for (int v = 0; v < 3; ++v) un[v] = 0.0;
    if constexpr (MODE != MODE_RECON) {
        if (tid < T && i0 + tid < a.nx && a.stage > 1) {
#pragma unroll
            for (int v = 0; v < 3; ++v) un[v] = a.Un[v * a.plane + i0 + tid + a.ng];
        }
    }
}

// SSP-RK3 stage combination (Sec. 2.1) of one value from the step-start
// value un, the stage input us and the residual Lx, with its multiply-adds
// written out: every kernel that updates a 1D cell rounds it alike,
// whatever the compiler would contract in its context.
__device__ __forceinline__ double rk3_combine(int stage, double un, double us, double dt, double Lx)
{
    if (stage == 1) return fma(dt, Lx, us);
    if (stage == 2) return fma(0.25 * dt, Lx, fma(0.75, un, 0.25 * us));
    return fma((2.0 / 3.0) * dt, Lx, fma(1.0 / 3.0, un, (2.0 / 3.0) * us));
}

// The phases of a tile once its window (state and strengths) is in LDS:
// reconstruct the T + 2 cells whose face values the tile's faces need, LF
// flux at the T + 1 faces, then the stage combination of the T cells.
// With LAM, lam returns the signal-speed sum (|u| + c) / dx of this lane's
// new cell (0 for a lane without one).  With LDS_OUT the new values of all
// T cells replace the stage input in L.sU (each lane its own cell, after the
// flux phase) and nothing is written to memory: the caller keeps a whole
// step in LDS and makes sure a.nx lets every cell through.
template <int R, int T, int NT, int MODE, bool LAM = false, bool LDS_OUT = false>
__device__ __forceinline__ void stage1d_compute(const Tile1D &a, int i0, const MethodConst &mc, Lds1D<R, T> &L,
                                                const double (&un)[3], double &lam)
{
    constexpr int NV = 3, OI = R - 1;
    const int tid = threadIdx.x;
    const int ox = i0 - 1 - R;
    const bool want_sigma = (mc.flags & ASE_FLAG_DF_FIRST_ORDER) == 0;
    lam = 0.0;

    for (int tx = tid; tx < T + 2; tx += NT) {
        const int lx = tx + R;
        const int x = ox + lx;
        if (x > a.nx) continue;
        double s[2 * R];
#pragma unroll
        for (int m = -R; m < R; ++m) s[m + R] = L.sS[lx + m];
        auto ld = [&](int v, int m) { return L.sU[v][lx + m]; };
        double out[NV][2];
        const int lvl = reconstruct_cell<R, NV, 2>(ld, s, mc, OI, 0, out);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            L.sTR[v][tx] = out[v][0];
            L.sTL[v][tx] = out[v][1];
        }
        if (MODE == MODE_RECON && a.level != nullptr && x >= 0 && x < a.nx) a.level[x] = (int8_t)lvl;
    }
    __syncthreads();

    for (int fx = tid; fx < T + 1; fx += NT) {
        const int x = i0 - 1 + fx;   // face x + 1/2
        if (x > a.nx - 1) continue;
        double Wl[NV], Wr[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Wl[v] = L.sTR[v][fx];
            Wr[v] = L.sTL[v][fx + 1];
        }
        if constexpr (MODE == MODE_RECON) {
            if (a.wl != nullptr) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    a.wl[(long long)v * a.nfaces + x + 1] = Wl[v];
                    a.wr[(long long)v * a.nfaces + x + 1] = Wr[v];
                }
            }
        } else {
            double F[NV];
            auto cl = [&](int v) { return L.sU[v][fx + R]; };
            auto cr = [&](int v) { return L.sU[v][fx + R + 1]; };
            const double sg = gauss_point<NV>(Wl, Wr, cl, cr, 0, mc, F, want_sigma);
#pragma unroll
            for (int v = 0; v < NV; ++v) L.sF[v][fx] = F[v];
            if (want_sigma && (fx > 0 || i0 == 0)) a.sig_out[x + a.ng] = sg;
        }
    }
    if constexpr (MODE == MODE_RECON) return;
    __syncthreads();

    const double dt = a.dt;
    const int cx = tid, x = i0 + cx;
    if constexpr (LDS_OUT) {
        if (cx < T) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double Lx = -(L.sF[v][cx + 1] - L.sF[v][cx]) * a.inv_dx;
                L.sU[v][cx + R + 1] = rk3_combine(a.stage, un[v], L.sU[v][cx + R + 1], dt, Lx);
            }
        }
        return;
    }
    if (cx < T && x < a.nx) {
        double W[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const long long e = v * a.plane + x + a.ng;
            const double Lx = -(L.sF[v][cx + 1] - L.sF[v][cx]) * a.inv_dx;
            // the stage input is U^n in stage 1
            const double o = rk3_combine(a.stage, un[v], L.sU[v][cx + R + 1], dt, Lx);
            a.Uout[e] = o;
            W[v] = o;
        }
        if constexpr (LAM) {
            const Prim q = primitives<NV>(W, 0, mc);
            lam = (fabs(q.un) + q.c) * a.inv_dx;
        }
    }
}

template <int R, int T, int NT, int MODE>
__device__ __forceinline__ void stage1d_tile(const Tile1D &a, int i0, const MethodConst &mc, Lds1D<R, T> &L)
{
    constexpr int NV = 3;
    constexpr int UX = Lds1D<R, T>::UX;
    const int tid = threadIdx.x;
    const int ox = i0 - 1 - R;
    double un[NV];
    stage1d_prefetch<T, NT, MODE>(a, i0, un);
    for (int lx = tid; lx < UX; lx += NT) {
        const int I = ox + lx + a.ng;
        const bool in = I < a.NX;
#pragma unroll
        for (int v = 0; v < NV; ++v) L.sU[v][lx] = in ? a.U[v * a.plane + I] : 0.0;
        L.sS[lx] = in ? a.sx[I] : 0.0;
    }
    __syncthreads();
    double lam;
    stage1d_compute<R, T, NT, MODE>(a, i0, mc, L, un, lam);
}

template <int R, int T, int MODE>
__global__ void __launch_bounds__(kThreads) k_stage1d(SweepArgs a)
{
    __shared__ Lds1D<R, T> L;
    const int i0 = blockIdx.x * T;
    if (MODE != MODE_RECON && a.skip != nullptr && *a.skip != 0.0) {
        for (int fx = threadIdx.x; fx < T + 1; fx += kThreads) {
            const int x = i0 - 1 + fx;
            if (x > a.nx - 1) continue;
            if (fx > 0 || i0 == 0) a.sig_out[x + a.ng] = a.sx[x + a.ng];
        }
        return;
    }
    Tile1D t;
    t.U = a.U; t.sx = a.sx; t.sig_out = a.sig_out; t.Un = a.Un; t.Uout = a.Uout;
    t.wl = a.wl; t.wr = a.wr; t.level = a.level;
    t.plane = a.plane; t.nx = a.nx; t.ng = a.ng; t.NX = a.NX; t.nfaces = a.nfaces; t.stage = a.stage;
    t.inv_dx = a.inv_dx;
    t.dt = (MODE == MODE_RECON) ? 0.0 : *a.dt;
    stage1d_tile<R, T, kThreads, MODE>(t, i0, a.mc, L);
}

// ---------------------------------------------------------------------------
// Batched persistent 1D kernel: every workgroup walks the instances of its
// bin (a packing computed on the host) and advances each one through all
// its steps -- ghost cells, DF state, its own dt, three stages over tiles of
// T cells -- without leaving the kernel.  Instances are independent, so no
// workgroup ever waits for another.
// ---------------------------------------------------------------------------
struct BatchArgs {
    const long long *offsets;   // first stored cell of each instance
    const int *ncells;
    const double *dx;
    double *U, *sig, *t, *dt_hist;
    const double *dt_in;        // optional [nsteps][ninst]: replayed time steps instead of the CFL rule
    int *status;                // optional [ninst]: 0, or s+1 if the instance stopped at step s
    double *U1, *U2, *sig2;     // workspace, same layout as U / sig
    const int *bin_start, *bin_list;
    const int *bc_inst;         // optional per-instance boundary code (else `bc` for all)
    const int *only;            // k_batched_sigma_init: optional [ninst], instances with only[k] > 0
    long long total;
    int ninst, ng, nsteps, bc, fo;
    double t_end, cfl, dt_cap;
    MethodConst mc;
};

// Boundary code of instance k: periodic, reflective, anything else
// transmissive.
__device__ __forceinline__ int inst_bc(const int *bc_inst, int bc, int k)
{
    const int b = bc_inst ? bc_inst[k] : bc;
    return (b == ASE_BC_PERIODIC || b == ASE_BC_REFLECTIVE) ? b : ASE_BC_TRANSMISSIVE;
}

// Ghost cells of one instance and the strengths its stage reads.
template <int NT>
__device__ __forceinline__ void batched_fill(const BatchArgs &a, int bc, double *U, double *sg, int N,
                                             const MethodConst &mc)
{
    const int ng = a.ng, NX = N + 2 * ng;
    const long long P = a.total;
    for (int k = threadIdx.x; k < 2 * ng; k += NT) {
        const int I = k < ng ? k : N + k;
        int Is;
        if (bc == ASE_BC_PERIODIC) Is = k < ng ? I + N : I - N;
        else if (bc == ASE_BC_REFLECTIVE) Is = k < ng ? 2 * ng - 1 - I : 2 * (N + ng) - 1 - I;
        else Is = k < ng ? ng : ng + N - 1;
        const double fm = bc == ASE_BC_REFLECTIVE ? -1.0 : 1.0;   // momentum sign at a wall
        U[I] = U[Is];
        U[P + I] = fm * U[P + Is];
        U[2 * P + I] = U[2 * P + Is];
    }
    __syncthreads();
    if (a.fo) {
        // every face from the cell averages beside it; each lane forms the
        // primitive variables of its cell once and takes its right
        // neighbour's from the next lane (the last lane of a wave forms them
        // itself).  Uniform trip count: all lanes take part in the swaps.
        for (int I0 = 0; I0 + 1 < NX; I0 += NT) {
            const int I = I0 + threadIdx.x;
            double Wa[3];
#pragma unroll
            for (int v = 0; v < 3; ++v) Wa[v] = I < NX ? U[v * P + I] : 1.0;
            const Prim qa = primitives<3>(Wa, 0, mc);
            Prim qb;
            qb.p = __shfl_down(qa.p, 1);
            qb.un = __shfl_down(qa.un, 1);
            qb.ut = __shfl_down(qa.ut, 1);
            qb.ic = __shfl_down(qa.ic, 1);
            qb.c = 0.0;
            qb.ok = __shfl_down((int)qa.ok, 1) != 0;
            if ((threadIdx.x & 63) == 63 && I + 1 < NX) {
                double Wb[3];
#pragma unroll
                for (int v = 0; v < 3; ++v) Wb[v] = U[v * P + I + 1];
                qb = primitives<3>(Wb, 0, mc);
            }
            if (I + 1 < NX) sg[I] = sigma_point(qa, qb);
        }
        __syncthreads();
        return;
    }
    for (int I = threadIdx.x; I + 1 < NX; I += NT) {
        const int f = I - ng;
        const bool produced = f >= -1 && f <= N - 1;
        if (!produced) {
            if (bc == ASE_BC_PERIODIC) {
                sg[I] = sg[((f % N) + N) % N + ng];
            } else if (bc == ASE_BC_REFLECTIVE) {
                sg[I] = sg[(f < -1 ? -f - 2 : 2 * N - f - 2) + ng];   // mirror face at a wall
            } else {
                double Wa[3], Wb[3];
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    Wa[v] = U[v * P + I];
                    Wb[v] = U[v * P + I + 1];
                }
                sg[I] = sigma_point(primitives<3>(Wa, 0, mc), primitives<3>(Wb, 0, mc));
            }
        }
    }
    __syncthreads();
}

template <int R, int NT>
__global__ void __launch_bounds__(NT) k_batched1d(BatchArgs a)
{
    // tile of NT - 2R - 2 cells: every per-cell and per-face loop of a tile
    // then takes one pass of the workgroup (a longer tile runs a second pass
    // on one wave while the others wait at the next barrier)
    constexpr int T = NT - 2 * R - 2;
    __shared__ Lds1D<R, T> L;
    __shared__ double red[NT / 64];
    __shared__ double s_dt;
    const MethodConst &mc = a.mc;
    for (int b = a.bin_start[blockIdx.x]; b < a.bin_start[blockIdx.x + 1]; ++b) {
        const int k = a.bin_list[b];
        const long long off = a.offsets[k];
        const int N = a.ncells[k];
        if (N < 1 || off < 0 || off + N + 2LL * a.ng > a.total) continue;   // malformed entry: skipped
        const int bc = inst_bc(a.bc_inst, a.bc, k);
        double *U = a.U + off, *U1 = a.U1 + off, *U2 = a.U2 + off;
        double *sA = a.sig + off, *sB = a.sig2 + off;
        const double inv_dx = 1.0 / a.dx[k];
        double t = a.t[k];
        if (a.status != nullptr && threadIdx.x == 0) a.status[k] = 0;
        int s = 0;
        for (; s < a.nsteps; ++s) {
            if (a.t_end > 0.0 && t >= a.t_end) break;
            batched_fill<NT>(a, bc, U, sA, N, mc);
            if (a.dt_in) {
                const double dtr = a.dt_in[(long long)s * a.ninst + k];
                if (!(dtr > 0.0)) break;
                if (threadIdx.x == 0) s_dt = dtr;
                __syncthreads();
            } else {
                // dt from the signal speeds of this instance
                double lam = 0.0;
                for (int i = threadIdx.x; i < N; i += NT) {
                    double W[3];
#pragma unroll
                    for (int v = 0; v < 3; ++v) W[v] = U[v * a.total + i + a.ng];
                    const Prim q = primitives<3>(W, 0, mc);
                    const double l = (fabs(q.un) + q.c) * inv_dx;
                    lam = max_nan(lam, l);
                }
                // the maximum is exact and NaN-sticky in any order: lanes of a
                // wave first, then the waves
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) lam = max_nan(lam, __shfl_xor(lam, o));
                if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lam;
                __syncthreads();
                if (threadIdx.x == 0) {
                    double m = red[0];
                    for (int w = 1; w < NT / 64; ++w) m = max_nan(m, red[w]);
                    double dt = a.cfl / m;
                    if (a.dt_cap > 0.0 && dt > a.dt_cap) dt = a.dt_cap;
                    if (a.t_end > 0.0 && t + dt > a.t_end) dt = a.t_end - t;
                    s_dt = dt;
                }
                __syncthreads();
            }
            const double dt = s_dt;
            if (a.status != nullptr && !a.dt_in && !(dt > 0.0)) {
                // a signal speed of the state is NaN (rho <= 0 or p <= 0
                // somewhere): the instance stops here and says so
                if (threadIdx.x == 0) a.status[k] = s + 1;
                break;
            }
            double *in_st[3] = {U, U1, U2};
            double *out_st[3] = {U1, U2, U};
            for (int st = 0; st < 3; ++st) {
                double *sin = (st == 1) ? sB : sA;
                double *sout = (st == 1) ? sA : sB;
                if (st > 0) batched_fill<NT>(a, bc, in_st[st], sin, N, mc);
                Tile1D tl;
                tl.U = in_st[st]; tl.sx = sin; tl.sig_out = sout; tl.Un = U; tl.Uout = out_st[st];
                tl.wl = tl.wr = nullptr; tl.level = nullptr;
                tl.plane = a.total; tl.nx = N; tl.ng = a.ng; tl.NX = N + 2 * a.ng; tl.nfaces = N + 1;
                tl.stage = st + 1; tl.inv_dx = inv_dx; tl.dt = dt;
                for (int i0 = 0; i0 < N; i0 += T) {
                    stage1d_tile<R, T, NT, MODE_FUSED_1D>(tl, i0, mc, L);
                    __syncthreads();
                }
            }
            // the new strengths are in sB: swap the roles
            double *tmp = sA;
            sA = sB;
            sB = tmp;
            t += dt;
            if (threadIdx.x == 0 && a.dt_hist) a.dt_hist[(long long)s * a.ninst + k] = dt;
            __syncthreads();
        }
        // first-order source: hand back the strengths of the final state
        if (a.fo && a.nsteps > 0) batched_fill<NT>(a, bc, U, sA, N, mc);
        if (threadIdx.x == 0) {
            a.t[k] = t;
            if (a.dt_hist)
                for (int r = s; r < a.nsteps; ++r) a.dt_hist[(long long)r * a.ninst + k] = 0.0;
        }
        if (sA != a.sig + off) {
            // the N + 2 ng - 1 stored faces; the last stored cell has no face
            // on its right, so its entry is neither written nor copied
            for (int I = threadIdx.x; I + 1 < N + 2 * a.ng; I += NT) a.sig[off + I] = sA[I];
        }
        __syncthreads();
    }
}

// First-order strengths of every instance (one workgroup per instance).
template <int NT>
__global__ void __launch_bounds__(NT) k_batched_sigma_init(BatchArgs a)
{
    const int k = blockIdx.x;
    if (a.only != nullptr && a.only[k] < 1) return;
    const long long off = a.offsets[k];
    const int N = a.ncells[k];
    if (N < 1 || off < 0 || off + N + 2LL * a.ng > a.total) return;
    BatchArgs b = a;
    b.fo = 1;
    batched_fill<NT>(b, inst_bc(a.bc_inst, a.bc, k), a.U + off, a.sig + off, N, a.mc);
}

// ---------------------------------------------------------------------------
// Wide form of the batched step for the largest instances: one launch per
// stage over all their tiles (many workgroups per instance, the launch
// boundary as the only barrier), beside the persistent launch that keeps the
// others.  First-order DF source only.  A tile loads its window of the stage
// input with the ghost cells taken from their boundary-mapped interior
// cells (the values batched_fill writes there), forms every strength of the
// window from the two cell averages beside the face, and runs the same
// stage as stage1d_tile.  The time step of an instance comes from the
// signal-speed maxima its tiles left (the prep launch from the initial
// state, each stage-3 launch from the new state): every tile of the
// instance forms the same dt, its first tile records it.
// ---------------------------------------------------------------------------
struct WideArgs {
    const long long *offsets;
    const int *ncells;
    const double *dx;
    double *U, *U1, *U2;
    double *t, *dt_hist;
    const double *dt_in;
    int *status;
    const int *bc_inst;
    const int *tile_inst, *tile_i0, *inst_tile0, *inst_ntiles;
    double *lam;       // [ntiles]: signal-speed maximum of each tile's cells
    double *dt_cur;    // [ninst]: the time step of the current step
    int *done;         // [ninst]: the instance has stopped
    long long total;
    int ninst, ntiles, ng, bc, step, stage;   // stage 0: prep
    int nsteps;                               // steps of the call (one-launch-per-step form)
    double t_end, cfl, dt_cap;
    MethodConst mc;
};

// The instance's tiles are those of a plan for this tile length T: tile b is
// number b - t0 at j T, the last one at (nt - 1) T, and they cover the N
// cells exactly once.  Every tile of an instance takes the same decision
// from the last tile's entry (a plan for another length is skipped as a
// whole: its instances do not advance).
__device__ __forceinline__ bool wide_tiles_fit(const WideArgs &a, int b, int i0, int t0, int nt, int N, int T)
{
    const long long last = (long long)(nt - 1) * T;
    return a.tile_i0[t0 + nt - 1] == last && last < N && N <= last + T && i0 == (long long)(b - t0) * T;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double *red)
{
    // the maximum is exact and NaN-sticky in any order: lanes, then waves
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max_nan(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) m = max_nan(m, red[w]);
    return m;
}

// Stage input u (instance base, ghost slots not read) at cell x in
// [-ng, N + ng): ghosts mapped as batched_fill copies them (periodic image,
// wall mirror with the momentum reversed, or the boundary cell); 0 beyond.
__device__ __forceinline__ void mapped_cell(const double *u, long long P, int N, int ng, int bc, int x,
                                            double (&W)[3])
{
    double fm = 1.0;
    const bool in_range = x >= -ng && x < N + ng;
    if (x < 0 || x >= N) {
        if (bc == ASE_BC_PERIODIC) x = x < 0 ? x + N : x - N;
        else if (bc == ASE_BC_REFLECTIVE) {
            x = x < 0 ? -1 - x : 2 * N - 1 - x;
            fm = -1.0;
        } else x = x < 0 ? 0 : N - 1;
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) W[v] = in_range ? u[v * P + ng + x] : 0.0;
    W[1] *= fm;
}

// The window x in [i0-1-R, i0+T+1+R) of the stage input u into L.sU (one
// cell per lane: the window is NT cells long) and the first-order strength
// of the face on each window cell's right into L.sS: the neighbour's
// primitive variables from the next lane (the last lane of a wave forms them
// itself), as in batched_fill.  Ends with a barrier.
template <int R, int NT>
__device__ __forceinline__ void wide_window(const double *u, long long P, int N, int ng, int bc, int i0,
                                            const MethodConst &mc, Lds1D<R, NT - 2 * R - 2> &L)
{
    constexpr int UX = Lds1D<R, NT - 2 * R - 2>::UX;
    static_assert(UX == NT, "one window cell per lane");
    const int tid = threadIdx.x;
    const int ox = i0 - 1 - R;
    double W[3];
    mapped_cell(u, P, N, ng, bc, ox + tid, W);
#pragma unroll
    for (int v = 0; v < 3; ++v) L.sU[v][tid] = W[v];
    const Prim qa = primitives<3>(W, 0, mc);
    Prim qb;
    qb.p = __shfl_down(qa.p, 1);
    qb.un = __shfl_down(qa.un, 1);
    qb.ut = __shfl_down(qa.ut, 1);
    qb.ic = __shfl_down(qa.ic, 1);
    qb.c = 0.0;
    qb.ok = __shfl_down((int)qa.ok, 1) != 0;
    if ((tid & 63) == 63 && tid + 1 < UX) {
        double Wb[3];
        mapped_cell(u, P, N, ng, bc, ox + tid + 1, Wb);
        qb = primitives<3>(Wb, 0, mc);
    }
    if (tid + 1 < UX) L.sS[tid] = sigma_point(qa, qb);
    __syncthreads();
}

template <int R, int NT>
__global__ void __launch_bounds__(NT) k_batched_wide(WideArgs a)
{
    constexpr int T = NT - 2 * R - 2;
    __shared__ Lds1D<R, T> L;
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int k = a.tile_inst[b], i0 = a.tile_i0[b];
    if (k < 0 || k >= a.ninst) return;   // malformed tile entry: skipped (the whole workgroup)
    const int N = a.ncells[k], ng = a.ng;
    const long long off = a.offsets[k], P = a.total;
    const int t0 = a.inst_tile0[k], nt = a.inst_ntiles[k];
    if (N < T || off < 0 || off + N + 2LL * ng > P || i0 < 0 || i0 >= N || t0 < 0 || nt < 1 ||
        t0 + nt > a.ntiles || b < t0 || b >= t0 + nt || !wide_tiles_fit(a, b, i0, t0, nt, N, T))
        return;
    const bool first = b == t0;
    const double inv_dx = 1.0 / a.dx[k];
    const MethodConst &mc = a.mc;

    if (a.stage == 0) {
        // prep: the instance runs, and the signal speeds of its initial state
        double l = 0.0;
        const int x = i0 + tid;
        if (tid < T && x < N) {
            double W[3];
#pragma unroll
            for (int v = 0; v < 3; ++v) W[v] = a.U[v * P + off + ng + x];
            const Prim q = primitives<3>(W, 0, mc);
            l = (fabs(q.un) + q.c) * inv_dx;
        }
        const double m = block_max<NT>(l, red);
        if (tid == 0) {
            a.lam[b] = m;
            if (first) {
                a.done[k] = 0;
                if (a.status != nullptr) a.status[k] = 0;
            }
        }
        return;
    }
    const int s = a.step;
    const long long hs = (long long)s * a.ninst + k;
    if (a.done[k]) {
        if (a.stage == 1 && first && tid == 0 && a.dt_hist) a.dt_hist[hs] = 0.0;
        return;
    }
    double dt;
    if (a.stage == 1) {
        const double t = a.t[k];
        bool stop = a.t_end > 0.0 && t >= a.t_end;
        dt = 0.0;
        if (!stop && a.dt_in) {
            dt = a.dt_in[hs];
            stop = !(dt > 0.0);
        } else if (!stop) {
            double m = 0.0;
            for (int j = tid; j < nt; j += NT) m = max_nan(m, a.lam[t0 + j]);
            m = block_max<NT>(m, red);
            dt = a.cfl / m;
            if (a.dt_cap > 0.0 && dt > a.dt_cap) dt = a.dt_cap;
            if (a.t_end > 0.0 && t + dt > a.t_end) dt = a.t_end - t;
            if (a.status != nullptr && !(dt > 0.0)) {
                // a signal speed of the state is NaN: the instance stops here
                if (first && tid == 0) a.status[k] = s + 1;
                stop = true;
            }
        }
        if (stop) {
            if (first && tid == 0) {
                a.done[k] = 1;
                if (a.dt_hist) a.dt_hist[hs] = 0.0;
            }
            return;
        }
        if (first && tid == 0) a.dt_cur[k] = dt;
    } else {
        dt = a.dt_cur[k];
    }

    double *in = a.stage == 1 ? a.U : a.stage == 2 ? a.U1 : a.U2;
    double *out = a.stage == 1 ? a.U1 : a.stage == 2 ? a.U2 : a.U;
    Tile1D tl;
    tl.U = in + off; tl.sx = nullptr; tl.sig_out = nullptr; tl.Un = a.U + off; tl.Uout = out + off;
    tl.wl = tl.wr = nullptr; tl.level = nullptr;
    tl.plane = P; tl.nx = N; tl.ng = ng; tl.NX = N + 2 * ng; tl.nfaces = N + 1;
    tl.stage = a.stage; tl.inv_dx = inv_dx; tl.dt = dt;
    double un[3];
    stage1d_prefetch<T, NT, MODE_FUSED_1D>(tl, i0, un);

    wide_window<R, NT>(in + off, P, N, ng, inst_bc(a.bc_inst, a.bc, k), i0, mc, L);
    double l;
    if (a.stage == 3) {
        stage1d_compute<R, T, NT, MODE_FUSED_1D, true>(tl, i0, mc, L, un, l);
        const double m = block_max<NT>(l, red);
        if (tid == 0) {
            a.lam[b] = m;
            if (first) {
                a.t[k] = a.t[k] + dt;
                if (a.dt_hist) a.dt_hist[hs] = dt;
            }
        }
    } else {
        stage1d_compute<R, T, NT, MODE_FUSED_1D>(tl, i0, mc, L, un, l);
    }
}

// ---------------------------------------------------------------------------
// Wide form with one launch per step.  A tile's window reaches 3 (R + 1)
// cells beyond the cells it owns on each side, the reach of three stages, so
// the tile runs all three RK stages in LDS and writes only its own cells of
// the new state.  Ghost cells of walls and open ends are taken again from
// their mapped cells of the window before each stage (a window that holds a
// ghost also holds its mapped cells, far enough inside to be exact at that
// stage); on a periodic instance the window simply wraps round, and a tile
// computes the wrapped cells itself from the same values the tile owning
// them uses.  Cells of the window whose inputs reach beyond it are computed
// from garbage and never used.  An instance shorter than a tile is one tile
// whose window holds all of it and its ghost cells (periodic and wall
// instances have at least ng cells, as everywhere).  The state and the
// instance times alternate between two buffers from step to step
// (neighbouring tiles read the halo of the step's input while others write
// the output), arranged so that the call's last step writes U and t; the
// per-tile signal-speed maxima alternate likewise.  Every output equals the per-stage form's and the
// persistent launch's bit for bit: each cell value is formed by the same
// operations on the same operands.
// ---------------------------------------------------------------------------

// Stage input u (instance base) at window cell x of a step's window: the
// periodic image of any x, or as mapped_cell for walls and open ends.
__device__ __forceinline__ void step_cell(const double *u, long long P, int N, int ng, int bc, int x,
                                          double (&W)[3])
{
    if (bc == ASE_BC_PERIODIC) {
        int xm = x % N;
        if (xm < 0) xm += N;
#pragma unroll
        for (int v = 0; v < 3; ++v) W[v] = u[v * P + ng + xm];
    } else {
        mapped_cell(u, P, N, ng, bc, x, W);
    }
}

// Window position p (cell x) of the stage values in LDS; a ghost cell of a
// wall or open end (x in [-ng, 0) or [N, N + ng)) reads its mapped cell of
// the window instead.  Returns whether p is such a ghost.
template <int R, int T>
__device__ __forceinline__ bool step_lds_cell(const Lds1D<R, T> &L, int p, int x, int N, int ng, int bc,
                                              double (&W)[3])
{
    constexpr int UX = Lds1D<R, T>::UX;
    int q = p;
    double fm = 1.0;
    const bool ghost = bc != ASE_BC_PERIODIC && ((x >= -ng && x < 0) || (x >= N && x < N + ng));
    if (ghost) {
        int y;
        if (bc == ASE_BC_REFLECTIVE) {
            y = x < 0 ? -1 - x : 2 * N - 1 - x;
            fm = -1.0;
        } else {
            y = x < 0 ? 0 : N - 1;
        }
        q = p + (y - x);
        q = q < 0 ? 0 : (q > UX - 1 ? UX - 1 : q);
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) W[v] = L.sU[v][q];
    W[1] *= fm;
    return ghost;
}

// First-order strength of the face on the right of window position tid from
// W (this lane's cell) and the next lane's cell (next: the last lane of a
// wave forms that one itself), as wide_window does.
template <int R, int T>
__device__ __forceinline__ void step_sigma(Lds1D<R, T> &L, const double (&W)[3], const double (&Wn)[3],
                                           const MethodConst &mc)
{
    constexpr int UX = Lds1D<R, T>::UX;
    const int tid = threadIdx.x;
    const Prim qa = primitives<3>(W, 0, mc);
    Prim qb;
    qb.p = __shfl_down(qa.p, 1);
    qb.un = __shfl_down(qa.un, 1);
    qb.ut = __shfl_down(qa.ut, 1);
    qb.ic = __shfl_down(qa.ic, 1);
    qb.c = 0.0;
    qb.ok = __shfl_down((int)qa.ok, 1) != 0;
    if ((tid & 63) == 63 && tid + 1 < UX) qb = primitives<3>(Wn, 0, mc);
    if (tid + 1 < UX) L.sS[tid] = sigma_point(qa, qb);
}

// Bounded to five waves per SIMD (83 registers, no spills).  The three
// stages are unrolled: as a loop, the constants and branch masks the stage
// code keeps in scalar registers across it spilled 109 of them into vector
// lanes, and the step ran 5 % slower.
template <int R, int NT>
__global__ void __launch_bounds__(NT, 5) k_batched_wide_step(WideArgs a)
{
    constexpr int T = NT - 2 * R - 2;   // cells one stage updates: window positions R + 1 .. NT - R - 2
    constexpr int H = 3 * (R + 1);      // halo of the step's window
    constexpr int TS = NT - 2 * H;      // cells a tile owns
    static_assert(TS > H, "tile shorter than its halo");
    __shared__ Lds1D<R, T> L;
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int k = a.tile_inst[b], i0 = a.tile_i0[b];
    if (k < 0 || k >= a.ninst) return;   // malformed tile entry: skipped (the whole workgroup)
    const int N = a.ncells[k], ng = a.ng;
    const long long off = a.offsets[k], P = a.total;
    const int t0 = a.inst_tile0[k], nt = a.inst_ntiles[k];
    if (N < 1 || off < 0 || off + N + 2LL * ng > P || i0 < 0 || i0 >= N || t0 < 0 || nt < 1 ||
        t0 + nt > a.ntiles || b < t0 || b >= t0 + nt || a.nsteps < 1 || !wide_tiles_fit(a, b, i0, t0, nt, N, TS))
        return;
    const bool first = b == t0;
    const double inv_dx = 1.0 / a.dx[k];
    const MethodConst &mc = a.mc;
    const int bc = inst_bc(a.bc_inst, a.bc, k);
    // buffer A (U, t) takes the output of the call's last step
    double *tA = a.t, *tB = a.dt_cur;
    const int x = i0 + tid;              // this lane's owned cell, tid < TS
    const bool owns = tid < TS && x < N;

    if (a.stage == 0) {
        // prep: the instance runs, the signal speeds of its initial state,
        // and with an odd step count the state and time into buffer B
        const bool to_b = (a.nsteps & 1) != 0;
        double l = 0.0;
        if (owns) {
            double W[3];
#pragma unroll
            for (int v = 0; v < 3; ++v) W[v] = a.U[v * P + off + ng + x];
            if (to_b) {
#pragma unroll
                for (int v = 0; v < 3; ++v) a.U1[v * P + off + ng + x] = W[v];
            }
            const Prim q = primitives<3>(W, 0, mc);
            l = (fabs(q.un) + q.c) * inv_dx;
        }
        const double m = block_max<NT>(l, red);
        if (tid == 0) {
            a.lam[b] = m;
            if (first) {
                a.done[k] = 0;
                if (a.status != nullptr) a.status[k] = 0;
                if (to_b) tB[k] = tA[k];
            }
        }
        return;
    }
    const int s = a.step;
    const bool dst_a = ((a.nsteps - 1 - s) & 1) == 0;
    const double *X = (dst_a ? a.U1 : a.U) + off;
    double *Y = (dst_a ? a.U : a.U1) + off;
    const double t = dst_a ? tB[k] : tA[k];
    double *tdst = dst_a ? tA : tB;
    const double *lam_in = a.lam + (s & 1) * (long long)a.ntiles;
    double *lam_out = a.lam + ((s + 1) & 1) * (long long)a.ntiles;
    const long long hs = (long long)s * a.ninst + k;

    bool stop = a.done[k] != 0;
    double dt = 0.0;
    if (!stop) {
        stop = a.t_end > 0.0 && t >= a.t_end;
        if (!stop && a.dt_in) {
            dt = a.dt_in[hs];
            stop = !(dt > 0.0);
        } else if (!stop) {
            double m = 0.0;
            for (int j = tid; j < nt; j += NT) m = max_nan(m, lam_in[t0 + j]);
            m = block_max<NT>(m, red);
            dt = a.cfl / m;
            if (a.dt_cap > 0.0 && dt > a.dt_cap) dt = a.dt_cap;
            if (a.t_end > 0.0 && t + dt > a.t_end) dt = a.t_end - t;
            if (a.status != nullptr && !(dt > 0.0)) {
                // a signal speed of the state is NaN: the instance stops here
                if (first && tid == 0) a.status[k] = s + 1;
                stop = true;
            }
        }
    }
    if (stop) {
        // the state and time carry over to the other buffer unchanged
        if (owns) {
#pragma unroll
            for (int v = 0; v < 3; ++v) Y[v * P + ng + x] = X[v * P + ng + x];
        }
        if (first && tid == 0) {
            a.done[k] = 1;
            tdst[k] = t;
            if (a.dt_hist) a.dt_hist[hs] = 0.0;
        }
        return;
    }

    // the step's window of the input state, and the strengths of its faces
    const int ox = i0 - H;   // window position p holds cell ox + p
    {
        double W[3], Wn[3];
        step_cell(X, P, N, ng, bc, ox + tid, W);
        if ((tid & 63) == 63 && tid + 1 < NT) step_cell(X, P, N, ng, bc, ox + tid + 1, Wn);
#pragma unroll
        for (int v = 0; v < 3; ++v) L.sU[v][tid] = W[v];
        step_sigma<R, T>(L, W, Wn, mc);
    }
    __syncthreads();
    double un[3];   // U^n of the cell this lane updates (window position tid + R + 1)
#pragma unroll
    for (int v = 0; v < 3; ++v) un[v] = tid < T ? L.sU[v][tid + R + 1] : 0.0;

    Tile1D tl;
    tl.U = nullptr; tl.sx = nullptr; tl.sig_out = nullptr; tl.Un = nullptr; tl.Uout = nullptr;
    tl.wl = tl.wr = nullptr; tl.level = nullptr;
    tl.plane = P; tl.nx = 1 << 30; tl.ng = ng; tl.NX = 1 << 30; tl.nfaces = 1 << 30;
    tl.inv_dx = inv_dx; tl.dt = dt;
#pragma unroll
    for (int stg = 1; stg <= 3; ++stg) {
        if (stg > 1) {
            // ghost cells of the new stage values again, then the strengths
            double W[3], Wn[3];
            const bool g = step_lds_cell<R, T>(L, tid, ox + tid, N, ng, bc, W);
            if ((tid & 63) == 63 && tid + 1 < NT) step_lds_cell<R, T>(L, tid + 1, ox + tid + 1, N, ng, bc, Wn);
            if (g) {
#pragma unroll
                for (int v = 0; v < 3; ++v) L.sU[v][tid] = W[v];
            }
            step_sigma<R, T>(L, W, Wn, mc);
            __syncthreads();
        }
        tl.stage = stg;
        double l;
        stage1d_compute<R, T, NT, MODE_FUSED_1D, false, true>(tl, ox + R + 1, mc, L, un, l);
        __syncthreads();
    }

    double l = 0.0;
    if (owns) {
        double W[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            W[v] = L.sU[v][H + tid];
            Y[v * P + ng + x] = W[v];
        }
        const Prim q = primitives<3>(W, 0, mc);
        l = (fabs(q.un) + q.c) * inv_dx;
    }
    const double m = block_max<NT>(l, red);
    if (tid == 0) {
        lam_out[b] = m;
        if (first) {
            tdst[k] = t + dt;
            if (a.dt_hist) a.dt_hist[hs] = dt;
        }
    }
}

// ---------------------------------------------------------------------------
// Discrete adjoint of the 1D step.  Frozen decisions: the time step, the
// strengths every stage read (hence DF factors and stencil levels), the side
// that gives the LF signal speed and the positivity replacements.  Everything
// else is differentiated exactly, including the WENO-Z-AO weights and the
// ghost copies of the boundary conditions.
//
// One workgroup owns an instance: it first re-runs the forward steps of the
// segment from the checkpoint with the recorded time steps, keeping every
// stage input (state and strengths) in a tape, then walks the steps back:
//   mu2 = 2/3 lam + J(U2)^T (2/3 dt lam)
//   mu1 = 1/4 mu2 + J(U1)^T (1/4 dt mu2)
//   lam = 1/3 lam + 3/4 mu2 + mu1 + J(Un)^T (dt mu1)
// with J the Jacobian of the residual L.  Each J^T g is a tile pass:
// traces, transposed LF flux per face, then per variable the transposed
// reconstruction of each cell scattered as 2R+1 tap contributions and
// gathered per output cell (no atomics, fixed summation order).
// ---------------------------------------------------------------------------
template <int R, int T>
struct LdsAdj {
    static constexpr int H = 2 * R + 2;       // state window halo
    static constexpr int WX = T + 2 * H;      // window cells [i0-H, i0+T+H)
    static constexpr int NC = T + 2 * R + 2;  // trace cells [i0-R-1, i0+T+R]
    static constexpr int NF = NC - 1;         // faces between consecutive trace cells
    double sV[3][WX];
    double sGL[3][NF], sGR[3][NF];
    union {
        // window strengths, adjoint weights and face traces (trace, flux and
        // decision phases), then the tap contributions (tap and gather
        // phases)
        struct {
            double sS[WX];
            double sG[3][NC];
            double tr[3][NC], tl[3][NC];
        } t;
        double c[2 * R + 1][NC];
    } u;
    uint8_t rep[NF];
};

// LDS of one phase: the forward tiles for the tape, the transposed tiles
// for the reverse sweep (each phase is its own kernel and allocates only its
// own, so the tape runs at the forward kernel's occupancy)
template <int R, int T, int PH>
using LdsAdjPhase = std::conditional_t<PH == ASE_ADJ_TAPE, Lds1D<R, T>, LdsAdj<R, T>>;

struct AdjTile {
    const double *V, *S;   // stage input (ghosts filled) and the strengths the stage read
    const double *g;       // adjoint weights (interior)
    double gscale;         // stage coefficient x dt
    const double *a0, *a1, *a2;
    double c0, c1, c2;     // out = c0 a0 + c1 a1 + c2 a2 + J^T (gscale g)
    double *out;
    long long plane;
    int N, ng;
    double inv_dx;
};

template <int R, int T, int NT, bool UNROLL_V = false>
__device__ __forceinline__ void adjoint1d_tile(const AdjTile &a, int i0, const MethodConst &mc, LdsAdj<R, T> &L)
{
    using LA = LdsAdj<R, T>;
    constexpr int H = LA::H, WX = LA::WX, NC = LA::NC, NF = LA::NF;
    const int tid = threadIdx.x;
    const int NXs = a.N + 2 * a.ng;
    const int xw = i0 - H;       // first window cell
    const int xc = i0 - R - 1;   // first trace cell
    const long long P = a.plane;

    (void)xw;
    (void)NXs;
    (void)WX;
    // the window (state, strengths, weights) is in LDS: adj_stage staged it

    // face traces of the cells -1..N that lie in the trace range
    for (int c = tid; c < NC; c += NT) {
        const int x = xc + c;
        if (x < -1 || x > a.N) continue;
        const int lx = c + (H - R - 1);
        double s[2 * R];
#pragma unroll
        for (int m = -R; m < R; ++m) s[m + R] = L.u.t.sS[lx + m];
        auto ld = [&](int v, int m) { return L.sV[v][lx + m]; };
        double out[3][2];
        reconstruct_cell<R, 3, 2>(ld, s, mc, R - 1, 0, out);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            L.u.t.tr[v][c] = out[v][0];
            L.u.t.tl[v][c] = out[v][1];
        }
    }
    __syncthreads();

    // transposed LF flux of face x + 1/2 between trace cells f and f + 1
    for (int f = tid; f < NF; f += NT) {
        const int x = xc + f;
        double gl[3] = {0.0, 0.0, 0.0}, gr[3] = {0.0, 0.0, 0.0};
        uint8_t rp = 0;
        if (x >= -1 && x <= a.N - 1) {
            double h[3], Wl[3], Wr[3];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                h[v] = (L.u.t.sG[v][f + 1] - L.u.t.sG[v][f]) * a.inv_dx;
                Wl[v] = L.u.t.tr[v][f];
                Wr[v] = L.u.t.tl[v][f + 1];
            }
            Prim ql = primitives<3>(Wl, 0, mc);
            Prim qr = primitives<3>(Wr, 0, mc);
            if (mc.flags & 1) {
                const int lx = f + (H - R - 1);
                if (!ql.ok) {
#pragma unroll
                    for (int v = 0; v < 3; ++v) Wl[v] = L.sV[v][lx];
                    ql = primitives<3>(Wl, 0, mc);
                    rp |= 1;
                }
                if (!qr.ok) {
#pragma unroll
                    for (int v = 0; v < 3; ++v) Wr[v] = L.sV[v][lx + 1];
                    qr = primitives<3>(Wr, 0, mc);
                    rp |= 2;
                }
            }
            const double sl = fabs(ql.un) + ql.c, sr = fabs(qr.un) + qr.c;
            const bool takel = sl > sr;
            const double hs = 0.5 * (takel ? sl : sr);
            double dsl[3], dsr[3];
            euler1d_vjp(Wl, ql, mc, h, 0.5, gl, dsl);
            euler1d_vjp(Wr, qr, mc, h, 0.5, gr, dsr);
            double hd = 0.0;
#pragma unroll
            for (int v = 0; v < 3; ++v) hd += h[v] * (Wr[v] - Wl[v]);
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                gl[v] += hs * h[v] - (takel ? 0.5 * hd * dsl[v] : 0.0);
                gr[v] += -hs * h[v] - (takel ? 0.0 : 0.5 * hd * dsr[v]);
            }
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            L.sGL[v][f] = gl[v];
            L.sGR[v][f] = gr[v];
        }
        L.rep[f] = rp;
    }
    // frozen level and DF factors of this lane's trace cell (one per lane:
    // NC = NT), once for all three variables, kept in registers
    static_assert(NC == NT, "one trace cell per lane");
    int lev = 0;
    double dal[4] = {0.0, 0.0, 0.0, 0.0};
    {
        const int c = tid, x = xc + c;
        if (c >= 1 && c <= NC - 2 && x >= -1 && x <= a.N) {
            const int lx = c + (H - R - 1);
            double s[2 * R];
#pragma unroll
            for (int m = -R; m < R; ++m) s[m + R] = L.u.t.sS[lx + m];
            lev = cell_decisions<R>(s, mc, dal);
        }
    }
    __syncthreads();

    const bool first = i0 == 0, last = i0 + T >= a.N;
    auto var_pass = [&](int v) {
        // this lane's first gather cell: its stage-combination terms, loaded
        // now and used after the tap phase
        double pa0 = 0.0, pa1 = 0.0, pa2 = 0.0;
        {
            const int j = i0 - a.ng + tid;
            const bool interior = tid < T + 2 * a.ng && j >= i0 && j < i0 + T && j < a.N;
            if (interior) {
                const long long e = v * P + j + a.ng;
                pa0 = a.a0[e];
                if (a.a1) pa1 = a.a1[e];
                if (a.a2) pa2 = a.a2[e];
            }
        }
        // tap contributions of each cell: c[m][cell] feeds output cell + m
        for (int c = tid; c < NC; c += NT) {
            const int x = xc + c;
            double cc[2 * R + 1];
#pragma unroll
            for (int m = 0; m < 2 * R + 1; ++m) cc[m] = 0.0;
            if (c >= 1 && c <= NC - 2 && x >= -1 && x <= a.N) {
                double gR = 0.0, gL = 0.0, d = 0.0;
                if (x <= a.N - 1) {
                    if (L.rep[c] & 1) d += L.sGL[v][c];
                    else gR = L.sGL[v][c];
                }
                if (x >= 0) {
                    if (L.rep[c - 1] & 2) d += L.sGR[v][c - 1];
                    else gL = L.sGR[v][c - 1];
                }
                const int lx = c + (H - R - 1);
                recon_vjp_var<R>([&](int m) { return L.sV[v][lx + m]; }, lev, dal, mc, gR, gL, cc);
                cc[R] += d;
            }
#pragma unroll
            for (int m = 0; m < 2 * R + 1; ++m) L.u.c[m][c] = cc[m];
        }
        __syncthreads();
        for (int jj = tid; jj < T + 2 * a.ng; jj += NT) {
            const int j = i0 - a.ng + jj;
            const bool interior = j >= i0 && j < i0 + T && j < a.N;
            const bool ghost = (first && j < 0) || (last && j >= a.N && j < a.N + a.ng);
            if (!interior && !ghost) continue;
            double G = 0.0;
#pragma unroll
            for (int m = -R; m <= R; ++m) {
                const int c = j - m - xc;
                if (c >= 1 && c <= NC - 2) G += L.u.c[m + R][c];
            }
            const long long e = v * P + j + a.ng;
            if (interior) {
                const bool pre = jj == tid;
                double o = a.c0 * (pre ? pa0 : a.a0[e]);
                if (a.a1) o += a.c1 * (pre ? pa1 : a.a1[e]);
                if (a.a2) o += a.c2 * (pre ? pa2 : a.a2[e]);
                G += o;
            }
            a.out[e] = G;
        }
        __syncthreads();
    };
    if constexpr (UNROLL_V) {
        // straight-line: the tap phase's constants and branch masks are
        // formed where they are used instead of living in scalar registers
        // across a loop (which spilled them into vector lanes)
#pragma unroll
        for (int v = 0; v < 3; ++v) var_pass(v);
    } else {
#pragma unroll 1
        for (int v = 0; v < 3; ++v) var_pass(v);
    }
}

// Add the ghost-cell gradients of `out` onto the interior cells the ghosts
// copy (transmissive: the boundary cell; periodic: the wrapped cell).  One
// thread per variable and side; the ghost values are summed in registers so
// the target sees a single read-modify-write.
__device__ __forceinline__ void adj_fold(double *out, long long P, int N, int ng, int bc)
{
    const int v = threadIdx.x >> 1, side = threadIdx.x & 1;
    if (threadIdx.x < 6) {
        double *o = out + v * P;
        if (bc == ASE_BC_PERIODIC && N >= 2 * ng) {
            // distinct targets: left ghosts -> N-ng..N-1, right ghosts -> 0..ng-1
            for (int k = 0; k < ng; ++k) {
                if (side == 0) o[N + k] += o[k];
                else o[ng + k] += o[N + ng + k];
            }
        } else if (bc == ASE_BC_PERIODIC) {
            if (side == 0) {
                for (int k = 0; k < ng; ++k) {
                    const int tgt = k - ng + N;
                    if (tgt >= 0 && tgt < N) o[tgt + ng] += o[k];
                }
                for (int k = 0; k < ng; ++k) {
                    const int tgt = k;
                    if (tgt >= 0 && tgt < N) o[tgt + ng] += o[N + ng + k];
                }
            }
        } else if (bc == ASE_BC_REFLECTIVE) {
            // ghost storage k copies storage 2ng-1-k (left), N+ng+k copies
            // N+ng-1-k (right); the momentum gradient changes sign
            const double fm = v == 1 ? -1.0 : 1.0;
            if (side == 0) {
                if (N >= 2 * ng) {
                    for (int k = 0; k < ng; ++k) o[2 * ng - 1 - k] += fm * o[k];
                } else {
                    for (int k = 0; k < ng; ++k) o[2 * ng - 1 - k] += fm * o[k];
                    for (int k = 0; k < ng; ++k) o[N + ng - 1 - k] += fm * o[N + ng + k];
                }
            } else if (N >= 2 * ng) {
                for (int k = 0; k < ng; ++k) o[N + ng - 1 - k] += fm * o[N + ng + k];
            }
        } else if (N > 1) {
            double acc = 0.0;
            const int base = side == 0 ? 0 : N + ng;
            for (int k = 0; k < ng; ++k) acc += o[base + k];
            o[side == 0 ? ng : ng + N - 1] += acc;
        } else if (side == 0) {
            // one cell: both sides fold onto it
            double acc = 0.0;
            for (int k = 0; k < ng; ++k) acc += o[k] + o[N + ng + k];
            o[ng] += acc;
        }
    }
    __syncthreads();
}

struct AdjArgs {
    const long long *offsets;   // nullptr: one instance at offset 0 with n1 cells of width dx1
    const int *ncells;
    const double *dx;
    int n1;
    double dx1;
    const double *ck_U, *ck_sig;   // checkpoint at the segment start
    const double *dt_hist;         // [nsteps][ninst]; 0 = step not taken
    double *lam;                   // in: adjoint at the segment end; out: at its start
    double *mu1, *mu2;
    double *tapeU, *tapeS;         // [3 nsteps][3][total], [3 nsteps][total]
    const int *bin_start, *bin_list;   // nullptr: instance = workgroup
    const int *bc_inst;                // optional per-instance boundary code
    long long total;
    int ninst, ng, nsteps, bc, fo;
    int phase;                         // bit 1: record the tape; bit 2: reverse sweep
    MethodConst mc;
};

// Window of one adjoint tile held in registers: state and strengths of cells
// [i0-H, i0+T+H), weights of the trace cells.  Loaded for the next tile
// while the current one computes.
template <int R, int T, int NT>
struct AdjWin {
    static constexpr int NW = (LdsAdj<R, T>::WX + NT - 1) / NT;
    static constexpr int NG = (LdsAdj<R, T>::NC + NT - 1) / NT;
    double v[NW][4];
    double g[NG][3];
};

template <int R, int T, int NT>
__device__ __forceinline__ void adj_fetch(const AdjTile &a, int i0, AdjWin<R, T, NT> &w)
{
    using LA = LdsAdj<R, T>;
    const int tid = threadIdx.x, NXs = a.N + 2 * a.ng;
    const long long P = a.plane;
#pragma unroll
    for (int q = 0; q < AdjWin<R, T, NT>::NW; ++q) {
        const int lx = tid + q * NT;
        const int I = i0 - LA::H + lx + a.ng;
        const bool in = lx < LA::WX && I >= 0 && I < NXs;
#pragma unroll
        for (int v = 0; v < 3; ++v) w.v[q][v] = in ? a.V[v * P + I] : 0.0;
        w.v[q][3] = in ? a.S[I] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < AdjWin<R, T, NT>::NG; ++q) {
        const int c = tid + q * NT;
        const int x = i0 - R - 1 + c;
        const bool in = c < LA::NC && x >= 0 && x < a.N;
#pragma unroll
        for (int v = 0; v < 3; ++v) w.g[q][v] = in ? a.gscale * a.g[v * P + x + a.ng] : 0.0;
    }
}

template <int R, int T, int NT>
__device__ __forceinline__ void adj_stage_window(const AdjWin<R, T, NT> &w, LdsAdj<R, T> &L)
{
    using LA = LdsAdj<R, T>;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < AdjWin<R, T, NT>::NW; ++q) {
        const int lx = tid + q * NT;
        if (lx < LA::WX) {
#pragma unroll
            for (int v = 0; v < 3; ++v) L.sV[v][lx] = w.v[q][v];
            L.u.t.sS[lx] = w.v[q][3];
        }
    }
#pragma unroll
    for (int q = 0; q < AdjWin<R, T, NT>::NG; ++q) {
        const int c = tid + q * NT;
        if (c < LA::NC) {
#pragma unroll
            for (int v = 0; v < 3; ++v) L.u.t.sG[v][c] = w.g[q][v];
        }
    }
}

template <int R, int T, int NT>
__device__ __forceinline__ void adj_stage(AdjTile &t, const MethodConst &mc, LdsAdj<R, T> &L, int bc)
{
    AdjWin<R, T, NT> w;
    adj_fetch<R, T, NT>(t, 0, w);
    for (int i0 = 0; i0 < t.N; i0 += T) {
        adj_stage_window<R, T, NT>(w, L);   // the previous tile ended with a barrier
        __syncthreads();
        if (i0 + T < t.N) adj_fetch<R, T, NT>(t, i0 + T, w);
        adjoint1d_tile<R, T, NT>(t, i0, mc, L);
    }
    adj_fold(t.out, t.plane, t.N, t.ng, bc);
}

// The tape phase is the forward kernel's work: bounded to 128 registers
// (four waves per SIMD) like k_batched1d.
template <int R, int NT, int PH>
__global__ void __launch_bounds__(NT, PH == ASE_ADJ_TAPE ? 4 : 1) k_adjoint1d(AdjArgs a)
{
    static_assert(PH == ASE_ADJ_TAPE || PH == ASE_ADJ_REVERSE, "one phase per kernel");
    constexpr int T = NT - 2 * R - 2;   // trace cells of a tile = NT (one pass per phase)
    __shared__ LdsAdjPhase<R, T, PH> L;
    const MethodConst &mc = a.mc;
    const int tid = threadIdx.x;
    const int b0 = a.bin_start ? a.bin_start[blockIdx.x] : (int)blockIdx.x;
    const int b1 = a.bin_start ? a.bin_start[blockIdx.x + 1] : (int)blockIdx.x + 1;
    for (int b = b0; b < b1; ++b) {
        const int k = a.bin_start ? a.bin_list[b] : b;
        long long off;
        int N;
        double dx;
        if (a.offsets) {
            off = a.offsets[k];
            N = a.ncells[k];
            dx = a.dx[k];
        } else {
            off = 0;
            N = a.n1;
            dx = a.dx1;
        }
        if (N < 1 || off < 0 || off + N + 2LL * a.ng > a.total) continue;   // malformed entry: skipped
        const int bc = inst_bc(a.bc_inst, a.bc, k);
        const int NX = N + 2 * a.ng;
        const long long P = a.total, SU = 3 * P;
        const double inv_dx = 1.0 / dx;
        int nact = 0;
        while (nact < a.nsteps && a.dt_hist[(long long)nact * a.ninst + k] > 0.0) ++nact;

        // forward over the segment with the recorded steps, keeping the tape
        if constexpr (PH == ASE_ADJ_TAPE) {
            for (int I = tid; I < NX; I += NT) {
#pragma unroll
                for (int v = 0; v < 3; ++v) a.tapeU[v * P + off + I] = a.ck_U[v * P + off + I];
                a.tapeS[off + I] = a.ck_sig[off + I];
            }
            __syncthreads();
            BatchArgs fb;
            fb.ng = a.ng;
            fb.total = a.total;
            fb.bc = bc;
            fb.fo = a.fo;
            for (int q = 0; q < nact; ++q) {
                const double dt = a.dt_hist[(long long)q * a.ninst + k];
                double *Un = a.tapeU + (3LL * q) * SU + off;
                for (int st = 0; st < 3; ++st) {
                    double *in = a.tapeU + (3LL * q + st) * SU + off;
                    double *sin = a.tapeS + (3LL * q + st) * P + off;
                    batched_fill<NT>(fb, bc, in, sin, N, mc);
                    if (st == 2 && q == nact - 1) break;
                    Tile1D tl;
                    tl.U = in; tl.sx = sin; tl.Un = Un;
                    tl.Uout = a.tapeU + (3LL * q + st + 1) * SU + off;
                    tl.sig_out = a.tapeS + (3LL * q + st + 1) * P + off;
                    tl.wl = tl.wr = nullptr; tl.level = nullptr;
                    tl.plane = P; tl.nx = N; tl.ng = a.ng; tl.NX = NX; tl.nfaces = N + 1;
                    tl.stage = st + 1; tl.inv_dx = inv_dx; tl.dt = dt;
                    for (int i0 = 0; i0 < N; i0 += T) {
                        stage1d_tile<R, T, NT, MODE_FUSED_1D>(tl, i0, mc, L);
                        __syncthreads();
                    }
                }
            }
        }
        if constexpr (PH == ASE_ADJ_REVERSE) {
            // reverse sweep
            double *lam = a.lam + off, *mu1 = a.mu1 + off, *mu2 = a.mu2 + off;
            for (int q = nact - 1; q >= 0; --q) {
                const double dt = a.dt_hist[(long long)q * a.ninst + k];
                AdjTile t;
                t.plane = P; t.N = N; t.ng = a.ng; t.inv_dx = inv_dx;
                t.a1 = t.a2 = nullptr;
                t.c1 = t.c2 = 0.0;
                // stage 3
                t.V = a.tapeU + (3LL * q + 2) * SU + off;
                t.S = a.tapeS + (3LL * q + 2) * P + off;
                t.g = lam; t.gscale = (2.0 / 3.0) * dt;
                t.a0 = lam; t.c0 = 2.0 / 3.0;
                t.out = mu2;
                adj_stage<R, T, NT>(t, mc, L, bc);
                // stage 2
                t.V = a.tapeU + (3LL * q + 1) * SU + off;
                t.S = a.tapeS + (3LL * q + 1) * P + off;
                t.g = mu2; t.gscale = 0.25 * dt;
                t.a0 = mu2; t.c0 = 0.25;
                t.out = mu1;
                adj_stage<R, T, NT>(t, mc, L, bc);
                // stage 1
                t.V = a.tapeU + (3LL * q) * SU + off;
                t.S = a.tapeS + (3LL * q) * P + off;
                t.g = mu1; t.gscale = dt;
                t.a0 = lam; t.c0 = 1.0 / 3.0;
                t.a1 = mu2; t.c1 = 0.75;
                t.a2 = mu1; t.c2 = 1.0;
                t.out = lam;
                adj_stage<R, T, NT>(t, mc, L, bc);
            }
            // ghost slots of the result carry no meaning: clear them
            for (int kk = tid; kk < 2 * a.ng; kk += NT) {
                const int I = kk < a.ng ? kk : N + kk;
    #pragma unroll
                for (int v = 0; v < 3; ++v) lam[v * P + I] = 0.0;
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Wide form of the reverse sweep for the largest instances: one launch per
// (step, transposed stage) over all their tiles, then a launch that folds
// each instance's ghost gradients onto the cells they copy (adj_fold), as
// adj_stage does after its tile loop.  The tape comes from the tape phase of
// the persistent kernel (every instance).  Within one transposed stage no
// tile reads what another writes (each reads the previous stage's folded
// output and its own cells' combination terms), so the launches give the
// persistent reverse sweep's results bit for bit.
// ---------------------------------------------------------------------------
struct AdjWideArgs {
    const long long *offsets;
    const int *ncells;
    const double *dx;
    const double *dt_hist;
    const double *ck_U;   // checkpoint at the segment start (tape phase)
    double *lam, *mu1, *mu2;
    double *tapeU, *tapeS;
    const int *bc_inst;
    const int *tile_inst, *tile_i0, *inst_ntiles;
    long long total;
    int ninst, ntiles, ng, nsteps, bc;
    int q, stage;   // step, transposed stage 3, 2 or 1; stage 0: clear the ghost slots of lam
                    // (tape kernel: forward stage 0, 1 or 2 of step q)
    MethodConst mc;
};

// Steps the segment took for instance k (the persistent kernel's count).
__device__ __forceinline__ int adj_nact(const AdjWideArgs &a, int k)
{
    int n = 0;
    while (n < a.nsteps && a.dt_hist[(long long)n * a.ninst + k] > 0.0) ++n;
    return n;
}

// The transposed stage `stage` of step q as adj_stage sets it up.
__device__ __forceinline__ AdjTile adj_wide_tile(const AdjWideArgs &a, int k, int q, int stage)
{
    const long long off = a.offsets[k], P = a.total, SU = 3 * P;
    const double dt = a.dt_hist[(long long)q * a.ninst + k];
    double *lam = a.lam + off, *mu1 = a.mu1 + off, *mu2 = a.mu2 + off;
    AdjTile t;
    t.plane = P; t.N = a.ncells[k]; t.ng = a.ng; t.inv_dx = 1.0 / a.dx[k];
    t.a1 = t.a2 = nullptr;
    t.c1 = t.c2 = 0.0;
    t.V = a.tapeU + (3LL * q + stage - 1) * SU + off;
    t.S = a.tapeS + (3LL * q + stage - 1) * P + off;
    if (stage == 3) {
        t.g = lam; t.gscale = (2.0 / 3.0) * dt;
        t.a0 = lam; t.c0 = 2.0 / 3.0;
        t.out = mu2;
    } else if (stage == 2) {
        t.g = mu2; t.gscale = 0.25 * dt;
        t.a0 = mu2; t.c0 = 0.25;
        t.out = mu1;
    } else {
        t.g = mu1; t.gscale = dt;
        t.a0 = lam; t.c0 = 1.0 / 3.0;
        t.a1 = mu2; t.c1 = 0.75;
        t.a2 = mu1; t.c2 = 1.0;
        t.out = lam;
    }
    return t;
}

template <int R, int NT>
__global__ void __launch_bounds__(NT, 4) k_adjoint_wide(AdjWideArgs a)
{
    constexpr int T = NT - 2 * R - 2;
    __shared__ LdsAdj<R, T> L;
    const int b = blockIdx.x;
    const int k = a.tile_inst[b], i0 = a.tile_i0[b];
    if (k < 0 || k >= a.ninst) return;   // malformed tile entry: skipped (the whole workgroup)
    const int N = a.ncells[k];
    const long long off = a.offsets[k];
    if (N < T || off < 0 || off + N + 2LL * a.ng > a.total || i0 < 0 || i0 >= N) return;
    const bool active = a.q < adj_nact(a, k);
    // a transmissive instance's boundary tile holds both its ghost cells and
    // the cell they copy: it folds them itself (and at the end of the sweep
    // clears the ghost slots of lam); the fold launch takes the others
    const int bc = inst_bc(a.bc_inst, a.bc, k);
    const bool local = bc != ASE_BC_PERIODIC && bc != ASE_BC_REFLECTIVE;
    const bool clear = local && a.q == 0 && a.stage == 1;
    if (!active && !clear) return;
    const AdjTile t = adj_wide_tile(a, k, a.q, a.stage);
    if (active) {
        AdjWin<R, T, NT> w;
        adj_fetch<R, T, NT>(t, i0, w);
        adj_stage_window<R, T, NT>(w, L);
        __syncthreads();
        adjoint1d_tile<R, T, NT, true>(t, i0, a.mc, L);   // ends with a barrier
    }
    if (local) {
        const int v = threadIdx.x >> 1, side = threadIdx.x & 1;
        const bool mine = side == 0 ? i0 == 0 : i0 + T >= N;
        if (threadIdx.x < 6 && mine) {
            // adj_fold's transmissive sum, in its order
            double *o = t.out + v * a.total;
            const int base = side == 0 ? 0 : N + a.ng;
            if (active) {
                double acc = 0.0;
                for (int kk = 0; kk < a.ng; ++kk) acc += o[base + kk];
                o[side == 0 ? a.ng : a.ng + N - 1] += acc;
            }
            if (clear)
                for (int kk = 0; kk < a.ng; ++kk) o[base + kk] = 0.0;
        }
    }
}

// Tape of the wide instances: forward stage `stage` (0, 1, 2) of step q of
// every tile, as the tape phase of k_adjoint1d runs it, with the recorded
// time step.  The stage input is tape slot 3q + stage (the checkpoint for
// the first); the launch writes that slot's ghost cells and every face
// strength the way batched_fill leaves them, the checkpoint's interior into
// slot 0, and the stage output into the interior of the next slot (the last
// stage of the last step taken has no output: the reverse sweep never reads
// it).
template <int R, int NT>
__global__ void __launch_bounds__(NT) k_tape_wide(AdjWideArgs a)
{
    constexpr int T = NT - 2 * R - 2;
    constexpr int UX = Lds1D<R, T>::UX;
    __shared__ Lds1D<R, T> L;
    const int tid = threadIdx.x, b = blockIdx.x;
    const int k = a.tile_inst[b], i0 = a.tile_i0[b];
    if (k < 0 || k >= a.ninst) return;   // malformed tile entry: skipped (the whole workgroup)
    const int N = a.ncells[k], ng = a.ng;
    const long long off = a.offsets[k], P = a.total, SU = 3 * P;
    if (N < T || off < 0 || off + N + 2LL * ng > P || i0 < 0 || i0 >= N) return;
    const int q = a.q, st = a.stage;
    const int nact = adj_nact(a, k);
    if (q >= nact) return;
    const int bc = inst_bc(a.bc_inst, a.bc, k);
    const bool from_ck = q == 0 && st == 0;
    double *slot = a.tapeU + (3LL * q + st) * SU + off;
    double *sslot = a.tapeS + (3LL * q + st) * P + off;
    const double *in = from_ck ? a.ck_U + off : slot;
    const bool last_stage = st == 2 && q == nact - 1;

    Tile1D tl;
    tl.U = const_cast<double *>(in); tl.sx = nullptr; tl.sig_out = nullptr;
    tl.Un = a.tapeU + (3LL * q) * SU + off;
    tl.Uout = a.tapeU + (3LL * q + st + 1) * SU + off;
    tl.wl = tl.wr = nullptr; tl.level = nullptr;
    tl.plane = P; tl.nx = N; tl.ng = ng; tl.NX = N + 2 * ng; tl.nfaces = N + 1;
    tl.stage = st + 1; tl.inv_dx = 1.0 / a.dx[k]; tl.dt = a.dt_hist[(long long)q * a.ninst + k];
    double un[3];
    stage1d_prefetch<T, NT, MODE_FUSED_1D>(tl, i0, un);
    wide_window<R, NT>(in, P, N, ng, bc, i0, a.mc, L);

    // the input slot as batched_fill leaves it: ghost cells (boundary
    // tiles), the checkpoint's interior (slot 0), and the strength of every
    // face x + 1/2, x in [-ng, N + ng - 1): own faces x in [i0, i0 + T),
    // ghost faces by the boundary tiles
    const int ox = i0 - 1 - R;
    const bool first = i0 == 0, last = i0 + T >= N;
    auto face = [&](int x) {
        const int lx = x - ox;
        if (lx >= 0 && lx + 1 < UX) return L.sS[lx];
        double Wa[3], Wb[3];
        mapped_cell(in, P, N, ng, bc, x, Wa);
        mapped_cell(in, P, N, ng, bc, x + 1, Wb);
        return sigma_point(primitives<3>(Wa, 0, a.mc), primitives<3>(Wb, 0, a.mc));
    };
    {
        const int x = i0 + tid;
        if (tid < T && x < N) {
            sslot[x + ng] = face(x);
            if (from_ck) {
#pragma unroll
                for (int v = 0; v < 3; ++v) slot[v * P + x + ng] = L.sU[v][x - ox];
            }
        }
    }
    if (first || last) {
        for (int kk = tid; kk < ng; kk += NT) {
            if (first) {
                const int x = -ng + kk;
                double W[3];
                mapped_cell(in, P, N, ng, bc, x, W);
#pragma unroll
                for (int v = 0; v < 3; ++v) slot[v * P + x + ng] = W[v];
                sslot[x + ng] = face(x);
            }
            if (last) {
                const int x = N + kk;
                double W[3];
                mapped_cell(in, P, N, ng, bc, x, W);
#pragma unroll
                for (int v = 0; v < 3; ++v) slot[v * P + x + ng] = W[v];
                if (x + 1 < N + ng) sslot[x + ng] = face(x);
            }
        }
    }
    if (last_stage) return;
    double l;
    stage1d_compute<R, T, NT, MODE_FUSED_1D>(tl, i0, a.mc, L, un, l);
}

// One workgroup of 64 lanes per instance; instances without tiles and
// transmissive ones return.
__global__ void __launch_bounds__(64) k_adjoint_wide_fold(AdjWideArgs a)
{
    const int k = blockIdx.x;
    if (a.inst_ntiles[k] < 1) return;
    const int N = a.ncells[k];
    const long long off = a.offsets[k], P = a.total;
    if (N < 1 || off < 0 || off + N + 2LL * a.ng > a.total) return;
    const int bc = inst_bc(a.bc_inst, a.bc, k);
    if (bc != ASE_BC_PERIODIC && bc != ASE_BC_REFLECTIVE) return;   // folded by its boundary tiles
    if (a.stage == 0) {
        double *lam = a.lam + off;
        for (int kk = threadIdx.x; kk < 2 * a.ng; kk += 64) {
            const int I = kk < a.ng ? kk : N + kk;
#pragma unroll
            for (int v = 0; v < 3; ++v) lam[v * P + I] = 0.0;
        }
        return;
    }
    if (a.q >= adj_nact(a, k)) return;
    double *out = (a.stage == 3 ? a.mu2 : a.stage == 2 ? a.mu1 : a.lam) + off;
    adj_fold(out, P, N, a.ng, bc);
}

// J_k = dx_k sum_i p_i over the interior of each instance and its gradient
// dJ/dU = dx (gamma-1) (u^2/2, -u, 1) (ghost slots 0).  One workgroup per
// instance, fixed-order tree reduction.
struct ObjArgs {
    const long long *offsets;
    const int *ncells;
    const double *dx;
    int n1;
    double dx1;
    const double *U;
    const double *w;   // optional per-instance weights of the gradient
    double *J, *lam;
    long long total;
    int ng;
    double gm1;
};

template <int NT>
__global__ void __launch_bounds__(NT) k_pressure_objective(ObjArgs a)
{
    __shared__ double red[NT];
    const int k = blockIdx.x;
    long long off;
    int N;
    double dx;
    if (a.offsets) {
        off = a.offsets[k];
        N = a.ncells[k];
        dx = a.dx[k];
    } else {
        off = 0;
        N = a.n1;
        dx = a.dx1;
    }
    if (N < 1 || off < 0 || off + N + 2LL * a.ng > a.total) return;
    const long long P = a.total;
    const double wdx = (a.w ? a.w[k] : 1.0) * dx;
    double acc = 0.0;
    for (int I = threadIdx.x; I < N + 2 * a.ng; I += NT) {
        const int i = I - a.ng;
        const long long e = off + I;
        if (i < 0 || i >= N) {
            if (a.lam) {
#pragma unroll
                for (int v = 0; v < 3; ++v) a.lam[v * P + e] = 0.0;
            }
            continue;
        }
        const double rho = a.U[e], m = a.U[P + e], E = a.U[2 * P + e];
        const double u = m / rho;
        acc += a.gm1 * (E - 0.5 * m * u);
        if (a.lam) {
            a.lam[e] = wdx * a.gm1 * 0.5 * u * u;
            a.lam[P + e] = -wdx * a.gm1 * u;
            a.lam[2 * P + e] = wdx * a.gm1;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && a.J) a.J[k] = red[0] * dx;
}

// ---------------------------------------------------------------------------
// Granular face kernels.
// ---------------------------------------------------------------------------
struct FaceGeo {
    int dim, nx, ny, ng, ld, nfaces, G, oi;
};

__device__ __forceinline__ long long face_plane_pos(const FaceGeo &f, int dir, long long id)
{
    if (f.dim == 1) return id - 1 + f.ng;
    if (dir == 0) {
        const long long j = id / (f.nx + 1), i = id % (f.nx + 1) - 1;
        return (j + f.ng) * f.ld + i + f.ng;
    }
    const long long j = id / f.nx - 1, i = id % f.nx;
    return (j + f.ng) * f.ld + i + f.ng;
}

template <int NV>
__global__ void __launch_bounds__(kThreads) k_df(FaceGeo f, MethodConst mc, int dir, const double *wl,
                                                 const double *wr, double *sig)
{
    const long long id = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (id >= f.nfaces) return;
    double s = 0.0;
    for (int k = 0; k < f.G; ++k) {
        double Wl[NV], Wr[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Wl[v] = wl[(long long)(v * f.G + k) * f.nfaces + id];
            Wr[v] = wr[(long long)(v * f.G + k) * f.nfaces + id];
        }
        s += sigma_point(primitives<NV>(Wl, dir, mc), primitives<NV>(Wr, dir, mc));
    }
    sig[face_plane_pos(f, dir, id)] = s / (double)f.G;
}

template <int NV>
__global__ void __launch_bounds__(kThreads) k_flux(FaceGeo f, MethodConst mc, int dir, const double *wl,
                                                   const double *wr, double *F)
{
    const long long id = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (id >= f.nfaces) return;
    double Fs[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fs[v] = 0.0;
    for (int k = 0; k < f.G; ++k) {
        double Wl[NV], Wr[NV], Fk[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Wl[v] = wl[(long long)(v * f.G + k) * f.nfaces + id];
            Wr[v] = wr[(long long)(v * f.G + k) * f.nfaces + id];
        }
        lf_flux<NV>(Wl, primitives<NV>(Wl, dir, mc), Wr, primitives<NV>(Wr, dir, mc), dir, Fk);
        const double eta = (f.dim == 1) ? 1.0 : kTab.eta[f.oi][k];
#pragma unroll
        for (int v = 0; v < NV; ++v) Fs[v] += eta * Fk[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) F[(long long)v * f.nfaces + id] = Fs[v];
}

template <int NV>
__global__ void __launch_bounds__(kThreads) k_stage_update(BCInfo b, int stage, const double *dtp, const double *Un,
                                                           const double *Us, const double *F, const double *Gf,
                                                           double inv_dx, double inv_dy, double *Uo)
{
    const int ny = b.dim == 1 ? 1 : b.ny;
    const long long n = (long long)ny * b.nx;
    const long long idx = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= n) return;
    const int j = (int)(idx / b.nx), i = (int)(idx % b.nx);
    const long long pos = (long long)(b.dim == 1 ? 0 : j + b.ng) * b.ld + i + b.ng;
    const long long nfx = b.dim == 1 ? b.nx + 1 : (long long)(b.nx + 1) * b.ny;
    const long long nfy = (long long)b.nx * (b.ny + 1);
    const double dt = *dtp;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const long long fx = (b.dim == 1) ? i + 1 : (long long)j * (b.nx + 1) + i + 1;
        double L = -(F[v * nfx + fx] - F[v * nfx + fx - 1]) * inv_dx;
        if constexpr (NV == 4) {
            const long long fy = (long long)(j + 1) * b.nx + i;
            L = L + -(Gf[v * nfy + fy] - Gf[v * nfy + fy - b.nx]) * inv_dy;
        }
        const long long e = v * b.plane + pos;
        double o;
        if (stage == 1) o = Un[e] + dt * L;
        else if (stage == 2) o = 0.75 * Un[e] + 0.25 * Us[e] + 0.25 * dt * L;
        else o = (1.0 / 3.0) * Un[e] + (2.0 / 3.0) * Us[e] + (2.0 / 3.0) * dt * L;
        Uo[e] = o;
    }
}

int grid_blocks(long long n)
{
    long long b = (n + kThreads - 1) / kThreads;
    if (b > 65535LL * 16) b = 65535LL * 16;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

void launch_bc_fill(const ase_grid_t &g, const Geo &geo, const MethodConst &mc, double *U, double *sx, double *sy,
                    hipStream_t st, const double *t, const double *dt, double ct)
{
    BCInfo b = make_bc(g, geo);
    b.t = t;
    b.dt = dt;
    b.ct = ct;
    const dim3 grid(grid_blocks(frame_size(b)), geo.dim == 2 ? 3 : 2);
    if (geo.nv == 4) k_bc_fill<4><<<grid, kThreads, 0, st>>>(b, mc, U, sx, sy);
    else k_bc_fill<3><<<grid, kThreads, 0, st>>>(b, mc, U, sx, sy);
}

void launch_sigma_init(const ase_grid_t &g, const Geo &geo, const MethodConst &mc, double *U, double *sx,
                       double *sy, hipStream_t st, const double *t, const double *dt, double ct, double *part)
{
    BCInfo b = make_bc(g, geo);
    b.t = t;
    b.dt = dt;
    b.ct = ct;
    const double idx = 1.0 / g.dx, idy = geo.dim == 2 ? 1.0 / g.dy : 0.0;
    if (geo.dim == 1) {
        const dim3 tiles((geo.NX + kFoTX1 - 1) / kFoTX1);
        k_fill_fo<3, kFoTX1, 1><<<tiles, kFoTX1, 0, st>>>(b, mc, U, sx, sy, idx, idy, part);
    } else {
        const dim3 tiles((geo.NX + kFoTX2 - 1) / kFoTX2, (geo.NY + kFoTY2 - 1) / kFoTY2);
        k_fill_fo<4, kFoTX2, kFoTY2><<<tiles, kFoTX2 * kFoTY2, 0, st>>>(b, mc, U, sx, sy, idx, idy, part);
    }
}

void launch_nonphysical(const ase_grid_t &g, const Geo &geo, const MethodConst &mc, const double *U, double *part,
                        int nparts, hipStream_t st)
{
    const BCInfo b = make_bc(g, geo);
    if (geo.nv == 4) k_nonphysical_partial<4><<<nparts, kThreads, 0, st>>>(b, mc, U, part);
    else k_nonphysical_partial<3><<<nparts, kThreads, 0, st>>>(b, mc, U, part);
}

void launch_cfl_final(const ase_grid_t &g, const Geo &geo, const ase_params_t &p, const MethodConst &mc,
                      const double *t_in, double *t_out, double t_end, double *dt, double *skip, double *dt_hist,
                      const double *part, int nparts, hipStream_t st)
{
    InflowSpeed inf;
    inf.on = (g.bc[0] == ASE_BC_INFLOW_SLOT || g.bc[1] == ASE_BC_INFLOW_SLOT) ? 1 : 0;
    inf.dim = geo.dim;
    for (int k = 0; k < 4; ++k) inf.W[k] = g.inflow[k];
    inf.inv_dx = 1.0 / g.dx;
    inf.inv_dy = geo.dim == 2 ? 1.0 / g.dy : 0.0;
    k_cfl_final<<<1, kFinalThreads, 0, st>>>(part, nparts, p.cfl, p.dt_cap, t_in, t_out, t_end, dt, skip, dt_hist,
                                             inf, mc);
}

void launch_cfl(const ase_grid_t &g, const Geo &geo, const ase_params_t &p, const MethodConst &mc, const double *U,
                const double *t_in, double *t_out, double t_end, double *dt, double *skip, double *dt_hist,
                double *part, int nparts, hipStream_t st)
{
    const BCInfo b = make_bc(g, geo);
    if (geo.nv == 4)
        k_cfl_partial<4><<<nparts, kThreads, 0, st>>>(b, mc, U, 1.0 / g.dx, 1.0 / g.dy, part);
    else
        k_cfl_partial<3><<<nparts, kThreads, 0, st>>>(b, mc, U, 1.0 / g.dx, 1.0 / g.dy, part);
    launch_cfl_final(g, geo, p, mc, t_in, t_out, t_end, dt, skip, dt_hist, part, nparts, st);
}

namespace {
constexpr int kT1D = 256;
// 2D sweeps: x faces on 15 x 16 tiles with 512 lanes, y faces on 16 x 7
// tiles with 256 lanes (the y sweep also streams the residual and the
// step-start state; more, smaller workgroups per CU hide that latency better).
// (T0 + 1) x T1 = 256 x-faces and T0 x (T1 + 1) = 128 y-faces: one face per
// lane pair of the block.
constexpr int kNTX = 512, kNTY = 256;
constexpr int kX_T0 = 15, kX_T1 = 16, kY_T0 = 16, kY_T1 = 7;

template <int R>
void sweep_r(const Geo &geo, int dir, int mode, const SweepArgs &a, hipStream_t st)
{
    if (geo.dim == 1) {
        constexpr int T1 = kT1D - 2 * R - 2;   // one pass of the workgroup per phase
        dim3 grid((geo.nx + T1 - 1) / T1);
        if (mode == MODE_RECON) k_stage1d<R, T1, MODE_RECON><<<grid, kThreads, 0, st>>>(a);
        else k_stage1d<R, T1, MODE_FUSED_1D><<<grid, kThreads, 0, st>>>(a);
        return;
    }
    if (dir == 0) {
        dim3 grid((geo.nx + kX_T0 - 1) / kX_T0, (geo.ny + kX_T1 - 1) / kX_T1);
        if (mode == MODE_RECON) k_sweep2d<0, R, kX_T0, kX_T1, kNTX, MODE_RECON><<<grid, kNTX, 0, st>>>(a);
        else k_sweep2d<0, R, kX_T0, kX_T1, kNTX, MODE_FUSED_X><<<grid, kNTX, 0, st>>>(a);
    } else {
        dim3 grid((geo.nx + kY_T0 - 1) / kY_T0, (geo.ny + kY_T1 - 1) / kY_T1);
        if (mode == MODE_RECON) k_sweep2d<1, R, kY_T0, kY_T1, kNTY, MODE_RECON><<<grid, kNTY, 0, st>>>(a);
        else k_sweep2d<1, R, kY_T0, kY_T1, kNTY, MODE_FUSED_Y><<<grid, kNTY, 0, st>>>(a);
    }
}
}  // namespace

void launch_sweep(const Geo &geo, int dir, int mode, const SweepArgs &a, hipStream_t st)
{
    switch (geo.R) {
    case 1: sweep_r<1>(geo, dir, mode, a, st); break;
    case 2: sweep_r<2>(geo, dir, mode, a, st); break;
    case 3: sweep_r<3>(geo, dir, mode, a, st); break;
    default: sweep_r<4>(geo, dir, mode, a, st); break;
    }
}

static FaceGeo face_geo(const Geo &geo, int dir)
{
    FaceGeo f;
    f.dim = geo.dim; f.nx = geo.nx; f.ny = geo.ny; f.ng = geo.ng; f.ld = geo.ld;
    f.G = geo.G; f.oi = geo.oi;
    if (geo.dim == 1) f.nfaces = geo.nx + 1;
    else f.nfaces = dir == 0 ? (geo.nx + 1) * geo.ny : geo.nx * (geo.ny + 1);
    return f;
}

void launch_df(const Geo &geo, const MethodConst &mc, int dir, const double *wl, const double *wr, double *sig,
               hipStream_t st)
{
    const FaceGeo f = face_geo(geo, dir);
    const int nb = (f.nfaces + kThreads - 1) / kThreads;
    if (geo.nv == 4) k_df<4><<<nb, kThreads, 0, st>>>(f, mc, dir, wl, wr, sig);
    else k_df<3><<<nb, kThreads, 0, st>>>(f, mc, dir, wl, wr, sig);
}

void launch_flux(const Geo &geo, const MethodConst &mc, int dir, const double *wl, const double *wr, double *F,
                 hipStream_t st)
{
    const FaceGeo f = face_geo(geo, dir);
    const int nb = (f.nfaces + kThreads - 1) / kThreads;
    if (geo.nv == 4) k_flux<4><<<nb, kThreads, 0, st>>>(f, mc, dir, wl, wr, F);
    else k_flux<3><<<nb, kThreads, 0, st>>>(f, mc, dir, wl, wr, F);
}

void launch_stage_update(const ase_grid_t &g, const Geo &geo, int stage, const double *dt, const double *Un,
                         const double *Us, const double *F, const double *Gf, double *Uout, hipStream_t st)
{
    const BCInfo b = make_bc(g, geo);
    const long long n = (long long)geo.nx * (geo.dim == 1 ? 1 : geo.ny);
    const int nb = (int)((n + kThreads - 1) / kThreads);
    if (geo.nv == 4)
        k_stage_update<4><<<nb, kThreads, 0, st>>>(b, stage, dt, Un, Us, F, Gf, 1.0 / g.dx, 1.0 / g.dy, Uout);
    else
        k_stage_update<3><<<nb, kThreads, 0, st>>>(b, stage, dt, Un, Us, F, Gf, 1.0 / g.dx, 1.0 / g.dy, Uout);
}

void launch_batched(const BatchLaunch &bl, hipStream_t st)
{
    BatchArgs a;
    a.offsets = bl.offsets; a.ncells = bl.ncells; a.dx = bl.dx;
    a.U = bl.U; a.sig = bl.sig; a.t = bl.t; a.dt_hist = bl.dt_hist; a.dt_in = bl.dt_in; a.status = bl.status;
    a.U1 = bl.U1; a.U2 = bl.U2; a.sig2 = bl.sig2;
    a.bin_start = bl.bin_start; a.bin_list = bl.bin_list; a.bc_inst = bl.bc_inst; a.only = bl.only;
    a.total = bl.total; a.ninst = bl.ninst; a.ng = bl.ng; a.nsteps = bl.nsteps; a.bc = bl.bc; a.fo = bl.fo;
    a.t_end = bl.t_end; a.cfl = bl.cfl; a.dt_cap = bl.dt_cap; a.mc = bl.mc;
    if (bl.init) {
        k_batched_sigma_init<256><<<bl.ninst, 256, 0, st>>>(a);
        return;
    }
#define ASE_BATCH(RR, NTT) k_batched1d<RR, NTT><<<bl.nbins, NTT, 0, st>>>(a)
    if (bl.threads == 1024) {
        switch (bl.R) {
        case 1: ASE_BATCH(1, 1024); break;
        case 2: ASE_BATCH(2, 1024); break;
        case 3: ASE_BATCH(3, 1024); break;
        default: ASE_BATCH(4, 1024); break;
        }
    } else if (bl.threads == 512) {
        switch (bl.R) {
        case 1: ASE_BATCH(1, 512); break;
        case 2: ASE_BATCH(2, 512); break;
        case 3: ASE_BATCH(3, 512); break;
        default: ASE_BATCH(4, 512); break;
        }
    } else {
        switch (bl.R) {
        case 1: ASE_BATCH(1, 256); break;
        case 2: ASE_BATCH(2, 256); break;
        case 3: ASE_BATCH(3, 256); break;
        default: ASE_BATCH(4, 256); break;
        }
    }
#undef ASE_BATCH
}

void launch_batched_wide(const WideLaunch &wl, hipStream_t st)
{
    WideArgs a;
    a.offsets = wl.offsets; a.ncells = wl.ncells; a.dx = wl.dx;
    a.U = wl.U; a.U1 = wl.U1; a.U2 = wl.U2; a.t = wl.t; a.dt_hist = wl.dt_hist; a.dt_in = wl.dt_in;
    a.status = wl.status; a.bc_inst = wl.bc_inst;
    a.tile_inst = wl.tile_inst; a.tile_i0 = wl.tile_i0; a.inst_tile0 = wl.inst_tile0; a.inst_ntiles = wl.inst_ntiles;
    a.lam = wl.lam; a.dt_cur = wl.dt_cur; a.done = wl.done;
    a.total = wl.total; a.ninst = wl.ninst; a.ntiles = wl.ntiles; a.ng = wl.ng; a.bc = wl.bc; a.step = wl.step;
    a.stage = wl.stage; a.nsteps = wl.nsteps;
    a.t_end = wl.t_end; a.cfl = wl.cfl; a.dt_cap = wl.dt_cap; a.mc = wl.mc;
#define ASE_WIDE(RR, NTT)                                                     \
    do {                                                                      \
        if (wl.per_step) k_batched_wide_step<RR, NTT><<<wl.ntiles, NTT, 0, st>>>(a); \
        else k_batched_wide<RR, NTT><<<wl.ntiles, NTT, 0, st>>>(a);           \
    } while (0)
    if (wl.threads == 512) {
        switch (wl.R) {
        case 1: ASE_WIDE(1, 512); break;
        case 2: ASE_WIDE(2, 512); break;
        case 3: ASE_WIDE(3, 512); break;
        default: ASE_WIDE(4, 512); break;
        }
    } else {
        switch (wl.R) {
        case 1: ASE_WIDE(1, 256); break;
        case 2: ASE_WIDE(2, 256); break;
        case 3: ASE_WIDE(3, 256); break;
        default: ASE_WIDE(4, 256); break;
        }
    }
#undef ASE_WIDE
}

void launch_tape_wide(const AdjWideLaunch &wl, hipStream_t st)
{
    AdjWideArgs a;
    std::memset(&a, 0, sizeof(a));
    a.offsets = wl.offsets; a.ncells = wl.ncells; a.dx = wl.dx; a.dt_hist = wl.dt_hist; a.ck_U = wl.ck_U;
    a.tapeU = wl.tapeU; a.tapeS = wl.tapeS;
    a.bc_inst = wl.bc_inst; a.tile_inst = wl.tile_inst; a.tile_i0 = wl.tile_i0; a.inst_ntiles = wl.inst_ntiles;
    a.total = wl.total; a.ninst = wl.ninst; a.ntiles = wl.ntiles; a.ng = wl.ng; a.nsteps = wl.nsteps;
    a.bc = wl.bc; a.mc = wl.mc;
    for (int q = 0; q < wl.nsteps; ++q) {
        for (int stage = 0; stage < 3; ++stage) {
            a.q = q;
            a.stage = stage;
            if (wl.threads == 512) {
                switch (wl.R) {
                case 1: k_tape_wide<1, 512><<<wl.ntiles, 512, 0, st>>>(a); break;
                case 2: k_tape_wide<2, 512><<<wl.ntiles, 512, 0, st>>>(a); break;
                case 3: k_tape_wide<3, 512><<<wl.ntiles, 512, 0, st>>>(a); break;
                default: k_tape_wide<4, 512><<<wl.ntiles, 512, 0, st>>>(a); break;
                }
            } else {
                switch (wl.R) {
                case 1: k_tape_wide<1, 256><<<wl.ntiles, 256, 0, st>>>(a); break;
                case 2: k_tape_wide<2, 256><<<wl.ntiles, 256, 0, st>>>(a); break;
                case 3: k_tape_wide<3, 256><<<wl.ntiles, 256, 0, st>>>(a); break;
                default: k_tape_wide<4, 256><<<wl.ntiles, 256, 0, st>>>(a); break;
                }
            }
        }
    }
}

void launch_adjoint_wide(const AdjWideLaunch &wl, hipStream_t st)
{
    AdjWideArgs a;
    std::memset(&a, 0, sizeof(a));
    a.offsets = wl.offsets; a.ncells = wl.ncells; a.dx = wl.dx; a.dt_hist = wl.dt_hist;
    a.lam = wl.lam; a.mu1 = wl.mu1; a.mu2 = wl.mu2; a.tapeU = wl.tapeU; a.tapeS = wl.tapeS;
    a.bc_inst = wl.bc_inst; a.tile_inst = wl.tile_inst; a.tile_i0 = wl.tile_i0; a.inst_ntiles = wl.inst_ntiles;
    a.total = wl.total; a.ninst = wl.ninst; a.ntiles = wl.ntiles; a.ng = wl.ng; a.nsteps = wl.nsteps;
    a.bc = wl.bc; a.mc = wl.mc;
    // the fold launches have work only for periodic and reflective instances
    const bool folds = wl.bc_inst != nullptr || wl.bc == ASE_BC_PERIODIC || wl.bc == ASE_BC_REFLECTIVE;
    // steps back, each as its three transposed stages and their folds
    for (int q = wl.nsteps - 1; q >= 0; --q) {
        for (int stage = 3; stage >= 1; --stage) {
            a.q = q;
            a.stage = stage;
            if (wl.threads == 512) {
                switch (wl.R) {
                case 1: k_adjoint_wide<1, 512><<<wl.ntiles, 512, 0, st>>>(a); break;
                case 2: k_adjoint_wide<2, 512><<<wl.ntiles, 512, 0, st>>>(a); break;
                case 3: k_adjoint_wide<3, 512><<<wl.ntiles, 512, 0, st>>>(a); break;
                default: k_adjoint_wide<4, 512><<<wl.ntiles, 512, 0, st>>>(a); break;
                }
            } else {
                switch (wl.R) {
                case 1: k_adjoint_wide<1, 256><<<wl.ntiles, 256, 0, st>>>(a); break;
                case 2: k_adjoint_wide<2, 256><<<wl.ntiles, 256, 0, st>>>(a); break;
                case 3: k_adjoint_wide<3, 256><<<wl.ntiles, 256, 0, st>>>(a); break;
                default: k_adjoint_wide<4, 256><<<wl.ntiles, 256, 0, st>>>(a); break;
                }
            }
            if (folds) k_adjoint_wide_fold<<<wl.ninst, 64, 0, st>>>(a);
        }
    }
    a.q = 0;
    a.stage = 0;
    if (folds) k_adjoint_wide_fold<<<wl.ninst, 64, 0, st>>>(a);
}

void launch_adjoint(const AdjLaunch &al, hipStream_t st)
{
    AdjArgs a;
    a.offsets = al.offsets; a.ncells = al.ncells; a.dx = al.dx; a.n1 = al.n1; a.dx1 = al.dx1;
    a.ck_U = al.ck_U; a.ck_sig = al.ck_sig; a.dt_hist = al.dt_hist; a.lam = al.lam;
    a.mu1 = al.mu1; a.mu2 = al.mu2; a.tapeU = al.tapeU; a.tapeS = al.tapeS;
    a.bin_start = al.bin_start; a.bin_list = al.bin_list; a.bc_inst = al.bc_inst;
    a.total = al.total; a.ninst = al.ninst; a.ng = al.ng; a.nsteps = al.nsteps; a.bc = al.bc; a.fo = al.fo;
    a.phase = al.phase;
    a.mc = al.mc;
    const int nblk = al.bin_start ? al.nbins : al.ninst;
    // the tape of every instance, then the reverse sweep of every instance
    // (instances are independent: the same results as one phase after the
    // other per instance)
#define ASE_ADJ(RR, NTT)                                                                         \
    do {                                                                                         \
        if (al.phase & ASE_ADJ_TAPE) k_adjoint1d<RR, NTT, ASE_ADJ_TAPE><<<nblk, NTT, 0, st>>>(a); \
        if (al.phase & ASE_ADJ_REVERSE)                                                          \
            k_adjoint1d<RR, NTT, ASE_ADJ_REVERSE><<<nblk, NTT, 0, st>>>(a);                      \
    } while (0)
    if (al.threads == 128) {
        switch (al.R) {
        case 1: ASE_ADJ(1, 128); break;
        case 2: ASE_ADJ(2, 128); break;
        case 3: ASE_ADJ(3, 128); break;
        default: ASE_ADJ(4, 128); break;
        }
    } else if (al.threads == 512) {
        switch (al.R) {
        case 1: ASE_ADJ(1, 512); break;
        case 2: ASE_ADJ(2, 512); break;
        case 3: ASE_ADJ(3, 512); break;
        default: ASE_ADJ(4, 512); break;
        }
    } else {
        switch (al.R) {
        case 1: ASE_ADJ(1, 256); break;
        case 2: ASE_ADJ(2, 256); break;
        case 3: ASE_ADJ(3, 256); break;
        default: ASE_ADJ(4, 256); break;
        }
    }
#undef ASE_ADJ
}

void launch_objective(const ObjLaunch &ol, hipStream_t st)
{
    ObjArgs a;
    a.offsets = ol.offsets; a.ncells = ol.ncells; a.dx = ol.dx; a.n1 = ol.n1; a.dx1 = ol.dx1;
    a.U = ol.U; a.w = ol.w; a.J = ol.J; a.lam = ol.lam; a.total = ol.total; a.ng = ol.ng; a.gm1 = ol.gm1;
    k_pressure_objective<256><<<ol.ninst, 256, 0, st>>>(a);
}


// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free batched entry point: the two
// stage states and the second strength array of k_batched1d live in this
// module-scope array instead of a caller workspace.  Every GPU the library
// runs on holds its own copy until the process ends.  Host code takes the
// address hipGetSymbolAddress returns on the current device (kept per
// device after the first call) and never the array's name, which on the
// host is only a stand-in for the symbol.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[ASE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;

int noalloc_scratch(void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(ASE_ERR_ARG, "device index beyond the scratch table");
    static std::mutex mu;
    static void *addr[kMaxScratchDevices];
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if ((reinterpret_cast<uintptr_t>(p) & 255u) != 0) return fail(ASE_ERR_ALIGN, "scratch not 256-byte aligned");
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return ASE_OK;
}

}  // namespace ase
