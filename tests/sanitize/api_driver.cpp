// Address/undefined-behaviour sanitizer run of the host side of libase's C
// ABI (test infrastructure): ase_api.cpp compiled with the host pass
// sanitized and linked against launchers that record nothing, so no GPU is
// needed.  Exercises the argument validation of every entry point (each must
// return its error before any launch), the workspace-size queries and the
// host packing of batches.  Exit status 0 when every check holds.
#include "../../paper_2410_05489_amd/csrc/ase_api.cpp"

#include <cstdio>
#include <vector>

namespace ase {
// launchers: never reached by the calls below (they fail validation first);
// defined so the library links without its kernels
void launch_bc_fill(const ase_grid_t &, const Geo &, const MethodConst &, double *, double *, double *, hipStream_t,
                    const double *, const double *, double) {}
void launch_sigma_init(const ase_grid_t &, const Geo &, const MethodConst &, double *, double *, double *,
                       hipStream_t, const double *, const double *, double, double *) {}
void launch_nonphysical(const ase_grid_t &, const Geo &, const MethodConst &, const double *, double *, int,
                        hipStream_t) {}
void launch_cfl(const ase_grid_t &, const Geo &, const ase_params_t &, const MethodConst &, const double *,
                const double *, double *, double, double *, double *, double *, double *, int, hipStream_t) {}
void launch_cfl_final(const ase_grid_t &, const Geo &, const ase_params_t &, const MethodConst &, const double *,
                      double *, double, double *, double *, double *, const double *, int, hipStream_t) {}
void launch_sweep(const Geo &, int, int, const SweepArgs &, hipStream_t) {}
void launch_df(const Geo &, const MethodConst &, int, const double *, const double *, double *, hipStream_t) {}
void launch_flux(const Geo &, const MethodConst &, int, const double *, const double *, double *, hipStream_t) {}
void launch_stage_update(const ase_grid_t &, const Geo &, int, const double *, const double *, const double *,
                         const double *, const double *, double *, hipStream_t) {}
void launch_batched(const BatchLaunch &, hipStream_t) {}
void launch_batched_wide(const WideLaunch &, hipStream_t) {}
int noalloc_scratch(void **ptr) { *ptr = nullptr; return ASE_OK; }
void launch_adjoint(const AdjLaunch &, hipStream_t) {}
void launch_adjoint_wide(const AdjWideLaunch &, hipStream_t) {}
void launch_tape_wide(const AdjWideLaunch &, hipStream_t) {}
void launch_objective(const ObjLaunch &, hipStream_t) {}
void launch_gks1d(int, int, const Gks1DArgs &, hipStream_t) {}
void launch_gks2d(int, int, bool, const Gks2DArgs &, hipStream_t) {}
void launch_gks2d_update(const Gks2DUpdate &, hipStream_t) {}
void launch_gks_points(const GksPointArgs &, hipStream_t) {}
}  // namespace ase

static int fails = 0, checks = 0;
#define EXPECT(cond)                                                              \
    do {                                                                          \
        ++checks;                                                                 \
        if (!(cond)) {                                                            \
            ++fails;                                                              \
            std::printf("FAILED line %d: %s (%s)\n", __LINE__, #cond, ase_last_error()); \
        }                                                                         \
    } while (0)

int main()
{
    ase_grid_t g;
    std::memset(&g, 0, sizeof(g));
    g.dim = 2; g.nx = 16; g.ny = 12; g.ng = 5; g.ld = 26;
    for (int k = 0; k < 4; ++k) g.bc[k] = ASE_BC_TRANSMISSIVE;
    g.dx = g.dy = 1.0 / 16;
    ase_params_t p;
    std::memset(&p, 0, sizeof(p));
    p.order = 9; p.gamma = 1.4; p.cfl = 0.4; p.sigma_thres = 2.0; p.eps = 1e-6; p.d_hi = p.d_lo = 0.85;
    double *dummy = reinterpret_cast<double *>(0x1000);   // never dereferenced: every call below fails first

    // validation of the grid and method
    ase_params_t bad = p;
    bad.order = 4;
    EXPECT(ase_step(&g, &bad, dummy, dummy, dummy, dummy, nullptr, 1, 0.0, dummy, 1 << 20, nullptr) == ASE_ERR_ORDER);
    ase_grid_t gb = g;
    gb.ng = 4;
    EXPECT(ase_step(&gb, &p, dummy, dummy, dummy, dummy, nullptr, 1, 0.0, dummy, 1 << 20, nullptr) == ASE_ERR_GHOST);
    gb = g;
    gb.ld = 20;
    EXPECT(ase_bc_fill(&gb, &p, dummy, dummy, dummy, nullptr) == ASE_ERR_ARG);
    gb = g;
    gb.bc[0] = ASE_BC_PERIODIC;
    EXPECT(ase_sigma_init(&gb, &p, dummy, dummy, dummy, nullptr) == ASE_ERR_ARG);
    gb = g;
    gb.nx = -3;
    EXPECT(ase_workspace_bytes(&gb, &p) == 0);
    EXPECT(ase_workspace_bytes(&g, &p) > 0);
    EXPECT(ase_gks_workspace_bytes(&g, &p) >= ase_workspace_bytes(&g, &p));
    EXPECT(ase_step(&g, &p, nullptr, dummy, dummy, dummy, nullptr, 1, 0.0, dummy, 1 << 30, nullptr) == ASE_ERR_ARG);
    EXPECT(ase_step(&g, &p, dummy, dummy, dummy, dummy, nullptr, 1, 0.0, nullptr, 0, nullptr) == ASE_ERR_WORKSPACE);
    EXPECT(ase_step(&g, &p, dummy, dummy, dummy, dummy, nullptr, -1, 0.0, dummy, 1 << 30, nullptr) == ASE_ERR_ARG);
    double *odd = reinterpret_cast<double *>(0x1003);
    EXPECT(ase_reconstruct(&g, &p, 2, dummy, dummy, dummy, dummy, dummy, nullptr, nullptr) != ASE_OK);
    EXPECT(ase_flux(&g, &p, 0, odd, dummy, dummy, nullptr) != ASE_OK);
    EXPECT(ase_stage_update(&g, &p, 4, dummy, dummy, dummy, dummy, dummy, dummy, nullptr) == ASE_ERR_ARG);
    EXPECT(ase_cfl_dt(&g, &p, dummy, dummy, 0.0, dummy, nullptr, 0, nullptr) == ASE_ERR_WORKSPACE);
    ase_gks_t gk;
    std::memset(&gk, 0, sizeof(gk));
    gk.c1 = -1.0;
    EXPECT(ase_step_gks(&g, &p, &gk, dummy, dummy, dummy, dummy, nullptr, 1, 0.0, dummy, 1 << 30, nullptr) != ASE_OK);
    EXPECT(ase_gks_flux(&p, &gk, -1, dummy, dummy, dummy, dummy, 0.1, dummy, dummy, nullptr) != ASE_OK);
    // adjoint: 1D only
    EXPECT(ase_adjoint_workspace_bytes(&g) == 0);
    EXPECT(ase_adjoint_step(&g, &p, dummy, dummy, dummy, dummy, dummy, dummy, 1 << 30, nullptr) != ASE_OK);

    // batched: host packing (longest first onto the least loaded bin)
    std::vector<int32_t> nc = {300, 17, 4096, 64, 64, 1200, 999, 5};
    const int nb = 3;
    std::vector<int32_t> start(nb + 1, -1), list(nc.size(), -1);
    EXPECT(ase_batched_plan((int32_t)nc.size(), nc.data(), nb, start.data(), list.data()) == ASE_OK);
    EXPECT(start[0] == 0 && start[nb] == (int32_t)nc.size());
    std::vector<int> seen(nc.size(), 0);
    for (int k : list) {
        EXPECT(k >= 0 && k < (int)nc.size());
        if (k >= 0 && k < (int)nc.size()) ++seen[k];
    }
    for (int s : seen) EXPECT(s == 1);
    EXPECT(ase_batched_plan(0, nc.data(), nb, start.data(), list.data()) == ASE_ERR_ARG);
    EXPECT(ase_batched_plan((int32_t)nc.size(), nc.data(), 0, start.data(), list.data()) == ASE_ERR_ARG);
    EXPECT(ase_batched_workspace_bytes(0) == 0 && ase_batched_workspace_bytes(1000) >= 7 * 1000 * 8);
    EXPECT(ase_step_batched(&p, ASE_BC_TRANSMISSIVE, nullptr, 0, nullptr, nullptr, nullptr, 5, 0, nullptr, nullptr,
                            nullptr, nullptr, nullptr, nullptr, 1, 0.0, nullptr, nullptr, 1, 256, nullptr, 0,
                            nullptr) == ASE_ERR_ARG);
    int64_t off = 0;
    int32_t n1 = 10;
    EXPECT(ase_step_batched(&p, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy, dummy,
                            nullptr, nullptr, nullptr, 1, 0.0, &n1, &n1, 1, 300, dummy, 1 << 20,
                            nullptr) == ASE_ERR_ARG);
    EXPECT(ase_step_batched_noalloc(&p, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 1198369, dummy, dummy,
                                    dummy, nullptr, nullptr, nullptr, 1, 0.0, &n1, &n1, 1, 256,
                                    nullptr) == ASE_ERR_WORKSPACE);
    // wide form: planning (tiles of 256 - 9 - 1 = 246 cells at order 9) and validation
    {
        std::vector<int32_t> ti(64, -1), t0(64, -1), b0(nb + 1, -1), bl2(nc.size(), -1), tin(nc.size(), -2),
            tnt(nc.size(), -2);
        int32_t ntl = -1;
        EXPECT(ase_batched_plan_wide((int32_t)nc.size(), nc.data(), 1000, 9, 256, nb, b0.data(), bl2.data(),
                                     nullptr, nullptr, tin.data(), tnt.data(), 0, &ntl) == ASE_ERR_ARG);
        EXPECT(ntl == 17 + 5);   // 4096 cells: 17 tiles, 1200: 5; 999 < min_cells
        EXPECT(ase_batched_plan_wide((int32_t)nc.size(), nc.data(), 1000, 9, 256, nb, b0.data(), bl2.data(),
                                     ti.data(), t0.data(), tin.data(), tnt.data(), 64, &ntl) == ASE_OK);
        EXPECT(ntl == 22 && tin[2] == 0 && tnt[2] == 17 && tin[5] == 17 && tnt[5] == 5);
        EXPECT(tin[0] == -1 && tnt[0] == 0 && b0[nb] == (int32_t)nc.size() - 2);
        EXPECT(ti[16] == 2 && t0[16] == 16 * 246 && ti[21] == 5 && t0[21] == 4 * 246);
        EXPECT(ase_batched_plan_wide((int32_t)nc.size(), nc.data(), 1000, 8, 256, nb, b0.data(), bl2.data(),
                                     ti.data(), t0.data(), tin.data(), tnt.data(), 64, &ntl) == ASE_ERR_ORDER);
        EXPECT(ase_batched_plan_wide((int32_t)nc.size(), nc.data(), 1000, 9, 1024, nb, b0.data(), bl2.data(),
                                     ti.data(), t0.data(), tin.data(), tnt.data(), 64, &ntl) == ASE_ERR_ARG);
        EXPECT(ase_batched_wide_workspace_bytes(1000, 2, 3) > ase_batched_workspace_bytes(1000));
        EXPECT(ase_batched_wide_workspace_bytes(0, 2, 3) == 0);
        // the wide form needs the first-order source
        const size_t wsb = ase_batched_wide_workspace_bytes(20, 1, 1);
        EXPECT(ase_step_batched_wide(&p, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                     dummy, nullptr, nullptr, nullptr, 1, 0.0, &n1, &n1, 1, 256, &n1, &n1, &n1,
                                     &n1, 1, 256, dummy, wsb, nullptr) == ASE_ERR_ARG);
        ase_params_t pf = p;
        pf.flags |= ASE_FLAG_DF_FIRST_ORDER;
        EXPECT(ase_step_batched_wide(&pf, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                     dummy, nullptr, nullptr, nullptr, 1, 0.0, &n1, &n1, 1, 256, &n1, &n1, &n1,
                                     &n1, 1, 384, dummy, wsb, nullptr) == ASE_ERR_ARG);
        EXPECT(ase_step_batched_wide(&pf, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                     dummy, nullptr, nullptr, nullptr, 1, 0.0, &n1, &n1, 1, 256, &n1, &n1, &n1,
                                     &n1, 1, 256, dummy, wsb - 8, nullptr) == ASE_ERR_WORKSPACE);
        EXPECT(ase_step_batched_wide(&pf, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                     dummy, nullptr, nullptr, nullptr, 1, 0.0, &n1, &n1, 1, 256, nullptr, &n1, &n1,
                                     &n1, 1, 256, dummy, wsb, nullptr) == ASE_ERR_ARG);
        // nothing to do: no launch, no stream
        EXPECT(ase_step_batched_wide(&pf, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                     dummy, nullptr, nullptr, nullptr, 0, 0.0, &n1, &n1, 1, 256, &n1, &n1, &n1,
                                     &n1, 1, 256, dummy, wsb, nullptr) == ASE_OK);
    }
    EXPECT(ase_adjoint_batched(&p, 7, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy, dummy, 1, dummy, &n1, &n1,
                               1, 256, ASE_ADJ_TAPE | ASE_ADJ_REVERSE, dummy, 1 << 20, nullptr) == ASE_ERR_ARG);
    EXPECT(ase_adjoint_batched(&p, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy, dummy, 1,
                               dummy, &n1, &n1, 1, 256, 0, dummy, 1 << 20, nullptr) == ASE_ERR_ARG);
    ase_params_t pfo = p;
    pfo.flags |= ASE_FLAG_DF_FIRST_ORDER;
    // the wide adjoint: first-order source only, 256 or 512 lanes, tile arrays, a phase
    EXPECT(ase_adjoint_batched_wide(&p, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                    dummy, 1, dummy, &n1, &n1, 1, 256, &n1, &n1, &n1, 1, 256, 2, dummy, 1 << 30,
                                    nullptr) == ASE_ERR_ARG);
    EXPECT(ase_adjoint_batched_wide(&pfo, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                    dummy, 1, dummy, &n1, &n1, 1, 256, &n1, &n1, &n1, 1, 384, 2, dummy, 1 << 30,
                                    nullptr) == ASE_ERR_ARG);
    EXPECT(ase_adjoint_batched_wide(&pfo, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                    dummy, 1, dummy, &n1, &n1, 1, 256, nullptr, &n1, &n1, 1, 256, 2, dummy, 1 << 30,
                                    nullptr) == ASE_ERR_ARG);
    EXPECT(ase_adjoint_batched_wide(&pfo, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                    dummy, 1, dummy, &n1, &n1, 1, 256, &n1, &n1, &n1, 1, 256, 4, dummy, 1 << 30,
                                    nullptr) == ASE_ERR_ARG);
    EXPECT(ase_adjoint_batched_wide(&p, ASE_BC_TRANSMISSIVE, nullptr, 1, &off, &n1, dummy, 5, 20, dummy, dummy,
                                    dummy, 1, dummy, &n1, &n1, 1, 256, &n1, &n1, &n1, 1, 256, 2, dummy, 64,
                                    nullptr) == ASE_ERR_WORKSPACE);
    EXPECT(ase_pressure_objective(nullptr, 1, &off, &n1, dummy, 5, 20, dummy, nullptr, nullptr, nullptr,
                                  nullptr) != ASE_OK);
    EXPECT(ase_profile_read(99, nullptr, nullptr) != ASE_OK);
    EXPECT(std::strlen(ase_last_error()) > 0);
    std::printf("api sanitizer run: %d checks, %d failed\n", checks, fails);
    return fails ? 1 : 0;
}
