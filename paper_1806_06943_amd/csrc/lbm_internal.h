// Host/device shared declarations of the HIP library (not part of the C-ABI).
#pragma once

#include "lbm.h"
#include "lbm_device.h"

namespace lbm {

// per-row partial quantities and per-instance results of the FP64 reductions
constexpr int NQR = 12;
constexpr int NRES = 24;
enum ResSlot {
    RES_MASSA = 0, RES_MASSB, RES_PX, RES_PY, RES_JX, RES_JY, RES_Q, RES_UMAX, RES_AMAX,
    RES_AMIN, RES_BAD, RES_AREA, RES_R, RES_CX, RES_CY, RES_PIN, RES_POUT, RES_NIN, RES_NOUT,
    RES_DP, RES_GAMMA, RES_W
};

// device-side tables of a context (all inside the caller's workspace)
struct Dev {
    KInst *insts;   // [ninst]
    int4 *tiles;    // [ntiles] {inst, x0, y0, 0}: 2-D tiles of the auxiliary kernels
    int4 *strips;   // [nstrips] {inst, X0, Y0, wo | ho << 16}: segments of the fused step
    int *first;     // [nwg + 1] workgroup g advances segments first[g] .. first[g+1]-1
    int2 *rows;     // [nrows]  {inst, y}
    int *row0s;     // [ninst]  first row index of each instance in rows
    double *part;   // [nrows][NQR]
    double *res;    // [ninst][NRES]
    int ninst, ntiles, nrows, nstrips;
    int nw;         // wavefronts per strip of the fused step (1, 2, 4 or 8)
    int nwg;        // workgroups of the fused step
    int forcing;    // 0: Guo term (Eq. 5), 1: velocity shift of the original model
    int fr;         // 1: full-row segments {inst, w0, Y0, k | ho << 16} (nx = 64 k)
};

// wavefronts per strip for a strip of `cols` output columns
constexpr int strip_waves(int cols) { return cols <= 58 ? 1 : cols <= 122 ? 2 : cols <= 250 ? 4 : 8; }
constexpr int MAX_STRIP_COLS = 8 * 64 - 6;

// output columns of a one-wavefront strip of the two-step kernel (six
// columns of halo on either side)
constexpr int SW2 = SW - 4 * (HALO + 1);

hipError_t launch_init(const Dev &d, const double *const *rho0s, hipStream_t st);
hipError_t launch_step(const Dev &d, int par, hipStream_t st);
// two steps in one launch (one-wavefront strips of at most SW2 output
// columns, no full rows): f[par] -> f[par ^ 1]
hipError_t launch_step2(const Dev &d, int par, hipStream_t st);
// Options of one launch of the fused step: buffers that replace one
// instance's ping-pong pair (a window recorded in place; inst < 0: none),
// and whether the launch writes rho(t + 1) of every instance (wrho 1) or of
// none (0: the step itself never reads it).
struct StepOvr {
    int inst;
    const float *fin;
    float *fout, *rout;
    int wrho;
};
hipError_t launch_step_ovr(const Dev &d, int par, const StepOvr &o, hipStream_t st);
hipError_t launch_density(const Dev &d, int par, hipStream_t st);
hipError_t launch_fields(const Dev &d, int par, hipStream_t st);
hipError_t launch_fields_out(const Dev &d, int inst, float *rho, float *u, hipStream_t st);
hipError_t launch_export(const Dev &d, int inst, int par, float *f, hipStream_t st);
hipError_t launch_import(const Dev &d, int inst, int par, const float *f, hipStream_t st);
hipError_t launch_forces(const Dev &d, int inst, int par, const float *rho, float *F, hipStream_t st);
// the reduction partials go to part[nrows][NQR], the per-instance results
// to res[ninst][NRES] (the workspace's, or any other device buffer)
hipError_t launch_observables(const Dev &d, int par, double margin, double *part, double *res,
                              hipStream_t st);
// per-instance results res[ninst][NRES] as lbm_obs records out[ninst] (device)
hipError_t launch_obs_pack(const Dev &d, const double *res, lbm_obs *out, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, uint64_t nbytes, hipStream_t st);
hipError_t lds_checks(unsigned int *bad, hipStream_t st);

// ------------------------------------------------------------------ adjoint
// Scratch planes of the instance's field region used by the adjoint passes:
// density deviations (the first 2 planes, holding one packed density buffer),
// force adjoints [k][d] (4), then FP64 block partials
// (NPART per 64 x 4 tile, a small part of one plane) followed by NPART final
// sums, the force transpose's addition to every lam_{k,i} of a node (2), and
// a second set of force adjoints (4): the steps of a run alternate between
// the two sets, each reading the one the step before wrote.
constexpr int SCR_RDEV = 0;
constexpr int SCR_FBAR = 2;
constexpr int SCR_PART = 6;
constexpr int SCR_ADD = 7;
constexpr int SCR_FBAR2 = 9;
constexpr int NPART = 8;
static_assert(SCR_FBAR2 + 4 <= NFLD, "adjoint scratch planes");

// Parameters of one instance for the adjoint kernels (passed by value).
struct AdjPar {
    int32_t nx, ny, walls, pitch;
    int64_t plane;          // floats between scratch planes
    float G1[2], G2[2];     // Eq. 8 couplings per component
    float gab;              // Eq. 9 coupling
    float it[2];            // 1 / tau_k
    float cg[2];            // 1 - 1 / (2 tau_k), Guo prefactor of Eq. 5
    float g[2][2];          // body acceleration per component
    float rho_ref[2], rho_wall[2], psi_wall[2];
    float rho0, inv_rho0;
    float qscale;           // 1 / nx (flow-rate objective)
    float *scr;             // scratch planes
    float *rscr;            // density deviations written by k_adj_density (packed, rho[y][x][k])
    const float *rdev;      // density deviations of the state being transposed (packed)
    int fbo;                // first of the 4 planes the local pass writes its force adjoints to
    int fbi;                // (folded runs) the planes the step before wrote its force adjoints to
    const float *rdev_next; // (folded runs) density deviations of the state after this one
    double *part;           // [blocks][NPART]
    double *res;            // [NPART]
};

hipError_t launch_adjoint_step(const AdjPar &A, const float *f, const float *lam_next, float *lam,
                               double *grad, hipStream_t st);
// Pieces of a run of adjoint steps: clear the partials and the pending
// addition, one step, final sums.  Between the steps of a run lam is held as
// the local part in the caller's buffer plus a pending per-component
// addition in scratch; launch_adjoint_combine folds it in (out = in + add,
// in place allowed).
hipError_t launch_adjoint_zero(const AdjPar &A, hipStream_t st);
// f: the state's populations in the library's packed layout; rdev: its
// density deviations (packed, recorded), or NULL to compute them
hipError_t launch_adjoint_body(const AdjPar &A, const float *f, const float *rdev,
                               const float *lam_next, float *lam, hipStream_t st);
hipError_t launch_adjoint_combine(const AdjPar &A, const float *in, float *out, hipStream_t st);
// The two passes of a step of a run, separately.  The local pass with fold
// forms the pending addition of the step before (force adjoints in planes
// A.fbi, densities A.rdev_next) itself where its gather reads it, instead of
// a force pass of the step before writing it; the force pass reads planes
// A.fbo and writes the pending addition.
hipError_t launch_adjoint_local(const AdjPar &A, bool fold, const float *f, const float *lam_next,
                                float *lam, hipStream_t st);
hipError_t launch_adjoint_force(const AdjPar &A, hipStream_t st);
hipError_t launch_adjoint_final(const AdjPar &A, double *grad, hipStream_t st);
hipError_t launch_objective_pass1(const AdjPar &A, int which, const float *f, float *lam,
                                  hipStream_t st);
hipError_t launch_objective_dp_seed(const AdjPar &A, float *lam, double mA, double mB, double SA,
                                    double SB, hipStream_t st);
int adjoint_blocks(int nx, int ny);
constexpr int N_ADJ_KERNELS = 5;
const char *adjoint_kernel_name(int j);
hipError_t launch_adjoint_kernel(const AdjPar &A, int j, const float *f, const float *lam_next,
                                 float *lam, double *grad, hipStream_t st);

// pressure tensor P[3][ny][nx] of instance inst and the FP64 sum of P_xx - P_yy
hipError_t launch_pressure(const Dev &d, const lbm_params &p, int inst, int par, float *out,
                           double *part, double *res, hipStream_t st);

// kernels of one step, for timing: number, names, and a launcher of kernel j
constexpr int N_STEP_KERNELS = 1;
const char *step_kernel_name(int j);
hipError_t launch_step_kernel(const Dev &d, int j, int par, hipStream_t st);

}  // namespace lbm
