/*
 * C-ABI of the MI355X (gfx950) implementation of the two-range
 * pseudopotential lattice Boltzmann step for binary mixtures with tunable
 * viscosity ratio (Fei, Scagliarini, Montessori, Lauricella, Succi, Luo,
 * arXiv:1806.06943, Sec. II).
 *
 * One time step advances both components of every lattice node:
 *   densities            rho_k = sum_i f_{k,i}                         (Eq. 6)
 *   pseudopotential      psi_k = rho0 (1 - exp(-rho_k / rho0))         (Sec. II B)
 *   forces               F_k = F^c_k (Eq. 8, D2Q9 attraction + D2Q25
 *                        repulsion) + F^r_k (Eq. 9) + rho_k g_k
 *   moments              j_k = sum_i f_{k,i} e_i + F_k / 2             (Eq. 6)
 *   common velocity      u^eq = sum_k j_k/tau_k / sum_k rho_k/tau_k     (Eq. 3)
 *   collision            BGK per component towards f^eq(rho_k, u^eq)
 *                        plus the Guo forcing term                     (Eqs. 1, 2, 5)
 *   (or, with the velocity-shift forcing of the original model: j_k without
 *   F_k/2 and BGK towards f^eq(rho_k, u^eq + tau_k F_k / rho_k), Sec. II A)
 *   streaming            periodic in x; periodic in y, or half-way
 *                        bounce-back walls half a link outside rows 0
 *                        and ny-1                                      (Eq. 1, Sec. III A)
 *
 * Arithmetic is FP32; populations are stored as FP32 deviations
 * f_{k,i} - w_i rho_ref[k].  FP64 is used on the device only in the
 * reductions behind lbm_observables, lbm_adjoint_seed and the parameter
 * gradients of lbm_adjoint_step.
 *
 * Memory ownership: the caller allocates ONE device workspace of
 * lbm_workspace_bytes() bytes and every device buffer passed to an entry
 * point; the library never allocates or frees device memory.  The library
 * owns host-side metadata and HIP graph objects of a context.  All device
 * work is enqueued on the stream given to lbm_init; entry points that
 * return host data synchronise that stream.
 *
 * Errors: every entry point returns LBM_OK (0) or a negative code and never
 * aborts; lbm_last_error() gives the message of the last failure of a
 * context.  A context is used from one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)       /* bad argument: sizes, tau <= 0.5, NULL, short buffer */
#define LBM_EHIP (-2)         /* HIP runtime failure                                 */
#define LBM_ENONFINITE (-3)   /* a reduction saw NaN or Inf in the state             */
#define LBM_EUNSUPPORTED (-4) /* valid request that the library does not provide    */

typedef struct lbm_ctx lbm_ctx;

#define LBM_FORCING_GUO 0
#define LBM_FORCING_SHIFT 1

/* Model parameters of one lattice instance, as the paper states the model. */
typedef struct {
    int32_t nx, ny;      /* lattice size, each >= 1 (small tori alias the 5x5 stencil)   */
    int32_t walls;       /* 0: periodic x and y; 1: periodic x, walls below row 0 and
                            above row ny-1 (half-way bounce-back, Sec. III A)            */
    int32_t forcing;     /* LBM_FORCING_GUO (0): the present model's forcing term with the
                            common velocity (Eq. 5); LBM_FORCING_SHIFT (1): the velocity
                            shift of the original two-range model (its explicit form C^SC,
                            Sec. II A), for comparison.  All instances of a context use
                            the same scheme.  The shift as Eq. 4 states it does not
                            reproduce the original model's numbers of Sec. III C: at the
                            emulsion couplings it is stable only for tau >= 1, where its
                            surface tension is about 0.16, not 0.043.                  */
    double G_AB;         /* inter-species coupling of Eq. 9 (> 0 repulsive)             */
    double G1[2];        /* short-range coupling of Eq. 8 per component {A, B}          */
    double G2[2];        /* mid-range coupling of Eq. 8 per component {A, B}            */
    double tau[2];       /* relaxation times of Eq. 1, each > 0.5                       */
    double psi_rho0;     /* rho0 of the pseudopotential (Sec. II B), > 0                */
    double g[2][2];      /* body acceleration per component, (x, y): F^b_k = rho_k g_k  */
    double rho_wall[2];  /* densities the force stencil sees beyond a wall (walls = 1)  */
    double rho_ref[2];   /* reference of the FP32 deviation storage, per component;
                            the library uses its FP32 rounding                         */
} lbm_params;

/* FP64 observables of one instance (lbm_observables). */
typedef struct {
    double mass[2];      /* sum_x rho_k                                              */
    double mom_raw[2];   /* sum_{x,k,i} f_{k,i} e_i (population momentum)            */
    double mom_bary[2];  /* sum_x sum_k j_k, j_k with F_k/2 (Eq. 6)                  */
    double max_speed;    /* max_x |u|, u barycentric (Eq. 7)                         */
    double rho_a_max;    /* max_x rho_A                                              */
    double rho_a_min;    /* min_x rho_A                                              */
    double flow_rate;    /* Q = sum_y ubar(y), ubar = x-mean of u_x (Sec. III D)     */
    double R_eff;        /* static-droplet radius sqrt(A/pi) (Laplace test, Sec. III B) */
    double cx, cy;       /* droplet centre (periodic circular mean)                  */
    double p_in, p_out;  /* mean bulk pressure (Eq. 11) inside / outside             */
    double dp;           /* p_in - p_out                                             */
    double gamma;        /* dp * R_eff                                               */
    double width;        /* interface width W along the row through the centre
                            (Fig. 2 caption)                                          */
    int64_t n_in, n_out; /* node counts of the two pressure averages                 */
    int64_t finite;      /* 1 if every density and velocity was finite               */
} lbm_obs;

/* Bytes of device workspace that lbm_init needs for n_inst instances whose
 * parameters are params[0..n_inst-1].  Returns LBM_EINVAL for bad sizes. */
int lbm_workspace_bytes(const lbm_params *params, int32_t n_inst, uint64_t *bytes);

/* Create a context for n_inst >= 1 independent instances (all with the same
 * forcing scheme; LBM_EUNSUPPORTED otherwise).
 *   params     host array [n_inst], copied
 *   rhoA0/B0   host FP64 initial densities, instance after instance, each
 *              row-major ny*nx; the initial state is equilibrium at rest
 *              f_{k,i} = w_i rho_k (Eq. 2 with u = 0)
 *   workspace  device pointer to workspace_bytes >= lbm_workspace_bytes(),
 *              256-byte aligned, owned by the caller, kept alive until
 *              lbm_destroy
 *   stream     hipStream_t on which all work of this context is enqueued
 *              (NULL = the default stream)
 * Every instance advances by the same number of steps per lbm_step. */
int lbm_init(lbm_ctx **out, const lbm_params *params, int32_t n_inst, const double *rhoA0,
             const double *rhoB0, void *workspace, uint64_t workspace_bytes, void *stream);

/* Advance every instance by nsteps >= 0 time steps (Eq. 1).  Asynchronous on
 * the context's stream; long runs replay a captured HIP graph.  The step
 * moves only the populations: the calls that read densities (observables,
 * fields, pressure tensor, recording) first compute those of the current
 * state with one density pass, once per state. */
int lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* Capture the step graphs that lbm_step replays (one per parity of the
 * state, 16 steps each) now, without running them; otherwise the first
 * lbm_step of 16 or more steps from each parity captures its graph.  Lets a
 * caller keep capture and instantiation out of a timed or latency-bound
 * region.  Changes no state; the graphs stay valid until a strip-plan call
 * discards them. */
int lbm_prepare(lbm_ctx *ctx);

/* Time steps taken since lbm_init (or the last lbm_set_populations). */
int64_t lbm_steps_done(const lbm_ctx *ctx);

/* FP64 observables of every instance into host out[n_inst]; if ubar is not
 * NULL it receives the x-mean of u_x per row, instance after instance
 * (sum of ny doubles).  Synchronises the stream.  Returns LBM_ENONFINITE
 * (after filling out) if any instance holds NaN or Inf. */
int lbm_observables(lbm_ctx *ctx, lbm_obs *out, double *ubar);

/* For callers that cannot allocate memory (code under stream capture, tight
 * serving loops, hosts that forbid allocation after start-up): the observables
 * of lbm_observables (same kernels, same results bit for bit) into host
 * out[n_inst], without ubar, allocating nothing on the host or the device.
 * The FP64 reduction partials, the per-instance results and the packed
 * records live in a static device array of the library, 4 MiB per GPU (held
 * from the first lbm_init on that GPU until the process ends), whose device
 * address lbm_init resolves.  A context whose 12 * (total rows) + 46 *
 * n_inst doubles exceed 2^19 gets LBM_EINVAL.  Every call on one GPU uses
 * that GPU's one array: calls that overlap in time on one GPU (contexts on
 * different streams or host threads) race and must be serialised by the
 * caller.  Each call writes every scratch word it reads, so nothing carries
 * over from an earlier call.  Synchronises the stream; LBM_ENONFINITE as
 * lbm_observables. */
int lbm_observables_noalloc(lbm_ctx *ctx, lbm_obs *out);

/* Density and barycentric velocity (Eq. 7) fields of instance inst, FP32,
 * into device buffers rho[2][ny][nx] and u[2][ny][nx] (either may be NULL).
 * Asynchronous. */
int lbm_fields(lbm_ctx *ctx, int32_t inst, float *rho_dev, float *u_dev);

/* Pressure tensor (Sec. II B) of instance inst into the device buffer
 * P_dev[3][ny][nx] (FP32; P_xx, P_yy, P_xy): P = P^int + P^kin, with
 *   P^int_k = 1/2 sum_e c_k(e) psi_k(x) psi_k(x+e) e e
 *           + 1/2 G_AB sum_i w_i rho_k(x) rho_kbar(x+e_i) e_i e_i
 *   (c_k(e) = G_{k,1} w(e) + G_{k,2} p(e)), the pair-sum form of the forces
 *   of Eqs. 8, 9, equal to the interaction part of Eq. 11 in bulk;
 *   P^kin = sum_{k,i} f_{k,i} e_i e_i for the Guo forcing (the static
 *   problem), sum_k rho_k cs^2 delta + K^tau of the original model for the
 *   velocity shift (density gradients by central differences).
 * If line_tension is not NULL it receives (1/ny) sum_{x,y} (P_xx - P_yy)
 * (FP64): the line tension of Eqs. 15, 16 for interfaces orthogonal to x
 * (per interface pair it is the overall line tension gamma_f; one interface
 * gives gamma), and the stream is synchronised; otherwise asynchronous.
 * Overwrites the instance's field scratch. */
int lbm_pressure(lbm_ctx *ctx, int32_t inst, float *P_dev, double *line_tension);

/* Copy the populations f_{k,i}(x, t) (post-streaming, pre-collision) of
 * instance inst as FP32 deviations f - w_i rho_ref[k] into the device buffer
 * f_dev[2][9][ny][nx] (D2Q9 order 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
 * 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)).  Asynchronous. */
int lbm_get_populations(lbm_ctx *ctx, int32_t inst, float *f_dev);

/* Replace the state of instance inst by f_dev (same layout and meaning as
 * lbm_get_populations).  Asynchronous. */
int lbm_set_populations(lbm_ctx *ctx, int32_t inst, const float *f_dev);

/* Interaction plus body forces F_k (Eqs. 8, 9, F^b) of instance inst for the
 * given densities rho_dev[2][ny][nx] (device, FP32) into F_dev[2][2][ny][nx]
 * (component, axis).  Uses the step's own force code and a scratch density
 * buffer of the context (not the current state's).  Asynchronous. */
int lbm_forces(lbm_ctx *ctx, int32_t inst, const float *rho_dev, float *F_dev);

/* Device-to-device copy of nbytes through the library's own streaming copy
 * kernel; used to measure the achievable HBM bandwidth.  Asynchronous. */
int lbm_copy_probe(lbm_ctx *ctx, void *dst_dev, const void *src_dev, uint64_t nbytes);

/* Time the kernels of one step: each kernel of the step is launched nrep
 * times back to back on the context's stream between two HIP events; ms[j]
 * receives the average duration of kernel j in milliseconds and names[j]
 * (if names is not NULL) a static string naming it.  *n_kernels receives the
 * number of kernels per step (at most max_k are written).  In two-step mode
 * (lbm_set_two_step) the kernel timed is the two-step one, "k_fused_step2",
 * and ms[0] covers two steps.  The state is left unchanged.  Synchronises
 * the stream. */
int lbm_profile_step(lbm_ctx *ctx, int32_t nrep, int32_t max_k, double *ms, const char **names,
                     int32_t *n_kernels);

/* Strip height of the fused step (lattice rows one strip advances per step,
 * default 16, at least 2); selects the uniform plan (every column strip cut
 * into ceil(ny / chunk_rows) chunks, one workgroup each).  Any value gives
 * the same results bit for bit; it trades halo recomputation against
 * parallelism.  Synchronises the stream and discards captured graphs. */
int lbm_set_tiling(lbm_ctx *ctx, int32_t chunk_rows);
int32_t lbm_get_tiling(const lbm_ctx *ctx);

/* Output columns per strip of the fused step, in [16, 506] (default 58).  A
 * strip is one workgroup of 1, 2, 4 or 8 wavefronts (up to 58, 122, 250 or
 * 506 columns).  A multiple of 16 places strips at multiples of cols, so
 * that every row of output starts on a 64-byte boundary; any other value
 * splits each row into ceil(nx / cols) strips of balanced width.  Results
 * are bitwise identical for every value.  Synchronises the stream and
 * discards captured graphs. */
int lbm_set_strip_width(lbm_ctx *ctx, int32_t cols);
int32_t lbm_get_strip_width(const lbm_ctx *ctx);

/* Balanced plan (wgs_per_cu in [1, 8]): the fused step runs as exactly
 * wgs_per_cu workgroups per compute unit, each advancing an equal share of
 * all strip rows (a share may cover two or more column strips), so no
 * compute unit holds more work than another.  0 returns to the uniform plan
 * of lbm_set_tiling.  Results are bitwise identical for every plan.
 * Synchronises the stream and discards captured graphs. */
int lbm_set_balance(lbm_ctx *ctx, int32_t wgs_per_cu);
int32_t lbm_get_balance(const lbm_ctx *ctx);

/* Full-row plan (on = 1) for contexts whose lattice widths are all multiples
 * of 64, at most 512: a group of nx / 64 wavefronts covers whole rows, every
 * lane loading, colliding and writing one column of its own, so no column
 * is read or collided twice; rows are cut into the uniform chunks of
 * lbm_set_tiling, and chunks of equal height share workgroups of 1, 2, 4 or
 * 8 wavefronts (the smallest that holds the widest lattice).  LBM_EUNSUPPORTED
 * for other widths.  on = 0, lbm_set_strip_width and lbm_set_balance return
 * to strips.  Results are bitwise identical for every plan.  Synchronises the
 * stream and discards captured graphs. */
int lbm_set_full_rows(lbm_ctx *ctx, int32_t on);
int32_t lbm_get_full_rows(const lbm_ctx *ctx);

/* Two steps per launch (on = 1): lbm_step then advances every instance two
 * time steps (Eqs. 1-9, twice) per launch of a second kernel that keeps the
 * intermediate state of each strip on chip, so the populations cross HBM
 * once per two steps; an odd remaining step runs alone.  Every node goes
 * through exactly the operations of two single steps: the states equal
 * those of the single-step kernel bit for bit.  It needs one-wavefront
 * strips of at most 52 output columns (lbm_set_strip_width(ctx, c) with
 * c <= 52, uniform or balanced, no full rows): LBM_EUNSUPPORTED otherwise,
 * and, while it is on, for the plan setters that would leave such strips.
 * Only lbm_step changes; recording, the adjoint and the observables run
 * the single step.  Discards captured graphs. */
int lbm_set_two_step(lbm_ctx *ctx, int32_t on);
int32_t lbm_get_two_step(const lbm_ctx *ctx);

/* Workgroups of one launch of the fused step under the current strip plan. */
int32_t lbm_get_workgroups(const lbm_ctx *ctx);

/* The same strip planner on the host, without a context or a device: for
 * params[0..n_inst-1], strips of cols output columns, and either uniform
 * chunks of chunk_rows rows (wgs = 0) or the balanced plan of exactly wgs
 * workgroups (wgs in [1, 8192]; lbm_set_balance asks for wgs_per_cu times
 * the compute units), or, with full_rows = 1, the full-row plan of chunks of
 * chunk_rows rows (cols and wgs ignored), *nwg receives the workgroups of one
 * launch and, if nsegs is not NULL, *nsegs the segments (full-row groups)
 * they advance.  LBM_EINVAL for arguments lbm_set_tiling /
 * lbm_set_strip_width / lbm_set_balance refuse, LBM_EUNSUPPORTED for a
 * full-row plan of lattices lbm_set_full_rows refuses. */
int lbm_plan_workgroups(const lbm_params *params, int32_t n_inst, int32_t cols, int32_t chunk_rows,
                        int32_t wgs, int32_t full_rows, int32_t *nwg, int32_t *nsegs);

/* ------------------------------------------------------------------------
 * Reverse-mode adjoint (gradients of objectives with respect to the state and
 * to theta = (G1, G2, G_AB, tau_A, tau_B), where G1 and G2 move the couplings
 * of Eq. 8 of both components together).  The paper has no adjoint; these
 * entry points differentiate the step defined by Eqs. 1, 2, 3, 5, 6, 8, 9
 * exactly as lbm_step computes it (same readings).  State and adjoint
 * buffers are the caller's, device FP32, in the lbm_get_populations layout
 * [2][9][ny][nx]; state buffers hold deviations as lbm_get_populations
 * writes them.  The adjoint kernels use the instance's field scratch (what
 * lbm_fields last left there is overwritten).
 * ------------------------------------------------------------------------ */

/* Objectives of lbm_adjoint_seed (built on the paper's observables). */
#define LBM_OBJ_DP 0      /* smooth pressure jump <p_b>_A - <p_b>_B, p_b of Eq. 11 averaged
                             with weights max(0, +-phi)^4, phi = (rho_A - rho_B)/(rho_A + rho_B)
                             (Laplace test of Sec. III B without a droplet centre)            */
#define LBM_OBJ_Q 1       /* flow rate Q = (1/nx) sum_x u_x, u barycentric (Eq. 7); the
                             relative effective viscosity of Sec. III D is Q_0 / Q           */
#define LBM_OBJ_MOM_A 2   /* x-momentum of the populations of A, sum f_{A,i} e_{i,x}          */
#define LBM_OBJ_MOM 3     /* total x-momentum of the populations (theta-gradient zero)      */
#define LBM_OBJ_MASS_A 4  /* mass of A (theta-gradient zero)                                */

/* Adjoint of one time step of instance inst taken from state f_dev (time t):
 * lam_out_dev = (d f(t+1) / d f(t))^T lam_in_dev, and
 * grad_dev[0..4] += (d f(t+1) / d theta)^T lam_in_dev (device FP64, may be
 * NULL to skip the gradient).  lam_out_dev must not overlap f_dev or
 * lam_in_dev.  Asynchronous on the context's stream; consecutive calls on
 * one context are ordered by the stream.  The adjoint entry points return
 * LBM_EUNSUPPORTED for the velocity-shift forcing. */
int lbm_adjoint_step(lbm_ctx *ctx, int32_t inst, const float *f_dev, const float *lam_in_dev,
                     float *lam_out_dev, double *grad_dev);

/* Floats per state that lbm_record stores for instance inst: the state in
 * the library's own (opaque, padded) layout, populations and their density
 * deviations.  -1 for a bad context or instance. */
int64_t lbm_record_floats(const lbm_ctx *ctx, int32_t inst);

/* Forward run that keeps its states, for checkpoint-recompute: stores the
 * state of instance inst before each of nsteps steps, state j at
 * f_store_dev + j*lbm_record_floats(ctx, inst), while advancing the context
 * by nsteps steps (every instance).  The steps write these states in place
 * (no copies beyond the first state).  Asynchronous. */
int lbm_record(lbm_ctx *ctx, int32_t inst, int64_t nsteps, float *f_store_dev);

/* nsteps adjoint steps back through a recorded window: on entry lam_dev holds
 * dJ/df(t0 + nsteps), on return dJ/df(t0); f_store_dev holds the states
 * f(t0 + j), j = 0..nsteps-1, as lbm_record writes them (the recorded
 * densities spare the adjoint its own density pass).  lam_dev and tmp_dev
 * are buffers of one population state in the lbm_get_populations layout
 * (18*nx*ny floats); neither may overlap the store or each other.
 * grad_dev[0..4] (device FP64, may be NULL) += the theta-gradient of the
 * window, reduced once in a fixed order.  The result equals nsteps calls of
 * lbm_adjoint_step bit for bit in lam (one launch per step: each step also
 * transposes the force stencils of the step after it).  Asynchronous. */
int lbm_adjoint_run(lbm_ctx *ctx, int32_t inst, int64_t nsteps, const float *f_store_dev,
                    float *lam_dev, float *tmp_dev, double *grad_dev);

/* Objective J(f) of state f_dev of instance inst (one of LBM_OBJ_*): *J
 * receives its value (FP64 accumulation), dtheta[0..4] the direct partial
 * derivatives dJ/dtheta at fixed f (host), and lam_dev (device, may be NULL
 * except for LBM_OBJ_Q) the seed dJ/df.  Synchronises the stream.  Returns
 * LBM_EINVAL if the pressure-jump objective finds only one phase. */
int lbm_adjoint_seed(lbm_ctx *ctx, int32_t inst, int32_t objective, const float *f_dev,
                     float *lam_dev, double *J, double *dtheta);

/* Replace the model parameters of instance inst (couplings, relaxation
 * times, body force, pseudopotential scale, wall densities); nx, ny, walls
 * and rho_ref must equal the current ones (LBM_EINVAL otherwise), so the
 * state stays valid.  Synchronises the stream; captured graphs stay valid
 * and use the new values. */
int lbm_set_params(lbm_ctx *ctx, int32_t inst, const lbm_params *params);

/* Time the kernels of one adjoint step of instance inst like
 * lbm_profile_step (nrep launches of each kernel between HIP events on the
 * context's stream): the density pass, the local transpose, the force
 * transpose, the final sums, and the local transpose with the force
 * transpose of the step before folded in (the kernel of an adjoint run's
 * later steps).  ms[j] and names[j] for j < min(max_k, *n_kernels).
 * lam_out_dev and grad_dev are overwritten with meaningless values.
 * Synchronises the stream. */
int lbm_profile_adjoint(lbm_ctx *ctx, int32_t inst, const float *f_dev, const float *lam_in_dev,
                        float *lam_out_dev, double *grad_dev, int32_t nrep, int32_t max_k,
                        double *ms, const char **names, int32_t *n_kernels);

/* Debugging: in the checked build of the library (compiled with
 * LBM_CHECK_LDS), every launch of the fused step checks the indices of its
 * LDS ring and edge arrays, and *violations receives the number of
 * out-of-range indices seen on this device since the previous call (the
 * counter is then reset; an out-of-range index is counted, not used).
 * Synchronises the stream.  LBM_EUNSUPPORTED in the plain build. */
int lbm_lds_checks(lbm_ctx *ctx, int64_t *violations);

/* Release host resources of the context (graphs, metadata).  Synchronises
 * the stream; never frees caller memory. */
int lbm_destroy(lbm_ctx *ctx);

/* Message of the last failure on ctx (or of the last failed lbm_init when
 * ctx is NULL). */
const char *lbm_last_error(const lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
