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
 *   streaming            periodic in x; periodic in y, or half-way
 *                        bounce-back walls half a link outside rows 0
 *                        and ny-1                                      (Eq. 1, Sec. III A)
 *
 * Arithmetic is FP32; populations are stored as FP32 deviations
 * f_{k,i} - w_i rho_ref[k].  FP64 is used on the device only in the
 * reductions behind lbm_observables and the parameter gradients.
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
#define LBM_EUNSUPPORTED (-4) /* valid request that this build does not provide      */

typedef struct lbm_ctx lbm_ctx;

/* Model parameters of one lattice instance, as the paper states the model. */
typedef struct {
    int32_t nx, ny;      /* lattice size, each >= 1 (small tori alias the 5x5 stencil)   */
    int32_t walls;       /* 0: periodic x and y; 1: periodic x, walls below row 0 and
                            above row ny-1 (half-way bounce-back, Sec. III A)            */
    int32_t reserved;    /* must be 0                                                    */
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

/* Create a context for n_inst >= 1 independent instances.
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
 * the context's stream; long runs replay a captured HIP graph. */
int lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* Time steps taken since lbm_init (or the last lbm_set_populations). */
int64_t lbm_steps_done(const lbm_ctx *ctx);

/* FP64 observables of every instance into host out[n_inst]; if ubar is not
 * NULL it receives the x-mean of u_x per row, instance after instance
 * (sum of ny doubles).  Synchronises the stream.  Returns LBM_ENONFINITE
 * (after filling out) if any instance holds NaN or Inf. */
int lbm_observables(lbm_ctx *ctx, lbm_obs *out, double *ubar);

/* Density and barycentric velocity (Eq. 7) fields of instance inst, FP32,
 * into device buffers rho[2][ny][nx] and u[2][ny][nx] (either may be NULL).
 * Asynchronous. */
int lbm_fields(lbm_ctx *ctx, int32_t inst, float *rho_dev, float *u_dev);

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
 * (component, axis).  Uses the step's own force code; overwrites the
 * instance's internal density buffer (the next lbm_step recomputes it).
 * Asynchronous. */
int lbm_forces(lbm_ctx *ctx, int32_t inst, const float *rho_dev, float *F_dev);

/* Device-to-device copy of nbytes through the library's own streaming copy
 * kernel; used to measure the achievable HBM bandwidth.  Asynchronous. */
int lbm_copy_probe(lbm_ctx *ctx, void *dst_dev, const void *src_dev, uint64_t nbytes);

/* Time the kernels of one step: each kernel of the step is launched nrep
 * times back to back on the context's stream between two HIP events; ms[j]
 * receives the average duration of kernel j in milliseconds and names[j]
 * (if names is not NULL) a static string naming it.  *n_kernels receives the
 * number of kernels per step (at most max_k are written).  The state is left
 * unchanged.  Synchronises the stream. */
int lbm_profile_step(lbm_ctx *ctx, int32_t nrep, int32_t max_k, double *ms, const char **names,
                     int32_t *n_kernels);

/* Strip height of the fused step (lattice rows one wavefront advances per
 * step, default 16, at least 4).  Any value gives the same results bit for
 * bit; it trades halo recomputation against parallelism.  Synchronises the
 * stream and discards captured graphs. */
int lbm_set_tiling(lbm_ctx *ctx, int32_t chunk_rows);
int32_t lbm_get_tiling(const lbm_ctx *ctx);

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
