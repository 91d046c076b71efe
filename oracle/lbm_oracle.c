/*
 * FP64 CPU oracle of the two-range pseudopotential lattice Boltzmann step
 * for a binary mixture with per-component relaxation times
 * (Fei, Scagliarini, Montessori, Lauricella, Succi, Luo,
 *  "Mesoscopic model for soft flowing systems with tunable viscosity ratio",
 *  arXiv:1806.06943, Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the HIP path is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant with the HIP library: every
 * weight below is typed here from the paper.
 *
 * Layout (all double precision, row-major, x fastest):
 *   f   [k][i][y][x]   k in {A=0,B=1}, i in 0..8 (D2Q9)
 *   rho [k][y][x]
 *   F   [k][d][y][x]   d in {x=0,y=1}
 *
 * D2Q9 ordering (the paper's Fig. 1 is not available; any consistent order
 * gives identical results):
 *   0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
 *
 * Forcing: the present model's Guo term with the common velocity (Eq. 5,
 * forcing = 0), or, for comparison, the velocity shift of the original
 * two-range model in its explicit form C^SC (Sec. II A, forcing = 1; the
 * common velocity then averages the bare population momenta).
 *
 * Readings of points the paper leaves open (each is listed with its reason
 * in the design notes of the repository):
 *   - equilibrium carries the usual factor 1/2 on the quadratic term
 *     (Eq. 2 as printed omits it; without it the second moment is wrong);
 *   - within a step: densities -> pseudopotential -> forces -> moments with
 *     F/2 -> common velocity -> BGK + Guo collision -> streaming;
 *   - the mid-range sum of Eq. 8 runs over all 25 vectors of D2Q25 (both
 *     belts), exactly as the equation is written;
 *   - body force F^b_k = rho_k g_k (g an acceleration per component);
 *   - walls (walls=1): x periodic, half-way bounce-back half a link below
 *     row 0 and above row ny-1; the force stencil sees virtual densities
 *     rho_wall[k] at rows outside the fluid.
 *
 * Parity pins: lattice moment sums, equilibrium/forcing moments, a
 * sinusoidal closed form of both stencils, an exact-rational brute force on
 * a 4x4 torus, mass and momentum identities, Laplace's law and the
 * two-component Poiseuille profile (Eq. 19) are checked by the tests.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int nx, ny, walls;
    double G_AB;        /* Eq. 9 inter-species coupling (>0 repulsive)   */
    double G1[2];       /* Eq. 8 short-range coupling per component       */
    double G2[2];       /* Eq. 8 mid-range coupling per component         */
    double tau[2];      /* Eq. 1 relaxation time per component            */
    double rho0;        /* pseudopotential reference density (Sec. II B)  */
    double g[2][2];     /* body acceleration per component, (x, y)        */
    double rho_wall[2]; /* virtual densities beyond the walls             */
    int forcing;        /* 0: Guo term with the common velocity (Eq. 5);
                           1: velocity shift of the original model (the
                           explicit form C^SC of Sec. II A)              */
} ora_params;

/* number of OpenMP threads the row loops use (1 without OpenMP) */
int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads for the following row loops (timing of the oracle on n cores) */
void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---- lattice tables, typed from Sec. II A (D2Q9) and Sec. II B (D2Q25) ---- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0;

/* w(|e|^2): w(0)=4/9, w(1)=1/9, w(2)=1/36 (Eq. 2) */
static double w_of(int e2)
{
    switch (e2) {
    case 0: return 4.0 / 9.0;
    case 1: return 1.0 / 9.0;
    case 2: return 1.0 / 36.0;
    }
    return 0.0;
}

/* p(|e|^2) for D2Q25 (Eq. 8): p(0)=247/420, p(1)=4/63, p(2)=4/135,
 * p(4)=1/180, p(5)=2/945, p(8)=1/15120; zero for every other |e|^2. */
static double p_of(int e2)
{
    switch (e2) {
    case 0: return 247.0 / 420.0;
    case 1: return 4.0 / 63.0;
    case 2: return 4.0 / 135.0;
    case 4: return 1.0 / 180.0;
    case 5: return 2.0 / 945.0;
    case 8: return 1.0 / 15120.0;
    }
    return 0.0;
}

static double wi(int i) { return w_of(EX[i] * EX[i] + EY[i] * EY[i]); }

/* Exported copy of the tables so that tests can check them against the
 * paper's numbers and the isotropy sums.  D2Q25 order: dy outer, dx inner,
 * both from -2 to 2. */
void ora_tables(int *ex9, int *ey9, int *opp9, double *w9,
                int *ex25, int *ey25, double *p25)
{
    for (int i = 0; i < 9; ++i) {
        ex9[i] = EX[i];
        ey9[i] = EY[i];
        opp9[i] = OPP[i];
        w9[i] = wi(i);
    }
    int j = 0;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            ex25[j] = dx;
            ey25[j] = dy;
            p25[j] = p_of(dx * dx + dy * dy);
            ++j;
        }
}

/* ---- indexing helpers ---- */
static int wrap(int a, int n)
{
    if (a >= 0 && a < n) return a;
    int r = a % n;
    return r < 0 ? r + n : r;
}

static size_t NODE(const ora_params *p, int x, int y)
{
    return (size_t)y * p->nx + x;
}

static size_t FIDX(const ora_params *p, int k, int i, int x, int y)
{
    size_t N = (size_t)p->nx * p->ny;
    return ((size_t)k * 9 + i) * N + NODE(p, x, y);
}

/* pseudopotential psi(rho) = rho0 (1 - exp(-rho/rho0)) (Sec. II B) */
static double psi_of(const ora_params *p, double rho)
{
    return p->rho0 * (1.0 - exp(-rho / p->rho0));
}

/* Source of densities for the force stencil: precomputed density and
 * pseudopotential arrays (rho != NULL), or, when rho is NULL, sums of the
 * populations taken on demand (used to step a single node of a large
 * lattice). */
typedef struct {
    const double *rho;
    const double *psi;
    const double *f;
} dens_src;

/* Density of component k seen at (x, y): periodic in x; periodic in y
 * without walls, the virtual wall density beyond the walls. */
static double rho_at(const ora_params *p, const dens_src *s, int k, int x, int y)
{
    x = wrap(x, p->nx);
    if (p->walls) {
        if (y < 0 || y >= p->ny) return p->rho_wall[k];
    } else {
        y = wrap(y, p->ny);
    }
    if (s->rho) return s->rho[(size_t)k * p->nx * p->ny + NODE(p, x, y)];
    double r = 0.0;
    for (int i = 0; i < 9; ++i) r += s->f[FIDX(p, k, i, x, y)];
    return r;
}

/* Pseudopotential of component k seen at (x, y), same wrapping rules. */
static double psi_at(const ora_params *p, const dens_src *s, int k, int x, int y)
{
    if (!s->psi) return psi_of(p, rho_at(p, s, k, x, y));
    x = wrap(x, p->nx);
    if (p->walls) {
        if (y < 0 || y >= p->ny) return psi_of(p, p->rho_wall[k]);
    } else {
        y = wrap(y, p->ny);
    }
    return s->psi[(size_t)k * p->nx * p->ny + NODE(p, x, y)];
}

/* psi[k][y][x] from rho[k][y][x] */
static void psi_field(const ora_params *p, const double *rho, double *psi)
{
    size_t n2 = 2 * (size_t)p->nx * p->ny;
    for (size_t n = 0; n < n2; ++n) psi[n] = psi_of(p, rho[n]);
}

/* ---- Eq. 6: component densities ---- */
void ora_density(const ora_params *p, const double *f, double *rho)
{
    size_t N = (size_t)p->nx * p->ny;
    for (int k = 0; k < 2; ++k)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double s = 0.0;
                for (int i = 0; i < 9; ++i) s += f[FIDX(p, k, i, x, y)];
                rho[(size_t)k * N + NODE(p, x, y)] = s;
            }
}

/* ---- Eqs. 8, 9 and the body force: total force on component k at one node ---- */
static void force_at(const ora_params *p, const dens_src *rho, int k, int x, int y,
                     double *Fx, double *Fy)
{
    int kb = 1 - k;
    double psi_x = psi_at(p, rho, k, x, y);
    double rho_x = rho_at(p, rho, k, x, y);

    /* short-range attraction within k: sum over D2Q9 with weights w */
    double s1x = 0.0, s1y = 0.0;
    for (int i = 0; i < 9; ++i) {
        double ps = psi_at(p, rho, k, x + EX[i], y + EY[i]);
        s1x += wi(i) * ps * EX[i];
        s1y += wi(i) * ps * EY[i];
    }
    /* mid-range repulsion within k: sum over all of D2Q25 with weights p */
    double s2x = 0.0, s2y = 0.0;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            double ps = psi_at(p, rho, k, x + dx, y + dy);
            double pw = p_of(dx * dx + dy * dy);
            s2x += pw * ps * dx;
            s2y += pw * ps * dy;
        }
    /* inter-species repulsion: density (not psi) of the other component */
    double srx = 0.0, sry = 0.0;
    for (int i = 0; i < 9; ++i) {
        double rb = rho_at(p, rho, kb, x + EX[i], y + EY[i]);
        srx += wi(i) * rb * EX[i];
        sry += wi(i) * rb * EY[i];
    }
    *Fx = -p->G1[k] * psi_x * s1x - p->G2[k] * psi_x * s2x - p->G_AB * rho_x * srx
          + rho_x * p->g[k][0];
    *Fy = -p->G1[k] * psi_x * s1y - p->G2[k] * psi_x * s2y - p->G_AB * rho_x * sry
          + rho_x * p->g[k][1];
}

void ora_forces(const ora_params *p, const double *rho_arr, double *F)
{
    size_t N = (size_t)p->nx * p->ny;
    double *psi = (double *)malloc(2 * N * sizeof(double));
    psi_field(p, rho_arr, psi);
    dens_src rho = {rho_arr, psi, NULL};
    for (int k = 0; k < 2; ++k)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double fx, fy;
                force_at(p, &rho, k, x, y, &fx, &fy);
                F[((size_t)k * 2 + 0) * N + NODE(p, x, y)] = fx;
                F[((size_t)k * 2 + 1) * N + NODE(p, x, y)] = fy;
            }
    free(psi);
}

/* ---- Eq. 2 with the 1/2 on the quadratic term ---- */
static double feq_i(int i, double rho, double ux, double uy)
{
    double eu = EX[i] * ux + EY[i] * uy;
    double uu = ux * ux + uy * uy;
    return wi(i) * rho * (1.0 + eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2));
}

void ora_feq(double rho, double ux, double uy, double *out9)
{
    for (int i = 0; i < 9; ++i) out9[i] = feq_i(i, rho, ux, uy);
}

/* ---- Eq. 5: Guo forcing term evaluated with the common velocity ---- */
static double guo_i(int i, double tau, double ux, double uy, double Fx, double Fy)
{
    double eu = EX[i] * ux + EY[i] * uy;
    double cx = (EX[i] - ux) / CS2 + eu * EX[i] / (CS2 * CS2);
    double cy = (EY[i] - uy) / CS2 + eu * EY[i] / (CS2 * CS2);
    return (1.0 - 1.0 / (2.0 * tau)) * wi(i) * (cx * Fx + cy * Fy);
}

void ora_guo(double tau, double ux, double uy, double Fx, double Fy, double *out9)
{
    for (int i = 0; i < 9; ++i) out9[i] = guo_i(i, tau, ux, uy, Fx, Fy);
}

/* ---- Eqs. 6 and 3: moments with F/2 and the common velocity at a node ----
 * jx, jy carry F/2 (Eq. 6) for the observables in either scheme; the common
 * velocity (Eq. 3) averages the component momenta of the scheme: with F/2
 * for the Guo term, the bare population momenta for the velocity shift. */
typedef struct {
    double rho[2], jx[2], jy[2], Fx[2], Fy[2], ux, uy;
} node_macro;

static void macro_at(const ora_params *p, const double *f, const dens_src *rho, int x,
                     int y, node_macro *m)
{
    double numx = 0.0, numy = 0.0, den = 0.0;
    for (int k = 0; k < 2; ++k) {
        double mx = 0.0, my = 0.0;
        for (int i = 0; i < 9; ++i) {
            double fi = f[FIDX(p, k, i, x, y)];
            mx += fi * EX[i];
            my += fi * EY[i];
        }
        m->rho[k] = rho_at(p, rho, k, x, y);
        force_at(p, rho, k, x, y, &m->Fx[k], &m->Fy[k]);
        m->jx[k] = mx + 0.5 * m->Fx[k];
        m->jy[k] = my + 0.5 * m->Fy[k];
        numx += (p->forcing ? mx : m->jx[k]) / p->tau[k];
        numy += (p->forcing ? my : m->jy[k]) / p->tau[k];
        den += m->rho[k] / p->tau[k];
    }
    m->ux = numx / den;
    m->uy = numy / den;
}

/* ---- velocity-shift forcing term of the original model (Sec. II A) ----
 * C^SC = [f^eq(rho, u + F tau / rho) - f^eq(rho, u)] / tau */
static double shift_i(int i, double tau, double rho, double ux, double uy, double Fx, double Fy)
{
    return (feq_i(i, rho, ux + Fx * tau / rho, uy + Fy * tau / rho) - feq_i(i, rho, ux, uy)) / tau;
}

void ora_shift(double tau, double rho, double ux, double uy, double Fx, double Fy, double *out9)
{
    for (int i = 0; i < 9; ++i) out9[i] = shift_i(i, tau, rho, ux, uy, Fx, Fy);
}

/* ---- Eq. 1 right-hand side: post-collision value of f_{k,i} at a node ---- */
static double post_collision(const ora_params *p, const double *f, const node_macro *m,
                             int k, int i, int x, int y)
{
    double fi = f[FIDX(p, k, i, x, y)];
    double tau = p->tau[k];
    double eq = feq_i(i, m->rho[k], m->ux, m->uy);
    double c = p->forcing ? shift_i(i, tau, m->rho[k], m->ux, m->uy, m->Fx[k], m->Fy[k])
                          : guo_i(i, tau, m->ux, m->uy, m->Fx[k], m->Fy[k]);
    return fi - (fi - eq) / tau + c;
}

/* ---- one full time step: fnew = stream(collide(f)) ----
 * work must hold 4*nx*ny doubles (densities and pseudopotentials). */
void ora_step(const ora_params *p, const double *f, double *fnew, double *work)
{
    size_t N = (size_t)p->nx * p->ny;
    ora_density(p, f, work);
    psi_field(p, work, work + 2 * N);
    dens_src rho = {work, work + 2 * N, NULL};
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            node_macro m;
            macro_at(p, f, &rho, x, y, &m);
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < 9; ++i) {
                    double fs = post_collision(p, f, &m, k, i, x, y);
                    int xd = wrap(x + EX[i], p->nx);
                    int yd = y + EY[i];
                    if (p->walls && (yd < 0 || yd >= p->ny)) {
                        /* half-way bounce-back: returns to the same node reversed */
                        fnew[FIDX(p, k, OPP[i], x, y)] = fs;
                    } else {
                        yd = wrap(yd, p->ny);
                        fnew[FIDX(p, k, i, xd, yd)] = fs;
                    }
                }
        }
}

/* Advance f in place by nsteps.  work must hold 22*nx*ny doubles. */
void ora_run(const ora_params *p, double *f, long nsteps, double *work)
{
    size_t N = (size_t)p->nx * p->ny;
    double *tmp = work;
    double *rho = work + 18 * N;
    for (long s = 0; s < nsteps; ++s) {
        ora_step(p, f, tmp, rho);
        memcpy(f, tmp, 18 * N * sizeof(double));
    }
}

/* Next-step populations of one node (x, y), in the pull form of the same
 * update: f_{k,i}(x, t+1) is the post-collision value at x - e_i, or, when
 * x - e_i lies beyond a wall, the reversed post-collision value of x itself.
 * Densities are summed on demand, so only the neighbourhood of (x, y) is
 * touched: used to check sampled nodes of lattices too large to step whole.
 * out18 = [k][i]. */
void ora_step_at(const ora_params *p, const double *f, int x, int y, double *out18)
{
    dens_src rho = {NULL, NULL, f};
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i) {
            int sx = x - EX[i], sy = y - EY[i], ii = i;
            if (p->walls && (sy < 0 || sy >= p->ny)) {
                sx = x;
                sy = y;
                ii = OPP[i];
            }
            sx = wrap(sx, p->nx);
            sy = wrap(sy, p->ny);
            node_macro m;
            macro_at(p, f, &rho, sx, sy, &m);
            out18[k * 9 + i] = post_collision(p, f, &m, k, ii, sx, sy);
        }
}

/* ---- initial state: equilibrium at rest from given densities (reading) ---- */
void ora_init(const ora_params *p, const double *rhoA, const double *rhoB, double *f)
{
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x)
            for (int i = 0; i < 9; ++i) {
                f[FIDX(p, 0, i, x, y)] = wi(i) * rhoA[NODE(p, x, y)];
                f[FIDX(p, 1, i, x, y)] = wi(i) * rhoB[NODE(p, x, y)];
            }
}

/* ---- macroscopic fields for observables ----
 * rho[k][y][x], j[k][d][y][x] (component momentum with F/2, Eq. 6),
 * F[k][d][y][x], ueq[d][y][x] (Eq. 3), u[d][y][x] (barycentric, Eq. 7),
 * pb[y][x] (bulk equation of state, Eq. 11).  Any output may be NULL. */
void ora_fields(const ora_params *p, const double *f, double *rho_out, double *j_out,
                double *F_out, double *ueq_out, double *u_out, double *pb_out)
{
    size_t N = (size_t)p->nx * p->ny;
    double *rho_arr = (double *)malloc(2 * N * sizeof(double));
    double *psi = (double *)malloc(2 * N * sizeof(double));
    ora_density(p, f, rho_arr);
    psi_field(p, rho_arr, psi);
    dens_src rho = {rho_arr, psi, NULL};
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            node_macro m;
            macro_at(p, f, &rho, x, y, &m);
            size_t n = NODE(p, x, y);
            double rt = m.rho[0] + m.rho[1];
            for (int k = 0; k < 2; ++k) {
                if (rho_out) rho_out[k * N + n] = m.rho[k];
                if (j_out) {
                    j_out[(k * 2 + 0) * N + n] = m.jx[k];
                    j_out[(k * 2 + 1) * N + n] = m.jy[k];
                }
                if (F_out) {
                    F_out[(k * 2 + 0) * N + n] = m.Fx[k];
                    F_out[(k * 2 + 1) * N + n] = m.Fy[k];
                }
            }
            if (ueq_out) {
                ueq_out[n] = m.ux;
                ueq_out[N + n] = m.uy;
            }
            if (u_out) {
                u_out[n] = (m.jx[0] + m.jx[1]) / rt;
                u_out[N + n] = (m.jy[0] + m.jy[1]) / rt;
            }
            if (pb_out) {
                double s = 0.0;
                for (int k = 0; k < 2; ++k) {
                    double ps = psi_of(p, m.rho[k]);
                    s += (m.rho[k] + 0.5 * (p->G1[k] + p->G2[k]) * ps * ps) * CS2;
                }
                s += p->G_AB * m.rho[0] * m.rho[1] * CS2;
                pb_out[n] = s;
            }
        }
    free(rho_arr);
    free(psi);
}

/* ======================================================================
 * Reverse-mode adjoint of one time step and differentiable objectives.
 *
 * The paper does not treat gradients; this section is the transpose of the
 * derivative of the step defined above (Eqs. 1, 2, 3, 5, 6, 8, 9 with the
 * readings listed at the top), written equation by equation in reverse
 * order.  For one step f(t+1) = Phi(f(t); theta), given
 * lam_next = dJ/df(t+1) it returns lam = (dPhi/df)^T lam_next and adds
 * (dPhi/dtheta)^T lam_next to grad, with
 *   theta = (G1, G2, G_AB, tau_A, tau_B),
 * where G1 and G2 move the couplings of both components together.
 * Everything is FP64, no blocking, one node at a time; the nonlocal part of
 * the force is transposed as a scatter (the literal transpose of the
 * gather in force_at).
 * ====================================================================== */

/* Sums of the three stencils of Eqs. 8 and 9 at one node (the bracketed
 * sums of force_at, without the prefactors). */
typedef struct {
    double s1x, s1y; /* sum_i w_i psi_k(x + e_i) e_i over D2Q9   */
    double s2x, s2y; /* sum_j p_j psi_k(x + e_j) e_j over D2Q25  */
    double srx, sry; /* sum_i w_i rho_kbar(x + e_i) e_i          */
} stencil_sums;

static void stencil_sums_at(const ora_params *p, const dens_src *rho, int k, int x, int y,
                            stencil_sums *s)
{
    int kb = 1 - k;
    memset(s, 0, sizeof(*s));
    for (int i = 0; i < 9; ++i) {
        double ps = psi_at(p, rho, k, x + EX[i], y + EY[i]);
        s->s1x += wi(i) * ps * EX[i];
        s->s1y += wi(i) * ps * EY[i];
        double rb = rho_at(p, rho, kb, x + EX[i], y + EY[i]);
        s->srx += wi(i) * rb * EX[i];
        s->sry += wi(i) * rb * EY[i];
    }
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            double ps = psi_at(p, rho, k, x + dx, y + dy);
            double pw = p_of(dx * dx + dy * dy);
            s->s2x += pw * ps * dx;
            s->s2y += pw * ps * dy;
        }
}

/* Lattice node seen at (x, y) with the force stencil's wrapping rules:
 * returns 0 when (x, y) lies beyond a wall (a fixed virtual density that no
 * adjoint flows into), else 1 with the wrapped node index in *n. */
static int node_in_lattice(const ora_params *p, int x, int y, size_t *n)
{
    x = wrap(x, p->nx);
    if (p->walls) {
        if (y < 0 || y >= p->ny) return 0;
    } else {
        y = wrap(y, p->ny);
    }
    *n = NODE(p, x, y);
    return 1;
}

/* Transpose of the force (Eqs. 8, 9 and F^b = rho g) for a field of force
 * adjoints Fbar[k][d][y][x]: adds d J / d rho_k to rhobar[k][y][x] (through
 * psi, the inter-species density and the body force) and the direct coupling
 * gradients to gG[3] = (G1, G2, G_AB). */
static void force_transpose(const ora_params *p, const dens_src *rho, const double *Fbar,
                            double *rhobar, double *gG)
{
    size_t N = (size_t)p->nx * p->ny;
    double *psibar = (double *)calloc(2 * N, sizeof(double));
    for (int k = 0; k < 2; ++k) {
        int kb = 1 - k;
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t n = NODE(p, x, y);
                double fbx = Fbar[((size_t)k * 2 + 0) * N + n];
                double fby = Fbar[((size_t)k * 2 + 1) * N + n];
                if (fbx == 0.0 && fby == 0.0) continue;
                stencil_sums s;
                stencil_sums_at(p, rho, k, x, y, &s);
                double psi_x = psi_at(p, rho, k, x, y);
                double rho_x = rho_at(p, rho, k, x, y);
                /* own-node factors: psi_k(x) and rho_k(x) */
                psibar[(size_t)k * N + n] +=
                    -p->G1[k] * (s.s1x * fbx + s.s1y * fby) - p->G2[k] * (s.s2x * fbx + s.s2y * fby);
                rhobar[(size_t)k * N + n] += -p->G_AB * (s.srx * fbx + s.sry * fby)
                                             + p->g[k][0] * fbx + p->g[k][1] * fby;
                /* coupling gradients */
                gG[0] += -psi_x * (s.s1x * fbx + s.s1y * fby);
                gG[1] += -psi_x * (s.s2x * fbx + s.s2y * fby);
                gG[2] += -rho_x * (s.srx * fbx + s.sry * fby);
                /* neighbours: psi_k(x + e) in the two psi stencils */
                for (int dy = -2; dy <= 2; ++dy)
                    for (int dx = -2; dx <= 2; ++dx) {
                        int e2 = dx * dx + dy * dy;
                        double c = p->G2[k] * p_of(e2) + (e2 <= 2 ? p->G1[k] * w_of(e2) : 0.0);
                        size_t m;
                        if (!node_in_lattice(p, x + dx, y + dy, &m)) continue;
                        psibar[(size_t)k * N + m] += -psi_x * c * (dx * fbx + dy * fby);
                    }
                /* neighbours: rho_kbar(x + e_i) in the inter-species stencil */
                for (int i = 0; i < 9; ++i) {
                    size_t m;
                    if (!node_in_lattice(p, x + EX[i], y + EY[i], &m)) continue;
                    rhobar[(size_t)kb * N + m] +=
                        -p->G_AB * rho_x * wi(i) * (EX[i] * fbx + EY[i] * fby);
                }
            }
    }
    /* psi_k = rho0 (1 - exp(-rho_k / rho0))  =>  dpsi/drho = exp(-rho_k / rho0) */
    for (int k = 0; k < 2; ++k)
        for (size_t n = 0; n < N; ++n)
            rhobar[(size_t)k * N + n] +=
                psibar[(size_t)k * N + n] * exp(-rho->rho[(size_t)k * N + n] / p->rho0);
    free(psibar);
}

/* Adjoint of one step.  f = state at t, lam_next = dJ/df(t+1), both
 * [k][i][y][x]; writes lam = dJ/df(t) and adds to grad[5].
 * work must hold 10*nx*ny doubles. */
void ora_adjoint_step(const ora_params *p, const double *f, const double *lam_next, double *lam,
                      double *grad, double *work)
{
    size_t N = (size_t)p->nx * p->ny;
    if (p->forcing) { /* the adjoint is written for the Guo term only */
        for (size_t n = 0; n < 18 * N; ++n) lam[n] = NAN;
        return;
    }
    double *rho_arr = work, *psi = work + 2 * N, *Fbar = work + 4 * N, *rhobar = work + 8 * N;
    ora_density(p, f, rho_arr);
    psi_field(p, rho_arr, psi);
    dens_src rho = {rho_arr, psi, NULL};
    memset(Fbar, 0, 4 * N * sizeof(double));
    memset(rhobar, 0, 2 * N * sizeof(double));
    double gtau[2] = {0.0, 0.0};

    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            size_t n = NODE(p, x, y);
            node_macro m;
            macro_at(p, f, &rho, x, y, &m);
            double D = m.rho[0] / p->tau[0] + m.rho[1] / p->tau[1];
            double uu = m.ux * m.ux + m.uy * m.uy;

            /* transpose of streaming: the post-collision f*_{k,i}(x) went to
             * x + e_i, or back to x reversed across a wall */
            double a[2][9];
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < 9; ++i) {
                    int yd = y + EY[i];
                    if (p->walls && (yd < 0 || yd >= p->ny))
                        a[k][i] = lam_next[FIDX(p, k, OPP[i], x, y)];
                    else
                        a[k][i] = lam_next[FIDX(p, k, i, wrap(x + EX[i], p->nx), wrap(yd, p->ny))];
                }

            /* transpose of Eq. 1 (BGK + Guo) at fixed rho_k, u, F_k */
            double ubx = 0.0, uby = 0.0;
            double rbar[2], Fbx[2], Fby[2];
            for (int k = 0; k < 2; ++k) {
                double tau = p->tau[k], c = 1.0 - 1.0 / (2.0 * tau);
                rbar[k] = 0.0;
                Fbx[k] = 0.0;
                Fby[k] = 0.0;
                for (int i = 0; i < 9; ++i) {
                    double eu = EX[i] * m.ux + EY[i] * m.uy;
                    double eF = EX[i] * m.Fx[k] + EY[i] * m.Fy[k];
                    double E = 1.0 + eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2);
                    /* f^eq = w rho E(u) */
                    rbar[k] += a[k][i] * wi(i) * E / tau;
                    double dEx = EX[i] / CS2 + eu * EX[i] / (CS2 * CS2) - m.ux / CS2;
                    double dEy = EY[i] / CS2 + eu * EY[i] / (CS2 * CS2) - m.uy / CS2;
                    ubx += a[k][i] / tau * wi(i) * m.rho[k] * dEx;
                    uby += a[k][i] / tau * wi(i) * m.rho[k] * dEy;
                    /* Guo term c w [ (e - u)/cs2 + (e.u) e / cs4 ] . F */
                    double gx = (EX[i] - m.ux) / CS2 + eu * EX[i] / (CS2 * CS2);
                    double gy = (EY[i] - m.uy) / CS2 + eu * EY[i] / (CS2 * CS2);
                    Fbx[k] += a[k][i] * c * wi(i) * gx;
                    Fby[k] += a[k][i] * c * wi(i) * gy;
                    ubx += a[k][i] * c * wi(i) * (-m.Fx[k] / CS2 + eF * EX[i] / (CS2 * CS2));
                    uby += a[k][i] * c * wi(i) * (-m.Fy[k] / CS2 + eF * EY[i] / (CS2 * CS2));
                    /* tau_k: -(f - feq)/tau and the (1 - 1/(2 tau)) factor */
                    double fi = f[FIDX(p, k, i, x, y)];
                    double eq = wi(i) * m.rho[k] * E;
                    gtau[k] += a[k][i] * (fi - eq) / (tau * tau);
                    gtau[k] += a[k][i] * wi(i) * (gx * m.Fx[k] + gy * m.Fy[k]) / (2.0 * tau * tau);
                }
            }
            /* transpose of Eq. 3: u = sum_k j_k/tau_k / D, D = sum_k rho_k/tau_k */
            double mbx[2], mby[2];
            for (int k = 0; k < 2; ++k) {
                double tau = p->tau[k];
                double jbx = ubx / (tau * D), jby = uby / (tau * D);
                rbar[k] += -(ubx * m.ux + uby * m.uy) / (tau * D);
                gtau[k] += (ubx * (m.ux * m.rho[k] - m.jx[k]) + uby * (m.uy * m.rho[k] - m.jy[k]))
                           / (tau * tau * D);
                /* Eq. 6: j = sum f e + F/2 */
                mbx[k] = jbx;
                mby[k] = jby;
                Fbx[k] += 0.5 * jbx;
                Fby[k] += 0.5 * jby;
            }
            for (int k = 0; k < 2; ++k) {
                double tau = p->tau[k];
                for (int i = 0; i < 9; ++i)
                    lam[FIDX(p, k, i, x, y)] =
                        (1.0 - 1.0 / tau) * a[k][i] + mbx[k] * EX[i] + mby[k] * EY[i];
                rhobar[(size_t)k * N + n] += rbar[k];
                Fbar[((size_t)k * 2 + 0) * N + n] = Fbx[k];
                Fbar[((size_t)k * 2 + 1) * N + n] = Fby[k];
            }
        }

    /* transpose of the forces, then of Eq. 6's density sum */
    double gG[3] = {0.0, 0.0, 0.0};
    force_transpose(p, &rho, Fbar, rhobar, gG);
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i)
            for (size_t n = 0; n < N; ++n) lam[((size_t)k * 9 + i) * N + n] += rhobar[(size_t)k * N + n];
    grad[0] += gG[0];
    grad[1] += gG[1];
    grad[2] += gG[2];
    grad[3] += gtau[0];
    grad[4] += gtau[1];
}

/* Differentiable objectives of a state f (not in the paper; built on its
 * observables).  Returns J; if lam is not NULL writes dJ/df [k][i][y][x];
 * if dtheta is not NULL adds the direct dJ/dtheta (theta as above).
 *   0  J_dp   smooth pressure jump <p_b>_A - <p_b>_B, p_b of Eq. 11,
 *             weights chi_A = max(0, phi)^4, chi_B = max(0, -phi)^4,
 *             phi = (rho_A - rho_B) / (rho_A + rho_B)  (bulk phases count,
 *             interfaces do not; tolerates drifting droplets)
 *   1  J_Q    flow rate Q = sum_y ubar(y) = (1/nx) sum_x u_x, u barycentric
 *             with F/2 (Eq. 7); the relative effective viscosity of
 *             Sec. III D is Q_0 / Q
 *   2  J_momA x-momentum of the populations of A, sum_{x,i} f_{A,i} e_{i,x}
 *   3  J_mom  total x-momentum of the populations (its theta-gradient is
 *             exactly zero: the interaction forces sum to zero)
 *   4  J_massA mass of A (theta-gradient exactly zero)
 * work must hold 10*nx*ny doubles. */
double ora_objective(const ora_params *p, const double *f, int which, double *lam, double *dtheta,
                     double *work)
{
    size_t N = (size_t)p->nx * p->ny;
    double *rho_arr = work, *psi = work + 2 * N, *Fbar = work + 4 * N, *rhobar = work + 8 * N;
    ora_density(p, f, rho_arr);
    psi_field(p, rho_arr, psi);
    dens_src rho = {rho_arr, psi, NULL};
    memset(Fbar, 0, 4 * N * sizeof(double));
    memset(rhobar, 0, 2 * N * sizeof(double));
    if (lam) memset(lam, 0, 18 * N * sizeof(double));
    double J = 0.0;

    if (which == 0) {
        double SA = 0.0, SB = 0.0, PA = 0.0, PB = 0.0;
        double dPA[3] = {0, 0, 0}, dPB[3] = {0, 0, 0};
        for (size_t n = 0; n < N; ++n) {
            double ra = rho_arr[n], rb = rho_arr[N + n];
            double pa = psi[n], pb_ = psi[N + n];
            double pr = CS2 * (ra + 0.5 * (p->G1[0] + p->G2[0]) * pa * pa + rb
                               + 0.5 * (p->G1[1] + p->G2[1]) * pb_ * pb_ + p->G_AB * ra * rb);
            double phi = (ra - rb) / (ra + rb);
            double ca = phi > 0 ? phi * phi * phi * phi : 0.0;
            double cb = phi < 0 ? phi * phi * phi * phi : 0.0;
            double dG12 = CS2 * 0.5 * (pa * pa + pb_ * pb_), dGab = CS2 * ra * rb;
            SA += ca;
            SB += cb;
            PA += pr * ca;
            PB += pr * cb;
            dPA[0] += dG12 * ca; dPA[1] += dG12 * ca; dPA[2] += dGab * ca;
            dPB[0] += dG12 * cb; dPB[1] += dG12 * cb; dPB[2] += dGab * cb;
        }
        double mA = PA / SA, mB = PB / SB;
        J = mA - mB;
        if (dtheta)
            for (int t = 0; t < 3; ++t) dtheta[t] += dPA[t] / SA - dPB[t] / SB;
        if (lam)
            for (size_t n = 0; n < N; ++n) {
                double ra = rho_arr[n], rb = rho_arr[N + n];
                double pa = psi[n], pb_ = psi[N + n];
                double pr = CS2 * (ra + 0.5 * (p->G1[0] + p->G2[0]) * pa * pa + rb
                                   + 0.5 * (p->G1[1] + p->G2[1]) * pb_ * pb_ + p->G_AB * ra * rb);
                double s = ra + rb, phi = (ra - rb) / s;
                double dphi[2] = {2.0 * rb / (s * s), -2.0 * ra / (s * s)};
                double dp[2] = {
                    CS2 * (1.0 + (p->G1[0] + p->G2[0]) * pa * exp(-ra / p->rho0) + p->G_AB * rb),
                    CS2 * (1.0 + (p->G1[1] + p->G2[1]) * pb_ * exp(-rb / p->rho0) + p->G_AB * ra)};
                double ca = phi > 0 ? phi * phi * phi * phi : 0.0;
                double cb = phi < 0 ? phi * phi * phi * phi : 0.0;
                double dca = phi > 0 ? 4.0 * phi * phi * phi : 0.0;
                double dcb = phi < 0 ? 4.0 * phi * phi * phi : 0.0;
                for (int k = 0; k < 2; ++k) {
                    double d = (dp[k] * ca + (pr - mA) * dca * dphi[k]) / SA
                               - (dp[k] * cb + (pr - mB) * dcb * dphi[k]) / SB;
                    for (int i = 0; i < 9; ++i) lam[((size_t)k * 9 + i) * N + n] = d;
                }
            }
        return J;
    }

    if (which == 1) {
        double inv_nx = 1.0 / p->nx;
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t n = NODE(p, x, y);
                node_macro m;
                macro_at(p, f, &rho, x, y, &m);
                double rt = m.rho[0] + m.rho[1];
                double ux = (m.jx[0] + m.jx[1]) / rt;
                J += ux * inv_nx;
                for (int k = 0; k < 2; ++k) {
                    /* u_x = (sum_k m_kx + F_kx / 2) / rho */
                    if (lam)
                        for (int i = 0; i < 9; ++i)
                            lam[FIDX(p, k, i, x, y)] = inv_nx * (EX[i] - ux) / rt;
                    Fbar[((size_t)k * 2 + 0) * N + n] = 0.5 * inv_nx / rt;
                }
            }
        double gG[3] = {0.0, 0.0, 0.0};
        force_transpose(p, &rho, Fbar, rhobar, gG);
        if (lam)
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < 9; ++i)
                    for (size_t n = 0; n < N; ++n)
                        lam[((size_t)k * 9 + i) * N + n] += rhobar[(size_t)k * N + n];
        if (dtheta)
            for (int t = 0; t < 3; ++t) dtheta[t] += gG[t];
        return J;
    }

    /* linear functionals of the populations */
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i) {
            double c;
            if (which == 2) c = k == 0 ? EX[i] : 0.0;
            else if (which == 3) c = EX[i];
            else c = k == 0 ? 1.0 : 0.0;
            for (size_t n = 0; n < N; ++n) {
                J += c * f[((size_t)k * 9 + i) * N + n];
                if (lam) lam[((size_t)k * 9 + i) * N + n] = c;
            }
        }
    return J;
}

/* ======================================================================
 * Pressure tensor (Sec. II B) and the flat-interface integrals of Sec. II C.
 *
 * P = P^int + P^kin.  The kinetic part of the static problem is the second
 * moment of the populations, sum_{k,i} f_{k,i} e_i e_i (present model).
 * The interaction part is fixed by the paper only through its divergence
 * (minus the total force); for the pairwise lattice forces of Eqs. 8 and 9
 * the pair-sum (virial) form
 *   P^int_k(x) = 1/2 sum_e c_k(e) psi_k(x) psi_k(x+e) e e
 *              + 1/2 G_AB sum_i w_i rho_k(x) rho_kbar(x+e_i) e_i e_i,
 *   c_k(e) = G_{k,1} w(e) + G_{k,2} p(e),
 * is used: it equals the interaction part of the bulk equation of state
 * (Eq. 11) in a uniform state, and its sum over a flat interface is the
 * total virial of the pairs that cross it, which is what the surface-tension
 * integral (Eq. 15) needs.  For the velocity-shift forcing the kinetic part
 * is the paper's explicit sum_k rho_k cs^2 delta + K^tau (the tau-dependent
 * terms), with tau = (rho_A tau_A + rho_B tau_B) / rho, F the total force
 * and the density gradients by central differences (a reading: the paper
 * does not state the discretisation).
 * Output per node: P[c][y][x], c = 0: xx, 1: yy, 2: xy.
 * ====================================================================== */
void ora_pressure(const ora_params *p, const double *f, double *P)
{
    size_t N = (size_t)p->nx * p->ny;
    double *rho_arr = (double *)malloc(2 * N * sizeof(double));
    double *psi = (double *)malloc(2 * N * sizeof(double));
    ora_density(p, f, rho_arr);
    psi_field(p, rho_arr, psi);
    dens_src rho = {rho_arr, psi, NULL};
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            size_t n = NODE(p, x, y);
            double pxx = 0.0, pyy = 0.0, pxy = 0.0;
            for (int k = 0; k < 2; ++k) {
                int kb = 1 - k;
                double ps = psi_at(p, &rho, k, x, y), rk = rho_at(p, &rho, k, x, y);
                for (int dy = -2; dy <= 2; ++dy)
                    for (int dx = -2; dx <= 2; ++dx) {
                        int e2 = dx * dx + dy * dy;
                        if (e2 == 0) continue;
                        double c = p->G1[k] * w_of(e2) + p->G2[k] * p_of(e2);
                        double v = 0.5 * c * ps * psi_at(p, &rho, k, x + dx, y + dy);
                        if (e2 <= 2)
                            v += 0.5 * p->G_AB * w_of(e2) * rk * rho_at(p, &rho, kb, x + dx, y + dy);
                        pxx += v * dx * dx;
                        pyy += v * dy * dy;
                        pxy += v * dx * dy;
                    }
                if (!p->forcing) {
                    for (int i = 0; i < 9; ++i) {
                        double fi = f[FIDX(p, k, i, x, y)];
                        pxx += fi * EX[i] * EX[i];
                        pyy += fi * EY[i] * EY[i];
                        pxy += fi * EX[i] * EY[i];
                    }
                } else {
                    pxx += rk * CS2;
                    pyy += rk * CS2;
                }
            }
            if (p->forcing) {
                /* K^tau of the original model */
                double ra = rho_arr[n], rb = rho_arr[N + n], rt = ra + rb;
                double t = (ra * p->tau[0] + rb * p->tau[1]) / rt, t2 = (t - 0.5) * (t - 0.5);
                double F[2] = {0.0, 0.0};
                for (int k = 0; k < 2; ++k) {
                    double fx, fy;
                    force_at(p, &rho, k, x, y, &fx, &fy);
                    F[0] += fx;
                    F[1] += fy;
                }
                double g[2];
                g[0] = (log(rho_at(p, &rho, 0, x + 1, y)) - log(rho_at(p, &rho, 0, x - 1, y))
                        - log(rho_at(p, &rho, 1, x + 1, y)) + log(rho_at(p, &rho, 1, x - 1, y))) * 0.5;
                g[1] = (log(rho_at(p, &rho, 0, x, y + 1)) - log(rho_at(p, &rho, 0, x, y - 1))
                        - log(rho_at(p, &rho, 1, x, y + 1)) + log(rho_at(p, &rho, 1, x, y - 1))) * 0.5;
                double cc = CS2 * CS2 * ra * rb / rt * t2;
                pxx += t2 * F[0] * F[0] / rt + cc * g[0] * g[0];
                pyy += t2 * F[1] * F[1] / rt + cc * g[1] * g[1];
                pxy += t2 * F[0] * F[1] / rt + cc * g[0] * g[1];
            }
            P[n] = pxx;
            P[N + n] = pyy;
            P[2 * N + n] = pxy;
        }
    free(rho_arr);
    free(psi);
}
