// HIP kernels of the two-range pseudopotential LBM step on gfx950
// (arXiv:1806.06943, Sec. II).  Every kernel walks a flat table of tiles
// (instance, x0, y0) or rows (instance, y), so one launch covers one lattice
// or many lattices of different sizes alike.
#include "lbm_internal.h"

namespace lbm {

// ------------------------------------------------------------------ init
// Equilibrium at rest, f_{k,i} = w_i rho_k (Eq. 2 with u = 0), written as the
// post-collision state of the step before: f*_i(x) = f_i(x + e_i, 0), or the
// node's own value when x + e_i lies beyond a wall.  rho0 holds FP64
// densities [k][ny][nx] (dense).
__global__ __launch_bounds__(NTHREADS) void k_init(const KInst *__restrict__ insts,
                                                    const int4 *__restrict__ tiles,
                                                    const double *const *__restrict__ rho0s,
                                                    int par)
{
    const int4 t = tiles[blockIdx.x];
    const KInst &P = insts[t.x];
    const int x = t.y + (int)(threadIdx.x % TX);
    const int y = t.z + (int)(threadIdx.x / TX);
    if (x >= P.nx || y >= P.ny) return;
    const double *rho0 = rho0s[t.x];
    const int64_t N = (int64_t)P.nx * P.ny;
    constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr double CI[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    float *out = P.f[par];
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i) {
            int xs = wrapi(x + EX[i], P.nx);
            int ys = y + EY[i];
            if (P.walls && (ys < 0 || ys >= P.ny)) {
                xs = x;
                ys = y;
            } else {
                ys = wrapi(ys, P.ny);
            }
            const double r = rho0[k * N + (int64_t)ys * P.nx + xs];
            out[(int64_t)(k * 9 + i) * P.plane + (int64_t)y * P.pitch + x] =
                (float)(CI[i] / 36.0 * (r - (double)P.rho_ref[k]));
        }
}

// ------------------------------------------------------------------ density pass
// rho_k(x) = rho_ref + sum_i f_i(x) (Eq. 6) for the pre-collision state.
__global__ __launch_bounds__(NTHREADS) void k_density(const KInst *__restrict__ insts,
                                                       const int4 *__restrict__ tiles, int par)
{
    const int4 t = tiles[blockIdx.x];
    const KInst &P = insts[t.x];
    const int x = t.y + (int)(threadIdx.x % TX);
    const int y = t.z + (int)(threadIdx.x / TX);
    if (x >= P.nx || y >= P.ny) return;
    float f[2][9];
    gather(P, P.f[par], x, y, f);
    const int64_t o = (int64_t)y * P.pitch + x;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        float hi, lo;
        sum9(f[k], hi, lo);
        P.rho[k * P.plane + o] = P.rho_ref[k] + (hi + lo);
    }
}

// ------------------------------------------------------------------ step
// Forces from the LDS density tile, moments, common velocity, BGK + Guo
// collision, pull streaming: reads f[par], writes f[par ^ 1].
__global__ __launch_bounds__(NTHREADS) void k_step(const KInst *__restrict__ insts,
                                                    const int4 *__restrict__ tiles, int par)
{
    __shared__ Tile T;
    const int4 t = tiles[blockIdx.x];
    const KInst &P = insts[t.x];
    stage_tile(P, t.y, t.z, T);
    __syncthreads();
    const int lx = (int)(threadIdx.x % TX), ly = (int)(threadIdx.x / TX);
    const int x = t.y + lx, y = t.z + ly;
    if (x >= P.nx || y >= P.ny) return;

    float f[2][9];
    gather(P, P.f[par], x, y, f);
    float F[2][2];
    tile_force(P, T, lx + HALO, ly + HALO, F);

    float dh[2], dl[2], rho[2], jx[2], jy[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        sum9(f[k], dh[k], dl[k]);
        rho[k] = T.rho[k][ly + HALO][lx + HALO];
        float mx, my;
        mom9(f[k], mx, my);
        jx[k] = mx + 0.5f * F[k][0];
        jy[k] = my + 0.5f * F[k][1];
    }
    float ux, uy;
    common_velocity(P, rho, jx, jy, ux, uy);

    float *out = P.f[par ^ 1];
    const int64_t o = (int64_t)y * P.pitch + x;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        float post[9];
        collide(P, k, f[k], dh[k], dl[k], rho[k], F[k][0], F[k][1], ux, uy, post);
#pragma unroll
        for (int i = 0; i < 9; ++i) out[(int64_t)(k * 9 + i) * P.plane + o] = post[i];
    }
}

// ------------------------------------------------------------------ fields
// Per-node FP32 fields for observables: rho_k, barycentric u (Eq. 7),
// bulk pressure p_b (Eq. 11), population momentum and total j (with F/2).
__global__ __launch_bounds__(NTHREADS) void k_fields(const KInst *__restrict__ insts,
                                                      const int4 *__restrict__ tiles, int par)
{
    __shared__ Tile T;
    const int4 t = tiles[blockIdx.x];
    const KInst &P = insts[t.x];
    stage_tile(P, t.y, t.z, T);
    __syncthreads();
    const int lx = (int)(threadIdx.x % TX), ly = (int)(threadIdx.x / TX);
    const int x = t.y + lx, y = t.z + ly;
    if (x >= P.nx || y >= P.ny) return;
    float f[2][9];
    gather(P, P.f[par], x, y, f);
    float F[2][2];
    tile_force(P, T, lx + HALO, ly + HALO, F);
    float rho[2], mxs = 0.f, mys = 0.f, jxs = 0.f, jys = 0.f;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        rho[k] = T.rho[k][ly + HALO][lx + HALO];
        float mx, my;
        mom9(f[k], mx, my);
        mxs += mx;
        mys += my;
        jxs += mx + 0.5f * F[k][0];
        jys += my + 0.5f * F[k][1];
    }
    const float rt = rho[0] + rho[1];
    const float pA = T.psi[0][ly + HALO][lx + HALO], pB = T.psi[1][ly + HALO][lx + HALO];
    const float pb = ((rho[0] + P.gpb[0] * pA * pA) + (rho[1] + P.gpb[1] * pB * pB) +
                      P.gab * rho[0] * rho[1]) / 3.0f;
    float *fl = P.fld;
    const int64_t o = (int64_t)y * P.pitch + x, pl = P.plane;
    fl[FLD_RHOA * pl + o] = rho[0];
    fl[FLD_RHOB * pl + o] = rho[1];
    fl[FLD_UX * pl + o] = jxs / rt;
    fl[FLD_UY * pl + o] = jys / rt;
    fl[FLD_PB * pl + o] = pb;
    fl[FLD_MX * pl + o] = mxs;
    fl[FLD_MY * pl + o] = mys;
    fl[FLD_JX * pl + o] = jxs;
    fl[FLD_JY * pl + o] = jys;
}

// Dense copies of rho and u of one instance (from the field scratch).
__global__ void k_fields_out(const KInst *__restrict__ insts, int inst, float *rho_out,
                             float *u_out)
{
    const KInst &P = insts[inst];
    const int64_t N = (int64_t)P.nx * P.ny;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(n / P.nx), x = (int)(n % P.nx);
        const int64_t o = (int64_t)y * P.pitch + x, pl = P.plane;
        if (rho_out) {
            rho_out[n] = P.fld[FLD_RHOA * pl + o];
            rho_out[N + n] = P.fld[FLD_RHOB * pl + o];
        }
        if (u_out) {
            u_out[n] = P.fld[FLD_UX * pl + o];
            u_out[N + n] = P.fld[FLD_UY * pl + o];
        }
    }
}

// ------------------------------------------------------------------ state import / export
__global__ __launch_bounds__(NTHREADS) void k_export(const KInst *__restrict__ insts,
                                                      const int4 *__restrict__ tiles, int inst,
                                                      int par, float *__restrict__ fout)
{
    const int4 t = tiles[blockIdx.x];
    if (t.x != inst) return;
    const KInst &P = insts[t.x];
    const int x = t.y + (int)(threadIdx.x % TX);
    const int y = t.z + (int)(threadIdx.x / TX);
    if (x >= P.nx || y >= P.ny) return;
    float f[2][9];
    gather(P, P.f[par], x, y, f);
    const int64_t N = (int64_t)P.nx * P.ny, n = (int64_t)y * P.nx + x;
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i) fout[(int64_t)(k * 9 + i) * N + n] = f[k][i];
}

// Inverse of k_export: pre-collision f(x) -> post-collision storage
// f*_i(x) = f_i(x + e_i), or f_opp(i)(x) when x + e_i lies beyond a wall.
__global__ __launch_bounds__(NTHREADS) void k_import(const KInst *__restrict__ insts,
                                                      const int4 *__restrict__ tiles, int inst,
                                                      int par, const float *__restrict__ fin)
{
    const int4 t = tiles[blockIdx.x];
    if (t.x != inst) return;
    const KInst &P = insts[t.x];
    const int x = t.y + (int)(threadIdx.x % TX);
    const int y = t.z + (int)(threadIdx.x / TX);
    if (x >= P.nx || y >= P.ny) return;
    constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    const int64_t N = (int64_t)P.nx * P.ny;
    float *out = P.f[par];
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 9; ++i) {
            int xs = wrapi(x + EX[i], P.nx), ys = y + EY[i], ii = i;
            if (P.walls && (ys < 0 || ys >= P.ny)) {
                xs = x;
                ys = y;
                ii = OPP[i];
            } else {
                ys = wrapi(ys, P.ny);
            }
            out[(int64_t)(k * 9 + i) * P.plane + (int64_t)y * P.pitch + x] =
                fin[(int64_t)(k * 9 + ii) * N + (int64_t)ys * P.nx + xs];
        }
}

// ------------------------------------------------------------------ forces only
__global__ void k_rho_in(const KInst *__restrict__ insts, int inst, const float *rho_in)
{
    const KInst &P = insts[inst];
    const int64_t N = (int64_t)P.nx * P.ny;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < 2 * N;
         n += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(n / N);
        const int64_t m = n % N;
        const int y = (int)(m / P.nx), x = (int)(m % P.nx);
        P.rho[k * P.plane + (int64_t)y * P.pitch + x] = rho_in[n];
    }
}

__global__ __launch_bounds__(NTHREADS) void k_forces(const KInst *__restrict__ insts,
                                                      const int4 *__restrict__ tiles, int inst,
                                                      float *__restrict__ Fout)
{
    __shared__ Tile T;
    const int4 t = tiles[blockIdx.x];
    if (t.x != inst) return;  // uniform per block: no thread reaches the barrier below
    const KInst &P = insts[t.x];
    stage_tile(P, t.y, t.z, T);
    __syncthreads();
    const int lx = (int)(threadIdx.x % TX), ly = (int)(threadIdx.x / TX);
    const int x = t.y + lx, y = t.z + ly;
    if (x >= P.nx || y >= P.ny) return;
    float F[2][2];
    tile_force(P, T, lx + HALO, ly + HALO, F);
    const int64_t N = (int64_t)P.nx * P.ny, n = (int64_t)y * P.nx + x;
    for (int k = 0; k < 2; ++k)
        for (int d = 0; d < 2; ++d) Fout[(int64_t)(k * 2 + d) * N + n] = F[k][d];
}

// ------------------------------------------------------------------ FP64 reductions
// One block per (instance, row); every quantity is accumulated in FP64 in a
// fixed order (per-thread strided loop, then an LDS tree), so results are
// bitwise reproducible.
constexpr int RT = 256;  // threads of reduction blocks

__device__ __forceinline__ double tree_sum(double v, double *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = RT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double tree_max(double v, double *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = RT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double tree_min(double v, double *s)
{
    return -tree_max(-v, s);
}

// pass 1 per row: masses and population momentum from the populations;
// total j, row sum of u_x, max |u|, extrema of rho_A, non-finite count.
__global__ __launch_bounds__(RT) void k_red_rows1(const KInst *__restrict__ insts,
                                                   const int2 *__restrict__ rows, int par,
                                                   double *__restrict__ part)
{
    __shared__ double s[RT];
    const int2 r = rows[blockIdx.x];
    const KInst &P = insts[r.x];
    const int y = r.y;
    const int64_t pl = P.plane;
    double mA = 0, mB = 0, px = 0, py = 0, jx = 0, jy = 0, su = 0, umax = 0;
    double amax = -INFINITY, amin = INFINITY, bad = 0;
    for (int x = threadIdx.x; x < P.nx; x += RT) {
        float f[2][9];
        gather(P, P.f[par], x, y, f);
        for (int i = 0; i < 9; ++i) {
            mA += (double)f[0][i];
            mB += (double)f[1][i];
        }
        constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        for (int k = 0; k < 2; ++k)
            for (int i = 0; i < 9; ++i) {
                px += (double)f[k][i] * EX[i];
                py += (double)f[k][i] * EY[i];
            }
        const int64_t o = (int64_t)y * P.pitch + x;
        const double ux = P.fld[FLD_UX * pl + o], uy = P.fld[FLD_UY * pl + o];
        const double ra = P.fld[FLD_RHOA * pl + o], rb = P.fld[FLD_RHOB * pl + o];
        jx += (double)P.fld[FLD_JX * pl + o];
        jy += (double)P.fld[FLD_JY * pl + o];
        su += ux;
        const double sp = sqrt(ux * ux + uy * uy);
        if (!(isfinite(ux) && isfinite(uy) && isfinite(ra) && isfinite(rb))) bad += 1;
        umax = fmax(umax, sp);
        amax = fmax(amax, ra);
        amin = fmin(amin, ra);
    }
    double *o = part + (int64_t)blockIdx.x * NQR;
    const double v0 = tree_sum(mA, s), v1 = tree_sum(mB, s), v2 = tree_sum(px, s),
                 v3 = tree_sum(py, s), v4 = tree_sum(jx, s), v5 = tree_sum(jy, s),
                 v6 = tree_sum(su, s), v7 = tree_max(umax, s), v8 = tree_max(amax, s),
                 v9 = tree_min(amin, s), v10 = tree_sum(bad, s);
    if (threadIdx.x == 0) {
        o[0] = v0; o[1] = v1; o[2] = v2; o[3] = v3; o[4] = v4; o[5] = v5;
        o[6] = v6; o[7] = v7; o[8] = v8; o[9] = v9; o[10] = v10;
    }
}

// fixed-order sum over the rows of one instance: thread t takes rows
// t, t + RT, ... in order, then the LDS tree combines the threads.
__device__ double rows_sum(const double *part, int row0, int nrow, int q, double *s)
{
    double a = 0;
    for (int r = threadIdx.x; r < nrow; r += RT) a += part[(int64_t)(row0 + r) * NQR + q];
    return tree_sum(a, s);
}

__device__ double rows_max(const double *part, int row0, int nrow, int q, double *s)
{
    double a = -INFINITY;
    for (int r = threadIdx.x; r < nrow; r += RT) a = fmax(a, part[(int64_t)(row0 + r) * NQR + q]);
    return tree_max(a, s);
}

__device__ double rows_min(const double *part, int row0, int nrow, int q, double *s)
{
    double a = INFINITY;
    for (int r = threadIdx.x; r < nrow; r += RT) a = fmin(a, part[(int64_t)(row0 + r) * NQR + q]);
    return tree_min(a, s);
}

// final pass 1: one block per instance
__global__ __launch_bounds__(RT) void k_red_final1(const KInst *__restrict__ insts,
                                                    const int *__restrict__ row0s,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ res)
{
    __shared__ double s[RT];
    const int inst = blockIdx.x;
    const KInst &P = insts[inst];
    const int row0 = row0s[inst], nrow = P.ny;
    const double N = (double)P.nx * (double)P.ny;
    double *R = res + (int64_t)inst * NRES;
    const double mA = rows_sum(part, row0, nrow, 0, s), mB = rows_sum(part, row0, nrow, 1, s);
    const double px = rows_sum(part, row0, nrow, 2, s), py = rows_sum(part, row0, nrow, 3, s);
    const double jx = rows_sum(part, row0, nrow, 4, s), jy = rows_sum(part, row0, nrow, 5, s);
    const double su = rows_sum(part, row0, nrow, 6, s);
    const double um = rows_max(part, row0, nrow, 7, s);
    const double am = rows_max(part, row0, nrow, 8, s), an = rows_min(part, row0, nrow, 9, s);
    const double bad = rows_sum(part, row0, nrow, 10, s);
    if (threadIdx.x == 0) {
        R[RES_MASSA] = N * (double)P.rho_ref[0] + mA;
        R[RES_MASSB] = N * (double)P.rho_ref[1] + mB;
        R[RES_PX] = px;
        R[RES_PY] = py;
        R[RES_JX] = jx;
        R[RES_JY] = jy;
        R[RES_Q] = su / (double)P.nx;
        R[RES_UMAX] = um;
        R[RES_AMAX] = am;
        R[RES_AMIN] = an;
        R[RES_BAD] = bad;
    }
}

// pass 2 per row: weights w = rho_A - rho_A,min for the droplet area and the
// periodic circular mean of its position.
__global__ __launch_bounds__(RT) void k_red_rows2(const KInst *__restrict__ insts,
                                                   const int2 *__restrict__ rows,
                                                   const double *__restrict__ res,
                                                   double *__restrict__ part)
{
    __shared__ double s[RT];
    const int2 r = rows[blockIdx.x];
    const KInst &P = insts[r.x];
    const double rmin = res[(int64_t)r.x * NRES + RES_AMIN];
    const int y = r.y;
    double w = 0, wc = 0, ws = 0;
    const double k = 2.0 * M_PI / (double)P.nx;
    for (int x = threadIdx.x; x < P.nx; x += RT) {
        const double v = (double)P.fld[FLD_RHOA * P.plane + (int64_t)y * P.pitch + x] - rmin;
        double sn, cs;
        sincos(k * x, &sn, &cs);
        w += v;
        wc += v * cs;
        ws += v * sn;
    }
    double *o = part + (int64_t)blockIdx.x * NQR;
    const double a = tree_sum(w, s), b = tree_sum(wc, s), c = tree_sum(ws, s);
    if (threadIdx.x == 0) {
        o[0] = a;
        o[1] = b;
        o[2] = c;
    }
}

__global__ __launch_bounds__(RT) void k_red_final2(const KInst *__restrict__ insts,
                                                    const int *__restrict__ row0s,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ res)
{
    __shared__ double s[RT];
    const int inst = blockIdx.x;
    const KInst &P = insts[inst];
    const int row0 = row0s[inst], nrow = P.ny;
    double *R = res + (int64_t)inst * NRES;
    const double W = rows_sum(part, row0, nrow, 0, s);
    const double Wc = rows_sum(part, row0, nrow, 1, s);
    const double Ws = rows_sum(part, row0, nrow, 2, s);
    // y moments: row weights times cos/sin of the row angle
    double yc = 0, ys = 0;
    const double k = 2.0 * M_PI / (double)P.ny;
    for (int rr = threadIdx.x; rr < nrow; rr += RT) {
        double sn, cs;
        sincos(k * rr, &sn, &cs);
        const double v = part[(int64_t)(row0 + rr) * NQR + 0];
        yc += v * cs;
        ys += v * sn;
    }
    const double Yc = tree_sum(yc, s), Ys = tree_sum(ys, s);
    if (threadIdx.x == 0) {
        const double span = R[RES_AMAX] - R[RES_AMIN];
        const double area = span > 0 ? W / span : 0.0;
        double cx = atan2(Ws, Wc) * (double)P.nx / (2.0 * M_PI);
        double cy = atan2(Ys, Yc) * (double)P.ny / (2.0 * M_PI);
        cx = fmod(cx, (double)P.nx);
        if (cx < 0) cx += P.nx;
        cy = fmod(cy, (double)P.ny);
        if (cy < 0) cy += P.ny;
        R[RES_AREA] = area;
        R[RES_R] = sqrt(area / M_PI);
        R[RES_CX] = cx;
        R[RES_CY] = cy;
    }
}

// pass 3 per row: bulk pressure sums inside r <= R/2 and outside r >= R + margin
__global__ __launch_bounds__(RT) void k_red_rows3(const KInst *__restrict__ insts,
                                                   const int2 *__restrict__ rows,
                                                   const double *__restrict__ res,
                                                   double margin, double *__restrict__ part)
{
    __shared__ double s[RT];
    const int2 r = rows[blockIdx.x];
    const KInst &P = insts[r.x];
    const double *R = res + (int64_t)r.x * NRES;
    const double cx = R[RES_CX], cy = R[RES_CY], Rd = R[RES_R];
    const int y = r.y;
    double dy = fabs((double)y - cy);
    dy = fmin(dy, (double)P.ny - dy);
    double pin = 0, nin = 0, pout = 0, nout = 0;
    for (int x = threadIdx.x; x < P.nx; x += RT) {
        double dx = fabs((double)x - cx);
        dx = fmin(dx, (double)P.nx - dx);
        const double rr = sqrt(dx * dx + dy * dy);
        const double pb = (double)P.fld[FLD_PB * P.plane + (int64_t)y * P.pitch + x];
        if (rr <= 0.5 * Rd) {
            pin += pb;
            nin += 1;
        }
        if (rr >= Rd + margin) {
            pout += pb;
            nout += 1;
        }
    }
    double *o = part + (int64_t)blockIdx.x * NQR;
    const double a = tree_sum(pin, s), b = tree_sum(nin, s), c = tree_sum(pout, s),
                 d = tree_sum(nout, s);
    if (threadIdx.x == 0) {
        o[0] = a;
        o[1] = b;
        o[2] = c;
        o[3] = d;
    }
}

__global__ __launch_bounds__(RT) void k_red_final3(const KInst *__restrict__ insts,
                                                    const int *__restrict__ row0s,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ res)
{
    __shared__ double s[RT];
    const int inst = blockIdx.x;
    const KInst &P = insts[inst];
    const int row0 = row0s[inst], nrow = P.ny;
    double *R = res + (int64_t)inst * NRES;
    const double pin = rows_sum(part, row0, nrow, 0, s), nin = rows_sum(part, row0, nrow, 1, s);
    const double pout = rows_sum(part, row0, nrow, 2, s), nout = rows_sum(part, row0, nrow, 3, s);
    if (threadIdx.x == 0) {
        const double a = nin > 0 ? pin / nin : NAN;
        const double b = nout > 0 ? pout / nout : NAN;
        R[RES_PIN] = a;
        R[RES_POUT] = b;
        R[RES_NIN] = nin;
        R[RES_NOUT] = nout;
        R[RES_DP] = a - b;
        R[RES_GAMMA] = (a - b) * R[RES_R];
        // interface width along the row through the centre, walking +x from it
        const int yr = wrapi((int)floor(R[RES_CY] + 0.5), P.ny);
        const int xs = wrapi((int)floor(R[RES_CX] + 0.5), P.nx);
        const float *row = P.fld + FLD_RHOA * P.plane + (int64_t)yr * P.pitch;
        double mx = -INFINITY, mn = INFINITY;
        for (int x = 0; x < P.nx; ++x) {
            mx = fmax(mx, (double)row[x]);
            mn = fmin(mn, (double)row[x]);
        }
        const double bar = 0.5 * (mx + mn);
        double Wd = NAN;
        int x = xs;
        for (int n = 0; n < P.nx; ++n) {
            const int xn = (x + 1 == P.nx) ? 0 : x + 1;
            const double a0 = row[x], a1 = row[xn];
            if (a0 >= bar && bar > a1) {
                Wd = (mx - mn) / (a0 - a1);
                break;
            }
            x = xn;
        }
        R[RES_W] = Wd;
    }
}

// ------------------------------------------------------------------ copy probe
__global__ void k_copy(float4 *__restrict__ dst, const float4 *__restrict__ src, int64_t n4)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_copy_tail(char *__restrict__ dst, const char *__restrict__ src, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------------ launchers
#define LAUNCH_CHECK()                                            \
    do {                                                          \
        hipError_t e_ = hipGetLastError();                        \
        if (e_ != hipSuccess) return e_;                          \
    } while (0)

hipError_t launch_init(const Dev &d, const double *const *rho0s, hipStream_t st)
{
    k_init<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, rho0s, 0);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_step(const Dev &d, int par, hipStream_t st)
{
    k_density<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, par);
    LAUNCH_CHECK();
    k_step<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, par);
    LAUNCH_CHECK();
    return hipSuccess;
}

const char *step_kernel_name(int j)
{
    static const char *names[N_STEP_KERNELS] = {"k_density", "k_step"};
    return (j >= 0 && j < N_STEP_KERNELS) ? names[j] : "";
}

// kernel j of the step alone; neither changes the state of buffer par
hipError_t launch_step_kernel(const Dev &d, int j, int par, hipStream_t st)
{
    if (j == 0)
        k_density<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, par);
    else
        k_step<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, par);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fields(const Dev &d, int par, hipStream_t st)
{
    k_density<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, par);
    LAUNCH_CHECK();
    k_fields<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, par);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fields_out(const Dev &d, int inst, float *rho, float *u, hipStream_t st)
{
    k_fields_out<<<1024, 256, 0, st>>>(d.insts, inst, rho, u);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_export(const Dev &d, int inst, int par, float *f, hipStream_t st)
{
    k_export<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, inst, par, f);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_import(const Dev &d, int inst, int par, const float *f, hipStream_t st)
{
    k_import<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, inst, par, f);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_forces(const Dev &d, int inst, const float *rho, float *F, hipStream_t st)
{
    k_rho_in<<<1024, 256, 0, st>>>(d.insts, inst, rho);
    LAUNCH_CHECK();
    k_forces<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, inst, F);
    LAUNCH_CHECK();
    return hipSuccess;
}

// fields, then three row passes with their per-instance final passes; the
// per-row u_x sums (slot 6 of pass 1) stay untouched by passes 2 and 3.
hipError_t launch_observables(const Dev &d, int par, double margin, hipStream_t st)
{
    hipError_t e = launch_fields(d, par, st);
    if (e != hipSuccess) return e;
    k_red_rows1<<<d.nrows, RT, 0, st>>>(d.insts, d.rows, par, d.part);
    LAUNCH_CHECK();
    k_red_final1<<<d.ninst, RT, 0, st>>>(d.insts, d.row0s, d.part, d.res);
    LAUNCH_CHECK();
    k_red_rows2<<<d.nrows, RT, 0, st>>>(d.insts, d.rows, d.res, d.part);
    LAUNCH_CHECK();
    k_red_final2<<<d.ninst, RT, 0, st>>>(d.insts, d.row0s, d.part, d.res);
    LAUNCH_CHECK();
    k_red_rows3<<<d.nrows, RT, 0, st>>>(d.insts, d.rows, d.res, margin, d.part);
    LAUNCH_CHECK();
    k_red_final3<<<d.ninst, RT, 0, st>>>(d.insts, d.row0s, d.part, d.res);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_copy(void *dst, const void *src, uint64_t nbytes, hipStream_t st)
{
    const int64_t n4 = (int64_t)(nbytes / 16);
    if (n4 > 0) {
        k_copy<<<4096, 256, 0, st>>>((float4 *)dst, (const float4 *)src, n4);
        LAUNCH_CHECK();
    }
    const int64_t tail = (int64_t)(nbytes - (uint64_t)n4 * 16);
    if (tail > 0) {
        k_copy_tail<<<1, 64, 0, st>>>((char *)dst + n4 * 16, (const char *)src + n4 * 16, tail);
        LAUNCH_CHECK();
    }
    return hipSuccess;
}

}  // namespace lbm
