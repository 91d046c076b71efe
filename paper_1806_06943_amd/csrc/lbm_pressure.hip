// Pressure tensor of the two-range model (Sec. II B) and the line-tension
// integral of a flat interface (Eqs. 15, 16), for gfx950.
//
// P = P^int + P^kin per node.  P^int is the pair-sum (virial) form of the
// pairwise lattice forces of Eqs. 8 and 9,
//   P^int_k = 1/2 sum_e c_k(e) psi_k(x) psi_k(x+e) e e
//           + 1/2 G_AB sum_i w_i rho_k(x) rho_kbar(x+e_i) e_i e_i,
// which equals the interaction part of the bulk equation of state (Eq. 11)
// in a uniform state and whose sum across a flat interface is the virial of
// the pairs crossing it.  P^kin is sum_{k,i} f e e for the Guo forcing (the
// static problem of Sec. II B), and sum_k rho_k cs^2 delta + K^tau (the
// tau-dependent terms the paper gives for the original model) for the
// velocity shift, density gradients by central differences.
#include <stdint.h>

#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int PW = TX + 2 * HALO, PH = TY + 2 * HALO;

__device__ __forceinline__ float ppsi(const KInst &P, float r) { return -P.rho0 * expm1f(-r * P.inv_rho0); }

// Per-node P_xx, P_yy, P_xy into out[3][ny][nx] (FP32), and FP64 partial
// sums of P_xx - P_yy per block into part[block].
__global__ __launch_bounds__(NTHREADS) void k_pressure(const KInst *__restrict__ insts, int inst,
                                                       int par, float G1a, float G1b, float G2a,
                                                       float G2b, float tauA, float tauB,
                                                       int forcing, float *__restrict__ out,
                                                       double *__restrict__ part)
{
    __shared__ float rho[2][PH][PW];
    __shared__ float psi[2][PH][PW];
    __shared__ double red[NTHREADS / 64];
    const KInst &P = insts[inst];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    for (int t = threadIdx.x; t < PW * PH; t += NTHREADS) {
        const int lx = t % PW, ly = t / PW;
        const int gx = wrapi(x0 + lx - HALO, P.nx);
        const int gy = y0 + ly - HALO;
        const bool wall = P.walls && (gy < 0 || gy >= P.ny);
        const int yy = wall ? 0 : wrapi(gy, P.ny);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float r = wall ? P.rho_wall[k] : P.rho_ref[k] + P.rho[par][ridx(P, k, gx, yy)];
            rho[k][ly][lx] = r;
            psi[k][ly][lx] = wall ? P.psi_wall[k] : ppsi(P, r);
        }
    }
    __syncthreads();
    const int lx = (int)(threadIdx.x % TX), ly = (int)(threadIdx.x / TX);
    const int x = x0 + lx, y = y0 + ly;
    double mis = 0.0;
    if (x < P.nx && y < P.ny) {
        const int cx = lx + HALO, cy = ly + HALO;
        const float G1[2] = {G1a, G1b}, G2[2] = {G2a, G2b};
        const float gab = P.gab;
        // weights w(|e|^2) for |e|^2 = 1, 2 and p(|e|^2) for 1, 2, 4, 5, 8
        const float w1 = 1.0f / 9.0f, w2 = 1.0f / 36.0f;
        const float p1 = 4.0f / 63.0f, p2 = 4.0f / 135.0f, p4 = 1.0f / 180.0f, p5 = 2.0f / 945.0f,
                    p8 = 1.0f / 15120.0f;
        double pxx = 0.0, pyy = 0.0, pxy = 0.0;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float ps = psi[k][cy][cx], rk = rho[k][cy][cx];
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx) {
                    const int e2 = dx * dx + dy * dy;
                    if (e2 == 0) continue;
                    const float pw = e2 == 1 ? p1 : e2 == 2 ? p2 : e2 == 4 ? p4 : e2 == 5 ? p5 : p8;
                    const float ww = e2 == 1 ? w1 : e2 == 2 ? w2 : 0.0f;
                    double v = 0.5 * (double)(G1[k] * ww + G2[k] * pw) * ps * psi[k][cy + dy][cx + dx];
                    if (e2 <= 2) v += 0.5 * (double)(gab * ww) * rk * rho[1 - k][cy + dy][cx + dx];
                    pxx += v * (dx * dx);
                    pyy += v * (dy * dy);
                    pxy += v * (dx * dy);
                }
        }
        if (!forcing) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                float f[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = P.f[par][fidx(P, k * 9 + i, x, y)];
                const double wr = (double)(k ? P.rho_ref[1] : P.rho_ref[0]);
                // second moment of the deviations plus that of w_i rho_ref (cs^2 rho_ref)
                pxx += (double)f[1] + f[3] + f[5] + f[6] + f[7] + f[8] + wr / 3.0;
                pyy += (double)f[2] + f[4] + f[5] + f[6] + f[7] + f[8] + wr / 3.0;
                pxy += (double)f[5] - f[6] + f[7] - f[8];
            }
        } else {
            const double ra = rho[0][cy][cx], rb = rho[1][cy][cx], rt = ra + rb;
            pxx += rt / 3.0;
            pyy += rt / 3.0;
            const double tm = (ra * tauA + rb * tauB) / rt, t2 = (tm - 0.5) * (tm - 0.5);
            // total force at the node (Eqs. 8, 9, body force)
            double Fx = 0.0, Fy = 0.0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const float ps = psi[k][cy][cx], rk = rho[k][cy][cx];
#pragma unroll
                for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
                    for (int dx = -2; dx <= 2; ++dx) {
                        const int e2 = dx * dx + dy * dy;
                        if (e2 == 0) continue;
                        const float pw = e2 == 1 ? p1 : e2 == 2 ? p2 : e2 == 4 ? p4 : e2 == 5 ? p5 : p8;
                        const float ww = e2 == 1 ? w1 : e2 == 2 ? w2 : 0.0f;
                        double c = -(double)(G1[k] * ww + G2[k] * pw) * ps * psi[k][cy + dy][cx + dx];
                        if (e2 <= 2) c -= (double)(gab * ww) * rk * rho[1 - k][cy + dy][cx + dx];
                        Fx += c * dx;
                        Fy += c * dy;
                    }
                Fx += (double)rk * P.g[k][0];
                Fy += (double)rk * P.g[k][1];
            }
            const double gx = 0.5 * (log((double)rho[0][cy][cx + 1]) - log((double)rho[0][cy][cx - 1]) -
                                     log((double)rho[1][cy][cx + 1]) + log((double)rho[1][cy][cx - 1]));
            const double gy = 0.5 * (log((double)rho[0][cy + 1][cx]) - log((double)rho[0][cy - 1][cx]) -
                                     log((double)rho[1][cy + 1][cx]) + log((double)rho[1][cy - 1][cx]));
            const double cc = ra * rb / rt * t2 / 9.0;
            pxx += t2 * Fx * Fx / rt + cc * gx * gx;
            pyy += t2 * Fy * Fy / rt + cc * gy * gy;
            pxy += t2 * Fx * Fy / rt + cc * gx * gy;
        }
        const int64_t N = (int64_t)P.nx * P.ny, n = (int64_t)y * P.nx + x;
        out[n] = (float)pxx;
        out[N + n] = (float)pyy;
        out[2 * N + n] = (float)pxy;
        mis = pxx - pyy;
    }
    // block sum in a fixed order
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mis += __shfl_xor(mis, o, 64);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = mis;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < NTHREADS / 64; ++w) s += red[w];
        part[blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void k_pressure_final(const double *__restrict__ part, int n,
                                                        double *__restrict__ res)
{
    __shared__ double red[256 / 64];
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < n; b += 256) v[0] += part[b];
    constexpr int op[1] = {RED_SUM};
    block_reduce<256>(v, op, red);
    if (threadIdx.x == 0) res[0] = v[0];
}

}  // namespace

hipError_t launch_pressure(const Dev &d, const lbm_params &p, int inst, int par, float *out,
                           double *part, double *res, hipStream_t st)
{
    const dim3 grid((p.nx + TX - 1) / TX, (p.ny + TY - 1) / TY);
    k_pressure<<<grid, NTHREADS, 0, st>>>(d.insts, inst, par, (float)p.G1[0], (float)p.G1[1],
                                          (float)p.G2[0], (float)p.G2[1], (float)p.tau[0],
                                          (float)p.tau[1], p.forcing, out, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pressure_final<<<1, 256, 0, st>>>(part, (int)(grid.x * grid.y), res);
    return hipGetLastError();
}

}  // namespace lbm
