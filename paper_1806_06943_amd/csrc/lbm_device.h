// Device-side pieces of the two-range pseudopotential LBM step for gfx950
// (arXiv:1806.06943, Sec. II): per-instance launch parameters, the D2Q9 pull
// gather, the two-belt force from an LDS density tile and the FP32 collision.
//
// Storage: the state at time t is the post-streaming, pre-collision
// populations f(t) as FP32 deviations f - w_i rho_ref.  Their density
// deviations sum_i (f_i - w_i rho_ref), correctly rounded, are formed by the
// step from the populations it loads (the collision needs exactly that
// rounded sum); density buffers (double-buffered with those of t+1) are
// written only for the kernels and calls that read densities.
//
// Layout: row-major rows; within a row the 18 populations q = 9 k + i of a
// node are packed into vector planes of `pitch` nodes: four float4 planes
// (q = 0-3, 4-7, 8-11, 12-15, i.e. f_A0..3, f_A4..7, f_A8 f_B0..2, f_B3..6)
// and one float2 plane (q = 16, 17: f_B7, f_B8), 18 pitch floats per row.
// The two density deviations of a node are one float2, rho[y][x][k].  A
// wavefront working on one lattice row then moves each plane of 64
// consecutive nodes with one 16-byte (8-byte) access per lane, 1 KiB per
// instruction; single-float accesses per lane would reach only about two
// thirds of the bandwidth of wide ones on this GPU.
//
// Numerical formulation (FP32 throughout the step):
//   * the density deviation sum is accumulated in FP64 and rounded once, so
//     the rest-state part of the collision sees the stored mass exactly;
//   * weights are w_i = c_i / 36 with integer c_i = 16, 4, 1; quantities per
//     unit weight are formed by a correctly rounded division by 36, so the
//     rounding of the weights cannot create or destroy mass systematically;
//   * the collision relaxes only the small part f_i - c_i a (a = drho / 36)
//     and adds the rest part back once;
//   * the force stencils of Eqs. 8 and 9 are evaluated as antisymmetric
//     differences psi(x+e) - psi(x-e) with the two couplings of Eq. 8 merged
//     per |e|^2 class, which keeps the exact pairwise momentum balance.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int TX = 64;   // auxiliary 2-D tiles: width (one wavefront of 64 lanes per row)
constexpr int TY = 4;    // auxiliary 2-D tiles: height (4 wavefronts per block)
constexpr int NTHREADS = TX * TY;
constexpr int HALO = 2;  // radius of the D2Q25 stencil

// fused step: the lanes of a strip load its output columns, one collided
// halo column and HALO stencil columns on each side
constexpr int SW = 64;                  // lanes of a one-wavefront strip
constexpr int SWO = SW - 2 - 2 * HALO;  // output columns of a full one-wavefront strip
constexpr int RR = 2 * HALO + 1;        // density-ring rows

// number of FP32 planes in the per-instance field scratch (the observables
// use the first nine, the adjoint passes all)
constexpr int NFLD = 13;
enum FieldPlane { FLD_RHOA = 0, FLD_RHOB, FLD_UX, FLD_UY, FLD_PB, FLD_MX, FLD_MY, FLD_JX, FLD_JY };

// Launch parameters of one instance (device copy lives in the workspace).
struct KInst {
    float *f[2];           // population buffers (packed rows, see fidx), paired with rho[]
    float *rho[2];         // density-deviation buffers rho[y][x][k]
    float *fld;            // field scratch planes [NFLD][ny][pitch]
    int64_t plane;         // floats between consecutive field planes
    int32_t nx, ny, pitch, walls;
    float cw[2][5];        // merged Eq. 8 weights G1 w + G2 p per |e|^2 in {1, 2, 4, 5, 8}
    float gr1, gr2;        // Eq. 9 weights G_AB w(1), G_AB w(2)
    float g[2][2];         // body acceleration per component
    float it[2];           // 1 / tau_k
    float cf[2];           // (1 - 1/(2 tau_k)) / 36
    float rho_ref[2];
    float rho_wall[2], psi_wall[2];
    float rho0, inv_rho0;  // pseudopotential scale
    float gpb[2];          // (G1 + G2) / 2 per component, for the bulk pressure of Eq. 11
    float gab;             // G_AB
    int32_t pad_;
};

// The arithmetic parameters of an instance, as plain values: kernels that
// loop over rows copy them once (a reference into global memory would be
// reloaded after every store).
struct KPar {
    float cw[2][5], gr1, gr2, g[2][2], it[2], cf[2], rho_ref[2], rho_wall[2], psi_wall[2];
    float rho0, inv_rho0;
};

__device__ __forceinline__ KPar kpar(const KInst &P)
{
    KPar q;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
#pragma unroll
        for (int c = 0; c < 5; ++c) q.cw[k][c] = P.cw[k][c];
        q.g[k][0] = P.g[k][0];
        q.g[k][1] = P.g[k][1];
        q.it[k] = P.it[k];
        q.cf[k] = P.cf[k];
        q.rho_ref[k] = P.rho_ref[k];
        q.rho_wall[k] = P.rho_wall[k];
        q.psi_wall[k] = P.psi_wall[k];
    }
    q.gr1 = P.gr1;
    q.gr2 = P.gr2;
    q.rho0 = P.rho0;
    q.inv_rho0 = P.inv_rho0;
    return q;
}

__device__ __forceinline__ int wrapi(int a, int n)
{
    if (a >= 0 && a < n) return a;
    int r = a % n;
    return r < 0 ? r + n : r;
}

// psi = rho0 (1 - exp(-rho/rho0)), through expm1f for accuracy at small rho
template <class Par>
__device__ __forceinline__ float psi_of(const Par &P, float r)
{
    return -P.rho0 * expm1f(-r * P.inv_rho0);
}

// index of population q = 9 k + i of node (x, y) in a population buffer
__device__ __forceinline__ int64_t fidx(const KInst &P, int q, int x, int y)
{
    return ((int64_t)y * 18 + (q & ~3)) * P.pitch + (int64_t)x * (q < 16 ? 4 : 2) + (q & 3);
}

// index of the density deviation of component k of node (x, y)
__device__ __forceinline__ int64_t ridx(const KInst &P, int k, int x, int y)
{
    return ((int64_t)y * P.pitch + x) * 2 + k;
}

// Populations of node (x, y) from buffer fb (D2Q9 order 0:(0,0) 1:(1,0)
// 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)).
__device__ __forceinline__ void load_node(const KInst &P, const float *__restrict__ fb, int x,
                                          int y, float f[2][9])
{
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int i = 0; i < 9; ++i) f[k][i] = fb[fidx(P, k * 9 + i, x, y)];
}

// Sum of the nine deviations, correctly rounded to FP32: the FP32 terms are
// added in FP64 (exactly, unless their exponents span more than 29 bits)
// and the total is rounded once.
__device__ __forceinline__ float sum9(const float f[9])
{
    double s = (double)f[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) s += (double)f[i];
    return (float)s;
}

// FP64 block reductions in a fixed order.  Each wavefront combines its 64
// values by an xor butterfly: every step combines the same two operands on
// both lanes of a pair, so all lanes end with the same bits and no barrier
// is needed.  Lane 0 of each wavefront parks its result in LDS; after one
// barrier thread 0 combines the wavefronts' results in wavefront order.  The
// result is valid in thread 0.  Bitwise reproducible for a given block size.
enum RedOp { RED_SUM = 0, RED_MAX = 1, RED_MIN = 2 };

__device__ __forceinline__ double red_op(int op, double a, double b)
{
    return op == RED_SUM ? a + b : op == RED_MAX ? fmax(a, b) : fmin(a, b);
}

// v[q] (per thread) -> v[q] (thread 0) reduced with op[q]; lds holds
// N * NT / 64 doubles
template <int NT, int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], const int (&op)[N], double *lds)
{
    constexpr int NWV = NT / 64;
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
#pragma unroll
    for (int q = 0; q < N; ++q)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v[q] = red_op(op[q], v[q], __shfl_xor(v[q], o, 64));
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) lds[q * NWV + wv] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double a = lds[q * NWV];
            for (int w = 1; w < NWV; ++w) a = red_op(op[q], a, lds[q * NWV + w]);
            v[q] = a;
        }
    __syncthreads();  // the LDS may be reused after the call
}

// LDS density tile: rho and psi of both components on the tile plus a halo
// of 2, laid out [k][row][col] with (TX + 4) columns.
struct Tile {
    float rho[2][TY + 2 * HALO][TX + 2 * HALO];
    float psi[2][TY + 2 * HALO][TX + 2 * HALO];
};

// Fill the LDS tile for the tile whose first node is (x0, y0).  Periodic wrap
// in x (and in y without walls); rows beyond a wall hold the wall densities.
// rb holds density deviations (absolute = false) or densities.
__device__ __forceinline__ void stage_tile(const KInst &P, const float *__restrict__ rb, int x0,
                                           int y0, Tile &T, bool absolute = false)
{
    constexpr int W = TX + 2 * HALO, H = TY + 2 * HALO;
    for (int t = threadIdx.x; t < W * H; t += NTHREADS) {
        const int lx = t % W, ly = t / W;
        const int gx = wrapi(x0 + lx - HALO, P.nx);
        int gy = y0 + ly - HALO;
        float rA, rB, pA, pB;
        if (P.walls && (gy < 0 || gy >= P.ny)) {
            rA = P.rho_wall[0];
            rB = P.rho_wall[1];
            pA = P.psi_wall[0];
            pB = P.psi_wall[1];
        } else {
            gy = wrapi(gy, P.ny);
            const float dA = rb[ridx(P, 0, gx, gy)], dB = rb[ridx(P, 1, gx, gy)];
            rA = absolute ? dA : P.rho_ref[0] + dA;
            rB = absolute ? dB : P.rho_ref[1] + dB;
            pA = psi_of(P, rA);
            pB = psi_of(P, rB);
        }
        T.rho[0][ly][lx] = rA;
        T.rho[1][ly][lx] = rB;
        T.psi[0][ly][lx] = pA;
        T.psi[1][ly][lx] = pB;
    }
}

// Total force on both components from a density/pseudopotential accessor:
// acc.psi(k, dx, dy) and acc.rho(k, dx, dy) give the values at the node
// displaced by (dx, dy).  F^c (Eq. 8) with merged weights, F^r (Eq. 9),
// F^b = rho g.
template <class Par, class Acc>
__device__ __forceinline__ void stencil_force(const Par &P, const Acc &acc, float F[2][2])
{
#pragma unroll
    for (int k = 0; k < 2; ++k) {
#define PSI(dx, dy) acc.psi(k, dx, dy)
#define RHB(dx, dy) acc.rho(1 - k, dx, dy)
        // antisymmetric pair differences d(e) = psi(x+e) - psi(x-e)
        const float d10 = PSI(1, 0) - PSI(-1, 0);
        const float d20 = PSI(2, 0) - PSI(-2, 0);
        const float d01 = PSI(0, 1) - PSI(0, -1);
        const float d02 = PSI(0, 2) - PSI(0, -2);
        const float d11 = PSI(1, 1) - PSI(-1, -1);
        const float dm11 = PSI(-1, 1) - PSI(1, -1);
        const float d21 = PSI(2, 1) - PSI(-2, -1);
        const float dm21 = PSI(-2, 1) - PSI(2, -1);
        const float d12 = PSI(1, 2) - PSI(-1, -2);
        const float dm12 = PSI(-1, 2) - PSI(1, -2);
        const float d22 = PSI(2, 2) - PSI(-2, -2);
        const float dm22 = PSI(-2, 2) - PSI(2, -2);
        const float c1 = P.cw[k][0], c2 = P.cw[k][1], c4 = P.cw[k][2], c5 = P.cw[k][3],
                    c8 = P.cw[k][4];
        const float sx = c1 * d10 + 2.0f * c4 * d20 + c2 * (d11 - dm11) +
                         c5 * (2.0f * (d21 - dm21) + (d12 - dm12)) + 2.0f * c8 * (d22 - dm22);
        const float sy = c1 * d01 + 2.0f * c4 * d02 + c2 * (d11 + dm11) +
                         c5 * ((d21 + dm21) + 2.0f * (d12 + dm12)) + 2.0f * c8 * (d22 + dm22);
        // inter-species repulsion acts through the other component's density
        const float r10 = RHB(1, 0) - RHB(-1, 0);
        const float r01 = RHB(0, 1) - RHB(0, -1);
        const float r11 = RHB(1, 1) - RHB(-1, -1);
        const float rm11 = RHB(-1, 1) - RHB(1, -1);
        const float rx = P.gr1 * r10 + P.gr2 * (r11 - rm11);
        const float ry = P.gr1 * r01 + P.gr2 * (r11 + rm11);
#undef PSI
#undef RHB
        const float psi0 = acc.psi(k, 0, 0);
        const float rho0 = acc.rho(k, 0, 0);
        F[k][0] = -psi0 * sx - rho0 * rx + rho0 * P.g[k][0];
        F[k][1] = -psi0 * sy - rho0 * ry + rho0 * P.g[k][1];
    }
}

// accessor into a 2-D LDS tile centred at (cx, cy)
struct TileAcc {
    const Tile &T;
    int cx, cy;
    __device__ float psi(int k, int dx, int dy) const { return T.psi[k][cy + dy][cx + dx]; }
    __device__ float rho(int k, int dx, int dy) const { return T.rho[k][cy + dy][cx + dx]; }
};

__device__ __forceinline__ void tile_force(const KInst &P, const Tile &T, int cx, int cy,
                                           float F[2][2])
{
    stencil_force(P, TileAcc{T, cx, cy}, F);
}

// Momentum sum_i f_i e_i of one component as antisymmetric differences.
__device__ __forceinline__ void mom9(const float f[9], float &mx, float &my)
{
    mx = (f[1] - f[3]) + (f[5] - f[7]) + (f[8] - f[6]);
    my = (f[2] - f[4]) + (f[5] - f[7]) + (f[6] - f[8]);
}

// x / 36 correctly rounded in the usual case, from a product and one FMA
// correction (the residual x - 36 q is exact): an unbiased scaling, unlike a
// product with the rounded constant 1/36, whose error has a fixed sign.
__device__ __forceinline__ float div36(float x)
{
    const float q = x * (1.0f / 36.0f);
    const float r = fmaf(-36.0f, q, x);
    return fmaf(r, 1.0f / 36.0f, q);
}

// 1 / d from the hardware reciprocal refined by one Newton step
__device__ __forceinline__ float recip(float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    const float e = fmaf(-d, r, 1.0f);
    return fmaf(e, r, r);
}

// Common velocity u^eq of Eq. 3 from the component momenta j_k (with F/2).
template <class Par>
__device__ __forceinline__ void common_velocity(const Par &P, const float rho[2],
                                                const float jx[2], const float jy[2], float &ux,
                                                float &uy)
{
    const float inv = recip(fmaf(rho[0], P.it[0], rho[1] * P.it[1]));
    ux = fmaf(jx[0], P.it[0], jx[1] * P.it[1]) * inv;
    uy = fmaf(jy[0], P.it[0], jy[1] * P.it[1]) * inv;
}

// BGK + Guo collision of one component (Eqs. 1, 2 with the 1/2 on the
// quadratic term, 5), in deviation form.  f: pre-collision deviations,
// drho: their correctly rounded sum, rho: density, F: force, (ux, uy): u^eq.
// Opposite directions share e.u and e.F: the equilibrium splits into the
// even part 4.5 (e.u)^2 - 1.5 u.u and the odd part 3 e.u, the Guo bracket
// into 9 (e.u)(e.F) - 3 u.F and 3 e.F.  GUO = false drops the Guo term (the
// velocity shift, whose force enters through u^eq; F is then ignored).
// e.u and e.F are formed from the lattice vectors' components directly
// (u_x, u_y, u_x + u_y, u_y - u_x): a product with a zero component would
// still be evaluated (it is not an exact zero for every input).
template <bool GUO = true, class Par>
__device__ __forceinline__ void collide(const Par &P, int k, const float f[9], float drho,
                                        float rho, float Fx, float Fy, float ux, float uy,
                                        float out[9])
{
    const float a = div36(drho);   // rest-state deviation per unit weight
    const float r36 = div36(rho);
    const float it = P.it[k];
    const float omit = 1.0f - it;
    const float cf = P.cf[k];
    const float uu = fmaf(ux, ux, uy * uy);
    const float uF = GUO ? fmaf(ux, Fx, uy * Fy) : 0.0f;
    // relaxation of the small part g = f - c a towards f^eq - c a, plus C
    auto relax = [&](float fi, float c, float feq_small, float C) {
        const float rest = c * a;
        const float g = fi - rest;
        return rest + fmaf(g, omit, GUO ? fmaf(feq_small, it, C) : feq_small * it);
    };
    // rest direction: e = 0
    out[0] = relax(f[0], 16.0f, 16.0f * (r36 * (-1.5f * uu)), 16.0f * (cf * (-3.0f * uF)));
    // pairs (i, opp(i)) with weight c, e_i . u = eu and e_i . F = eF
    auto pair = [&](int i, int j, float eu, float eF, float c) {
        const float qe = fmaf(4.5f * eu, eu, -1.5f * uu);
        const float qo = 3.0f * eu;
        const float rc = c * r36;
        if constexpr (GUO) {
            const float ce = fmaf(9.0f * eu, eF, -3.0f * uF);
            const float co = 3.0f * eF;
            const float fc = c * cf;
            out[i] = relax(f[i], c, rc * (qe + qo), fc * (ce + co));
            out[j] = relax(f[j], c, rc * (qe - qo), fc * (ce - co));
        } else {
            out[i] = relax(f[i], c, rc * (qe + qo), 0.0f);
            out[j] = relax(f[j], c, rc * (qe - qo), 0.0f);
        }
    };
    pair(1, 3, ux, Fx, 4.0f);                 // e = (1, 0)
    pair(2, 4, uy, Fy, 4.0f);                 // e = (0, 1)
    pair(5, 7, ux + uy, Fx + Fy, 1.0f);       // e = (1, 1)
    pair(6, 8, uy - ux, Fy - Fx, 1.0f);       // e = (-1, 1)
}

}  // namespace lbm
