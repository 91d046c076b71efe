// Reverse-mode adjoint of the two-range pseudopotential LBM step and the
// seeds of differentiable objectives, for gfx950.
//
// The step (arXiv:1806.06943, Eqs. 1, 2, 3, 5, 6, 8, 9; Sec. II B) maps the
// populations f(t) to f(t+1) = Phi(f(t); theta).  Given lam_next = dJ/df(t+1)
// the adjoint step returns lam = (dPhi/df)^T lam_next and adds
// (dPhi/dtheta)^T lam_next to a gradient, theta = (G1, G2, G_AB, tau_A,
// tau_B) with G1 and G2 moving both components together.
//
// The state (FP32 deviations f - w_i rho_ref, and its density deviations) is
// read in the library's packed layout: a recorded window's slots, or the
// instance's spare buffer into which the entry points import a caller's
// state.  lam is the caller's, in the export layout [2][9][ny][nx].  One
// adjoint step is up to three passes over 2-D tiles (64 x 4 nodes; 64 x 8,
// two nodes per thread, for the local transpose):
//   k_adj_density  density deviations of f (rounded as the forward step's)
//                  into scratch (a recorded state brings the densities the
//                  step wrote, bitwise the same);
//   k_adj_local    per node: recompute rho, psi, the stencil sums of Eqs. 8
//                  and 9 (LDS tile with a halo of 2), F, j, u^eq; gather
//                  lam*_{k,i}(x) = lam_next_{k,i}(x + e_i) (transpose of
//                  streaming, reversed across a wall); transpose the
//                  collision, Eq. 3 and Eq. 6; write the force adjoint Fbar
//                  and the partial lam (everything but the force stencil's
//                  neighbour terms); accumulate the theta terms in FP64;
//   k_adj_force    per node: gather the neighbour terms of the transposed
//                  force stencils from psi Fbar and rho Fbar of the 5 x 5
//                  neighbourhood (LDS tile); their sum adds the same density
//                  adjoint to all nine lam_{k,i} of a component, so it is
//                  kept as one pending value per node and component, which
//                  the next step's gather (or k_adj_combine) adds;
// followed by a fixed-order FP64 reduction of the per-block theta partials.
// Within a run of steps (swept from the last time step back) the force pass
// of step j + 1 is folded into the local pass of step j: that pass stages
// psi Fbar and rho Fbar of step j + 1 around its tile and forms the pending
// addition where its gather reads it (the same operations, so the same
// bits), one launch per step instead of two.  "The step before" below is
// the step the sweep processed before, j + 1.
// Scratch (densities, Fbar, block partials, the pending additions) lives in
// the instance's field planes of the workspace.
#include <stdint.h>

#include <type_traits>

#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int AW = TX + 2 * HALO;  // staged tile width
constexpr int AH = TY + 2 * HALO;  // staged tile height

// Element indices in 32-bit arithmetic: every instance buffer stays below
// 2 GiB (checked at init), so no index reaches 2^31.
__device__ __forceinline__ int64_t xidx(const AdjPar &A, int q, int x, int y)
{
    return (int64_t)(((uint32_t)q * (uint32_t)A.ny + (uint32_t)y) * (uint32_t)A.nx + (uint32_t)x);  // [q][y][x]
}

// the library's packed state layout (pitch A.pitch): population q = 9 k + i
// in four float4 planes and one float2 plane per row, densities rho[y][x][k]
__device__ __forceinline__ int64_t pidx(const AdjPar &A, int q, int x, int y)
{
    return (int64_t)(((uint32_t)y * 18u + (uint32_t)(q & ~3)) * (uint32_t)A.pitch +
                     (uint32_t)x * (q < 16 ? 4u : 2u) + (uint32_t)(q & 3));
}

__device__ __forceinline__ int64_t didx(const AdjPar &A, int k, int x, int y)
{
    return (int64_t)(((uint32_t)y * (uint32_t)A.pitch + (uint32_t)x) * 2u + (uint32_t)k);
}

// periodic wrap of an index at most one period outside [0, n)
__device__ __forceinline__ int wrap1(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ int64_t sidx(const AdjPar &A, int plane, int x, int y)
{
    return (int64_t)((uint32_t)plane * (uint32_t)A.plane + (uint32_t)y * (uint32_t)A.pitch +
                     (uint32_t)x);  // scratch planes
}

__device__ __forceinline__ float apsi(const AdjPar &A, float r)
{
    return -A.rho0 * expm1f(-r * A.inv_rho0);
}

// D2Q9 (order 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1)
// 7:(-1,-1) 8:(1,-1)) with weights c_i / 36
// compile-time tables: in the unrolled direction loops every component is a
// known 0 or +-1
constexpr int c_ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int c_ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int c_op[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// e v for a lattice component e in {-1, 0, 1}, without a multiply (exact)
template <class T>
__device__ __forceinline__ T emul(int e, T v)
{
    return e == 0 ? T(0) : (e > 0 ? v : -v);
}

constexpr float W0 = 4.0f / 9.0f, W1 = 1.0f / 9.0f, W2 = 1.0f / 36.0f;
__device__ __forceinline__ float wgt(int i) { return i == 0 ? W0 : (i < 5 ? W1 : W2); }
constexpr double wgt9[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// D2Q25 weights p(|e|^2) of Eq. 8 for |e|^2 = 1, 2, 4, 5, 8
constexpr float P1 = 4.0f / 63.0f, P2 = 4.0f / 135.0f, P4 = 1.0f / 180.0f, P5 = 2.0f / 945.0f,
                P8 = 1.0f / 15120.0f;
constexpr double DW1 = 1.0 / 9.0, DW2 = 1.0 / 36.0;
constexpr double DP1 = 4.0 / 63.0, DP2 = 4.0 / 135.0, DP4 = 1.0 / 180.0, DP5 = 2.0 / 945.0,
                 DP8 = 1.0 / 15120.0;

// Stencil sum sum_e c(|e|^2) v(x + e) e over the 24 non-zero D2Q25 vectors,
// as antisymmetric pairs v(x+e) - v(x-e); v(dx, dy) reads the staged tile.
// T is the accumulation type: FP64 sums of FP32 tile values are exact in
// the pair differences and keep the relative accuracy of a result much
// smaller than its terms (interfaces), which the parameter gradients need.
template <class T, class V>
__device__ __forceinline__ void sum25(const V &v, T c1, T c2, T c4, T c5, T c8, T &sx, T &sy)
{
    auto d = [&](int ax, int ay, int bx, int by) { return (T)v(ax, ay) - (T)v(bx, by); };
    const T d10 = d(1, 0, -1, 0), d01 = d(0, 1, 0, -1);
    const T d20 = d(2, 0, -2, 0), d02 = d(0, 2, 0, -2);
    const T d11 = d(1, 1, -1, -1), dm11 = d(-1, 1, 1, -1);
    const T d21 = d(2, 1, -2, -1), dm21 = d(-2, 1, 2, -1);
    const T d12 = d(1, 2, -1, -2), dm12 = d(-1, 2, 1, -2);
    const T d22 = d(2, 2, -2, -2), dm22 = d(-2, 2, 2, -2);
    sx = c1 * d10 + (T)2 * c4 * d20 + c2 * (d11 - dm11) + c5 * ((T)2 * (d21 - dm21) + (d12 - dm12)) +
         (T)2 * c8 * (d22 - dm22);
    sy = c1 * d01 + (T)2 * c4 * d02 + c2 * (d11 + dm11) + c5 * ((d21 + dm21) + (T)2 * (d12 + dm12)) +
         (T)2 * c8 * (d22 + dm22);
}

// the D2Q9 part only (|e|^2 = 1, 2)
template <class T, class V>
__device__ __forceinline__ void sum9s(const V &v, T c1, T c2, T &sx, T &sy)
{
    auto d = [&](int ax, int ay, int bx, int by) { return (T)v(ax, ay) - (T)v(bx, by); };
    const T d10 = d(1, 0, -1, 0), d01 = d(0, 1, 0, -1);
    const T d11 = d(1, 1, -1, -1), dm11 = d(-1, 1, 1, -1);
    sx = c1 * d10 + c2 * (d11 - dm11);
    sy = c1 * d01 + c2 * (d11 + dm11);
}

// The pending addition of component k at one node: the neighbour terms of
// the transposed force stencils, psibar_k exp(-rho_k / rho0) + rhobar_k, from
// q(kk, d, dx, dy) = psi_kk Fbar_kk,d and r(kk, d, dx, dy) = rho_kk Fbar_kk,d
// of the node displaced by (dx, dy); rk is the node's own density.  With
//   psibar_k(y) = sum_e c_k(e) e . (q_k(y + e) - q_k(y - e))   (e over half of D2Q25,
//                 c_k(e) = G1_k w(e) + G2_k p(e))
//   rhobar_k(y) = G_AB sum_e w(e) e . (r_kb(y + e) - r_kb(y - e))   (half of D2Q9)
template <class QA, class RA>
__device__ __forceinline__ float force_add(const AdjPar &A, int k, const QA &q, const RA &r,
                                           float rk)
{
    float ax, ay, bx, by, cx_, cy_, dx_, dy_;
    auto qx = [&](int dx, int dy) { return q(k, 0, dx, dy); };
    auto qy = [&](int dx, int dy) { return q(k, 1, dx, dy); };
    const float c1 = A.G1[k] * W1 + A.G2[k] * P1, c2 = A.G1[k] * W2 + A.G2[k] * P2;
    const float c4 = A.G2[k] * P4, c5 = A.G2[k] * P5, c8 = A.G2[k] * P8;
    sum25<float>(qx, c1, c2, c4, c5, c8, ax, ay);  // uses the x component along e_x, e_y
    sum25<float>(qy, c1, c2, c4, c5, c8, bx, by);
    const float psibar = ax + by;  // e . q summed: e_x q_x + e_y q_y
    // inter-species: r of the other component
    auto rx = [&](int dx, int dy) { return r(1 - k, 0, dx, dy); };
    auto ry = [&](int dx, int dy) { return r(1 - k, 1, dx, dy); };
    sum9s<float>(rx, W1, W2, cx_, cy_);
    sum9s<float>(ry, W1, W2, dx_, dy_);
    (void)ay;
    (void)bx;
    (void)cy_;
    (void)dx_;
    return psibar * expf(-rk * A.inv_rho0) + A.gab * (cx_ + dy_);
}

// The staging loops below issue every global load of a thread's share of
// the tile before the first use: loads under a per-element branch (the
// rows beyond a wall) would each wait for their data before the next is
// issued.  An element past the tile, or in a row beyond a wall, loads a
// valid node (row 0, the last element) whose value goes unused.
template <int N>
constexpr int stage_iters() { return (N + NTHREADS - 1) / NTHREADS; }

// psi Fbar and rho Fbar of the force adjoints in planes fb (state densities
// rdev) over a tile of W x H staged nodes whose first node is lattice node
// (x0, y0) (periodic wrap; zero beyond a wall, where no force acts)
template <int W, int H>
__device__ __forceinline__ void stage_qr(const AdjPar &A, const float *__restrict__ rdev, int fb,
                                         int x0, int y0, float (&q)[2][2][H][W],
                                         float (&r)[2][2][H][W])
{
    constexpr int N = W * H, IT = stage_iters<N>();
    float rv[IT][2], fv[IT][2][2];
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const int t = min((int)threadIdx.x + j * NTHREADS, N - 1);
        const int lx = t % W, ly = t / W;
        const int gx = wrapi(x0 + lx, A.nx);
        const int gy = y0 + ly;
        const bool ghost = A.walls && (gy < 0 || gy >= A.ny);
        const int yy = ghost ? 0 : wrapi(gy, A.ny);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            rv[j][k] = rdev[didx(A, k, gx, yy)];
#pragma unroll
            for (int d = 0; d < 2; ++d) fv[j][k][d] = A.scr[sidx(A, fb + 2 * k + d, gx, yy)];
        }
    }
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const int t = (int)threadIdx.x + j * NTHREADS;
        if (t >= N) break;
        const int lx = t % W, ly = t / W;
        const int gy = y0 + ly;
        const bool ghost = A.walls && (gy < 0 || gy >= A.ny);  // no force acts there
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float rk = A.rho_ref[k] + rv[j][k];
            const float p = apsi(A, rk);
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const float fbv = ghost ? 0.0f : fv[j][k][d];
                q[k][d][ly][lx] = p * fbv;
                r[k][d][ly][lx] = rk * fbv;
            }
        }
    }
}

// Sum of NV doubles over the block (256 threads = 4 wavefronts) in a fixed
// order; thread 0 writes out[0..NV).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out, bool accumulate = false)
{
    __shared__ double red[NTHREADS / 64][NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double s = v[j];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        v[j] = s;
    }
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64;
    if (ln == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) red[wv][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double s = 0.0;
            for (int w = 0; w < NTHREADS / 64; ++w) s += red[w][j];
            out[j] = accumulate ? out[j] + s : s;
        }
}

__device__ __forceinline__ int block_id() { return blockIdx.y * gridDim.x + blockIdx.x; }

// ---------------------------------------------------------------- densities
__global__ __launch_bounds__(NTHREADS) void k_adj_density(AdjPar A, const float *__restrict__ f)
{
    const int x = blockIdx.x * TX + (int)(threadIdx.x % TX);
    const int y = blockIdx.y * TY + (int)(threadIdx.x / TX);
    if (x >= A.nx || y >= A.ny) return;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        float v[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = f[pidx(A, k * 9 + i, x, y)];
        A.rscr[didx(A, k, x, y)] = sum9(v);
    }
}

// The local transpose takes tiles of 64 x LTY nodes, each thread LSUB
// nodes of one column: a lattice of 512 x 512 then gives every lane of the
// GPU two nodes in one round of blocks, where one node per thread would
// leave a second, thinly occupied round (its 168 registers allow three
// wavefronts per SIMD, 1.33 rounds of 64 x 4 tiles there), and the staged
// halo rows are shared by more nodes.
constexpr int LSUB = 2;
constexpr int LTY = TY * LSUB;

// Stage rho and psi of both components over a tile of H rows and its halo
// of 2 (periodic in x, periodic in y or the wall densities beyond a wall).
template <int H>
struct RTile {
    float rho[2][H + 2 * HALO][AW];
    float psi[2][H + 2 * HALO][AW];
};

template <int H>
__device__ __forceinline__ void stage_rho(const AdjPar &A, int x0, int y0, RTile<H> &T)
{
    constexpr int N = AW * (H + 2 * HALO), IT = stage_iters<N>();
    float dv[IT][2];
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const int t = min((int)threadIdx.x + j * NTHREADS, N - 1);
        const int lx = t % AW, ly = t / AW;
        const int gx = wrapi(x0 + lx - HALO, A.nx);
        const int gy = y0 + ly - HALO;
        const int yy = (A.walls && (gy < 0 || gy >= A.ny)) ? 0 : wrapi(gy, A.ny);
#pragma unroll
        for (int k = 0; k < 2; ++k) dv[j][k] = A.rdev[didx(A, k, gx, yy)];
    }
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const int t = (int)threadIdx.x + j * NTHREADS;
        if (t >= N) break;
        const int lx = t % AW, ly = t / AW;
        const int gy = y0 + ly - HALO;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            float r, p;
            if (A.walls && (gy < 0 || gy >= A.ny)) {
                r = A.rho_wall[k];
                p = A.psi_wall[k];
            } else {
                r = A.rho_ref[k] + dv[j][k];
                p = apsi(A, r);
            }
            T.rho[k][ly][lx] = r;
            T.psi[k][ly][lx] = p;
        }
    }
}

// ---------------------------------------------------------------- local transpose
// MODE 0: adjoint step.  MODE 1: seed of J_Q = (1/nx) sum_x u_x.
// Block partials: [0..4] theta, [5] J.
// The folded force pass of the step before: psi Fbar and rho Fbar staged
// with a halo of FH = 3 (the gather reads the addition one node beyond the
// tile, whose stencil reaches two nodes further), and the addition itself
// over the tile and a halo of 1.
constexpr int FH = 3;
struct FoldTile {
    float q[2][2][LTY + 2 * FH][TX + 2 * FH];
    float r[2][2][LTY + 2 * FH][TX + 2 * FH];
    float add[2][LTY + 2][TX + 2];
};

// FOLD 1 (MODE 0 only): the gather adds the pending addition of the step
// before formed here from its force adjoints (planes A.fbi, densities
// A.rdev_next); FOLD 0: read from scratch (SCR_ADD, written by k_adj_force
// or cleared).
template <int MODE, int FOLD>
// two wavefronts per SIMD (the populations and the stencil sums are not
// held across the transpose), LDS 38 KB per block (73 KB folded)
__global__ __launch_bounds__(NTHREADS, 2) void k_adj_local(AdjPar A, const float *__restrict__ f,
                                                        const float *__restrict__ lam_next,
                                                        float *__restrict__ lam)
{
    static_assert(MODE == 0 || !FOLD, "the seed has no step before");
    __shared__ RTile<LTY> T;
    // each thread's FP64 stencil sums [k][s1x s1y s2x s2y srx sry], parked in
    // LDS between the force recompute and the own-node terms
    __shared__ double SS[NTHREADS][2][6];
    __shared__ typename std::conditional<FOLD != 0, FoldTile, char>::type FT;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * LTY;
    stage_rho(A, x0, y0, T);
    if constexpr (FOLD != 0) {
        stage_qr<TX + 2 * FH, LTY + 2 * FH>(A, A.rdev_next, A.fbi, x0 - FH, y0 - FH, FT.q, FT.r);
        __syncthreads();
        // the addition at the tile's nodes and one node around (rows beyond a
        // wall are never gathered: bounce-back reads the node itself); the
        // densities are loaded first, as in the staging loops
        constexpr int NA = (TX + 2) * (LTY + 2), IA = stage_iters<NA>();
        float rn[IA][2];
#pragma unroll
        for (int j = 0; j < IA; ++j) {
            const int t = min((int)threadIdx.x + j * NTHREADS, NA - 1);
            const int ax = t % (TX + 2), ay = t / (TX + 2);
            const int gx = wrapi(x0 + ax - 1, A.nx), gy = y0 + ay - 1;
            const int yy = (A.walls && (gy < 0 || gy >= A.ny)) ? 0 : wrapi(gy, A.ny);
#pragma unroll
            for (int k = 0; k < 2; ++k) rn[j][k] = A.rdev_next[didx(A, k, gx, yy)];
        }
#pragma unroll
        for (int j = 0; j < IA; ++j) {
            const int t = (int)threadIdx.x + j * NTHREADS;
            if (t >= NA) break;
            const int ax = t % (TX + 2), ay = t / (TX + 2);
            const int gy = y0 + ay - 1;
            if (A.walls && (gy < 0 || gy >= A.ny)) {
                FT.add[0][ay][ax] = FT.add[1][ay][ax] = 0.0f;
                continue;
            }
            const int qx = ax + FH - 1, qy = ay + FH - 1;  // the node in the staged tile
            auto q = [&](int k, int d, int dx, int dy) { return FT.q[k][d][qy + dy][qx + dx]; };
            auto r = [&](int k, int d, int dx, int dy) { return FT.r[k][d][qy + dy][qx + dx]; };
#pragma unroll
            for (int k = 0; k < 2; ++k)
                FT.add[k][ay][ax] = force_add(A, k, q, r, A.rho_ref[k] + rn[j][k]);
        }
    }
    __syncthreads();
    double acc[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
    for (int sub = 0; sub < LSUB; ++sub) {
    const int lx = (int)(threadIdx.x % TX), ly = (int)(threadIdx.x / TX) + TY * sub;
    const int x = x0 + lx, y = y0 + ly;
    if (x < A.nx && y < A.ny) {
        const int cx = lx + HALO, cy = ly + HALO;
        float rho[2], psi[2], drho[2], mx[2], my[2], F[2][2];
        // the three stencil sums of a component at this node (FP64)
        auto sums = [&](int k, double (&s1)[2], double (&s2)[2], double (&sr)[2]) {
            auto vp = [&](int dx, int dy) { return T.psi[k][cy + dy][cx + dx]; };
            auto vr = [&](int dx, int dy) { return T.rho[1 - k][cy + dy][cx + dx]; };
            sum9s<double>(vp, DW1, DW2, s1[0], s1[1]);
            sum25<double>(vp, DP1, DP2, DP4, DP5, DP8, s2[0], s2[1]);
            sum9s<double>(vr, DW1, DW2, sr[0], sr[1]);
        };
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            float dev[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) dev[i] = f[pidx(A, k * 9 + i, x, y)];
            rho[k] = T.rho[k][cy][cx];
            psi[k] = T.psi[k][cy][cx];
            drho[k] = A.rdev[didx(A, k, x, y)];
            mx[k] = (dev[1] - dev[3]) + (dev[5] - dev[7]) + (dev[8] - dev[6]);
            my[k] = (dev[2] - dev[4]) + (dev[5] - dev[7]) + (dev[6] - dev[8]);
            double s1[2], s2[2], sr[2];
            sums(k, s1, s2, sr);
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                F[k][d] = (float)(-(double)psi[k] * ((double)A.G1[k] * s1[d] + (double)A.G2[k] * s2[d]) -
                                  (double)A.gab * (double)rho[k] * sr[d]) +
                          rho[k] * A.g[k][d];
                SS[threadIdx.x][k][d] = s1[d];
                SS[threadIdx.x][k][2 + d] = s2[d];
                SS[threadIdx.x][k][4 + d] = sr[d];
            }
        }
        float jx[2], jy[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            jx[k] = mx[k] + 0.5f * F[k][0];
            jy[k] = my[k] + 0.5f * F[k][1];
        }
        const float D = rho[0] * A.it[0] + rho[1] * A.it[1];
        const float iD = 1.0f / D;
        const float ux = (jx[0] * A.it[0] + jx[1] * A.it[1]) * iD;
        const float uy = (jy[0] * A.it[0] + jy[1] * A.it[1]) * iD;
        // Compiler-only barrier (no instruction): the populations (from
        // cache) and the stencil sums (from LDS) are read again below instead
        // of being held in registers across the FP64 transpose, which keeps
        // the kernel within the register budget of two wavefronts per SIMD
        // without spilling.
        asm volatile("" ::: "memory");

        // The transpose is evaluated in FP64 from the FP32 linearisation point:
        // for adjoints of conserved or nearly conserved quantities its terms
        // cancel node by node (the exact adjoint of a conserved functional is
        // invariant), and FP32 arithmetic there would leave a noise floor on
        // small gradients.  Only the stored lam is rounded to FP32.
        using R = double;
        R Fb[2][2];
        R gtau[2] = {0.0, 0.0};
        // the local part of lam is lam_c[k] + lam_a[k] a_i + mb[k] . e_i (MODE 0:
        // lam_a = 1 - 1/tau_k; MODE 1: lam_a = 0, a = 0)
        R lam_c[2] = {0.0, 0.0}, lam_a[2] = {0.0, 0.0}, mbx[2] = {0.0, 0.0}, mby[2] = {0.0, 0.0};
        float a[2][9];
        const R Ux = ux, Uy = uy, UU = (R)ux * ux + (R)uy * uy, ID = (R)1 / ((R)rho[0] * A.it[0] + (R)rho[1] * A.it[1]);
        if (MODE == 0) {
            // transpose of streaming (pull of the downstream adjoint)
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int yd = y + c_ey[i];
                const bool bounce = A.walls && (yd < 0 || yd >= A.ny);
                const int xs = bounce ? x : wrap1(x + c_ex[i], A.nx);
                const int ys = bounce ? y : wrap1(yd, A.ny);
                const int is = bounce ? c_op[i] : i;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    float add;
                    if constexpr (FOLD != 0)
                        add = FT.add[k][ly + 1 + (bounce ? 0 : c_ey[i])][lx + 1 + (bounce ? 0 : c_ex[i])];
                    else
                        add = A.scr[sidx(A, SCR_ADD + k, xs, ys)];
                    a[k][i] = lam_next[xidx(A, k * 9 + is, xs, ys)] + add;
                }
            }
            // transpose of Eq. 1 (BGK + Guo) at fixed rho_k, u, F_k
            R ubx = 0.0, uby = 0.0, rbar[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const R it = A.it[k], c = A.cg[k], Fx = F[k][0], Fy = F[k][1], rk = rho[k];
                R rb = 0.0, fbx = 0.0, fby = 0.0, gt = 0.0, gg = 0.0;
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const int ex = c_ex[i], ey = c_ey[i];
                    const R w = (R)wgt9[i];
                    const R eu = emul(ex, Ux) + emul(ey, Uy);
                    const R eF = emul(ex, Fx) + emul(ey, Fy);
                    const R Em1 = 3.0 * eu + 4.5 * eu * eu - 1.5 * UU;  // E - 1
                    const R ai = (R)a[k][i];
                    rb += ai * w * (1.0 + Em1);
                    const R awr = ai * w * rk * it;
                    const R eu9 = 9.0 * eu, eF9 = 9.0 * eF;
                    ubx += awr * (emul(ex, 3.0 + eu9) - 3.0 * Ux);
                    uby += awr * (emul(ey, 3.0 + eu9) - 3.0 * Uy);
                    const R gx = emul(ex, 3.0 + eu9) - 3.0 * Ux;
                    const R gy = emul(ey, 3.0 + eu9) - 3.0 * Uy;
                    fbx += ai * w * gx;
                    fby += ai * w * gy;
                    ubx += ai * c * w * (emul(ex, eF9) - 3.0 * Fx);
                    uby += ai * c * w * (emul(ey, eF9) - 3.0 * Fy);
                    // f - feq in deviation form: dev - w (drho + rho (E - 1))
                    const R fneq = (R)f[pidx(A, k * 9 + i, x, y)] - w * ((R)drho[k] + rk * Em1);
                    gt += ai * fneq;
                    gg += ai * w * (gx * Fx + gy * Fy);
                }
                rbar[k] = rb * it;
                Fb[k][0] = c * fbx;
                Fb[k][1] = c * fby;
                gtau[k] = (gt + 0.5 * gg) * it * it;
            }
            // transpose of Eq. 3 and of Eq. 6 (j = m + F/2)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const R it = A.it[k];
                const R jbx = ubx * it * ID, jby = uby * it * ID;
                rbar[k] -= (ubx * Ux + uby * Uy) * it * ID;
                gtau[k] += (ubx * (Ux * rho[k] - jx[k]) + uby * (Uy * rho[k] - jy[k])) * it * it * ID;
                mbx[k] = jbx;
                mby[k] = jby;
                Fb[k][0] += 0.5 * jbx;
                Fb[k][1] += 0.5 * jby;
                lam_c[k] = rbar[k];
                lam_a[k] = 1.0 - it;
            }
        } else {
            // J_Q: u_x = (sum_k m_kx + F_kx / 2) / rho, summed over x and / nx
            const R rt = (R)rho[0] + rho[1];
            const R irt = 1.0 / rt;
            const R ubar = ((R)jx[0] + jx[1]) * irt;
            acc[5] += ubar * (R)A.qscale;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                // q (e_x - u_x) / rho
                lam_c[k] = -(R)A.qscale * ubar * irt;
                mbx[k] = (R)A.qscale * irt;
                Fb[k][0] = 0.5 * (R)A.qscale * irt;
                Fb[k][1] = 0.0;
#pragma unroll
                for (int i = 0; i < 9; ++i) a[k][i] = 0.0f;
            }
        }
        // own-node terms of the force transpose and the coupling gradients
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double *ss = SS[threadIdx.x][k];
            const double s1[2] = {ss[0], ss[1]}, s2[2] = {ss[2], ss[3]}, sr[2] = {ss[4], ss[5]};
            const R s1F = s1[0] * Fb[k][0] + s1[1] * Fb[k][1];
            const R s2F = s2[0] * Fb[k][0] + s2[1] * Fb[k][1];
            const R srF = sr[0] * Fb[k][0] + sr[1] * Fb[k][1];
            const R psibar = -((R)A.G1[k] * s1F + (R)A.G2[k] * s2F);
            const R rown = psibar * (R)expf(-rho[k] * A.inv_rho0) - (R)A.gab * srF +
                           (R)A.g[k][0] * Fb[k][0] + (R)A.g[k][1] * Fb[k][1];
#pragma unroll
            for (int i = 0; i < 9; ++i)
                lam[xidx(A, k * 9 + i, x, y)] =
                    (float)((lam_a[k] * (R)a[k][i] + emul(c_ex[i], mbx[k]) + emul(c_ey[i], mby[k]) + lam_c[k]) + rown);
            A.scr[sidx(A, A.fbo + 2 * k, x, y)] = (float)Fb[k][0];
            A.scr[sidx(A, A.fbo + 2 * k + 1, x, y)] = (float)Fb[k][1];
            acc[0] += -(R)psi[k] * s1F;
            acc[1] += -(R)psi[k] * s2F;
            acc[2] += -(R)rho[k] * srF;
            acc[3 + k] += gtau[k];
        }
    }
    }  // sub
    // adjoint steps add into their block's slot (cleared by k_adj_zero before a
    // run; launches on one stream are ordered, so no two blocks share a slot)
    block_sum(acc, A.part + (int64_t)block_id() * NPART, MODE == 0);
}

// clear the per-block partial sums (a kernel, not a memset: graph-safe)
__global__ __launch_bounds__(256) void k_adj_zero(AdjPar A, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) A.part[i] = 0.0;
}

// ---------------------------------------------------------------- force transpose
// Neighbour terms (force_add): with q_k = psi_k Fbar_k and r_k = rho_k Fbar_k,
// lam_{k,i}(y) += psibar_k(y) exp(-rho_k / rho0) + rhobar_k(y), the same for
// all i: the kernel writes that addition per component (SCR_ADD), and the
// next step's gather, or the combine pass, adds it where lam is read.
struct QTile {
    float q[2][2][AH][AW];  // [k][d]
    float r[2][2][AH][AW];
};

__global__ __launch_bounds__(NTHREADS) void k_adj_force(AdjPar A)
{
    __shared__ QTile T;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    stage_qr<AW, AH>(A, A.rdev, A.fbo, x0 - HALO, y0 - HALO, T.q, T.r);
    __syncthreads();
    const int lx = (int)(threadIdx.x % TX), ly = (int)(threadIdx.x / TX);
    const int x = x0 + lx, y = y0 + ly;
    if (x >= A.nx || y >= A.ny) return;
    const int cx = lx + HALO, cy = ly + HALO;
    auto q = [&](int k, int d, int dx, int dy) { return T.q[k][d][cy + dy][cx + dx]; };
    auto r = [&](int k, int d, int dx, int dy) { return T.r[k][d][cy + dy][cx + dx]; };
    float add[2];
#pragma unroll
    for (int k = 0; k < 2; ++k)
        add[k] = force_add(A, k, q, r, A.rho_ref[k] + A.rdev[didx(A, k, x, y)]);
#pragma unroll
    for (int k = 0; k < 2; ++k) A.scr[sidx(A, SCR_ADD + k, x, y)] = add[k];
}

// out_{k,i} = in_{k,i} + add_k (the pending force-transpose addition)
__global__ __launch_bounds__(NTHREADS) void k_adj_combine(AdjPar A, const float *in,
                                                          float *out)
{
    const int x = blockIdx.x * TX + (int)(threadIdx.x % TX);
    const int y = blockIdx.y * TY + (int)(threadIdx.x / TX);
    if (x >= A.nx || y >= A.ny) return;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float a = A.scr[sidx(A, SCR_ADD + k, x, y)];
#pragma unroll
        for (int i = 0; i < 9; ++i) out[xidx(A, k * 9 + i, x, y)] = in[xidx(A, k * 9 + i, x, y)] + a;
    }
}

// no pending addition (before the first step of a run)
__global__ __launch_bounds__(NTHREADS) void k_adj_clear_add(AdjPar A)
{
    const int x = blockIdx.x * TX + (int)(threadIdx.x % TX);
    const int y = blockIdx.y * TY + (int)(threadIdx.x / TX);
    if (x >= A.nx || y >= A.ny) return;
#pragma unroll
    for (int k = 0; k < 2; ++k) A.scr[sidx(A, SCR_ADD + k, x, y)] = 0.0f;
}

// ---------------------------------------------------------------- objectives
// J_dp sums per block: [0] S_A [1] S_B [2] P_A [3] P_B [4] dP_A/dG12 [5] dP_B/dG12
// [6] dP_A/dG_AB [7] dP_B/dG_AB (p_b of Eq. 11, weights chi = max(0, +-phi)^4)
__device__ __forceinline__ float bulk_pressure(const AdjPar &A, float ra, float rb, float pa,
                                               float pb)
{
    return (ra + 0.5f * (A.G1[0] + A.G2[0]) * pa * pa + rb + 0.5f * (A.G1[1] + A.G2[1]) * pb * pb +
            A.gab * ra * rb) *
           (1.0f / 3.0f);
}

__global__ __launch_bounds__(NTHREADS) void k_obj_dp_sums(AdjPar A)
{
    const int x = blockIdx.x * TX + (int)(threadIdx.x % TX);
    const int y = blockIdx.y * TY + (int)(threadIdx.x / TX);
    double acc[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (x < A.nx && y < A.ny) {
        const float ra = A.rho_ref[0] + A.rdev[didx(A, 0, x, y)];
        const float rb = A.rho_ref[1] + A.rdev[didx(A, 1, x, y)];
        const float pa = apsi(A, ra), pb = apsi(A, rb);
        const float pr = bulk_pressure(A, ra, rb, pa, pb);
        const float phi = (ra - rb) / (ra + rb);
        const float p2 = phi * phi;
        const float ca = phi > 0.0f ? p2 * p2 : 0.0f, cb = phi < 0.0f ? p2 * p2 : 0.0f;
        const float dG12 = (0.5f / 3.0f) * (pa * pa + pb * pb), dGab = ra * rb * (1.0f / 3.0f);
        acc[0] = ca;
        acc[1] = cb;
        acc[2] = (double)pr * ca;
        acc[3] = (double)pr * cb;
        acc[4] = (double)dG12 * ca;
        acc[5] = (double)dG12 * cb;
        acc[6] = (double)dGab * ca;
        acc[7] = (double)dGab * cb;
    }
    block_sum(acc, A.part + (int64_t)block_id() * NPART);
}

// seed of J_dp: dJ/df_{k,i} = dJ/drho_k for every i; m = {<p>_A, <p>_B, S_A, S_B}
__global__ __launch_bounds__(NTHREADS) void k_obj_dp_seed(AdjPar A, float *__restrict__ lam,
                                                          float mA, float mB, float iSA, float iSB)
{
    const int x = blockIdx.x * TX + (int)(threadIdx.x % TX);
    const int y = blockIdx.y * TY + (int)(threadIdx.x / TX);
    if (x >= A.nx || y >= A.ny) return;
    const float ra = A.rho_ref[0] + A.rdev[didx(A, 0, x, y)];
    const float rb = A.rho_ref[1] + A.rdev[didx(A, 1, x, y)];
    const float pa = apsi(A, ra), pb = apsi(A, rb);
    const float pr = bulk_pressure(A, ra, rb, pa, pb);
    const float s = ra + rb, is2 = 1.0f / (s * s);
    const float phi = (ra - rb) / s;
    const float dphi[2] = {2.0f * rb * is2, -2.0f * ra * is2};
    const float dp[2] = {
        (1.0f + (A.G1[0] + A.G2[0]) * pa * expf(-ra * A.inv_rho0) + A.gab * rb) * (1.0f / 3.0f),
        (1.0f + (A.G1[1] + A.G2[1]) * pb * expf(-rb * A.inv_rho0) + A.gab * ra) * (1.0f / 3.0f)};
    const float p2 = phi * phi;
    const float ca = phi > 0.0f ? p2 * p2 : 0.0f, cb = phi < 0.0f ? p2 * p2 : 0.0f;
    const float dca = phi > 0.0f ? 4.0f * p2 * phi : 0.0f, dcb = phi < 0.0f ? 4.0f * p2 * phi : 0.0f;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float d = (dp[k] * ca + (pr - mA) * dca * dphi[k]) * iSA -
                        (dp[k] * cb + (pr - mB) * dcb * dphi[k]) * iSB;
#pragma unroll
        for (int i = 0; i < 9; ++i) lam[xidx(A, k * 9 + i, x, y)] = d;
    }
}

// linear functionals J = sum c_{k,i} f_{k,i}: which 2 (x-momentum of A),
// 3 (total x-momentum), 4 (mass of A); block partial slot 5 holds J
__global__ __launch_bounds__(NTHREADS) void k_obj_lin(AdjPar A, const float *__restrict__ f,
                                                      float *__restrict__ lam, int which)
{
    const int x = blockIdx.x * TX + (int)(threadIdx.x % TX);
    const int y = blockIdx.y * TY + (int)(threadIdx.x / TX);
    double acc[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (x < A.nx && y < A.ny) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const float c = which == 4 ? (k == 0 ? 1.0f : 0.0f)
                                           : (which == 2 && k == 1 ? 0.0f : (float)c_ex[i]);
                const float fi = f[pidx(A, k * 9 + i, x, y)] + wgt(i) * A.rho_ref[k];
                s += (double)c * (double)fi;
                if (lam) lam[xidx(A, k * 9 + i, x, y)] = c;
            }
        acc[5] = s;
    }
    block_sum(acc, A.part + (int64_t)block_id() * NPART);
}

// Fixed-order sum of the per-block partials into res[0..NPART); if grad is
// not NULL, grad[0..4] += res[0..4].
__global__ __launch_bounds__(256) void k_adj_final(AdjPar A, int nblocks, double *__restrict__ grad)
{
    __shared__ double red[NPART * (256 / 64)];
    double v[NPART];
    int op[NPART];
    for (int j = 0; j < NPART; ++j) {
        v[j] = 0.0;
        op[j] = RED_SUM;
        for (int b = threadIdx.x; b < nblocks; b += 256) v[j] += A.part[(int64_t)b * NPART + j];
    }
    block_reduce<256>(v, op, red);
    if (threadIdx.x == 0)
        for (int j = 0; j < NPART; ++j) {
            A.res[j] = v[j];
            if (grad && j < 5) grad[j] += v[j];
        }
}

dim3 agrid(const AdjPar &A) { return dim3((A.nx + TX - 1) / TX, (A.ny + TY - 1) / TY); }
int nblk(const AdjPar &A) { return (int)(((A.nx + TX - 1) / TX) * ((A.ny + TY - 1) / TY)); }
// grid of the local transpose (tiles of LTY rows; its partial slots are the
// first lblk of the nblk)
dim3 lgrid(const AdjPar &A) { return dim3((A.nx + TX - 1) / TX, (A.ny + LTY - 1) / LTY); }
int lblk(const AdjPar &A) { return (int)(((A.nx + TX - 1) / TX) * ((A.ny + LTY - 1) / LTY)); }

}  // namespace

#define LAUNCH_CHECK()                                            \
    do {                                                          \
        hipError_t e_ = hipGetLastError();                        \
        if (e_ != hipSuccess) return e_;                          \
    } while (0)

hipError_t launch_adjoint_zero(const AdjPar &A, hipStream_t st)
{
    const int n = nblk(A) * NPART;
    k_adj_zero<<<(n + 255) / 256, 256, 0, st>>>(A, n);
    LAUNCH_CHECK();
    k_adj_clear_add<<<agrid(A), NTHREADS, 0, st>>>(A);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_adjoint_combine(const AdjPar &A, const float *in, float *out, hipStream_t st)
{
    k_adj_combine<<<agrid(A), NTHREADS, 0, st>>>(A, in, out);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_adjoint_body(const AdjPar &A, const float *f, const float *rdev,
                               const float *lam_next, float *lam, hipStream_t st)
{
    AdjPar B = A;
    if (rdev) {
        B.rdev = rdev;
    } else {
        k_adj_density<<<agrid(A), NTHREADS, 0, st>>>(A, f);
        LAUNCH_CHECK();
        B.rdev = A.rscr;
    }
    k_adj_local<0, 0><<<lgrid(B), NTHREADS, 0, st>>>(B, f, lam_next, lam);
    LAUNCH_CHECK();
    k_adj_force<<<agrid(B), NTHREADS, 0, st>>>(B);
    LAUNCH_CHECK();
    return hipSuccess;
}


hipError_t launch_adjoint_local(const AdjPar &A, bool fold, const float *f, const float *lam_next,
                                float *lam, hipStream_t st)
{
    if (fold)
        k_adj_local<0, 1><<<lgrid(A), NTHREADS, 0, st>>>(A, f, lam_next, lam);
    else
        k_adj_local<0, 0><<<lgrid(A), NTHREADS, 0, st>>>(A, f, lam_next, lam);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_adjoint_force(const AdjPar &A, hipStream_t st)
{
    k_adj_force<<<agrid(A), NTHREADS, 0, st>>>(A);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_adjoint_final(const AdjPar &A, double *grad, hipStream_t st)
{
    k_adj_final<<<1, 256, 0, st>>>(A, nblk(A), grad);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_adjoint_step(const AdjPar &A, const float *f, const float *lam_next, float *lam,
                               double *grad, hipStream_t st)
{
    hipError_t e = launch_adjoint_zero(A, st);
    if (e == hipSuccess) e = launch_adjoint_body(A, f, nullptr, lam_next, lam, st);
    if (e == hipSuccess) e = launch_adjoint_combine(A, lam, lam, st);
    if (e == hipSuccess) e = launch_adjoint_final(A, grad, st);
    return e;
}

hipError_t launch_objective_pass1(const AdjPar &A, int which, const float *f, float *lam,
                                  hipStream_t st)
{
    k_adj_density<<<agrid(A), NTHREADS, 0, st>>>(A, f);
    LAUNCH_CHECK();
    if (which == 0) {
        k_obj_dp_sums<<<agrid(A), NTHREADS, 0, st>>>(A);
    } else if (which == 1) {
        k_adj_local<1, 0><<<lgrid(A), NTHREADS, 0, st>>>(A, f, nullptr, lam);
        LAUNCH_CHECK();
        k_adj_force<<<agrid(A), NTHREADS, 0, st>>>(A);
        LAUNCH_CHECK();
        k_adj_combine<<<agrid(A), NTHREADS, 0, st>>>(A, lam, lam);
    } else {
        k_obj_lin<<<agrid(A), NTHREADS, 0, st>>>(A, f, lam, which);
    }
    LAUNCH_CHECK();
    // the local transpose writes the partials of its own (fewer) blocks
    k_adj_final<<<1, 256, 0, st>>>(A, which == 1 ? lblk(A) : nblk(A), nullptr);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_objective_dp_seed(const AdjPar &A, float *lam, double mA, double mB, double SA,
                                    double SB, hipStream_t st)
{
    k_obj_dp_seed<<<agrid(A), NTHREADS, 0, st>>>(A, lam, (float)mA, (float)mB, (float)(1.0 / SA),
                                                 (float)(1.0 / SB));
    LAUNCH_CHECK();
    return hipSuccess;
}

int adjoint_blocks(int nx, int ny) { return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY); }

const char *adjoint_kernel_name(int j)
{
    static const char *names[] = {"k_adj_density", "k_adj_local", "k_adj_force", "k_adj_final",
                                  "k_adj_local_fold"};
    return j >= 0 && j < N_ADJ_KERNELS ? names[j] : "";
}

hipError_t launch_adjoint_kernel(const AdjPar &A, int j, const float *f, const float *lam_next,
                                 float *lam, double *grad, hipStream_t st)
{
    switch (j) {
    case 0: k_adj_density<<<agrid(A), NTHREADS, 0, st>>>(A, f); break;
    // (the timed local pass accumulates into its partial slots; cleared before use)
    case 1: k_adj_local<0, 0><<<lgrid(A), NTHREADS, 0, st>>>(A, f, lam_next, lam); break;
    case 2: k_adj_force<<<agrid(A), NTHREADS, 0, st>>>(A); break;
    case 3: k_adj_final<<<1, 256, 0, st>>>(A, nblk(A), grad); break;
    // the local pass of a run's later steps, with the force pass of the step
    // before folded in (here: the force adjoints in the second set of planes
    // and the same state's densities, for timing)
    default: {
        AdjPar B = A;
        B.fbi = A.fbo == SCR_FBAR ? SCR_FBAR2 : SCR_FBAR;
        B.rdev_next = A.rdev;
        k_adj_local<0, 1><<<lgrid(B), NTHREADS, 0, st>>>(B, f, lam_next, lam);
        break;
    }
    }
    LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace lbm
