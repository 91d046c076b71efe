// HIP kernels of the two-range pseudopotential LBM step on gfx950
// (arXiv:1806.06943, Sec. II).  Every kernel walks a flat table of strips,
// tiles or rows tagged with their instance, so one launch covers one lattice
// or many lattices of different sizes alike.
#include "lbm_internal.h"

#include <type_traits>

namespace lbm {

// ------------------------------------------------------------------ init
// Equilibrium at rest, f_{k,i} = w_i rho_k (Eq. 2 with u = 0), from FP64
// densities rho0s[inst][k][ny][nx] (dense), rounded once to FP32 deviations.
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
    constexpr double CI[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    float *out = P.f[par];
    for (int k = 0; k < 2; ++k) {
        const double r = rho0[k * N + (int64_t)y * P.nx + x];
        for (int i = 0; i < 9; ++i)
            out[fidx(P, k * 9 + i, x, y)] = (float)(CI[i] / 36.0 * (r - (double)P.rho_ref[k]));
    }
}

// ------------------------------------------------------------------ density pass
// Density deviation sum_i f_i(x) (Eq. 6, deviation form), correctly rounded,
// of the state in buffer par; the fused step writes the same quantity for
// the next state itself.
__global__ __launch_bounds__(NTHREADS) void k_density(const KInst *__restrict__ insts,
                                                       const int4 *__restrict__ tiles, int par)
{
    const int4 t = tiles[blockIdx.x];
    const KInst &P = insts[t.x];
    const int x = t.y + (int)(threadIdx.x % TX);
    const int y = t.z + (int)(threadIdx.x / TX);
    if (x >= P.nx || y >= P.ny) return;
    float f[2][9];
    load_node(P, P.f[par], x, y, f);
#pragma unroll
    for (int k = 0; k < 2; ++k) P.rho[par][ridx(P, k, x, y)] = sum9(f[k]);
}

// ------------------------------------------------------------------ fused step
// Buffer descriptor over one population or density buffer of an instance:
// accesses are (scalar plane offset, per-lane byte offset) pairs, and the
// hardware range check returns 0 for (and drops) anything beyond `bytes`.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, 0x00020000);
}

// FP32 load / store through a buffer descriptor (the b32 builtins move raw bits)
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                       uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// 16- and 8-byte loads, 8-byte stores through a buffer descriptor (raw bits)
__device__ __forceinline__ u32x4 bload4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
}

__device__ __forceinline__ u32x2 bload2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
}

__device__ __forceinline__ void bstore2(float a, float b, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                        uint32_t soff)
{
    u32x2 v = {__float_as_uint(a), __float_as_uint(b)};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
}

// A float4 plane entry as two 8-byte stores.  A 16-byte buffer store with a
// register soffset whose data registers the very next VALU instruction
// overwrote (a 64-bit result) stored the new values on this GPU under load;
// the compiler inserts no wait for that form.  8-byte stores, which bandwidth
// does not distinguish from 16-byte ones here, showed no such window.
__device__ __forceinline__ void bstore4(float a, float b, float c, float d,
                                        __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    bstore2(a, b, r, voff, soff);
    bstore2(c, d, r, voff, soff + 8u);
}

// Lane shifts of a wavefront through DPP (lane l receives lane l - 1, resp.
// l + 1; the end lanes, which no output consumes, receive 0: with the
// bound control set the shift needs no copy of its source to keep)
__device__ __forceinline__ float from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}

__device__ __forceinline__ float from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

// Density ring of a strip of NW wavefronts: RR rows (a rolling window over
// lattice rows) of 64 NW columns (plus 4 that no stencil of a used lane
// reads), column j holding lattice column X0 - 1 - HALO + j.  In full-row
// mode (FR) the group of wavefronts that starts at wavefront w0 owns the
// 68 w0 ... columns: lattice column X at 68 w0 + HALO + X, with the HALO
// columns on either side holding the periodic wrap of the row.
// A slot holds one row of the three fields with the two components side by
// side: the stencil reads of a row are immediate offsets from one address
// per slot.
template <int NW, int FR>
struct RingW {
    static constexpr int W = FR ? 68 * NW : 64 * NW + 2 * HALO;
    struct Row {
        float2 psi[W];
        float2 rho[W];
        float2 dev[W];  // density deviations (own-node term of the collision)
    };
    Row row[RR];
};

// Index checks of the LDS ring and edge arrays, compiled in with
// LBM_CHECK_LDS (the checked build of the library): an index outside its
// array is counted in g_lds_bad (read back by lbm_lds_checks) instead of
// being used; the plain build compiles them out.
#ifdef LBM_CHECK_LDS
__device__ unsigned int g_lds_bad;
#define LDS_CHECK(ok)                                     \
    do {                                                  \
        if (!(ok)) atomicAdd(&g_lds_bad, 1u);              \
    } while (0)
#else
#define LDS_CHECK(ok) \
    do {              \
    } while (0)
#endif

// accessor into the ring: slot[dy + 2] is the ring row of lattice row c + dy,
// cx the ring column of the node
template <class RT>
struct RingAccW {
    const RT &R;
    const int *slot;
    int cx;
    __device__ float psi(int k, int dx, int dy) const
    {
        const float2 v = R.row[slot[dy + HALO]].psi[cx + dx];
        return k ? v.y : v.x;
    }
    __device__ float rho(int k, int dx, int dy) const
    {
        const float2 v = R.row[slot[dy + HALO]].rho[cx + dx];
        return k ? v.y : v.x;
    }
};

// Barrier of a fused-step workgroup.  A one-wavefront workgroup needs none:
// the LDS accesses of a wavefront take effect in the order it issues them,
// so a lane reads what another lane of the same wavefront stored before; a
// scheduling barrier keeps the compiler from moving them across.  Waiting
// for every LDS access to complete at each barrier would only expose the
// LDS latency of a wavefront that is alone on its SIMD.
template <bool MULTI>
__device__ __forceinline__ void wg_sync()
{
    if constexpr (MULTI)
        __syncthreads();
    else
        __builtin_amdgcn_wave_barrier();
}

// One workgroup of NW wavefronts advances its segments, one after the
// other, by one time step; a segment is a strip of wo <= 64 NW - 6 output
// columns [X0, X0 + wo) and ho output rows [Y0, Y0 + ho).
// Thread L owns lattice column X0 - 3 + L: threads 0 .. wo + 5 load their
// column, threads 2 .. wo + 3 collide it (threads 2 and wo + 3 are the
// one-column halo whose collision the neighbouring strips also compute).
// The workgroup marches down the rows:
//   * the populations of each row are read once, three rows ahead of their
//     collision: their sums give rho and psi of that row in an LDS ring that
//     holds rows c-2 .. c+2 for the force stencil of collided row c, and the
//     populations of rows c .. c+2 wait in registers;
//   * collided rows c-2 (upward populations) and c-1 (all) stay in registers;
//   * output row o = c - 1 pulls f_i(x, o) = f*_i(x - e_i) from rows o-1, o,
//     o+1: the x shift by one column is a DPP lane shift inside a wavefront
//     and, across the boundary between two wavefronts, an exchange of the
//     six edge values per component through LDS; bounce-back takes the
//     node's own reflected population next to a wall;
//   * f(t+1) of the output row is written, and rho(t+1) when the launch
//     asks for it (for the other kernels and the caller: the step itself
//     never reads it).
// The loop body has no lane-divergent branches on global memory: every lane
// loads a valid column or, where nothing it loads is used (idle lanes beyond
// the halo), zeros, rows beyond a wall read a clamped row whose values are
// not used, and lanes that must not write give an offset beyond the buffer,
// which the descriptor's range check drops
// (buffers stay below 2 GiB, so that offset plus any segment offset cannot
// wrap into range).  Memory waits are then exact.  The loads of row c + 3
// are in flight while row c is collided.  Two barriers per row: after the
// collision (the ring row of c - 2 and the edge values are then free /
// published) and after the ring update; in a one-wavefront workgroup they
// are scheduling barriers only (wg_sync).
// FS selects the forcing: 0 the Guo term with the common velocity (Eq. 5),
// 1 the velocity shift of the original model (momenta without F/2, BGK
// towards the equilibrium at u^eq + tau_k F_k / rho_k, no explicit term).
// Reads f[par]; writes f[par ^ 1] and, with ovr.wrho, rho[par ^ 1].
// Register budget: two waves per SIMD (at most 256 VGPRs; the instances
// use 198-220), which every strip width meets without spilling although
// four rows of populations are live across the collision.
//
// FR = 1 (full rows): for lattices whose width is a multiple of 64, a group
// of k = nx / 64 wavefronts covers whole rows, lane l of the group's j-th
// wavefront owning column 64 j + l: every lane loads, collides and writes
// its own column, and no column is loaded or collided twice.  The ring holds
// the row with its periodic wrap, and the x shift of the pull crosses from
// the group's last wavefront to its first through the edge exchange.  A
// workgroup then advances several groups at once (the segments of its
// table entry range, each {inst, w0, Y0, k | ho << 16}, all with the same
// ho); wavefronts that no group uses only keep the workgroup's barriers.
template <int NW, int FS, int FR>
__global__ __launch_bounds__(64 * NW, 2) void k_fused_step(
    const KInst *__restrict__ insts, const int4 *__restrict__ segs, const int *__restrict__ first,
    int par, StepOvr ovr)
{
    __shared__ RingW<NW, FR> R;
    // edge values of each wavefront for its neighbours: [wave][side][6]
    __shared__ float edge[NW][2][6];
    const int L = (int)threadIdx.x;
    const int l = L & 63;
    // the wavefront index, as a scalar (it is uniform within a wavefront)
    const int wv = __builtin_amdgcn_readfirstlane(L >> 6);
    // the workgroup's segments, one after the other (a segment ends with a
    // barrier after which no thread reads the ring or the edges again); in
    // full-row mode one pass over concurrent groups
    const int sg_begin = first[blockIdx.x], sg_end = first[blockIdx.x + 1];
    const int npass = FR ? 1 : sg_end - sg_begin;
    for (int pass = 0; pass < npass; ++pass) {
    int sg = sg_begin + pass;
    int w0 = 0, gk = 0;  // full-row group: first wavefront and wavefront count
    if constexpr (FR) {
        int mine = -1;
        for (int e = sg_begin; e < sg_end; ++e) {
            const int4 te = segs[e];
            const int k = te.w & 0xffff;
            if (wv >= te.y && wv < te.y + k) {
                mine = e;
                w0 = te.y;
                gk = k;
            }
        }
        if (mine < 0) {
            // no group here: keep the barriers of the others (one after the
            // ring fill, two per row of the common height)
            const int nitw = (int)((uint32_t)segs[sg_begin].w >> 16) + 2;
            for (int b = 0; b < 1 + 2 * nitw; ++b) __syncthreads();
            continue;
        }
        sg = mine;
    }
    const int4 t = segs[sg];
    const KInst &G = insts[t.x];
    // arithmetic parameters copied once: the buffer stores below could
    // otherwise alias them
    const KPar P = kpar(G);
    const int X0 = FR ? 0 : t.y, Y0 = t.z, wo = t.w & 0xffff, ho = (int)((uint32_t)t.w >> 16);
    const int nx = G.nx, ny = G.ny, walls = G.walls;
    const uint32_t pb = (uint32_t)G.pitch;        // nodes per row (with padding)
    const uint32_t frowb = 72u * pb;              // bytes per population row
    const uint32_t rrowb = 8u * pb;               // bytes per density row
    // the instance's ping-pong pair, or the override's buffers (same layout)
    const bool ov = t.x == ovr.inst;
    const __amdgpu_buffer_rsrc_t fin = make_rsrc(ov ? ovr.fin : G.f[par], (uint32_t)ny * frowb);
    const __amdgpu_buffer_rsrc_t fout = make_rsrc(ov ? ovr.fout : G.f[par ^ 1], (uint32_t)ny * frowb);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(ov ? ovr.rout : G.rho[par ^ 1], (uint32_t)ny * rrowb);
    // out-of-range offset: a load returns 0 without a memory request, a store
    // is dropped (offsets below 2 GiB plus this one cannot wrap into range)
    constexpr uint32_t DROP = 0x80000000u;
    // Thread L owns lattice column X0 - 1 - HALO + L.  Lanes 0 .. wo + 1 +
    // 2 HALO load that column's populations: their densities fill ring
    // column L, and the populations wait in registers for the node's own
    // collision three rows later.  Lanes HALO .. wo + 1 + HALO collide (the
    // outer two are the one-column halo whose collision the neighbouring
    // strips also compute), lanes HALO + 1 .. wo + HALO write.  Lanes beyond
    // read zeros and write nothing.
    // In full-row mode lane l of the group's wavefront wv - w0 owns column
    // X = 64 (wv - w0) + l < nx, loads, collides and writes it; its ring
    // column is 68 w0 + HALO + X, and the lanes of the first and last HALO
    // columns also fill the wrap columns at the other end of the row.
    const int jmax = wo + 1 + 2 * HALO;
    const int X = FR ? 64 * (wv - w0) + l : X0 - 1 - HALO + L;
    const bool outl = FR ? true : (L >= HALO + 1) && (L <= wo + HALO);
    const uint32_t xl = FR ? (uint32_t)X : (uint32_t)wrapi(X, nx);
    const bool needf = FR ? true : L <= jmax;
    const uint32_t xf16 = needf ? xl * 16u : DROP, xf8 = needf ? xl * 8u : DROP;
    const int rbase = 68 * w0 + HALO;
    const int cl = FR ? rbase + X : L;  // this lane's ring column
    const int cw = !FR ? -1 : X >= nx - HALO ? rbase + X - nx : X < HALO ? rbase + nx + X : -1;
    // the stencil's centre column: the two load-only lanes at the left edge
    // of a strip (their collision is never used) take lane 2's, so that no
    // stencil reaches left of the ring
    const int cs = FR ? cl : (cl < HALO ? HALO : cl);
    [[maybe_unused]] constexpr int RW = RingW<NW, FR>::W;
    LDS_CHECK(cl >= 0 && cl < RW && cs >= HALO && cs + HALO < RW);
    LDS_CHECK(cw < RW);
    LDS_CHECK(!FR || (w0 >= 0 && w0 + gk <= NW));

    // lattice row r -> wrapped row index, or -1 beyond a wall (general
    // form, used once per cursor); cursors then advance by one row
    struct Cursor {
        int r, i;  // lattice row, its index (or -1)
    };
    auto cursor = [&](int r) {
        if (walls) return Cursor{r, (r >= 0 && r < ny) ? r : -1};
        return Cursor{r, wrapi(r, ny)};
    };
    auto advance = [&](Cursor &q) {
        ++q.r;
        if (walls)
            q.i = (q.r >= 0 && q.r < ny) ? q.r : -1;
        else
            q.i = (q.i + 1 == ny) ? 0 : q.i + 1;
    };
    // four float4 planes and one float2 plane per row (q = 9 k + i in order);
    // rows beyond a wall read row 0 (valid memory, never used), and a row
    // that nothing needs (live false: the loads of the last iteration)
    // reads zeros instead of memory
    auto load_f = [&](int ri, bool live, float f[2][9]) {
        const uint32_t ro = (uint32_t)(ri < 0 ? 0 : ri) * frowb;
        const uint32_t o16 = live ? ro + xf16 : DROP, o8 = live ? ro + xf8 : DROP;
        float q[18];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const u32x4 v = bload4(fin, o16, (uint32_t)g * 16u * pb);
            q[4 * g + 0] = __uint_as_float(v.x);
            q[4 * g + 1] = __uint_as_float(v.y);
            q[4 * g + 2] = __uint_as_float(v.z);
            q[4 * g + 3] = __uint_as_float(v.w);
        }
        const u32x2 w = bload2(fin, o8, 64u * pb);
        q[16] = __uint_as_float(w.x);
        q[17] = __uint_as_float(w.y);
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int i = 0; i < 9; ++i) f[k][i] = q[9 * k + i];
    };
    // ring column L of a row from that row's populations at column L: the
    // density deviations are the same correctly rounded sums that the step
    // writes as rho(t + 1) (Eq. 6); a row beyond a wall takes the wall's
    // densities instead
    auto ring_store = [&](int slot, int ri, const float q[2][9]) {
        LDS_CHECK(slot >= 0 && slot < RR);
        const float da = sum9(q[0]), db = sum9(q[1]);
        float ra = P.rho_ref[0] + da, rb = P.rho_ref[1] + db;
        float pa = psi_of(P, ra), pbv = psi_of(P, rb);
        if (ri < 0) {  // a row beyond a wall (uniform): no selects on the other rows
            ra = P.rho_wall[0];
            rb = P.rho_wall[1];
            pa = P.psi_wall[0];
            pbv = P.psi_wall[1];
        }
        R.row[slot].rho[cl] = make_float2(ra, rb);
        R.row[slot].psi[cl] = make_float2(pa, pbv);
        R.row[slot].dev[cl] = make_float2(da, db);
        if constexpr (FR) {
            if (cw >= 0) {  // the row's periodic wrap (stencil values only)
                R.row[slot].rho[cw] = make_float2(ra, rb);
                R.row[slot].psi[cw] = make_float2(pa, pbv);
            }
        }
    };

    // ring rows Y0 - 3 .. Y0 + 1 into slots 0..4 (slot[d] is the slot of row
    // c - 2 + d for the row c being collided); the populations of rows
    // Y0 - 1, Y0 and Y0 + 1 stay in fa, fb, fc for their collisions
    int slot[RR];
    Cursor cr = cursor(Y0 - 1 - HALO);  // next row to enter the ring
    float fa[2][9], fb[2][9], fc[2][9];
    {
        float t0[2][9], t1[2][9];
        int ri[RR];
#pragma unroll
        for (int q = 0; q < RR; ++q) {
            ri[q] = cr.i;
            slot[q] = q;
            advance(cr);
        }
        load_f(ri[0], true, t0);
        load_f(ri[1], true, t1);
        load_f(ri[2], true, fa);
        load_f(ri[3], true, fb);
        load_f(ri[4], true, fc);
        ring_store(0, ri[0], t0);
        ring_store(1, ri[1], t1);
        ring_store(2, ri[2], fa);
        ring_store(3, ri[3], fb);
        ring_store(4, ri[4], fc);
    }
    wg_sync<(NW > 1 || FR)>();

    Cursor cc = cursor(Y0 - 1);  // row being collided
    // collided values of two consecutive rows (S of row c, Sprev of row
    // c - 1) and the upward populations of row c - 2
    float Sa[2][9], Sb[2][9], Uprev[2][3], fd[2][9];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
#pragma unroll
        for (int i = 0; i < 9; ++i) Sb[k][i] = 0.0f;
        Uprev[k][0] = Uprev[k][1] = Uprev[k][2] = 0.0f;
    }

    // One row: collide row c from fa, load row c + 3 into fn.  The four
    // population buffers and the two collided rows change roles from row to
    // row by renaming (the loop below is unrolled by four), not by copies.
    auto row = [&](int it, const int nit, float (&fa)[2][9], float (&fn)[2][9], float (&S)[2][9],
                   const float (&Sprev)[2][9]) {
        // the populations of row c + 3, for the ring after this collision
        // and for their own collision three rows on (the last row needs
        // neither: its loads read zeros)
        const bool more = it + 1 < nit;
        const int rnext = cr.i;
        load_f(rnext, more, fn);

        // collide row c (a row beyond a wall is collided from clamped data
        // and never used)
        {
            float F[2][2];
            stencil_force(P, RingAccW<RingW<NW, FR>>{R, slot, cs}, F);
            // the node's own terms (at the stencil centre: the same column
            // except on the two load-only lanes, whose collision is unused)
            const float2 dv = R.row[slot[HALO]].dev[cs], rv = R.row[slot[HALO]].rho[cs];
            float drho[2] = {dv.x, dv.y}, rho[2] = {rv.x, rv.y}, jx[2], jy[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                float mx, my;
                mom9(fa[k], mx, my);
                jx[k] = FS ? mx : fmaf(0.5f, F[k][0], mx);
                jy[k] = FS ? my : fmaf(0.5f, F[k][1], my);
            }
            float ux, uy;
            common_velocity(P, rho, jx, jy, ux, uy);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if constexpr (FS) {
                    // equilibrium velocity shifted by tau_k F_k / rho_k
                    const float s = recip(rho[k] * P.it[k]);
                    collide<false>(P, k, fa[k], drho[k], rho[k], 0.0f, 0.0f,
                                   fmaf(F[k][0], s, ux), fmaf(F[k][1], s, uy), S[k]);
                } else {
                    collide(P, k, fa[k], drho[k], rho[k], F[k][0], F[k][1], ux, uy, S[k]);
                }
            }
        }

        // the values that cross a wavefront boundary in the x shift: lane 63
        // publishes the right-moving ones (1, 5, 8) for the next wavefront's
        // lane 0, lane 0 the left-moving ones (3, 6, 7) for the previous
        // wavefront's lane 63
        if constexpr (NW > 1 || FR) {
            if (l == 63) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    edge[wv][1][3 * k + 0] = Sprev[k][1];
                    edge[wv][1][3 * k + 1] = Uprev[k][1];
                    edge[wv][1][3 * k + 2] = S[k][8];
                }
            }
            if (l == 0) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    edge[wv][0][3 * k + 0] = Sprev[k][3];
                    edge[wv][0][3 * k + 1] = Uprev[k][2];
                    edge[wv][0][3 * k + 2] = S[k][7];
                }
            }
        }
        // every collision of row c is done: the ring row of c - 2 is free and
        // the edge values are visible
        wg_sync<(NW > 1 || FR)>();
        // neighbouring wavefronts of the x shift: inside the strip, or, in
        // full-row mode, around the group's row (its last wavefront's right
        // neighbour is its first)
        const int wl = FR ? (wv == w0 ? w0 + gk - 1 : wv - 1) : (wv > 0 ? wv - 1 : 0);
        const int wr = FR ? (wv == w0 + gk - 1 ? w0 : wv + 1) : (wv < NW - 1 ? wv + 1 : NW - 1);
        const bool takel = FR ? l == 0 : NW > 1 && l == 0 && wv > 0;
        const bool taker = FR ? l == 63 : NW > 1 && l == 63 && wv < NW - 1;
        LDS_CHECK(wl >= 0 && wl < NW && wr >= 0 && wr < NW && wv < NW);

        // stream into output row o = c - 1; the first two iterations have no
        // output row yet and write nothing
        {
            const int o = cc.r - 1;
            const bool st = outl && it >= 2;
            const uint32_t xo = (uint32_t)X;
            const uint32_t off4 = st ? (uint32_t)o * frowb + xo * 16u : DROP;
            const uint32_t off2 = st ? (uint32_t)o * frowb + xo * 8u : DROP;
            const uint32_t roff = st && ovr.wrho ? (uint32_t)o * rrowb + xo * 8u : DROP;
            float g[2][9];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                float l1 = from_left(Sprev[k][1]), l5 = from_left(Uprev[k][1]), l8 = from_left(S[k][8]);
                float r3 = from_right(Sprev[k][3]), r6 = from_right(Uprev[k][2]), r7 = from_right(S[k][7]);
                if constexpr (NW > 1 || FR) {
                    l1 = takel ? edge[wl][1][3 * k + 0] : l1;
                    l5 = takel ? edge[wl][1][3 * k + 1] : l5;
                    l8 = takel ? edge[wl][1][3 * k + 2] : l8;
                    r3 = taker ? edge[wr][0][3 * k + 0] : r3;
                    r6 = taker ? edge[wr][0][3 * k + 1] : r6;
                    r7 = taker ? edge[wr][0][3 * k + 2] : r7;
                }
                g[k][0] = Sprev[k][0];
                g[k][1] = l1;
                g[k][3] = r3;
                g[k][2] = Uprev[k][0];
                g[k][5] = l5;
                g[k][6] = r6;
                g[k][4] = S[k][4];
                g[k][7] = r7;
                g[k][8] = l8;
            }
            // bounce-back next to a wall: a branch on the (uniform) row, so
            // that rows away from walls pay no selects
            if (walls && o == 0) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    g[k][2] = Sprev[k][4];
                    g[k][5] = Sprev[k][7];
                    g[k][6] = Sprev[k][8];
                }
            }
            if (walls && o == ny - 1) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    g[k][4] = Sprev[k][2];
                    g[k][7] = Sprev[k][5];
                    g[k][8] = Sprev[k][6];
                }
            }
            // component A fills planes 0, 1 and the first lane of plane 2;
            // component B the rest of plane 2, plane 3 and the float2 plane
            bstore4(g[0][0], g[0][1], g[0][2], g[0][3], fout, off4, 0u);
            bstore4(g[0][4], g[0][5], g[0][6], g[0][7], fout, off4, 16u * pb);
            bstore4(g[0][8], g[1][0], g[1][1], g[1][2], fout, off4, 32u * pb);
            bstore4(g[1][3], g[1][4], g[1][5], g[1][6], fout, off4, 48u * pb);
            bstore2(g[1][7], g[1][8], fout, off2, 64u * pb);
            // uniform: no sums when no densities are written
            if (ovr.wrho) bstore2(sum9(g[0]), sum9(g[1]), rout, roff, 0u);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            Uprev[k][0] = Sprev[k][2];
            Uprev[k][1] = Sprev[k][5];
            Uprev[k][2] = Sprev[k][6];
        }
        {
            // the slot of row c - 2 takes row c + 3 (after the last row too,
            // where it is simply not read)
            const int freed = slot[0];
#pragma unroll
            for (int d = 0; d < RR - 1; ++d) slot[d] = slot[d + 1];
            slot[RR - 1] = freed;
            ring_store(freed, rnext, fn);
            wg_sync<(NW > 1 || FR)>();  // the new ring row and the consumed edges before reuse
            advance(cr);
        }
        advance(cc);
    };
    const int nit = ho + 2;
    for (int it = 0; it < nit; it += 4) {
        row(it, nit, fa, fd, Sa, Sb);
        if (it + 1 < nit) row(it + 1, nit, fb, fa, Sb, Sa);
        if (it + 2 < nit) row(it + 2, nit, fc, fb, Sa, Sb);
        if (it + 3 < nit) row(it + 3, nit, fd, fc, Sb, Sa);
    }
    }  // segments
}

// ------------------------------------------------------------------ two steps per pass
// Two time steps in one pass over the lattice (temporal blocking) as a
// pipeline of two wavefronts per one-strip workgroup.  Wavefront 0 (stage A)
// is the single step above: it loads f(t), collides row c1 and pulls output
// row o1 = c1 - 1 of f(t+1), which goes to LDS instead of memory, together
// with its densities (the sums the step would write as rho(t + 1)) in a
// second density ring.  Wavefront 1 (stage B) advances f(t+1) the same way
// from those rows, one barrier phase and two rows behind, and writes f(t+2).
// Every node goes through exactly the operations of two single steps, in
// the same order, so the result equals two launches of k_fused_step bit for
// bit; the populations cross HBM once per two steps.  Each stage has the
// registers of one wavefront to itself, and the two wavefronts of a SIMD
// (two workgroups per SIMD pair) overlap one stage's memory waits with the
// other's arithmetic.
// Lane L of either wavefront owns lattice column X0 - 6 + L: stage A loads
// lanes 0 .. wo + 11, collides lanes 2 .. wo + 9 and produces f(t+1) for
// lanes 3 .. wo + 8; stage B collides lanes 5 .. wo + 6 and writes lanes
// 6 .. wo + 5, the segment's wo <= SW2 output columns.  A segment of ho
// output rows takes ho + 9 phases, one barrier each.  In phase p, stage A
// collides row Y0 - 4 + p (loading Y0 - 1 + p) and, from p = 2 on, writes
// row o1(p) = Y0 - 5 + p of f(t+1) to slot p mod 4 and its densities to ring
// slot p mod 6; stage B collides row o1(p - 3) (p >= 7), whose stencil rows
// o1(p - 5) .. o1(p - 1) were written in earlier phases, and from p = 9 on
// writes row Y0 - 9 + p of f(t+2).  Stage B never reads a slot stage A
// writes in the same phase, and the barrier that ends a phase orders the
// rest.

// Density ring of the two-step kernel: NS row slots of a one-wavefront
// strip's columns (column j: lattice column X0 - 6 + j).  A slot holds one
// row of the three fields with the two components side by side, so that all
// reads of a row by one lane's stencil lie within 2 KiB after the first:
// one address register per slot and immediate offsets, with no address
// arithmetic per read.
template <int NS_>
struct RingP {
    static constexpr int NS = NS_;
    static constexpr int W = RingW<1, 0>::W;
    struct Row {
        float2 psi[W];
        float2 rho[W];
        float2 dev[W];  // density deviations (own-node term of the collision)
    };
    Row row[NS];
};

// accessor into a packed ring: slot[dy + 2] is the slot of lattice row
// c + dy, cb the ring column of the stencil's left edge (centre - HALO)
template <class RT>
struct RingAccP {
    const RT &R;
    const int *slot;
    int cb;
    __device__ float psi(int k, int dx, int dy) const
    {
        const float2 v = R.row[slot[dy + HALO]].psi[cb + HALO + dx];
        return k ? v.y : v.x;
    }
    __device__ float rho(int k, int dx, int dy) const
    {
        const float2 v = R.row[slot[dy + HALO]].rho[cb + HALO + dx];
        return k ? v.y : v.x;
    }
};

template <int FS>
__global__ __launch_bounds__(128, 2) void k_fused_step2(const KInst *__restrict__ insts,
                                                        const int4 *__restrict__ segs,
                                                        const int *__restrict__ first, int par)
{
    constexpr int RB6 = 6;
    __shared__ RingP<RR> RA;          // densities of f(t): stage A only
    __shared__ RingP<RB6> RB;         // densities of f(t+1)
    __shared__ float4 FQ[4][4][64];   // f(t+1) rows: four float4 planes per slot
    __shared__ float2 FQ2[4][64];     // and the float2 plane
    const int L = (int)threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int sg_begin = first[blockIdx.x], sg_end = first[blockIdx.x + 1];
    for (int sg = sg_begin; sg < sg_end; ++sg) {
    const int4 t = segs[sg];
    const KInst &G = insts[t.x];
    const KPar P = kpar(G);
    const int X0 = t.y, Y0 = t.z, wo = t.w & 0xffff, ho = (int)((uint32_t)t.w >> 16);
    const int nx = G.nx, ny = G.ny, walls = G.walls;
    const uint32_t pb = (uint32_t)G.pitch;
    const uint32_t frowb = 72u * pb;
    constexpr uint32_t DROP = 0x80000000u;
    constexpr int H2 = 2 * (HALO + 1);  // columns left of the output for the two stages
    const int X = X0 - H2 + L;
    const int cl = L;                        // ring column of this lane
    // left edge of the stencil (never left of the ring): the lane's centre
    // is cb + HALO, which differs from cl only on lanes 0 and 1, whose
    // collisions no output uses
    const int cb = cl < HALO ? 0 : cl - HALO;
    LDS_CHECK((cb + 2 * HALO < RingP<RR>::W));
    const int nph = ho + 9;  // phases of the segment

    struct Cursor {
        int r, i;
    };
    auto cursor = [&](int r) {
        if (walls) return Cursor{r, (r >= 0 && r < ny) ? r : -1};
        return Cursor{r, wrapi(r, ny)};
    };
    auto advance = [&](Cursor &q) {
        ++q.r;
        if (walls)
            q.i = (q.r >= 0 && q.r < ny) ? q.r : -1;
        else
            q.i = (q.i + 1 == ny) ? 0 : q.i + 1;
    };
    // ring row `slot` of R from a row's populations (as ring_store of the
    // single step: the same sums, the wall's densities beyond a wall)
    auto ring_store = [&](auto &R, int slot, int ri, const float q[2][9]) {
        LDS_CHECK(slot >= 0 && slot < R.NS);
        const float da = sum9(q[0]), db = sum9(q[1]);
        float ra = P.rho_ref[0] + da, rb = P.rho_ref[1] + db;
        float pa = psi_of(P, ra), pbv = psi_of(P, rb);
        if (ri < 0) {  // a row beyond a wall (uniform): no selects on the other rows
            ra = P.rho_wall[0];
            rb = P.rho_wall[1];
            pa = P.psi_wall[0];
            pbv = P.psi_wall[1];
        }
        R.row[slot].rho[cl] = make_float2(ra, rb);
        R.row[slot].psi[cl] = make_float2(pa, pbv);
        R.row[slot].dev[cl] = make_float2(da, db);
    };
    // collision of one row of populations fa with ring R (slots sl of rows
    // c - 2 .. c + 2), into S
    auto collide_row = [&](const auto &R, const int (&sl)[RR], const float (&fa)[2][9],
                           float (&S)[2][9]) {
        using RT = typename std::remove_cv<typename std::remove_reference<decltype(R)>::type>::type;
        float F[2][2];
        stencil_force(P, RingAccP<RT>{R, sl, cb}, F);
        const float2 dv = R.row[sl[HALO]].dev[cb + HALO], rv = R.row[sl[HALO]].rho[cb + HALO];
        float drho[2] = {dv.x, dv.y}, rho[2] = {rv.x, rv.y}, jx[2], jy[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            float mx, my;
            mom9(fa[k], mx, my);
            jx[k] = FS ? mx : fmaf(0.5f, F[k][0], mx);
            jy[k] = FS ? my : fmaf(0.5f, F[k][1], my);
        }
        float ux, uy;
        common_velocity(P, rho, jx, jy, ux, uy);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if constexpr (FS) {
                const float s = recip(rho[k] * P.it[k]);
                collide<false>(P, k, fa[k], drho[k], rho[k], 0.0f, 0.0f,
                               fmaf(F[k][0], s, ux), fmaf(F[k][1], s, uy), S[k]);
            } else {
                collide(P, k, fa[k], drho[k], rho[k], F[k][0], F[k][1], ux, uy, S[k]);
            }
        }
    };
    // pull of output row o (its lattice row number; walls decide
    // bounce-back) from the collided rows o - 1 (U: upward populations),
    // o (Sp) and o + 1 (S): g[k][i] = f_{k,i}(x, o) after streaming
    auto pull = [&](int o, const float (&Sp)[2][9], const float (&U)[2][3], const float (&S)[2][9],
                    float (&g)[2][9]) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            g[k][0] = Sp[k][0];
            g[k][1] = from_left(Sp[k][1]);
            g[k][3] = from_right(Sp[k][3]);
            g[k][2] = U[k][0];
            g[k][5] = from_left(U[k][1]);
            g[k][6] = from_right(U[k][2]);
            g[k][4] = S[k][4];
            g[k][7] = from_right(S[k][7]);
            g[k][8] = from_left(S[k][8]);
        }
        // bounce-back next to a wall: a branch on the (uniform) row, so that
        // rows away from walls pay no selects
        if (walls && o == 0) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                g[k][2] = Sp[k][4];
                g[k][5] = Sp[k][7];
                g[k][6] = Sp[k][8];
            }
        }
        if (walls && o == ny - 1) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                g[k][4] = Sp[k][2];
                g[k][7] = Sp[k][5];
                g[k][8] = Sp[k][6];
            }
        }
    };

    if (wv == 0) {
        // ---------------------------------------------------------- stage A
        const __amdgpu_buffer_rsrc_t fin = make_rsrc(G.f[par], (uint32_t)ny * frowb);
        const bool needf = L <= wo + 2 * H2 - 1;
        const uint32_t xl = (uint32_t)wrapi(X, nx);
        const uint32_t xf16 = needf ? xl * 16u : DROP, xf8 = needf ? xl * 8u : DROP;
        auto load_f = [&](int ri, bool live, float f[2][9]) {
            const uint32_t ro = (uint32_t)(ri < 0 ? 0 : ri) * frowb;
            const uint32_t o16 = live ? ro + xf16 : DROP, o8 = live ? ro + xf8 : DROP;
            float q[18];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const u32x4 v = bload4(fin, o16, (uint32_t)g * 16u * pb);
                q[4 * g + 0] = __uint_as_float(v.x);
                q[4 * g + 1] = __uint_as_float(v.y);
                q[4 * g + 2] = __uint_as_float(v.z);
                q[4 * g + 3] = __uint_as_float(v.w);
            }
            const u32x2 w = bload2(fin, o8, 64u * pb);
            q[16] = __uint_as_float(w.x);
            q[17] = __uint_as_float(w.y);
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int i = 0; i < 9; ++i) f[k][i] = q[9 * k + i];
        };
        // ring rows Y0 - 6 .. Y0 - 2, populations of rows Y0 - 4 .. Y0 - 2
        int slA[RR];
        Cursor cr = cursor(Y0 - 6);  // next row to load
        float fa[2][9], fb[2][9], fc[2][9], fd[2][9];
        {
            float t0[2][9], t1[2][9];
            int ri[RR];
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                ri[q] = cr.i;
                slA[q] = q;
                advance(cr);
            }
            load_f(ri[0], true, t0);
            load_f(ri[1], true, t1);
            load_f(ri[2], true, fa);
            load_f(ri[3], true, fb);
            load_f(ri[4], true, fc);
            ring_store(RA, 0, ri[0], t0);
            ring_store(RA, 1, ri[1], t1);
            ring_store(RA, 2, ri[2], fa);
            ring_store(RA, 3, ri[3], fb);
            ring_store(RA, 4, ri[4], fc);
        }
        wg_sync<false>();  // ring A is this wavefront's alone
        Cursor o1c = cursor(Y0 - 5);
        float Sa[2][9], Sb[2][9], U[2][3];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
#pragma unroll
            for (int i = 0; i < 9; ++i) Sb[k][i] = 0.0f;
            U[k][0] = U[k][1] = U[k][2] = 0.0f;
        }
        auto phase = [&](int p, float (&fa)[2][9], float (&fn)[2][9], float (&S)[2][9],
                         const float (&Sp)[2][9]) {
            const int rnext = cr.i;
            load_f(rnext, p <= ho + 6, fn);  // rows beyond Y0 + ho + 5 are not needed
            collide_row(RA, slA, fa, S);
            if (p >= 2) {
                float g[2][9];
                pull(o1c.r, Sp, U, S, g);
                const int fs = p & 3;
                FQ[fs][0][L] = make_float4(g[0][0], g[0][1], g[0][2], g[0][3]);
                FQ[fs][1][L] = make_float4(g[0][4], g[0][5], g[0][6], g[0][7]);
                FQ[fs][2][L] = make_float4(g[0][8], g[1][0], g[1][1], g[1][2]);
                FQ[fs][3][L] = make_float4(g[1][3], g[1][4], g[1][5], g[1][6]);
                FQ2[fs][L] = make_float2(g[1][7], g[1][8]);
                ring_store(RB, p % RB6, o1c.i, g);
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                U[k][0] = Sp[k][2];
                U[k][1] = Sp[k][5];
                U[k][2] = Sp[k][6];
            }
            const int freed = slA[0];
#pragma unroll
            for (int d = 0; d < RR - 1; ++d) slA[d] = slA[d + 1];
            slA[RR - 1] = freed;
            ring_store(RA, freed, rnext, fn);
            advance(cr);
            advance(o1c);
            __syncthreads();  // f(t+1) row and densities published; stage B's reads done
        };
        for (int p = 0; p < nph; p += 4) {
            phase(p, fa, fd, Sa, Sb);
            if (p + 1 < nph) phase(p + 1, fb, fa, Sb, Sa);
            if (p + 2 < nph) phase(p + 2, fc, fb, Sa, Sb);
            if (p + 3 < nph) phase(p + 3, fd, fc, Sb, Sa);
        }
    } else {
        // ---------------------------------------------------------- stage B
        const __amdgpu_buffer_rsrc_t fout = make_rsrc(G.f[par ^ 1], (uint32_t)ny * frowb);
        const bool outl = (L >= H2) && (L < wo + H2);
        Cursor o2c = cursor(Y0 - 9);  // output row of phase p: Y0 - 9 + p
        float Sa[2][9], Sb[2][9], U[2][3];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
#pragma unroll
            for (int i = 0; i < 9; ++i) Sb[k][i] = 0.0f;
            U[k][0] = U[k][1] = U[k][2] = 0.0f;
        }
        // slB[d]: ring slot of row o1(p - 5 + d), i.e. (p - 5 + d) mod 6,
        // rotated by one each phase (as stage A's slots, so that the compiler
        // can carry each slot's LDS address from phase to phase)
        int slB[RB6];
#pragma unroll
        for (int d = 0; d < RB6; ++d) slB[d] = (d + 1) % RB6;
        auto phase = [&](int p, float (&S)[2][9], const float (&Sp)[2][9]) {
            if (p >= 7) {
                // collide row c2 = o1(p - 3), its populations in slot (p - 3) mod 4
                const int fs = (p - 3) & 3;
                float f2[2][9];
                {
                    const float4 a = FQ[fs][0][L], b = FQ[fs][1][L], c = FQ[fs][2][L], d = FQ[fs][3][L];
                    const float2 e = FQ2[fs][L];
                    const float q[18] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x,
                                         c.y, c.z, c.w, d.x, d.y, d.z, d.w, e.x, e.y};
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int i = 0; i < 9; ++i) f2[k][i] = q[9 * k + i];
                }
                int sl[RR];  // ring slots of rows c2 - 2 .. c2 + 2 = o1(p - 5) .. o1(p - 1)
#pragma unroll
                for (int d = 0; d < RR; ++d) {
                    sl[d] = slB[d];
                    LDS_CHECK(sl[d] == (p - 5 + d) % RB6);
                }
                collide_row(RB, sl, f2, S);
                if (p >= 9) {
                    float g[2][9];
                    pull(o2c.r, Sp, U, S, g);
                    const uint32_t xo = (uint32_t)X;
                    const uint32_t off4 = outl ? (uint32_t)o2c.r * frowb + xo * 16u : DROP;
                    const uint32_t off2 = outl ? (uint32_t)o2c.r * frowb + xo * 8u : DROP;
                    bstore4(g[0][0], g[0][1], g[0][2], g[0][3], fout, off4, 0u);
                    bstore4(g[0][4], g[0][5], g[0][6], g[0][7], fout, off4, 16u * pb);
                    bstore4(g[0][8], g[1][0], g[1][1], g[1][2], fout, off4, 32u * pb);
                    bstore4(g[1][3], g[1][4], g[1][5], g[1][6], fout, off4, 48u * pb);
                    bstore2(g[1][7], g[1][8], fout, off2, 64u * pb);
                }
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    U[k][0] = Sp[k][2];
                    U[k][1] = Sp[k][5];
                    U[k][2] = Sp[k][6];
                }
            }
            const int oldest = slB[0];
#pragma unroll
            for (int d = 0; d < RB6 - 1; ++d) slB[d] = slB[d + 1];
            slB[RB6 - 1] = oldest;
            advance(o2c);
            __syncthreads();  // the end of the phase (stage A's next rows may now overwrite)
        };
        for (int p = 0; p < nph; p += 2) {
            phase(p, Sa, Sb);
            if (p + 1 < nph) phase(p + 1, Sb, Sa);
        }
    }
    }  // segments
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
    stage_tile(P, P.rho[par], t.y, t.z, T);
    __syncthreads();
    const int lx = (int)(threadIdx.x % TX), ly = (int)(threadIdx.x / TX);
    const int x = t.y + lx, y = t.z + ly;
    if (x >= P.nx || y >= P.ny) return;
    float f[2][9];
    load_node(P, P.f[par], x, y, f);
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
    const int64_t N = (int64_t)P.nx * P.ny, n = (int64_t)y * P.nx + x;
    for (int j = 0; j < 18; ++j) fout[(int64_t)j * N + n] = P.f[par][fidx(P, j, x, y)];
}

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
    const int64_t N = (int64_t)P.nx * P.ny, n = (int64_t)y * P.nx + x;
    for (int j = 0; j < 18; ++j) P.f[par][fidx(P, j, x, y)] = fin[(int64_t)j * N + n];
}

// ------------------------------------------------------------------ forces only
// densities of lbm_forces go to rho[par ^ 1], which the next step overwrites
__global__ void k_rho_in(const KInst *__restrict__ insts, int inst, int par, const float *rho_in)
{
    const KInst &P = insts[inst];
    const int64_t N = (int64_t)P.nx * P.ny;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < 2 * N;
         n += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(n / N);
        const int64_t m = n % N;
        const int y = (int)(m / P.nx), x = (int)(m % P.nx);
        P.rho[par ^ 1][ridx(P, k, x, y)] = rho_in[n];
    }
}

__global__ __launch_bounds__(NTHREADS) void k_forces(const KInst *__restrict__ insts,
                                                      const int4 *__restrict__ tiles, int inst,
                                                      int par, float *__restrict__ Fout)
{
    __shared__ Tile T;
    const int4 t = tiles[blockIdx.x];
    if (t.x != inst) return;  // uniform per block: no thread reaches the barrier below
    const KInst &P = insts[t.x];
    stage_tile(P, P.rho[par ^ 1], t.y, t.z, T, true);
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
// One block per (instance, row) for the row passes, one per instance for the
// final passes; every quantity is accumulated in FP64 in a fixed order (a
// per-thread strided loop, then block_reduce: wavefront butterflies and one
// LDS pass in wavefront order), so results are bitwise reproducible.
constexpr int RT = 256;  // threads of reduction blocks

// per-thread partials of the rows [row0, row0 + nrow) of quantity q
__device__ __forceinline__ double rows_acc(const double *part, int row0, int nrow, int q, int op)
{
    double a = op == RED_SUM ? 0.0 : op == RED_MAX ? -INFINITY : INFINITY;
    for (int r = threadIdx.x; r < nrow; r += RT) a = red_op(op, a, part[(int64_t)(row0 + r) * NQR + q]);
    return a;
}

// pass 1 per row: masses and population momentum from the populations;
// total j, row sum of u_x, max |u|, extrema of rho_A, non-finite count.
__global__ __launch_bounds__(RT) void k_red_rows1(const KInst *__restrict__ insts,
                                                   const int2 *__restrict__ rows, int par,
                                                   double *__restrict__ part)
{
    __shared__ double s[11 * (RT / 64)];
    const int2 r = rows[blockIdx.x];
    const KInst &P = insts[r.x];
    const int y = r.y;
    const int64_t pl = P.plane;
    double mA = 0, mB = 0, px = 0, py = 0, jx = 0, jy = 0, su = 0, umax = 0;
    double amax = -INFINITY, amin = INFINITY, bad = 0;
    for (int x = threadIdx.x; x < P.nx; x += RT) {
        float f[2][9];
        load_node(P, P.f[par], x, y, f);
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
    double v[11] = {mA, mB, px, py, jx, jy, su, umax, amax, amin, bad};
    constexpr int op[11] = {RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM,
                            RED_SUM, RED_MAX, RED_MAX, RED_MIN, RED_SUM};
    block_reduce<RT>(v, op, s);
    if (threadIdx.x == 0) {
        double *o = part + (int64_t)blockIdx.x * NQR;
        for (int q = 0; q < 11; ++q) o[q] = v[q];
    }
}

// final pass 1: one block per instance
__global__ __launch_bounds__(RT) void k_red_final1(const KInst *__restrict__ insts,
                                                    const int *__restrict__ row0s,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ res)
{
    __shared__ double s[11 * (RT / 64)];
    const int inst = blockIdx.x;
    const KInst &P = insts[inst];
    const int row0 = row0s[inst], nrow = P.ny;
    const double N = (double)P.nx * (double)P.ny;
    double *R = res + (int64_t)inst * NRES;
    constexpr int op[11] = {RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM,
                            RED_SUM, RED_MAX, RED_MAX, RED_MIN, RED_SUM};
    double v[11];
    for (int q = 0; q < 11; ++q) v[q] = rows_acc(part, row0, nrow, q, op[q]);
    block_reduce<RT>(v, op, s);
    if (threadIdx.x == 0) {
        R[RES_MASSA] = N * (double)P.rho_ref[0] + v[0];
        R[RES_MASSB] = N * (double)P.rho_ref[1] + v[1];
        R[RES_PX] = v[2];
        R[RES_PY] = v[3];
        R[RES_JX] = v[4];
        R[RES_JY] = v[5];
        R[RES_Q] = v[6] / (double)P.nx;
        R[RES_UMAX] = v[7];
        R[RES_AMAX] = v[8];
        R[RES_AMIN] = v[9];
        R[RES_BAD] = v[10];
    }
}

// pass 2 per row: weights w = rho_A - rho_A,min for the droplet area and the
// periodic circular mean of its position.
__global__ __launch_bounds__(RT) void k_red_rows2(const KInst *__restrict__ insts,
                                                   const int2 *__restrict__ rows,
                                                   const double *__restrict__ res,
                                                   double *__restrict__ part)
{
    __shared__ double s[3 * (RT / 64)];
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
    double v[3] = {w, wc, ws};
    constexpr int op[3] = {RED_SUM, RED_SUM, RED_SUM};
    block_reduce<RT>(v, op, s);
    if (threadIdx.x == 0) {
        double *o = part + (int64_t)blockIdx.x * NQR;
        o[0] = v[0];
        o[1] = v[1];
        o[2] = v[2];
    }
}

__global__ __launch_bounds__(RT) void k_red_final2(const KInst *__restrict__ insts,
                                                    const int *__restrict__ row0s,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ res)
{
    __shared__ double s[5 * (RT / 64)];
    const int inst = blockIdx.x;
    const KInst &P = insts[inst];
    const int row0 = row0s[inst], nrow = P.ny;
    double *R = res + (int64_t)inst * NRES;
    // x sums of the rows, then y moments: row weights times cos/sin of the row angle
    double yc = 0, ys = 0;
    const double k = 2.0 * M_PI / (double)P.ny;
    for (int rr = threadIdx.x; rr < nrow; rr += RT) {
        double sn, cs;
        sincos(k * rr, &sn, &cs);
        const double v = part[(int64_t)(row0 + rr) * NQR + 0];
        yc += v * cs;
        ys += v * sn;
    }
    double v[5] = {rows_acc(part, row0, nrow, 0, RED_SUM), rows_acc(part, row0, nrow, 1, RED_SUM),
                   rows_acc(part, row0, nrow, 2, RED_SUM), yc, ys};
    constexpr int op[5] = {RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_SUM};
    block_reduce<RT>(v, op, s);
    if (threadIdx.x == 0) {
        const double W = v[0], Wc = v[1], Ws = v[2], Yc = v[3], Ys = v[4];
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
    __shared__ double s[4 * (RT / 64)];
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
    double v[4] = {pin, nin, pout, nout};
    constexpr int op[4] = {RED_SUM, RED_SUM, RED_SUM, RED_SUM};
    block_reduce<RT>(v, op, s);
    if (threadIdx.x == 0) {
        double *o = part + (int64_t)blockIdx.x * NQR;
        o[0] = v[0];
        o[1] = v[1];
        o[2] = v[2];
        o[3] = v[3];
    }
}

__global__ __launch_bounds__(RT) void k_red_final3(const KInst *__restrict__ insts,
                                                    const int *__restrict__ row0s,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ res)
{
    __shared__ double s[4 * (RT / 64)];
    const int inst = blockIdx.x;
    const KInst &P = insts[inst];
    const int row0 = row0s[inst], nrow = P.ny;
    double *R = res + (int64_t)inst * NRES;
    double v[4];
    constexpr int op[4] = {RED_SUM, RED_SUM, RED_SUM, RED_SUM};
    for (int q = 0; q < 4; ++q) v[q] = rows_acc(part, row0, nrow, q, RED_SUM);
    block_reduce<RT>(v, op, s);
    if (threadIdx.x == 0) {
        const double pin = v[0], nin = v[1], pout = v[2], nout = v[3];
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
// each thread moves CPT 16-byte vectors, all loads issued before the stores
// (one per thread in 256-thread blocks was the fastest shape measured on
// MI355X, ahead of 4 or 8 per thread and of grid-stride loops)
constexpr int CPT = 1;
__global__ __launch_bounds__(256) void k_copy(float4 *__restrict__ dst,
                                              const float4 *__restrict__ src, int64_t n4)
{
    const int64_t base = (int64_t)blockIdx.x * 256 * CPT + threadIdx.x;
    float4 v[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int64_t i = base + (int64_t)j * 256;
        if (i < n4) v[j] = src[i];
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int64_t i = base + (int64_t)j * 256;
        if (i < n4) dst[i] = v[j];
    }
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
    k_density<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, 0);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_density(const Dev &d, int par, hipStream_t st)
{
    k_density<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, par);
    LAUNCH_CHECK();
    return hipSuccess;
}

template <int FS, int FR>
static hipError_t launch_fused(const Dev &d, int par, const StepOvr &o, hipStream_t st)
{
    switch (d.nw) {
    case 1: k_fused_step<1, FS, FR><<<d.nwg, 64, 0, st>>>(d.insts, d.strips, d.first, par, o); break;
    case 2: k_fused_step<2, FS, FR><<<d.nwg, 128, 0, st>>>(d.insts, d.strips, d.first, par, o); break;
    case 4: k_fused_step<4, FS, FR><<<d.nwg, 256, 0, st>>>(d.insts, d.strips, d.first, par, o); break;
    case 8: k_fused_step<8, FS, FR><<<d.nwg, 512, 0, st>>>(d.insts, d.strips, d.first, par, o); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step2(const Dev &d, int par, hipStream_t st)
{
    if (d.nw != 1 || d.fr) return hipErrorInvalidValue;
    if (d.forcing)
        k_fused_step2<1><<<d.nwg, 128, 0, st>>>(d.insts, d.strips, d.first, par);
    else
        k_fused_step2<0><<<d.nwg, 128, 0, st>>>(d.insts, d.strips, d.first, par);
    return hipGetLastError();
}

hipError_t launch_step_ovr(const Dev &d, int par, const StepOvr &o, hipStream_t st)
{
    if (d.forcing)
        return d.fr ? launch_fused<1, 1>(d, par, o, st) : launch_fused<1, 0>(d, par, o, st);
    return d.fr ? launch_fused<0, 1>(d, par, o, st) : launch_fused<0, 0>(d, par, o, st);
}

// count of out-of-range LDS indices the checked build has seen (and reset),
// or hipErrorNotSupported in the plain build
hipError_t lds_checks(unsigned int *bad, hipStream_t st)
{
#ifdef LBM_CHECK_LDS
    hipError_t e = hipMemcpyFromSymbolAsync(bad, HIP_SYMBOL(g_lds_bad), sizeof(unsigned int), 0,
                                            hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const unsigned int zero = 0;
    if (e == hipSuccess)
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_lds_bad), &zero, sizeof zero, 0,
                                   hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
#else
    (void)bad;
    (void)st;
    return hipErrorNotSupported;
#endif
}

hipError_t launch_step(const Dev &d, int par, hipStream_t st)
{
    return launch_step_ovr(d, par, StepOvr{-1, nullptr, nullptr, nullptr, 0}, st);
}

const char *step_kernel_name(int j)
{
    static const char *names[N_STEP_KERNELS] = {"k_fused_step"};
    return (j >= 0 && j < N_STEP_KERNELS) ? names[j] : "";
}

// kernel j of the step alone; it writes only the buffers of the next state
hipError_t launch_step_kernel(const Dev &d, int j, int par, hipStream_t st)
{
    (void)j;
    return launch_step(d, par, st);
}

hipError_t launch_fields(const Dev &d, int par, hipStream_t st)
{
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
    k_density<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, par);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_forces(const Dev &d, int inst, int par, const float *rho, float *F, hipStream_t st)
{
    k_rho_in<<<1024, 256, 0, st>>>(d.insts, inst, par, rho);
    LAUNCH_CHECK();
    k_forces<<<d.ntiles, NTHREADS, 0, st>>>(d.insts, d.tiles, inst, par, F);
    LAUNCH_CHECK();
    return hipSuccess;
}

// fields, then three row passes with their per-instance final passes; the
// per-row u_x sums (slot 6 of pass 1) stay untouched by passes 2 and 3.
hipError_t launch_observables(const Dev &d, int par, double margin, double *part, double *res,
                              hipStream_t st)
{
    hipError_t e = launch_fields(d, par, st);
    if (e != hipSuccess) return e;
    k_red_rows1<<<d.nrows, RT, 0, st>>>(d.insts, d.rows, par, part);
    LAUNCH_CHECK();
    k_red_final1<<<d.ninst, RT, 0, st>>>(d.insts, d.row0s, part, res);
    LAUNCH_CHECK();
    k_red_rows2<<<d.nrows, RT, 0, st>>>(d.insts, d.rows, res, part);
    LAUNCH_CHECK();
    k_red_final2<<<d.ninst, RT, 0, st>>>(d.insts, d.row0s, part, res);
    LAUNCH_CHECK();
    k_red_rows3<<<d.nrows, RT, 0, st>>>(d.insts, d.rows, res, margin, part);
    LAUNCH_CHECK();
    k_red_final3<<<d.ninst, RT, 0, st>>>(d.insts, d.row0s, part, res);
    LAUNCH_CHECK();
    return hipSuccess;
}

// The per-instance results as lbm_obs records, one thread per instance (the
// same assignments lbm_observables makes on the host).
__global__ void k_obs_pack(const double *__restrict__ res, int ninst, lbm_obs *__restrict__ out)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= ninst) return;
    const double *R = res + (int64_t)i * NRES;
    lbm_obs o;
    o.mass[0] = R[RES_MASSA];
    o.mass[1] = R[RES_MASSB];
    o.mom_raw[0] = R[RES_PX];
    o.mom_raw[1] = R[RES_PY];
    o.mom_bary[0] = R[RES_JX];
    o.mom_bary[1] = R[RES_JY];
    o.max_speed = R[RES_UMAX];
    o.rho_a_max = R[RES_AMAX];
    o.rho_a_min = R[RES_AMIN];
    o.flow_rate = R[RES_Q];
    o.R_eff = R[RES_R];
    o.cx = R[RES_CX];
    o.cy = R[RES_CY];
    o.p_in = R[RES_PIN];
    o.p_out = R[RES_POUT];
    o.dp = R[RES_DP];
    o.gamma = R[RES_GAMMA];
    o.width = R[RES_W];
    o.n_in = (int64_t)R[RES_NIN];
    o.n_out = (int64_t)R[RES_NOUT];
    o.finite = R[RES_BAD] == 0.0 && isfinite(R[RES_MASSA]) && isfinite(R[RES_MASSB]);
    out[i] = o;
}

hipError_t launch_obs_pack(const Dev &d, const double *res, lbm_obs *out, hipStream_t st)
{
    k_obs_pack<<<(d.ninst + 63) / 64, 64, 0, st>>>(res, d.ninst, out);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_copy(void *dst, const void *src, uint64_t nbytes, hipStream_t st)
{
    const int64_t n4 = (int64_t)(nbytes / 16);
    if (n4 > 0) {
        const int64_t nb = (n4 + 256 * CPT - 1) / (256 * CPT);
        if (nb > 0x7fffffff) return hipErrorInvalidValue;
        k_copy<<<(unsigned)nb, 256, 0, st>>>((float4 *)dst, (const float4 *)src, n4);
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
