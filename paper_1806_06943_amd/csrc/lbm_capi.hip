// C-ABI entry points (include/lbm.h): validation, workspace layout, context
// bookkeeping and HIP-graph replay of the step loop.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

constexpr int GRAPH_STEPS = 16;  // steps per captured graph (even: parity unchanged)
constexpr uint64_t ALIGN = 256;
constexpr int MIN_CHUNK = 2;     // smallest strip height the workspace is sized for
constexpr int DEFAULT_CHUNK = 16;
constexpr int MIN_WIDTH = 16;    // narrowest strip the workspace is sized for
constexpr int DEFAULT_WIDTH = SWO;

thread_local std::string g_init_error;

// Reduction scratch of lbm_observables_noalloc: FP64 row partials, per-instance
// results and the packed lbm_obs records of one call.  One copy per GPU,
// held until the process ends.  Host code never passes the array's name to
// a kernel or a copy: it uses the device address that hipGetSymbolAddress
// gives for the current device (scratch_address, resolved by lbm_init).
constexpr uint64_t SCRATCH_DOUBLES = (uint64_t)1 << 19;  // 4 MiB
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this GPU's scratch array (device dev must be current).
hipError_t scratch_address(int dev, double **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// doubles of scratch that lbm_observables_noalloc needs for this context
uint64_t noalloc_doubles(int nrows, int ninst)
{
    const uint64_t obs_words = (sizeof(lbm_obs) + 7) / 8;
    return (uint64_t)nrows * NQR + (uint64_t)ninst * (NRES + obs_words);
}

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

struct InstLayout {
    int32_t pitch;
    int64_t plane;       // floats per field plane
    int64_t fsize;       // floats per population buffer
    int64_t rsize;       // floats per density buffer
    uint64_t bytes;      // per-instance bytes (f0, f1, rho0, rho1, fields)
};

InstLayout inst_layout(const lbm_params &p)
{
    InstLayout L;
    L.pitch = (int32_t)align_up((uint64_t)p.nx, 64);
    // buffers end on a 256-byte boundary plus 64 floats, so that consecutive
    // buffers do not sit at the same offset modulo large powers of two
    L.plane = (int64_t)align_up((uint64_t)p.ny * L.pitch, 64) + 64;
    L.fsize = (int64_t)align_up((uint64_t)18 * p.ny * L.pitch, 64) + 64;
    L.rsize = (int64_t)align_up((uint64_t)2 * p.ny * L.pitch, 64) + 64;
    L.bytes = align_up((uint64_t)(2 * L.fsize + 2 * L.rsize + NFLD * L.plane) * sizeof(float), ALIGN);
    return L;
}

struct Layout {
    uint64_t off_insts, off_tiles, off_strips, off_rows, off_row0s, off_rho0p, off_part, off_res,
        off_data;
    std::vector<uint64_t> off_inst;
    std::vector<InstLayout> inst;
    int ntiles = 0, nrows = 0, max_strips = 0;
    uint64_t total = 0;
};

int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Work of the fused step: segments {inst, X0, Y0, wo | ho << 16} (both
// fields unsigned 16-bit: wo <= 506, ho <= 65535) and, per
// workgroup g, the range first[g] .. first[g+1]-1 of segments it advances.
struct StripPlan {
    std::vector<int4> segs;
    std::vector<int> first;
};

// Column strips of an instance for output width W (<= 506; a strip of W
// columns is one workgroup of strip_waves(W) wavefronts): ceil(nx / W)
// strips, either of balanced width (W not a multiple of 16) or starting at
// multiples of W (W a multiple of 16), so that every output row segment
// starts on a 64-byte boundary (the writes of neighbouring strips then never
// share a 64-byte block).  Returns {x0, width} pairs.
std::vector<int2> column_strips(int nx, int W)
{
    std::vector<int2> out;
    const int ns = ceil_div(nx, W);
    const bool aligned = W % 16 == 0;
    for (int sx = 0; sx < ns; ++sx) {
        const int x0 = aligned ? W * sx : (int)((int64_t)nx * sx / ns);
        const int x1 = aligned ? std::min(nx, W * (sx + 1)) : (int)((int64_t)nx * (sx + 1) / ns);
        out.push_back(make_int2(x0, x1 - x0));
    }
    return out;
}

constexpr int NXCD = 8;  // XCDs of the chip; workgroup g is dealt to XCD g % 8

// width and height of a segment in one word, as unsigned 16-bit fields (a
// height of 32768 or more sets the word's sign bit; the kernel decodes the
// word as unsigned)
int pack_wh(int wo, int ho) { return (int)((uint32_t)wo | ((uint32_t)ho << 16)); }

// Every segment of a plan fits a strip of nw wavefronts: its lanes cover
// the output columns, a collided halo column and HALO stencil columns on
// each side (the fused step assumes this for its LDS ring).
bool plan_fits(const StripPlan &P, int nw)
{
    for (const int4 &t : P.segs)
        if ((t.w & 0xffff) > 64 * nw - 2 - 2 * HALO) return false;
    return true;
}

// Uniform plan: rows split into ceil(ny / H) chunks of balanced height, one
// segment per workgroup.  The segments are ordered so that consecutive
// workgroup indices, which the hardware deals round-robin to the eight
// XCDs, give each XCD a contiguous run of neighbouring strips (shared halo
// columns and rows stay in that XCD's L2).
StripPlan plan_uniform(const lbm_params *p, int n, int H, int W)
{
    std::vector<int4> tab;
    for (int i = 0; i < n; ++i) {
        const std::vector<int2> cols = column_strips(p[i].nx, W);
        const int nc = ceil_div(p[i].ny, H);
        for (int c = 0; c < nc; ++c) {
            const int y0 = (int)((int64_t)p[i].ny * c / nc), y1 = (int)((int64_t)p[i].ny * (c + 1) / nc);
            for (const int2 &cs : cols) tab.push_back(make_int4(i, cs.x, y0, pack_wh(cs.y, y1 - y0)));
        }
    }
    const int T = (int)tab.size(), q = ceil_div(T, NXCD);
    StripPlan P;
    P.segs.reserve(T);
    for (int m = 0; m < q; ++m)
        for (int j = 0; j < NXCD; ++j)
            if (j * q + m < T) P.segs.push_back(tab[j * q + m]);
    for (int g = 0; g <= (int)P.segs.size(); ++g) P.first.push_back(g);
    return P;
}

// Balanced plan for G workgroups: every strip-row costs the same (one row
// of one workgroup), so each workgroup gets an equal share of all
// strip-rows, as runs of rows in one column strip (a share that crosses the
// end of a column becomes two or more segments).  The strip-rows are listed
// by horizontal band (eight bands of rows per instance), then instance,
// column and row; workgroup g takes share (g % 8) G/8 + g / 8, so each XCD
// advances one band: vertically neighbouring shares and the strips beside
// them meet in the same L2.
StripPlan plan_balanced(const lbm_params *p, int n, int W, int G)
{
    struct Unit {
        int inst, x0, wo, y0, y1;
    };
    std::vector<Unit> units;
    int64_t T = 0;
    for (int b = 0; b < NXCD; ++b)
        for (int i = 0; i < n; ++i) {
            const int y0 = (int)((int64_t)p[i].ny * b / NXCD), y1 = (int)((int64_t)p[i].ny * (b + 1) / NXCD);
            if (y1 <= y0) continue;
            for (const int2 &cs : column_strips(p[i].nx, W)) {
                units.push_back({i, cs.x, cs.y, y0, y1});
                T += y1 - y0;
            }
        }
    if (G > T) G = (int)T;
    if (G < 1) G = 1;
    // shares of logical index l: rows [T l / G, T (l + 1) / G) of the list
    std::vector<std::vector<int4>> share(G);
    size_t u = 0;
    int64_t ubase = 0;  // strip-rows before unit u
    for (int l = 0; l < G; ++l) {
        int64_t a = T * l / G;
        const int64_t b = T * (l + 1) / G;
        while (a < b) {
            while (ubase + (units[u].y1 - units[u].y0) <= a) {
                ubase += units[u].y1 - units[u].y0;
                ++u;
            }
            const Unit &U = units[u];
            const int64_t uend = ubase + (U.y1 - U.y0);
            const int64_t e = std::min(b, uend);
            const int ys = U.y0 + (int)(a - ubase), ho = (int)(e - a);
            share[l].push_back(make_int4(U.inst, U.x0, ys, pack_wh(U.wo, ho)));
            a = e;
        }
    }
    StripPlan P;
    const bool xcd = G % NXCD == 0;
    for (int g = 0; g < G; ++g) {
        const int l = xcd ? (g % NXCD) * (G / NXCD) + g / NXCD : g;
        P.first.push_back((int)P.segs.size());
        for (const int4 &sgm : share[l]) P.segs.push_back(sgm);
    }
    P.first.push_back((int)P.segs.size());
    return P;
}

// Full-row plans: lattices whose width is a multiple of 64 are advanced by
// groups of k = nx / 64 wavefronts covering whole rows.  0 if some instance
// is not of that form or wider than eight wavefronts, else the workgroup
// size in wavefronts (the smallest of 1, 2, 4, 8 that holds the widest).
int fullrow_waves(const lbm_params *p, int n)
{
    int kmax = 0;
    for (int i = 0; i < n; ++i) {
        if (p[i].nx % 64 != 0 || p[i].nx > 8 * 64) return 0;
        kmax = std::max(kmax, p[i].nx / 64);
    }
    return kmax <= 1 ? 1 : kmax <= 2 ? 2 : kmax <= 4 ? 4 : 8;
}

// Full-row plan for workgroups of NW wavefronts: every instance's rows cut
// into ceil(ny / H) chunks of balanced height, one group of k = nx / 64
// wavefronts each ({inst, first wavefront w0, Y0, k | ho << 16}).  Groups of
// equal height share workgroups (best fit, widest first), so every group of a
// workgroup runs the same number of rows; a workgroup's groups are its
// segment range.  Workgroups are then ordered like the uniform plan's, so
// that each XCD advances a run of neighbouring chunks.
StripPlan plan_fullrow(const lbm_params *p, int n, int H, int NW)
{
    struct Grp {
        int inst, k, y0, ho;
    };
    std::vector<Grp> grp;
    for (int i = 0; i < n; ++i) {
        const int nc = ceil_div(p[i].ny, H);
        for (int c = 0; c < nc; ++c) {
            const int y0 = (int)((int64_t)p[i].ny * c / nc), y1 = (int)((int64_t)p[i].ny * (c + 1) / nc);
            grp.push_back({i, p[i].nx / 64, y0, y1 - y0});
        }
    }
    // by height, then widest first (stable: instance and chunk order kept)
    std::stable_sort(grp.begin(), grp.end(), [](const Grp &a, const Grp &b) {
        return a.ho != b.ho ? a.ho > b.ho : a.k > b.k;
    });
    std::vector<std::vector<int4>> wgs;
    std::vector<int> fill;
    // open workgroups of the current height by free wavefronts
    std::vector<std::vector<int>> open(NW + 1);
    int cur_h = -1;
    for (const Grp &g : grp) {
        if (g.ho != cur_h) {
            for (auto &o : open) o.clear();
            cur_h = g.ho;
        }
        int w = -1;
        for (int f = g.k; f <= NW && w < 0; ++f)
            if (!open[f].empty()) {
                w = open[f].back();
                open[f].pop_back();
            }
        if (w < 0) {
            w = (int)wgs.size();
            wgs.emplace_back();
            fill.push_back(0);
        }
        wgs[w].push_back(make_int4(g.inst, fill[w], g.y0, pack_wh(g.k, g.ho)));
        fill[w] += g.k;
        if (fill[w] < NW) open[NW - fill[w]].push_back(w);
    }
    const int T = (int)wgs.size(), q = ceil_div(T, NXCD);
    StripPlan P;
    for (int m = 0; m < q; ++m)
        for (int j = 0; j < NXCD; ++j)
            if (j * q + m < T) {
                P.first.push_back((int)P.segs.size());
                for (const int4 &e : wgs[j * q + m]) P.segs.push_back(e);
            }
    P.first.push_back((int)P.segs.size());
    return P;
}

// segments a plan may need: uniform plans of any allowed width and height,
// balanced plans of up to MAX_WG workgroups
constexpr int MAX_WG = 8192;
int max_strips(const lbm_params *p, int n)
{
    int t = 0, cols = 0;
    for (int i = 0; i < n; ++i) {
        t += ceil_div(p[i].nx, MIN_WIDTH) * ceil_div(p[i].ny, MIN_CHUNK);
        cols += ceil_div(p[i].nx, MIN_WIDTH);
    }
    return std::max(t, MAX_WG + NXCD * cols);
}

Layout make_layout(const lbm_params *p, int n)
{
    Layout L;
    for (int i = 0; i < n; ++i) {
        L.ntiles += ((p[i].nx + TX - 1) / TX) * ((p[i].ny + TY - 1) / TY);
        L.nrows += p[i].ny;
    }
    L.max_strips = max_strips(p, n);
    uint64_t o = 0;
    L.off_insts = o; o = align_up(o + sizeof(KInst) * n, ALIGN);
    L.off_tiles = o; o = align_up(o + sizeof(int4) * L.ntiles, ALIGN);
    L.off_strips = o; o = align_up(o + (sizeof(int4) + sizeof(int)) * L.max_strips + sizeof(int), ALIGN);
    L.off_rows = o;  o = align_up(o + sizeof(int2) * L.nrows, ALIGN);
    L.off_row0s = o; o = align_up(o + sizeof(int) * n, ALIGN);
    L.off_rho0p = o; o = align_up(o + sizeof(double *) * n, ALIGN);
    L.off_part = o;  o = align_up(o + sizeof(double) * NQR * (uint64_t)L.nrows, ALIGN);
    L.off_res = o;   o = align_up(o + sizeof(double) * NRES * (uint64_t)n, ALIGN);
    L.off_data = o;
    for (int i = 0; i < n; ++i) {
        L.inst.push_back(inst_layout(p[i]));
        L.off_inst.push_back(o);
        o += L.inst.back().bytes;
    }
    L.total = o;
    return L;
}

bool finite_all(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

// returns an empty string when p is valid
std::string check_params(const lbm_params &p)
{
    char buf[256];
    if (p.nx < 1 || p.ny < 1) {
        snprintf(buf, sizeof buf, "lattice size must be >= 1 (got %d x %d)", p.nx, p.ny);
        return buf;
    }
    // byte offsets inside a population buffer must stay below 2^31
    if ((uint64_t)inst_layout(p).fsize * sizeof(float) >= ((uint64_t)1 << 31))
        return "lattice too large: a population buffer must stay below 2 GiB";
    if (p.walls != 0 && p.walls != 1) return "walls must be 0 or 1";
    if (p.forcing != LBM_FORCING_GUO && p.forcing != LBM_FORCING_SHIFT)
        return "forcing must be LBM_FORCING_GUO or LBM_FORCING_SHIFT";
    const double *d = &p.G_AB;
    if (!finite_all(d, (int)((sizeof(lbm_params) - offsetof(lbm_params, G_AB)) / sizeof(double))))
        return "parameters must be finite";
    for (int k = 0; k < 2; ++k)
        if (!(p.tau[k] > 0.5)) {
            snprintf(buf, sizeof buf, "tau[%d] = %g must exceed 0.5", k, p.tau[k]);
            return buf;
        }
    if (!(p.psi_rho0 > 0)) return "psi_rho0 must be positive";
    return "";
}

KInst make_kinst(const lbm_params &p, const InstLayout &L, char *base)
{
    KInst K;
    std::memset(&K, 0, sizeof K);
    float *b = (float *)base;
    K.f[0] = b;
    K.f[1] = b + L.fsize;
    K.rho[0] = b + 2 * L.fsize;
    K.rho[1] = b + 2 * L.fsize + L.rsize;
    K.fld = b + 2 * L.fsize + 2 * L.rsize;
    K.plane = L.plane;
    K.nx = p.nx;
    K.ny = p.ny;
    K.pitch = L.pitch;
    K.walls = p.walls;
    // merged weights of Eq. 8 per |e|^2 class {1, 2, 4, 5, 8}
    const double w[5] = {1.0 / 9.0, 1.0 / 36.0, 0.0, 0.0, 0.0};
    const double pw[5] = {4.0 / 63.0, 4.0 / 135.0, 1.0 / 180.0, 2.0 / 945.0, 1.0 / 15120.0};
    for (int k = 0; k < 2; ++k) {
        for (int c = 0; c < 5; ++c) K.cw[k][c] = (float)(p.G1[k] * w[c] + p.G2[k] * pw[c]);
        K.g[k][0] = (float)p.g[k][0];
        K.g[k][1] = (float)p.g[k][1];
        K.it[k] = (float)(1.0 / p.tau[k]);
        K.cf[k] = (float)((1.0 - 0.5 / p.tau[k]) / 36.0);
        K.rho_ref[k] = (float)p.rho_ref[k];
        K.rho_wall[k] = (float)p.rho_wall[k];
        K.psi_wall[k] = (float)(p.psi_rho0 * -std::expm1(-p.rho_wall[k] / p.psi_rho0));
        K.gpb[k] = (float)(0.5 * (p.G1[k] + p.G2[k]));
    }
    K.gr1 = (float)(p.G_AB / 9.0);
    K.gr2 = (float)(p.G_AB / 36.0);
    K.gab = (float)p.G_AB;
    K.rho0 = (float)p.psi_rho0;
    K.inv_rho0 = (float)(1.0 / p.psi_rho0);
    return K;
}

}  // namespace

struct lbm_ctx {
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;        // private stream used only for graph capture
    int n_inst = 0;
    std::vector<lbm_params> params;
    std::vector<KInst> hinst;
    Layout layout;
    Dev dev{};
    char *ws = nullptr;
    int par = 0;
    int64_t steps = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int chunk = DEFAULT_CHUNK;
    int width = DEFAULT_WIDTH;
    int balance = 0;   // workgroups per CU of a balanced plan (0: uniform chunks)
    int full_rows = 0; // 1: full-row plan of uniform chunks (lattice widths 64 k)
    int two_step = 0;  // 1: lbm_step advances two steps per launch (k_fused_step2)
    int ncu = 256;     // compute units of the device
    // rho[par] holds the densities of the state in f[par] (the plain step
    // does not write them; ensure_rho computes them when a kernel reads them)
    bool rho_ok[2] = {false, false};
    double *scratch = nullptr;  // this device's scratch array (lbm_observables_noalloc)
    std::string err;
};

#define CTX_CHECK(ctx)                                   \
    do {                                                 \
        if (!(ctx)) return LBM_EINVAL;                   \
    } while (0)

static int fail(lbm_ctx *ctx, int code, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    else
        g_init_error = msg;
    return code;
}

static int hip_fail(lbm_ctx *ctx, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, LBM_EHIP, m);
}

#define HIP_TRY(ctx, call)                                              \
    do {                                                                \
        hipError_t e__ = (call);                                        \
        if (e__ != hipSuccess) return hip_fail((ctx), e__, #call);      \
    } while (0)

extern "C" {

int lbm_workspace_bytes(const lbm_params *params, int32_t n_inst, uint64_t *bytes)
{
    if (!params || !bytes || n_inst < 1) return fail(nullptr, LBM_EINVAL, "null argument or n_inst < 1");
    for (int i = 0; i < n_inst; ++i) {
        std::string m = check_params(params[i]);
        if (!m.empty()) return fail(nullptr, LBM_EINVAL, "instance " + std::to_string(i) + ": " + m);
    }
    *bytes = make_layout(params, n_inst).total;
    return LBM_OK;
}

int lbm_init(lbm_ctx **out, const lbm_params *params, int32_t n_inst, const double *rhoA0,
             const double *rhoB0, void *workspace, uint64_t workspace_bytes, void *stream)
{
    if (!out || !params || !rhoA0 || !rhoB0 || !workspace || n_inst < 1)
        return fail(nullptr, LBM_EINVAL, "null argument or n_inst < 1");
    *out = nullptr;
    if ((uintptr_t)workspace % ALIGN)
        return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
    for (int i = 0; i < n_inst; ++i) {
        std::string m = check_params(params[i]);
        if (!m.empty()) return fail(nullptr, LBM_EINVAL, "instance " + std::to_string(i) + ": " + m);
        if (params[i].forcing != params[0].forcing)
            return fail(nullptr, LBM_EUNSUPPORTED, "all instances of a context need the same forcing");
    }
    Layout L = make_layout(params, n_inst);
    if (workspace_bytes < L.total)
        return fail(nullptr, LBM_EINVAL, "workspace too small: need " + std::to_string(L.total) +
                                              " bytes, got " + std::to_string(workspace_bytes));

    lbm_ctx *ctx = new lbm_ctx();
    ctx->stream = (hipStream_t)stream;
    ctx->n_inst = n_inst;
    ctx->params.assign(params, params + n_inst);
    ctx->layout = L;
    ctx->ws = (char *)workspace;

    // host tables
    std::vector<int4> tiles;
    std::vector<int2> rows;
    std::vector<int> row0s;
    std::vector<const double *> rho0p;
    for (int i = 0; i < n_inst; ++i) {
        const lbm_params &p = params[i];
        ctx->hinst.push_back(make_kinst(p, L.inst[i], ctx->ws + L.off_inst[i]));
        for (int y0 = 0; y0 < p.ny; y0 += TY)
            for (int x0 = 0; x0 < p.nx; x0 += TX) tiles.push_back(make_int4(i, x0, y0, 0));
        row0s.push_back((int)rows.size());
        for (int y = 0; y < p.ny; ++y) rows.push_back(make_int2(i, y));
        // FP64 initial densities are staged in the instance's field scratch
        rho0p.push_back((const double *)ctx->hinst.back().fld);
    }
    Dev &d = ctx->dev;
    d.insts = (KInst *)(ctx->ws + L.off_insts);
    d.tiles = (int4 *)(ctx->ws + L.off_tiles);
    d.rows = (int2 *)(ctx->ws + L.off_rows);
    d.row0s = (int *)(ctx->ws + L.off_row0s);
    d.part = (double *)(ctx->ws + L.off_part);
    d.res = (double *)(ctx->ws + L.off_res);
    d.strips = (int4 *)(ctx->ws + L.off_strips);
    d.first = (int *)(d.strips + L.max_strips);
    d.ninst = n_inst;
    d.ntiles = L.ntiles;
    d.nrows = L.nrows;
    {
        int dev = 0, ncu = 0;
        hipError_t de = hipGetDevice(&dev);
        if (de == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            ncu > 0)
            ctx->ncu = ncu;
        // this device's reduction scratch for lbm_observables_noalloc, with
        // the context's device current
        if (de == hipSuccess) de = scratch_address(dev, &ctx->scratch);
        if (de != hipSuccess) {
            std::string m = std::string("scratch address: ") + hipGetErrorString(de);
            delete ctx;
            return fail(nullptr, LBM_EHIP, m);
        }
    }
    StripPlan plan = plan_uniform(params, n_inst, ctx->chunk, ctx->width);
    if (!plan_fits(plan, strip_waves(ctx->width))) {
        delete ctx;
        return fail(nullptr, LBM_EINVAL, "strip wider than its workgroup");
    }
    const std::vector<int4> &strips = plan.segs;
    d.nstrips = (int)strips.size();
    d.nwg = (int)plan.first.size() - 1;
    d.nw = strip_waves(ctx->width);
    d.forcing = params[0].forcing;

    hipStream_t st = ctx->stream;
    auto bail = [&](hipError_t e, const char *what) {
        std::string m = std::string(what) + ": " + hipGetErrorString(e);
        delete ctx;
        return fail(nullptr, LBM_EHIP, m);
    };
    hipError_t e;
    if ((e = hipMemcpyAsync(d.insts, ctx->hinst.data(), sizeof(KInst) * n_inst,
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e, "copy instance table");
    if ((e = hipMemcpyAsync(d.tiles, tiles.data(), sizeof(int4) * tiles.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e, "copy tile table");
    if ((e = hipMemcpyAsync(d.strips, strips.data(), sizeof(int4) * strips.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e, "copy strip table");
    if ((e = hipMemcpyAsync(d.first, plan.first.data(), sizeof(int) * plan.first.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e, "copy workgroup table");
    if ((e = hipMemcpyAsync(d.rows, rows.data(), sizeof(int2) * rows.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e, "copy row table");
    if ((e = hipMemcpyAsync(d.row0s, row0s.data(), sizeof(int) * row0s.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e, "copy row offsets");
    const double **drho0p = (const double **)(ctx->ws + L.off_rho0p);
    if ((e = hipMemcpyAsync(drho0p, rho0p.data(), sizeof(double *) * n_inst,
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e, "copy density pointers");
    uint64_t off = 0;
    for (int i = 0; i < n_inst; ++i) {
        const uint64_t N = (uint64_t)params[i].nx * params[i].ny;
        double *dst = (double *)rho0p[i];
        if ((e = hipMemcpyAsync(dst, rhoA0 + off, N * sizeof(double), hipMemcpyHostToDevice, st)) !=
            hipSuccess)
            return bail(e, "copy initial rho_A");
        if ((e = hipMemcpyAsync(dst + N, rhoB0 + off, N * sizeof(double), hipMemcpyHostToDevice,
                                st)) != hipSuccess)
            return bail(e, "copy initial rho_B");
        off += N;
    }
    if ((e = launch_init(d, drho0p, st)) != hipSuccess) return bail(e, "init kernel");
    // the pageable host sources must stay valid until the copies complete
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e, "synchronise after init");
    ctx->rho_ok[0] = true;  // the init kernels write the densities of f[0]
    *out = ctx;
    return LBM_OK;
}

// Densities of the current state for the kernels that read rho[par]
// (observables, fields, the pressure tensor, a recorded window's first slot).
static int ensure_rho(lbm_ctx *ctx)
{
    if (ctx->rho_ok[ctx->par]) return LBM_OK;
    hipError_t e = launch_density(ctx->dev, ctx->par, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "density kernel");
    ctx->rho_ok[ctx->par] = true;
    return LBM_OK;
}

// n steps as launches on stream st: pairs of steps in one launch each in
// two-step mode (the last odd step alone), else one launch per step; every
// launch moves the state to the other buffer
static hipError_t launch_steps(lbm_ctx *ctx, int64_t n, int &par, hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (ctx->two_step)
        for (; n >= 2 && e == hipSuccess; n -= 2) {
            e = launch_step2(ctx->dev, par, st);
            par ^= 1;
        }
    for (; n > 0 && e == hipSuccess; --n) {
        e = launch_step(ctx->dev, par, st);
        par ^= 1;
    }
    return e;
}

static int step_eager(lbm_ctx *ctx, int64_t n, hipStream_t st)
{
    hipError_t e = launch_steps(ctx, n, ctx->par, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "step launch");
    return LBM_OK;
}

static int ensure_graph(lbm_ctx *ctx, int par)
{
    if (ctx->graph[par]) return LBM_OK;
    if (!ctx->cap) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
    int p = par;
    // GRAPH_STEPS is even: in either mode the graph ends on the parity it starts from
    hipError_t le = launch_steps(ctx, GRAPH_STEPS, p, ctx->cap);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(ctx->cap, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(ctx, le, "step launch during capture");
    }
    if (ee != hipSuccess) return hip_fail(ctx, ee, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&ctx->graph[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        ctx->graph[par] = nullptr;
        return hip_fail(ctx, ie, "hipGraphInstantiate");
    }
    return LBM_OK;
}

int lbm_step(lbm_ctx *ctx, int64_t nsteps)
{
    CTX_CHECK(ctx);
    if (nsteps < 0) return fail(ctx, LBM_EINVAL, "nsteps must be >= 0");
    hipStream_t st = ctx->stream;
    int64_t q = nsteps / GRAPH_STEPS, r = nsteps % GRAPH_STEPS;
    if (q > 0) {
        int rc = ensure_graph(ctx, ctx->par);
        if (rc != LBM_OK) return rc;
        for (int64_t i = 0; i < q; ++i) HIP_TRY(ctx, hipGraphLaunch(ctx->graph[ctx->par], st));
    }
    int rc = step_eager(ctx, r, st);
    if (rc != LBM_OK) return rc;
    if (nsteps > 0) ctx->rho_ok[0] = ctx->rho_ok[1] = false;
    ctx->steps += nsteps;
    return LBM_OK;
}

int lbm_prepare(lbm_ctx *ctx)
{
    CTX_CHECK(ctx);
    for (int par = 0; par < 2; ++par) {
        int rc = ensure_graph(ctx, par);
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}

int64_t lbm_steps_done(const lbm_ctx *ctx) { return ctx ? ctx->steps : -1; }

int lbm_observables(lbm_ctx *ctx, lbm_obs *out, double *ubar)
{
    CTX_CHECK(ctx);
    if (!out) return fail(ctx, LBM_EINVAL, "null output");
    int rc = ensure_rho(ctx);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    const double margin = 12.0;  // outer pressure shell starts 12 lattice units beyond R_eff
    hipError_t e = launch_observables(ctx->dev, ctx->par, margin, ctx->dev.part, ctx->dev.res, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "observable kernels");
    std::vector<double> res((size_t)NRES * ctx->n_inst);
    HIP_TRY(ctx, hipMemcpyAsync(res.data(), ctx->dev.res, sizeof(double) * res.size(),
                                hipMemcpyDeviceToHost, st));
    std::vector<double> part;
    if (ubar) {
        part.resize((size_t)NQR * ctx->dev.nrows);
        HIP_TRY(ctx, hipMemcpyAsync(part.data(), ctx->dev.part, sizeof(double) * part.size(),
                                    hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(ctx, hipStreamSynchronize(st));
    bool bad = false;
    int row = 0;
    for (int i = 0; i < ctx->n_inst; ++i) {
        const double *R = res.data() + (size_t)NRES * i;
        lbm_obs &o = out[i];
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
        o.finite = R[RES_BAD] == 0.0 && std::isfinite(R[RES_MASSA]) && std::isfinite(R[RES_MASSB]);
        if (!o.finite) bad = true;
        if (ubar) {
            const lbm_params &p = ctx->params[i];
            for (int y = 0; y < p.ny; ++y) ubar[row + y] = part[(size_t)(row + y) * NQR + 6] / p.nx;
        }
        row += ctx->params[i].ny;
    }
    if (bad) return fail(ctx, LBM_ENONFINITE, "non-finite density or velocity in the state");
    return LBM_OK;
}

int lbm_observables_noalloc(lbm_ctx *ctx, lbm_obs *out)
{
    CTX_CHECK(ctx);
    if (!out) return fail(ctx, LBM_EINVAL, "null output");
    const Dev &d = ctx->dev;
    if (noalloc_doubles(d.nrows, d.ninst) > SCRATCH_DOUBLES)
        return fail(ctx, LBM_EINVAL,
                    "lbm_observables_noalloc: " + std::to_string(d.nrows) + " rows and " +
                        std::to_string(d.ninst) + " instances need " +
                        std::to_string(noalloc_doubles(d.nrows, d.ninst) * 8) +
                        " bytes of scratch, more than its " + std::to_string(SCRATCH_DOUBLES * 8));
    int rc = ensure_rho(ctx);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    double *part = ctx->scratch;
    double *res = part + (uint64_t)d.nrows * NQR;
    lbm_obs *packed = (lbm_obs *)(res + (uint64_t)d.ninst * NRES);
    const double margin = 12.0;  // as lbm_observables
    hipError_t e = launch_observables(d, ctx->par, margin, part, res, st);
    if (e == hipSuccess) e = launch_obs_pack(d, res, packed, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "observable kernels");
    HIP_TRY(ctx, hipMemcpyAsync(out, packed, sizeof(lbm_obs) * d.ninst, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int i = 0; i < d.ninst; ++i)
        if (!out[i].finite) return fail(ctx, LBM_ENONFINITE, "non-finite density or velocity in the state");
    return LBM_OK;
}

static int check_inst(lbm_ctx *ctx, int32_t inst)
{
    if (inst < 0 || inst >= ctx->n_inst)
        return fail(ctx, LBM_EINVAL, "instance index out of range");
    return LBM_OK;
}

int lbm_fields(lbm_ctx *ctx, int32_t inst, float *rho_dev, float *u_dev)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (!rc) rc = ensure_rho(ctx);
    if (rc) return rc;
    hipError_t e = launch_fields(ctx->dev, ctx->par, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "fields kernels");
    e = launch_fields_out(ctx->dev, inst, rho_dev, u_dev, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "fields copy kernel");
    return LBM_OK;
}

int lbm_get_populations(lbm_ctx *ctx, int32_t inst, float *f_dev)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (!f_dev) return fail(ctx, LBM_EINVAL, "null output");
    hipError_t e = launch_export(ctx->dev, inst, ctx->par, f_dev, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "export kernel");
    return LBM_OK;
}

int lbm_set_populations(lbm_ctx *ctx, int32_t inst, const float *f_dev)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (!f_dev) return fail(ctx, LBM_EINVAL, "null input");
    hipError_t e = launch_import(ctx->dev, inst, ctx->par, f_dev, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "import kernel");
    ctx->rho_ok[ctx->par] = true;  // the import recomputes the densities of every instance
    ctx->steps = 0;
    return LBM_OK;
}

int lbm_forces(lbm_ctx *ctx, int32_t inst, const float *rho_dev, float *F_dev)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (!rho_dev || !F_dev) return fail(ctx, LBM_EINVAL, "null argument");
    ctx->rho_ok[ctx->par ^ 1] = false;  // the caller's densities go to rho[par ^ 1]
    hipError_t e = launch_forces(ctx->dev, inst, ctx->par, rho_dev, F_dev, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "force kernels");
    return LBM_OK;
}

int lbm_copy_probe(lbm_ctx *ctx, void *dst_dev, const void *src_dev, uint64_t nbytes)
{
    CTX_CHECK(ctx);
    if (!dst_dev || !src_dev) return fail(ctx, LBM_EINVAL, "null argument");
    if (((uintptr_t)dst_dev | (uintptr_t)src_dev) % 16)
        return fail(ctx, LBM_EINVAL, "copy buffers must be 16-byte aligned");
    hipError_t e = launch_copy(dst_dev, src_dev, nbytes, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy kernel");
    return LBM_OK;
}

int lbm_profile_step(lbm_ctx *ctx, int32_t nrep, int32_t max_k, double *ms, const char **names,
                     int32_t *n_kernels)
{
    CTX_CHECK(ctx);
    if (nrep < 1 || !ms || !n_kernels || max_k < 0) return fail(ctx, LBM_EINVAL, "bad arguments");
    *n_kernels = N_STEP_KERNELS;
    hipStream_t st = ctx->stream;
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    int rc = LBM_OK;
    ctx->rho_ok[ctx->par ^ 1] = false;  // the launches overwrite f[par ^ 1]
    for (int j = 0; j < N_STEP_KERNELS && j < max_k && rc == LBM_OK; ++j) {
        // in two-step mode the step kernel is the two-step one (two steps per launch)
        auto launch = [&]() {
            return ctx->two_step ? launch_step2(ctx->dev, ctx->par, st)
                                 : launch_step_kernel(ctx->dev, j, ctx->par, st);
        };
        hipError_t e = launch();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < nrep && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) {
            rc = hip_fail(ctx, e, "profile launches");
            break;
        }
        ms[j] = (double)t / nrep;
        if (names) names[j] = ctx->two_step ? "k_fused_step2" : step_kernel_name(j);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

static void drop_graphs(lbm_ctx *ctx)
{
    for (int i = 0; i < 2; ++i)
        if (ctx->graph[i]) {
            (void)hipGraphExecDestroy(ctx->graph[i]);
            ctx->graph[i] = nullptr;
        }
}

// a strip plan the two-step kernel can run: one-wavefront strips of at most
// SW2 output columns
static bool two_step_plan(int cols, int full_rows)
{
    return !full_rows && strip_waves(cols) == 1 && cols <= SW2;
}

static int set_strips(lbm_ctx *ctx, int rows, int cols, int balance, int full_rows = 0)
{
    if (ctx->two_step && !two_step_plan(cols, full_rows))
        return fail(ctx, LBM_EUNSUPPORTED, "two steps per launch need one-wavefront strips of at "
                                           "most 52 columns (lbm_set_two_step(ctx, 0) first)");
    const int frw = full_rows ? fullrow_waves(ctx->params.data(), ctx->n_inst) : 0;
    if (full_rows && !frw)
        return fail(ctx, LBM_EUNSUPPORTED, "full rows need every lattice width a multiple of 64, at most 512");
    StripPlan plan = full_rows    ? plan_fullrow(ctx->params.data(), ctx->n_inst, rows, frw)
                     : balance > 0 ? plan_balanced(ctx->params.data(), ctx->n_inst, cols, balance * ctx->ncu)
                                   : plan_uniform(ctx->params.data(), ctx->n_inst, rows, cols);
    if ((int)plan.segs.size() > ctx->layout.max_strips)
        return fail(ctx, LBM_EINVAL, "strip table overflow");
    if (!full_rows && !plan_fits(plan, strip_waves(cols)))
        return fail(ctx, LBM_EINVAL, "strip wider than its workgroup");
    // the tables are read by kernels already queued: order the copies after them
    HIP_TRY(ctx, hipMemcpyAsync(ctx->dev.strips, plan.segs.data(), sizeof(int4) * plan.segs.size(),
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->dev.first, plan.first.data(), sizeof(int) * plan.first.size(),
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->dev.nstrips = (int)plan.segs.size();
    ctx->dev.nwg = (int)plan.first.size() - 1;
    ctx->dev.nw = full_rows ? frw : strip_waves(cols);
    ctx->dev.fr = full_rows ? 1 : 0;
    ctx->chunk = rows;
    ctx->width = cols;
    ctx->balance = full_rows ? 0 : balance;
    ctx->full_rows = full_rows;
    drop_graphs(ctx);
    return LBM_OK;
}

int lbm_set_tiling(lbm_ctx *ctx, int32_t chunk_rows)
{
    CTX_CHECK(ctx);
    if (chunk_rows < MIN_CHUNK || chunk_rows > 65535)
        return fail(ctx, LBM_EINVAL, "chunk_rows must be in [2, 65535]");
    return set_strips(ctx, chunk_rows, ctx->width, 0, ctx->full_rows);
}

int lbm_set_full_rows(lbm_ctx *ctx, int32_t on)
{
    CTX_CHECK(ctx);
    if (on != 0 && on != 1) return fail(ctx, LBM_EINVAL, "on must be 0 or 1");
    return set_strips(ctx, ctx->chunk, ctx->width, 0, on);
}

int32_t lbm_get_full_rows(const lbm_ctx *ctx) { return ctx ? ctx->full_rows : -1; }

int lbm_set_two_step(lbm_ctx *ctx, int32_t on)
{
    CTX_CHECK(ctx);
    if (on != 0 && on != 1) return fail(ctx, LBM_EINVAL, "on must be 0 or 1");
    if (on && !two_step_plan(ctx->width, ctx->full_rows))
        return fail(ctx, LBM_EUNSUPPORTED, "two steps per launch need one-wavefront strips of at "
                                           "most 52 columns");
    if (on != ctx->two_step) drop_graphs(ctx);
    ctx->two_step = on;
    return LBM_OK;
}

int32_t lbm_get_two_step(const lbm_ctx *ctx) { return ctx ? ctx->two_step : -1; }

int lbm_set_strip_width(lbm_ctx *ctx, int32_t cols)
{
    CTX_CHECK(ctx);
    if (cols < MIN_WIDTH || cols > MAX_STRIP_COLS)
        return fail(ctx, LBM_EINVAL, "cols must be in [16, 506]");
    return set_strips(ctx, ctx->chunk, cols, ctx->balance);
}

int32_t lbm_get_strip_width(const lbm_ctx *ctx) { return ctx ? ctx->width : -1; }

int lbm_set_balance(lbm_ctx *ctx, int32_t wgs_per_cu)
{
    CTX_CHECK(ctx);
    if (wgs_per_cu < 0 || wgs_per_cu > 8 || wgs_per_cu * ctx->ncu > MAX_WG)
        return fail(ctx, LBM_EINVAL, "wgs_per_cu must be in [0, 8]");
    return set_strips(ctx, ctx->chunk, ctx->width, wgs_per_cu);
}

int32_t lbm_get_balance(const lbm_ctx *ctx) { return ctx ? ctx->balance : -1; }

int32_t lbm_get_workgroups(const lbm_ctx *ctx) { return ctx ? ctx->dev.nwg : -1; }

int lbm_plan_workgroups(const lbm_params *params, int32_t n_inst, int32_t cols, int32_t chunk_rows,
                        int32_t wgs, int32_t full_rows, int32_t *nwg, int32_t *nsegs)
{
    if (!params || !nwg || n_inst < 1) return fail(nullptr, LBM_EINVAL, "null argument or n_inst < 1");
    for (int i = 0; i < n_inst; ++i) {
        std::string m = check_params(params[i]);
        if (!m.empty()) return fail(nullptr, LBM_EINVAL, "instance " + std::to_string(i) + ": " + m);
    }
    if (cols < MIN_WIDTH || cols > MAX_STRIP_COLS)
        return fail(nullptr, LBM_EINVAL, "cols must be in [16, 506]");
    if (wgs < 0 || wgs > MAX_WG) return fail(nullptr, LBM_EINVAL, "wgs must be in [0, 8192]");
    if (wgs == 0 && (chunk_rows < MIN_CHUNK || chunk_rows > 65535))
        return fail(nullptr, LBM_EINVAL, "chunk_rows must be in [2, 65535]");
    if (full_rows) {
        if (!fullrow_waves(params, n_inst))
            return fail(nullptr, LBM_EUNSUPPORTED,
                        "full rows need every lattice width a multiple of 64, at most 512");
        if (chunk_rows < MIN_CHUNK || chunk_rows > 65535)
            return fail(nullptr, LBM_EINVAL, "chunk_rows must be in [2, 65535]");
    }
    StripPlan plan = full_rows ? plan_fullrow(params, n_inst, chunk_rows, fullrow_waves(params, n_inst))
                     : wgs > 0 ? plan_balanced(params, n_inst, cols, wgs)
                               : plan_uniform(params, n_inst, chunk_rows, cols);
    if (!full_rows && !plan_fits(plan, strip_waves(cols)))
        return fail(nullptr, LBM_EINVAL, "strip wider than its workgroup");
    if ((int)plan.segs.size() > max_strips(params, n_inst))
        return fail(nullptr, LBM_EINVAL, "strip table overflow");
    *nwg = (int32_t)plan.first.size() - 1;
    if (nsegs) *nsegs = (int32_t)plan.segs.size();
    return LBM_OK;
}

int32_t lbm_get_tiling(const lbm_ctx *ctx) { return ctx ? ctx->chunk : -1; }

int lbm_destroy(lbm_ctx *ctx)
{
    if (!ctx) return LBM_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < 2; ++i)
        if (ctx->graph[i]) (void)hipGraphExecDestroy(ctx->graph[i]);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    delete ctx;
    return LBM_OK;
}

// ------------------------------------------------------------------ adjoint
static AdjPar adj_par(const lbm_ctx *ctx, int inst)
{
    const lbm_params &p = ctx->params[inst];
    const KInst &K = ctx->hinst[inst];
    AdjPar A;
    std::memset(&A, 0, sizeof A);
    A.nx = p.nx;
    A.ny = p.ny;
    A.walls = p.walls;
    A.pitch = K.pitch;
    A.plane = K.plane;
    for (int k = 0; k < 2; ++k) {
        A.G1[k] = (float)p.G1[k];
        A.G2[k] = (float)p.G2[k];
        A.it[k] = (float)(1.0 / p.tau[k]);
        A.cg[k] = (float)(1.0 - 0.5 / p.tau[k]);
        A.g[k][0] = (float)p.g[k][0];
        A.g[k][1] = (float)p.g[k][1];
        A.rho_ref[k] = K.rho_ref[k];
        A.rho_wall[k] = K.rho_wall[k];
        A.psi_wall[k] = K.psi_wall[k];
    }
    A.gab = (float)p.G_AB;
    A.rho0 = K.rho0;
    A.inv_rho0 = K.inv_rho0;
    A.qscale = (float)(1.0 / p.nx);
    A.scr = K.fld;
    A.rscr = K.fld + (int64_t)SCR_RDEV * K.plane;  // one packed density buffer <= 2 planes
    A.rdev = A.rscr;
    A.fbo = SCR_FBAR;
    A.fbi = SCR_FBAR2;
    A.rdev_next = nullptr;
    A.part = (double *)(K.fld + (int64_t)SCR_PART * K.plane);
    A.res = A.part + (int64_t)adjoint_blocks(p.nx, p.ny) * NPART;
    return A;
}

// [a, a + na) and [b, b + nb) share a byte
static bool overlaps(const void *a, uint64_t na, const void *b, uint64_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

// The caller's state f_dev (lbm_get_populations layout) in the packed layout
// of the adjoint kernels, in the instance's spare population buffer f[par ^ 1]
// (free between steps: the next step overwrites it).
static const float *packed_state(lbm_ctx *ctx, int inst, const float *f_dev, hipError_t *e)
{
    ctx->rho_ok[ctx->par ^ 1] = false;
    *e = launch_import(ctx->dev, inst, ctx->par ^ 1, f_dev, ctx->stream);
    return ctx->hinst[inst].f[ctx->par ^ 1];
}

int lbm_adjoint_step(lbm_ctx *ctx, int32_t inst, const float *f_dev, const float *lam_in_dev,
                     float *lam_out_dev, double *grad_dev)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (ctx->params[inst].forcing != LBM_FORCING_GUO)
        return fail(ctx, LBM_EUNSUPPORTED, "the adjoint is written for the Guo forcing");
    if (!f_dev || !lam_in_dev || !lam_out_dev) return fail(ctx, LBM_EINVAL, "null argument");
    const lbm_params &p = ctx->params[inst];
    const uint64_t nb = (uint64_t)18 * p.nx * p.ny * sizeof(float);
    if (overlaps(lam_out_dev, nb, lam_in_dev, nb) || overlaps(lam_out_dev, nb, f_dev, nb))
        return fail(ctx, LBM_EINVAL, "lam_out must not overlap f or lam_in");
    hipError_t e;
    const float *fp = packed_state(ctx, inst, f_dev, &e);
    if (e == hipSuccess)
        e = launch_adjoint_step(adj_par(ctx, inst), fp, lam_in_dev, lam_out_dev, grad_dev, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "adjoint kernels");
    return LBM_OK;
}

int lbm_pressure(lbm_ctx *ctx, int32_t inst, float *P_dev, double *line_tension)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (!P_dev) return fail(ctx, LBM_EINVAL, "null output");
    rc = ensure_rho(ctx);
    if (rc) return rc;
    const lbm_params &p = ctx->params[inst];
    const KInst &K = ctx->hinst[inst];
    // block partials and the final sum in the instance's field scratch
    double *part = (double *)(K.fld + (int64_t)SCR_PART * K.plane);
    double *res = part + adjoint_blocks(p.nx, p.ny);
    hipError_t e = launch_pressure(ctx->dev, p, inst, ctx->par, P_dev, part, res, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "pressure kernels");
    if (line_tension) {
        double sum = 0.0;
        HIP_TRY(ctx, hipMemcpyAsync(&sum, res, sizeof sum, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        *line_tension = sum / p.ny;
    }
    return LBM_OK;
}

int64_t lbm_record_floats(const lbm_ctx *ctx, int32_t inst)
{
    if (!ctx || inst < 0 || inst >= ctx->n_inst) return -1;
    const InstLayout &L = ctx->layout.inst[inst];
    return L.fsize + L.rsize;
}

int lbm_record(lbm_ctx *ctx, int32_t inst, int64_t nsteps, float *f_store_dev)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (nsteps < 0 || (nsteps > 0 && !f_store_dev)) return fail(ctx, LBM_EINVAL, "bad arguments");
    if (nsteps == 0) return LBM_OK;
    const InstLayout &L = ctx->layout.inst[inst];
    const KInst &K = ctx->hinst[inst];
    const int64_t S = L.fsize + L.rsize;
    rc = ensure_rho(ctx);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    // slot 0 = the current state; step j reads slot j and writes slot j + 1
    // (the last step the context's own buffers, so the context advances);
    // these launches write the densities of every instance
    HIP_TRY(ctx, hipMemcpyAsync(f_store_dev, K.f[ctx->par], L.fsize * sizeof(float),
                                hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(f_store_dev + L.fsize, K.rho[ctx->par], L.rsize * sizeof(float),
                                hipMemcpyDeviceToDevice, st));
    for (int64_t j = 0; j < nsteps; ++j) {
        float *cur = f_store_dev + j * S, *nxt = f_store_dev + (j + 1) * S;
        const bool last = j + 1 == nsteps;
        const StepOvr o{inst, cur, last ? K.f[ctx->par ^ 1] : nxt,
                        last ? K.rho[ctx->par ^ 1] : nxt + L.fsize, 1};
        hipError_t e = launch_step_ovr(ctx->dev, ctx->par, o, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "step launch");
        ctx->par ^= 1;
        ctx->rho_ok[ctx->par] = true;
        ctx->rho_ok[ctx->par ^ 1] = false;
    }
    ctx->steps += nsteps;
    return LBM_OK;
}

int lbm_adjoint_run(lbm_ctx *ctx, int32_t inst, int64_t nsteps, const float *f_store_dev,
                    float *lam_dev, float *tmp_dev, double *grad_dev)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (ctx->params[inst].forcing != LBM_FORCING_GUO)
        return fail(ctx, LBM_EUNSUPPORTED, "the adjoint is written for the Guo forcing");
    if (nsteps < 0 || !lam_dev || !tmp_dev || (nsteps > 0 && !f_store_dev))
        return fail(ctx, LBM_EINVAL, "bad arguments");
    const lbm_params &p = ctx->params[inst];
    const InstLayout &L = ctx->layout.inst[inst];
    const int64_t N = (int64_t)p.nx * p.ny, S = L.fsize + L.rsize;
    const uint64_t nb = (uint64_t)18 * N * sizeof(float), ns = (uint64_t)S * sizeof(float);
    if (overlaps(lam_dev, nb, tmp_dev, nb)) return fail(ctx, LBM_EINVAL, "lam and tmp overlap");
    if (nsteps > 0 && (overlaps(lam_dev, nb, f_store_dev, ns * nsteps) ||
                       overlaps(tmp_dev, nb, f_store_dev, ns * nsteps)))
        return fail(ctx, LBM_EINVAL, "lam or tmp overlaps the state store");
    if (nsteps == 0) return LBM_OK;
    const AdjPar A = adj_par(ctx, inst);
    hipStream_t st = ctx->stream;
    hipError_t e = launch_adjoint_zero(A, st);  // also: no pending addition before the first step
    float *cur = lam_dev, *nxt = tmp_dev;
    // Step j writes its force adjoints to one of two plane sets (by the
    // parity of j); every step after the first forms the pending addition of
    // the step before from that step's set and state (the force pass folded
    // into its local pass), so only the last step runs the force pass.
    auto fb_set = [](int64_t j) { return (j & 1) ? SCR_FBAR2 : SCR_FBAR; };
    for (int64_t j = nsteps - 1; j >= 0 && e == hipSuccess; --j) {
        AdjPar B = A;
        B.rdev = f_store_dev + j * S + L.fsize;
        B.fbo = fb_set(j);
        const bool fold = j < nsteps - 1;
        if (fold) {
            B.fbi = fb_set(j + 1);
            B.rdev_next = f_store_dev + (j + 1) * S + L.fsize;
        }
        e = launch_adjoint_local(B, fold, f_store_dev + j * S, cur, nxt, st);
        std::swap(cur, nxt);
    }
    if (e == hipSuccess) {
        AdjPar B = A;
        B.rdev = f_store_dev + L.fsize;  // state 0
        B.fbo = fb_set(0);
        e = launch_adjoint_force(B, st);
    }
    if (e == hipSuccess) e = launch_adjoint_final(A, grad_dev, st);
    // the last step's pending addition, into lam_dev
    if (e == hipSuccess) e = launch_adjoint_combine(A, cur, lam_dev, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "adjoint run");
    return LBM_OK;
}

int lbm_adjoint_seed(lbm_ctx *ctx, int32_t inst, int32_t objective, const float *f_dev,
                     float *lam_dev, double *J, double *dtheta)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (ctx->params[inst].forcing != LBM_FORCING_GUO)
        return fail(ctx, LBM_EUNSUPPORTED, "the adjoint is written for the Guo forcing");
    if (!f_dev || !J || !dtheta) return fail(ctx, LBM_EINVAL, "null argument");
    if (objective < LBM_OBJ_DP || objective > LBM_OBJ_MASS_A)
        return fail(ctx, LBM_EINVAL, "unknown objective");
    if (!lam_dev && objective == LBM_OBJ_Q)
        return fail(ctx, LBM_EINVAL, "the flow-rate objective needs lam_dev");
    const lbm_params &p = ctx->params[inst];
    const uint64_t nb = (uint64_t)18 * p.nx * p.ny * sizeof(float);
    if (lam_dev && overlaps(lam_dev, nb, f_dev, nb))
        return fail(ctx, LBM_EINVAL, "lam_dev must not overlap f_dev");
    const AdjPar A = adj_par(ctx, inst);
    hipStream_t st = ctx->stream;
    hipError_t e;
    const float *fp = packed_state(ctx, inst, f_dev, &e);
    if (e == hipSuccess) e = launch_objective_pass1(A, objective, fp, lam_dev, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "objective kernels");
    double res[NPART];
    HIP_TRY(ctx, hipMemcpyAsync(res, A.res, sizeof res, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int t = 0; t < 5; ++t) dtheta[t] = 0.0;
    if (objective == LBM_OBJ_DP) {
        // res: S_A, S_B, P_A, P_B, dP_A/dG12, dP_B/dG12, dP_A/dG_AB, dP_B/dG_AB
        if (!(res[0] > 0.0) || !(res[1] > 0.0))
            return fail(ctx, LBM_EINVAL, "pressure-jump objective needs both phases present");
        const double mA = res[2] / res[0], mB = res[3] / res[1];
        *J = mA - mB;
        dtheta[0] = dtheta[1] = res[4] / res[0] - res[5] / res[1];
        dtheta[2] = res[6] / res[0] - res[7] / res[1];
        if (lam_dev) {
            e = launch_objective_dp_seed(A, lam_dev, mA, mB, res[0], res[1], st);
            if (e != hipSuccess) return hip_fail(ctx, e, "objective seed kernel");
        }
    } else {
        *J = res[5];
        if (objective == LBM_OBJ_Q)
            for (int t = 0; t < 3; ++t) dtheta[t] = res[t];
    }
    if (!std::isfinite(*J)) return fail(ctx, LBM_ENONFINITE, "objective is not finite");
    return LBM_OK;
}

int lbm_set_params(lbm_ctx *ctx, int32_t inst, const lbm_params *params)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (!params) return fail(ctx, LBM_EINVAL, "null argument");
    std::string m = check_params(*params);
    if (!m.empty()) return fail(ctx, LBM_EINVAL, m);
    const lbm_params &old = ctx->params[inst];
    if (params->forcing != old.forcing)
        return fail(ctx, LBM_EUNSUPPORTED, "the forcing scheme of a context cannot change");
    if (params->nx != old.nx || params->ny != old.ny || params->walls != old.walls ||
        (float)params->rho_ref[0] != (float)old.rho_ref[0] ||
        (float)params->rho_ref[1] != (float)old.rho_ref[1])
        return fail(ctx, LBM_EINVAL, "nx, ny, walls and rho_ref of an instance cannot change");
    const InstLayout &L = ctx->layout.inst[inst];
    KInst K = make_kinst(*params, L, ctx->ws + ctx->layout.off_inst[inst]);
    // kernels already queued read the old block: order the update after them
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->dev.insts + inst, &K, sizeof K, hipMemcpyHostToDevice,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->params[inst] = *params;
    ctx->hinst[inst] = K;
    return LBM_OK;
}

int lbm_profile_adjoint(lbm_ctx *ctx, int32_t inst, const float *f_dev, const float *lam_in_dev,
                        float *lam_out_dev, double *grad_dev, int32_t nrep, int32_t max_k,
                        double *ms, const char **names, int32_t *n_kernels)
{
    CTX_CHECK(ctx);
    int rc = check_inst(ctx, inst);
    if (rc) return rc;
    if (!f_dev || !lam_in_dev || !lam_out_dev || !grad_dev || nrep < 1 || !ms || !n_kernels ||
        max_k < 0)
        return fail(ctx, LBM_EINVAL, "bad arguments");
    const AdjPar A = adj_par(ctx, inst);
    hipStream_t st = ctx->stream;
    *n_kernels = N_ADJ_KERNELS;
    hipError_t ei;
    const float *fp = packed_state(ctx, inst, f_dev, &ei);
    if (ei != hipSuccess) return hip_fail(ctx, ei, "import");
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    rc = LBM_OK;
    for (int j = 0; j < N_ADJ_KERNELS && j < max_k && rc == LBM_OK; ++j) {
        hipError_t e = launch_adjoint_zero(A, st);
        if (e == hipSuccess) e = launch_adjoint_kernel(A, j, fp, lam_in_dev, lam_out_dev, grad_dev, st);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < nrep && e == hipSuccess; ++r)
            e = launch_adjoint_kernel(A, j, fp, lam_in_dev, lam_out_dev, grad_dev, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) {
            rc = hip_fail(ctx, e, "profile launches");
            break;
        }
        ms[j] = (double)t / nrep;
        if (names) names[j] = adjoint_kernel_name(j);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int lbm_lds_checks(lbm_ctx *ctx, int64_t *violations)
{
    CTX_CHECK(ctx);
    if (!violations) return fail(ctx, LBM_EINVAL, "null output");
    unsigned int bad = 0;
    hipError_t e = lds_checks(&bad, ctx->stream);
    if (e == hipErrorNotSupported)
        return fail(ctx, LBM_EUNSUPPORTED, "LDS index checks need the checked build (LBM_CHECK_LDS)");
    if (e != hipSuccess) return hip_fail(ctx, e, "reading the LDS check counter");
    *violations = (int64_t)bad;
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

}  // extern "C"
