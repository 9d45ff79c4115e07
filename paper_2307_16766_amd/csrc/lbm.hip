// lbm.hip -- host side of the C ABI declared in include/lbm.h (liblbm_hip.so, gfx950).
//
// The library owns no device memory: the caller's workspace is carved into two population
// buffers, two parity copies of the boundary solver state, the Dirichlet profiles and the
// diagnostics scratch.  One step is one kernel launch (k_step) on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "adjoint.h"
#include "kernels.h"
#include "lbm.h"

using namespace lbm;

// Scratch of lbm_diagnostics_noalloc: the first pass's partials ([8][NOALLOC_PARTIALS],
// component-major) and nothing else; every device the library runs on holds its own copy until
// the process ends.  Host code never passes `scratch` itself to a kernel (on the host it names a
// stand-in, not device memory): lbm_init looks up each device's address once.
constexpr int NOALLOC_PARTIALS = 16384;
static __device__ __align__(256) double scratch[8 * NOALLOC_PARTIALS];

namespace {

std::string g_err;

// per-device address of `scratch` (hipGetSymbolAddress with that device current)
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

hipError_t scratch_address(int dev, double** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool is_char(int b) { return b >= BC_LODI && b <= BC_CBC_RELAX; }
bool is_relax(int b) { return b == BC_LODI_RELAX || b == BC_CBC_RELAX; }
bool is_full(int b) { return b == BC_CBC || b == BC_CBC_RELAX; }

int stencil_M(int st) { return st == 9 ? 1 : 3; }
double stencil_cs2(int st) { return st == 9 ? Lat<9>::cs2 : st == 17 ? Lat<17>::cs2 : Lat<37>::cs2; }
int chunk_rows(int M) { return 192 / M - 8; }   // must match ChunkShape::CR - 8 in char_chunk
// Sides normal to x (rows along y) take shorter chunks where the bulk update is short: their strip
// pull reads one population per row and plane, each from its own cache line, and a work-group's
// lines go through one CU's vector memory path; spreading the rows over more work-groups shortens
// the pull and the reconstruction (256^2 D2Q37: 21.0 -> 17.1 us per step in FP64, C3-sized grids
// 39 -> 34 us in FP32).  Where the bulk runs far longer than a chunk (from 8192 bulk work-groups
// on), the boundary is hidden behind it and the extra work-groups only take CU slots (4096 x 2048:
// 398.5 -> 404 us), so the chunks stay full height.
bool short_x_chunks(int nx, int ny) { return (long long)((nx + 255) / 256) * ny < 8192; }
// D2Q37 takes 12 rows, and 8 on CBC sides, whose four pulls per row (x_f and the three
// viscous-moment nodes) are the slowest loads under the bulk's traffic (1024 x 512 FP32, CBC-RELAX
// outflow: 35.4 -> 31.3 us per step; 256^2 FP64 15.6 -> 15.4 us); D2Q9 takes 16 rows (256 x 128:
// 7.7 -> 6.8 us per step).
int chunk_rows_x(int M, int nx, int ny, bool cbc) {
    if (!short_x_chunks(nx, ny)) return chunk_rows(M);
    return M == 3 ? (cbc ? 8 : 12) : M == 2 ? 24 : 16;
}
// sides normal to y (coalesced pulls) take half-height chunks on the same small grids: their
// reconstruction and corner chunks then end sooner
int chunk_rows_y(int M, int nx, int ny) { return short_x_chunks(nx, ny) ? chunk_rows(M) / 2 : chunk_rows(M); }
// Reverse chunks of the adjoint (halo of 8 rows on each side): on the same small grids every
// side takes the short height, since a reverse chunk's load phase grows with its rows whatever
// the side's orientation and the sweep waits for the slowest chunk (256^2 D2Q37: sides normal to
// y at 69 -> 17 rows took the reverse step from 39.7 to 37.7 us)
int adj_rows(int M) { return 256 / M - 16; }   // must match NR - 2 H in adj_chunk
int adj_rows_short(int M, int nx, int ny) {
    if (!short_x_chunks(nx, ny)) return adj_rows(M);
    return M == 3 ? 12 : M == 2 ? 24 : 48;   // D2Q37: 16 -> 12 rows, 36.34 -> 36.07 us per 256^2 reverse step
}

struct Layout {
    int Q = 0, M = 0, MS = 0;
    size_t esz = 0;
    unsigned long long pitch = 0;   // padded row length of a population plane (elements)
    size_t f_bytes = 0, region_bytes = 0, off_region = 0, off_inlet[4] = {0, 0, 0, 0}, off_diag = 0, total = 0;
    int diag_blocks = 0;
    SideDev s[4];
    CornerDev c[4];
};

int validate(const lbm_config* c, std::string& err) {
    if (!c) { err = "null config"; return LBM_E_ARG; }
    if (c->stencil != 9 && c->stencil != 17 && c->stencil != 37) { err = "stencil must be LBM_D2Q9, LBM_D2Q17 or LBM_D2Q37"; return LBM_E_ARG; }
    if (c->precision != LBM_FP64 && c->precision != LBM_FP32DEV) { err = "unknown precision"; return LBM_E_ARG; }
    if (!(c->tau > 0.5) || !std::isfinite(c->tau)) { err = "tau must be a finite value above 1/2"; return LBM_E_ARG; }
    for (int s = 0; s < 4; ++s)
        if (c->bc[s] < 0 || c->bc[s] > 6) { err = "unknown boundary type"; return LBM_E_ARG; }
    if ((c->bc[0] == BC_PERIODIC) != (c->bc[1] == BC_PERIODIC) || (c->bc[2] == BC_PERIODIC) != (c->bc[3] == BC_PERIODIC)) {
        err = "periodic sides must come in pairs"; return LBM_E_ARG;
    }
    const int M = stencil_M(c->stencil);
    const bool xp = c->bc[0] == BC_PERIODIC, yp = c->bc[2] == BC_PERIODIC;
    if (c->nx < (xp ? M + 1 : 2 * M + 3) || c->ny < (yp ? M + 1 : 2 * M + 3)) { err = "grid too small"; return LBM_E_ARG; }
    // the viscous terms of a CBC side are evaluated at x_f - M .. x_f - M - 2, which must be bulk nodes
    if (((is_full(c->bc[0]) || is_full(c->bc[1])) && c->nx < 3 * M + 3) ||
        ((is_full(c->bc[2]) || is_full(c->bc[3])) && c->ny < 3 * M + 3)) {
        err = "CBC sides need at least 3M + 3 nodes along their normal"; return LBM_E_ARG;
    }
    if ((double)c->nx * (double)c->ny > 2.0e9) { err = "grid too large"; return LBM_E_ARG; }
    {   // the step kernel's row of bulk tile t is umulhi(t, floor(2^32 / bpr) + 1): exact while t * bpr < 2^32
        const unsigned long long bpr = ((unsigned long long)c->nx + 255) / 256;
        if (bpr * bpr * (unsigned long long)c->ny >= (1ull << 32)) { err = "grid too large for the step kernel's tile indexing"; return LBM_E_UNSUPPORTED; }
    }
    if (!xp && !yp)
        for (int sx = 0; sx < 2; ++sx)
            for (int sy = 2; sy < 4; ++sy) {
                const bool ok = (is_char(c->bc[sx]) && is_char(c->bc[sy])) || (c->bc[sx] == BC_ZG && c->bc[sy] == BC_ZG);
                if (!ok) { err = "corner between these boundary types is not supported"; return LBM_E_UNSUPPORTED; }
            }
    if (c->stencil == 9)
        for (int s = 0; s < 4; ++s)
            if (is_full(c->bc[s])) { err = "CBC with viscous terms needs a thermal stencil (D2Q17 or D2Q37)"; return LBM_E_UNSUPPORTED; }
    return LBM_OK;
}

void make_layout(const lbm_config* c, Layout& L) {
    L.Q = c->stencil;
    L.M = stencil_M(c->stencil);
    L.MS = L.M == 1 ? 2 : 1;
    L.esz = c->precision == LBM_FP64 ? 8 : 4;
    L.pitch = ((unsigned long long)c->nx + 63) / 64 * 64;
    L.f_bytes = align_up((size_t)L.Q * L.pitch * c->ny * L.esz);
    const bool xp = c->bc[0] == BC_PERIODIC, yp = c->bc[2] == BC_PERIODIC;
    size_t reg = 0;
    int blk = 0;
    for (int s = 0; s < 4; ++s) {
        SideDev& d = L.s[s];
        std::memset(&d, 0, sizeof(d));
        const int b = c->bc[s];
        d.scheme = b;
        d.kind = b == BC_PERIODIC ? KIND_NONE : is_char(b) ? KIND_CHAR : b == BC_ZG ? KIND_ZG : KIND_DIRICHLET;
        d.nax = s < 2 ? 0 : 1;
        d.sn = (s % 2 == 0) ? -1 : 1;
        d.Nn = d.nax == 0 ? c->nx : c->ny;
        d.Nt = d.nax == 0 ? c->ny : c->nx;
        d.tper = d.nax == 0 ? yp : xp;
        d.r0 = d.tper ? 0 : L.M;
        d.len = d.tper ? d.Nt : d.Nt - 2 * L.M;
        d.xf = d.sn > 0 ? d.Nn - 1 - L.M : L.M;
        d.corner_lo = d.corner_hi = -1;
        if (!d.tper) {
            if (d.nax == 0) { d.corner_lo = (s & 1); d.corner_hi = (s & 1) | 2; }
            else { d.corner_lo = ((s - 2) << 1); d.corner_hi = 1 | ((s - 2) << 1); }
        }
        d.owns_corners = d.nax == 0;
        d.Pinf = 0;
        if (d.kind == KIND_CHAR) {
            d.rows = d.nax == 0 ? chunk_rows_x(L.M, c->nx, c->ny, is_full(b)) : chunk_rows_y(L.M, c->nx, c->ny);
            d.nblk = (d.len + d.rows - 1) / d.rows;
            d.off_ub = reg; reg += align_up((size_t)L.M * d.len * 4 * 8);
            d.off_strip = reg; reg += align_up((size_t)L.MS * d.len * 4 * 8);
            d.off_stage = reg; reg += align_up((size_t)3 * L.M * d.len * 4 * 8);
            if (is_full(b)) { d.off_vis = reg; reg += align_up((size_t)3 * d.len * 6 * 8); }
        } else if (d.kind == KIND_ZG) {
            d.rows = 256;
            d.nblk = (d.len + 255) / 256;
        }
        d.blk0 = blk;
        blk += d.nblk;
    }
    for (int ci = 0; ci < 4; ++ci) {
        CornerDev& k = L.c[ci];
        std::memset(&k, 0, sizeof(k));
        const int sx = ci & 1, sy = 2 + (ci >> 1);
        k.active = !xp && !yp;
        if (!k.active) continue;
        k.zg = c->bc[sx] == BC_ZG;
        const SideDev &X = L.s[sx], &Y = L.s[sy];
        k.xc = X.xf + X.sn;
        k.yc = Y.xf + Y.sn;
        k.vx = -X.sn;
        k.vy = -Y.sn;
        k.x0 = X.xf + X.sn; k.sxn = X.sn;
        k.y0 = Y.xf + Y.sn; k.syn = Y.sn;
        k.ndx = X.sn / std::sqrt(2.0);
        k.ndy = Y.sn / std::sqrt(2.0);
        if (!k.zg) {
            k.off_cu = reg; reg += ALIGN;
            k.off_cd = reg; reg += ALIGN;
            k.off_cs = reg; reg += ALIGN;
        }
    }
    L.region_bytes = align_up(reg > 0 ? reg : ALIGN);
    size_t off = 2 * L.f_bytes;
    L.off_region = off;
    off += 2 * L.region_bytes;
    for (int s = 0; s < 4; ++s) {
        L.off_inlet[s] = off;
        if (L.s[s].kind == KIND_DIRICHLET) off += align_up((size_t)L.s[s].len * 4 * 8);
    }
    L.diag_blocks = (int)(((unsigned long long)c->nx + 255) / 256 * c->ny);   // one per 256-node row tile
    L.off_diag = off;
    off += align_up((size_t)(L.diag_blocks + 1) * 8 * 8);
    L.total = off;
}

}  // namespace

// Tape of a recorded run (the caller's device buffer): checkpoints every K steps, and the
// scratch of the reverse sweep.
struct Tape {
    char* base = nullptr;
    int N = 0, K = 0, nchk = 0;
    long step_end = -1;
    // two recomputation sets (populations R, moments, boundary states), so that the recomputation
    // of one segment overlaps the reverse sweep of the next one
    size_t chk_stride = 0, off_R[2][2] = {{0, 0}, {0, 0}}, off_V[2] = {0, 0}, off_mom[2] = {0, 0}, mom_bytes = 0, off_rh[2] = {0, 0};
    size_t off_adj[2] = {0, 0}, off_ccon = 0, off_gm = 0, off_acc = 0, total = 0;
    size_t off_neep[4] = {0, 0, 0, 0};   // per characteristic / ZG side: [len][Q + 4] terms of nu^{n+1}(x_f)
    size_t off_zgc = 0;                  // per zero-gradient corner: [Q + 4] terms of nu^{n+1}(c + v)
    size_t off_dacc[4] = {0, 0, 0, 0};   // per Dirichlet side: [M][len][4] adjoint of a default profile
    int ablk0[4] = {0, 0, 0, 0}, anblk[4] = {0, 0, 0, 0}, arows[4] = {0, 0, 0, 0}, nadj = 0;
};

struct lbm_ctx {
    lbm_config cfg;
    Layout L;
    char* ws = nullptr;
    void* f[2] = {nullptr, nullptr};
    char* region[2] = {nullptr, nullptr};
    double* inlet[4] = {nullptr, nullptr, nullptr, nullptr};
    int inlet_set[4] = {0, 0, 0, 0};   // Dirichlet profile given by lbm_dirichlet_profile
    double* diag = nullptr;
    int cur = 0;
    long steps = 0;
    int diag_every = 0;            // lbm_step checks for non-finite populations every n steps (0: off)
    int device = 0;                // HIP device current at lbm_init
    double* scratch = nullptr;     // that device's copy of the file-scope `scratch` (device address)
    long save_hdr[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // checkpoint header staging: steps, Dirichlet profile flags
    hipStream_t stream = nullptr;
    int nbnd = 0;
    lbm_relax relax[4];
    int meso[4] = {0, 0, 0, 0};   // mesoscopic BC per side (LBM_RECON_*)
    int vfd[4] = {0, 0, 0, 0};    // viscous terms per CBC side (LBM_VISC_*)
    BulkArgs bulk;
    std::string err;
    // bulk kernel timing (measurement only)
    int timing = 0;                // time every timing-th step launch (0: off)
    size_t tcalls = 0;             // step launches since timing was set
    std::vector<hipEvent_t> tev;   // pairs: start, end
    size_t tcount = 0;             // recorded pairs
    Tape tape;
    // the adjoint's second stream (non-blocking, default priority) and its events, made on the
    // first lbm_adjoint: ev[0..1] recomputation set b ready, ev[2..3] set b released, ev[4] start
    hipStream_t aux = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

int fail(lbm_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg; else g_err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return fail(ctx, LBM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

BndArgs make_bnd(const lbm_ctx* c) {
    BndArgs a;
    std::memset(&a, 0, sizeof(a));
    const lbm_config& g = c->cfg;
    a.nx = g.nx; a.ny = g.ny;
    a.xper = g.bc[0] == BC_PERIODIC;
    a.yper = g.bc[2] == BC_PERIODIC;
    a.pitch = c->L.pitch;
    a.omega = 1.0 / g.tau;
    a.tau = g.tau;
    a.reg_cur = c->region[c->cur];
    a.reg_next = c->region[c->cur ^ 1];
    const double cs2 = stencil_cs2(g.stencil);
    const bool thermal = g.stencil != 9;
    for (int s = 0; s < 4; ++s) {
        a.s[s] = c->L.s[s];
        const lbm_relax& p = c->relax[s];
        const double cinf = thermal ? std::sqrt(2.0 * cs2 * p.T_inf) : std::sqrt(cs2);
        const double len = p.length > 0 ? p.length : (double)a.s[s].Nn;
        a.s[s].K = p.sigma * (1.0 - p.mach * p.mach) * cinf / len;
        a.s[s].alpha = p.alpha;
        a.s[s].meso = c->meso[s];
        a.s[s].vfd = c->vfd[s];
        a.s[s].Pinf = p.rho_inf * cs2 * (thermal ? p.T_inf : 1.0);
    }
    for (int ci = 0; ci < 4; ++ci) {
        a.c[ci] = c->L.c[ci];
        const int sx = ci & 1;
        a.c[ci].relax = is_relax(g.bc[sx]);
        a.c[ci].K = a.s[sx].K;
        a.c[ci].Pinf = a.s[sx].Pinf;
    }
    return a;
}

constexpr size_t MAX_TIMED = 65536;

// launch the step kernel, bracketed by timing events when kernel timing is on
template <typename F>
hipError_t timed_launch(lbm_ctx* c, F&& launch) {
    const bool rec = c->timing > 0 && (c->tcalls++ % (size_t)c->timing) == 0 && c->tcount < MAX_TIMED;
    if (rec) {
        while (c->tev.size() < 2 * (c->tcount + 1)) {
            hipEvent_t e;
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            c->tev.push_back(e);
        }
        const hipError_t r = hipEventRecord(c->tev[2 * c->tcount], c->stream);
        if (r != hipSuccess) return r;
    }
    launch(c->stream);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    if (rec) {
        r = hipEventRecord(c->tev[2 * c->tcount + 1], c->stream);
        if (r != hipSuccess) return r;
        c->tcount += 1;
    }
    return hipSuccess;
}

template <int Q, typename T, bool HIST>
void launch_step_raw(const lbm_ctx* c, const T* A, T* B, char* reg_cur, char* reg_next, double* mom, hipStream_t s) {
    BndArgs a = make_bnd(c);
    a.reg_cur = reg_cur;
    a.reg_next = reg_next;
    BulkArgs g = c->bulk;
    g.mom = mom;
    const int bpr = (g.x1 + 1 + 255) / 256;   // bulk tiles per row, aligned to x = 0
    const int nbnd = c->nbnd;
    const int nbnd_pad = sizeof(T) == 8 ? (nbnd + 7) & ~7 : nbnd;   // FP64 tile order, see k_step
    const int nblk = nbnd_pad + bpr * (g.y1 - g.y0 + 1);
    const unsigned magic = bpr > 1 ? (unsigned)((1ull << 32) / (unsigned long long)bpr + 1ull) : 0u;   // row = umulhi(t, magic)
    const bool px = c->cfg.bc[0] == BC_PERIODIC, py = c->cfg.bc[2] == BC_PERIODIC;
    if (px && py) hipLaunchKernelGGL((k_step<Q, T, true, true, HIST>), dim3(nblk), dim3(256), 0, s, A, B, a, g, nbnd, bpr, magic);
    else if (px) hipLaunchKernelGGL((k_step<Q, T, true, false, HIST>), dim3(nblk), dim3(256), 0, s, A, B, a, g, nbnd, bpr, magic);
    else if (py) hipLaunchKernelGGL((k_step<Q, T, false, true, HIST>), dim3(nblk), dim3(256), 0, s, A, B, a, g, nbnd, bpr, magic);
    else hipLaunchKernelGGL((k_step<Q, T, false, false, HIST>), dim3(nblk), dim3(256), 0, s, A, B, a, g, nbnd, bpr, magic);
}

template <int Q, typename T>
int launch_step(lbm_ctx* c) {
    const T* A = (const T*)c->f[c->cur];
    T* B = (T*)c->f[c->cur ^ 1];
    char* rc = c->region[c->cur];
    char* rn = c->region[c->cur ^ 1];
    auto step = [&](hipStream_t s) { launch_step_raw<Q, T, false>(c, A, B, rc, rn, nullptr, s); };
    HIPCHK(c, timed_launch(c, step));
    c->cur ^= 1;
    c->steps += 1;
    return LBM_OK;
}

template <int Q, typename T>
int launch_init(lbm_ctx* c, const double* rho, const double* ux, const double* uy, const double* Tf) {
    const int n = c->cfg.nx * c->cfg.ny;
    hipLaunchKernelGGL((k_init_fields<Q, T>), dim3((n + 255) / 256), dim3(256), 0, c->stream, rho, ux, uy,
                       Lat<Q>::thermal ? Tf : nullptr, (T*)c->f[0], (T*)c->f[1], c->cfg.nx, n, c->L.pitch);
    HIPCHK(c, hipGetLastError());
    const BndArgs a = make_bnd(c);
    int maxlen = 1;
    for (int s = 0; s < 4; ++s) maxlen = std::max(maxlen, c->L.s[s].len);
    hipLaunchKernelGGL((k_init_boundary<Q>), dim3((maxlen + 255) / 256, 4), dim3(256), 0, c->stream, a, rho, ux, uy,
                       Lat<Q>::thermal ? Tf : nullptr, c->inlet[0], c->inlet[1], c->inlet[2], c->inlet[3]);
    HIPCHK(c, hipGetLastError());
    for (int s = 0; s < 4; ++s) {
        if (c->L.s[s].kind != KIND_DIRICHLET) continue;
        const int tot = c->L.s[s].len * c->L.M;
        hipLaunchKernelGGL((k_dirichlet<Q, T>), dim3((tot + 255) / 256), dim3(256), 0, c->stream, a, s, c->inlet[s],
                           (T*)c->f[0], (T*)c->f[1]);
        HIPCHK(c, hipGetLastError());
    }
    return LBM_OK;
}

// ---------------------------------------------------------------- discrete adjoint (host side)
int adjoint_supported(const lbm_ctx* c, std::string& err) {
    const lbm_config& g = c->cfg;
    if (g.stencil == 9 && g.bc[0] != BC_PERIODIC && g.bc[2] != BC_PERIODIC) {
        err = "the D2Q9 adjoint needs one periodic axis (no corners)";
        return LBM_E_UNSUPPORTED;
    }
    return LBM_OK;
}

void tape_layout(const Layout& L, int nx, int ny, int N, int K, Tape& t) {
    t.N = N;
    t.K = K;
    t.nchk = (N + K - 1) / K;
    t.chk_stride = L.f_bytes + L.region_bytes;
    size_t off = (size_t)t.nchk * t.chk_stride;
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 2; ++k) { t.off_R[b][k] = off; off += L.f_bytes; }
    const size_t vbytes = align_up((size_t)L.Q * L.pitch * ny * 8);
    for (int k = 0; k < 2; ++k) { t.off_V[k] = off; off += vbytes; }
    t.mom_bytes = align_up((size_t)4 * L.pitch * ny * 8);
    for (int b = 0; b < 2; ++b) { t.off_mom[b] = off; off += (size_t)(K + 1) * t.mom_bytes; }
    for (int b = 0; b < 2; ++b) { t.off_rh[b] = off; off += (size_t)(K + 1) * L.region_bytes; }
    for (int k = 0; k < 2; ++k) { t.off_adj[k] = off; off += L.region_bytes; }
    t.off_ccon = off; off += align_up(4 * 2 * 2 * 4 * 8);
    t.off_gm = off; off += align_up(16 * 4 * 8);
    t.nadj = 0;
    for (int s = 0; s < 4; ++s) {
        t.arows[s] = adj_rows_short(L.M, nx, ny);
        t.ablk0[s] = t.nadj;
        t.anblk[s] = L.s[s].kind == KIND_CHAR ? (L.s[s].len + t.arows[s] - 1) / t.arows[s]
                   : L.s[s].kind == KIND_ZG ? (L.s[s].len + 255) / 256 : 0;
        t.nadj += t.anblk[s];
    }
    t.off_acc = off; off += align_up((size_t)(2 * t.nadj + 4) * 8);
    for (int s = 0; s < 4; ++s)
        if (L.s[s].kind == KIND_CHAR || L.s[s].kind == KIND_ZG) {
            t.off_neep[s] = off;
            off += align_up((size_t)L.s[s].len * (L.Q + 4) * 8);
        }
    t.off_zgc = off; off += align_up((size_t)4 * (L.Q + 4) * 8);
    for (int s = 0; s < 4; ++s)
        if (L.s[s].kind == KIND_DIRICHLET) {
            t.off_dacc[s] = off;
            off += align_up((size_t)L.M * L.s[s].len * 4 * 8);
        }
    t.total = off;
}

template <int Q, typename T>
int run_adjoint(lbm_ctx* c, const double* seed, double* grad, double* h_relax) {
    const Tape& t = c->tape;
    const Layout& L = c->L;
    hipStream_t st = c->stream;
    char* base = t.base;
    const BulkArgs& bk = c->bulk;
    const int nx = c->cfg.nx, ny = c->cfg.ny;
    const int bpr = (nx + 255) / 256;
    const bool px = c->cfg.bc[0] == BC_PERIODIC, py = c->cfg.bc[2] == BC_PERIODIC;
    double* V[2] = {(double*)(base + t.off_V[0]), (double*)(base + t.off_V[1])};
    auto mom_slot = [&](int b, int j) { return (double*)(base + t.off_mom[b] + (size_t)j * t.mom_bytes); };
    auto reg_slot = [&](int b, int j) { return base + t.off_rh[b] + (size_t)j * L.region_bytes; };
    if (!c->aux) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
        for (hipEvent_t& e : c->ev) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    hipStream_t ax = c->aux;

    hipLaunchKernelGGL((k_adj_seed<Q, T>), dim3(bpr * ny), dim3(256), 0, st, (const T*)c->f[c->cur], seed, V[t.N & 1], bk, bpr);
    HIPCHK(c, hipGetLastError());
    for (int k = 0; k < 2; ++k) HIPCHK(c, hipMemsetAsync(base + t.off_adj[k], 0, L.region_bytes, st));
    HIPCHK(c, hipMemsetAsync(base + t.off_ccon, 0, 4 * 2 * 2 * 4 * 8, st));
    HIPCHK(c, hipMemsetAsync(base + t.off_gm, 0, 16 * 4 * 8, st));
    HIPCHK(c, hipMemsetAsync(base + t.off_acc, 0, (size_t)(2 * t.nadj + 4) * 8, st));
    HIPCHK(c, hipMemsetAsync(base + t.off_zgc, 0, (size_t)4 * (L.Q + 4) * 8, st));

    AdjArgs g;
    std::memset(&g, 0, sizeof(g));
    g.b = make_bnd(c);
    g.ccon = (double*)(base + t.off_ccon);
    g.gm = (double*)(base + t.off_gm);
    g.acc = (double*)(base + t.off_acc);
    g.grad = grad;
    for (int s = 0; s < 4; ++s) { g.ablk0[s] = t.ablk0[s]; g.anblk[s] = t.anblk[s]; }
    for (int s = 0; s < 4; ++s) g.arows[s] = t.arows[s];
    g.nadj = t.nadj;
    for (int ci = 0; ci < 4; ++ci)
        for (int ax = 0; ax < 2; ++ax) {
            g.cside[ci][ax] = -1;
            g.crow[ci][ax] = 0;
            if (!L.c[ci].active) continue;
            const int s = ax == 0 ? (ci & 1) : 2 + (ci >> 1);
            g.cside[ci][ax] = s;
            g.crow[ci][ax] = L.s[s].corner_lo == ci ? 0 : L.s[s].len - 1;
        }
    bool any_corner = false;
    for (int ci = 0; ci < 4; ++ci) any_corner = any_corner || L.c[ci].active;
    // the sides' transverse terms reach the corner values through transverse relaxation (LODI-RELAX)
    // and always on CBC sides
    g.coupled = 0;
    for (int s = 0; s < 4; ++s)
        if (any_corner && ((c->cfg.bc[s] == BC_LODI_RELAX && c->relax[s].alpha != 0.0) || is_full(c->cfg.bc[s])))
            g.coupled = 1;
    bool any_full = false;
    for (int s = 0; s < 4; ++s) any_full = any_full || is_full(c->cfg.bc[s]);
    g.vism = 0;
    for (int s = 0; s < 4; ++s)
        if (is_full(c->cfg.bc[s]) && c->vfd[s] == LBM_VISC_MESO) g.vism = 1;
    g.neep_any = 0;
    for (int s = 0; s < 4; ++s) {
        g.neep[s] = nullptr;
        if ((L.s[s].kind == KIND_CHAR && c->meso[s] == LBM_RECON_NEEP) || L.s[s].kind == KIND_ZG) {
            g.neep[s] = (double*)(base + t.off_neep[s]);
            g.neep_any = 1;
        }
    }
    g.zgc = (double*)(base + t.off_zgc);
    g.zgc_any = 0;
    for (int ci = 0; ci < 4; ++ci) g.zgc_any = g.zgc_any || (L.c[ci].active && L.c[ci].zg);
    // Dirichlet sides with the default profile: the layers follow the initial fields of the first
    // layer at every time level
    g.dir_any = 0;
    for (int s = 0; s < 4; ++s) {
        g.dacc[s] = nullptr;
        g.dprof[s] = c->inlet[s];
        if (L.s[s].kind != KIND_DIRICHLET || c->inlet_set[s]) continue;
        g.dacc[s] = (double*)(base + t.off_dacc[s]);
        g.dir_any = 1;
        HIPCHK(c, hipMemsetAsync(g.dacc[s], 0, (size_t)L.M * L.s[s].len * 4 * 8, st));
    }
    const int nside_blocks = t.nadj + ((any_corner && !g.coupled) ? 4 : 0);

    // Segment seg is recomputed from its checkpoint on the second stream into recomputation set
    // seg & 1 (populations, and per step the moments and boundary states the reverse sweep
    // reads), while the caller's stream sweeps segment seg + 1 backwards from the other set.
    // Events order the two: the sweep of seg waits for its set to be filled, the recomputation
    // of seg - 1 waits for the sweep of seg + 1 to have released that set.
    auto recompute = [&](int seg) -> int {
        const int b = seg & 1;
        const int n0 = seg * t.K, n1 = std::min(n0 + t.K, t.N);
        const char* chk = base + (size_t)seg * t.chk_stride;
        T* R[2] = {(T*)(base + t.off_R[b][0]), (T*)(base + t.off_R[b][1])};
        HIPCHK(c, hipMemcpyAsync(R[0], chk, L.f_bytes, hipMemcpyDeviceToDevice, ax));
        HIPCHK(c, hipMemcpyAsync(reg_slot(b, 0), chk + L.f_bytes, L.region_bytes, hipMemcpyDeviceToDevice, ax));
        hipLaunchKernelGGL((k_adj_moments<Q, T>), dim3(bpr * ny), dim3(256), 0, ax, (const T*)R[0], mom_slot(b, 0), bk, bpr);
        HIPCHK(c, hipGetLastError());
        // the step kernel never writes Dirichlet layers (their profile is fixed): give the second
        // recomputation buffer the same layers as the checkpoint
        for (int s = 0; s < 4; ++s) {
            if (L.s[s].kind != KIND_DIRICHLET) continue;
            const int tot = L.s[s].len * L.M;
            hipLaunchKernelGGL((k_dirichlet<Q, T>), dim3((tot + 255) / 256), dim3(256), 0, ax, g.b, s, c->inlet[s], R[0], R[1]);
            HIPCHK(c, hipGetLastError());
        }
        for (int j = 0; j < n1 - n0; ++j) {
            launch_step_raw<Q, T, true>(c, R[j & 1], R[(j + 1) & 1], reg_slot(b, j), reg_slot(b, j + 1), mom_slot(b, j + 1), ax);
            HIPCHK(c, hipGetLastError());
        }
        HIPCHK(c, hipEventRecord(c->ev[b], ax));
        return LBM_OK;
    };
    HIPCHK(c, hipEventRecord(c->ev[4], st));   // the seed and the clears above come first
    HIPCHK(c, hipStreamWaitEvent(ax, c->ev[4], 0));
    int rc = recompute(t.nchk - 1);
    if (rc != LBM_OK) return rc;
    for (int seg = t.nchk - 1; seg >= 0; --seg) {
        const int b = seg & 1;
        const int n0 = seg * t.K, n1 = std::min(n0 + t.K, t.N);
        HIPCHK(c, hipStreamWaitEvent(st, c->ev[b], 0));
        if (seg > 0) {
            if (seg + 1 < t.nchk) HIPCHK(c, hipStreamWaitEvent(ax, c->ev[2 + (b ^ 1)], 0));
            rc = recompute(seg - 1);
            if (rc != LBM_OK) return rc;
        }
        for (int n = n1 - 1; n >= n0; --n) {
            const int j = n - n0;
            g.b.reg_cur = reg_slot(b, j);
            g.b.reg_next = reg_slot(b, j + 1);
            g.adj_cur = base + t.off_adj[n & 1];
            g.adj_next = base + t.off_adj[(n + 1) & 1];
            g.V1 = V[(n + 1) & 1];
            g.V0 = V[n & 1];
            g.mom = mom_slot(b, j);
            g.mom1 = mom_slot(b, j + 1);
            if (nside_blocks > 0) {
                if (any_full) hipLaunchKernelGGL((k_adj_side<Q, true>), dim3(nside_blocks), dim3(256), 0, st, g);
                else hipLaunchKernelGGL((k_adj_side<Q, false>), dim3(nside_blocks), dim3(256), 0, st, g);
                HIPCHK(c, hipGetLastError());
            }
            if (any_corner && g.coupled) {
                hipLaunchKernelGGL((k_adj_corner<Q>), dim3(4), dim3(256), 0, st, g);
                HIPCHK(c, hipGetLastError());
            }
            const dim3 grid(bpr * ny);
            if (n > 0) {
                if (px && py) hipLaunchKernelGGL((k_adj_bulk<Q, true, true, false>), grid, dim3(256), 0, st, g, bk, bpr);
                else if (px) hipLaunchKernelGGL((k_adj_bulk<Q, true, false, false>), grid, dim3(256), 0, st, g, bk, bpr);
                else if (py) hipLaunchKernelGGL((k_adj_bulk<Q, false, true, false>), grid, dim3(256), 0, st, g, bk, bpr);
                else hipLaunchKernelGGL((k_adj_bulk<Q, false, false, false>), grid, dim3(256), 0, st, g, bk, bpr);
            } else {
                if (px && py) hipLaunchKernelGGL((k_adj_bulk<Q, true, true, true>), grid, dim3(256), 0, st, g, bk, bpr);
                else if (px) hipLaunchKernelGGL((k_adj_bulk<Q, true, false, true>), grid, dim3(256), 0, st, g, bk, bpr);
                else if (py) hipLaunchKernelGGL((k_adj_bulk<Q, false, true, true>), grid, dim3(256), 0, st, g, bk, bpr);
                else hipLaunchKernelGGL((k_adj_bulk<Q, false, false, true>), grid, dim3(256), 0, st, g, bk, bpr);
            }
            HIPCHK(c, hipGetLastError());
        }
        HIPCHK(c, hipEventRecord(c->ev[2 + b], st));
    }
    for (int s = 0; s < 4; ++s) {
        if (!g.dacc[s]) continue;
        hipLaunchKernelGGL((k_adj_dir_collect<Q>), dim3((L.s[s].len + 255) / 256), dim3(256), 0, st, g, s, nx, ny);
        HIPCHK(c, hipGetLastError());
    }
    g.adj_cur = base + t.off_adj[0];
    hipLaunchKernelGGL((k_adj_final<Q>), dim3(1), dim3(256), 0, st, g);
    HIPCHK(c, hipGetLastError());
    std::vector<double> acc((size_t)2 * t.nadj + 4);
    HIPCHK(c, hipMemcpyAsync(acc.data(), base + t.off_acc, acc.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    // dK / dsigma per side, as in make_bnd
    const double cs2 = Lat<Q>::cs2;
    for (int s = 0; s < 4; ++s) {
        const lbm_relax& p = c->relax[s];
        const double cinf = Lat<Q>::thermal ? std::sqrt(2.0 * cs2 * p.T_inf) : std::sqrt(cs2);
        const double len = p.length > 0 ? p.length : (double)L.s[s].Nn;
        const double kf = (1.0 - p.mach * p.mach) * cinf / len;
        double dK = 0.0, dA = 0.0;
        for (int b = t.ablk0[s]; b < t.ablk0[s] + t.anblk[s]; ++b) { dK += acc[2 * b]; dA += acc[2 * b + 1]; }
        if (s < 2)
            for (int ci = 0; ci < 4; ++ci)
                if (L.c[ci].active && (ci & 1) == s) dK += acc[2 * t.nadj + ci];
        const bool rel = is_relax(c->cfg.bc[s]);
        h_relax[2 * s] = rel ? dK * kf : 0.0;
        h_relax[2 * s + 1] = rel ? dA : 0.0;
    }
    return LBM_OK;
}

template <typename F>
int dispatch(const lbm_ctx* c, F&& f) {
    if (c->cfg.stencil == 9) return c->cfg.precision == LBM_FP64 ? f.template operator()<9, double>() : f.template operator()<9, float>();
    if (c->cfg.stencil == 17) return c->cfg.precision == LBM_FP64 ? f.template operator()<17, double>() : f.template operator()<17, float>();
    return c->cfg.precision == LBM_FP64 ? f.template operator()<37, double>() : f.template operator()<37, float>();
}

// Diagnostics of the current state into d_out[8] (device), on the context's stream: the first
// pass writes nparts partials per quantity into `partials` (component-major, [8][nparts]), each
// work-group covering tpw consecutive 256-node row tiles (tpw = 1: one tile each, nparts = the
// tile count), the second pass folds them in a fixed order.
int enqueue_diag(lbm_ctx* c, double* partials, int nparts, int tpw, double* d_out) {
    const BulkArgs& g = c->bulk;
    const int bpr = (c->cfg.nx + 255) / 256;
    const int ntiles = c->L.diag_blocks;
    return dispatch(c, [&]<int Q, typename T>() -> int {
        if (tpw == 1)
            hipLaunchKernelGGL((k_diag_partial<Q, T, false>), dim3(nparts), dim3(256), 0, c->stream, (const T*)c->f[c->cur],
                               c->cfg.nx, bpr, c->L.pitch, g.x0, g.x1, g.y0, g.y1, partials, ntiles, 1);
        else
            hipLaunchKernelGGL((k_diag_partial<Q, T, true>), dim3(nparts), dim3(256), 0, c->stream, (const T*)c->f[c->cur],
                               c->cfg.nx, bpr, c->L.pitch, g.x0, g.x1, g.y0, g.y1, partials, ntiles, tpw);
        HIPCHK(c, hipGetLastError());
        hipLaunchKernelGGL(k_diag_final, dim3(8), dim3(1024), 0, c->stream, partials, nparts, d_out, (double)c->steps);
        HIPCHK(c, hipGetLastError());
        return LBM_OK;
    });
}

// Diagnostics into h_out[8] (host) from the workspace's scratch; synchronises the stream.
int host_diag(lbm_ctx* c, double* h_out) {
    const int nb = c->L.diag_blocks;
    const int rc = enqueue_diag(c, c->diag, nb, 1, c->diag + (size_t)nb * 8);
    if (rc != LBM_OK) return rc;
    HIPCHK(c, hipMemcpyAsync(h_out, c->diag + (size_t)nb * 8, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

}  // namespace

// =========================================================================== C ABI
extern "C" {

size_t lbm_workspace_bytes(const lbm_config* cfg) {
    std::string err;
    if (validate(cfg, err) != LBM_OK) { g_err = err; return 0; }
    Layout L;
    make_layout(cfg, L);
    return L.total;
}

int lbm_init(const lbm_config* cfg, void* d_workspace, size_t workspace_bytes, void* hip_stream, const double* d_rho0,
             const double* d_ux0, const double* d_uy0, const double* d_T0, lbm_ctx** out) {
    if (!out) return fail(nullptr, LBM_E_ARG, "out is NULL");
    *out = nullptr;
    std::string err;
    const int v = validate(cfg, err);
    if (v != LBM_OK) return fail(nullptr, v, err);
    if (!d_workspace || ((uintptr_t)d_workspace % ALIGN) != 0) return fail(nullptr, LBM_E_ARG, "workspace must be non-NULL and 256-byte aligned");
    if (!d_rho0 || !d_ux0 || !d_uy0 || (cfg->stencil != 9 && !d_T0)) return fail(nullptr, LBM_E_ARG, "initial field pointer is NULL");
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_E_ARG, "out of host memory");
    c->cfg = *cfg;
    make_layout(cfg, c->L);
    if (workspace_bytes < c->L.total) {
        delete c;
        return fail(nullptr, LBM_E_ARG, "workspace smaller than lbm_workspace_bytes(cfg)");
    }
    c->ws = (char*)d_workspace;
    c->f[0] = c->ws;
    c->f[1] = c->ws + c->L.f_bytes;
    c->region[0] = c->ws + c->L.off_region;
    c->region[1] = c->region[0] + c->L.region_bytes;
    for (int s = 0; s < 4; ++s) c->inlet[s] = (double*)(c->ws + c->L.off_inlet[s]);
    c->diag = (double*)(c->ws + c->L.off_diag);
    c->stream = (hipStream_t)hip_stream;
    {
        hipError_t e = hipGetDevice(&c->device);
        if (e == hipSuccess && (c->device < 0 || c->device >= MAX_DEVICES)) e = hipErrorInvalidDevice;
        if (e == hipSuccess) e = scratch_address(c->device, &c->scratch);
        if (e != hipSuccess) {
            delete c;
            return fail(nullptr, LBM_E_HIP, std::string("device scratch lookup: ") + hipGetErrorString(e));
        }
    }
    for (int s = 0; s < 4; ++s) c->relax[s] = lbm_relax{0.0, 0.0, 1.0, 1.0, 0.0, 0.0};
    c->nbnd = 0;
    for (int s = 0; s < 4; ++s) c->nbnd += c->L.s[s].nblk;
    const int M = c->L.M;
    const bool xp = cfg->bc[0] == BC_PERIODIC, yp = cfg->bc[2] == BC_PERIODIC;
    c->bulk.nx = cfg->nx; c->bulk.ny = cfg->ny;
    c->bulk.x0 = xp ? 0 : M; c->bulk.x1 = xp ? cfg->nx - 1 : cfg->nx - 1 - M;
    c->bulk.y0 = yp ? 0 : M; c->bulk.y1 = yp ? cfg->ny - 1 : cfg->ny - 1 - M;
    c->bulk.pitch = c->L.pitch;
    c->bulk.omega_d = 1.0 / cfg->tau;
    c->bulk.omega_f = (float)(1.0 / cfg->tau);
    const int rc = dispatch(c, [&]<int Q, typename T>() -> int { return launch_init<Q, T>(c, d_rho0, d_ux0, d_uy0, d_T0); });
    if (rc != LBM_OK) {
        g_err = c->err;
        lbm_destroy(c);
        return rc;
    }
    *out = c;
    return LBM_OK;
}

int lbm_cbc_params(lbm_ctx* c, int side, const lbm_relax* p) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (!p || side < -1 || side > 3) return fail(c, LBM_E_ARG, "bad side or params");
    const double vals[6] = {p->sigma, p->alpha, p->rho_inf, p->T_inf, p->mach, p->length};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(c, LBM_E_ARG, "non-finite relaxation parameter");
    if (!(p->rho_inf > 0) || !(p->T_inf > 0)) return fail(c, LBM_E_ARG, "rho_inf and T_inf must be positive");
    for (int s = 0; s < 4; ++s)
        if (side < 0 || s == side) c->relax[s] = *p;
    c->tape = Tape{};   // a recorded run no longer matches the boundary settings
    return LBM_OK;
}

int lbm_reconstruction(lbm_ctx* c, int side, int mode) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (side < -1 || side > 3 || (mode != LBM_RECON_EQUILIBRIUM && mode != LBM_RECON_NEEP))
        return fail(c, LBM_E_ARG, "bad side or reconstruction mode");
    for (int s = 0; s < 4; ++s) {
        if (side >= 0 && s != side) continue;
        if (mode == LBM_RECON_NEEP && c->L.s[s].kind != KIND_CHAR) {
            if (side >= 0) return fail(c, LBM_E_STATE, "NEEP applies to characteristic sides only");
            continue;
        }
        c->meso[s] = mode;
    }
    c->tape = Tape{};   // a recorded run no longer matches the boundary settings
    return LBM_OK;
}

int lbm_viscous(lbm_ctx* c, int side, int mode) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (side < -1 || side > 3 || (mode != LBM_VISC_MESO && mode != LBM_VISC_FD))
        return fail(c, LBM_E_ARG, "bad side or viscous mode");
    for (int s = 0; s < 4; ++s) {
        if (side >= 0 && s != side) continue;
        if (mode == LBM_VISC_FD && !is_full(c->cfg.bc[s])) {
            if (side >= 0) return fail(c, LBM_E_STATE, "finite-difference viscous terms apply to CBC sides only");
            continue;
        }
        c->vfd[s] = mode;
    }
    c->tape = Tape{};   // a recorded run no longer matches the boundary settings
    return LBM_OK;
}

int lbm_dirichlet_profile(lbm_ctx* c, int side, const double* d_U) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (side < 0 || side > 3 || !d_U) return fail(c, LBM_E_ARG, "bad side or profile pointer");
    if (c->L.s[side].kind != KIND_DIRICHLET) return fail(c, LBM_E_STATE, "side is not a Dirichlet side");
    const size_t bytes = (size_t)c->L.s[side].len * 4 * 8;
    HIPCHK(c, hipMemcpyAsync(c->inlet[side], d_U, bytes, hipMemcpyDeviceToDevice, c->stream));
    c->inlet_set[side] = 1;
    c->tape = Tape{};   // a recorded run no longer matches the boundary data
    return dispatch(c, [&]<int Q, typename T>() -> int {
        const BndArgs a = make_bnd(c);
        const int tot = c->L.s[side].len * c->L.M;
        hipLaunchKernelGGL((k_dirichlet<Q, T>), dim3((tot + 255) / 256), dim3(256), 0, c->stream, a, side,
                           c->inlet[side], (T*)c->f[0], (T*)c->f[1]);
        HIPCHK(c, hipGetLastError());
        return LBM_OK;
    });
}

int lbm_step(lbm_ctx* c, int nsteps) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (nsteps < 0) return fail(c, LBM_E_ARG, "nsteps < 0");
    for (int k = 0; k < nsteps; ++k) {
        const int rc = dispatch(c, [&]<int Q, typename T>() -> int { return launch_step<Q, T>(c); });
        if (rc != LBM_OK) return rc;
        if (c->diag_every > 0 && c->steps % c->diag_every == 0) {
            double out[8];
            const int rd = host_diag(c, out);
            if (rd != LBM_OK) return rd;
            if (out[6] > 0)
                return fail(c, LBM_E_NONFINITE, "non-finite populations after step " + std::to_string(c->steps));
        }
    }
    return LBM_OK;
}

int lbm_macroscopic(lbm_ctx* c, double* rho, double* ux, double* uy, double* Tf) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (!rho || !ux || !uy) return fail(c, LBM_E_ARG, "output pointer is NULL");
    const int n = c->cfg.nx * c->cfg.ny;
    return dispatch(c, [&]<int Q, typename T>() -> int {
        hipLaunchKernelGGL((k_macro<Q, T>), dim3((n + 255) / 256), dim3(256), 0, c->stream, (const T*)c->f[c->cur],
                           c->cfg.nx, n, c->L.pitch, rho, ux, uy, Tf);
        HIPCHK(c, hipGetLastError());
        return LBM_OK;
    });
}

int lbm_boundary_state(lbm_ctx* c, int side, double* d_out) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (side < 0 || side > 3 || !d_out) return fail(c, LBM_E_ARG, "bad side or output pointer");
    const SideDev& s = c->L.s[side];
    if (s.kind != KIND_CHAR) return fail(c, LBM_E_STATE, "side is not a characteristic side");
    HIPCHK(c, hipMemcpyAsync(d_out, c->region[c->cur] + s.off_ub, (size_t)c->L.M * s.len * 4 * 8, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

int lbm_diagnostics(lbm_ctx* c, double* h_out) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (!h_out) return fail(c, LBM_E_ARG, "output pointer is NULL");
    double out[8];
    const int rc = host_diag(c, out);
    if (rc != LBM_OK) return rc;
    std::memcpy(h_out, out, sizeof(out));
    if (out[6] > 0) return fail(c, LBM_E_NONFINITE, "non-finite populations");
    return LBM_OK;
}

int lbm_diagnostics_noalloc(lbm_ctx* c, double* d_out) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (!d_out) return fail(c, LBM_E_ARG, "output pointer is NULL");
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev != c->device || !c->scratch) return fail(c, LBM_E_STATE, "the context's device is not the current device");
    const int ntiles = c->L.diag_blocks;
    const int tpw = (ntiles + NOALLOC_PARTIALS - 1) / NOALLOC_PARTIALS;   // row tiles per work-group
    const int nparts = (ntiles + tpw - 1) / tpw;
    if (tpw < 1 || nparts > NOALLOC_PARTIALS) return fail(c, LBM_E_ARG, "grid too large for the fixed diagnostics scratch");
    return enqueue_diag(c, c->scratch, nparts, tpw, d_out);
}

int lbm_diag_every(lbm_ctx* c, int n) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (n < 0) return fail(c, LBM_E_ARG, "n must be 0 (off) or a positive step count");
    c->diag_every = n;
    return LBM_OK;
}

// Checkpoint layout: a 256-byte header (steps done, the four Dirichlet-profile flags), the
// current population buffer, the current boundary state region, the Dirichlet profiles.
size_t lbm_state_bytes(const lbm_ctx* c) {
    if (!c) return 0;
    return ALIGN + c->L.f_bytes + c->L.region_bytes + (c->L.off_diag - c->L.off_inlet[0]);
}

int lbm_save(lbm_ctx* c, void* d_buf) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (!d_buf) return fail(c, LBM_E_ARG, "buffer is NULL");
    char* b = (char*)d_buf;
    c->save_hdr[0] = c->steps;
    for (int s = 0; s < 4; ++s) c->save_hdr[1 + s] = c->inlet_set[s];
    HIPCHK(c, hipMemcpyAsync(b, c->save_hdr, sizeof(c->save_hdr), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b + ALIGN, c->f[c->cur], c->L.f_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(b + ALIGN + c->L.f_bytes, c->region[c->cur], c->L.region_bytes, hipMemcpyDeviceToDevice, c->stream));
    const size_t pbytes = c->L.off_diag - c->L.off_inlet[0];
    if (pbytes > 0)
        HIPCHK(c, hipMemcpyAsync(b + ALIGN + c->L.f_bytes + c->L.region_bytes, c->ws + c->L.off_inlet[0], pbytes,
                                 hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_restore(lbm_ctx* c, const void* d_buf) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (!d_buf) return fail(c, LBM_E_ARG, "buffer is NULL");
    const char* b = (const char*)d_buf;
    long hdr[8];
    HIPCHK(c, hipMemcpyAsync(hdr, b, sizeof(hdr), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->f[0], b + ALIGN, c->L.f_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->region[0], b + ALIGN + c->L.f_bytes, c->L.region_bytes, hipMemcpyDeviceToDevice, c->stream));
    const size_t pbytes = c->L.off_diag - c->L.off_inlet[0];
    if (pbytes > 0)
        HIPCHK(c, hipMemcpyAsync(c->ws + c->L.off_inlet[0], b + ALIGN + c->L.f_bytes + c->L.region_bytes, pbytes,
                                 hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->cur = 0;
    c->steps = hdr[0];
    for (int s = 0; s < 4; ++s) c->inlet_set[s] = (int)hdr[1 + s];
    c->tape = Tape();
    // the step kernel never writes the layers of a Dirichlet side: both population buffers get
    // the equilibrium of the restored profile
    return dispatch(c, [&]<int Q, typename T>() -> int {
        const BndArgs a = make_bnd(c);
        for (int s = 0; s < 4; ++s) {
            if (c->L.s[s].kind != KIND_DIRICHLET) continue;
            const int tot = c->L.s[s].len * c->L.M;
            hipLaunchKernelGGL((k_dirichlet<Q, T>), dim3((tot + 255) / 256), dim3(256), 0, c->stream, a, s, c->inlet[s],
                               (T*)c->f[0], (T*)c->f[1]);
            HIPCHK(c, hipGetLastError());
        }
        return LBM_OK;
    });
}

size_t lbm_tape_bytes(const lbm_ctx* c, int nsteps, int every) {
    if (!c || nsteps < 1 || every < 1) return 0;
    Tape t;
    tape_layout(c->L, c->cfg.nx, c->cfg.ny, nsteps, std::min(every, nsteps), t);
    return t.total;
}

int lbm_record(lbm_ctx* c, int nsteps, int every, void* d_tape, size_t tape_bytes) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    std::string err;
    const int sup = adjoint_supported(c, err);
    if (sup != LBM_OK) return fail(c, sup, err);
    if (nsteps < 1 || every < 1) return fail(c, LBM_E_ARG, "nsteps and every must be positive");
    if (!d_tape || ((uintptr_t)d_tape % ALIGN) != 0) return fail(c, LBM_E_ARG, "tape must be non-NULL and 256-byte aligned");
    if (c->steps != 0) return fail(c, LBM_E_STATE, "recording starts from the initial state (no steps taken)");
    Tape t;
    tape_layout(c->L, c->cfg.nx, c->cfg.ny, nsteps, std::min(every, nsteps), t);
    if (tape_bytes < t.total) return fail(c, LBM_E_ARG, "tape smaller than lbm_tape_bytes");
    t.base = (char*)d_tape;
    for (int n = 0; n < nsteps; ++n) {
        if (n % t.K == 0) {
            char* chk = t.base + (size_t)(n / t.K) * t.chk_stride;
            HIPCHK(c, hipMemcpyAsync(chk, c->f[c->cur], c->L.f_bytes, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(chk + c->L.f_bytes, c->region[c->cur], c->L.region_bytes, hipMemcpyDeviceToDevice, c->stream));
        }
        const int rc = dispatch(c, [&]<int Q, typename T>() -> int { return launch_step<Q, T>(c); });
        if (rc != LBM_OK) return rc;
    }
    t.step_end = c->steps;
    c->tape = t;
    return LBM_OK;
}

int lbm_adjoint(lbm_ctx* c, const double* d_seed, double* d_grad_fields, double* h_grad_relax) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (!d_grad_fields || !h_grad_relax) return fail(c, LBM_E_ARG, "output pointer is NULL");
    if (!c->tape.base) return fail(c, LBM_E_STATE, "no recorded run (call lbm_record first)");
    if (c->steps != c->tape.step_end) return fail(c, LBM_E_STATE, "the context has stepped since lbm_record");
    std::string err;
    const int sup = adjoint_supported(c, err);
    if (sup != LBM_OK) return fail(c, sup, err);
    return dispatch(c, [&]<int Q, typename T>() -> int { return run_adjoint<Q, T>(c, d_seed, d_grad_fields, h_grad_relax); });
}

long lbm_steps_done(const lbm_ctx* c) { return c ? c->steps : -1; }

int lbm_set_kernel_timing(lbm_ctx* c, int enable) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (enable < 0) return fail(c, LBM_E_ARG, "enable must be 0 or a positive stride");
    c->timing = enable;
    c->tcount = 0;
    c->tcalls = 0;
    return LBM_OK;
}

int lbm_bulk_kernel_time(lbm_ctx* c, double* total_ms, long* launches) {
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (!total_ms || !launches) return fail(c, LBM_E_ARG, "output pointer is NULL");
    double sum = 0.0;
    for (size_t k = 0; k < c->tcount; ++k) {
        HIPCHK(c, hipEventSynchronize(c->tev[2 * k + 1]));
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->tev[2 * k], c->tev[2 * k + 1]));
        sum += ms;
    }
    *total_ms = sum;
    *launches = (long)c->tcount;
    return LBM_OK;
}

int lbm_lattice_info(int stencil, int* M, double* cs2, double* w, int* cxo, int* cyo) {
    if (stencil == 9) {
        if (M) *M = 1;
        if (cs2) *cs2 = Lat<9>::cs2;
        for (int i = 0; i < 9; ++i) { if (w) w[i] = wt<9>(i); if (cxo) cxo[i] = cx<9>(i); if (cyo) cyo[i] = cy<9>(i); }
        return 9;
    }
    if (stencil == 17) {
        if (M) *M = 3;
        if (cs2) *cs2 = Lat<17>::cs2;
        for (int i = 0; i < 17; ++i) { if (w) w[i] = wt<17>(i); if (cxo) cxo[i] = cx<17>(i); if (cyo) cyo[i] = cy<17>(i); }
        return 17;
    }
    if (stencil == 37) {
        if (M) *M = 3;
        if (cs2) *cs2 = Lat<37>::cs2;
        for (int i = 0; i < 37; ++i) { if (w) w[i] = wt<37>(i); if (cxo) cxo[i] = cx<37>(i); if (cyo) cyo[i] = cy<37>(i); }
        return 37;
    }
    g_err = "unknown stencil";
    return LBM_E_ARG;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

void lbm_destroy(lbm_ctx* c) {
    if (!c) return;
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    if (c->aux) {
        (void)hipStreamSynchronize(c->aux);
        for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(c->aux);
    }
    delete c;
}

}  // extern "C"
