// lbm3d.hip -- host side of the three-dimensional C ABI (include/lbm3d.h) in liblbm_hip.so.
//
// The caller's workspace holds two population buffers, two parity copies of the face state, the
// RK4 stage buffers, the viscous terms, the diagnostics scratch, the staged layer populations and
// the compact face strips.  One step is the bulk kernel
// followed by the face kernels, all on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels3.h"
#include "lbm3d.h"

using namespace lbm3;

namespace {

std::string g_err3;
constexpr size_t ALIGN3 = 256;
size_t al3(size_t v) { return (v + ALIGN3 - 1) / ALIGN3 * ALIGN3; }

struct Layout3 {
    size_t esz = 0;
    unsigned long long pitch = 0;
    int rows = 0;
    size_t f_bytes = 0, region_bytes = 0, off_region = 0, off_Ya = 0, off_Yb = 0, off_V = 0, off_diag = 0, total = 0;
    size_t off_lay = 0;   // staged layer populations of the new level [face][rows][M][Q] (storage type)
    size_t off_strip = 0; // face strips [face][rows][sm.blk] (storage type; see StripMap3)
    int diag_blocks = 0;
    Face3 f[2];
    StripMap3 sm;
};

// the configuration on the library's internal grid: the face axis becomes x, the two axes that
// follow it cyclically become y and z
lbm3d_config internal3(const lbm3d_config* u) {
    lbm3d_config c = *u;
    const int d[3] = {u->nx, u->ny, u->nz}, a = u->axis;
    c.nx = d[a]; c.ny = d[(a + 1) % 3]; c.nz = d[(a + 2) % 3];
    c.axis = 0;
    return c;
}

int validate3(const lbm3d_config* u, std::string& err) {
    if (!u) { err = "null config"; return LBM_E_ARG; }
    if (u->axis < 0 || u->axis > 2) { err = "axis must be 0 (x), 1 (y) or 2 (z)"; return LBM_E_ARG; }
    const lbm3d_config ic = internal3(u);
    const lbm3d_config* c = &ic;
    if (c->stencil != LBM_D3Q39) { err = "stencil must be LBM_D3Q39"; return LBM_E_ARG; }
    if (c->precision != LBM_FP64 && c->precision != LBM_FP32DEV) { err = "unknown precision"; return LBM_E_ARG; }
    if (!(c->tau > 0.5) || !std::isfinite(c->tau)) { err = "tau must be a finite value above 1/2"; return LBM_E_ARG; }
    for (int s = 0; s < 2; ++s)
        if (c->bc[s] != LBM_BC_PERIODIC && c->bc[s] != LBM_BC_LODI && c->bc[s] != LBM_BC_LODI_RELAX &&
            c->bc[s] != LBM_BC_CBC && c->bc[s] != LBM_BC_CBC_RELAX && c->bc[s] != LBM_BC_ZG) {
            err = "face type must be periodic, LODI, LODI_RELAX, CBC, CBC_RELAX or ZG"; return LBM_E_ARG;
        }
    if ((c->bc[0] == LBM_BC_PERIODIC) != (c->bc[1] == LBM_BC_PERIODIC)) { err = "periodic faces must come in pairs"; return LBM_E_ARG; }
    const bool xp = c->bc[0] == LBM_BC_PERIODIC;
    if (c->nx < (xp ? L3::M + 1 : 2 * L3::M + 3) || c->ny < L3::M + 1 || c->nz < L3::M + 1) { err = "grid too small"; return LBM_E_ARG; }
    // the viscous terms of a CBC face are evaluated at x_f - M .. x_f - M - 2, which must be bulk nodes
    if ((c->bc[0] == LBM_BC_CBC || c->bc[0] == LBM_BC_CBC_RELAX || c->bc[1] == LBM_BC_CBC || c->bc[1] == LBM_BC_CBC_RELAX) &&
        c->nx < 3 * L3::M + 3) { err = "CBC faces need 3M + 3 nodes across"; return LBM_E_ARG; }
    const double n = (double)c->nx * (double)c->ny * (double)c->nz;
    if (n > 2.0e9) { err = "grid too large"; return LBM_E_ARG; }
    const unsigned long long bpr = ((unsigned long long)c->nx + 255) / 256;
    const unsigned long long rows = (unsigned long long)c->ny * (unsigned long long)c->nz;
    if (bpr * bpr * rows >= (1ull << 32) || bpr * rows >= (1ull << 31)) {
        err = "grid too large for the bulk kernel's tile indexing"; return LBM_E_UNSUPPORTED;
    }
    return LBM_OK;
}

void make_layout3(const lbm3d_config* c, Layout3& L) {
    L.esz = c->precision == LBM_FP64 ? 8 : 4;
    L.pitch = ((unsigned long long)c->nx + 63) / 64 * 64;
    L.rows = c->ny * c->nz;
    L.f_bytes = al3((size_t)L3::Q * L.pitch * L.rows * L.esz);
    size_t reg = 0;
    for (int s = 0; s < 2; ++s) {
        Face3& f = L.f[s];
        std::memset(&f, 0, sizeof(f));
        f.scheme = c->bc[s];
        f.sn = s == 0 ? -1 : 1;
        f.xf = s == 0 ? L3::M : c->nx - 1 - L3::M;
        if (c->bc[s] >= LBM_BC_LODI && c->bc[s] <= LBM_BC_CBC_RELAX) {
            f.off_ub = reg; reg += al3((size_t)L3::M * L.rows * 5 * 8);
            f.off_strip = reg; reg += al3((size_t)L.rows * 5 * 8);
            if (c->bc[s] == LBM_BC_CBC || c->bc[s] == LBM_BC_CBC_RELAX) { f.off_vis = reg; reg += al3((size_t)3 * L.rows * 10 * 8); }
        }
    }
    L.region_bytes = al3(reg == 0 ? ALIGN3 : reg);
    L.off_region = 2 * L.f_bytes;
    L.off_Ya = L.off_region + 2 * L.region_bytes;
    L.off_Yb = L.off_Ya + al3((size_t)2 * L3::M * L.rows * 5 * 8);
    L.off_V = L.off_Yb + al3((size_t)2 * L3::M * L.rows * 5 * 8);
    L.off_diag = L.off_V + al3((size_t)2 * L.rows * 5 * 8);
    L.diag_blocks = 1024;
    L.off_lay = L.off_diag + al3((size_t)(L.diag_blocks + 1) * 8 * 8);
    std::memset(&L.sm, 0, sizeof(L.sm));
    bool any = false;
    for (int s = 0; s < 2; ++s) {
        const int b = c->bc[s];
        const bool ch = b >= LBM_BC_LODI && b <= LBM_BC_CBC_RELAX, full = b == LBM_BC_CBC || b == LBM_BC_CBC_RELAX;
        L.sm.nk[s] = !ch || L.esz != 8 ? 0 : full ? 4 : 1;   // strips in FP64 storage only (see StripMap3)
        L.sm.xf[s] = L.f[s].xf;
        L.sm.sn[s] = L.f[s].sn;
        // x of the pulled nodes X_k - c_x, |c_x| <= M: x_f - 3 .. x_f + 3 with the strip node only,
        // also the three viscous-moment nodes inward of it otherwise
        L.sm.w[s] = L.sm.nk[s] == 4 ? 12 : 7;
        L.sm.lo[s] = (s == 0 || L.sm.nk[s] != 4) ? L.f[s].xf - L3::M : L.f[s].xf - L3::M - (L3::M + 2);
        any = any || L.sm.nk[s] > 0;
    }
    for (int s = 0; s < 2; ++s)
        L.sm.blk[s] = (int)((((size_t)L3::Q * L.sm.nk[s] * L.esz + 127) / 128 * 128) / L.esz);
    L.off_strip = L.off_lay + al3((size_t)2 * L.rows * L3::M * L3::Q * L.esz);
    L.total = L.off_strip + (any ? al3((size_t)L.rows * (L.sm.blk[0] + L.sm.blk[1]) * L.esz) : 0);
}

}  // namespace

struct lbm3d_ctx {
    lbm3d_config cfg;              // on the internal grid (faces normal to its x axis)
    int axis = 0;                  // the caller's face axis
    UStride3 us;                   // caller index of internal nodes
    VMap3 vm;                      // library velocity of each caller-frame velocity
    Layout3 L;
    char* ws = nullptr;
    void* f[2] = {nullptr, nullptr};
    char* region[2] = {nullptr, nullptr};
    double* diag = nullptr;
    int cur = 0;
    long steps = 0;
    hipStream_t stream = nullptr;
    lbm_relax relax[2];
    int meso[2] = {0, 0};
    std::string err;
    int timing = 0;                // time every timing-th bulk launch (0: off)
    size_t tcalls = 0;             // bulk launches since timing was set
    std::vector<hipEvent_t> tev;
    size_t tcount = 0;
};

namespace {

int fail3(lbm3d_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg; else g_err3 = msg;
    return code;
}

#define HIPCHK3(ctx, call)                                                                 \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return fail3(ctx, LBM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

Args3 make_args3(const lbm3d_ctx* c) {
    Args3 a;
    std::memset(&a, 0, sizeof(a));
    a.nx = c->cfg.nx; a.ny = c->cfg.ny; a.nz = c->cfg.nz;
    a.xper = c->cfg.bc[0] == LBM_BC_PERIODIC;
    a.rows = c->L.rows;
    a.pitch = c->L.pitch;
    a.omega = 1.0 / c->cfg.tau;
    a.tau = c->cfg.tau;
    a.reg_cur = c->region[c->cur];
    a.reg_next = c->region[c->cur ^ 1];
    a.Ya = (double*)(c->ws + c->L.off_Ya);
    a.Yb = (double*)(c->ws + c->L.off_Yb);
    a.V = (double*)(c->ws + c->L.off_V);
    for (int s = 0; s < 2; ++s) {
        a.f[s] = c->L.f[s];
        const lbm_relax& p = c->relax[s];
        const double cinf = std::sqrt(GAMMA * L3::cs2 * p.T_inf);
        const double len = p.length > 0 ? p.length : (double)c->cfg.nx;
        a.f[s].K = p.sigma * (1.0 - p.mach * p.mach) * cinf / len;
        a.f[s].alpha = p.alpha;
        a.f[s].Pinf = p.rho_inf * L3::cs2 * p.T_inf;
        a.f[s].meso = c->meso[s];
    }
    return a;
}

Bulk3 make_bulk3(const lbm3d_ctx* c) {
    Bulk3 g;
    const bool xp = c->cfg.bc[0] == LBM_BC_PERIODIC;
    g.nx = c->cfg.nx; g.ny = c->cfg.ny; g.nz = c->cfg.nz;
    g.x0 = xp ? 0 : L3::M;
    g.x1 = xp ? c->cfg.nx - 1 : c->cfg.nx - 1 - L3::M;
    g.pitch = c->L.pitch;
    g.omega_d = 1.0 / c->cfg.tau;
    g.omega_f = (float)(1.0 / c->cfg.tau);
    g.rows = c->L.rows;
    g.lay = c->ws + c->L.off_lay;
    g.strip = (c->L.sm.nk[0] || c->L.sm.nk[1]) ? (void*)(c->ws + c->L.off_strip) : nullptr;
    return g;
}

template <typename F>
int dispatch3(const lbm3d_ctx* c, F&& f) {
    return c->cfg.precision == LBM_FP64 ? f.template operator()<double>() : f.template operator()<float>();
}

template <typename T>
int launch_step3(lbm3d_ctx* c) {
    const T* A = (const T*)c->f[c->cur];
    T* B = (T*)c->f[c->cur ^ 1];
    const Args3 a = make_args3(c);
    const Bulk3 g = make_bulk3(c);
    const int rows = c->L.rows;
    const int bpr = (g.nx + 255) / 256;
    const unsigned magic = bpr > 1 ? (unsigned)((1ull << 32) / (unsigned long long)bpr + 1ull) : 0u;
    const unsigned nblk = (unsigned)bpr * (unsigned)rows;
    // faces first (they read only A): characteristic solve, then the layers' new populations,
    // staged for the bulk kernel's boundary-layer lanes
    if (!a.xper) {
        if (c->cfg.bc[0] != LBM_BC_ZG || c->cfg.bc[1] != LBM_BC_ZG) {
            hipLaunchKernelGGL((k3_prep<T>), dim3((4 * rows + 255) / 256, 2), dim3(256), 0, c->stream, A,
                               g.strip ? (const T*)g.strip : nullptr, c->L.sm, a);
            HIPCHK3(c, hipGetLastError());
            for (int st = 0; st < 4; ++st) {
                hipLaunchKernelGGL(k3_stage, dim3((L3::M * rows + 255) / 256, 2), dim3(256), 0, c->stream, a, st);
                HIPCHK3(c, hipGetLastError());
            }
        }
        hipLaunchKernelGGL((k3_final<T>), dim3((L3::M * rows + 255) / 256, 2), dim3(256), 0, c->stream, A,
                           (T*)(c->ws + c->L.off_lay), a);
        HIPCHK3(c, hipGetLastError());
    }
    const bool rec = c->timing > 0 && (c->tcalls++ % (size_t)c->timing) == 0 && c->tcount < 65536;
    if (rec) {
        while (c->tev.size() < 2 * (c->tcount + 1)) {
            hipEvent_t e;
            HIPCHK3(c, hipEventCreate(&e));
            c->tev.push_back(e);
        }
        HIPCHK3(c, hipEventRecord(c->tev[2 * c->tcount], c->stream));
    }
    // FP32: an unused dynamic LDS reservation of 54000 bytes caps the bulk kernel at 3 work-groups
    // per CU (160 KiB of LDS), where the many-stream pull pattern streams best (73.6 % against
    // 71.2 % at the register-limited 5 per CU on 512 x 256 x 256); FP64 is at 2 per CU anyway.
    // (less the kernel's own static LDS for the face strips)
    const unsigned lds = sizeof(T) == 4 ? 54000u - (unsigned)(sizeof(T) * (2 * 12 * L3::Q)) : 0u;
    if (a.xper) hipLaunchKernelGGL((k3_bulk<T, true>), dim3(nblk), dim3(256), lds, c->stream, A, B, g, c->L.sm, bpr, magic);
    else hipLaunchKernelGGL((k3_bulk<T, false>), dim3(nblk), dim3(256), lds, c->stream, A, B, g, c->L.sm, bpr, magic);
    HIPCHK3(c, hipGetLastError());
    if (rec) {
        HIPCHK3(c, hipEventRecord(c->tev[2 * c->tcount + 1], c->stream));
        c->tcount += 1;
    }
    c->cur ^= 1;
    c->steps += 1;
    return LBM_OK;
}

}  // namespace

// =========================================================================== C ABI
extern "C" {

size_t lbm3d_workspace_bytes(const lbm3d_config* cfg) {
    std::string err;
    if (validate3(cfg, err) != LBM_OK) { g_err3 = err; return 0; }
    const lbm3d_config ic = internal3(cfg);
    Layout3 L;
    make_layout3(&ic, L);
    return L.total;
}

int lbm3d_init(const lbm3d_config* cfg, void* d_workspace, size_t workspace_bytes, void* hip_stream,
               const double* d_rho0, const double* d_ux0, const double* d_uy0, const double* d_uz0,
               const double* d_T0, lbm3d_ctx** out) {
    if (!out) return fail3(nullptr, LBM_E_ARG, "out is NULL");
    *out = nullptr;
    std::string err;
    const int v = validate3(cfg, err);
    if (v != LBM_OK) return fail3(nullptr, v, err);
    if (!d_workspace || ((uintptr_t)d_workspace % ALIGN3) != 0) return fail3(nullptr, LBM_E_ARG, "workspace must be non-NULL and 256-byte aligned");
    if (!d_rho0 || !d_ux0 || !d_uy0 || !d_uz0 || !d_T0) return fail3(nullptr, LBM_E_ARG, "initial field pointer is NULL");
    lbm3d_ctx* c = new (std::nothrow) lbm3d_ctx();
    if (!c) return fail3(nullptr, LBM_E_ARG, "out of host memory");
    c->cfg = internal3(cfg);
    c->axis = cfg->axis;
    {
        const long long ustr[3] = {1, cfg->nx, (long long)cfg->nx * cfg->ny};
        for (int k = 0; k < 3; ++k) c->us.s[k] = ustr[(c->axis + k) % 3];
        // caller-frame velocity j = (c_x, c_y, c_z) is the internal velocity with components
        // (c[axis], c[axis + 1], c[axis + 2])
        for (int j = 0; j < L3::Q; ++j) {
            const int cu[3] = {cx3(j), cy3(j), cz3(j)};
            const int ci[3] = {cu[c->axis], cu[(c->axis + 1) % 3], cu[(c->axis + 2) % 3]};
            c->vm.i[j] = -1;
            for (int i = 0; i < L3::Q; ++i)
                if (cx3(i) == ci[0] && cy3(i) == ci[1] && cz3(i) == ci[2]) c->vm.i[j] = i;
            if (c->vm.i[j] < 0) {   // the velocity set is closed under axis permutations
                delete c;
                return fail3(nullptr, LBM_E_UNSUPPORTED, "velocity set not closed under the axis permutation");
            }
        }
    }
    make_layout3(&c->cfg, c->L);
    if (workspace_bytes < c->L.total) {
        delete c;
        return fail3(nullptr, LBM_E_ARG, "workspace smaller than lbm3d_workspace_bytes(cfg)");
    }
    c->ws = (char*)d_workspace;
    c->f[0] = c->ws;
    c->f[1] = c->ws + c->L.f_bytes;
    c->region[0] = c->ws + c->L.off_region;
    c->region[1] = c->region[0] + c->L.region_bytes;
    c->diag = (double*)(c->ws + c->L.off_diag);
    c->stream = (hipStream_t)hip_stream;
    for (int s = 0; s < 2; ++s) c->relax[s] = lbm_relax{0.0, 0.0, 1.0, 1.0, 0.0, 0.0};
    const long long n = (long long)cfg->nx * cfg->ny * cfg->nz;
    // velocity components on the internal axes
    const double* uin[3] = {d_ux0, d_uy0, d_uz0};
    const double* u0 = uin[c->axis];
    const double* u1 = uin[(c->axis + 1) % 3];
    const double* u2 = uin[(c->axis + 2) % 3];
    const int rc = dispatch3(c, [&]<typename T>() -> int {
        hipLaunchKernelGGL((k3_init<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, d_rho0, u0, u1, u2,
                           d_T0, (T*)c->f[0], (T*)c->f[1], c->cfg.nx, c->cfg.ny, n, c->L.pitch, c->us);
        HIPCHK3(c, hipGetLastError());
        const Args3 a = make_args3(c);
        hipLaunchKernelGGL(k3_init_faces, dim3((c->L.rows + 255) / 256, 2), dim3(256), 0, c->stream, a, d_rho0, u0, u1, u2,
                           d_T0, c->us);
        HIPCHK3(c, hipGetLastError());
        const Bulk3 g = make_bulk3(c);
        if (g.strip) {   // the face strips of f^0, which the first step's k3_prep reads
            const long long ne = (long long)c->L.rows * L3::Q * 4;   // covers either face's entries
            hipLaunchKernelGGL((k3_fill_strip<T>), dim3((unsigned)((ne + 255) / 256), 2), dim3(256), 0, c->stream,
                               (const T*)c->f[0], g, c->L.sm);
            HIPCHK3(c, hipGetLastError());
        }
        return LBM_OK;
    });
    if (rc != LBM_OK) {
        g_err3 = c->err;
        lbm3d_destroy(c);
        return rc;
    }
    *out = c;
    return LBM_OK;
}

int lbm3d_cbc_params(lbm3d_ctx* c, int face, const lbm_relax* p) {
    if (!c) return fail3(nullptr, LBM_E_ARG, "null context");
    if (!p || face < -1 || face > 1) return fail3(c, LBM_E_ARG, "bad face or params");
    const double vals[6] = {p->sigma, p->alpha, p->rho_inf, p->T_inf, p->mach, p->length};
    for (double v : vals)
        if (!std::isfinite(v)) return fail3(c, LBM_E_ARG, "non-finite relaxation parameter");
    if (!(p->rho_inf > 0) || !(p->T_inf > 0)) return fail3(c, LBM_E_ARG, "rho_inf and T_inf must be positive");
    for (int s = 0; s < 2; ++s)
        if (face < 0 || s == face) c->relax[s] = *p;
    return LBM_OK;
}

int lbm3d_reconstruction(lbm3d_ctx* c, int face, int mode) {
    if (!c) return fail3(nullptr, LBM_E_ARG, "null context");
    if (face < -1 || face > 1 || (mode != LBM_RECON_EQUILIBRIUM && mode != LBM_RECON_NEEP))
        return fail3(c, LBM_E_ARG, "bad face or reconstruction mode");
    for (int s = 0; s < 2; ++s) {
        if (face >= 0 && s != face) continue;
        const int b = c->cfg.bc[s];
        if (mode == LBM_RECON_NEEP && !(b >= LBM_BC_LODI && b <= LBM_BC_CBC_RELAX)) {
            if (face >= 0) return fail3(c, LBM_E_STATE, "NEEP applies to characteristic faces only");
            continue;
        }
        c->meso[s] = mode;
    }
    return LBM_OK;
}

int lbm3d_step(lbm3d_ctx* c, int nsteps) {
    if (!c) return fail3(nullptr, LBM_E_ARG, "null context");
    if (nsteps < 0) return fail3(c, LBM_E_ARG, "nsteps < 0");
    for (int k = 0; k < nsteps; ++k) {
        const int rc = dispatch3(c, [&]<typename T>() -> int { return launch_step3<T>(c); });
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}

int lbm3d_macroscopic(lbm3d_ctx* c, double* rho, double* ux, double* uy, double* uz, double* Tf) {
    if (!c) return fail3(nullptr, LBM_E_ARG, "null context");
    if (!rho || !ux || !uy || !uz || !Tf) return fail3(c, LBM_E_ARG, "output pointer is NULL");
    const long long n = (long long)c->cfg.nx * c->cfg.ny * c->cfg.nz;
    double* uo[3] = {ux, uy, uz};
    return dispatch3(c, [&]<typename T>() -> int {
        hipLaunchKernelGGL((k3_macro<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, (const T*)c->f[c->cur],
                           c->cfg.nx, c->cfg.ny, n, c->L.pitch, rho, uo[c->axis], uo[(c->axis + 1) % 3],
                           uo[(c->axis + 2) % 3], Tf, c->us);
        HIPCHK3(c, hipGetLastError());
        return LBM_OK;
    });
}

int lbm3d_populations(lbm3d_ctx* c, double* d_out) {
    if (!c) return fail3(nullptr, LBM_E_ARG, "null context");
    if (!d_out) return fail3(c, LBM_E_ARG, "output pointer is NULL");
    const long long n = (long long)c->cfg.nx * c->cfg.ny * c->cfg.nz;
    return dispatch3(c, [&]<typename T>() -> int {
        hipLaunchKernelGGL((k3_pops<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, (const T*)c->f[c->cur],
                           c->cfg.nx, c->cfg.ny, n, c->L.pitch, d_out, c->us, c->vm);
        HIPCHK3(c, hipGetLastError());
        return LBM_OK;
    });
}

int lbm3d_diagnostics(lbm3d_ctx* c, double* h_out) {
    if (!c) return fail3(nullptr, LBM_E_ARG, "null context");
    if (!h_out) return fail3(c, LBM_E_ARG, "output pointer is NULL");
    const Bulk3 g = make_bulk3(c);
    const int nb = c->L.diag_blocks;
    const long long n = (long long)c->cfg.nx * c->cfg.ny * c->cfg.nz;
    const int rc = dispatch3(c, [&]<typename T>() -> int {
        hipLaunchKernelGGL((k3_diag_partial<T>), dim3(nb), dim3(256), 0, c->stream, (const T*)c->f[c->cur], c->cfg.nx,
                           c->cfg.ny, n, c->L.pitch, g.x0, g.x1, c->diag);
        HIPCHK3(c, hipGetLastError());
        hipLaunchKernelGGL(k3_diag_final, dim3(8), dim3(1024), 0, c->stream, c->diag, nb, c->diag + (size_t)nb * 8);
        HIPCHK3(c, hipGetLastError());
        return LBM_OK;
    });
    if (rc != LBM_OK) return rc;
    double out[8];
    HIPCHK3(c, hipMemcpyAsync(out, c->diag + (size_t)nb * 8, sizeof(out), hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    // momentum components of the internal axes to the caller's
    const double j[3] = {out[1], out[2], out[3]};
    for (int k = 0; k < 3; ++k) out[1 + (c->axis + k) % 3] = j[k];
    std::memcpy(h_out, out, sizeof(out));
    if (out[7] > 0) return fail3(c, LBM_E_NONFINITE, "non-finite populations");
    return LBM_OK;
}

int lbm3d_set_kernel_timing(lbm3d_ctx* c, int enable) {
    if (!c) return fail3(nullptr, LBM_E_ARG, "null context");
    if (enable < 0) return fail3(c, LBM_E_ARG, "enable must be 0 or a positive stride");
    c->timing = enable;
    c->tcount = 0;
    c->tcalls = 0;
    return LBM_OK;
}

int lbm3d_bulk_kernel_time(lbm3d_ctx* c, double* total_ms, long* launches) {
    if (!c) return fail3(nullptr, LBM_E_ARG, "null context");
    if (!total_ms || !launches) return fail3(c, LBM_E_ARG, "output pointer is NULL");
    HIPCHK3(c, hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (size_t k = 0; k < c->tcount; ++k) {
        float ms = 0.0f;
        HIPCHK3(c, hipEventElapsedTime(&ms, c->tev[2 * k], c->tev[2 * k + 1]));
        sum += ms;
    }
    *total_ms = sum;
    *launches = (long)c->tcount;
    return LBM_OK;
}

int lbm3d_lattice_info(int stencil, int* M, double* cs2, double* w, int* cxo, int* cyo, int* czo) {
    if (stencil != LBM_D3Q39) { g_err3 = "unknown stencil"; return LBM_E_ARG; }
    if (M) *M = L3::M;
    if (cs2) *cs2 = L3::cs2;
    for (int i = 0; i < L3::Q; ++i) {
        if (w) w[i] = wt3(i);
        if (cxo) cxo[i] = cx3(i);
        if (cyo) cyo[i] = cy3(i);
        if (czo) czo[i] = cz3(i);
    }
    return L3::Q;
}

const char* lbm3d_last_error(const lbm3d_ctx* c) { return c ? c->err.c_str() : g_err3.c_str(); }

void lbm3d_destroy(lbm3d_ctx* c) {
    if (!c) return;
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
