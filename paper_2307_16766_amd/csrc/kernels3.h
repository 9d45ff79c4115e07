// kernels3.h -- HIP kernels of the three-dimensional path (Appendix A): thermal BGK on D3Q39
// with characteristic (LODI / CBC) boundaries on the two x-faces of a box periodic in y and z.
//
// Data layout in HBM: populations as deviations f - w_i, row-interleaved SoA f[z][y][i][x] (a
// "row" is one (y, z) pair; its q planes are contiguous, the x pitch is padded to 64 elements).
// Face state (FP64, two parity copies): U_b[M][rows][5], the bulk value of x_f [rows][5] and the
// viscous moments of x_f - M, x_f - M - 1, x_f - M - 2 [3][rows][10] (CBC schemes); RK4 stage inputs and the
// viscous terms are single buffers.
//
// One time step = face kernels, which need only the old level A: k3_prep (strip and viscous
// moments of the new level from pulls of A -- in FP64, read from the compact face strips that the
// previous bulk launch wrote, see StripMap3 --, viscous terms of the old level), four k3_stage
// launches (one per RK4 stage of the coupled face system) and k3_final (new layer populations:
// equilibrium, eq. NEEP or zero gradient, staged in a small buffer); then the bulk kernel (fused
// pull-stream + moments + BGK, HBM-bound), whose boundary-layer lanes store the staged layer
// populations with the bulk's own whole-line stores.  Separate launches replace the
// halo recomputation of the two-dimensional boundary chunks: a face couples its rows in y and z,
// so a chunk's halo would grow in two directions, while the face work is a small fraction of a
// 3D step.
#pragma once

#include "lattice3.h"

namespace lbm3 {

enum { F3_PERIODIC = 0, F3_LODI = 1, F3_LODI_RELAX = 2, F3_CBC = 3, F3_CBC_RELAX = 4, F3_ZG = 5 };
constexpr double CV = 1.5, GAMMA = 5.0 / 3.0;   // c_v = d/2, gamma = c_p / c_v in d = 3

struct Face3 {
    int scheme, meso, sn, xf;    // xf: bulk node next to the layers; layer j at xf + sn j
    double K, alpha, Pinf;       // relaxation (eq. LODI-Relax / CBC-Relax)
    unsigned long long off_ub, off_strip, off_vis;   // byte offsets inside one parity region
};

struct Args3 {
    int nx, ny, nz, xper, rows;
    unsigned long long pitch;
    double omega, tau;
    char* reg_cur;
    char* reg_next;
    double* Ya;   // RK4 stage inputs [2][M][rows][5]
    double* Yb;
    double* V;    // viscous terms of the old level [2][rows][5]
    Face3 f[2];
};

// Caller arrays [nz][ny][nx] (x fastest) indexed from the library's internal grid, whose x axis is
// the axis normal to the faces: the caller's linear index of internal node (x, y, z) is
// x s[0] + y s[1] + z s[2]; with faces normal to x, s = (1, nx, nx ny).
struct UStride3 {
    long long s[3];
};

// library velocity index of each velocity of the caller's frame (populations output)
struct VMap3 {
    int i[39];
};

__device__ __forceinline__ int wrap3(int v, int n) {
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

__device__ __forceinline__ unsigned long long pix3(unsigned long long pitch, int ny, int i, int x, int y, int z) {
    return (((unsigned long long)z * ny + y) * L3::Q + i) * pitch + x;
}

__device__ __forceinline__ bool is_char3(int b) { return b >= F3_LODI && b <= F3_CBC_RELAX; }
__device__ __forceinline__ bool is_full3(int b) { return b == F3_CBC || b == F3_CBC_RELAX; }

// pull of one node at the new level (FP64), periodic in y and z, in x when configured
template <typename T>
__device__ __forceinline__ void pull3(const T* __restrict__ A, const Args3& a, int x, int y, int z, double* d) {
#pragma unroll
    for (int i = 0; i < L3::Q; ++i) {
        int xs = x - cx3(i);
        if (a.xper) xs = wrap3(xs, a.nx);
        d[i] = (double)A[pix3(a.pitch, a.ny, i, xs, wrap3(y - cy3(i), a.ny), wrap3(z - cz3(i), a.nz))];
    }
}

// ================================================================== bulk: fused stream + collide
struct Bulk3 {
    int nx, ny, nz, x0, x1, rows;
    unsigned long long pitch;
    float omega_f;
    double omega_d;
    const void* lay;   // layer populations of the new level staged by k3_final, [face][rows][M][Q] of T
    void* strip;       // face strips of the new level (see StripMap3), NULL without characteristic faces
};

// Face strips: per characteristic face and row (y, z), the populations that the next step's face
// pulls read from this row, entry i nk + k of the row's block = f(X_k - c_ix, y, z, i), X_0 = x_f
// (the strip node) and X_k = x_f - sn (M + k - 1), k = 1..3 (the viscous-moment nodes of the CBC
// schemes; nk = 4 there, 1 for the LODI schemes).  A row's block is padded to whole 128-byte lines
// and written whole (padding included) by the bulk kernel's work-group holding the row's window of
// x (12 nodes with the viscous-moment nodes, else 7): partly written lines would cost a
// read-modify-write each.  k3_prep then reads 160-640 bytes per row and face instead of one
// 128-byte line per population.  Kept in FP64 storage only: there it shortens the 3D step by
// 2.3 % on 512 x 256 x 256, while in FP32 the window wavefront's extra work lengthens every bulk
// work-group of a launch held at 3 per CU, which costs more (1.4 %) than the pulls it saves.
struct StripMap3 {
    int nk[2];     // k slots per face: 4 (CBC schemes), 1 (LODI schemes), 0 (no strip)
    int lo[2];     // first x of the face's window
    int w[2];      // window width
    int xf[2], sn[2];
    int blk[2];    // elements per row block (Q nk, padded to 128 bytes)
};
// first element of face s's blocks
__device__ __forceinline__ size_t strip_base(const StripMap3& m, int s, int rows) {
    return s == 0 ? 0 : (size_t)rows * m.blk[0];
}
// c_x of population i for a per-lane i, from two packed constants (3 bits per velocity): a lookup
// in the constant table would be a global load
__host__ __device__ constexpr unsigned long long pack_cx3(int from) {
    unsigned long long v = 0;
    for (int j = 0; j < 21 && from + j < L3::Q; ++j) v |= (unsigned long long)(cx3(from + j) + 3) << (3 * j);
    return v;
}
__device__ __forceinline__ int cx3_dyn(int i) {
    constexpr unsigned long long lo = pack_cx3(0), hi = pack_cx3(21);
    const unsigned long long v = i < 21 ? (lo >> (3 * i)) : (hi >> (3 * (i - 21)));
    return (int)(v & 7ull) - 3;
}
__device__ __forceinline__ int strip_x(const StripMap3& m, int s, int k) {
    return k == 0 ? m.xf[s] : m.xf[s] - m.sn[s] * (L3::M + k - 1);
}

// One thread per node of a 256-node x-tile of one row (the tiles cover x = 0 .. nx - 1).  Loads
// are issued source row by source row (49 (dy, dz) combinations, unrolled; only those holding
// populations generate loads); stores are non-temporal.  The row of tile t is umulhi(t, magic),
// magic = floor(2^32 / bpr) + 1 (exact while t * bpr < 2^32, checked on the host), and t itself
// when bpr == 1.
// XCD-aware order: work-group b runs on XCD b % 8, so tiles are assigned such that each XCD
// walks one contiguous range of rows; a node's up to 25 source rows (y - c_y, z - c_z) then sit
// in the L2 of the XCD that reads them instead of being fetched by several XCDs (measured on
// 512 x 256 x 256: FP64 62 % -> 72 % of HBM bandwidth, FP32 unchanged within 1 %).
// Boundary-layer lanes store the layers' new populations, which k3_final has staged before this
// launch (the faces are solved from the old level alone), so every plane's first and last cache
// line of a row is written whole by one store instruction: layer lanes run the bulk lanes'
// instruction stream (pulls with the periodic wrap in x, always in bounds; a bulk lane has
// M <= x <= nx - 1 - M and |c_x| <= M, so the wrap never acts for it) and take the staged values
// before the stores.  Partial-line stores cost read-modify-write bandwidth: k3_final writing 12
// bytes per plane row into lines the bulk had written took 180 us per step on 512 x 256 x 256;
// computing the layers' populations here instead doubles the bulk kernel's registers (the FP64
// reconstruction) and was slower.
template <typename T, bool PX>
__global__ __launch_bounds__(256, (sizeof(T) == 4 ? 3 : 2)) void k3_bulk(const T* __restrict__ A, T* __restrict__ B, Bulk3 g,
                                                                          StripMap3 sm, int bpr, unsigned magic) {
    const unsigned t0 = blockIdx.x;
    const unsigned per = gridDim.x >> 3;
    const unsigned t = (gridDim.x & 7u) ? t0 : (t0 & 7u) * per + (t0 >> 3);
    const unsigned row = bpr == 1 ? t : __umulhi(t, magic);
    const int xt0 = (int)(t - row * (unsigned)bpr) * 256;
    const int x = xt0 + (int)threadIdx.x;
    const int z = (int)(row / (unsigned)g.ny), y = (int)(row - (unsigned)z * (unsigned)g.ny);
    // the face strips: whether this tile holds part of a face's window (uniform per work-group)
    bool win[2] = {false, false};
    if (!PX && g.strip)
        for (int s = 0; s < 2; ++s) win[s] = sm.nk[s] > 0 && sm.lo[s] <= xt0 + 255 && sm.lo[s] + sm.w[s] - 1 >= xt0;
    if (x >= g.nx && !win[0] && !win[1]) return;
    const bool act = PX || (x >= g.x0 && x <= g.x1);
    T d[L3::Q];
    if (x < g.nx) {
#pragma unroll
    for (int dz = -L3::M; dz <= L3::M; ++dz) {
#pragma unroll
        for (int dy = -L3::M; dy <= L3::M; ++dy) {
            bool any = false;
#pragma unroll
            for (int i = 0; i < L3::Q; ++i) any = any || (cy3(i) == dy && cz3(i) == dz);
            if (!any) continue;
            const int ys = wrap3(y - dy, g.ny), zs = wrap3(z - dz, g.nz);
            const T* Ar = A + pix3(g.pitch, g.ny, 0, 0, ys, zs);
#pragma unroll
            for (int i = 0; i < L3::Q; ++i) {
                if (cy3(i) != dy || cz3(i) != dz) continue;
                const int xs = wrap3(x - cx3(i), g.nx);
                d[i] = Ar[(unsigned long long)i * g.pitch + xs];
            }
        }
    }
    const T omega = sizeof(T) == 4 ? (T)g.omega_f : (T)g.omega_d;
    collide3_dev<T>(d, omega);
    if (!act) {   // a boundary-layer node: its staged new populations
        const int face = x < g.x0 ? 0 : 1, j = face == 0 ? g.x0 - x : x - g.x1;
        const T* Ls = (const T*)g.lay + (((size_t)face * g.rows + (size_t)row) * L3::M + (j - 1)) * L3::Q;
#pragma unroll
        for (int i = 0; i < L3::Q; ++i) d[i] = Ls[i];
    }
    T* Bo = B + pix3(g.pitch, g.ny, 0, x, y, z);
#pragma unroll
    for (int i = 0; i < L3::Q; ++i) __builtin_nontemporal_store(d[i], Bo + (unsigned long long)i * g.pitch);
    }
    if (PX || !(win[0] || win[1])) return;
    // the window's values through LDS, then the row's strip blocks with contiguous stores.  When
    // the window lies in one wavefront (the usual case) that wavefront does it alone, with no
    // work-group barrier (a barrier made every bulk work-group wait for its slowest wavefront:
    // -6 % of the FP32 bulk rate on 512 x 256 x 256); a window across wavefronts or tiles takes
    // the barrier.
    __shared__ T sW[2][12][L3::Q];
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    bool solo[2] = {false, false}, shared = false;
    for (int s = 0; s < 2; ++s) {
        if (!win[s]) continue;
        const int l0 = sm.lo[s] - xt0, l1 = l0 + sm.w[s] - 1;
        solo[s] = l0 >= 0 && l1 <= 255 && (l0 >> 6) == (l1 >> 6);
        shared = shared || !solo[s];
    }
    for (int s = 0; s < 2; ++s)
        if (win[s] && x < g.nx && x >= sm.lo[s] && x < sm.lo[s] + sm.w[s]) {
#pragma unroll
            for (int i = 0; i < L3::Q; ++i) sW[s][x - sm.lo[s]][i] = d[i];
        }
    if (shared) __syncthreads();
    for (int s = 0; s < 2; ++s) {
        if (!win[s]) continue;
        int e0 = (int)threadIdx.x, de = 256;
        if (solo[s]) {   // only the window's wavefront, after its own LDS writes
            if (wave != ((sm.lo[s] - xt0) >> 6)) continue;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            e0 = lane;
            de = 64;
        }
        T* blk = (T*)g.strip + strip_base(sm, s, g.rows) + (size_t)row * sm.blk[s];
        const int nk = sm.nk[s];
        for (int e = e0; e < sm.blk[s]; e += de) {
            if (e >= L3::Q * nk) {   // padding, written so that the block's lines are whole
                blk[e] = (T)0;
                continue;
            }
            const int i = e / nk, k = e - i * nk;
            const int xs = strip_x(sm, s, k) - cx3_dyn(i);
            if (xs >= xt0 && xs <= xt0 + 255) blk[e] = sW[s][xs - sm.lo[s]][i];
        }
    }
}

// the face strips of the initial state (f^0), in the layout the bulk kernel writes them
template <typename T>
__global__ __launch_bounds__(256) void k3_fill_strip(const T* __restrict__ A, Bulk3 g, StripMap3 sm) {
    const int s = blockIdx.y;
    const int nk = sm.nk[s];
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (nk == 0 || e >= (long long)g.rows * L3::Q * nk) return;
    const int row = (int)(e / (L3::Q * nk)), q = (int)(e - (long long)row * L3::Q * nk), i = q / nk, k = q % nk;
    const int z = row / g.ny, y = row - z * g.ny;
    ((T*)g.strip)[strip_base(sm, s, g.rows) + (size_t)row * sm.blk[s] + q] =
        A[pix3(g.pitch, g.ny, i, strip_x(sm, s, k) - cx3(i), y, z)];
}

// ================================================================== initialisation
template <typename T>
__global__ __launch_bounds__(256) void k3_init(const double* __restrict__ rho, const double* __restrict__ ux,
                                               const double* __restrict__ uy, const double* __restrict__ uz,
                                               const double* __restrict__ Tf, T* __restrict__ A, T* __restrict__ B,
                                               int nx, int ny, long long n, unsigned long long pitch, UStride3 us) {
    const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
    if (id >= n) return;
    const int x = (int)(id % nx);
    const long long r = id / nx;
    const int y = (int)(r % ny), z = (int)(r / ny);
    const long long u = x * us.s[0] + y * us.s[1] + z * us.s[2];
    double fe[L3::Q];
    feq3_dev<double>(rho[u] - 1.0, ux[u], uy[u], uz[u], Tf[u] - 1.0, fe);
#pragma unroll
    for (int i = 0; i < L3::Q; ++i) {
        A[pix3(pitch, ny, i, x, y, z)] = (T)fe[i];
        B[pix3(pitch, ny, i, x, y, z)] = (T)fe[i];
    }
}

// Face state arrays are component-major (structure of arrays over the rows): U_b and the stage
// buffers [M][5][rows], the strip [5][rows], the viscous moments [3][10][rows], V [5][rows], so
// that consecutive threads (consecutive rows) read consecutive doubles.
__device__ __forceinline__ size_t iub(int rows, int j, int m, int r) { return ((size_t)j * 5 + m) * rows + r; }
__device__ __forceinline__ size_t ivis(int rows, int k, int c, int r) { return ((size_t)k * 10 + c) * rows + r; }

// face state at time 0 from the initial fields (both parities); an equilibrium state has no
// viscous stress and no heat flux
__global__ __launch_bounds__(256) void k3_init_faces(Args3 a, const double* __restrict__ rho, const double* __restrict__ ux,
                                                     const double* __restrict__ uy, const double* __restrict__ uz,
                                                     const double* __restrict__ Tf, UStride3 us) {
    const int s = blockIdx.y;
    const Face3& fc = a.f[s];
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (!is_char3(fc.scheme) || r >= a.rows) return;
    const int y = r % a.ny, z = r / a.ny;
    auto field = [&](int x, double* u5) {
        const long long id = x * us.s[0] + y * us.s[1] + z * us.s[2];
        u5[0] = rho[id]; u5[1] = ux[id]; u5[2] = uy[id]; u5[3] = uz[id]; u5[4] = Tf[id];
    };
    for (int p = 0; p < 2; ++p) {
        char* reg = p == 0 ? a.reg_cur : a.reg_next;
        double* ub = (double*)(reg + fc.off_ub);
        double* st = (double*)(reg + fc.off_strip);
        double u5[5];
        for (int j = 1; j <= L3::M; ++j) {
            field(fc.xf + fc.sn * j, u5);
            for (int m = 0; m < 5; ++m) ub[iub(a.rows, j - 1, m, r)] = u5[m];
        }
        field(fc.xf, u5);
        for (int m = 0; m < 5; ++m) st[(size_t)m * a.rows + r] = u5[m];
        if (is_full3(fc.scheme)) {
            double* vis = (double*)(reg + fc.off_vis);
            for (int k = 0; k < 3; ++k) {
                field(fc.xf - fc.sn * (L3::M + k), u5);
                for (int c = 0; c < 10; ++c) vis[ivis(a.rows, k, c, r)] = c == 0 ? u5[0] : 0.0;
            }
        }
    }
}

// ================================================================== face: viscous data
// (rho, Pi'_nn, Pi'_n1, Pi'_n2, Pi'_11, Pi'_12, Pi'_22, q_n, q_1, q_2) in the face frame, from the
// pre-collision populations: Pi' = -(1 - 1/(2 tau)) sum c c (f - f^eq),
// q = (1 - 1/(2 tau)) 1/2 sum f |c - u|^2 (c - u)
__device__ __forceinline__ void visc_moments3(int sn, const double* d, double tau, double* o) {
    double rm1, u, v, w, th;
    moments3_dev<double>(d, rm1, u, v, w, th);
    double fe[L3::Q];
    feq3_dev<double>(rm1, u, v, w, th, fe);
    const double fac = 1.0 - 0.5 / tau;
    double pxx = 0, pxy = 0, pxz = 0, pyy = 0, pyz = 0, pzz = 0, qx = 0, qy = 0, qz = 0;
#pragma unroll
    for (int i = 0; i < L3::Q; ++i) {
        const double c0 = cx3(i), c1 = cy3(i), c2 = cz3(i);
        const double fn = d[i] - fe[i];
        pxx -= c0 * c0 * fn; pxy -= c0 * c1 * fn; pxz -= c0 * c2 * fn;
        pyy -= c1 * c1 * fn; pyz -= c1 * c2 * fn; pzz -= c2 * c2 * fn;
        const double ex = c0 - u, ey = c1 - v, ez = c2 - w;
        const double e = (wt3(i) + d[i]) * (ex * ex + ey * ey + ez * ez);
        qx += e * ex; qy += e * ey; qz += e * ez;
    }
    o[0] = 1.0 + rm1;
    o[1] = fac * pxx; o[2] = sn * fac * pxy; o[3] = sn * fac * pxz;
    o[4] = fac * pyy; o[5] = fac * pyz; o[6] = fac * pzz;
    o[7] = sn * 0.5 * fac * qx; o[8] = 0.5 * fac * qy; o[9] = 0.5 * fac * qz;
}

// Four threads per face row, one per node: x_f (k = 0) and x_f - sn (M + k - 1) (k = 1, 2, 3),
// pulling from the face strips the previous bulk launch (or k3_fill_strip) wrote, or from A where
// no strips are kept (consecutive threads then pull nearby x of the same row).  New level: moments of x_f (the
// strip) and, for the CBC schemes, the viscous moments of the other three nodes.  Old level (CBC
// schemes, thread k = 0): the viscous terms V (eq. NSF-CHAR, Appendix A), frozen during the RK4
// stages -- div Pi' / rho and (-div q + Pi':Pi' / (2 rho nu)) / (rho c_v cs^2), normal derivatives
// one-sided over x_f - M .. x_f - M - 2 (eq. FD-dx-bw), tangential ones central in y and z
// (eq. FD-dx-center).
template <typename T>
__global__ __launch_bounds__(256) void k3_prep(const T* __restrict__ A, const T* __restrict__ strip, StripMap3 sm, Args3 a) {
    const int s = blockIdx.y;
    const Face3& fc = a.f[s];
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (!is_char3(fc.scheme) || t >= 4 * a.rows) return;
    // four threads per row: k = 0 the strip node x_f, k = 1..3 the viscous-moment nodes
    // x_f - M - (k - 1), the first nodes inward of x_f none of whose populations streamed from
    // the layers (bulk nodes: the configuration keeps nx >= 3M + 3 for CBC faces)
    const int r = t / 4, k = t - 4 * r;
    const int y = r % a.ny, z = r / a.ny;
    const bool full = is_full3(fc.scheme);
    if (!full && k > 0) return;
    // the pull of node X_k: from the face strips when kept (population i of it is strip entry
    // (i, k) of the row (y - c_iy, z - c_iz)), else from A
    double d[L3::Q];
    if (strip) {
        const T* sb = strip + strip_base(sm, s, a.rows);
        const int nk = sm.nk[s], bl = sm.blk[s];
#pragma unroll
        for (int i = 0; i < L3::Q; ++i)
            d[i] = (double)sb[(size_t)(wrap3(z - cz3(i), a.nz) * a.ny + wrap3(y - cy3(i), a.ny)) * bl + i * nk + k];
    } else {
        pull3<T>(A, a, k == 0 ? fc.xf : fc.xf - fc.sn * (L3::M + k - 1), y, z, d);
    }
    if (k == 0) {
        double rm1, u, v, w, th;
        moments3_dev<double>(d, rm1, u, v, w, th);
        double* stn = (double*)(a.reg_next + fc.off_strip);
        const double o[5] = {1.0 + rm1, u, v, w, 1.0 + th};
        for (int m = 0; m < 5; ++m) stn[(size_t)m * a.rows + r] = o[m];
    } else {
        double o[10];
        visc_moments3(fc.sn, d, a.tau, o);
        double* visn = (double*)(a.reg_next + fc.off_vis);
        for (int c = 0; c < 10; ++c) visn[ivis(a.rows, k - 1, c, r)] = o[c];
    }
    if (!full || k != 0) return;
    const double* vis = (const double*)(a.reg_cur + fc.off_vis);
    auto at = [&](int kk, int yy, int zz, int c) {
        return vis[ivis(a.rows, kk, c, wrap3(zz, a.nz) * a.ny + wrap3(yy, a.ny))];
    };
    auto dn = [&](int c) { return 0.5 * (3.0 * at(0, y, z, c) - 4.0 * at(1, y, z, c) + at(2, y, z, c)); };
    auto d1 = [&](int c) { return 0.5 * (at(0, y + 1, z, c) - at(0, y - 1, z, c)); };
    auto d2 = [&](int c) { return 0.5 * (at(0, y, z + 1, c) - at(0, y, z - 1, c)); };
    double p[10];
    for (int c = 0; c < 10; ++c) p[c] = at(0, y, z, c);
    const double rho = p[0];
    const double nu = (a.tau - 0.5) * L3::cs2;
    const double pp = p[1] * p[1] + p[4] * p[4] + p[6] * p[6] + 2.0 * (p[2] * p[2] + p[3] * p[3] + p[5] * p[5]);
    double* V = a.V + (size_t)s * 5 * a.rows;
    V[r] = 0.0;
    V[(size_t)1 * a.rows + r] = (dn(1) + d1(2) + d2(3)) / rho;
    V[(size_t)2 * a.rows + r] = (dn(2) + d1(4) + d2(5)) / rho;
    V[(size_t)3 * a.rows + r] = (dn(3) + d1(5) + d2(6)) / rho;
    V[(size_t)4 * a.rows + r] = (-(dn(7) + d1(8) + d2(9)) + pp / (2.0 * rho * nu)) / (rho * CV * L3::cs2);
}

// ================================================================== face: characteristic rate
// dU/dt in the face frame (rho, u_n, u_t1, u_t2, T) of one layer node (Appendix A): amplitudes
// L = Lambda S dU/dn, incoming ones by scheme (Tab. CBCs; relaxation on the incoming acoustic
// wave with the acoustic rows' pressure coefficient 1/(5 rho cs^2)), then -S^-1 Lbar (+ T + V
// for the CBC schemes).  yp/ym, zp/zm: the node's neighbours in y and z (same layer); U0: the
// node at time t, which fixes the wave directions.
__device__ __forceinline__ void char_rate3(const double* U, const double* dn, const double* yp, const double* ym,
                                           const double* zp, const double* zm, const double* V, const double* U0,
                                           int scheme, double K, double alpha, double Pinf, double* rate) {
    constexpr double cs2 = L3::cs2;
    const bool full = is_full3(scheme);
    const bool relax = scheme == F3_LODI_RELAX || scheme == F3_CBC_RELAX;
    const double rho = U[0], un = U[1], v = U[2], w = U[3], T = U[4];
    const double ir = 1.0 / rho;
    auto h = [](double a, double b) { return 0.5 * (a - b); };
    // transverse terms (Appendix A), central differences in y and z
    double Tt[5];
    Tt[0] = -h(yp[0] * yp[2], ym[0] * ym[2]) - h(zp[0] * zp[3], zm[0] * zm[3]);
    Tt[1] = -(v * h(yp[1], ym[1]) + w * h(zp[1], zm[1]));
    Tt[2] = -cs2 * ir * h(yp[0] * yp[4], ym[0] * ym[4]) - (v * h(yp[2], ym[2]) + w * h(zp[2], zm[2]));
    Tt[3] = -cs2 * ir * h(zp[0] * zp[4], zm[0] * zm[4]) - (v * h(yp[3], ym[3]) + w * h(zp[3], zm[3]));
    Tt[4] = -(T * (1.0 / CV)) * (h(yp[2], ym[2]) + h(zp[3], zm[3])) - (v * h(yp[4], ym[4]) + w * h(zp[4], zm[4]));
    const double er = T * ir;                          // T~ / (rho cs^2)
    const double r15 = sqrt(T * (1.0 / (15.0 * cs2)));
    auto Sx = [&](const double* x, double* o) {
        o[0] = -0.4 * er * x[0] + 0.6 * x[4];
        o[1] = x[2];
        o[2] = x[3];
        o[3] = 0.2 * er * x[0] - r15 * x[1] + 0.2 * x[4];
        o[4] = 0.2 * er * x[0] + r15 * x[1] + 0.2 * x[4];
    };
    const double s = sqrt(GAMMA * cs2 * T), s0 = sqrt(GAMMA * cs2 * U0[4]), u0 = U0[1];
    double Sd[5], ST[5];
    Sx(dn, Sd);
    Sx(Tt, ST);
    const double lam[5] = {un, un, un, un - s, un + s};
    const double lam0[5] = {u0, u0, u0, u0 - s0, u0 + s0};
    double in[5] = {0, 0, 0, 0, 0};
    if (full) {
        double TV[5], STV[5];
        for (int m = 0; m < 5; ++m) TV[m] = Tt[m] + V[m];
        Sx(TV, STV);
        for (int m = 0; m < 5; ++m) in[m] = STV[m];
    }
    if (relax) {
        const double pr = K * (rho * cs2 * T - Pinf) * ir * (1.0 / (5.0 * cs2));
        in[3] += pr - alpha * ST[3];
        in[4] += pr - alpha * ST[4];
    }
    double Bv[5];
    for (int m = 0; m < 5; ++m) Bv[m] = lam0[m] >= 0.0 ? lam[m] * Sd[m] : in[m];
    const double rT = rho / T, q15 = sqrt(15.0 * cs2 / (4.0 * T));
    rate[0] = rT * Bv[0] - 1.5 * rT * (Bv[3] + Bv[4]);
    rate[1] = q15 * (Bv[3] - Bv[4]);
    rate[2] = -Bv[1];
    rate[3] = -Bv[2];
    rate[4] = -(Bv[0] + Bv[3] + Bv[4]);
    if (full)
        for (int m = 0; m < 5; ++m) rate[m] += Tt[m] + V[m];
}

// One RK4 stage of the coupled face system, one thread per layer node (face s, layer j, row r;
// consecutive threads take consecutive rows).  Stage st reads its inputs Y_st (st = 0: U_b^n)
// and writes Y_{st+1} = U_b^n + a_{st+1} K_st into the other stage buffer and the running sum
// U_b^{n+1} += b_st K_st / 6 into the next parity region.  Bulk values at stage time
// t + theta: (1 - theta) strip^n + theta strip^{n+1}.
__global__ __launch_bounds__(256) void k3_stage(Args3 a, int st) {
    const int s = blockIdx.y;
    const Face3& fc = a.f[s];
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (!is_char3(fc.scheme) || t >= L3::M * a.rows) return;
    const int jj = t / a.rows, r = t - jj * a.rows, j = jj + 1;
    const int y = r % a.ny, z = r / a.ny;
    const int R = a.rows;
    const double thv[4] = {0.0, 0.5, 0.5, 1.0}, bst[4] = {1.0, 2.0, 2.0, 1.0};
    const double th = thv[st];
    const double* ub = (const double*)(a.reg_cur + fc.off_ub);
    double* ubn = (double*)(a.reg_next + fc.off_ub);
    const size_t fo = (size_t)s * L3::M * 5 * R;   // this face's part of the stage buffers
    const double* Ys = st == 0 ? ub : (st == 2 ? a.Yb + fo : a.Ya + fo);
    double* Yd = st == 0 ? a.Ya + fo : (st == 1 ? a.Yb + fo : (st == 2 ? a.Ya + fo : nullptr));
    const double* sc = (const double*)(a.reg_cur + fc.off_strip);
    const double* sx = (const double*)(a.reg_next + fc.off_strip);
    auto loc = [&](const double* g, double* l) { l[0] = g[0]; l[1] = fc.sn * g[1]; l[2] = g[2]; l[3] = g[3]; l[4] = g[4]; };
    auto val_n = [&](int k, double* l) {   // outward index k at this row (k = 0: x_f)
        double g[5];
        if (k >= 1) {
            for (int m = 0; m < 5; ++m) g[m] = Ys[iub(R, k - 1, m, r)];
        } else {
            for (int m = 0; m < 5; ++m) g[m] = (1.0 - th) * sc[(size_t)m * R + r] + th * sx[(size_t)m * R + r];
        }
        loc(g, l);
    };
    auto val_t = [&](int yy, int zz, double* l) {
        const int rr = wrap3(zz, a.nz) * a.ny + wrap3(yy, a.ny);
        double g[5];
        for (int m = 0; m < 5; ++m) g[m] = Ys[iub(R, jj, m, rr)];
        loc(g, l);
    };
    double U[5], dn[5], yp[5], ym[5], zp[5], zm[5], U0[5];
    val_n(j, U);
    if (j == L3::M) {   // eq. FD-dx-bw
        double b1[5], b2[5];
        val_n(j - 1, b1); val_n(j - 2, b2);
        for (int m = 0; m < 5; ++m) dn[m] = 0.5 * (3.0 * U[m] - 4.0 * b1[m] + b2[m]);
    } else {            // eq. FD-dx-center
        double p1[5], m1[5];
        val_n(j + 1, p1); val_n(j - 1, m1);
        for (int m = 0; m < 5; ++m) dn[m] = 0.5 * (p1[m] - m1[m]);
    }
    val_t(y + 1, z, yp); val_t(y - 1, z, ym); val_t(y, z + 1, zp); val_t(y, z - 1, zm);
    double g0[5];
    for (int m = 0; m < 5; ++m) g0[m] = ub[iub(R, jj, m, r)];
    loc(g0, U0);
    double Vl[5] = {0, 0, 0, 0, 0};
    if (is_full3(fc.scheme))   // already in the face frame
        for (int m = 0; m < 5; ++m) Vl[m] = a.V[((size_t)s * 5 + m) * R + r];
    double rl[5];
    char_rate3(U, dn, yp, ym, zp, zm, Vl, U0, fc.scheme, fc.K, fc.alpha, fc.Pinf, rl);
    rl[1] *= fc.sn;   // back to global components
    for (int m = 0; m < 5; ++m) {
        const size_t o = iub(R, jj, m, r);
        const double base = st == 0 ? g0[m] : ubn[o];
        ubn[o] = base + bst[st] * (1.0 / 6.0) * rl[m];
        if (Yd) Yd[o] = g0[m] + thv[st + 1] * rl[m];
    }
}

// New layer populations, three threads per face row (one per layer; neighbouring x of the same
// row, so the stores of a plane cover contiguous bytes): the equilibrium of U_b^{n+1}, plus with
// NEEP (eq. NEEP) the post-collision non-equilibrium part of x_f; zero-gradient faces copy x_f
// (eq. zg-bc) from the new bulk populations in B.
template <typename T>
__global__ __launch_bounds__(256) void k3_final(const T* __restrict__ A, T* __restrict__ S, Args3 a) {
    const int s = blockIdx.y;
    const Face3& fc = a.f[s];
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (fc.scheme == F3_PERIODIC || t >= L3::M * a.rows) return;
    const int r = t / L3::M, jj = t - L3::M * r;
    const int y = r % a.ny, z = r / a.ny;
    T* o = S + (((size_t)s * a.rows + r) * L3::M + jj) * L3::Q;
    if (fc.scheme == F3_ZG) {
        // eq. zg-bc: the post-collision populations of x_f, as the bulk kernel computes them
        T d[L3::Q];
#pragma unroll
        for (int i = 0; i < L3::Q; ++i)
            d[i] = A[pix3(a.pitch, a.ny, i, fc.xf - cx3(i), wrap3(y - cy3(i), a.ny), wrap3(z - cz3(i), a.nz))];
        collide3_dev<T>(d, (T)a.omega);
#pragma unroll
        for (int i = 0; i < L3::Q; ++i) o[i] = d[i];
        return;
    }
    const double* ubn = (const double*)(a.reg_next + fc.off_ub);
    double u5[5];
    for (int m = 0; m < 5; ++m) u5[m] = ubn[iub(a.rows, jj, m, r)];
    double fe[L3::Q];
    feq3_dev<double>(u5[0] - 1.0, u5[1], u5[2], u5[3], u5[4] - 1.0, fe);
    if (fc.meso == 1) {
        double d[L3::Q], fx[L3::Q];
        pull3<T>(A, a, fc.xf, y, z, d);
        double rm1, u, v, w, th;
        moments3_dev<double>(d, rm1, u, v, w, th);
        feq3_dev<double>(rm1, u, v, w, th, fx);
        const double c = 1.0 - a.omega;
#pragma unroll
        for (int i = 0; i < L3::Q; ++i) fe[i] += c * (d[i] - fx[i]);
    }
#pragma unroll
    for (int i = 0; i < L3::Q; ++i) o[i] = (T)fe[i];
}

// ================================================================== output and diagnostics
template <typename T>
__global__ __launch_bounds__(256) void k3_macro(const T* __restrict__ A, int nx, int ny, long long n, unsigned long long pitch,
                                                double* __restrict__ rho, double* __restrict__ ux, double* __restrict__ uy,
                                                double* __restrict__ uz, double* __restrict__ Tf, UStride3 us) {
    const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
    if (id >= n) return;
    const int x = (int)(id % nx);
    const long long rr = id / nx;
    const int y = (int)(rr % ny), z = (int)(rr / ny);
    double d[L3::Q];
#pragma unroll
    for (int i = 0; i < L3::Q; ++i) d[i] = (double)A[pix3(pitch, ny, i, x, y, z)];
    double rm1, u, v, w, th;
    moments3_dev<double>(d, rm1, u, v, w, th);
    const long long o = x * us.s[0] + y * us.s[1] + z * us.s[2];
    rho[o] = 1.0 + rm1; ux[o] = u; uy[o] = v; uz[o] = w; Tf[o] = 1.0 + th;
}

// full populations f = w_i + d_i, FP64 [q][nz][ny][nx] in the caller's frame: plane j holds the
// library velocity vm.i[j] of the internal grid (the same velocity as j, axes permuted)
template <typename T>
__global__ __launch_bounds__(256) void k3_pops(const T* __restrict__ A, int nx, int ny, long long n, unsigned long long pitch,
                                               double* __restrict__ out, UStride3 us, VMap3 vm) {
    const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
    if (id >= n) return;
    const int x = (int)(id % nx);
    const long long rr = id / nx;
    const int y = (int)(rr % ny), z = (int)(rr / ny);
    const long long o = x * us.s[0] + y * us.s[1] + z * us.s[2];
#pragma unroll
    for (int j = 0; j < L3::Q; ++j) {
        const int i = vm.i[j];
        out[(long long)j * n + o] = wt3(i) + (double)A[pix3(pitch, ny, i, x, y, z)];
    }
}

__device__ __forceinline__ double wsum3(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wmax3(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// partial[8][nblk] (component-major, nblk = gridDim.x): mass, jx, jy, jz, energy
// (1/2 sum f |c|^2), loss (sum over bulk nodes of (P - P_inf)^2, P_inf = cs^2), max |u|,
// non-finite count.  A grid-stride loop over the nodes (one work-group per 256-node row tile, as
// in 2D, measured no faster here and needs a longer second pass).
template <typename T>
__global__ __launch_bounds__(256) void k3_diag_partial(const T* __restrict__ A, int nx, int ny, long long n,
                                                       unsigned long long pitch, int bx0, int bx1,
                                                       double* __restrict__ partial) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long long id = (long long)blockIdx.x * 256 + threadIdx.x; id < n; id += (long long)gridDim.x * 256) {
        const int x = (int)(id % nx);
        const long long rr = id / nx;
        const int y = (int)(rr % ny), z = (int)(rr / ny);
        double d[L3::Q], bad = 0.0;
#pragma unroll
        for (int i = 0; i < L3::Q; ++i) {
            d[i] = (double)A[pix3(pitch, ny, i, x, y, z)];
            bad += isfinite(d[i]) ? 0.0 : 1.0;
        }
        double rm1, u, v, w, th;
        moments3_dev<double>(d, rm1, u, v, w, th);
        const double r = 1.0 + rm1;
        double e = 1.5 * L3::cs2;   // 1/2 sum w |c|^2
#pragma unroll
        for (int i = 0; i < L3::Q; ++i) e += 0.5 * (double)c2_3(i) * d[i];
        acc[0] += r; acc[1] += r * u; acc[2] += r * v; acc[3] += r * w; acc[4] += e;
        if (x >= bx0 && x <= bx1) {
            const double p = L3::cs2 * (rm1 + th + rm1 * th);
            acc[5] += p * p;
        }
        const double um = sqrt(u * u + v * v + w * w);
        acc[6] = (um == um) ? fmax(acc[6], um) : acc[6];
        acc[7] += bad;
    }
    __shared__ double red[4][8];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < 8; ++k) {
        const double v = k == 6 ? wmax3(acc[k]) : wsum3(acc[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int q = 1; q < 4; ++q) v = k == 6 ? fmax(v, red[q][k]) : v + red[q][k];
        partial[(size_t)k * gridDim.x + blockIdx.x] = v;
    }
}

// second pass: one 1024-thread work-group per quantity (k = 6 is a maximum, the others sums),
// each thread folding partials t, t + 1024, ... in order with eight loads in flight, then a fixed
// tree (deterministic)
__global__ __launch_bounds__(1024) void k3_diag_final(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
    const int k = blockIdx.x;
    __shared__ double red[1024];
    const double* pk = partial + (size_t)k * nblk;
    double v = 0.0;   // identity of both (the maximum is over |u| >= 0)
    for (int b0 = threadIdx.x; b0 < nblk; b0 += 8 * 1024) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + u * 1024;
            t[u] = b < nblk ? pk[b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v = k == 6 ? fmax(v, t[u]) : v + t[u];
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] = k == 6 ? fmax(red[threadIdx.x], red[threadIdx.x + w]) : red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
}

}  // namespace lbm3
