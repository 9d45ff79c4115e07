// kernels.h -- HIP kernels of the thermal LBM with characteristic boundaries (gfx950).
//
// Data layout in HBM (one context):
//   f[2]   : two population buffers in row-interleaved structure-of-arrays order f[y][i][x]
//            (the q planes of one row are contiguous; row pitch padded to a multiple of 64
//            elements so every plane segment starts on a 256-byte boundary), storing the
//            deviations f_i - w_i in T = double or float.  Interleaving the planes per row keeps
//            the write stream of a row of work-groups in one contiguous region.
//   region : two parity copies of the boundary solver state (FP64): per characteristic side
//            U_b[M][len][4], the bulk strip U[MS][len][4] at x_f (and x_f - 1 for M = 1), the
//            viscous moments [3][len][6] at x_f-M .. x_f-M-2; per corner U_c[4] and the two
//            inward diagonal bulk nodes [2][4].  Parity p holds time level n with n % 2 = p.
// One time step n -> n+1 is one launch of k_step: its first work-groups each take a chunk of
// rows of a boundary side (re-pull of the strip from A, RK4 of the characteristic system in
// LDS, equilibrium populations of the M boundary layers of B); the remaining work-groups each
// take 256 bulk nodes of one row (pull-stream + moments + equilibrium + BGK, A -> B).  Both
// kinds only read A and write disjoint nodes of B, so they need no ordering among themselves.
// The boundary path's LDS (and registers) cap the launch at 2-3 work-groups per CU, which is
// also the occupancy at which this many-stream access pattern streams fastest from HBM.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.h"

namespace lbm {

enum { BC_PERIODIC = 0, BC_LODI = 1, BC_LODI_RELAX = 2, BC_CBC = 3, BC_CBC_RELAX = 4, BC_ZG = 5, BC_DIRICHLET = 6 };
enum { KIND_NONE = 0, KIND_CHAR = 1, KIND_ZG = 2, KIND_DIRICHLET = 3 };

struct SideDev {
    int kind, scheme;
    int meso;                    // mesoscopic BC of a characteristic side: 0 equilibrium, 1 NEEP
    int vfd;                     // viscous terms of a CBC side: 0 mesoscopic moments, 1 differences
    int nax, sn, Nn, Nt, r0, len, xf, tper;
    int blk0, nblk, rows;        // boundary work-groups of this side in k_step, rows per work-group
    int corner_lo, corner_hi;    // corners at row -1 / row len (non-periodic tangent), else -1
    int owns_corners;            // x-sides write the corner blocks
    double K, alpha, Pinf;       // relaxation (eq. LODI-Relax / CBC-Relax)
    unsigned long long off_ub, off_strip, off_vis;   // byte offsets inside one parity region
    unsigned long long off_stage;   // RK4 stage inputs Y_1..Y_3 [3][M][len][4] (recomputation for the adjoint)
};

struct CornerDev {
    int active, zg, relax;
    int xc, yc, vx, vy;          // innermost corner node and inward diagonal step
    int x0, y0, sxn, syn;        // corner block: x0 + sxn*j, y0 + syn*j, j = 0..M-1
    double K, Pinf, ndx, ndy;    // relaxation of the x-side, outward diagonal normal
    unsigned long long off_cu, off_cd;
    unsigned long long off_cs;   // RK4 stage inputs Y_1..Y_3 [3][4] (recomputation for the adjoint)
};

struct BndArgs {
    int nx, ny, nbulk_x0, nbulk_x1, nbulk_y0, nbulk_y1, xper, yper;
    unsigned long long pitch;   // padded row length (elements) of one population plane row
    double omega, tau;
    char* reg_cur;    // parity region of time level n
    char* reg_next;   // parity region of time level n+1
    SideDev s[4];
    CornerDev c[4];
};

__device__ __forceinline__ int wrapi(int v, int n) {
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

// element of population i at node (x, y)
template <int Q>
__device__ __forceinline__ unsigned long long pix(unsigned long long pitch, int i, int x, int y) {
    return ((unsigned long long)y * Q + i) * pitch + x;
}

// node of side s at outward index k (k = 0: x_f, k = j: layer x_{b,j}) and physical row r
__device__ __forceinline__ void side_node(const SideDev& s, int k, int r, int& x, int& y) {
    const int nc = s.xf + s.sn * k;
    const int tc = s.r0 + r;
    if (s.nax == 0) { x = nc; y = tc; } else { x = tc; y = nc; }
}

// ------------------------------------------------------------------ pull of one node (FP64)
template <int Q, typename T>
__device__ __forceinline__ void pull_node(const T* __restrict__ A, const BndArgs& a, int x, int y, double* d) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int xs = x - cx<Q>(i), ys = y - cy<Q>(i);
        if (a.xper) xs = wrapi(xs, a.nx);
        if (a.yper) ys = wrapi(ys, a.ny);
        d[i] = (double)A[pix<Q>(a.pitch, i, xs, ys)];
    }
}

// ================================================================== bulk: fused stream + collide
struct BulkArgs {
    int nx, ny, x0, x1, y0, y1;   // bulk node range (inclusive)
    unsigned long long pitch;
    float omega_f;
    double omega_d;
    double* mom;                  // HIST only: (rho, ux, uy, T) planes [4][ny][pitch] of the new state
};

// One thread per node.  Work-group x-ranges start at x = 0 (multiples of 256), so every
// wavefront's store of a plane is one aligned 256 B (float) / 512 B (double) segment; lanes
// outside the bulk range do nothing.  Loads are ordinary (cached) loads, issued source row by
// source row: the shifted pulls of neighbouring wavefronts share cache lines at their edges,
// which L2 serves once.  Stores are non-temporal: the output is not re-read in this step.
// HIST (recomputation for the adjoint) also stores the node's moments.
template <int Q, typename T, bool PX, bool PY, bool HIST>
__device__ __forceinline__ void bulk_node(const T* __restrict__ A, T* __restrict__ B, const BulkArgs& g, int x, int y) {
    if (x < g.x0 || x > g.x1) return;
    T d[Q];
#pragma unroll
    for (int dy = -Lat<Q>::M; dy <= Lat<Q>::M; ++dy) {
        int ys = y - dy;
        if (PY) ys = wrapi(ys, g.ny);
        const T* Ar = A + pix<Q>(g.pitch, 0, 0, ys);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (cy<Q>(i) != dy) continue;
            int xs = x - cx<Q>(i);
            if (PX) xs = wrapi(xs, g.nx);
            d[i] = Ar[(unsigned long long)i * g.pitch + xs];
        }
    }
    if (HIST) {
        T rm1, u, v, th;
        moments_dev<Q, T>(d, rm1, u, v, th);
        const unsigned long long plane = (unsigned long long)g.ny * g.pitch, o = (unsigned long long)y * g.pitch + x;
        g.mom[o] = 1.0 + (double)rm1;
        g.mom[plane + o] = (double)u;
        g.mom[2 * plane + o] = (double)v;
        g.mom[3 * plane + o] = 1.0 + (double)th;
    }
    const T omega = sizeof(T) == 4 ? (T)g.omega_f : (T)g.omega_d;
    collide_dev<Q, T>(d, omega);
    T* Bo = B + pix<Q>(g.pitch, 0, x, y);
#pragma unroll
    for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(d[i], Bo + (unsigned long long)i * g.pitch);
}

// ================================================================== initialisation
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_init_fields(const double* __restrict__ rho, const double* __restrict__ ux,
                                                     const double* __restrict__ uy, const double* __restrict__ Tf,
                                                     T* __restrict__ A, T* __restrict__ B, int nx, int n,
                                                     unsigned long long pitch) {
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= n) return;
    const int x = id % nx, y = id / nx;
    double fe[Q];
    const double th = (Lat<Q>::thermal && Tf) ? Tf[id] - 1.0 : 0.0;
    feq_dev<Q, double>(rho[id] - 1.0, ux[id], uy[id], th, fe);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        A[pix<Q>(pitch, i, x, y)] = (T)fe[i];
        B[pix<Q>(pitch, i, x, y)] = (T)fe[i];
    }
}

// macroscopic field value (rho, ux, uy, T) of node (x, y) from the initial arrays
__device__ __forceinline__ void field_at(const double* rho, const double* ux, const double* uy, const double* Tf,
                                         int nx, int x, int y, double* u4) {
    const int id = y * nx + x;
    u4[0] = rho[id]; u4[1] = ux[id]; u4[2] = uy[id]; u4[3] = Tf ? Tf[id] : 1.0;
}

// boundary solver state at time 0 from the initial fields; both parities' viscous moments 0
template <int Q>
__global__ __launch_bounds__(256) void k_init_boundary(BndArgs a, const double* __restrict__ rho, const double* __restrict__ ux,
                                                       const double* __restrict__ uy, const double* __restrict__ Tf,
                                                       double* __restrict__ inlet0, double* __restrict__ inlet1,
                                                       double* __restrict__ inlet2, double* __restrict__ inlet3) {
    constexpr int M = Lat<Q>::M, MS = (M == 1) ? 2 : 1;
    const int s = blockIdx.y;
    const SideDev& sd = a.s[s];
    const bool thermal = Lat<Q>::thermal;
    const double* Tuse = thermal ? Tf : nullptr;
    for (int r = blockIdx.x * 256 + threadIdx.x; r < sd.len; r += gridDim.x * 256) {
        if (sd.kind == KIND_CHAR) {
            double* ub = (double*)(a.reg_cur + sd.off_ub);
            double* st = (double*)(a.reg_cur + sd.off_strip);
            for (int j = 1; j <= M; ++j) {
                int x, y; side_node(sd, j, r, x, y);
                field_at(rho, ux, uy, Tuse, a.nx, x, y, &ub[((size_t)(j - 1) * sd.len + r) * 4]);
            }
            for (int k = 0; k < MS; ++k) {
                int x, y; side_node(sd, -k, r, x, y);
                field_at(rho, ux, uy, Tuse, a.nx, x, y, &st[((size_t)k * sd.len + r) * 4]);
            }
            if (sd.scheme == BC_CBC || sd.scheme == BC_CBC_RELAX) {
                // equilibrium initial state: no stress, no heat flux; density of the fields
                double* v0 = (double*)(a.reg_cur + sd.off_vis);
                double* v1 = (double*)(a.reg_next + sd.off_vis);
                for (int k = 0; k < 3; ++k) {
                    int x, y; side_node(sd, -(M + k), r, x, y);
                    const double rk = rho[y * a.nx + x];
                    for (int c = 0; c < 6; ++c) {
                        v0[((size_t)k * sd.len + r) * 6 + c] = c == 0 ? rk : 0.0;
                        v1[((size_t)k * sd.len + r) * 6 + c] = c == 0 ? rk : 0.0;
                    }
                }
            }
        } else if (sd.kind == KIND_DIRICHLET) {
            double* inl = s == 0 ? inlet0 : s == 1 ? inlet1 : s == 2 ? inlet2 : inlet3;
            int x, y; side_node(sd, 1, r, x, y);
            field_at(rho, ux, uy, Tuse, a.nx, x, y, &inl[(size_t)r * 4]);
        }
    }
    if (s == 0 && blockIdx.x == 0 && threadIdx.x < 4) {
        const CornerDev& c = a.c[threadIdx.x];
        if (c.active && !c.zg) {
            double* cu = (double*)(a.reg_cur + c.off_cu);
            double* cd = (double*)(a.reg_cur + c.off_cd);
            field_at(rho, ux, uy, Tuse, a.nx, c.xc, c.yc, cu);
            field_at(rho, ux, uy, Tuse, a.nx, c.xc + c.vx, c.yc + c.vy, cd);
            field_at(rho, ux, uy, Tuse, a.nx, c.xc + 2 * c.vx, c.yc + 2 * c.vy, cd + 4);
        }
    }
}

// equilibrium populations of a fixed profile on every layer of a Dirichlet side, both buffers
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_dirichlet(BndArgs a, int s, const double* __restrict__ prof, T* __restrict__ A,
                                                   T* __restrict__ B) {
    constexpr int M = Lat<Q>::M;
    const SideDev& sd = a.s[s];
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= sd.len * M) return;
    const int r = t / M, j = 1 + t % M;
    int x, y; side_node(sd, j, r, x, y);
    const double* u = prof + (size_t)r * 4;
    double fe[Q];
    feq_dev<Q, double>(u[0] - 1.0, u[1], u[2], Lat<Q>::thermal ? u[3] - 1.0 : 0.0, fe);
#pragma unroll
    for (int i = 0; i < Q; ++i) { A[pix<Q>(a.pitch, i, x, y)] = (T)fe[i]; B[pix<Q>(a.pitch, i, x, y)] = (T)fe[i]; }
}

// ================================================================== macroscopic output
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_macro(const T* __restrict__ A, int nx, int n, unsigned long long pitch,
                                               double* __restrict__ rho, double* __restrict__ ux, double* __restrict__ uy,
                                               double* __restrict__ Tf) {
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= n) return;
    const int x = id % nx, y = id / nx;
    double d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = (double)A[pix<Q>(pitch, i, x, y)];
    double rm1, u, v, th;
    moments_dev<Q, double>(d, rm1, u, v, th);
    rho[id] = 1.0 + rm1; ux[id] = u; uy[id] = v;
    if (Tf) Tf[id] = 1.0 + th;
}

// ================================================================== diagnostics (two passes)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Diagnostics of one node, accumulated into acc: mass, jx, jy, energy, loss (bulk nodes only),
// max |u|, non-finite count.
template <int Q, typename T>
__device__ __forceinline__ void diag_node(const T* __restrict__ A, int x, int y, unsigned long long pitch, int bx0,
                                          int bx1, int by0, int by1, double* acc) {
    double d[Q];
    double bad = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        d[i] = (double)A[pix<Q>(pitch, i, x, y)];
        bad += (isfinite(d[i]) ? 0.0 : 1.0);
    }
    double rm1, u, v, th;
    moments_dev<Q, double>(d, rm1, u, v, th);
    const double r = 1.0 + rm1;
    double e = Lat<Q>::cs2;   // 1/2 sum w |c|^2
#pragma unroll
    for (int i = 0; i < Q; ++i) e += 0.5 * (double)c2<Q>(i) * d[i];
    acc[0] += r; acc[1] += r * u; acc[2] += r * v; acc[3] += e;
    if (x >= bx0 && x <= bx1 && y >= by0 && y <= by1) {
        const double p = Lat<Q>::cs2 * (rm1 + th + rm1 * th);   // P - cs^2
        acc[4] += p * p;
    }
    const double um = sqrt(u * u + v * v);
    acc[5] = (um == um) ? fmax(acc[5], um) : acc[5];
    acc[6] += bad;
}

// partial[8][nblk] (component-major, nblk = gridDim.x): mass, jx, jy, energy, loss, max|u|,
// non-finite count, 0.  One work-group per 256-node x tile of one row (bpr tiles per row), one
// node per thread: a grid-stride loop over fewer work-groups keeps fewer loads in flight and read
// 60 % of the HBM rate in FP32 against ~85 % for this mapping (measured on 4096 x 2048).  With
// TPW, work-group b takes the tpw consecutive tiles b tpw .. b tpw + tpw - 1 (< ntiles), so that
// the partials fit a fixed-size buffer.
template <int Q, typename T, bool TPW>
__global__ __launch_bounds__(256) void k_diag_partial(const T* __restrict__ A, int nx, int bpr, unsigned long long pitch,
                                                      int bx0, int bx1, int by0, int by1, double* __restrict__ partial,
                                                      int ntiles, int tpw) {
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    if (!TPW) {
        const int x = (blockIdx.x % bpr) * 256 + threadIdx.x, y = blockIdx.x / bpr;
        if (x < nx) diag_node<Q, T>(A, x, y, pitch, bx0, bx1, by0, by1, acc);
    } else {
        const int t0 = blockIdx.x * tpw, t1 = min(ntiles, t0 + tpw);
        for (int t = t0; t < t1; ++t) {
            const int x = (t % bpr) * 256 + threadIdx.x, y = t / bpr;
            if (x < nx) diag_node<Q, T>(A, x, y, pitch, bx0, bx1, by0, by1, acc);
        }
    }
    __shared__ double red[4][8];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = 0; k < 7; ++k) {
        const double v = k == 5 ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wid][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int w = 1; w < 4; ++w) v = (k == 5) ? fmax(v, red[w][k]) : v + red[w][k];
        partial[(size_t)k * gridDim.x + blockIdx.x] = v;
    }
    if (threadIdx.x == 7) partial[(size_t)7 * gridDim.x + blockIdx.x] = 0.0;
}

// second pass: one 1024-thread work-group per quantity (k = 5 is a maximum, the others sums).
// Thread t folds partials t, t + 1024, ... in that order, eight loads in flight at a time, then a
// fixed tree over the threads: the result does not depend on timing (deterministic).  out[7]
// receives v7 (the step count).
__global__ __launch_bounds__(1024) void k_diag_final(const double* __restrict__ partial, int nblk, double* __restrict__ out,
                                                     double v7) {
    const int k = blockIdx.x;   // 0..7
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
        for (int u = 0; u < 8; ++u) v = (k == 5) ? fmax(v, t[u]) : v + t[u];
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] = (k == 5) ? fmax(red[threadIdx.x], red[threadIdx.x + w]) : red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = k == 7 ? v7 : red[0];
}

// ================================================================== characteristic boundary
// Rate dU/dt (side-local (rho, u_n, u_t, T)) of one boundary node: wave amplitudes of
// eq. thermal_WAV written out with T~ = cs^2 T, incoming amplitudes by scheme (Tab. CBCs), the
// relaxation acting on the incoming acoustic wave, then -S^-1 Lbar (+ T + V for CBC variants).
// up / dw: node values at the neighbouring rows (transverse central differences); u0, s0: normal
// velocity and sound speed of the node at time t, which fix the wave directions.
template <int Q>
__device__ __forceinline__ void char_rate_dir(const double* U, const double* dn, const double* up, const double* dw,
                                              const double* V, double u0, double s0, int scheme, double K,
                                              double alpha, double Pinf, double* rate) {
    constexpr bool THERMAL = Lat<Q>::thermal;
    constexpr double cs2 = Lat<Q>::cs2;
    constexpr double cs = Lat<Q>::cs;
    const bool full = scheme == BC_CBC || scheme == BC_CBC_RELAX;
    const bool relax = scheme == BC_LODI_RELAX || scheme == BC_CBC_RELAX;
    const double rho = U[0], u = U[1], v = U[2], T = U[3];
    const double ir = 1.0 / rho;
    // transverse terms (eq. NSF-CHAR), central in the row direction
    const double T1 = -0.5 * (up[0] * up[2] - dw[0] * dw[2]);
    const double T2 = -v * 0.5 * (up[1] - dw[1]);
    double T3, T4;
    if (THERMAL) {
        T3 = -cs2 * ir * 0.5 * (up[0] * up[3] - dw[0] * dw[3]) - v * 0.5 * (up[2] - dw[2]);
        T4 = -0.5 * (up[3] * up[2] - dw[3] * dw[2]);
    } else {
        T3 = -cs2 * ir * 0.5 * (up[0] - dw[0]) - v * 0.5 * (up[2] - dw[2]);
        T4 = 0.0;
    }
    if (THERMAL) {
        const double s = sqrt(2.0 * cs2 * T);
        const double a = 0.25 * T * ir, b = s * (0.25 / cs2);
        const double L1 = u * (-2.0 * a * dn[0] + 0.5 * dn[3]);
        const double L2 = u * dn[2];
        const double L3 = (u - s) * (a * dn[0] - b * dn[1] + 0.25 * dn[3]);
        const double L4 = (u + s) * (a * dn[0] + b * dn[1] + 0.25 * dn[3]);
        // S T and S V
        const double ST1 = -2.0 * a * T1 + 0.5 * T4, ST2 = T3;
        const double ST3 = a * T1 - b * T2 + 0.25 * T4, ST4 = a * T1 + b * T2 + 0.25 * T4;
        double in1 = 0.0, in2 = 0.0, in3 = 0.0, in4 = 0.0;
        if (full) {
            in1 = ST1 + 0.5 * V[3];
            in2 = ST2 + V[2];
            in3 = ST3 - b * V[1] + 0.25 * V[3];
            in4 = ST4 + b * V[1] + 0.25 * V[3];
        }
        if (relax) {
            const double pr = K * (rho * cs2 * T - Pinf) * ir * (0.25 / cs2);
            in3 += pr - alpha * ST3;
            in4 += pr - alpha * ST4;
        }
        const double B1 = u0 >= 0.0 ? L1 : in1;
        const double B2 = u0 >= 0.0 ? L2 : in2;
        const double B3 = u0 - s0 >= 0.0 ? L3 : in3;
        const double B4 = u0 + s0 >= 0.0 ? L4 : in4;
        rate[0] = rho / T * (B1 - B3 - B4);
        rate[1] = 2.0 * cs2 / s * (B3 - B4);
        rate[2] = -B2;
        rate[3] = -(B1 + B3 + B4);
        if (full) {
            rate[0] += T1;
            rate[1] += T2 + V[1];
            rate[2] += T3 + V[2];
            rate[3] += T4 + V[3];
        }
    } else {
        const double c = cs;
        const double L0 = u * dn[2];
        const double Lm = (u - c) * (cs2 * dn[0] - rho * c * dn[1]);
        const double Lp = (u + c) * (cs2 * dn[0] + rho * c * dn[1]);
        double inm = 0.0, inp = 0.0;
        if (relax) {
            const double pr = K * (cs2 * rho - Pinf);
            inm = pr - alpha * (cs2 * T1 - rho * c * T2);
            inp = pr - alpha * (cs2 * T1 + rho * c * T2);
        }
        const double B0 = u0 >= 0.0 ? L0 : 0.0;
        const double Bm = u0 - s0 >= 0.0 ? Lm : inm;
        const double Bp = u0 + s0 >= 0.0 ? Lp : inp;
        rate[0] = -(Bm + Bp) * (0.5 / cs2);
        rate[1] = (Bm - Bp) * (0.5 / c) * ir;
        rate[2] = -B0;
        rate[3] = 0.0;
    }
}

// sound speed that sets the wave directions at a node of side-local value U0 (time t)
template <int Q>
__device__ __forceinline__ double char_speed(const double* U0) {
    return Lat<Q>::thermal ? sqrt(2.0 * Lat<Q>::cs2 * U0[3]) : Lat<Q>::cs;
}

// U0: the node's side-local value at time t
template <int Q>
__device__ __forceinline__ void char_rate(const double* U, const double* dn, const double* up, const double* dw,
                                          const double* V, const double* U0, int scheme, double K, double alpha,
                                          double Pinf, double* rate) {
    char_rate_dir<Q>(U, dn, up, dw, V, U0[1], char_speed<Q>(U0), scheme, K, alpha, Pinf, rate);
}

__device__ __forceinline__ void to_local(const SideDev& s, const double* g, double* l) {
    l[0] = g[0];
    l[1] = s.sn * g[1 + s.nax];
    l[2] = g[2 - s.nax];
    l[3] = g[3];
}
__device__ __forceinline__ void rate_to_global(const SideDev& s, const double* l, double* g) {
    g[0] = l[0];
    g[1 + s.nax] = s.sn * l[1];
    g[2 - s.nax] = l[2];
    g[3] = l[3];
}

template <int Q>
__device__ __forceinline__ void moments_u4(const double* d, double* u4) {
    double rm1, th;
    moments_dev<Q, double>(d, rm1, u4[1], u4[2], th);
    u4[0] = 1.0 + rm1;
    u4[3] = 1.0 + th;
}

// viscous moments at a node in side-local components (rho, Pi'_nn, Pi'_nt, Pi'_tt, q_n, q_t),
// Pi' = -(1 - 1/(2 tau)) sum c c (f - f^eq), q = (1 - 1/(2 tau)) 1/2 sum f |c - u|^2 (c - u)
template <int Q>
__device__ __forceinline__ void visc_moments(const SideDev& s, const double* d, double tau, double* o6) {
    double rm1, u, v, th;
    moments_dev<Q, double>(d, rm1, u, v, th);
    double fe[Q];
    feq_dev<Q, double>(rm1, u, v, th, fe);
    const double fac = 1.0 - 0.5 / tau;
    double pxx = 0, pxy = 0, pyy = 0, qx = 0, qy = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double c0 = cx<Q>(i), c1 = cy<Q>(i);
        const double fn = d[i] - fe[i];
        pxx -= c0 * c0 * fn; pxy -= c0 * c1 * fn; pyy -= c1 * c1 * fn;
        const double dx = c0 - u, dy = c1 - v;
        const double e = (wt<Q>(i) + d[i]) * (dx * dx + dy * dy);
        qx += e * dx; qy += e * dy;
    }
    pxx *= fac; pxy *= fac; pyy *= fac;
    qx *= 0.5 * fac; qy *= 0.5 * fac;
    o6[0] = 1.0 + rm1;
    o6[1] = s.nax == 0 ? pxx : pyy;
    o6[2] = s.sn * pxy;
    o6[3] = s.nax == 0 ? pyy : pxx;
    o6[4] = s.sn * (s.nax == 0 ? qx : qy);
    o6[5] = s.nax == 0 ? qy : qx;
}

// Mesoscopic viscous terms V (side-local: 0, V_n, V_t, V_T of eq. NSF-CHAR with eq. LaplaceU /
// LaplaceT) of one side row rp from the viscous moments vis[k][len][6] of x_f - M - k, k = 0..2:
// divergence of Pi' and q one-sided along the normal at x_f - M (eq. FD-dx-bw) and central along the
// side between rows rup and rdw (-1: no row there, its moments taken as 0), plus the viscous
// heating Pi':Pi' / mu.
template <int Q>
__device__ __forceinline__ void visc_terms_row(const double* vis, int len, int rp, int rup, int rdw, double nu,
                                               double* V) {
    const double* v0 = &vis[((size_t)0 * len + rp) * 6];
    const double* v1 = &vis[((size_t)1 * len + rp) * 6];
    const double* v2 = &vis[((size_t)2 * len + rp) * 6];
    double upv[6] = {0, 0, 0, 0, 0, 0}, dwv[6] = {0, 0, 0, 0, 0, 0};
    if (rup >= 0) for (int m = 0; m < 6; ++m) upv[m] = vis[((size_t)0 * len + rup) * 6 + m];
    if (rdw >= 0) for (int m = 0; m < 6; ++m) dwv[m] = vis[((size_t)0 * len + rdw) * 6 + m];
    auto dn_ = [&](int m) { return 0.5 * (3.0 * v0[m] - 4.0 * v1[m] + v2[m]); };
    auto dt_ = [&](int m) { return 0.5 * (upv[m] - dwv[m]); };
    const double rho = v0[0];
    V[0] = 0.0;
    V[1] = (dn_(1) + dt_(2)) / rho;
    V[2] = (dn_(2) + dt_(3)) / rho;
    double vt = 0.0;
    if (Lat<Q>::thermal) {
        const double heat = (0.5 * (v0[1] * v0[1] + v0[3] * v0[3]) + v0[2] * v0[2]) / (rho * rho * nu * Lat<Q>::cs2);
        vt = -(dn_(4) + dt_(5)) / (rho * Lat<Q>::cs2) + heat;
    }
    V[3] = vt;
}

// corner LODI along the outward diagonal, rate in global components; ln, s0: the corner's time-n
// value in diagonal-local components and its sound speed (fix the wave directions)
template <int Q>
__device__ __forceinline__ void corner_rate(const CornerDev& c, const double* Uc, const double* U1, const double* U2,
                                            const double* ln, double s0, double* rate) {
    const double tdx = -c.ndy, tdy = c.ndx;
    double l0[4], l1[4], l2[4];
    auto loc = [&](const double* g, double* l) {
        l[0] = g[0]; l[1] = g[1] * c.ndx + g[2] * c.ndy; l[2] = g[1] * tdx + g[2] * tdy; l[3] = g[3];
    };
    loc(Uc, l0); loc(U1, l1); loc(U2, l2);
    constexpr double inv = 0.35355339059327376220;   // 1 / (2 sqrt 2): diagonal spacing sqrt 2
    double dn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) dn[k] = (3.0 * l0[k] - 4.0 * l1[k] + l2[k]) * inv;
    const double zero[4] = {0, 0, 0, 0};
    double rl[4];
    char_rate_dir<Q>(l0, dn, l0, l0, zero, ln[1], s0, c.relax ? BC_LODI_RELAX : BC_LODI, c.K, 0.0, c.Pinf, rl);
    rate[0] = rl[0];
    rate[1] = rl[1] * c.ndx + rl[2] * tdx;
    rate[2] = rl[1] * c.ndy + rl[2] * tdy;
    rate[3] = rl[3];
}

template <int Q, typename T>
__device__ __forceinline__ void write_feq(T* __restrict__ B, unsigned long long pitch, int x, int y, const double* u4) {
    double fe[Q];
    feq_dev<Q, double>(u4[0] - 1.0, u4[1], u4[2], Lat<Q>::thermal ? u4[3] - 1.0 : 0.0, fe);
#pragma unroll
    for (int i = 0; i < Q; ++i) B[pix<Q>(pitch, i, x, y)] = (T)fe[i];
}

// one corner: RK4 of the diagonal LODI system from the moments of the two inward diagonal nodes
// at time n (cdn[8]) and n+1 (D1p, D2p: of their pulled populations); Un: U_c at time n.
// U_c^{n+1} goes to cp_out and, for the owning (x-side) work-group, to the next parity region
template <int Q, bool HIST>
__device__ void corner_rk4(const BndArgs& a, const CornerDev& c, bool owner, const double* D1p, const double* D2p,
                           const double* cdn, const double* Un, double* cp_out) {
    double D1n[4], D2n[4];
    for (int k = 0; k < 4; ++k) { D1n[k] = cdn[k]; D2n[k] = cdn[4 + k]; }
    const double ast[4] = {0.0, 0.5, 0.5, 1.0}, bst[4] = {1.0, 2.0, 2.0, 1.0};
    double k4[4] = {0, 0, 0, 0}, acc[4];
    for (int m = 0; m < 4; ++m) acc[m] = Un[m];
    const double ln[4] = {Un[0], Un[1] * c.ndx + Un[2] * c.ndy, -Un[1] * c.ndy + Un[2] * c.ndx, Un[3]};
    const double s0 = char_speed<Q>(ln);
    for (int st = 0; st < 4; ++st) {
        const double th = ast[st];
        double Y[4], B1[4], B2[4];
        for (int m = 0; m < 4; ++m) {
            Y[m] = Un[m] + ast[st] * k4[m];
            B1[m] = (1.0 - th) * D1n[m] + th * D1p[m];
            B2[m] = (1.0 - th) * D2n[m] + th * D2p[m];
        }
        if (HIST && owner && st > 0)
            for (int m = 0; m < 4; ++m) ((double*)(a.reg_next + c.off_cs))[(st - 1) * 4 + m] = Y[m];
        corner_rate<Q>(c, Y, B1, B2, ln, s0, k4);
        for (int m = 0; m < 4; ++m) acc[m] += bst[st] * (1.0 / 6.0) * k4[m];
    }
    for (int m = 0; m < 4; ++m) cp_out[m] = acc[m];
    if (owner) {
        double* cun = (double*)(a.reg_next + c.off_cu);
        double* cdn_next = (double*)(a.reg_next + c.off_cd);
        for (int m = 0; m < 4; ++m) { cun[m] = acc[m]; cdn_next[m] = D1p[m]; cdn_next[4 + m] = D2p[m]; }
    }
}

// ---------------------------------------------------------------- chunk of a characteristic side
// LDS row lr <-> side row r = r0 - 4 + lr: CR rows, of which CR - 8 are owned, plus 4 halo rows on
// each side (one per RK stage, so chunks need no grid-wide synchronisation).  Node threads
// t < NN = CR M (three wavefronts) each own node (lr = t / M, layer j = t % M + 1) for the whole
// step and keep its time-n value, stage value and RK4 sum in registers; the fourth wavefront pulls
// the strip and fills the strip and corner slots of the stage buffers; lanes of the first pull the
// corners' inward diagonal nodes and run the corner RK4 while the strip pull is in flight.  The
// stage buffers hold every node in side-local components (rho, u_n, u_t, T), slots
// k = -(MS - 1) .. M along the normal (strip nodes, then layers) at slot index k + MS - 1, and are
// double-buffered, so an RK stage needs one barrier.
// A descriptor in the kernel arguments read with a uniform index, its fields passed through
// readfirstlane: selecting between two such copies per lane then selects values.  (A per-lane
// choice between two descriptors is otherwise turned into a load through a per-lane address: a
// vector load from the kernel arguments, each waited for before the next, and the wait also holds
// every load issued before it.)
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uni(unsigned long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double uni(double v) {
    return __longlong_as_double((long long)uni((unsigned long long)__double_as_longlong(v)));
}
__device__ __forceinline__ CornerDev uniform_corner(const CornerDev& c) {
    CornerDev u;
    u.active = uni(c.active); u.zg = uni(c.zg); u.relax = uni(c.relax);
    u.xc = uni(c.xc); u.yc = uni(c.yc); u.vx = uni(c.vx); u.vy = uni(c.vy);
    u.x0 = uni(c.x0); u.y0 = uni(c.y0); u.sxn = uni(c.sxn); u.syn = uni(c.syn);
    u.K = uni(c.K); u.Pinf = uni(c.Pinf); u.ndx = uni(c.ndx); u.ndy = uni(c.ndy);
    u.off_cu = uni(c.off_cu); u.off_cd = uni(c.off_cd); u.off_cs = uni(c.off_cs);
    return u;
}
// corner descriptor of the low (h = false) or high end, per lane, from uniform copies
__device__ __forceinline__ CornerDev pick_corner(const CornerDev& lo, const CornerDev& hi, bool h) {
    CornerDev c;
    c.active = h ? hi.active : lo.active;
    c.zg = h ? hi.zg : lo.zg;
    c.relax = h ? hi.relax : lo.relax;
    c.xc = h ? hi.xc : lo.xc;
    c.yc = h ? hi.yc : lo.yc;
    c.vx = h ? hi.vx : lo.vx;
    c.vy = h ? hi.vy : lo.vy;
    c.x0 = h ? hi.x0 : lo.x0;
    c.y0 = h ? hi.y0 : lo.y0;
    c.sxn = h ? hi.sxn : lo.sxn;
    c.syn = h ? hi.syn : lo.syn;
    c.K = h ? hi.K : lo.K;
    c.Pinf = h ? hi.Pinf : lo.Pinf;
    c.ndx = h ? hi.ndx : lo.ndx;
    c.ndy = h ? hi.ndy : lo.ndy;
    c.off_cu = h ? hi.off_cu : lo.off_cu;
    c.off_cd = h ? hi.off_cd : lo.off_cd;
    c.off_cs = h ? hi.off_cs : lo.off_cs;
    return c;
}

template <int Q> struct ChunkShape {
    static constexpr int M = Lat<Q>::M, MS = (M == 1) ? 2 : 1;
    static constexpr int CR = 192 / M;      // LDS rows per work-group
    static constexpr int NN = CR * M;       // node threads (192: three wavefronts)
    static constexpr int S = M + MS;        // normal slots per row
};

template <int Q, typename T, bool HIST>
__device__ void char_chunk(const T* __restrict__ A, T* __restrict__ B, const BndArgs& a, const SideDev& sd, int chunk) {
    using CS = ChunkShape<Q>;
    constexpr int M = CS::M, MS = CS::MS, CR = CS::CR, NN = CS::NN, S = CS::S;
    constexpr bool TH = Lat<Q>::thermal;
    static_assert(NN == 192, "chunk layout");
    __shared__ double sY[2][CR * S * 4];                  // stage values (side-local)
    __shared__ double sBn[CR * MS * 4], sBp[CR * MS * 4];  // strip at time n, n+1 (side-local)
    __shared__ double sV[CR * 4];                         // mesoscopic viscous terms of time n
    __shared__ double sC[2][2][4];                        // corners [lo, hi][time n, n+1] (global)
    __shared__ double sCn[2][8];                          // time-n moments of their inward diagonal nodes
    __shared__ double sCp[2][2][4];                       // their moments at n+1
    const int tid = threadIdx.x;
    const int len = sd.len, tper = sd.tper;
    const int r0 = chunk * sd.rows;
    const int r1 = min(r0 + sd.rows, len);
    // corners beyond the ends of a side with non-periodic rows (row -1, row len): needed by every
    // chunk whose rows computed in stage 0 (within 3 of its own) reach row 0 / row len - 1, i.e.
    // also by the last-but-one chunk when the last one has fewer than 4 rows; their state and
    // blocks are written by the chunk that owns the end row
    const bool need_c[2] = {!tper && r0 <= 3, !tper && r1 >= len - 3};
    const bool own_c[2] = {!tper && r0 == 0, !tper && r1 == len};
    const bool full = sd.scheme == BC_CBC || sd.scheme == BC_CBC_RELAX;
    const double* ub = (const double*)(a.reg_cur + sd.off_ub);
    double* ubn = (double*)(a.reg_next + sd.off_ub);
    const double* st = (const double*)(a.reg_cur + sd.off_strip);
    double* stn = (double*)(a.reg_next + sd.off_strip);
    const double* vis = (const double*)(a.reg_cur + sd.off_vis);
    double* visn = (double*)(a.reg_next + sd.off_vis);
    auto valid = [&](int r) { return tper || (r >= 0 && r < len); };
    auto phys = [&](int r) { return tper ? ((r % len) + len) % len : r; };
    auto Yat = [&](int buf, int lr, int slot) { return &sY[buf][(lr * S + slot) * 4]; };
    // LDS rows of the corner rows (row -1, row len) where need_c holds: 3 - r0 >= 0, and
    // len - r0 + 4 <= CR - 1 since r1 >= len - 3 and r1 - r0 <= CR - 8
    const int lr_c[2] = {3 - r0, len - r0 + 4};
    const CornerDev cLo = uniform_corner(a.c[sd.corner_lo < 0 ? 0 : sd.corner_lo]);
    const CornerDev cHi = uniform_corner(a.c[sd.corner_hi < 0 ? 0 : sd.corner_hi]);

    const int nlr = min(CR, r1 - r0 + 8);                 // LDS rows in use
    const bool node = tid < NN;
    const int lr = tid / M, jj = tid % M, sj = jj + MS;   // node threads: LDS row, layer j - 1, slot
    const int r = r0 - 4 + lr;
    const bool vr = node && lr < nlr && valid(r);
    const int pr = vr ? phys(r) : 0;

    // ---- phase A: load time level n, re-pull time level n+1 ------------------------------
    // loads first (node value, strip values, corner inputs), uses after the pulls, so that their
    // latencies overlap
    double g_u[4];
    {
        const double* src = &ub[((size_t)jj * len + pr) * 4];
        for (int m = 0; m < 4; ++m) g_u[m] = src[m];
    }
    constexpr int KB = (MS + M - 1) / M;   // strip slots loaded per node thread (2 for M = 1)
    double g_b[KB][4];
    for (int kb = 0; kb < KB; ++kb) {
        const int k = jj + kb * M;
        const double* src = &st[((size_t)(k < MS ? k : 0) * len + pr) * 4];
        for (int m = 0; m < 4; ++m) g_b[kb][m] = src[m];
    }
    // corner inputs: threads 0..3 pull the corners' inward diagonal nodes (corner tid / 2, node
    // tid % 2 + 1 steps in; one whole pull per thread, so the lattice offsets are constants), threads
    // 4..27 load the 2 x 4 time-n values and the 2 x 8 time-n moments of those nodes
    double g_c = 0.0;
    const bool cpull = tid < 4 && need_c[tid >> 1];
    const int cv = tid - 4, cve = cv / 12, cvm = cv % 12;
    const bool cval = cv >= 0 && cv < 24 && need_c[cve];
    if (cval) {
        const CornerDev c = pick_corner(cLo, cHi, cve == 1);
        g_c = cvm < 4 ? ((const double*)(a.reg_cur + c.off_cu))[cvm] : ((const double*)(a.reg_cur + c.off_cd))[cvm - 4];
    }
    // viscous terms of time level n (frozen during the RK stages)
    if (full && !sd.vfd) {
        const double nu = (a.tau - 0.5) * Lat<Q>::cs2;
        for (int l2 = tid; l2 < nlr; l2 += blockDim.x) {
            const int rr = r0 - 4 + l2;
            if (!valid(rr)) continue;
            visc_terms_row<Q>(vis, len, phys(rr), valid(rr + 1) ? phys(rr + 1) : -1, valid(rr - 1) ? phys(rr - 1) : -1,
                              nu, &sV[l2 * 4]);
        }
    }
    // pulls, the fourth wavefront first: per row the strip nodes x_f (.. x_f - MS + 1), then for
    // CBC sides the three nodes of the viscous moments, x_f - M - kv (kv = 0, 1, 2): the first nodes
    // inward of x_f none of whose populations streamed from the layers (a node there that is no
    // bulk node holds an equilibrium, whose non-equilibrium moments are 0)
    const int KP = full ? MS + 3 : MS;
    for (int p = (tid + 256 - NN) & 255; p < nlr * KP; p += 256) {
        const int lp = p / KP, k = p % KP, rq = r0 - 4 + lp;
        if (!valid(rq)) continue;
        const int rp = phys(rq);
        const bool owned = rq >= r0 && rq < r1;
        if (k < MS) {
            int x, y; side_node(sd, -k, rp, x, y);
            double d[Q];
            pull_node<Q, T>(A, a, x, y, d);
            double u4[4];
            moments_u4<Q>(d, u4);
            if (owned) for (int m = 0; m < 4; ++m) stn[((size_t)k * len + rp) * 4 + m] = u4[m];
            to_local(sd, u4, &sBp[(lp * MS + k) * 4]);
            continue;
        }
        if (!owned) continue;
        const int kv = k - MS;
        int x, y; side_node(sd, -(M + kv), rp, x, y);
        const bool bulk = (a.xper || (x >= M && x <= a.nx - 1 - M)) && (a.yper || (y >= M && y <= a.ny - 1 - M));
        double o6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (bulk) {
            double d[Q];
            pull_node<Q, T>(A, a, x, y, d);
            visc_moments<Q>(sd, d, a.tau, o6);
        }
        for (int m = 0; m < 6; ++m) visn[((size_t)kv * len + rp) * 6 + m] = o6[m];
    }
    if (cpull) {   // (after the pulls: no node thread of a LODI side pulls, so these loads overlap the rest)
        const CornerDev c = pick_corner(cLo, cHi, (tid >> 1) == 1);
        const int x = c.xc + ((tid & 1) + 1) * c.vx, y = c.yc + ((tid & 1) + 1) * c.vy;
        double d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = (double)A[pix<Q>(a.pitch, i, x - cx<Q>(i), y - cy<Q>(i))];
        moments_u4<Q>(d, sCp[tid >> 1][tid & 1]);
    }
    // stage-0 inputs: node values, strip at time n, corner values at time n in the corner rows
    double Y0[4] = {0.0, 0.0, 0.0, 0.0};
    if (vr) {
        to_local(sd, g_u, Y0);
        for (int m = 0; m < 4; ++m) Yat(0, lr, sj)[m] = Y0[m];
        for (int kb = 0; kb < KB; ++kb) {
            const int k = jj + kb * M;
            if (k >= MS) continue;
            double l[4];
            to_local(sd, g_b[kb], l);
            for (int m = 0; m < 4; ++m) { sBn[(lr * MS + k) * 4 + m] = l[m]; Yat(0, lr, MS - 1 - k)[m] = l[m]; }
        }
    }
    if (cval) {
        if (cvm < 4) {
            sC[cve][0][cvm] = g_c;
            sC[cve][1][cvm] = g_c;
            // the corner row of the stage-0 input: this component, side-local, on every layer
            const int lm = cvm == 0 || cvm == 3 ? cvm : (cvm == 1 + sd.nax ? 1 : 2);
            const double v = cvm == 1 + sd.nax ? sd.sn * g_c : g_c;
            for (int k = MS; k < S; ++k) Yat(0, lr_c[cve], k)[lm] = v;
        } else {
            sCn[cve][cvm - 4] = g_c;
        }
    }
    // corner RK4 (time-n values and n+1 moments written above by lanes of this same wavefront, in
    // program order): lane 0 the low corner, lane 2 the high corner, while the fourth wavefront
    // is still pulling the strip
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (tid < 4 && (tid & 1) == 0 && need_c[tid >> 1]) {
        const int e = tid >> 1;
        corner_rk4<Q, HIST>(a, pick_corner(cLo, cHi, e == 1), sd.owns_corners && own_c[e], sCp[e][0], sCp[e][1], sCn[e],
                            sC[e][0], sC[e][1]);
    }
    __syncthreads();

    // ---- phase B: RK4; stage st computes rates on rows within 3 - st of the owned range --------
    const double ast[4] = {0.0, 0.5, 0.5, 1.0}, bst[4] = {1.0, 2.0, 2.0, 1.0};
    // normal differences at layer j: eq. FD-dx-bw at j = M (and the backward second difference of
    // the -FD variant, Sec. 4.2, for M = 3), eq. FD-dx-center below; offsets -3 .. +1 from slot sj
    const bool one = jj == M - 1;
    const int sm1 = sj - 1, sm2 = max(sj - 2, 0), sm3 = max(sj - 3, 0), sp1 = min(sj + 1, S - 1);
    const double u0 = Y0[1], s0 = char_speed<Q>(Y0);
    double Ys[4], acc[4], Vl[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m = 0; m < 4; ++m) { Ys[m] = Y0[m]; acc[m] = Y0[m]; }
    if (node && full && !sd.vfd)
        for (int m = 0; m < 4; ++m) Vl[m] = sV[lr * 4 + m];
    const bool owned = vr && r >= r0 && r < r1;
    for (int stg = 0; stg < 4; ++stg) {
        const int cur = stg & 1, nxt = cur ^ 1;
        const int he = 3 - stg;
        if (node) {
            if (vr && r >= r0 - he && r < r1 + he) {
                const double* vm1 = Yat(cur, lr, sm1);
                const double* vm2 = Yat(cur, lr, sm2);
                const double* vp1 = Yat(cur, lr, sp1);
                const double* up = Yat(cur, lr + 1, sj);
                const double* dw = Yat(cur, lr - 1, sj);
                double dn[4];
                for (int m = 0; m < 4; ++m)
                    dn[m] = one ? 0.5 * (3.0 * Ys[m] - 4.0 * vm1[m] + vm2[m]) : 0.5 * (vp1[m] - vm1[m]);
                if (full && sd.vfd) {
                    // the -FD variant (Sec. 4.2, treatment of viscous terms): Laplacians of eq.
                    // NSF-CHAR by second differences of the stage values, heating from the first
                    // differences; c_p / Pr = 2
                    const double* vm3 = Yat(cur, lr, sm3);
                    const double nu = (a.tau - 0.5) * Lat<Q>::cs2;
                    double lap[4];
                    for (int m = 1; m < 4; ++m) {
                        const double d2n = one ? (M == 3 ? 2.0 * Ys[m] - 5.0 * vm1[m] + 4.0 * vm2[m] - vm3[m] : 0.0)
                                               : vp1[m] - 2.0 * Ys[m] + vm1[m];
                        lap[m] = d2n + up[m] - 2.0 * Ys[m] + dw[m];
                    }
                    Vl[1] = nu * lap[1];
                    Vl[2] = nu * lap[2];
                    if (TH) {
                        const double sa = dn[1] - 0.5 * (up[2] - dw[2]), sb = 0.5 * (up[1] - dw[1]) + dn[2];
                        Vl[3] = 2.0 * nu * lap[3] + nu * (1.0 / Lat<Q>::cs2) * (sa * sa + sb * sb);
                    }
                }
                double rl[4];
                char_rate_dir<Q>(Ys, dn, up, dw, Vl, u0, s0, sd.scheme, sd.K, sd.alpha, sd.Pinf, rl);
                for (int m = 0; m < 4; ++m) acc[m] += bst[stg] * (1.0 / 6.0) * rl[m];
                if (stg < 3) {
                    for (int m = 0; m < 4; ++m) Ys[m] = Y0[m] + ast[stg + 1] * rl[m];
                    for (int m = 0; m < 4; ++m) Yat(nxt, lr, sj)[m] = Ys[m];
                    if (HIST && owned) {
                        double g[4];
                        rate_to_global(sd, Ys, g);
                        double* ys = (double*)(a.reg_next + sd.off_stage);
                        for (int m = 0; m < 4; ++m) ys[(((size_t)stg * M + jj) * len + r) * 4 + m] = g[m];
                    }
                }
            }
        } else if (stg < 3) {
            const int u = tid - NN;
            const double th = ast[stg + 1];
            if (u < 2 && need_c[u]) {   // corner rows of the next stage input
                double g[4], l[4];
                for (int m = 0; m < 4; ++m) g[m] = (1.0 - th) * sC[u][0][m] + th * sC[u][1][m];
                to_local(sd, g, l);
                for (int k = MS; k < S; ++k)
                    for (int m = 0; m < 4; ++m) Yat(nxt, lr_c[u], k)[m] = l[m];
            }
            for (int l2 = u; l2 < nlr; l2 += 256 - NN)   // strip slots of the next stage input
                for (int k = 0; k < MS; ++k)
                    for (int m = 0; m < 4; ++m)
                        Yat(nxt, l2, MS - 1 - k)[m] = (1.0 - th) * sBn[(l2 * MS + k) * 4 + m] + th * sBp[(l2 * MS + k) * 4 + m];
        }
        if (stg < 3) __syncthreads();
    }

    // ---- phase C: new boundary state and reconstruction of the layers ------------------------
    if (owned) {
        double u4[4];
        rate_to_global(sd, acc, u4);
        for (int m = 0; m < 4; ++m) ubn[((size_t)jj * len + r) * 4 + m] = u4[m];
        int x, y; side_node(sd, jj + 1, r, x, y);
        if (sd.meso == 0) {   // equilibrium BC: all populations at equilibrium
            write_feq<Q, T>(B, a.pitch, x, y, u4);
        } else {              // eq. NEEP: plus the post-collision non-equilibrium part of x_f
            int xf, yf; side_node(sd, 0, r, xf, yf);
            double d[Q], fe[Q];
            pull_node<Q, T>(A, a, xf, yf, d);
            double rm1, ux, uy, thv;
            moments_dev<Q, double>(d, rm1, ux, uy, thv);
            feq_dev<Q, double>(rm1, ux, uy, thv, fe);
            const double c = 1.0 - a.omega;
#pragma unroll
            for (int i = 0; i < Q; ++i) d[i] = c * (d[i] - fe[i]);
            feq_dev<Q, double>(u4[0] - 1.0, u4[1], u4[2], Lat<Q>::thermal ? u4[3] - 1.0 : 0.0, fe);
#pragma unroll
            for (int i = 0; i < Q; ++i) B[pix<Q>(a.pitch, i, x, y)] = (T)(fe[i] + d[i]);
        }
    }
    // the x-side's work-groups write the M x M corner blocks (fourth wavefront; the corner values
    // at n+1 were set in stage 0)
    if (sd.owns_corners && !node) {
        const int u = tid - NN;
        if (u < 2 * M * M) {
            const int e = u / (M * M), jx = (u / M) % M, jy = u % M;
            if (own_c[e]) {
                const CornerDev c = pick_corner(cLo, cHi, e == 1);
                write_feq<Q, T>(B, a.pitch, c.x0 + c.sxn * jx, c.y0 + c.syn * jy, sC[e][1]);
            }
        }
    }
}

// ---------------------------------------------------------------- zero-gradient side (eq. zg-bc)
template <int Q, typename T>
__device__ void zg_chunk(const T* __restrict__ A, T* __restrict__ B, const BndArgs& a, const SideDev& sd, int chunk) {
    constexpr int M = Lat<Q>::M;
    const T omega = sizeof(T) == 4 ? (T)(float)a.omega : (T)a.omega;
    const int r = chunk * sd.rows + threadIdx.x;
    if (threadIdx.x < sd.rows && r < sd.len) {
        int x, y; side_node(sd, 0, r, x, y);
        T d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int xs = x - cx<Q>(i), ys = y - cy<Q>(i);
            if (a.xper) xs = wrapi(xs, a.nx);
            if (a.yper) ys = wrapi(ys, a.ny);
            d[i] = A[pix<Q>(a.pitch, i, xs, ys)];
        }
        collide_dev<Q, T>(d, omega);
        for (int j = 1; j <= M; ++j) {
            int xb, yb; side_node(sd, j, r, xb, yb);
#pragma unroll
            for (int i = 0; i < Q; ++i) B[pix<Q>(a.pitch, i, xb, yb)] = d[i];
        }
    }
    // corner blocks copy the post-collision state of the inward diagonal node
    if (!sd.tper && sd.owns_corners && threadIdx.x == 0) {
        for (int e = 0; e < 2; ++e) {
            const int ci = e == 0 ? sd.corner_lo : sd.corner_hi;
            const bool mine = e == 0 ? (chunk == 0) : ((chunk + 1) * sd.rows >= sd.len);
            if (ci < 0 || !mine) continue;
            const CornerDev& c = a.c[ci];
            const int x = c.xc + c.vx, y = c.yc + c.vy;
            T d[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                int xs = x - cx<Q>(i), ys = y - cy<Q>(i);
                d[i] = A[pix<Q>(a.pitch, i, xs, ys)];
            }
            collide_dev<Q, T>(d, omega);
            for (int jx = 0; jx < M; ++jx)
                for (int jy = 0; jy < M; ++jy) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) B[pix<Q>(a.pitch, i, c.x0 + c.sxn * jx, c.y0 + c.syn * jy)] = d[i];
                }
        }
    }
}

// one boundary work-group: find its side and chunk
template <int Q, typename T, bool HIST>
__device__ __forceinline__ void boundary_job(const T* __restrict__ A, T* __restrict__ B, const BndArgs& a, int b) {
    int s = 0;
    while (s < 4 && !(a.s[s].nblk > 0 && b >= a.s[s].blk0 && b < a.s[s].blk0 + a.s[s].nblk)) ++s;
    if (s == 4) return;
    const SideDev& sd = a.s[s];
    if (sd.kind == KIND_CHAR) char_chunk<Q, T, HIST>(A, B, a, sd, b - sd.blk0);
    else if (sd.kind == KIND_ZG) zg_chunk<Q, T>(A, B, a, sd, b - sd.blk0);
}

// Waves per SIMD the step kernel is compiled for: 3 for D2Q37 in float (caps registers at 168
// and matches the 3 work-groups per CU that the boundary LDS allows), 2 otherwise.
template <int Q, typename T> struct StepOcc { static constexpr int waves = (Q == 37 && sizeof(T) == 4) ? 3 : 2; };

// One full time step: work-groups [0, nbnd) are boundary chunks (dispatched first), the rest bulk
// tiles of 256 nodes, bpr tiles per row, rows from g.y0.  FP32: row-major order (the whole chip
// sweeps the rows in order, which streams best from HBM; an XCD-aware order that keeps a row's
// tiles on one L2 removes the ~10 % duplicate edge-line fetches but streams slower, 77.6 % ->
// 74.2 %).  FP64: XCD-aware order -- work-group b runs on XCD b % 8, and each XCD walks one
// contiguous range of tiles (74.5 % -> 75.7 % on 4096 x 2048); the host rounds the boundary
// work-groups up to a multiple of 8 for it (the extra ones return at once).  The row of tile t is
// t / bpr computed as umulhi(t, magic) with magic = floor(2^32 / bpr) + 1 for bpr > 1 (exact
// while t * bpr < 2^32, checked on the host), which stays on the scalar unit.
template <int Q, typename T, bool PX, bool PY, bool HIST>
__global__ __launch_bounds__(256, (StepOcc<Q, T>::waves)) void k_step(const T* __restrict__ A, T* __restrict__ B, BndArgs a,
                                                                     BulkArgs g, int nbnd, int bpr, unsigned magic) {
    const int b = (int)blockIdx.x;
    if (b < nbnd) {
        boundary_job<Q, T, HIST>(A, B, a, b);
        return;
    }
    unsigned t = (unsigned)(b - nbnd);
    if (sizeof(T) == 8) {
        const int nbnd8 = (nbnd + 7) & ~7;
        if (b < nbnd8) return;
        const unsigned t0 = (unsigned)(b - nbnd8), nt = gridDim.x - (unsigned)nbnd8, per = nt >> 3;
        t = (nt & 7u) ? t0 : (t0 & 7u) * per + (t0 >> 3);
    }
    const unsigned row = bpr == 1 ? t : __umulhi(t, magic);   // (2^32 + 1 does not fit for bpr = 1)
    const int tile = (int)(t - row * (unsigned)bpr);
    bulk_node<Q, T, PX, PY, HIST>(A, B, g, tile * 256 + (int)threadIdx.x, g.y0 + (int)row);
}

}  // namespace lbm
