/*
 * lbm3d.h -- C ABI of the three-dimensional path of liblbm_hip.so: thermal lattice Boltzmann
 * on the D3Q39 stencil with characteristic (LODI / CBC) boundaries on the two faces normal to one
 * axis (x, y or z) of a box that is periodic along the other two, on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Klass, Gabbana & Bartel, "Characteristic Boundary Condition for Thermal Lattice
 * Boltzmann Methods" (arXiv 2307.16766), Appendix A (CBC and LODI for the Navier-Stokes-Fourier
 * equations in d = 3):
 *   - bulk: BGK lattice Boltzmann (Sec. 2, eq. lbe and eq. bgk) on D3Q39, the degree-7
 *     Gauss-Hermite rule with cs^2 = 2/3, with the 3rd-order Hermite equilibrium of eq. feq-3
 *     (d = 3 in its polynomials); T = sum f |c - u|^2 / (3 rho cs^2);
 *   - faces: the characteristic system of Appendix A (A, S, S^-1, Lambda in the local frame
 *     (rho, u_n, u_t1, u_t2, T), c_v = 3/2, gamma = 5/3), its transverse terms along the two
 *     tangential axes and
 *     viscous terms from the mesoscopic moments at x_f - M, x_f - M - 1, x_f - M - 2 (the first
 *     bulk nodes none of whose populations streamed from the layers); incoming amplitudes by
 *     the four schemes of Tab. CBCs; RK4 as in two dimensions; equilibrium or NEEP
 *     reconstruction of all populations on the M = 3 layers.
 *   The paper gives no edge or corner treatment in 3D: the two axes along the faces are always
 *   periodic.
 *
 * Conventions as in lbm.h: lattice units, T dimensionless with reference 1, caller-owned device
 * memory (d_* pointers) and stream, asynchronous calls except lbm3d_diagnostics, negative error
 * codes from enum lbm_status, messages from lbm3d_last_error.  Macroscopic arrays are FP64
 * [nz][ny][nx] with x fastest.  Face order: low end, high end of the face axis.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include <stddef.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

enum lbm3d_stencil { LBM_D3Q39 = 39 };

/* Face types: LBM_BC_PERIODIC (both faces), LBM_BC_LODI .. LBM_BC_CBC_RELAX, LBM_BC_ZG. */
typedef struct lbm3d_config {
    int stencil;     /* LBM_D3Q39 */
    int precision;   /* lbm_precision: LBM_FP64 or LBM_FP32DEV (deviations f - w_i in float) */
    int nx, ny, nz;  /* nodes; along the face axis >= 2M+3 = 9 with boundary faces, 3M+3 = 12 with a
                        CBC face (>= 4 if periodic); along the other axes >= 4 */
    double tau;      /* BGK relaxation time, > 1/2; nu = (tau - 1/2) cs^2 */
    int bc[2];       /* lbm_bc of the faces at the low and the high end of the face axis */
    int axis;        /* face axis: 0 = x (faces x = 0, nx - 1), 1 = y, 2 = z; the other two axes
                        are periodic.  Appendix A's system is written for the normal along x; a
                        face normal to y or z uses it rotated, with the local frame (u_n, u_t1,
                        u_t2) = (u_y, u_z, u_x) or (u_z, u_x, u_y).  Internally the library
                        stores the grid with the face axis as its fastest axis; input and output
                        arrays keep the caller's [nz][ny][nx] layout. */
} lbm3d_config;

typedef struct lbm3d_ctx lbm3d_ctx;

/* Device workspace for this configuration (bytes); 0 for an invalid configuration. */
size_t lbm3d_workspace_bytes(const lbm3d_config* cfg);

/* Create a context and set f = f^eq(rho0, u0, T0) at every node (face states from the same
 * fields).  d_workspace: device buffer of at least lbm3d_workspace_bytes(cfg) bytes, 256-byte
 * aligned.  hip_stream: hipStream_t (NULL for the null stream).  d_rho0 .. d_T0: device FP64
 * [nz][ny][nx].  On success *out receives the context. */
int lbm3d_init(const lbm3d_config* cfg, void* d_workspace, size_t workspace_bytes, void* hip_stream,
               const double* d_rho0, const double* d_ux0, const double* d_uy0, const double* d_uz0,
               const double* d_T0, lbm3d_ctx** out);

/* Relaxation of face 0..1, or of both with face = -1 (eq. LODI-Relax / CBC-Relax).  The
 * incoming acoustic amplitude receives -alpha * T_x,i + K (P - P_inf) / (5 rho cs^2) (the
 * pressure coefficient of the acoustic rows of S in d = 3), K = sigma (1 - mach^2) c_inf / length,
 * c_inf = sqrt(5/3 cs^2 T_inf), P_inf = rho_inf cs^2 T_inf; length <= 0 selects nx. */
int lbm3d_cbc_params(lbm3d_ctx* ctx, int face, const lbm_relax* p);

/* Mesoscopic BC (lbm_recon) of face 0..1 or of both characteristic faces (face = -1). */
int lbm3d_reconstruction(lbm3d_ctx* ctx, int face, int mode);

/* Advance nsteps time steps: bulk kernel, then the face kernels (strip and viscous moments, four
 * RK4 stages, reconstruction) on the caller's stream. */
int lbm3d_step(lbm3d_ctx* ctx, int nsteps);

/* FP64 rho, u_x, u_y, u_z, T [nz][ny][nx] of the current state (device pointers). */
int lbm3d_macroscopic(lbm3d_ctx* ctx, double* d_rho, double* d_ux, double* d_uy, double* d_uz, double* d_T);

/* Full populations f_i (FP64, library velocity order, [q][nz][ny][nx]) into device memory. */
int lbm3d_populations(lbm3d_ctx* ctx, double* d_out);

/* Synchronising diagnostics into host h_out[8]: mass, momentum x/y/z, energy (1/2 sum f |c|^2),
 * loss (sum over bulk nodes of (P - cs^2)^2), max |u|, non-finite population count.  Returns
 * LBM_E_NONFINITE when that count is non-zero. */
int lbm3d_diagnostics(lbm3d_ctx* ctx, double* h_out);

/* Bulk-kernel timing with HIP events on the context's stream (measurement only): enable = n > 0
 * times every n-th bulk launch (the first after this call included), 0 turns it off, negative
 * values return LBM_E_ARG; lbm3d_bulk_kernel_time returns the summed milliseconds and the number
 * of timed launches. */
int lbm3d_set_kernel_timing(lbm3d_ctx* ctx, int enable);
int lbm3d_bulk_kernel_time(lbm3d_ctx* ctx, double* total_ms, long* launches);

/* Lattice of the library: returns q and fills M, cs2, w[q], cx[q], cy[q], cz[q] (any may be
 * NULL); negative for an unknown stencil.  Host only. */
int lbm3d_lattice_info(int stencil, int* M, double* cs2, double* w, int* cx, int* cy, int* cz);

const char* lbm3d_last_error(const lbm3d_ctx* ctx);
void lbm3d_destroy(lbm3d_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H */
