/*
 * lbm.h -- C ABI of liblbm_hip.so: thermal lattice Boltzmann method with characteristic
 * (LODI / CBC) non-reflecting boundary conditions on one AMD Instinct MI355X (gfx950).
 *
 * Method: Klass, Gabbana & Bartel, "Characteristic Boundary Condition for Thermal Lattice
 * Boltzmann Methods" (arXiv 2307.16766).
 *   - bulk: BGK lattice Boltzmann equation (Sec. 2, eq. lbe and eq. bgk) on the single-speed
 *     D2Q9 stencil (isothermal, 2nd-order equilibrium) or the multi-speed D2Q17 (Tab. d2q17;
 *     3rd-order Hermite equilibrium, eq. feq-3) and D2Q37 stencils (Tab. d2q37; 4th-order
 *     Hermite equilibrium, eq. feq-4);
 *   - boundary: layerwise characteristic analysis on the M outer layers (Sec. 3.3), wave
 *     amplitudes of eq. thermal_WAV, incoming amplitudes by one of the four schemes of
 *     Tab. CBCs (eq. PNR, LODI-Relax, CBC-PNR, CBC-Relax), RK4 in time, equilibrium or NEEP
 *     Dirichlet reconstruction of all populations on the layers (Sec. 3.3 "Mesoscopic BC",
 *     eq. NEEP).
 *
 * Conventions
 *   - Grid: nx * ny nodes, row-major, x fastest.  Side order: x = 0, x = nx-1, y = 0, y = ny-1.
 *   - Units: lattice units (dx = dt = 1).  T is dimensionless with reference T = 1; the lattice
 *     temperature is cs^2 T and the pressure P = rho cs^2 T.  D2Q9 is isothermal (T = 1).
 *   - Memory: every pointer argument named d_* is device memory on the current HIP device.
 *     The caller owns all device memory (workspace, fields, checkpoint buffers) and the HIP
 *     stream; the library borrows them until lbm_destroy.  The library owns only its host-side
 *     context (and, while kernel timing is enabled, the timing events).
 *   - Asynchrony: every call that takes a context enqueues work on the caller's stream and
 *     returns without synchronising, except lbm_diagnostics, lbm_save, lbm_restore,
 *     lbm_adjoint and lbm_step's non-finite checks (lbm_diag_every), which synchronise.
 *   - Errors: functions return LBM_OK (0) or a negative code; nothing throws across the ABI.
 *     lbm_last_error(ctx) gives a message for the last failure on that context
 *     (lbm_last_error(NULL) for failures before a context exists).
 *   - Macroscopic input and output are FP64 [ny][nx] arrays whatever the storage precision.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lbm_status {
    LBM_OK = 0,
    LBM_E_ARG = -1,          /* invalid argument or configuration */
    LBM_E_HIP = -2,          /* a HIP runtime call failed */
    LBM_E_NONFINITE = -3,    /* diagnostics found a non-finite population */
    LBM_E_STATE = -4,        /* call not valid in the context's current state */
    LBM_E_UNSUPPORTED = -5   /* valid but not supported combination */
};

enum lbm_stencil { LBM_D2Q9 = 9, LBM_D2Q17 = 17, LBM_D2Q37 = 37 };

/* Storage precision of the populations.  FP64 stores f - w_i in double.  FP32DEV stores the
 * deviation f - w_i from the lattice weight in float and runs the bulk update in float; the
 * boundary solve, the macroscopic output and the diagnostics are FP64 in both modes. */
enum lbm_precision { LBM_FP64 = 0, LBM_FP32DEV = 1 };

/* Boundary types (Tab. CBCs, eq. zg-bc).  Periodic sides must come in pairs (x0 with x1,
 * y0 with y1).  Corners (both axes non-periodic) are supported between characteristic sides
 * (LODI..CBC_RELAX) and between zero-gradient sides. */
enum lbm_bc {
    LBM_BC_PERIODIC = 0,
    LBM_BC_LODI = 1,        /* eq. thermal_LODI_macro_evo with eq. PNR */
    LBM_BC_LODI_RELAX = 2,  /* eq. thermal_LODI_macro_evo with eq. LODI-Relax */
    LBM_BC_CBC = 3,         /* eq. thermal_CBC_macro_evo with eq. CBC-PNR (thermal stencils) */
    LBM_BC_CBC_RELAX = 4,   /* eq. thermal_CBC_macro_evo with eq. CBC-Relax (thermal stencils) */
    LBM_BC_ZG = 5,          /* zero-gradient copy of the adjacent bulk node, eq. zg-bc */
    LBM_BC_DIRICHLET = 6    /* equilibrium populations of a fixed profile (inlet) */
};

typedef struct lbm_config {
    int stencil;     /* LBM_D2Q9, LBM_D2Q17 or LBM_D2Q37 */
    int precision;   /* lbm_precision */
    int nx, ny;      /* nodes; non-periodic axes need >= 2M+3 nodes (3M+3 normal to a CBC side),
                        periodic ones >= M+1 */
    double tau;      /* BGK relaxation time, > 1/2; nu = (tau - 1/2) cs^2 (Sec. 2) */
    int bc[4];       /* lbm_bc for sides x0, x1, y0, y1 */
} lbm_config;

/* Relaxation parameters of one characteristic side (eq. LODI-Relax / eq. CBC-Relax).  The
 * incoming acoustic amplitude receives  -alpha * T_x,i + K (P - P_inf) / (4 rho cs^2)
 * (thermal stencils) or  -alpha * T_x,i + K (P - P_inf)  (D2Q9), with
 * K = sigma (1 - mach^2) c_inf / length, c_inf = sqrt(2 cs^2 T_inf) (thermal) or cs (D2Q9),
 * P_inf = rho_inf cs^2 T_inf.  length <= 0 selects the domain extent normal to the side.
 * Sides without relaxation (LODI, CBC) ignore these values.  Defaults: all zero except
 * rho_inf = T_inf = 1. */
typedef struct lbm_relax {
    double sigma;
    double alpha;
    double rho_inf;
    double T_inf;
    double mach;
    double length;
} lbm_relax;

/* Mesoscopic BC of a characteristic side (Sec. 3.3 "Mesoscopic BC"): the populations of the M
 * layers are set from the new boundary state U_b either to the equilibrium f^eq(U_b) (default) or,
 * with NEEP (eq. NEEP), to f^eq(U_b) plus the non-equilibrium part f - f^eq(U) of the adjacent
 * bulk node x_f of the same row (post-collision, like every stored population).  Corner blocks
 * stay at equilibrium. */
enum lbm_recon { LBM_RECON_EQUILIBRIUM = 0, LBM_RECON_NEEP = 1 };

/* Viscous terms V of a CBC side (eq. NSF-CHAR).  MESO (default): from the non-equilibrium
 * moments of the populations (Sec. 3.3 "Evaluation of viscous terms", eq. LaplaceU and eq.
 * LaplaceT) at x_f - M, x_f - M - 1, x_f - M - 2, the first bulk nodes of the row none of whose
 * populations streamed from the layers, one-sided along the normal and central along the side;
 * frozen at time t during the RK4 stages and shared by the M layers of a row.  FD: the -FD variant of Sec. 4.2 ("Treatment of viscous terms"): nu lap(u) and
 * 2 nu lap(T) by second differences of the macroscopic values of each layer (the backward
 * four-point formula on the outermost layer, central differences on inner layers and along the
 * side) plus the viscous heating from first differences, evaluated at every RK4 stage. */
enum lbm_visc { LBM_VISC_MESO = 0, LBM_VISC_FD = 1 };

typedef struct lbm_ctx lbm_ctx;

/* Device workspace the caller must provide to lbm_init for this configuration (bytes).
 * Returns 0 for an invalid configuration. */
size_t lbm_workspace_bytes(const lbm_config* cfg);

/* Create a context and set the initial state f = f^eq(rho0, u0, T0) at every node (Sec. 2,
 * "Initialize"); boundary states start from the same fields.  d_workspace: device buffer of
 * at least lbm_workspace_bytes(cfg) bytes, 256-byte aligned.  hip_stream: hipStream_t (NULL
 * for the null stream).  d_rho0, d_ux0, d_uy0, d_T0: device FP64 [ny][nx]; d_T0 may be NULL
 * for D2Q9.  On success *out receives the context. */
int lbm_init(const lbm_config* cfg, void* d_workspace, size_t workspace_bytes, void* hip_stream,
             const double* d_rho0, const double* d_ux0, const double* d_uy0, const double* d_T0,
             lbm_ctx** out);

/* Set the relaxation parameters of side 0..3, or of every side with side = -1.  Takes effect
 * from the next lbm_step.  Discards a run recorded with lbm_record (lbm_adjoint then returns
 * LBM_E_STATE), as do lbm_reconstruction and lbm_viscous. */
int lbm_cbc_params(lbm_ctx* ctx, int side, const lbm_relax* p);

/* Reconstruction mode (lbm_recon) of side 0..3, or of every characteristic side with side = -1;
 * NEEP on a non-characteristic side returns LBM_E_STATE.  Takes effect from the next lbm_step. */
int lbm_reconstruction(lbm_ctx* ctx, int side, int mode);

/* Viscous-term mode (lbm_visc) of side 0..3, or of every CBC side with side = -1; FD on a side
 * that is not CBC or CBC_RELAX returns LBM_E_STATE.  Takes effect from the next lbm_step. */
int lbm_viscous(lbm_ctx* ctx, int side, int mode);

/* Fixed profile of a Dirichlet side: d_U is device FP64 [len][4] = (rho, u_x, u_y, T) per row
 * along the side (len = ny for x-sides, nx for y-sides).  Default: the initial fields on the
 * first boundary layer.  Writes the equilibrium populations of every layer immediately, and
 * discards a run recorded with lbm_record (lbm_adjoint then returns LBM_E_STATE). */
int lbm_dirichlet_profile(lbm_ctx* ctx, int side, const double* d_U);

/* Advance nsteps time steps: fused stream + collide on the bulk, characteristic boundary solve
 * and reconstruction on the boundary layers (Sec. 3.3, Fig. flowchart-cbc-lbm).  With a check
 * interval n > 0 set by lbm_diag_every, every step that brings the step count to a multiple of
 * n is followed by the diagnostics' non-finite count (one read of the populations, and the
 * call synchronises the stream there); when it is positive lbm_step stops and returns
 * LBM_E_NONFINITE, with the state of that step kept and lbm_steps_done telling which step. */
int lbm_step(lbm_ctx* ctx, int nsteps);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the diagnostics of lbm_diagnostics, enqueued on the
 * context's stream without synchronising, allocating nothing and touching no workspace scratch.
 * d_out: device FP64 [8], the same quantities as lbm_diagnostics' h_out ([7] = the step count
 * when the call is made); the caller reads [6] for non-finite populations (this call does not
 * return LBM_E_NONFINITE).  The partial sums live in a fixed device array of the library
 * (16384 partials per quantity, 1 MiB per device, kept until the process ends); grids of more
 * than 16384 row tiles of 256 nodes let each work-group fold several tiles, so every grid that
 * lbm_init accepts fits, and up to that size the result equals lbm_diagnostics' bit for bit
 * (beyond it the sums differ by rounding only).  All calls on one device share that array:
 * calls in flight at the same time on one device (other streams, other threads) race; calls on
 * one stream are ordered.  The device current at the call must be the context's (else
 * LBM_E_STATE). */
int lbm_diagnostics_noalloc(lbm_ctx* ctx, double* d_out);

/* Interval of lbm_step's non-finite check: n > 0 checks after every n-th step (counted since
 * lbm_init, or the restored checkpoint's count), 0 (the default) turns it off; negative n
 * returns LBM_E_ARG. */
int lbm_diag_every(lbm_ctx* ctx, int n);

/* Macroscopic fields (eq. macro) of the current state at every node, FP64 [ny][nx] device
 * arrays; d_T may be NULL. */
int lbm_macroscopic(lbm_ctx* ctx, double* d_rho, double* d_ux, double* d_uy, double* d_T);

/* Boundary solver state of a characteristic side: device FP64 [M][len][4], layer j = 1..M
 * (x_{b,j}, j = M outermost) then row, (rho, u_x, u_y, T). */
int lbm_boundary_state(lbm_ctx* ctx, int side, double* d_out);

/* Diagnostics of the current state (synchronises the stream).  h_out (host) receives
 * [0] total mass, [1] x momentum, [2] y momentum, [3] energy 1/2 sum f |c|^2,
 * [4] loss = sum over bulk nodes of (P - cs^2)^2, [5] max |u|, [6] number of non-finite
 * populations, [7] steps done.  Returns LBM_E_NONFINITE when [6] > 0.  The sums are
 * deterministic: one FP64 partial per 256-node row tile (wavefront reductions), folded in a
 * fixed order. */
int lbm_diagnostics(lbm_ctx* ctx, double* h_out);

/* Checkpoint of the complete state (populations, boundary solver state and the Dirichlet
 * profiles): device buffer of lbm_state_bytes(ctx) bytes.  Save then restore reproduces the run
 * bit for bit, also when a Dirichlet profile was changed in between.  lbm_restore discards a
 * run recorded with lbm_record. */
size_t lbm_state_bytes(const lbm_ctx* ctx);
int lbm_save(lbm_ctx* ctx, void* d_buf);
int lbm_restore(lbm_ctx* ctx, const void* d_buf);

/* Number of steps taken since lbm_init (or the restored checkpoint's count). */
long lbm_steps_done(const lbm_ctx* ctx);

/* Kernel timing for measurement.  With enable = n > 0, lbm_step records a pair of HIP events
 * around every n-th step kernel launch (fused bulk stream-collide and boundary solve; the first
 * launch after this call is timed) on the caller's stream, resetting earlier records; 0 turns
 * timing off, a negative value returns LBM_E_ARG.  Each timed launch adds about 7 us of event
 * work to the stream, so a stride above 1 keeps a timed run's step rate close to an untimed
 * one.  lbm_bulk_kernel_time synchronises on the events and returns the summed elapsed
 * milliseconds and the number of timed launches.  Disabled by default; at most 65536 launches
 * are recorded. */
int lbm_set_kernel_timing(lbm_ctx* ctx, int enable);
int lbm_bulk_kernel_time(lbm_ctx* ctx, double* total_ms, long* launches);

/* Discrete adjoint with checkpointing.  The paper has no adjoint: these calls differentiate
 * the discrete map that lbm_step computes (bulk stream + BGK collide, the RK4 characteristic
 * solve of every side and corner with wave directions frozen at the start of the step, and the
 * equilibrium reconstruction), in FP64 whatever the storage precision.  Supported boundaries:
 * periodic, LODI, LODI_RELAX, CBC and CBC_RELAX (mesoscopic or finite-difference viscous
 * terms), with the equilibrium or the NEEP reconstruction, zero-gradient sides with their
 * corners, and Dirichlet sides: with a profile given by lbm_dirichlet_profile the layers are
 * constants and the gradient with respect to the initial fields is 0 on them; with the default
 * profile every layer of a row holds, at every step, the equilibrium of the initial fields on the
 * first layer, which then carry the whole row's gradient (the other layers 0).  D2Q9
 * additionally needs one periodic axis (else LBM_E_UNSUPPORTED).  lbm_adjoint recomputes the
 * recorded steps, so the boundary settings must stay those of the recording: lbm_cbc_params,
 * lbm_reconstruction, lbm_viscous, lbm_dirichlet_profile and lbm_restore discard it.
 *
 * lbm_tape_bytes: device bytes of the tape for nsteps steps with a checkpoint every `every`
 * steps (0 for invalid arguments).  The tape holds ceil(nsteps / every) checkpoints of the
 * state plus the reverse sweep's scratch: two adjoint population buffers and two recomputation
 * sets, each of two population buffers and (every + 1) slots of per-node moments and boundary
 * state.
 *
 * lbm_record: from the initial state (no step taken since lbm_init; else LBM_E_STATE), advance
 * nsteps steps exactly as lbm_step does while storing the checkpoints in d_tape (caller-owned,
 * 256-byte aligned, at least lbm_tape_bytes bytes, borrowed until the next lbm_record, the
 * context's destruction, or lbm_restore, which discards the recording).
 *
 * lbm_adjoint: gradient of a scalar loss L of the final macroscopic fields with respect to the
 * initial fields and the relaxation parameters.  d_seed: device FP64 [4][ny][nx] =
 * dL/d(rho, u_x, u_y, T) at the final step and every node (the T plane is ignored for D2Q9),
 * or NULL for the pressure loss of lbm_diagnostics ([4]: sum over bulk nodes of
 * (P - cs^2)^2).  d_grad_fields (device FP64 [4][ny][nx]) receives
 * dL/d(rho0, u_x0, u_y0, T0) of the fields given to lbm_init; h_grad_relax (host [4][2])
 * receives dL/dsigma and dL/dalpha of each side (0 for sides without relaxation).  Runs the
 * reverse sweep segment by segment from the last checkpoint: each segment is recomputed from
 * its checkpoint, then reversed step by step.  The recomputation runs on a second stream that
 * the library makes on the context's first lbm_adjoint (non-blocking, default priority, on the
 * device current at that call, which must be the context's; released by lbm_destroy), one
 * segment ahead of the reverse sweep on the context's stream; events order the two.  The
 * context must not have stepped since lbm_record (LBM_E_STATE); its state is left unchanged,
 * and the call may be repeated with other seeds.  Synchronises the stream before returning. */
size_t lbm_tape_bytes(const lbm_ctx* ctx, int nsteps, int every);
int lbm_record(lbm_ctx* ctx, int nsteps, int every, void* d_tape, size_t tape_bytes);
int lbm_adjoint(lbm_ctx* ctx, const double* d_seed, double* d_grad_fields, double* h_grad_relax);

/* Lattice constants used by the library (host pointers, arrays of q entries, library order).
 * Returns q, or a negative code for an unknown stencil. */
int lbm_lattice_info(int stencil, int* M, double* cs2, double* w, int* cx, int* cy);

const char* lbm_last_error(const lbm_ctx* ctx);
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
