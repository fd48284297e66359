/*
 * lbm.h - C ABI of the MI355X (gfx950) library for the double-distribution
 * cascaded (central-moment, multiple-relaxation-time) lattice Boltzmann
 * method for 3D thermal convection of Hajabdollahi & Premnath,
 * arXiv:1710.04751.
 *
 * Problem (Sec. 3 of the paper): a box of nx * ny * nz fluid cells with
 * walls half a link outside the first and last cells (L = nx).  The wall
 * x = -1/2 is held at T_hot, the wall x = nx - 1/2 at T_cold, the other four
 * faces are adiabatic, the fluid sticks to every wall, and buoyancy
 * F = g beta (T - T0) acts along +z with T0 = (T_hot + T_cold)/2.
 *
 * Method per time step and cell (the fused update this library launches):
 *   pull streaming, eq. (2b) and (13b), with half-way bounce-back for the
 *   flow, anti-bounce-back on the two Dirichlet walls and bounce-back on the
 *   adiabatic faces for the scalar;
 *   macroscopic fields: T = sum gbar + R/2 (eq. 25; R the optional uniform
 *   heat source), F = g beta (T - T0) z-hat, rho = sum f,
 *   rho u = sum f e + F/2 (eq. 3);
 *   flow collision: the D3Q15 cascaded central-moment kernel of Appendix A
 *   with the body-force source, eq. (2a);
 *   scalar collision: the D3Q15 kernel of Sec. 2.2 or the D3Q7 kernel of
 *   Appendix C, eq. (13a), with the flow velocity of the same step and the
 *   source populations S^phi of eq. (19) / Appendix B, C.
 *
 * Conventions for every function:
 *   - Return an lbm_status; nothing throws across this ABI.
 *   - lbm_last_error() returns a thread-local message for the last failure.
 *   - "device pointer" means memory on the HIP device the handle was created
 *     on; the caller allocates and owns it.  "host pointer" means ordinary
 *     host memory.
 *   - Work is enqueued on the stream given at creation (hipStream_t passed
 *     as void*; NULL is the default stream).  Only functions documented as
 *     synchronising wait for the device.
 *   - Field layout: one value per cell, x fastest: index (z*ny + y)*nx + x.
 *   - Population arrays exchanged with the caller: population a of cell c
 *     at [a*ncell + c].  The stored state itself groups rows (see
 *     lbm_state_info).
 */
#ifndef LBM_H_
#define LBM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_ERR_ARG = -1,      /* invalid argument or parameter set */
    LBM_ERR_HIP = -2,      /* a HIP runtime call failed */
    LBM_ERR_UNSTABLE = -3, /* NaN or Inf found in the solution */
    LBM_ERR_STATE = -4     /* call not valid in the handle's current state */
} lbm_status;

/* Storage and arithmetic of the distributions.
 * LBM_FP64: FP64 arithmetic, FP64 storage.
 * LBM_FP32: FP32 arithmetic, FP32 storage.
 * LBM_FP32_S16: FP32 arithmetic, FP16 storage (round to nearest even).
 * In every mode the flow populations are stored as deviations f - w_a from
 * the rest state (rho = 1, u = 0) and the scalar populations as g (T_ref =
 * 0), so storage rounding acts on small numbers. */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP32_S16 = 2 } lbm_precision;

/* Problem and method parameters.  Fill with lbm_params_init, then adjust. */
typedef struct lbm_params {
    int32_t nx, ny, nz;     /* fluid cells per axis (each >= 4) */
    int32_t thermal_q;      /* scalar lattice: 7 (Appendix C) or 15 (Sec. 2.2) */
    int32_t precision;      /* lbm_precision */
    int32_t fourth_maxwell; /* flow 4th-order equilibrium: 0 = kxx~ kyy~ / rho
                               (post-collision second-order central moments,
                               Appendix A), 1 = c_s^4 rho */
    double Ra, Pr;          /* Rayleigh and Prandtl numbers (Sec. 3) */
    double u0;              /* velocity scale sqrt(g beta dT L) in lattice units */
    double T_hot, T_cold;   /* wall temperatures at x = -1/2 and x = nx - 1/2 */
    double cs2_T;           /* c_sphi^2 of the scalar equilibrium (eq. 6); 1/3 */
    double omega_bulk;      /* flow trace rate omega_9; <= 0 means the shear rate */
    double omega_hi;        /* flow rates omega_10..omega_14 (third/fourth order); 1 */
    double omega_hi_T;      /* scalar rates of orders >= 2; 1 */
    double R;               /* uniform scalar source of the convection-diffusion
                               equation (eq. 4), per cell and time step in
                               lattice units; finite.  R != 0 runs the general
                               collision kernels (source populations of eq. 19,
                               Appendix B/C; T = sum gbar + R/2, eq. 25) */
    int32_t lattice_units;  /* 0: derive nu, alpha, gbeta from Ra, Pr, u0 and
                               L = nx; 1: take nu, alpha, gbeta below as given */
    int32_t block_x;        /* threads per block along x (0 = default) */
    int32_t block_y;        /* threads per block along y (0 = default) */
    int32_t round_stochastic; /* FP16 storage only: 0 = round to nearest even
                                 (default), 1 = stochastic rounding (unbiased,
                                 keyed by step, population and cell; a batch
                                 member draws the bits a single run of it
                                 draws) */
    int32_t scalar_specular;  /* zero-gradient condition of the scalar on the
                                 four adiabatic faces (Sec. 3): 0 = bounce-back
                                 of g (default), 1 = specular reflection (the
                                 crossed velocity components reversed, so each
                                 link keeps its tangential flux; differs from
                                 bounce-back only on D3Q15) */
    double nu, alpha, gbeta; /* used only when lattice_units == 1 */
} lbm_params;

/* Lattice-unit values a handle runs with. */
typedef struct lbm_lattice {
    double nu, alpha, gbeta; /* viscosity, diffusivity, g beta */
    double omega_nu;         /* shear rate: nu = (1/omega - 1/2)/3 (Appendix A) */
    double omega_bulk;       /* trace rate actually used */
    double omega_T;          /* alpha = c_sphi^2 (1/omega_T - 1/2) (eq. 23) */
    double T_ref;            /* T0 of the buoyancy force */
} lbm_lattice;

/* Wall heat transfer (FP64).  Local Nu is the heat crossing a wall per unit
 * area and step times L / (alpha dT), taken from the links that cross the
 * wall (anti-bounce-back returns 2 (w_a T_wall - g_out) per link), so pure
 * conduction gives exactly 1. */
typedef struct lbm_nu {
    double nu_hot_wall, nu_cold_wall; /* means over the two Dirichlet faces */
    double nu_hot_mid, nu_cold_mid;   /* means along z on the mid-plane y = L/2 */
    double nu_max, z_max;             /* max of hot-wall local Nu on that line, at z/L */
    double nu_min, z_min;             /* min, at z/L */
} lbm_nu;

/* Peak velocities on the symmetry plane y = L/2, the quantities Table 1 of
 * the paper reports, in units of u0.  Positions follow the paper's axes
 * (heated axis from the cold wall, height from the bottom), in units of L. */
typedef struct lbm_peaks {
    double u_max; /* max over height of the velocity along the heated axis
                     pointing from the cold to the hot wall (-u_x), on the
                     vertical centreline x = L/2 */
    double u_pos; /* its height z/L */
    double w_max; /* max of the vertical velocity u_z on the horizontal
                     centreline z = L/2 */
    double w_pos; /* its distance from the cold wall, over L */
} lbm_peaks;

/* How a run to steady state ended. */
typedef enum {
    LBM_STEADY_TOL = 0,       /* residual below the tolerance */
    LBM_STEADY_PLATEAU = 1,   /* residual stopped falling above the tolerance
                                 (the precision's floor) */
    LBM_STEADY_MAX_STEPS = 2, /* step limit reached first */
    LBM_STEADY_UNSTABLE = 3,  /* NaN or Inf appeared */
    LBM_STEADY_STALLED = 4    /* residual stopped reaching new minima above the
                                 plateau floor: the run approached a steady
                                 state and then left it (a steady state that
                                 the discrete dynamics does not hold) */
} lbm_steady;

typedef struct lbm_handle lbm_handle;
typedef struct lbm_batch lbm_batch;

/* Thread-local text of the last error (never NULL). */
const char* lbm_last_error(void);

/* Defaults: n^3 cavity at Rayleigh number Ra, Pr = 0.71, u0 = 0.05,
 * T_hot = +0.5, T_cold = -0.5, D3Q7 scalar, FP32, c_sphi^2 = 1/3, bulk rate
 * equal to the shear rate, higher-order rates 1, factorised 4th-order
 * equilibrium. */
lbm_status lbm_params_init(lbm_params* p, int32_t n, double Ra);

/* Derived lattice values of a parameter set (host pointers). */
lbm_status lbm_params_lattice(const lbm_params* p, lbm_lattice* out);

/* Bytes of device workspace lbm_create needs for p; 0 if p is invalid. */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Create a solver.  Validates p (LBM_ERR_ARG: a size < 4, thermal_q not 7 or
 * 15, R not finite, Ra, Pr or u0 <= 0, u0 / c_s > 0.3, a relaxation rate outside
 * (0, 2), block sizes not a multiple of 64 threads or above 1024).
 * workspace: device pointer of at least lbm_workspace_bytes(p) bytes, 256-byte
 * aligned, borrowed until lbm_destroy.  stream: hipStream_t or NULL.
 * The state is the fluid at rest with T = 0 (lbm_init_rest is enqueued). */
lbm_status lbm_create(const lbm_params* p, void* workspace, size_t workspace_bytes, void* stream,
                      lbm_handle** out);

/* Release the host-side state; the workspace is not freed (caller owns it). */
lbm_status lbm_destroy(lbm_handle* h);

/* Lattice values the handle runs with (host pointer). */
lbm_status lbm_get_lattice(const lbm_handle* h, lbm_lattice* out);

/* Number of steps taken since the last initialisation. */
int64_t lbm_steps_done(const lbm_handle* h);

/* Rest state: rho = 1, u = 0, T = 0 (f = w_a; g = 0, or with a source the
 * scalar equilibrium at -R/2, so the first step sees T = 0).  Asynchronous. */
lbm_status lbm_init_rest(lbm_handle* h);

/* Equilibrium state from fields (device pointers, float, ncell each; NULL
 * means 0): rho = 1, velocity (ux, uy, uz), temperature T (with a source the
 * scalar equilibrium is taken at T - R/2, so the first step sees T).  Used
 * to start from a prediction.  The staggered part of the velocity is first set as a
 * start from rest has it.  With pull streaming and bounce-back walls every
 * population that carries x-momentum changes the parity of x at each step
 * and the collision conserves momentum, so Qx = sum (-1)^x rho u_x only
 * changes sign from step to step (likewise Qy); along z the collision adds
 * S = g beta sum (-1)^z (T - T0), so Qz alternates about S/2.  Any other
 * staggered momentum never decays: it stays as a period-2 oscillation.
 * Hence ux -= (-1)^x Sx / ncell with Sx = sum (-1)^x ux, the same for uy,
 * and uz -= (-1)^z (Sz - S/2) / ncell with Sz = sum (-1)^z uz.
 * Asynchronous. */
lbm_status lbm_init_macros(lbm_handle* h, const float* ux, const float* uy, const float* uz,
                           const float* T);

/* Advance nsteps >= 0 time steps.  Asynchronous. */
lbm_status lbm_step(lbm_handle* h, int64_t nsteps);

/* Macroscopic fields of the current step: rho, ux, uy, uz, T (device
 * pointers, ncell values each, double if fp64 != 0 else float; NULL skips a
 * field).  They equal the pre-collision moments of the last step (eq. 3, 25),
 * recovered from the stored post-collision populations (collision conserves
 * rho, adds F to the momentum and R to the scalar sum: T = sum g~ - R/2).
 * Asynchronous. */
lbm_status lbm_macros(lbm_handle* h, void* rho, void* ux, void* uy, void* uz, void* T, int fp64);

/* Wall Nusselt numbers of the current state (FP64 reduction on the device),
 * after the definition of Sec. 3 of the paper: the local Nusselt number is
 * the wall-normal temperature gradient at a Dirichlet wall scaled by L/dT
 * (the paper prints it with its axes mixed up), its average over the wall
 * the mean Nusselt number, and Table 1 reports its mean, maximum and minimum
 * on the symmetry plane.  The gradient is taken as the lattice's heat flux
 * through the wall (see lbm_nu), which equals alpha times the gradient for
 * pure conduction exactly.  out: host pointer.  Synchronises the stream.
 * Optional profiles (device pointers, double, may be NULL): local Nu of the
 * hot and cold walls, [nz][ny] each.  Returns LBM_ERR_UNSTABLE if a result
 * is not finite. */
lbm_status lbm_nusselt(lbm_handle* h, lbm_nu* out, double* local_hot, double* local_cold);

/* lbm_nusselt for callers that cannot allocate or hand over scratch memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results (bit for bit), with the local
 * profiles and the reduced values in a device array that the library holds
 * on each device it runs on until the process ends (2 * 2^20 + 8 doubles,
 * 16 MiB), instead of in the handle's workspace.  Limit: ny * nz <= 2^20
 * (LBM_ERR_ARG beyond it, before any launch).  The handle's device must be
 * current (LBM_ERR_STATE otherwise).  Allocates nothing.  Every call on a
 * device shares that device's array: calls that overlap on one device (from
 * several threads or streams) race and must be serialised by the caller.
 * out: host pointer; local_hot, local_cold: optional device pointers as in
 * lbm_nusselt.  Synchronises the stream. */
lbm_status lbm_nusselt_noalloc(lbm_handle* h, lbm_nu* out, double* local_hot,
                               double* local_cold);

/* Steady-state residual: max over cells of |T_now - T_snapshot| (host
 * pointer), then T_now becomes the snapshot.  The first call after an
 * initialisation only takes the snapshot and reports +inf.  Returns
 * LBM_ERR_UNSTABLE if any T is NaN or Inf.  Synchronises the stream. */
lbm_status lbm_residual(lbm_handle* h, double* max_dT);

/* Velocity profiles on the symmetry plane y = L/2 (FP64, device kernel):
 * u_line[nz] = -u_x / u0 along the vertical centreline x = L/2, w_line[nx]
 * = u_z / u0 along the horizontal centreline z = L/2, pre-collision moments
 * of the current step as in lbm_macros.  An even number of cells across a
 * centreline averages the two middle cells.  u_line, w_line: device
 * pointers, may be NULL.  peaks (host pointer, may be NULL): maxima of the
 * two profiles, each refined by the parabola through the largest sample and
 * its two neighbours (cell centres sit at (i + 1/2)/N).  Synchronises the
 * stream when peaks is given. */
lbm_status lbm_centerlines(lbm_handle* h, double* u_line, double* w_line, lbm_peaks* peaks);

/* Project fields onto the symmetries of the cavity problem (Sec. 3): the
 * mirror y -> ny-1-y, under which uy changes sign, and the half turn about
 * the y axis through the centre, (x, z) -> (nx-1-x, nz-1-z), under which ux,
 * uz and T - T0 change sign (the walls swap temperatures, buoyancy
 * reverses).  Each value becomes the signed mean over its four images.
 * In place on device pointers (float, ncell each, the handle's grid; NULL
 * skips a field).  A start from rest keeps these symmetries exactly; an
 * initial field that breaks them seeds modes that the symmetric steady
 * state does not damp at high Rayleigh numbers on coarse grids, so a
 * predicted start is projected first.  Asynchronous. */
lbm_status lbm_symmetrize(lbm_handle* h, float* ux, float* uy, float* uz, float* T);

/* Step until steady: every check_every steps (even, > 0) take lbm_residual;
 * stop when it is below tol (LBM_STEADY_TOL), or when plateau_checks > 0,
 * its smallest value so far is below plateau_floor and it has not reached a
 * new minimum for plateau_checks checks in a row (LBM_STEADY_PLATEAU: the
 * state wanders at the storage precision's floor, e.g. FP32 stalls at a few
 * units in the last place of T; *steps is then the step at which the
 * minimum was first seen), or when stall_checks > 0 and it has not reached
 * a new minimum for stall_checks checks in a row while its smallest value
 * stays at or above plateau_floor (LBM_STEADY_STALLED: the state came near
 * a steady state and left it again), or after max_steps
 * (LBM_STEADY_MAX_STEPS).  A residual that falls slowly with oscillations
 * keeps the run going as long as new minima come within stall_checks
 * checks.  The first check only takes the snapshot.  Outputs (host
 * pointers, may be NULL): steps taken to the stopping criterion (-1 unless
 * it ended with TOL or PLATEAU), how it ended (lbm_steady), the last
 * residual.  Returns LBM_ERR_UNSTABLE (with *how = LBM_STEADY_UNSTABLE) on
 * NaN/Inf.  Synchronises. */
lbm_status lbm_run_to_steady(lbm_handle* h, double tol, int64_t check_every, int64_t max_steps,
                             int32_t plateau_checks, double plateau_floor, int32_t stall_checks,
                             int64_t* steps, int32_t* how, double* last_residual);

/* Full populations as FP64 (device pointers): F [15][ncell], G [q][ncell]
 * (f itself, not the stored deviation).  Either may be NULL.  Asynchronous. */
lbm_status lbm_get_populations(lbm_handle* h, double* F, double* G);

/* Overwrite the state with full FP64 populations (device pointers, same
 * layout; rounded to the storage precision).  Resets the step counter.
 * Asynchronous. */
lbm_status lbm_set_populations(lbm_handle* h, const double* F, const double* G);

/* Full FP64 populations of n listed cells (device pointers): cells [n]
 * (linear cell indices, each in [0, ncell)), F [n][15], G [n][q].  Indices
 * out of range are reported as LBM_ERR_ARG before any launch only when
 * check != 0 (the check copies cells to the host and synchronises).
 * Asynchronous otherwise. */
lbm_status lbm_gather_cells(lbm_handle* h, const int64_t* cells, int64_t n, double* F, double* G,
                            int check);

/* Device buffers of the current state, for inspection: F and G base
 * pointers, elements between two populations of one cell (pop_stride), bytes
 * per stored value.  The state interleaves groups of Rg = pop_stride / nx
 * consecutive x-rows (Rg a power of two, chosen so that one population's
 * run of a group spans about 32 KB): with r = z*ny + y, population a of
 * cell (x, y, z) is
 *   F[((r / Rg)*(15 + q) + a)*pop_stride + (r % Rg)*nx + x]  (flow, a < 15),
 *   G[((r / Rg)*(15 + q) + a)*pop_stride + (r % Rg)*nx + x]  (scalar, a < q),
 * with G = F + 15 pop_stride. */
lbm_status lbm_state_info(const lbm_handle* h, const void** F, const void** G,
                          int64_t* pop_stride, int32_t* value_bytes);

/* Name of the step kernel the handle launches (for profiler summaries). */
const char* lbm_step_kernel_name(const lbm_handle* h);

/* Threads per block of the step kernel: set (each a multiple of 64 total,
 * at most 1024) or time candidates with HIP events on the handle's stream
 * and keep the fastest.  lbm_autotune advances the state by the steps it
 * times (it is meant for warm-up); results: the chosen block_x, block_y. */
lbm_status lbm_set_block(lbm_handle* h, int32_t block_x, int32_t block_y);
lbm_status lbm_autotune(lbm_handle* h, int32_t steps_per_trial, int32_t* block_x,
                        int32_t* block_y);

/* Plain device copy of bytes (device pointers, 16-byte aligned, bytes a
 * multiple of 16) on stream: the reference kernel for bandwidth and
 * memory-counter calibration.  Asynchronous. */
lbm_status lbm_copy_probe(void* dst, const void* src, size_t bytes, void* stream);


/* ------------------------------------------------------------------------
 * Batched form: many independent cavities (any sizes and parameters, one
 * precision, scalar lattice and rate set) advanced together.  One step is
 * one persistent launch over a device list of tiles (a tile is a few whole
 * x-rows of one z-plane of one cavity); each member is updated exactly as
 * by lbm_step.  Steps are replayed from a captured hipGraph.  Converged
 * members leave the tile list (compacted on the device), so the graph is
 * never re-captured for that.
 * ---------------------------------------------------------------------- */

/* Bytes of device workspace for n cavities p[0..n-1] (host array); 0 if any
 * is invalid, if they differ in precision, thermal_q, round_stochastic or in
 * whether the general collision kernels run, or if n is not in [1, 255]. */
size_t lbm_batch_workspace_bytes(const lbm_params* p, int32_t n);

/* Create a batch over caller device memory (256-byte aligned, borrowed
 * until lbm_batch_destroy) on stream; every member starts at rest and is
 * active.  Launch shape: 256 threads per block, 8 blocks per compute unit,
 * graphs of 100 steps (change with lbm_batch_set_launch or
 * lbm_batch_autotune). */
lbm_status lbm_batch_create(const lbm_params* p, int32_t n, void* workspace, size_t bytes,
                            void* stream, lbm_batch** out);
lbm_status lbm_batch_destroy(lbm_batch* b);

/* Member i as a solver handle, for the observables (lbm_macros,
 * lbm_nusselt, lbm_get_populations, lbm_init_macros, ...).  lbm_step and
 * lbm_destroy refuse members.  Members may be re-initialised only while the
 * batch has taken an even number of steps. NULL if i is out of range. */
lbm_handle* lbm_batch_member(lbm_batch* b, int32_t i);

/* Advance every active member nsteps steps.  Asynchronous. */
lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps);

/* Residual of every member (host arrays of n): max |T - T_snapshot| over its
 * cells, then the snapshot is renewed (+inf on a member's first call;
 * inactive members report their last value).  status[i] = LBM_OK or
 * LBM_ERR_UNSTABLE (NaN/Inf).  Synchronises the stream. */
lbm_status lbm_batch_residuals(lbm_batch* b, double* max_dT, int32_t* status);

/* Set which members take part in later steps (host array of n, 0/1).
 * Rebuilds the device tile list; asynchronous. */
lbm_status lbm_batch_set_active(lbm_batch* b, const int32_t* active);

/* Run every active member to steady state with the rule of
 * lbm_run_to_steady (tolerance, plateau, stall, step limit), checking all
 * members every check_every steps (even) and retiring each as it stops.
 * Outputs (host arrays of n, may be NULL): steps each member took to its
 * stopping criterion (-1 unless it ended with TOL or PLATEAU), how it ended
 * (lbm_steady), last residual.  Synchronises. */
lbm_status lbm_batch_run_to_steady(lbm_batch* b, double tol, int64_t check_every,
                                   int64_t max_steps, int32_t plateau_checks,
                                   double plateau_floor, int32_t stall_checks, int64_t* steps,
                                   int32_t* how, double* last_residual);

/* Launch shape: threads per block (a multiple of 64, >= the largest nx, at
 * most 1024), blocks per compute unit (1..32: a persistent grid whose blocks
 * walk the tile list; 0: one block per tile of the whole batch, blocks past
 * the active tiles returning at once), steps per captured graph (even, 0
 * disables graphs). */
lbm_status lbm_batch_set_launch(lbm_batch* b, int32_t threads, int32_t blocks_per_cu,
                                int32_t graph_steps);

/* Time candidate (threads, blocks per CU) shapes with HIP events over
 * steps_per_trial steps each and keep the fastest; the trial steps advance
 * the members.  Returns the chosen shape. */
lbm_status lbm_batch_autotune(lbm_batch* b, int32_t steps_per_trial, int32_t* threads,
                              int32_t* blocks_per_cu);

/* Current launch: threads per block, grid blocks, active tiles (synchronises
 * to read the device count), steps per graph, batch steps taken. */
lbm_status lbm_batch_launch_info(lbm_batch* b, int32_t* threads, int32_t* grid_blocks,
                                 int32_t* active_tiles, int32_t* graph_steps, int64_t* steps);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H_ */
