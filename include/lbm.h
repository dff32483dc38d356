/*
 * lbm.h -- C ABI of libcplbm, the MI355X (gfx950) solver for the
 * chemical-potential multiphase lattice Boltzmann method of Wen, Zhao, Qiu,
 * Ye and Shan, "Chemical-Potential Multiphase Lattice Boltzmann Method with
 * Superlarge Density Ratios" (arXiv:1906.09530).
 *
 * One time step (Sec. 2-4 of the paper) on an nx x ny D2Q9 mesh, FP64:
 *   1. moments rho = sum f_i, rho u = sum e_i f_i                     (Eq. 3)
 *   2. bulk chemical potential psi'(rho) of the chosen EOS   (Eqs. 15/17/19/21)
 *      bounded by an upper limit                                   (Sec. 5.6)
 *   3. mesh chemical potential mu = k^2 psi'(rho) - kappa lap(rho)    (Eq. 33)
 *      with derivatives from the periodic compact scheme     (Eqs. 37-39) and
 *      the Laplacian as the first-derivative scheme applied twice   (Sec. 4.3)
 *   4. nonideal force F = -rho grad mu + c_s^2 grad rho                (Eq. 12)
 *   5. BGK collision with the exact-difference force term          (Eqs. 1, 5)
 *      and streaming.
 *
 * Units: mesh lattice units (mesh step 1, time step 1, c_s^2 = 1/3).  The
 * EOS constants, T and psi' live in momentum space; k links the two
 * (Eq. 25) and enters only as the factor k^2 of Eq. 33.
 *
 * Layout: a scalar field is nx*ny doubles, row-major, node (x, y) at index
 * y*nx + x.  The distribution state at the ABI is 9 such planes, f[i][y][x],
 * with the D2Q9 velocities e_0..e_8 = (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),
 * (-1,1),(-1,-1),(1,-1) (Sec. 2).  The stored state is the pre-collision
 * f(t).  (A context keeps each row's nine populations side by side on the
 * device, f[y][i][x]; lbm_get_state and lbm_set_state convert.)
 *
 * Boundaries: x is periodic.  y is periodic (bc_y = 0) or closed by
 * half-way bounce-back walls at y = -1/2 and y = ny - 1/2 (bc_y = 1) that may
 * slide along x with speed wall_ux; along y between walls the derivatives
 * act on the even extension of each column about the walls, which gives the
 * neighbour-node chemical-potential condition of Sec. 5.5.
 *
 * Streams: every device operation of a context is enqueued on the HIP
 * stream given to lbm_init (NULL: the default stream).  Calls that return
 * data to the host synchronise that stream.
 *
 * Errors: every entry point returns an lbm_status; nothing is thrown across
 * the ABI.  LBM_E_NONFINITE is sticky: once a non-finite density has been
 * seen, every later call on the context returns it.  lbm_last_error() gives
 * a human-readable reason for the last failure of a context.
 *
 * Threading: a context may be used by one host thread at a time.
 */
#ifndef CPLBM_LBM_H
#define CPLBM_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_NOT_CONVERGED = 1,  /* run_until_converged reached max_steps */
    LBM_E_INVALID = -1,     /* a parameter or size is outside what is supported */
    LBM_E_DOMAIN = -2,      /* initial density outside the EOS domain */
    LBM_E_NOMEM = -3,       /* device allocation failed or workspace too small */
    LBM_E_DEVICE = -4,      /* a HIP call failed */
    LBM_E_NONFINITE = -5    /* the density field became NaN or infinite */
} lbm_status;

/* Equations of state of Sec. 3.2. */
typedef enum {
    LBM_EOS_VDW = 0,  /* van der Waals, Eqs. 14-15 */
    LBM_EOS_RK = 1,   /* Redlich-Kwong, alpha(T) = T^-1/2, Eqs. 16-17 */
    LBM_EOS_RKS = 2,  /* Soave-Redlich-Kwong, Eqs. 16-17 */
    LBM_EOS_PR = 3,   /* Peng-Robinson, Eqs. 18-19 */
    LBM_EOS_CS = 4    /* Carnahan-Starling, Eqs. 20-21 */
} lbm_eos;

typedef struct {
    int32_t nx, ny;     /* mesh nodes; 8 <= nx, ny <= 2^20; lines longer than
                           4096 nodes: nx a multiple of 4, ny a multiple of 8 */
    int32_t bc_y;       /* 0: periodic in y; 1: bounce-back walls in y */
    int32_t eos;        /* lbm_eos */
    double a, b, R;     /* EOS constants in momentum space (Sec. 3.2) */
    double omega;       /* acentric factor (RKS, PR) */
    double T_r;         /* reduced temperature T/T_c, 0 < T_r < 1 */
    double kappa;       /* surface-tension coefficient on the mesh, >= 0 (Eq. 33) */
    double tau;         /* BGK relaxation time, > 1/2 (Eq. 1) */
    double k;           /* proportional coefficient mesh/momentum step, > 0 (Eq. 25) */
    double mu_cap;      /* upper limit of psi'(rho), momentum units (Sec. 5.6);
                           +INFINITY switches it off */
    double cfd_alpha;   /* compact scheme: 1/3 (sixth order, Eq. 39) or 1/4 (Eq. 38) */
    double wall_ux;     /* x-velocity of both walls (bc_y = 1); 0 for resting walls */
    int32_t collision;  /* lbm_collision: BGK (Eq. 1) or MRT (Eq. 4) */
    int32_t force;      /* lbm_force: chemical potential (Eq. 12) or pseudopotential */
    double s_e, s_eps, s_q;  /* MRT rates of the energy, energy-square and energy-flux
                                moments, each in (0, 2) (Eq. 4; the paper uses 1.64,
                                1.54, 1.9); the stress moments relax at 1/tau.
                                Ignored by BGK. */
    int32_t wetting;    /* walls (bc_y = 1) only: 0 the neighbour-node chemical-potential
                           condition of Sec. 5.5 (mu on the far side of a wall mirrors the
                           fluid, zero normal derivative); 1 a wetting wall that holds mu at
                           k^2 mu_wall (the chemical-potential boundary of ref. [45]; mu is
                           extended oddly about the wall value).  Chemical-potential force
                           only. */
    double mu_wall;     /* wall chemical potential, momentum units (as psi') */
} lbm_params;

/* Collision operator (Sec. 2). */
typedef enum {
    LBM_COLLISION_BGK = 0,  /* single relaxation time tau, Eq. 1 */
    LBM_COLLISION_MRT = 1   /* multiple relaxation times, Eq. 4: moments (rho, e, eps,
                               j_x, q_x, j_y, q_y, p_xx, p_xy) relaxed by
                               S = diag(0, s_e, s_eps, 0, s_q, 0, s_q, 1/tau, 1/tau) */
} lbm_collision;

/* Nonideal force. */
typedef enum {
    LBM_FORCE_CP = 0,  /* chemical potential, F = -rho grad mu + c_s^2 grad rho (Eq. 12) */
    LBM_FORCE_SC = 1   /* pseudopotential comparison model of Sec. 5.1 with k and the
                          compact scheme: F = -G c_s^2 psi grad psi, G = -1, effective
                          mass psi = sqrt(2 (rho c_s^2 - k^2 p0(rho)) / c_s^2) from the EOS
                          (Eq. 29; 0 where the root's argument is negative).  kappa and
                          mu_cap do not apply; lbm_force_fields returns psi as mu. */
} lbm_force;

/* ---- host-only thermodynamics (no device needed) ----------------------- */

/* Critical point of the EOS in p (T_r is ignored): dp0/drho = d2p0/drho2 = 0
 * with alpha(T_c) = 1 for RKS and PR and alpha = T^-1/2 for RK (Sec. 3.2).
 * Outputs in momentum units; any output pointer may be NULL. */
lbm_status lbm_critical_point(const lbm_params *p, double *T_c, double *rho_c, double *p_c);

/* Maxwell equal-area coexistence densities at p->T_r: equal psi'(rho) and
 * equal p0(rho) on both branches (Sec. 5.1).  Used to build the initial
 * tanh fields of Eq. 41.  LBM_E_INVALID if T_r is not in (0, 1). */
lbm_status lbm_maxwell(const lbm_params *p, double *rho_g, double *rho_l);

/* Bulk pressure p0(rho) (Eqs. 14, 16, 18, 20) and chemical potential psi'(rho)
 * (Eqs. 15, 17, 19, 21) at p->T_r, momentum units (either output may be
 * NULL).  LBM_E_DOMAIN unless 0 < rho < 1/b (4/b for CS). */
lbm_status lbm_eos_values(const lbm_params *p, double rho, double *p0, double *mu0);

/* ---- solver ----------------------------------------------------------- */

/* Device bytes a context for these parameters needs (for device_ws). */
size_t lbm_workspace_bytes(const lbm_params *p);

/* Create a context and set f = f^eq(rho0, u0) (Eq. 2).
 *   rho0, ux0, uy0: nx*ny doubles each, host memory, or device memory when
 *                   src_on_device != 0 (ux0/uy0 may be NULL for rest);
 *                   read during the call only; caller keeps ownership.
 *   hip_stream:     hipStream_t to enqueue on, or NULL for the default stream.
 *   device_ws:      NULL (the library allocates) or a caller-owned device
 *                   buffer of lbm_workspace_bytes(p) bytes, 256-byte aligned,
 *                   that must outlive the context.
 * With LBM_FORCE_SC the initial density must lie inside the EOS domain.
 * Fails with LBM_E_INVALID for unsupported parameters, LBM_E_DOMAIN when a
 * density is not positive and finite, or (with the limit switched off)
 * outside the EOS domain (rho >= 1/b, or b rho / 4 >= 1 for CS).  *out is
 * NULL on failure. */
lbm_status lbm_init(const lbm_params *p, const double *rho0, const double *ux0, const double *uy0,
                    int src_on_device, void *hip_stream, void *device_ws, lbm_ctx **out);

/* Enqueue nsteps time steps (nsteps >= 0).  Returns once the work is
 * enqueued; a non-finite state is only detected by the calls below. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* Observables of the current state: rho, and the velocity
 * v = u + F/(2 rho) (Sec. 2, after Eq. 5).  Each output holds nx*ny
 * doubles in host memory, or device memory if dst_on_device != 0; any
 * output may be NULL.  Synchronises the stream. */
lbm_status lbm_moments(lbm_ctx *ctx, double *rho, double *vx, double *vy, int dst_on_device);

/* The mesh chemical potential mu of Eq. 33 and the force F of Eq. 12 at
 * the current state (same conventions as lbm_moments). */
lbm_status lbm_force_fields(lbm_ctx *ctx, double *mu, double *Fx, double *Fy, int dst_on_device);

/* Step until max_x |rho(t) - rho(t - check_every)| < tol, testing every
 * check_every steps, at most max_steps steps.  Returns LBM_OK when
 * converged, LBM_NOT_CONVERGED at max_steps, LBM_E_NONFINITE on a NaN or
 * infinite density.  *steps_done and *last_delta may be NULL. */
lbm_status lbm_run_until_converged(lbm_ctx *ctx, double tol, int64_t check_every,
                                   int64_t max_steps, int64_t *steps_done, double *last_delta);

/* Copy the state f[9][ny][nx] out of / into the context (checkpoint and
 * resume; resuming reproduces a run bit for bit), converting from / to the
 * context's row-interleaved layout with one strided copy per population. */
lbm_status lbm_get_state(lbm_ctx *ctx, double *f, int dst_on_device);
lbm_status lbm_set_state(lbm_ctx *ctx, const double *f, int src_on_device);

/* Diagnostic: average device time in milliseconds of each kernel of a step
 * on the current state, each launched nsteps times back to back between two
 * HIP events on the context's stream: ms_per_pass[0] = row pass (rho,
 * d2/dx2 rho), [1] = column pass (mu, F_y), [2] = row pass (F_x,
 * collision, streaming into the spare buffer).  The state and the step
 * count are not changed.  Synchronises the stream. */
lbm_status lbm_time_passes(lbm_ctx *ctx, int64_t nsteps, double *ms_per_pass);

/* Diagnostic: run nsteps time steps (the state advances as with lbm_step)
 * with a HIP event recorded on the context's stream before and after every
 * kernel, so each kernel is timed inside the real step sequence.  ms[k]
 * receives the average milliseconds of kernel k and *count the number of
 * kernels per step: 3 (row pass A, column pass B, collision pass C in the
 * selected variant).  ms needs room for 3.
 * Synchronises the stream. */
lbm_status lbm_time_step_kernels(lbm_ctx *ctx, int64_t nsteps, double *ms, int *count);

/* Give the fluid the velocity (vx, vy) (arrays of nx*ny, host or device per
 * src_on_device; NULL for zero): the state becomes f = feq(rho, u) with rho
 * the current density and u = v - F/(2 rho), F the force of Eq. 12 of that
 * density, so that the velocity v of Sec. 2 (the observed velocity
 * u + F/(2 rho), Eq. 5) equals the given one.  With NULL, the fluid starts
 * at rest in that sense rather than with zero bare velocity.  Synchronises. */
lbm_status lbm_set_velocity(lbm_ctx *c, const double *vx, const double *vy, int src_on_device);

/* Autotuner: for each strip width of the column pass (columns per
 * workgroup) in {1, 2, 4, 8, 16} that one workgroup's LDS holds and, for the
 * factorised solve, each chunk length (column nodes per thread) in
 * {4, 8, 16}; for column tiles with windows (see lbm_set_column_shape) of
 * width 4, 8 or 16 and chunk 8 or 16 where the columns are long enough; for
 * streamed strips of width 8, 16 and 32 where the mesh allows them; then
 * for each collision pass variant of
 * lbm_set_collision_variant that the mesh allows, time `repeats` whole steps
 * (the three passes from the current state into the spare buffers, HIP
 * events), so that every candidate meets the caches as a real step leaves
 * them; keep the fastest of each for the context.  ms[] reports the time
 * per step.  The state f is
 * not changed.  widths[], chunks[] and ms[] (room for 27 entries each, may be
 * NULL) receive the candidates and their average time in milliseconds --
 * column candidates as (width, chunk; chunk 0 = general reduction kernel,
 * chunk < 0 = tiles of chunk -chunk, chunk LBM_COLUMN_STREAM = streamed
 * strips), collision candidates as (0, variant)
 * -- and *count (may be NULL) their number.  Synchronises. */
lbm_status lbm_autotune(lbm_ctx *ctx, int repeats, int *widths, int *chunks, double *ms,
                        int *count);

/* Collision pass variant (pass C of Eqs. 1, 2, 5, 12), for meshes whose rows
 * take the factorised-inverse kernels; the autotuner picks among them.
 *   0  one kernel over whole rows, reading the populations twice;
 *   1  one kernel over whole rows holding the populations in registers
 *      (rows of at most 1024 nodes; the default there);
 *   2  over row segments of 896 nodes (rows longer than 896 nodes, a
 *      multiple of 4; the last segment may be shorter): one workgroup per
 *      segment holds its populations in registers and takes F_x from the
 *      density and mu planes over a window of 52 nodes past each end of the
 *      segment, with the same values as whole-row derivatives of those
 *      planes.  F_x then takes rho from pass A (the sum of the density
 *      groups) instead of the collision's own sum of f, so results differ
 *      from variants 0 and 1 in the last bits.  Rows longer than 4096 nodes
 *      take this variant only, and their pass A and observations run over
 *      segments as well.
 * LBM_E_INVALID if the variant is not available for this mesh. */
lbm_status lbm_set_collision_variant(lbm_ctx *ctx, int variant);

/* Set the column-pass shape directly (width in columns per workgroup, chunk
 * in column nodes per thread of the factorised solve, 0 for the general
 * reduction kernel).  A negative chunk (-4, -8 or -16; width 4, 8 or 16)
 * cuts the columns into tiles of rows, one workgroup per tile, each tile
 * taking its three chained derivatives over a window of 3 (M + 1) chunks
 * above and below it (M the carries of the factorised solve: 11, 6, 3) --
 * mirrored about a wall -- so that strips stay wide on long columns (the
 * default for columns of more than 4096 nodes: width 4, chunk 8; tiles of
 * 1712 rows, where the streamed strips below do not apply); it needs
 * columns of more than one tile.  chunk =
 * LBM_COLUMN_STREAM (width 8, 16 or 32) streams each strip down the columns:
 * one workgroup per strip (512 threads) walks down it in tiles of chunks (8
 * nodes where ny is a multiple of 8, else 4), its three chained derivatives
 * pipelined one tile apart, so that each row of a plane is read and written
 * in whole strip-wide pieces (16 columns: one 128-byte line) and once --
 * between walls each solve closes with the mirror image's edge values and
 * carries; periodic columns add windows above and below (168 rows with
 * 8-node chunks, 144 with 4); it needs nx a multiple of the width, ny a
 * multiple of 4 of at least 64 nodes (periodic: at least the window), and the
 * chemical-potential force (not the pseudopotential model); the default,
 * 16 wide, for meshes of at least
 * 4096 x 2048 nodes.  LBM_E_INVALID if the shape does not fit.  Results of
 * every shape agree to round-off. */
#define LBM_COLUMN_STREAM 1
lbm_status lbm_set_column_shape(lbm_ctx *ctx, int width, int chunk);

/* Allocation-free stepping, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Advances the state f[9][ny][nx] (device memory, caller-owned,
 * the layout of lbm_get_state) by nsteps time steps in place, with the same
 * kernels, pass shapes and results as lbm_init + lbm_step on a new context
 * (no autotuning).  Every intermediate (the spare distribution buffer, the
 * density groups, the scalar planes) lives in a static device array of
 * 38 MiB that the library holds on each GPU it runs on until the process
 * ends: the call allocates nothing.  Meshes of at most
 * LBM_NOALLOC_MAX_NODES nodes; larger ones return LBM_E_INVALID before any
 * work is enqueued.  The work is enqueued on hip_stream (NULL: the default
 * stream) and the call returns without synchronising; the initial density
 * is not checked (a non-finite result shows in f).  Every call on one GPU
 * shares that GPU's array, so calls that overlap in time on one GPU (other
 * streams, other host threads) race; calls on one stream are ordered.
 * Errors: LBM_E_INVALID (parameters, size, NULL f, nsteps < 0),
 * LBM_E_DEVICE (a HIP call failed), with the reason in lbm_last_error(NULL). */
#define LBM_NOALLOC_MAX_NODES 262144
lbm_status lbm_step_noalloc(const lbm_params *p, double *f, int64_t nsteps, void *hip_stream);

/* Replay runs of steps from captured HIP graphs: lbm_step and
 * lbm_run_until_converged then enqueue every whole run of `steps` time steps
 * (rounded up to an even count, so that a run ends in the buffer it started
 * from) as one graph launch, and the rest kernel by kernel.  The kernels,
 * their order and the results are those of the launches one by one; on
 * small meshes, whose kernels take a few microseconds, the launches
 * themselves set the step time, and one graph launch replaces 3 x steps of
 * them.  Two graphs (one per starting buffer) are captured on first use, on
 * a stream the context creates, and captured again after the autotuner or
 * the collision or column settings change the pass shapes.  0 launches
 * every kernel separately.  Default: 100 for meshes of at most 512 x 512
 * nodes, 0 for larger ones (whose kernels hide the launches).
 * LBM_E_INVALID for steps outside [0, 100000]. */
lbm_status lbm_set_graph_steps(lbm_ctx *ctx, int64_t steps);

/* Steps taken since lbm_init. */
int64_t lbm_steps_taken(const lbm_ctx *ctx);

/* Wait for all work of the context. */
lbm_status lbm_synchronize(lbm_ctx *ctx);

/* Release the context and the memory the library allocated for it. */
void lbm_destroy(lbm_ctx *ctx);

/* Reason for the last failure of ctx (or of the last failed lbm_init when
 * ctx is NULL); empty when there was none.  Valid until the next call. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Name of a status code. */
const char *lbm_status_string(lbm_status s);

/* ---- batches of independent simulations --------------------------------
 * A sweep (temperatures for the coexistence curve of Sec. 5.1, radii for
 * Laplace's law of Sec. 5.3) runs as one batch: every pass of a time step is
 * a single launch over the workgroups of all active simulations, a chunk of
 * steps between convergence tests is replayed from one captured HIP graph,
 * and simulations that have converged drop out of the launches.  Each
 * simulation has its own parameters, sizes and state and evolves exactly as
 * it would in its own context with the same column-pass shape.  The batch
 * owns its device memory and a HIP stream of its own (default priority). */
typedef struct lbm_batch lbm_batch;

/* Create a batch of nsims simulations.  params[s], rho0[s], ux0[s], uy0[s]
 * as for lbm_init (host arrays; ux0/uy0 may be NULL, or hold NULL entries,
 * for rest).  Each simulation needs 64 <= nx, ny <= 1024 with nx and ny
 * multiples of 8, and all use the same collision operator.  Fails as lbm_init would, naming the simulation in
 * lbm_batch_last_error(NULL). */
lbm_status lbm_batch_create(int32_t nsims, const lbm_params *params, const double *const *rho0,
                            const double *const *ux0, const double *const *uy0, lbm_batch **out);

/* Set the column-pass shape of the batch: col_elems (2048 or 4096) nodes per
 * workgroup, i.e. col_elems / ny columns of each simulation, in chunks of
 * chunk (4 or 8) nodes per thread.  Results do not depend on col_elems. */
lbm_status lbm_batch_set_column_shape(lbm_batch *b, int col_elems, int chunk);

/* Autotuner: time the batched column pass for each shape above (repeats
 * launches each, HIP events), keep the fastest.  State unchanged.
 * col_elems[], chunks[], ms[] (room for 4, may be NULL) and *count report
 * the candidates. */
lbm_status lbm_batch_autotune(lbm_batch *b, int repeats, int *col_elems, int *chunks,
                              double *ms, int *count);

/* Enqueue nsteps steps of every active simulation (eager launches). */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Step all active simulations, test each every check_every steps for
 * max_x |rho(t) - rho(t - check_every)| < tol, and retire the ones that pass;
 * stop when none is active or after max_steps steps.  use_graph != 0 replays
 * each chunk from a captured HIP graph (re-captured when the set of active
 * simulations changes); 0 launches eagerly.  Per-simulation outputs
 * (arrays of nsims, each may be NULL): steps taken, last difference, and
 * status (LBM_OK converged, LBM_NOT_CONVERGED, LBM_E_NONFINITE, which also
 * retires the simulation).  Returns LBM_OK when all converged,
 * LBM_E_NONFINITE if any diverged, else LBM_NOT_CONVERGED. */
lbm_status lbm_batch_run_until_converged(lbm_batch *b, double tol, int64_t check_every,
                                         int64_t max_steps, int use_graph, int64_t *steps_done,
                                         double *last_delta, int32_t *status);

/* rho and v = u + F/(2 rho) of simulation sim, host arrays of nx*ny (any may
 * be NULL); the state f[9][ny][nx] of simulation sim (host).  Synchronise. */
lbm_status lbm_batch_moments(lbm_batch *b, int32_t sim, double *rho, double *vx, double *vy);
lbm_status lbm_batch_get_state(lbm_batch *b, int32_t sim, double *f);

/* lbm_set_velocity for simulation sim (host arrays, NULL for zero). */
lbm_status lbm_batch_set_velocity(lbm_batch *b, int32_t sim, const double *vx, const double *vy);

/* Steps taken by simulation sim (-1 for an invalid index). */
int64_t lbm_batch_steps(const lbm_batch *b, int32_t sim);

void lbm_batch_destroy(lbm_batch *b);

/* Reason for the last failure of b, or of the last failed lbm_batch_create
 * when b is NULL. */
const char *lbm_batch_last_error(const lbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* CPLBM_LBM_H */
