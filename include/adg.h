/*
 * adg.h -- C ABI of the MI355X (gfx950) ADER-DG library for 2D compressible
 * Navier-Stokes with gravity and the total-variation refinement indicator.
 *
 * Method: Krenz, Rannabauer, Bader, "A High-Order Discontinuous Galerkin
 * Solver with Dynamic Adaptive Mesh Refinement to Simulate Cloud Formation
 * Processes" (arXiv:1905.05524).  Equation set: Section 2 (eqs.
 * equation-set, eos, temperature, stress-tensor, heat-conduction-coeff,
 * hydrostatic-balance, momentum-equation-split).  Scheme: Section 3 (ADER-DG
 * predictor/corrector with a Rusanov-type viscous flux).  Indicator: Section 3
 * (eqs. tv, refinement-criterion, chebychev).
 *
 * Conventions shared by every call
 *   - FP64 throughout.  Node sets are Gauss-Legendre (GL) points on [0,1].
 *   - State Q is device memory, cell-major: Q[cell][var][jz][ix], var =
 *     (rho, rho*u, rho*w, rho*E), n = N+1 nodes per direction; node (jz, ix)
 *     of a cell with lower-left corner (x0, z0) and size h sits at
 *     (x0 + h*xi_ix, z0 + h*xi_jz).  Energy includes the geopotential rho*g*z.
 *   - Cell order: for a uniform grid, c = j*nx + i; otherwise the order of
 *     the leaf list given to adg_init_mesh.
 *   - clock: device double[4] = (t, dt, unused, step count).
 *     Time and time step live on the device so that a step needs no host
 *     scalar; the caller may write t and dt before a step.
 *   - Ownership: every device buffer passed in (Q, workspace, clock, tv,
 *     flags, stats, adjoint buffers) belongs to the caller and is never freed
 *     by the library.  A handle owns only its metadata and constant tables
 *     (allocated in adg_init_mesh, freed in adg_destroy).
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *     stream).  Enqueuing calls are asynchronous and capturable in a HIP
 *     graph, except adg_regrid_apply and adg_check_health, which synchronise.
 *   - Errors: every call returns an adg status; parameter and launch errors
 *     are reported immediately, with a message from adg_last_error().  Device
 *     state errors (non-finite values, rho <= 0, p <= 0) are reported by
 *     adg_check_health.  Handles are not thread-safe.
 */
#ifndef ADG_H
#define ADG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ADG_OK = 0,
  ADG_EINVAL = -1,       /* bad argument or inconsistent parameters          */
  ADG_ENOMEM = -2,       /* handle-owned allocation failed                    */
  ADG_EHIP = -3,         /* HIP runtime or launch error                       */
  ADG_ESTATE = -4,       /* no state bound, or unhealthy state on the device  */
  ADG_EUNSUPPORTED = -5  /* valid request that this build does not support    */
};

enum { ADG_BC_PERIODIC = 0, ADG_BC_WALL = 1 };
enum { ADG_VAR_THETA = 0, ADG_VAR_RHO = 1 };
enum { ADG_SHAPE_COSINE = 0, ADG_SHAPE_PLATEAU_GAUSS = 1 };

/* Physical and numerical parameters.
 *   order N in 1..7 (n = N+1 <= 8 GL nodes per direction);
 *   picard_iters: number of predictor sweeps, 0 -> N+1;
 *   gamma, Pr, R, cp, mu: ideal gas and viscosity, kappa = mu*cp/Pr
 *     (eq. heat-conduction-coeff);
 *   gravity != 0: geopotential rho*g*z in the EOS, momentum flux with the
 *     perturbation pressure p - p_bar(z), source -g (rho - rho_bar(z)) in the
 *     vertical momentum (eq. momentum-equation-split); the background is the
 *     hydrostatic atmosphere of constant potential temperature theta_bg
 *     (eq. hydrostatic-balance) with reference pressure p0;
 *   mms = 1: adds the energy source of the manufactured advected density
 *     wave rho = 1 + mms_amp sin(mms_kx (x - mms_u t)) sin(mms_kz (z - mms_w t)),
 *     velocity (mms_u, mms_w), pressure mms_p (for convergence checks);
 *   mms = 2: adds the source of the paper's manufactured solution (CFD
 *     scenarios, eq. manufactured-solution): with xi = (pi/5)(x + z) - 2 pi t,
 *     p = 1/gamma + cos(xi)/10, rho = 1 + sin(xi)/2, u = w = sin(xi)/4, on
 *     every conserved variable (EINVAL with gravity; the mms_* fields are
 *     not used);
 *   cfl: Courant number of the time-step rule;
 *   fixed_dt != 0: keep clock[1] unchanged (no CFL update after a step). */
typedef struct {
  int order;
  int picard_iters;
  double gamma, Pr, R, cp, mu, g, p0, theta_bg;
  int gravity;
  int mms;
  double mms_amp, mms_u, mms_w, mms_kx, mms_kz, mms_p;
  double cfl;
  int fixed_dt;
} adg_params;

/* Mesh: a coarse grid of nx x nz square cells on [x0,x0+Lx] x [z0,z0+Lz]
 * (Lx/nx == Lz/nz) refined by 3-way splits per level and dimension (paper,
 * Sections 3 and 4.3) up to max_level.  bc[4] = (west, east, south, north).
 * leaf_level/leaf_i/leaf_j (host arrays of n_leaves entries; all NULL for the
 * uniform coarse grid) list the leaves; leaf (l, i, j) has size
 * h = Lx/(nx 3^l) and corner (x0 + i h, z0 + j h).  Neighbouring leaves may
 * differ by at most one level. */
typedef struct {
  double x0, z0, Lx, Lz;
  int nx, nz;
  int max_level;
  int bc[4];
  int n_leaves;
  const int32_t* leaf_level;
  const int32_t* leaf_i;
  const int32_t* leaf_j;
} adg_mesh_desc;

typedef struct adg_mesh adg_mesh;

/* Create a handle: validates parameters, builds the GL basis and the face
 * tables, uploads constant tables.  EINVAL on bad parameters or an invalid
 * leaf list.  *out is set only on success. */
int adg_init_mesh(const adg_params* prm, const adg_mesh_desc* mesh, adg_mesh** out);
int adg_destroy(adg_mesh* m);

/* Number of cells, nodes per direction, and the size in bytes of the
 * workspace the caller must provide to adg_set_state. */
int adg_mesh_info(const adg_mesh* m, int* n_cells, int* n_nodes);
int adg_workspace_bytes(const adg_mesh* m, size_t* bytes);

/* Bind caller-owned device buffers: Q [C][4][n][n] (updated in place by each
 * step), workspace (adg_workspace_bytes, 256-byte aligned), clock double[4]. */
int adg_set_state(adg_mesh* m, double* Q, void* workspace, double* clock);

/* Initial state by nodal interpolation (paper, Section 4.2: hydrostatic
 * background of constant potential temperature, perturbed in theta at fixed
 * pressure; cosine bubble eq. cos-pertubation read with cos(pi r / a);
 * bubbles of eq. bubbles-pertubation).  bubbles: host array [n_bubbles][6] =
 * (shape, A, a, s, xc, zc); perturbations add.  kind 0 = bubbles, 1 = the
 * manufactured density wave at time t0, 2 = the paper's manufactured
 * solution at time t0.  Writes the bound Q. */
int adg_init_state(adg_mesh* m, int kind, int n_bubbles, const double* bubbles, double t0,
                   void* stream);

/* Time step by the CFL rule from the bound Q:
 *   dt = cfl * min_cells h / (2 (2N+1) (lambda + 2 lambda_v (2N+1)/h)),
 * lambda = max(|u|,|w|) + c, lambda_v = max(4 mu/(3 rho), gamma mu/(Pr rho));
 * writes clock[1]. */
int adg_compute_dt(adg_mesh* m, void* stream);

/* Space-time predictor (ADER-DG, Section 3): Picard sweeps on the GL
 * space-time nodes of every cell, then the time-averaged state and flux, the
 * volume-plus-source update Q* and the face data, into the workspace. */
int adg_predictor(adg_mesh* m, void* stream);

/* Corrector: viscous Rusanov flux on every face from the face data (walls:
 * background-state ghosts with the background heat flux, Section 4.2), the
 * surface update Q = Q* - lifting, the next CFL time step (unless fixed_dt),
 * then t += dt and step count += 1 in clock. */
int adg_corrector(adg_mesh* m, void* stream);

/* One full step: adg_predictor + adg_corrector. */
int adg_step(adg_mesh* m, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one step
 * exactly like adg_step, of Q (device [C][4][n][n], updated in place) with
 * clock (device double[4], as for adg_set_state), whose workspace (the
 * predictor's partial update, the face data and the per-cell time-step
 * bounds) lives in a static device buffer of the library of
 * ADG_STATIC_SCRATCH_BYTES (32 MiB, enough for about 9,900 cells at order
 * 6), one per GPU, held until the process ends.  Allocates nothing and does
 * not use the buffers bound by adg_set_state.  Must be called with the
 * handle's device current.  EINVAL if Q or clock is null or misaligned, if
 * the mesh's workspace (adg_workspace_bytes) exceeds the buffer, or if the
 * current device is not the handle's; EHIP if the buffer's device address
 * could not be looked up when the handle was created.  Every call on one
 * GPU shares the buffer, which keeps the last call's contents (nothing in
 * it must start at zero: each step writes every entry it reads): calls that
 * overlap on one GPU (other streams or threads) race and must be
 * serialised by the caller. */
#define ADG_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
int adg_step_static(adg_mesh* m, double* Q, double* clock, void* stream);

/* TV indicator (eq. tv) of theta (ADG_VAR_THETA) or rho per cell, read as
 * the l1 norm of the physical gradient integrated by GL quadrature with the
 * reference element's weights (which sum to one), i.e. the mean of
 * |df/dx| + |df/dz| over the cell:
 *   TV = (1/h) sum_ji w_i w_j (|sum_m D_im f_jm| + |sum_m D_jm f_mi|),
 * so a cell's TV does not scale with its size; the
 * population mean/std of TV over all cells merged with the pairwise updates of
 * Chan, Golub and LeVeque, and the flags of eq. refinement-criterion:
 * +1 refine if TV >= mu + T_refine sigma, -1 coarsen if TV < mu + T_coarsen
 * sigma, else 0 (sigma == 0 keeps all).  tv: device double[C], flags: device
 * int8[C], stats: device double[3] = (count, mean, sigma).  Above 65,536
 * cells the statistics go through per-workgroup partials in a small
 * handle-owned buffer: calls on one handle that overlap in time race. */
int adg_tv_indicator(adg_mesh* m, int var, double T_refine, double T_coarsen, double* tv,
                     int8_t* flags, double* stats, void* stream);

/* Synchronises the stream, then checks the bound state: ESTATE if any value
 * is non-finite or any node has rho <= 0 or p <= 0. */
int adg_check_health(adg_mesh* m, void* stream);

/* Message of the last failing call on this thread. */
const char* adg_last_error(void);

/* Read back the handle's GL nodes/weights and matrices (n, n, n*n, n*n):
 * D[i*n+j] = phi_j'(xi_i), P = K1^{-1} W of the time predictor. */
int adg_basis(const adg_mesh* m, double* xi, double* w, double* D, double* P);

/* Leaf list of the current mesh (host arrays of n_cells entries, may be
 * NULL), in cell order. */
int adg_get_leaves(const adg_mesh* m, int32_t* level, int32_t* i, int32_t* j);

/* Regrid, step 1 (host only): from per-cell flags (host int8[C]: +1 refine,
 * -1 coarsen, 0 keep; e.g. the output of adg_tv_indicator copied to the
 * host) build the new leaf list: refine is dropped at max_level and coarsen
 * at level 0; a family of nine siblings becomes its parent only if all nine
 * are leaves flagged coarsen (paper, Section 3); refined leaves are replaced
 * by their 3x3 children.  New order: old leaves in order, children row by
 * row in place of their parent, a coarsened family at its first sibling.
 * Returns the new cell count and workspace size.  EUNSUPPORTED if the result
 * has neighbours more than one level apart. */
int adg_regrid_plan(adg_mesh* m, const int8_t* flags_host, int* n_cells_new, size_t* ws_bytes_new);

/* Regrid, step 2: transfer the bound state into Q_new (caller-owned,
 * n_cells_new*4*n*n doubles, must not alias Q): copy for kept leaves, exact
 * interpolation of the parent polynomial for new children, L2 projection of
 * the nine children for a new parent; then install the face tables the plan
 * built (in the handle's device buffers, which grow when the mesh does) and
 * bind (Q_new, workspace_new, clock).  Synchronises the device (every kernel
 * that reads the old tables, on any stream, has finished).  The old Q and
 * workspace are the caller's to free.  ENOMEM or EHIP after the transfer
 * leaves the handle without a usable mesh (its cell count reads 0): destroy
 * it and create a new one. */
int adg_regrid_apply(adg_mesh* m, double* Q_new, void* workspace_new, double* clock, void* stream);

/* Launch shape of the predictor and corrector: cells per wavefront (1, 2 or
 * 4, with cells_per_wave * n^2 <= 64) and wavefronts per workgroup (1, 2 or
 * 4); cells_per_wave 0 selects the time-level predictor, for meshes too
 * small to fill the GPU with one wavefront per cell: one workgroup per cell
 * whose wavefronts share the time levels of the Picard sweeps, one
 * wavefront per level (waves_per_block 1) or the levels spread over 2 or 4
 * wavefronts (waves_per_block 2 or 4; with n or fewer levels the same as 1).
 * Results do not depend on the shape (up to the order of sums).
 * Default: one wavefront per time level while n_cells * (order + 1) <= 3072
 * (about three wavefronts per SIMD), else (order >= 4) the levels over four
 * wavefronts while n_cells * 4 <= 3072, else 1, 1.
 * adg_autotune reports the time-level predictor as cells_per_wave 0 with its
 * waves_per_block as above. */
int adg_set_launch(adg_mesh* m, int cells_per_wave, int waves_per_block);

/* Time every launch shape on the bound state (reps predictor + corrector
 * pairs each; the corrector writes into the workspace so Q and clock are left
 * unchanged), keep the fastest and return it.  Synchronises the stream. */
int adg_autotune(adg_mesh* m, int reps, void* stream, int* cells_per_wave, int* waves_per_block);

/* --------------------------------------------------------------- adjoint
 * Hand-written reverse mode of one step with a frozen time step (clock[1];
 * clock[0] is the step's start time), of the initial state built from a
 * potential-temperature perturbation, and of the potential-temperature loss.
 * Conforming meshes only (EUNSUPPORTED otherwise).  Non-smooth points: the
 * Rusanov speed takes the subgradient of the first maximum over the face
 * nodes in the order (lower side nodes 0..n-1, upper side nodes 0..n-1);
 * d|x|/dx = 0 at x = 0. */

/* Size of the adjoint workspace (Picard iterate store of one step, face
 * adjoints, loss partials). */
int adg_adjoint_workspace_bytes(const adg_mesh* m, size_t* bytes);

/* lam_n = (dQ^{n+1}/dQ^n)^T lam_np1 for the step that starts from the
 * checkpoint Q_n (device [C][4][n][n]).  Recomputes that step's predictor
 * (overwrites the bound workspace); lam_n must not alias lam_np1. */
int adg_step_adjoint(adg_mesh* m, const double* Q_n, const double* lam_np1, double* lam_n, void* adj_ws,
                     void* stream);

/* The same step adjoint without the predictor recompute, for callers that
 * kept the forward step's Picard iterates and face data in device memory
 * (288 GB of HBM hold them for thousands of steps of a mid-size mesh):
 *   adg_keep_bytes: sizes of one step's iterate store [C][I][n][4][n][n]
 *     and face data [C][4][2][4][n];
 *   adg_step_keep: one step like adg_step (predictor, corrector, clock),
 *     writing that step's iterates to store and its face data to fd
 *     (caller-owned device buffers of those sizes); the bound workspace's
 *     face data are not used;
 *   adg_step_adjoint_kept: as adg_step_adjoint for the step that started
 *     from Q_n, reading store and fd as adg_step_keep wrote them; the
 *     result equals adg_step_adjoint's (the same iterates, not recomputed).
 * Conforming meshes only (EUNSUPPORTED otherwise). */
int adg_keep_bytes(const adg_mesh* m, size_t* store_bytes, size_t* fd_bytes);
int adg_step_keep(adg_mesh* m, double* store, double* fd, void* stream);

/* adg_step (store = fd = NULL) or adg_step_keep (both given) with the new
 * state Q^{n+1} written to Q_out (device [C][4][n][n], caller-owned; may be
 * the bound state, which gives the in-place step) instead of the bound state,
 * which keeps Q^n: a rollout writes each step into the next checkpoint slot
 * and binds it (adg_set_state) for the next step, with no copy.  The clock
 * advances as in adg_step.  Keeping iterates: conforming meshes only
 * (EUNSUPPORTED otherwise); EINVAL when only one of store and fd is given. */
int adg_step_to(adg_mesh* m, double* Q_out, double* store, double* fd, void* stream);
int adg_step_adjoint_kept(adg_mesh* m, const double* Q_n, const double* store, const double* fd,
                          const double* lam_np1, double* lam_n, void* adj_ws, void* stream);

/* Bound Q <- initial state of the nodal perturbation theta_prime (device
 * [C][n][n]): hydrostatic background of constant potential temperature,
 * theta = theta_bg + theta' at fixed pressure, at rest (paper, Section 4.2).
 * grad = (dQ/dtheta')^T lam (device [C][n][n]). */
int adg_ic_theta(adg_mesh* m, const double* theta_prime, void* stream);
int adg_ic_theta_adjoint(adg_mesh* m, const double* theta_prime, const double* lam, double* grad, void* stream);

/* loss (device double[1]) = sqrt(sum_cells h^2 sum_ji w_i w_j (theta - theta_bg)^2)
 * of the bound Q; the adjoint writes lam = grad_loss[0] * dloss/dQ (device
 * [C][4][n][n]) given the loss value. */
int adg_loss_theta(adg_mesh* m, double* loss, void* adj_ws, void* stream);
int adg_loss_theta_adjoint(adg_mesh* m, const double* loss, const double* grad_loss, double* lam, void* stream);

/* ---------------------------------------------------------------- batches
 * Many independent scenarios (own mesh, own order, own clock) stepped
 * together.  All scenarios share the physical parameters; orders may differ.
 * Scenarios are grouped by order; each group is one concatenated cell array.
 * One step forks one stream per order group (predictor, corrector), joins,
 * and updates every scenario's clock (t, dt, steps) with its own CFL step.
 * The state is one device array: scenario s occupies
 * [q_offset, q_offset + n_cells*4*n*n) with the single-mesh layout; clocks
 * is device double[n_scen][4]. */
typedef struct adg_batch adg_batch;

/* prm and mesh: host arrays of n_scen entries.  EINVAL if parameters other
 * than the order differ between scenarios or a mesh is invalid. */
int adg_batch_create(const adg_params* prm, const adg_mesh_desc* mesh, int n_scen, adg_batch** out);
int adg_batch_destroy(adg_batch* b);
int adg_batch_info(const adg_batch* b, int* n_groups, int* total_cells, size_t* q_doubles, size_t* ws_bytes);
int adg_batch_scenario(const adg_batch* b, int s, size_t* q_offset, int* n_cells, int* n_nodes);
/* Bind caller-owned device buffers (Q of q_doubles, workspace of ws_bytes,
 * clocks [n_scen][4]); drops a captured graph. */
int adg_batch_set_state(adg_batch* b, double* Q, void* workspace, double* clocks);
/* As adg_init_state, for scenario s (synchronises). */
int adg_batch_init_state(adg_batch* b, int s, int kind, int n_bubbles, const double* bubbles, double t0,
                         void* stream);
/* CFL time step of every scenario (writes clocks[s][1]). */
int adg_batch_compute_dt(adg_batch* b, void* stream);
/* One step of every scenario, launched eagerly. */
int adg_batch_step(adg_batch* b, void* stream);
/* One step of every scenario as one HIP graph launch: the first call on a
 * stream captures the step (fork/join over the group streams) and
 * instantiates it; later calls replay it.  stream must not be NULL. */
int adg_batch_step_graph(adg_batch* b, void* stream);
/* Autotune the launch shape of every order group (outputs: host arrays of
 * n_groups entries, may be NULL).  Drops a captured graph.  Synchronises. */
int adg_batch_autotune(adg_batch* b, int reps, void* stream, int* cells_per_wave, int* waves_per_block);
int adg_batch_set_launch(adg_batch* b, int group, int cells_per_wave, int waves_per_block);
/* Predictor of a batch step: ADG_BATCH_PER_ORDER (default) launches one
 * predictor grid per order group over its cells, on the group's forked
 * stream; ADG_BATCH_PERSISTENT launches, per order group, a persistent grid
 * of resident wavefronts that take work items (one wavefront's cells) from
 * a device counter (reset by the grid's last wavefront), each order's grid
 * sized by its share of the modelled predictor work (cells x (N+1)^4).
 * Its bits are those of the per-order mode with one wavefront per cell
 * (adg_batch_set_launch with cells_per_wave >= 1); a group that the
 * per-order mode runs with one wavefront per time level (small groups, by
 * default) sums the levels in another order and agrees to rounding.  The
 * persistent mode measured slower (its loop
 * around the order-6 body spills registers) and exists for comparison.
 * Drops a captured graph; EUNSUPPORTED for the paper's manufactured
 * solution in persistent mode. */
enum { ADG_BATCH_PER_ORDER = 0, ADG_BATCH_PERSISTENT = 1 };
int adg_batch_set_mode(adg_batch* b, int mode);

#ifdef __cplusplus
}
#endif
#endif /* ADG_H */
