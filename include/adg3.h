/*
 * adg3.h -- C ABI of the three-dimensional ADER-DG step of the MI355X
 * (gfx950) library: compressible Navier-Stokes with gravity on a uniform grid
 * of cubes with periodic or no-slip wall boundaries.
 *
 * Method: Krenz, Rannabauer, Bader, arXiv:1905.05524.  The equation set of
 * Section 2 is written for two or three space dimensions (eqs. equation-set,
 * eos, temperature, stress-tensor, heat-conduction-coeff, hydrostatic-balance,
 * momentum-equation-split); the scheme of Section 3 (ADER-DG predictor and
 * corrector with a Rusanov-type viscous flux) is the same in both.  The
 * three-dimensional set-ups of Section 4 are the ABC flow (eq. abc-flow,
 * order 3 on 27^3 cells) and the cosine bubble (eq. cos-pertubation with
 * y_c = x_c, order 3 on 40 m cells, mu = 0.005).
 *
 * Conventions (shared with adg.h where not stated otherwise)
 *   - FP64; Gauss-Legendre nodes on [0,1]; n = N+1 nodes per direction.
 *   - State Q is device memory, cell-major: Q[cell][var][kz][jy][ix] with
 *     var = (rho, rho*u, rho*v, rho*w, rho*E); gravity acts along -z and
 *     the energy includes the geopotential rho*g*z.  Cell (i, j, k) of the
 *     grid is c = (k*ny + j)*nx + i; its corner is
 *     (x0 + i*h, y0 + j*h, z0 + k*h); node (kz, jy, ix) sits at
 *     corner + h*(xi_ix, xi_jy, xi_kz).
 *   - Faces of a cell: 0 = -x, 1 = +x, 2 = -y, 3 = +y, 4 = -z, 5 = +z.
 *   - clock: device double[4] = (t, dt, unused, step count), as in adg.h.
 *   - Ownership, streams and errors as in adg.h: caller-owned device
 *     buffers are never freed by the library; enqueuing calls are
 *     asynchronous on the given hipStream_t (void*, NULL = default stream)
 *     and capturable, except adg3_check_health, which synchronises;
 *     every call returns an adg status (ADG_OK, ADG_EINVAL, ...) with the
 *     message in adg_last_error().  Handles are not thread-safe.
 */
#ifndef ADG3_H
#define ADG3_H

#include <stddef.h>
#include <stdint.h>

#include "adg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Uniform grid of nx x ny x nz cubes of edge h with lower corner
 * (x0, y0, z0).  bc[6] per face of the domain (order as the cell faces):
 * ADG_BC_PERIODIC or ADG_BC_WALL; periodic faces come in pairs. */
typedef struct {
  double x0, y0, z0, h;
  int nx, ny, nz;
  int bc[6];
} adg3_mesh_desc;

typedef struct adg3_mesh adg3_mesh;

/* Create a handle.  prm as in adg.h with order N in 1..5 (n^3 <= 216 nodes
 * per cell); mms must be 0 (EUNSUPPORTED otherwise).  EINVAL on invalid
 * parameters or mesh. */
int adg3_init_mesh(const adg_params* prm, const adg3_mesh_desc* mesh, adg3_mesh** out);
int adg3_destroy(adg3_mesh* m);

/* Number of cells, nodes per direction, and the workspace size in bytes. */
int adg3_mesh_info(const adg3_mesh* m, int* n_cells, int* n_nodes);
int adg3_workspace_bytes(const adg3_mesh* m, size_t* bytes);

/* Bind caller-owned device buffers: Q [C][5][n][n][n] (updated in place by
 * each step), workspace (adg3_workspace_bytes, 256-byte aligned), clock
 * double[4].  Workspace layout (byte offsets rounded up to 256):
 * Q* [C][5][n][n][n], then the face data [C][6][2][5][n][n] (per face: the
 * time-averaged state and normal flux extrapolated to the face, nodes
 * ordered by the two tangential directions in (z, y, x) order), then the
 * per-cell time-step candidates [C], then a health flag. */
int adg3_set_state(adg3_mesh* m, double* Q, void* workspace, double* clock);

/* Initial state by nodal interpolation.  kind 0: the hydrostatic background
 * of constant potential temperature theta_bg (Section 4.2; needs gravity),
 * perturbed in theta at fixed pressure by bubbles (host array
 * [n_bubbles][7] = (shape, A, a, s, xc, yc, zc); shape ADG_SHAPE_COSINE:
 * (A/2)(1 + cos(pi r/a)) for r <= a, ADG_SHAPE_PLATEAU_GAUSS: A for r <= a,
 * A exp(-(r-a)^2/s^2) beyond; perturbations add), at rest.  kind 1: the ABC
 * flow of eq. abc-flow at time t0 (rho = 1, constant C = 100/gamma), meant
 * for the periodic cube [-pi, pi]^3.  At most 16 bubbles. */
int adg3_init_state(adg3_mesh* m, int kind, int n_bubbles, const double* bubbles, double t0, void* stream);

/* CFL time step from the bound Q:
 *   dt = cfl * h / (3 (2N+1) (lambda + 2 lambda_v (2N+1)/h)),
 * lambda = max over nodes of max(|u|,|v|,|w|) + c, lambda_v =
 * max(4 mu/(3 rho), gamma mu/(Pr rho)); writes clock[1]. */
int adg3_compute_dt(adg3_mesh* m, void* stream);

/* Space-time predictor of every cell (Section 3): Picard sweeps on the GL
 * space-time nodes, time averages of state, flux and source, the volume and
 * source update Q* and the face data, into the workspace.  Uses dt =
 * clock[1]. */
int adg3_predictor(adg3_mesh* m, void* stream);

/* Corrector: viscous Rusanov flux on the six faces of every cell from the
 * face data (walls: background-state ghost with mirrored velocity and the
 * background heat flux through horizontal walls, Section 4.2), the surface
 * update Q = Q* - lifting, the next CFL candidate per cell; then t += dt,
 * steps += 1 and, unless fixed_dt, dt <- the CFL step of the new state. */
int adg3_corrector(adg3_mesh* m, void* stream);

/* One full step: adg3_predictor + adg3_corrector. */
int adg3_step(adg3_mesh* m, void* stream);

/* Synchronises the stream, then ESTATE if any value of the bound Q is
 * non-finite or any node has rho <= 0 or p <= 0. */
int adg3_check_health(adg3_mesh* m, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ADG3_H */
