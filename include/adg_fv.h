/*
 * adg_fv.h -- C ABI of the finite-volume scheme of the MI355X (gfx950)
 * library: MUSCL-Hancock with the van Albada limiter for the 2D compressible
 * Euler equations with gravity on a uniform grid of square cells.
 *
 * Method: Krenz, Rannabauer, Bader, arXiv:1905.05524.  Section 3 (Numerics)
 * names the engine's second scheme, MUSCL-Hancock finite volumes stabilised
 * with the van Albada limiter, with the Rusanov-type flux of the ADER-DG
 * scheme; Section 4.2 runs it without viscosity on the colliding bubbles
 * (7^2 patches of 90^2 cells: a uniform 630 x 630 grid on the 1000 m box).
 * The equation set is that of Section 2 with mu = 0 (eqs. equation-set,
 * eos, hydrostatic-balance, momentum-equation-split).
 *
 * One step, per cell (one value per cell, standing for its centre):
 *   1. slopes of the conserved variables along x and z from the backward
 *      and forward differences a, b, limited with van Albada:
 *      a b (a + b) / (a^2 + b^2) if a b > 0, else 0; at a wall the missing
 *      neighbour is the wall ghost state (below) at the ghost cell centre;
 *   2. Hancock half step: the four face values Q -+ slope/2 all move by
 *      dt/(2h) times the flux differences across the cell (each face value's
 *      flux at the face height) plus dt/2 times the gravity source;
 *   3. Rusanov flux G = (F_L + F_R)/2 - s/2 (Q_R - Q_L) of the evolved face
 *      values of the two cells of a face, s = max of |v.n| + c over both;
 *      at a wall the other side is the ghost of the evolved value: the
 *      background density and pressure at the face height with the velocity
 *      mirrored (without gravity the interior density and pressure), with
 *      the mass and energy fluxes mirrored and the momentum fluxes kept;
 *   4. Q <- Q - dt/h (G_east - G_west + G_north - G_south)
 *           + dt * source(Q + half-step increment).
 * Time step: the Courant rule of the DG scheme at N = 0 without viscosity,
 * dt = cfl h / (2 lambda), lambda = max over cells of max(|u|,|w|) + c.
 *
 * Conventions
 *   - FP64.  State Q: device memory, Q[cell][4], var = (rho, rho*u,
 *     rho*w, rho*E), cell (i, j) at c = j*nx + i with centre
 *     (x0 + (i + 1/2) h, z0 + (j + 1/2) h); the energy includes the
 *     geopotential rho*g*z; gravity acts along -z.
 *   - clock: device double[4] = (t, dt, unused, step count), as in adg.h.
 *   - Ownership, streams and errors as in adg.h: caller-owned device
 *     buffers are never freed by the library; enqueuing calls are
 *     asynchronous on the given hipStream_t (void*, NULL = default stream)
 *     and capturable, except adg_fv_check_health, which synchronises; every
 *     call returns an adg status with the message in adg_last_error().
 *     Handles are not thread-safe.
 */
#ifndef ADG_FV_H
#define ADG_FV_H

#include <stddef.h>
#include <stdint.h>

#include "adg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Uniform grid of nx x nz square cells of edge h, lower-left corner
 * (x0, z0); bc[4] = (west, east, south, north), ADG_BC_PERIODIC or
 * ADG_BC_WALL, periodic faces in pairs. */
typedef struct {
  double x0, z0, h;
  int nx, nz;
  int bc[4];
} adg_fv_desc;

typedef struct adg_fv adg_fv;

/* Create a handle.  prm as in adg.h with order 0 (the scheme has no
 * polynomial order), mu 0 and mms 0 (EUNSUPPORTED otherwise); Pr and
 * picard_iters are not used.  Builds the background table (density and
 * pressure at the cell centres, horizontal faces and wall ghost centres of
 * every row).  EINVAL on invalid parameters or mesh. */
int adg_fv_init(const adg_params* prm, const adg_fv_desc* mesh, adg_fv** out);
int adg_fv_destroy(adg_fv* m);

/* Number of cells and the workspace size in bytes. */
int adg_fv_info(const adg_fv* m, int* n_cells);
int adg_fv_workspace_bytes(const adg_fv* m, size_t* bytes);

/* Bind caller-owned device buffers: Q [C][4] (updated in place by each
 * step), workspace (adg_fv_workspace_bytes, 256-byte aligned), clock
 * double[4].  Workspace layout (offsets rounded up to 256 bytes): evolved
 * face values [4 faces (west, east, south, north)][4 vars][C], half-step
 * density increments [C], one time-step bound per workgroup of the
 * corrector or tile of adg_fv_step, a health flag. */
int adg_fv_set_state(adg_fv* m, double* Q, void* workspace, double* clock);

/* Initial cell values at the centres.  kind 0: the hydrostatic background
 * of constant potential temperature perturbed in theta at fixed pressure by
 * bubbles (host array [n_bubbles][6] = (shape, A, a, s, xc, zc) as in
 * adg_init_state; at most 16), at rest; needs gravity.  kind 1: the
 * advected density wave rho = 1 + mms_amp sin(mms_kx (x - mms_u t0))
 * sin(mms_kz (z - mms_w t0)) with velocity (mms_u, mms_w) and pressure
 * mms_p (its manufactured source is not applied: it solves the Euler
 * equations). */
int adg_fv_init_state(adg_fv* m, int kind, int n_bubbles, const double* bubbles, double t0, void* stream);

/* Time step by the Courant rule above from the bound Q; writes clock[1]. */
int adg_fv_compute_dt(adg_fv* m, void* stream);

/* Steps 1-2: slopes and Hancock half step of every cell, into the
 * workspace.  Uses dt = clock[1]. */
int adg_fv_predictor(adg_fv* m, void* stream);

/* Steps 3-4 and the clock: face fluxes, update of Q, then t += dt,
 * steps += 1 and, unless fixed_dt, dt <- the Courant step of the new Q. */
int adg_fv_corrector(adg_fv* m, void* stream);

/* One full step with the arithmetic of adg_fv_predictor + adg_fv_corrector
 * (and the same clock update), fused into one kernel on tiles of 16 x 16
 * cells whose face values stay in on-chip memory and whose face fluxes are
 * evaluated once per face, plus a copy-back kernel that also advances the
 * clock.  Interior cells of a tile are updated in place; the two outer
 * layers of every tile pass through the workspace's face-value area (its
 * contents afterwards are not the evolved face values).  The horizontal
 * faces inside a tile take their height from the row above the face, so a
 * result may differ from the split path in the last bits. */
int adg_fv_step(adg_fv* m, void* stream);

/* Synchronises the stream, then ESTATE if any value of the bound Q is
 * non-finite or any cell has rho <= 0 or p <= 0. */
int adg_fv_check_health(adg_fv* m, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ADG_FV_H */
