// MUSCL-Hancock finite volumes with the van Albada limiter (the engine's
// second scheme, Section 3; run without viscosity on the colliding bubbles,
// Section 4.2) for gfx950: kernels and the host side of include/adg_fv.h.
//
// One thread per cell, x fastest so that a wavefront reads consecutive cells
// (32 B each) and the x neighbours come from the same cache lines.
// The step (adg_fv_step) is one fused kernel on tiles of 16 x 16 cells:
//   k_fv_fused    each thread predicts its cell (slopes, Hancock half step),
//                 a fifth wavefront the ring of cells around the tile
//                 (only the face value the tile needs); the evolved face
//                 values meet in LDS; every face of the tile gets its
//                 Rusanov flux once (one job per face, 2.25 per cell); each
//                 thread then updates its cell and writes the new value: in
//                 place for the tile's interior cells, to a second buffer
//                 for its two outer layers (the only cells neighbouring tiles
//                 read: their ring cells and the ring cells' neighbours); and
//                 the tile's time-step bound of the new values;
//   k_fv_commit   copies the outer layers' new values into Q; its first
//                 workgroup reduces the tile bounds and advances the clock.
// HBM traffic is the state read (plus the halo) and written once, plus the
// outer layers (44 % of the cells) written and copied again.  The split
// entry points keep the two halves apart, with the evolved face values in
// the workspace (structure-of-arrays, one coalesced segment per face,
// variable and wavefront):
//   k_fv_predict  slopes and half step of every cell;
//   k_fv_correct  face fluxes and update in place (a thread reads no other
//                 cell's Q), and the workgroup's time-step bound.
// Both paths share the per-cell predictor; the face loop of the split path
// and the face jobs of the fused one take the same arithmetic.
// The background density and pressure of every row (centre, horizontal
// faces, wall ghost centres) come from a host-built table, so no kernel
// evaluates pow().
#include <algorithm>
#include <cmath>
#include <new>

#include "adg_fv.h"
#include "adg_internal.h"

namespace adg {

int launch_clock(double* clock, const double* dtc, const int* beg, const int* end, int nscen, int C, int advance,
                 int update, hipStream_t s);

constexpr int kFvThreads = 256;
constexpr int kFvBubbles = 16;

// Row table: for row j, 5 heights x (z, rho_bar, p_bar): the cell centre,
// the south and north faces, the south and north wall ghost centres.
enum { kBgC = 0, kBgS = 1, kBgN = 2, kBgGS = 3, kBgGN = 4 };

struct FvArgs {
  double* Q;            // [C][4]
  double* E;            // [4 faces][4 vars][C]
  double* inc;          // [C] half-step density increment
  double* dtb;          // [blocks] time-step bounds
  const double* clock;  // (t, dt, -, steps)
  const double* bg;     // [nz][5][3]
  int nx, nz, C, wall;  // wall: bit f set for a wall on face f (W, E, S, N)
  double h, ih;         // cell size and its reciprocal
};

struct FvBubbles {
  int nb;
  double b[kFvBubbles * 6];
};

__device__ inline double fv_pressure(const Phys& ph, const double q[4], double z) {
  return ph.gm1 * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) * recip(q[0]) - q[0] * (ph.geff * z));
}

// inviscid flux along d (0: x, 1: z) at height z with the perturbation
// pressure p - p_bar in the momentum flux (pb = 0 without gravity); returns
// the signal speed |v_d| + c of the state
__device__ inline double fv_flux(const Phys& ph, const double q[4], double z, double pb, int d, double F[4]) {
  const double ir = recip(q[0]);
  const double u = q[1] * ir, w = q[2] * ir;
  const double p = ph.gm1 * (q[3] - 0.5 * (q[1] * u + q[2] * w) - q[0] * (ph.geff * z));
  const double pm = p - pb;
  const double un = d ? w : u;
  F[0] = q[1 + d];
  F[1] = q[1] * un + (d == 0 ? pm : 0.0);
  F[2] = q[2] * un + (d == 1 ? pm : 0.0);
  F[3] = un * (q[3] + p);
  return fabs(un) + sqrt(ph.gamma * p * ir);
}

// wall ghost state of q at height z (background rb, pb there)
__device__ inline void fv_ghost(const Phys& ph, const double q[4], double z, double rb, double pb, double g[4]) {
  const double ir = recip(q[0]);
  const double u = q[1] * ir, w = q[2] * ir;
  double r = rb, p = pb;
  if (!ph.gravity) { r = q[0]; p = fv_pressure(ph, q, z); }
  const double geo = ph.gravity ? r * (ph.g * z) : 0.0;
  g[0] = r;
  g[1] = -(r * u);
  g[2] = -(r * w);
  g[3] = p / ph.gm1 + 0.5 * r * (u * u + w * w) + geo;
}

__device__ inline double van_albada(double a, double b) {
  if (!(a * b > 0.0)) return 0.0;
  return a * b * (a + b) * recip(a * a + b * b);
}

// G = (F_L + F_R)/2 - s/2 (Q_R - Q_L), s the larger of the two signal speeds
__device__ inline void rusanov_fv(double s, const double QL[4], const double FL[4], const double QR[4],
                                  const double FR[4], double G[4]) {
  for (int v = 0; v < 4; ++v) G[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * s * (QR[v] - QL[v]);
}

__device__ inline void load4(const double* p, double q[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  q[0] = a.x; q[1] = a.y; q[2] = b.x; q[3] = b.y;
}

// Steps 1-2 of the scheme for cell (i, j) inside the domain: the evolved
// face values fv[W, E, S, N][var] and the half-step density increment.  One
// direction at a time (its two neighbours, then its two face fluxes), so few
// values are live at once.
__device__ inline void fv_predict_cell(const Phys& ph, const FvArgs& a, int i, int j, double dt, double fv[4][4],
                                       double& inc0) {
  const int c = j * a.nx + i;
  const double* bg = a.bg + 15 * j;
  double q[4];
  load4(a.Q + 4 * (size_t)c, q);
  {  // x: west and east neighbours (wall ghost or periodic image at the domain edge)
    double nw[4], ne[4];
    if (i > 0) load4(a.Q + 4 * (size_t)(c - 1), nw);
    else if (a.wall & 1) fv_ghost(ph, q, bg[3 * kBgC], bg[3 * kBgC + 1], bg[3 * kBgC + 2], nw);
    else load4(a.Q + 4 * (size_t)(c + a.nx - 1), nw);
    if (i < a.nx - 1) load4(a.Q + 4 * (size_t)(c + 1), ne);
    else if (a.wall & 2) fv_ghost(ph, q, bg[3 * kBgC], bg[3 * kBgC + 1], bg[3 * kBgC + 2], ne);
    else load4(a.Q + 4 * (size_t)(c - a.nx + 1), ne);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double sx = van_albada(q[v] - nw[v], ne[v] - q[v]);
      fv[0][v] = q[v] - 0.5 * sx;
      fv[1][v] = q[v] + 0.5 * sx;
    }
  }
  {  // z: south and north neighbours
    double ns[4], nn[4];
    if (j > 0) load4(a.Q + 4 * (size_t)(c - a.nx), ns);
    else if (a.wall & 4) fv_ghost(ph, q, bg[3 * kBgGS], bg[3 * kBgGS + 1], bg[3 * kBgGS + 2], ns);
    else load4(a.Q + 4 * ((size_t)(a.nz - 1) * a.nx + i), ns);
    if (j < a.nz - 1) load4(a.Q + 4 * (size_t)(c + a.nx), nn);
    else if (a.wall & 8) fv_ghost(ph, q, bg[3 * kBgGN], bg[3 * kBgGN + 1], bg[3 * kBgGN + 2], nn);
    else load4(a.Q + 4 * (size_t)i, nn);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double sz = van_albada(q[v] - ns[v], nn[v] - q[v]);
      fv[2][v] = q[v] - 0.5 * sz;
      fv[3][v] = q[v] + 0.5 * sz;
    }
  }
  // flux differences across the cell: (F_W - F_E) + (F_S - F_N)
  double d[4];
  {
    double Fa[4], Fb[4];
    fv_flux(ph, fv[0], bg[3 * kBgC], bg[3 * kBgC + 2], 0, Fa);
    fv_flux(ph, fv[1], bg[3 * kBgC], bg[3 * kBgC + 2], 0, Fb);
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = Fa[v] - Fb[v];
  }
  {
    double Fa[4], Fb[4];
    fv_flux(ph, fv[2], bg[3 * kBgS], bg[3 * kBgS + 2], 1, Fa);
    fv_flux(ph, fv[3], bg[3 * kBgN], bg[3 * kBgN + 2], 1, Fb);
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = d[v] + (Fa[v] - Fb[v]);
  }
  const double Sw = -ph.geff * (q[0] - bg[3 * kBgC + 1]);
  const double k = 0.5 * dt * a.ih;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double inc = k * d[v];
    if (v == 2) inc += 0.5 * dt * Sw;
    if (v == 0) inc0 = inc;
#pragma unroll
    for (int f = 0; f < 4; ++f) fv[f][v] += inc;
  }
}

// Steps 3-4 for cell (i, j): Rusanov flux of its four faces from its own
// evolved face value and the facing value of the neighbour (or the wall
// ghost where the face is a wall), and the update.  fetch(f, own, nb) loads
// face f's two values, so that only one face's data is live at a time.
template <class Fetch>
__device__ inline void fv_update_cell(const Phys& ph, const FvArgs& a, int i, int j, double dt, Fetch fetch,
                                      double inc0, double out[4]) {
  const double* bg = a.bg + 15 * j;
  const int wall = (i == 0 ? a.wall & 1 : 0) | (i == a.nx - 1 ? a.wall & 2 : 0) | (j == 0 ? a.wall & 4 : 0) |
                   (j == a.nz - 1 ? a.wall & 8 : 0);
  double dx[4] = {0, 0, 0, 0}, dz[4] = {0, 0, 0, 0};   // G_east - G_west, G_north - G_south
  // a rolled loop: one face's values live at a time (the face index is
  // uniform, so its branches are scalar)
#pragma unroll 1
  for (int f = 0; f < 4; ++f) {
    const int d = f >> 1, hi = f & 1;
    const int row = d == 0 ? kBgC : (hi ? kBgN : kBgS);
    const double zf = bg[3 * row], rbf = bg[3 * row + 1], pbf = bg[3 * row + 2];
    double own[4], Qn[4], Fo[4], Fn[4], G[4], sn;
    fetch(f, own, Qn);
    const double so = fv_flux(ph, own, zf, pbf, d, Fo);
    if ((wall >> f) & 1) {
      fv_ghost(ph, own, zf, rbf, pbf, Qn);
      Fn[0] = -Fo[0]; Fn[1] = Fo[1]; Fn[2] = Fo[2]; Fn[3] = -Fo[3];
      const double pg = fv_pressure(ph, Qn, zf), irg = recip(Qn[0]);
      sn = fabs(Qn[1 + d] * irg) + sqrt(ph.gamma * pg * irg);
    } else {
      sn = fv_flux(ph, Qn, zf, pbf, d, Fn);
    }
    const double sp = fmax(so, sn);
    if (hi) rusanov_fv(sp, own, Fo, Qn, Fn, G);
    else rusanov_fv(sp, Qn, Fn, own, Fo, G);
    if (d == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) dx[v] = hi ? G[v] + dx[v] : -G[v];
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) dz[v] = hi ? G[v] + dz[v] : -G[v];
    }
  }
  double q[4];
  load4(a.Q + 4 * ((size_t)j * a.nx + i), q);
  const double Sh = -ph.geff * ((q[0] + inc0) - bg[3 * kBgC + 1]);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    out[v] = q[v] - dt * a.ih * (dx[v] + dz[v]);
    if (v == 2) out[v] += dt * Sh;
  }
}

// largest signal speed max(|u|,|w|) + c of a cell value at height z
__device__ inline double fv_lambda(const Phys& ph, const double q[4], double z) {
  const double ir = recip(q[0]);
  const double cs = sqrt(ph.gamma * fv_pressure(ph, q, z) * ir);
  return fmax(fabs(q[1]), fabs(q[2])) * ir + cs;
}

// workgroup maximum of lam -> time-step bound dtb[blockIdx]
template <int NT = kFvThreads>
__device__ inline void fv_block_bound(const Phys& ph, const FvArgs& a, double lam, int block) {
  __shared__ double smax[NT / kWave];
  lam = wave_max(lam);
  if ((threadIdx.x & (kWave - 1)) == 0) smax[threadIdx.x / kWave] = lam;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = smax[0];
    for (int w = 1; w < NT / kWave; ++w) m = fmax(m, smax[w]);
    a.dtb[block] = ph.cfl * a.h / (2.0 * m);
  }
}

// Steps 1-2, one thread per cell, face values to the workspace.
__global__ __launch_bounds__(kFvThreads) void k_fv_predict(Phys ph, FvArgs a) {
  const int c = blockIdx.x * kFvThreads + threadIdx.x;
  if (c >= a.C) return;
  double fv[4][4], inc0;
  fv_predict_cell(ph, a, c % a.nx, c / a.nx, a.clock[1], fv, inc0);
  const size_t C = (size_t)a.C;
  a.inc[c] = inc0;   // the half-step density feeds the source of the update
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int v = 0; v < 4; ++v) a.E[(size_t)(4 * f + v) * C + c] = fv[f][v];
}

// Steps 3-4, one thread per cell, from the workspace's face values; Q is
// updated in place (no thread reads another cell's Q), then the workgroup's
// time-step bound of the new values.
__global__ __launch_bounds__(kFvThreads) void k_fv_correct(Phys ph, FvArgs a) {
  const int c = blockIdx.x * kFvThreads + threadIdx.x;
  double lam = 0.0;
  if (c < a.C) {
    const int i = c % a.nx, j = c / a.nx;
    const size_t C = (size_t)a.C;
    const int nbr[4] = {i > 0 ? c - 1 : c + a.nx - 1, i < a.nx - 1 ? c + 1 : c - a.nx + 1,
                        j > 0 ? c - a.nx : (a.nz - 1) * a.nx + i, j < a.nz - 1 ? c + a.nx : i};
    auto fetch = [&](int f, double own[4], double nb[4]) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        own[v] = a.E[(size_t)(4 * f + v) * C + c];
        nb[v] = a.E[(size_t)(4 * (f ^ 1) + v) * C + nbr[f]];
      }
    };
    double out[4];
    fv_update_cell(ph, a, i, j, a.clock[1], fetch, a.inc[c], out);
    double2* o = reinterpret_cast<double2*>(a.Q + 4 * (size_t)c);
    o[0] = make_double2(out[0], out[1]);
    o[1] = make_double2(out[2], out[3]);
    lam = fv_lambda(ph, out, a.bg[15 * j]);
  }
  fv_block_bound(ph, a, lam, blockIdx.x);
}

// Rusanov flux of one face along d (0: x, 1: z) at height zf from the
// evolved values lo and hi on its low (west or south) and high side; d may
// differ between lanes (selects, no branches).  out = 1: the low side is a
// wall, its value is the wall ghost of hi; out = 2: the high side is a wall.
// The same arithmetic as the face loop of fv_update_cell.
__device__ inline double fv_flux_sel(const Phys& ph, const double q[4], double z, double pb, int d, double F[4]) {
  const double ir = recip(q[0]);
  const double u = q[1] * ir, w = q[2] * ir;
  const double p = ph.gm1 * (q[3] - 0.5 * (q[1] * u + q[2] * w) - q[0] * (ph.geff * z));
  const double pm = p - pb;
  const double un = d ? w : u;
  F[0] = d ? q[2] : q[1];
  F[1] = q[1] * un + (d == 0 ? pm : 0.0);
  F[2] = q[2] * un + (d == 1 ? pm : 0.0);
  F[3] = un * (q[3] + p);
  return fabs(un) + sqrt(ph.gamma * p * ir);
}

__device__ inline void fv_face(const Phys& ph, int d, double zf, double rbf, double pbf, int out, const double lo[4],
                               const double hi[4], double G[4]) {
  if (out == 0) {
    double Fl[4], Fh[4];
    const double sl = fv_flux_sel(ph, lo, zf, pbf, d, Fl);
    const double sh = fv_flux_sel(ph, hi, zf, pbf, d, Fh);
    rusanov_fv(fmax(sl, sh), lo, Fl, hi, Fh, G);
  } else {
    const double* in = out == 1 ? hi : lo;
    double qi[4], Fo[4], g[4], Fg[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) qi[v] = in[v];
    const double so = fv_flux_sel(ph, qi, zf, pbf, d, Fo);
    fv_ghost(ph, qi, zf, rbf, pbf, g);
    Fg[0] = -Fo[0]; Fg[1] = Fo[1]; Fg[2] = Fo[2]; Fg[3] = -Fo[3];
    const double pg = fv_pressure(ph, g, zf), irg = recip(g[0]);
    const double sg = fabs((d ? g[2] : g[1]) * irg) + sqrt(ph.gamma * pg * irg);
    const double sp = fmax(so, sg);
    if (out == 1) rusanov_fv(sp, g, Fg, qi, Fo, G);
    else rusanov_fv(sp, qi, Fo, g, Fg, G);
  }
}

// One step fused into one kernel on tiles of kTX x kTZ cells: every thread
// predicts its cell, the first threads also the ring of cells around the
// tile (each only for the face value the tile needs); the evolved face
// values meet in LDS; the update goes to Qn (other tiles still read Q), and
// the workgroup's time-step bound of the new values goes to dtb[tile].
constexpr int kTX = 16, kTZ = 16, kFT = kTX * kTZ;   // tile (one thread per tile cell)
constexpr int kRing = 2 * (kTX + kTZ), kFTR = kFT + kRing;   // workgroup: tile cells, then the ring
static_assert(kFT % kWave == 0 && kRing % kWave == 0, "tile and ring fill whole wavefronts");

__global__ __launch_bounds__(kFTR) void k_fv_fused(Phys ph, FvArgs a, double* Qn) {
  // evolved face values by face type, variable, row, column; each array is
  // padded by one in the direction of the neighbour that reads it:
  // west values of columns 0..kTX (kTX: east ring), east values of columns
  // -1..kTX-1 (stored at column + 1), south values of rows 0..kTZ (kTZ:
  // north ring), north values of rows -1..kTZ-1 (stored at row + 1)
  __shared__ double sWv[4][kTZ][kTX + 1], sEv[4][kTZ][kTX + 1];
  __shared__ double sSv[4][kTZ + 1][kTX], sNv[4][kTZ + 1][kTX];
  const int t = threadIdx.x, tx = t % kTX, tz = t / kTX;
  const int x0 = blockIdx.x * kTX, z0 = blockIdx.y * kTZ;
  const int ew = min(kTX, a.nx - x0), eh = min(kTZ, a.nz - z0);   // extent of the tile inside the domain
  const double dt = a.clock[1];
  const bool inside = t < kFT && tx < ew && tz < eh;
  // ring (threads kFT..kFTR-1, wavefronts of their own): left and right
  // columns (the face towards the tile), bottom and top rows
  if (t >= kFT) {
    const int q = t - kFT;
    int rx, rz, f;
    if (q < kTZ) { rx = -1; rz = q; f = 1; }
    else if (q < 2 * kTZ) { rx = ew; rz = q - kTZ; f = 0; }
    else if (q < 2 * kTZ + kTX) { rx = q - 2 * kTZ; rz = -1; f = 3; }
    else { rx = q - 2 * kTZ - kTX; rz = eh; f = 2; }
    const bool used = (f < 2) ? rz < eh : rx < ew;
    int gi = x0 + rx, gj = z0 + rz;
    bool ok = used;
    if (gi < 0 || gi >= a.nx) { ok = ok && !(a.wall & 3); gi = gi < 0 ? gi + a.nx : gi - a.nx; }
    if (gj < 0 || gj >= a.nz) { ok = ok && !(a.wall & 12); gj = gj < 0 ? gj + a.nz : gj - a.nz; }
    if (ok) {
      double rv[4][4], rinc;
      fv_predict_cell(ph, a, gi, gj, dt, rv, rinc);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f is known only at run time: select with constant indices so rv stays in registers
        if (f == 1) sEv[v][rz][0] = rv[1][v];
        else if (f == 0) sWv[v][rz][ew] = rv[0][v];
        else if (f == 3) sNv[v][0][rx] = rv[3][v];
        else sSv[v][eh][rx] = rv[2][v];
      }
    }
  }
  double inc0 = 0.0;
  if (inside) {
    double fv[4][4];
    fv_predict_cell(ph, a, x0 + tx, z0 + tz, dt, fv, inc0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sWv[v][tz][tx] = fv[0][v];
      sEv[v][tz][tx + 1] = fv[1][v];
      sSv[v][tz][tx] = fv[2][v];
      sNv[v][tz + 1][tx] = fv[3][v];
    }
  }
  __syncthreads();
  // every face of the tile once: z faces (rows 0..eh, the south face of each
  // row of cells and the tile's top), then x faces (columns 0..ew); a job's
  // flux replaces the low side's value, which only this job reads
  constexpr int kZJobs = (kTZ + 1) * kTX, kXJobs = kTZ * (kTX + 1);
  constexpr int zvs = (kTZ + 1) * kTX, xvs = kTZ * (kTX + 1);   // variable strides of the two array shapes
  for (int k = t; k < kZJobs + kXJobs; k += kFTR) {
    const bool zj = k < kZJobs;
    const int kk = zj ? k : k - kZJobs;
    const int r = zj ? kk / kTX : kk / (kTX + 1), col = zj ? kk % kTX : kk % (kTX + 1);
    if (!(zj ? (r <= eh && col < ew) : (r < eh && col <= ew))) continue;
    const int d = zj ? 1 : 0, vs = zj ? zvs : xvs;
    double* plo = zj ? &sNv[0][r][col] : &sEv[0][r][col];
    const double* phi = zj ? &sSv[0][r][col] : &sWv[0][r][col];
    const int gj = z0 + r;
    // face height: x faces at the row centre; z faces at the south face of
    // row gj, the tile's top face at the north face of the row below it
    const double* bf = !zj ? a.bg + 15 * gj + 3 * kBgC
                           : (r < eh ? a.bg + 15 * gj + 3 * kBgS : a.bg + 15 * (gj - 1) + 3 * kBgN);
    int out = 0;
    if (zj) {
      if (r == 0 && z0 == 0 && (a.wall & 4)) out = 1;
      else if (r == eh && z0 + eh == a.nz && (a.wall & 8)) out = 2;
    } else {
      if (col == 0 && x0 == 0 && (a.wall & 1)) out = 1;
      else if (col == ew && x0 + ew == a.nx && (a.wall & 2)) out = 2;
    }
    double lo[4], hi[4], G[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) { lo[v] = plo[v * vs]; hi[v] = phi[v * vs]; }
    fv_face(ph, d, bf[0], bf[1], bf[2], out, lo, hi, G);
#pragma unroll
    for (int v = 0; v < 4; ++v) plo[v * vs] = G[v];
  }
  __syncthreads();
  double lam = 0.0;
  if (inside) {
    const int i = x0 + tx, j = z0 + tz;
    double q[4], out[4];
    load4(a.Q + 4 * ((size_t)j * a.nx + i), q);
    const double Sh = -ph.geff * ((q[0] + inc0) - a.bg[15 * j + 3 * kBgC + 1]);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double dx = sEv[v][tz][tx + 1] - sEv[v][tz][tx];   // G_east - G_west
      const double dz = sNv[v][tz + 1][tx] - sNv[v][tz][tx];   // G_north - G_south
      out[v] = q[v] - dt * a.ih * (dx + dz);
      if (v == 2) out[v] += dt * Sh;
    }
    // other tiles read only the two outer layers of this tile (their ring
    // cells and the ring cells' neighbours): interior cells take the new
    // value in place, the outer layers go through Qn and the copy-back
    const bool edge = tx <= 1 || tx >= ew - 2 || tz <= 1 || tz >= eh - 2;
    double2* o = reinterpret_cast<double2*>((edge ? Qn : a.Q) + 4 * ((size_t)j * a.nx + i));
    o[0] = make_double2(out[0], out[1]);
    o[1] = make_double2(out[2], out[3]);
    lam = fv_lambda(ph, out, a.bg[15 * j]);
  }
  fv_block_bound<kFTR>(ph, a, lam, blockIdx.y * gridDim.x + blockIdx.x);
}

// Q <- Qn on the two outer layers of every tile of the fused step (workgroup
// b >= 1: tile b - 1, one thread per cell); workgroup 0 instead reduces the
// tiles' time-step bounds and advances the clock (t += dt, steps += 1, then
// dt <- the minimum unless update is 0), the work of k_clock, beside the copy.
__global__ __launch_bounds__(kFT) void k_fv_commit(const double* __restrict__ Qn, double* __restrict__ Q,
                                                          int nx, int nz, double* clock, const double* dtb, int nb,
                                                          int update) {
  const int t = threadIdx.x;
  if (blockIdx.x == 0) {
    __shared__ double sm[kFT / kWave];
    double m = __builtin_inf();
    if (update) {
      // four independent loads in flight per thread
      int k = t;
      for (; k + 3 * kFT < nb; k += 4 * kFT) {
        const double a0 = dtb[k], a1 = dtb[k + kFT], a2 = dtb[k + 2 * kFT], a3 = dtb[k + 3 * kFT];
        m = fmin(m, fmin(fmin(a0, a1), fmin(a2, a3)));
      }
      for (; k < nb; k += kFT) m = fmin(m, dtb[k]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmin(m, __shfl_xor(m, o, kWave));
    if ((t & (kWave - 1)) == 0) sm[t / kWave] = m;
    __syncthreads();
    if (t == 0) {
      double r = sm[0];
      for (int k = 1; k < kFT / kWave; ++k) r = fmin(r, sm[k]);
      clock[0] += clock[1];
      clock[3] += 1.0;
      if (update) clock[1] = r;
    }
    return;
  }
  const int tiles_x = (nx + kTX - 1) / kTX, b = blockIdx.x - 1;
  const int x0 = (b % tiles_x) * kTX, z0 = (b / tiles_x) * kTZ;
  const int ew = min(kTX, nx - x0), eh = min(kTZ, nz - z0);
  const int tx = t % kTX, tz = t / kTX;
  if (tx >= ew || tz >= eh) return;
  if (!(tx <= 1 || tx >= ew - 2 || tz <= 1 || tz >= eh - 2)) return;
  const size_t c = (size_t)(z0 + tz) * nx + x0 + tx;
  const double2* src = reinterpret_cast<const double2*>(Qn + 4 * c);
  double2* dst = reinterpret_cast<double2*>(Q + 4 * c);
  const double2 v0 = src[0], v1 = src[1];
  dst[0] = v0;
  dst[1] = v1;
}

// time-step bound of every workgroup of cells from the current Q
__global__ __launch_bounds__(kFvThreads) void k_fv_dt(Phys ph, FvArgs a) {
  const int c = blockIdx.x * kFvThreads + threadIdx.x;
  double lam = 0.0;
  if (c < a.C) {
    double q[4];
    load4(a.Q + 4 * (size_t)c, q);
    lam = fv_lambda(ph, q, a.bg[15 * (c / a.nx)]);
  }
  fv_block_bound(ph, a, lam, blockIdx.x);
}

// cell-centre initial values (kind 0 bubbles, kind 1 advected density wave)
__global__ void k_fv_init(Phys ph, FvArgs a, double x0, int kind, FvBubbles B, double t0) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.C) return;
  const int i = c % a.nx, j = c / a.nx;
  const double x = x0 + (i + 0.5) * a.h, z = a.bg[15 * j];
  double q[4];
  if (kind == 1) {
    const double X = x - ph.mms_u * t0, Z = z - ph.mms_w * t0;
    const double rho = 1.0 + ph.mms_amp * sin(ph.mms_kx * X) * sin(ph.mms_kz * Z);
    q[0] = rho; q[1] = rho * ph.mms_u; q[2] = rho * ph.mms_w;
    q[3] = ph.mms_p / ph.gm1 + 0.5 * rho * (ph.mms_u * ph.mms_u + ph.mms_w * ph.mms_w);
  } else {
    double th = 0.0;
    for (int b = 0; b < B.nb; ++b) {
      const double* bb = B.b + 6 * b;
      const double r = sqrt((x - bb[4]) * (x - bb[4]) + (z - bb[5]) * (z - bb[5]));
      if (bb[0] == 0.0) th += r <= bb[2] ? 0.5 * bb[1] * (1.0 + cos(M_PI * r / bb[2])) : 0.0;
      else th += r <= bb[2] ? bb[1] : bb[1] * exp(-(r - bb[2]) * (r - bb[2]) / (bb[3] * bb[3]));
    }
    const double pi = 1.0 - ph.g * z / (ph.cp * ph.theta);
    const double pb = a.bg[15 * j + 2];
    const double rho = pb / (ph.R * (ph.theta + th) * pi);
    q[0] = rho; q[1] = 0.0; q[2] = 0.0;
    q[3] = pb / ph.gm1 + rho * ph.g * z;
  }
  double2* o = reinterpret_cast<double2*>(a.Q + 4 * (size_t)c);
  o[0] = make_double2(q[0], q[1]);
  o[1] = make_double2(q[2], q[3]);
}

__global__ void k_fv_health(Phys ph, FvArgs a, int* flag) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.C) return;
  double q[4];
  load4(a.Q + 4 * (size_t)c, q);
  bool bad = !(isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && isfinite(q[3])) || !(q[0] > 0.0);
  if (!bad) bad = !(fv_pressure(ph, q, a.bg[15 * (c / a.nx)]) > 0.0);
  if (bad) atomicOr(flag, 1);
}

static size_t align256_fv(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace adg

using namespace adg;

struct adg_fv {
  adg_params prm{};
  adg_fv_desc desc{};
  Phys ph{};
  int C = 0, blocks = 0, tiles = 0;   // cell workgroups, tiles of the fused step
  double* d_bg = nullptr;
  double* Q = nullptr;
  void* ws = nullptr;
  double* clock = nullptr;
  size_t off_e = 0, off_inc = 0, off_dtb = 0, off_h = 0, ws_bytes = 0;
};

namespace {

int fv_validate(const adg_params* p, const adg_fv_desc* d) {
  if (!p || !d) return fail(ADG_EINVAL, "null argument");
  if (p->order != 0) return fail(ADG_EINVAL, "order must be 0 for the finite-volume scheme");
  if (!(p->gamma > 1.0) || !(p->R > 0.0) || !(p->cp > 0.0)) return fail(ADG_EINVAL, "invalid gas constants");
  if (p->gravity && (!(p->theta_bg > 0.0) || !(p->p0 > 0.0) || !(p->g >= 0.0)))
    return fail(ADG_EINVAL, "invalid background atmosphere");
  if (!(p->cfl > 0.0)) return fail(ADG_EINVAL, "cfl must be > 0");
  if (p->mu != 0.0) return fail(ADG_EUNSUPPORTED, "the finite-volume scheme is inviscid (mu must be 0)");
  if (p->mms) return fail(ADG_EUNSUPPORTED, "no manufactured source in the finite-volume scheme");
  if (d->nx < 1 || d->nz < 1 || !(d->h > 0.0) || !std::isfinite(d->h) || !std::isfinite(d->x0) ||
      !std::isfinite(d->z0))
    return fail(ADG_EINVAL, "invalid domain");
  for (int f = 0; f < 4; ++f)
    if (d->bc[f] != ADG_BC_PERIODIC && d->bc[f] != ADG_BC_WALL) return fail(ADG_EINVAL, "invalid bc");
  if ((d->bc[0] == ADG_BC_PERIODIC) != (d->bc[1] == ADG_BC_PERIODIC) ||
      (d->bc[2] == ADG_BC_PERIODIC) != (d->bc[3] == ADG_BC_PERIODIC))
    return fail(ADG_EINVAL, "periodic boundaries must come in pairs");
  if ((long long)d->nx * d->nz > (1LL << 28)) return fail(ADG_EINVAL, "too many cells");
  return ADG_OK;
}

// hydrostatic background of constant potential temperature at height z
void fv_background(const adg_params& p, double z, double& rb, double& pb) {
  if (!p.gravity) { rb = 0.0; pb = 0.0; return; }
  const double pi = 1.0 - p.g * z / (p.cp * p.theta_bg);
  pb = p.p0 * std::pow(pi, p.cp / p.R);
  rb = pb / (p.R * p.theta_bg * pi);
}

FvArgs fv_args(const adg_fv* m) {
  FvArgs a{};
  char* ws = static_cast<char*>(m->ws);
  a.Q = m->Q;
  a.E = ws ? reinterpret_cast<double*>(ws + m->off_e) : nullptr;
  a.inc = ws ? reinterpret_cast<double*>(ws + m->off_inc) : nullptr;
  a.dtb = ws ? reinterpret_cast<double*>(ws + m->off_dtb) : nullptr;
  a.clock = m->clock; a.bg = m->d_bg;
  a.nx = m->desc.nx; a.nz = m->desc.nz; a.C = m->C; a.h = m->desc.h; a.ih = 1.0 / m->desc.h;
  a.wall = 0;
  for (int f = 0; f < 4; ++f)
    if (m->desc.bc[f] == ADG_BC_WALL) a.wall |= 1 << f;
  return a;
}

int fv_need_state(adg_fv* m) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (!m->Q || !m->ws || !m->clock) return fail(ADG_ESTATE, "no state bound (adg_fv_set_state)");
  return ADG_OK;
}

}  // namespace

extern "C" {

int adg_fv_init(const adg_params* prm, const adg_fv_desc* mesh, adg_fv** out) {
  if (!out) return fail(ADG_EINVAL, "null out");
  int rc = fv_validate(prm, mesh);
  if (rc) return rc;
  adg_fv* m = new (std::nothrow) adg_fv();
  if (!m) return fail(ADG_ENOMEM, "out of host memory");
  m->prm = *prm;
  m->desc = *mesh;
  m->C = mesh->nx * mesh->nz;
  m->blocks = (m->C + kFvThreads - 1) / kFvThreads;
  m->tiles = ((mesh->nx + kTX - 1) / kTX) * ((mesh->nz + kTZ - 1) / kTZ);
  adg_params p1 = *prm;
  p1.order = 1;   // make_phys reads the order only for the DG time-step rule
  m->ph = make_phys(p1);
  m->ph.N = 0;
  // background table: centre, south face, north face, south and north ghost centres
  const double h = mesh->h;
  std::vector<double> bg((size_t)mesh->nz * 15);
  for (int j = 0; j < mesh->nz; ++j) {
    const double zc = mesh->z0 + (j + 0.5) * h;
    const double zs[5] = {zc, zc - 0.5 * h, zc + 0.5 * h, zc - h, zc + h};
    for (int k = 0; k < 5; ++k) {
      double rb, pb;
      fv_background(*prm, zs[k], rb, pb);
      bg[15 * j + 3 * k] = zs[k];
      bg[15 * j + 3 * k + 1] = rb;
      bg[15 * j + 3 * k + 2] = pb;
    }
  }
  if (hipMalloc(&m->d_bg, sizeof(double) * bg.size()) != hipSuccess) {
    delete m;
    return fail(ADG_ENOMEM, "device allocation failed");
  }
  if (hipMemcpy(m->d_bg, bg.data(), sizeof(double) * bg.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(m->d_bg);
    delete m;
    return fail(ADG_EHIP, "upload failed");
  }
  const size_t C = (size_t)m->C;
  size_t off = 0;
  m->off_e = off; off = align256_fv(off + sizeof(double) * 16 * C);
  m->off_inc = off; off = align256_fv(off + sizeof(double) * C);
  m->off_dtb = off; off = align256_fv(off + sizeof(double) * std::max(m->blocks, m->tiles));
  m->off_h = off; off = align256_fv(off + sizeof(int));
  m->ws_bytes = off;
  *out = m;
  return ADG_OK;
}

int adg_fv_destroy(adg_fv* m) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (m->d_bg) (void)hipFree(m->d_bg);
  delete m;
  return ADG_OK;
}

int adg_fv_info(const adg_fv* m, int* n_cells) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (n_cells) *n_cells = m->C;
  return ADG_OK;
}

int adg_fv_workspace_bytes(const adg_fv* m, size_t* bytes) {
  if (!m || !bytes) return fail(ADG_EINVAL, "null argument");
  *bytes = m->ws_bytes;
  return ADG_OK;
}

int adg_fv_set_state(adg_fv* m, double* Q, void* workspace, double* clock) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (!Q || !workspace || !clock) return fail(ADG_EINVAL, "null buffer");
  if (((uintptr_t)workspace & 255) != 0) return fail(ADG_EINVAL, "workspace must be 256-byte aligned");
  if (((uintptr_t)Q & 15) != 0 || ((uintptr_t)clock & 7) != 0) return fail(ADG_EINVAL, "misaligned buffer");
  m->Q = Q; m->ws = workspace; m->clock = clock;
  return ADG_OK;
}

int adg_fv_init_state(adg_fv* m, int kind, int n_bubbles, const double* bubbles, double t0, void* stream) {
  int rc = fv_need_state(m);
  if (rc) return rc;
  if (kind != 0 && kind != 1) return fail(ADG_EINVAL, "kind must be 0 (bubbles) or 1 (density wave)");
  if (kind == 0 && !m->prm.gravity) return fail(ADG_EINVAL, "bubble states need gravity (background)");
  if (n_bubbles < 0 || n_bubbles > kFvBubbles || (n_bubbles > 0 && !bubbles))
    return fail(ADG_EINVAL, "bad bubble list");
  FvBubbles B{};
  B.nb = kind == 0 ? n_bubbles : 0;
  for (int b = 0; b < B.nb; ++b) {
    const double* bb = bubbles + 6 * b;
    if (bb[0] != ADG_SHAPE_COSINE && bb[0] != ADG_SHAPE_PLATEAU_GAUSS) return fail(ADG_EINVAL, "bad bubble shape");
    if (bb[0] == ADG_SHAPE_COSINE && !(bb[2] > 0.0)) return fail(ADG_EINVAL, "cosine bubble radius must be > 0");
    if (bb[0] == ADG_SHAPE_PLATEAU_GAUSS && !(bb[3] > 0.0)) return fail(ADG_EINVAL, "decay s must be > 0");
    for (int k = 0; k < 6; ++k) B.b[6 * b + k] = bb[k];
  }
  hipLaunchKernelGGL(k_fv_init, dim3(m->blocks), dim3(kFvThreads), 0, (hipStream_t)stream, m->ph, fv_args(m),
                     m->desc.x0, kind, B, t0);
  return check_launch("fv_init");
}

int adg_fv_compute_dt(adg_fv* m, void* stream) {
  int rc = fv_need_state(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const FvArgs a = fv_args(m);
  hipLaunchKernelGGL(k_fv_dt, dim3(m->blocks), dim3(kFvThreads), 0, s, m->ph, a);
  rc = check_launch("fv_dt");
  if (rc) return rc;
  return launch_clock(m->clock, a.dtb, nullptr, nullptr, 1, m->blocks, 0, 1, s);
}

int adg_fv_predictor(adg_fv* m, void* stream) {
  int rc = fv_need_state(m);
  if (rc) return rc;
  hipLaunchKernelGGL(k_fv_predict, dim3(m->blocks), dim3(kFvThreads), 0, (hipStream_t)stream, m->ph, fv_args(m));
  return check_launch("fv_predict");
}

int adg_fv_corrector(adg_fv* m, void* stream) {
  int rc = fv_need_state(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const FvArgs a = fv_args(m);
  hipLaunchKernelGGL(k_fv_correct, dim3(m->blocks), dim3(kFvThreads), 0, s, m->ph, a);
  rc = check_launch("fv_correct");
  if (rc) return rc;
  return launch_clock(m->clock, a.dtb, nullptr, nullptr, 1, m->blocks, 1, m->prm.fixed_dt ? 0 : 1, s);
}

int adg_fv_step(adg_fv* m, void* stream) {
  int rc = fv_need_state(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const FvArgs a = fv_args(m);
  double* Qn = a.E;   // the fused step keeps its new values in the face-value area
  const dim3 tiles((m->desc.nx + kTX - 1) / kTX, (m->desc.nz + kTZ - 1) / kTZ);
  hipLaunchKernelGGL(k_fv_fused, tiles, dim3(kFTR), 0, s, m->ph, a, Qn);
  rc = check_launch("fv_fused");
  if (rc) return rc;
  // copy-back of the tiles' edge cells plus one workgroup for the clock
  hipLaunchKernelGGL(k_fv_commit, dim3(m->tiles + 1), dim3(kFT), 0, s, (const double*)Qn, m->Q,
                     m->desc.nx, m->desc.nz, m->clock, (const double*)a.dtb, m->tiles, m->prm.fixed_dt ? 0 : 1);
  return check_launch("fv_commit");
}

int adg_fv_check_health(adg_fv* m, void* stream) {
  int rc = fv_need_state(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  int* flag = reinterpret_cast<int*>(static_cast<char*>(m->ws) + m->off_h);
  if (hipMemsetAsync(flag, 0, sizeof(int), s) != hipSuccess) return fail(ADG_EHIP, "memset");
  hipLaunchKernelGGL(k_fv_health, dim3(m->blocks), dim3(kFvThreads), 0, s, m->ph, fv_args(m), flag);
  rc = check_launch("fv_health");
  if (rc) return rc;
  int hf = 0;
  if (hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return fail(ADG_EHIP, "copy");
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ADG_EHIP, "sync");
  if (hf) return fail(ADG_ESTATE, "state has non-finite values or non-positive density/pressure");
  return ADG_OK;
}

}  // extern "C"
