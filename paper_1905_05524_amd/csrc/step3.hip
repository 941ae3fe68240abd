// Three-dimensional ADER-DG step kernels for gfx950 on a uniform grid of
// cubes: space-time predictor, corrector with the viscous Rusanov face flux
// (periodic and wall faces) and the CFL candidate of every cell, initial
// states and the health check.
//
// Work decomposition.  A workgroup of kThreads3 threads holds CB cells; the
// thread t owns spatial node t % nd (nd = n^3) of cell slot t / nd, so a
// cell's nodes are consecutive lanes.  For n = 2 and n = 4 every cell lies in
// one wavefront and the LDS hand-offs between its nodes need only a
// wavefront barrier; otherwise cells straddle wavefronts and the workgroup
// synchronises.  Threads past CB * nd (when nd does not divide the
// workgroup) mirror the threads of slot 0: same cell, same node, hence the
// same values written to the same LDS addresses, and no global stores.  Tensor-product contractions along x, y and z read n values of an
// LDS slice per output; the space-time iterate of a node (n time levels x 5
// variables) stays in registers.
#include "adg3_internal.h"

namespace adg {

constexpr int kThreads3 = 256;

template <int n>
struct Cfg3 {
  static constexpr int nn = n * n, nd = n * n * n;
  static constexpr int CB = kThreads3 / nd;               // cells per workgroup
  static constexpr bool spare = CB * nd != kThreads3;      // threads without a cell
  static constexpr bool WL = (kWave % nd == 0);           // cells never straddle a wavefront
  static constexpr int pred_slot = 20 * nd;               // state slice [5][nd] + fluxes [3][5][nd]
  static constexpr int corr_slot = 30 * nn + 12 * nn + 2; // G [6][5][nn], speeds [2][6 nn], maxima [2]
};

template <bool WL>
__device__ inline void sync3() {
  if constexpr (WL) wave_sync();
  else __syncthreads();
}

// ---------------------------------------------------------------- physics
__device__ inline double pressure3(const Phys& ph, const double q[5], double z) {
  const double geo = q[0] * (ph.geff * z);
  return ph.gm1 * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0] - geo);
}

// Flux along x, y, z and the gravity source of the vertical momentum at one
// node: the equation set of Section 2 in three dimensions (eqs. equation-set,
// eos, temperature, stress-tensor, heat-conduction-coeff,
// momentum-equation-split).  g[d]: gradient of the conserved state along d in
// reference coordinates (h times the physical one); the 1/h of the viscous
// and heat fluxes is carried by mu_h = mu/h and kappa_h = kappa/h, the
// hydrostatic part of the vertical pressure gradient by gh = g h (0 without
// gravity).  rb, pb: background density and pressure at the node height z.
__device__ inline void flux_source3(const Phys& ph, const double q[5], const double g[3][5], double z, double rb,
                                    double pb, double mu_h, double kappa_h, double gh, double F[3][5],
                                    double& Sw) {
  const double rho = q[0], E = q[4];
  const double ir = recip(rho);
  const double u[3] = {q[1] * ir, q[2] * ir, q[3] * ir};
  const double gzz = ph.geff * z;
  const double p = ph.gm1 * (E - 0.5 * (q[1] * u[0] + q[2] * u[1] + q[3] * u[2]) - rho * gzz);
  const double pm = p - pb;
  const double T = p * ir * ph.iR;
  double du[3][3];   // du[a][d] = d u_a / d x_d (reference coordinates)
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d) du[a][d] = (g[d][1 + a] - u[a] * g[d][0]) * ir;
  const double hv2 = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + gzz;
  double dT[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double dp = ph.gm1 * (g[d][4] - hv2 * g[d][0] - rho * (u[0] * du[0][d] + u[1] * du[1][d] + u[2] * du[2][d]));
    if (d == 2) dp -= ph.gm1 * rho * gh;
    dT[d] = (dp - ph.R * T * g[d][0]) * ir * ph.iR;
  }
  const double div = du[0][0] + du[1][1] + du[2][2];
  double sig[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      sig[a][b] = mu_h * ((a == b ? (2.0 / 3.0) * div : 0.0) - (du[a][b] + du[b][a]));
  const double H = E + p;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    F[d][0] = q[1 + d];
#pragma unroll
    for (int a = 0; a < 3; ++a) F[d][1 + a] = q[1 + a] * u[d] + (a == d ? pm : 0.0) + sig[a][d];
    F[d][4] = u[d] * H + (u[0] * sig[0][d] + u[1] * sig[1][d] + u[2] * sig[2][d]) - kappa_h * dT[d];
  }
  Sw = -ph.geff * (rho - rb);
}

// largest wave speed along d and the viscous speed at a face node
__device__ inline void eig3(const Phys& ph, int d, const double q[5], double zf, double& lam, double& lv) {
  const double ir = 1.0 / q[0];
  const double p = pressure3(ph, q, zf);
  const double un = d == 0 ? q[1] : (d == 1 ? q[2] : q[3]);
  lam = fabs(un * ir) + sqrt(ph.gamma * p * ir);
  lv = ph.lv_coef * ir;
}

// No-slip wall with normal direction d (Section 4.2): the ghost carries the
// background density and pressure at the face height with the mirrored
// velocity; its normal flux mirrors the interior one for mass and energy
// (the energy flux around twice the background heat flux kappa g / cp through
// horizontal walls) and repeats it for the momenta.  Without gravity the
// interior density and pressure stand in for the background.
__device__ inline void wall_ghost3(const Phys& ph, int d, double zf, const double Qi[5], const double Fi[5],
                                   double Qg[5], double Fg[5]) {
  const double ir = 1.0 / Qi[0];
  const double u[3] = {Qi[1] * ir, Qi[2] * ir, Qi[3] * ir};
  double rb, pb;
  if (ph.gravity) background(ph, zf, rb, pb);
  else { rb = Qi[0]; pb = pressure3(ph, Qi, zf); }
  const double geo = ph.gravity ? rb * (ph.g * zf) : 0.0;
  Qg[0] = rb;
#pragma unroll
  for (int a = 0; a < 3; ++a) Qg[1 + a] = -(rb * u[a]);
  Qg[4] = pb / ph.gm1 + 0.5 * rb * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + geo;
  const double qbg = (ph.gravity && d == 2) ? ph.kappa * ph.g / ph.cp : 0.0;
  Fg[0] = -Fi[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) Fg[1 + a] = Fi[1 + a];
  Fg[4] = 2.0 * qbg - Fi[4];
}

// ---------------------------------------------------------------- predictor
// Gradient of the slice src ([5][nd] in LDS) at node (k, j, i) along x, y, z
// with the derivative-matrix rows of the node, then the flux and source.
template <int n>
__device__ inline void grad_flux3(const Phys& ph, const double* src, int i, int j, int k, const double Di[n],
                                  const double Dj[n], const double Dk[n], const double q[5], double z, double rb,
                                  double pb, double mu_h, double kappa_h, double gh, double F[3][5], double& Sw) {
  constexpr int nn = n * n, nd = nn * n;
  double g[3][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double* s = src + v * nd;
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) {
      gx = fma(Di[m], s[(k * n + j) * n + m], gx);
      gy = fma(Dj[m], s[(k * n + m) * n + i], gy);
      gz = fma(Dk[m], s[(m * n + j) * n + i], gz);
    }
    g[0][v] = gx; g[1][v] = gy; g[2][v] = gz;
  }
  flux_source3(ph, q, g, z, rb, pb, mu_h, kappa_h, gh, F, Sw);
}

// sum over the three directions of the contraction of the flux components
// ([3][5][nd] in LDS) with the rows Ti, Tj, Tk: the divergence for the
// derivative matrix, the volume term for the weighted transposed one
template <int n>
__device__ inline double div3(const double* sF, int v, int i, int j, int k, const double Ti[n], const double Tj[n],
                              const double Tk[n]) {
  constexpr int nn = n * n, nd = nn * n;
  const double* fx = sF + v * nd;
  const double* fy = sF + (5 + v) * nd;
  const double* fz = sF + (10 + v) * nd;
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < n; ++m) {
    s = fma(Ti[m], fx[(k * n + j) * n + m], s);
    s = fma(Tj[m], fy[(k * n + m) * n + i], s);
    s = fma(Tk[m], fz[(m * n + j) * n + i], s);
  }
  return s;
}

// Face data FD[f][kind][v][s][t] of one cell from its averaged state sq
// ([5][nd]) and fluxes sF ([3][5][nd]) in LDS: kind 0 the state, 1 the normal
// flux, extrapolated along the face normal with the boundary values of the
// basis.  The cell's nd threads (r = node index) share the 60 n^2 outputs.
template <int n>
__device__ inline void face_data3(const Tab<n>& tb, const double* sq, const double* sF, double* FDc, int r) {
  constexpr int nn = n * n, nd = nn * n;
  for (int o = r; o < 60 * nn; o += nd) {
    const int f = o / (10 * nn), rem = o - f * 10 * nn;
    const int kind = rem / (5 * nn), v = (rem / nn) % 5, st = rem % nn, s = st / n, t = st % n;
    const int d = f >> 1;
    const double* src = kind ? sF + (d * 5 + v) * nd : sq + v * nd;
    const int base = d == 0 ? (s * n + t) * n : (d == 1 ? s * nn + t : s * n + t);
    const int stride = d == 0 ? 1 : (d == 1 ? n : nn);
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) acc = fma((f & 1) ? tb.e1[m] : tb.e0[m], src[base + m * stride], acc);
    FDc[o] = acc;
  }
}

// Space-time predictor (Section 3): Picard sweeps
//   X_a = Q + dt sum_b P_ab R(X_b),  R = S - div F,  P = K1^{-1} W,
// from X_a = Q, then the time averages of state, flux and source, the update
// Q* = Q + dt (volume term of the averaged flux / h + averaged source) and
// the face data (averaged state and normal flux extrapolated to each face).
template <int n>
__global__ __launch_bounds__(kThreads3) void k_pred3(Phys ph, Tab<n> tb, Args3 a) {
  using G = Cfg3<n>;
  constexpr int nn = G::nn, nd = G::nd;
  constexpr bool WL = G::WL;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, r = tid % nd;
  const bool mirror = G::spare && tid >= G::CB * nd;
  const int slot = mirror ? 0 : tid / nd;
  const int cell = blockIdx.x * G::CB + slot;
  const bool valid = !mirror && cell < a.C;
  const int c = cell < a.C ? cell : a.C - 1;   // loads stay in bounds; only valid threads store
  double* sq = lds + slot * G::pred_slot;
  double* sF = sq + 5 * nd;
  const int i = r % n, j = (r / n) % n, k = r / nn;
  const double h = a.h;
  const int ck = c / (a.nx * a.ny);
  const double z = (a.z0 + ck * h) + h * a.gtab[GTab::XI * n + k];
  double rb, pb;
  background(ph, z, rb, pb);
  const double mu_h = ph.mu / h, kappa_h = ph.kappa / h, gh = ph.geff * h;
  const double dt = a.clock[1], sdt = -dt / h;
  double Di[n], Dj[n], Dk[n];
#pragma unroll
  for (int m = 0; m < n; ++m) {
    Di[m] = a.gtab[GTab::d(n) + i * n + m];
    Dj[m] = a.gtab[GTab::d(n) + j * n + m];
    Dk[m] = a.gtab[GTab::d(n) + k * n + m];
  }
  const double* Qc = a.Q + (size_t)c * 5 * nd;
  double Q0[5], X[n][5], R[n][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) Q0[v] = Qc[v * nd + r];
#pragma unroll
  for (int b = 0; b < n; ++b)
#pragma unroll
    for (int v = 0; v < 5; ++v) X[b][v] = Q0[v];

  for (int it = 0; it < a.iters; ++it) {
#pragma unroll
    for (int b = 0; b < n; ++b) {
      if (b > 0 && it == 0) {
        // the first sweep starts from Q^n at every time level: all levels
        // share level 0's residual (bit for bit)
#pragma unroll
        for (int v = 0; v < 5; ++v) R[b][v] = R[0][v];
        continue;
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) sq[v * nd + r] = X[b][v];
      sync3<WL>();
      double F[3][5], Sw;
      grad_flux3<n>(ph, sq, i, j, k, Di, Dj, Dk, X[b], z, rb, pb, mu_h, kappa_h, gh, F, Sw);
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = 0; v < 5; ++v) sF[(d * 5 + v) * nd + r] = F[d][v];
      sync3<WL>();
#pragma unroll
      for (int v = 0; v < 5; ++v) R[b][v] = sdt * div3<n>(sF, v, i, j, k, Di, Dj, Dk);
      R[b][3] = fma(dt, Sw, R[b][3]);
    }
#pragma unroll
    for (int a2 = 0; a2 < n; ++a2)
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < n; ++b) s = fma(tb.P[a2][b], R[b][v], s);
        X[a2][v] = Q0[v] + s;
      }
  }

  // time averages; the slice alternates between two LDS buffers so that one
  // barrier per time level suffices
  double Qb[5], Fb[3][5], Sb = 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Qb[v] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) Fb[d][v] = 0.0;
  }
#pragma unroll
  for (int b = 0; b < n; ++b) {
    double* buf = (b & 1) ? sF : sq;
#pragma unroll
    for (int v = 0; v < 5; ++v) buf[v * nd + r] = X[b][v];
    sync3<WL>();
    double F[3][5], Sw;
    grad_flux3<n>(ph, buf, i, j, k, Di, Dj, Dk, X[b], z, rb, pb, mu_h, kappa_h, gh, F, Sw);
    const double w = tb.w[b];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Qb[v] = fma(w, X[b][v], Qb[v]);
#pragma unroll
      for (int d = 0; d < 3; ++d) Fb[d][v] = fma(w, F[d][v], Fb[d][v]);
    }
    Sb = fma(w, Sw, Sb);
  }
  sync3<WL>();
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    sq[v * nd + r] = Qb[v];
#pragma unroll
    for (int d = 0; d < 3; ++d) sF[(d * 5 + v) * nd + r] = Fb[d][v];
  }
  sync3<WL>();

  // volume term (Dw[i][m] = w_m D[m][i] / w_i along each direction) and Q*
  double Wi[n], Wj[n], Wk[n];
#pragma unroll
  for (int m = 0; m < n; ++m) {
    Wi[m] = a.gtab[GTab::dw(n) + i * n + m];
    Wj[m] = a.gtab[GTab::dw(n) + j * n + m];
    Wk[m] = a.gtab[GTab::dw(n) + k * n + m];
  }
  const double ih = 1.0 / h;
  if (valid) {
    double* Qsc = a.Qs + (size_t)c * 5 * nd;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double vol = div3<n>(sF, v, i, j, k, Wi, Wj, Wk);
      Qsc[v * nd + r] = Q0[v] + dt * (vol * ih + (v == 3 ? Sb : 0.0));
    }
    face_data3<n>(tb, sq, sF, a.FD + (size_t)c * 60 * nn, r);
  }
}

// ------------------------------------------------ predictor, n = 4 (N = 3)
// One cell per wavefront, lane l = 16 k + 4 j + i.  The contractions along x
// and y run on the lanes of a quad (x) and of a 16-lane row (y) through the
// DPP network: rotation r brings each lane the value of the node r steps
// further along the line, multiplied by the matching entry of the lane's
// derivative-matrix row.  Only the z contractions go through LDS (one slice
// of 5 variables, read 4 values per output), so an LDS round trip per time
// level moves 10 writes and 40 reads per lane instead of 20 and 120.

// lane exchange of a double through the DPP network (two 32-bit moves; every
// lane of a quad or row has a source, so no lane keeps an old value)
template <int ctrl>
__device__ inline double dpp_d(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
// quad_perm control word: lane i of every quad reads lane (i + r) & 3
template <int r>
constexpr int quad_rot() {
  return ((0 + r) & 3) | (((1 + r) & 3) << 2) | (((2 + r) & 3) << 4) | (((3 + r) & 3) << 6);
}
constexpr int kRowRor = 0x120;   // row_ror:s control word base (rotation by s lanes within a row of 16)

// sum_r c[r] x(node r steps along x), the r = 0 term the lane's own value
__device__ inline double cx4(const double c[4], double x) {
  double s = c[0] * x;
  s = fma(c[1], dpp_d<quad_rot<1>()>(x), s);
  s = fma(c[2], dpp_d<quad_rot<2>()>(x), s);
  s = fma(c[3], dpp_d<quad_rot<3>()>(x), s);
  return s;
}
// the same along y (rows of 16 lanes hold the 4 x 4 nodes of one z level)
__device__ inline double cy4(const double c[4], double x) {
  double s = c[0] * x;
  s = fma(c[1], dpp_d<kRowRor + 4>(x), s);
  s = fma(c[2], dpp_d<kRowRor + 8>(x), s);
  s = fma(c[3], dpp_d<kRowRor + 12>(x), s);
  return s;
}
// z contraction of a [nd] LDS slice at node (j, i) = l & 15
__device__ inline double cz4(const double c[4], const double* s, int ji) {
  double acc = c[0] * s[ji];
  acc = fma(c[1], s[16 + ji], acc);
  acc = fma(c[2], s[32 + ji], acc);
  acc = fma(c[3], s[48 + ji], acc);
  return acc;
}

// rows of a node-indexed matrix table T (n = 4) matched to the lane
// exchanges: cx[r] = T[i][i'] and cy[r] = T[j][j'] with i', j' the node
// indices that rotation r delivers (found by sending the indices themselves
// through the same exchange), cz[m] = T[k][m]
__device__ inline void rot_rows4(const double* T, int i, int j, int k, double cx[4], double cy[4], double cz[4]) {
  const int pi1 = __builtin_amdgcn_mov_dpp(i, quad_rot<1>(), 0xF, 0xF, true);
  const int pi2 = __builtin_amdgcn_mov_dpp(i, quad_rot<2>(), 0xF, 0xF, true);
  const int pi3 = __builtin_amdgcn_mov_dpp(i, quad_rot<3>(), 0xF, 0xF, true);
  const int pj1 = __builtin_amdgcn_mov_dpp(j, kRowRor + 4, 0xF, 0xF, true);
  const int pj2 = __builtin_amdgcn_mov_dpp(j, kRowRor + 8, 0xF, 0xF, true);
  const int pj3 = __builtin_amdgcn_mov_dpp(j, kRowRor + 12, 0xF, 0xF, true);
  cx[0] = T[i * 4 + i]; cx[1] = T[i * 4 + pi1]; cx[2] = T[i * 4 + pi2]; cx[3] = T[i * 4 + pi3];
  cy[0] = T[j * 4 + j]; cy[1] = T[j * 4 + pj1]; cy[2] = T[j * 4 + pj2]; cy[3] = T[j * 4 + pj3];
#pragma unroll
  for (int m = 0; m < 4; ++m) cz[m] = T[k * 4 + m];
}

__global__ __launch_bounds__(kThreads3, 3) void k_pred3_w64(Phys ph, Tab<4> tb, Args3 a) {
  constexpr int n = 4, nd = 64;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, slot = tid >> 6, r = tid & 63;
  const int cell = blockIdx.x * (kThreads3 / kWave) + slot;
  const bool valid = cell < a.C;
  const int c = valid ? cell : a.C - 1;   // loads stay in bounds; nothing is stored for such lanes
  double* sq = lds + slot * 20 * nd;      // state slice [5][nd]; the averaged state in the epilogue
  double* sF = sq + 5 * nd;               // z fluxes [5][nd]; all averaged fluxes [3][5][nd] in the epilogue
  const int i = r & 3, j = (r >> 2) & 3, k = r >> 4, ji = r & 15;
  const double h = a.h;
  const int ck = c / (a.nx * a.ny);
  const double z = (a.z0 + ck * h) + h * a.gtab[GTab::XI * n + k];
  double rb, pb;
  background(ph, z, rb, pb);
  const double mu_h = ph.mu / h, kappa_h = ph.kappa / h, gh = ph.geff * h;
  const double dt = a.clock[1], sdt = -dt / h;
  double Cx[4], Cy[4], Cz[4];
  rot_rows4(a.gtab + GTab::d(n), i, j, k, Cx, Cy, Cz);
  const double* Qc = a.Q + (size_t)c * 5 * nd;
  double Q0[5], X[n][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) Q0[v] = Qc[v * nd + r];
#pragma unroll
  for (int b = 0; b < n; ++b)
#pragma unroll
    for (int v = 0; v < 5; ++v) X[b][v] = Q0[v];

  auto grad_flux = [&](const double q[5], double F[3][5], double& Sw) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sq[v * nd + r] = q[v];
    wave_sync();
    double g[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      g[0][v] = cx4(Cx, q[v]);
      g[1][v] = cy4(Cy, q[v]);
      g[2][v] = cz4(Cz, sq + v * nd, ji);
    }
    flux_source3(ph, q, g, z, rb, pb, mu_h, kappa_h, gh, F, Sw);
  };

  for (int it = 0; it < a.iters; ++it) {
#pragma unroll
    for (int b = 0; b < n; ++b) {
      if (b > 0 && it == 0) {
        // the first sweep starts from Q^n at every time level: all levels
        // share level 0's residual (bit for bit)
#pragma unroll
        for (int v = 0; v < 5; ++v) X[b][v] = X[0][v];
        continue;
      }
      double F[3][5], Sw;
      grad_flux(X[b], F, Sw);
#pragma unroll
      for (int v = 0; v < 5; ++v) sF[v * nd + r] = F[2][v];
      wave_sync();
      // the residual of time level b (times dt) replaces its iterate
#pragma unroll
      for (int v = 0; v < 5; ++v)
        X[b][v] = sdt * (cx4(Cx, F[0][v]) + cy4(Cy, F[1][v]) + cz4(Cz, sF + v * nd, ji));
      X[b][3] = fma(dt, Sw, X[b][3]);
      wave_sync();
    }
    // X <- Q + K1^{-1} W X: in-place solve with the unpivoted LU factors
    const double* lu = a.gtab + GTab::lu(n);
    int o = 0;
#pragma unroll
    for (int ii = 0; ii < n; ++ii) {
      const double wi = lu[o++];
#pragma unroll
      for (int v = 0; v < 5; ++v) X[ii][v] *= wi;
#pragma unroll
      for (int jj = 0; jj < ii; ++jj) {
        const double l = lu[o++];
#pragma unroll
        for (int v = 0; v < 5; ++v) X[ii][v] = fma(-l, X[jj][v], X[ii][v]);
      }
    }
#pragma unroll
    for (int ii = n - 1; ii >= 0; --ii) {
      const double iu = lu[o++];
#pragma unroll
      for (int v = 0; v < 5; ++v) X[ii][v] *= iu;
#pragma unroll
      for (int jj = ii + 1; jj < n; ++jj) {
        const double u = lu[o++];
#pragma unroll
        for (int v = 0; v < 5; ++v) X[ii][v] = fma(-u, X[jj][v], X[ii][v]);
      }
    }
#pragma unroll
    for (int a2 = 0; a2 < n; ++a2)
#pragma unroll
      for (int v = 0; v < 5; ++v) X[a2][v] += Q0[v];
  }

  // time averages; the averaged fluxes accumulate in the lane's own LDS
  // words [3][5][nd] (registers are short here), the state in registers
  double Qb[5], Sb = 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v) Qb[v] = 0.0;
#pragma unroll
  for (int b = 0; b < n; ++b) {
    double F[3][5], Sw;
    grad_flux(X[b], F, Sw);
    const double w = tb.w[b];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Qb[v] = fma(w, X[b][v], Qb[v]);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double* acc = sF + (d * 5 + v) * nd + r;
        *acc = b == 0 ? w * F[d][v] : fma(w, F[d][v], *acc);
      }
    }
    Sb = fma(w, Sw, Sb);
    wave_sync();
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) sq[v * nd + r] = Qb[v];
  wave_sync();

  // Lane indices and cell again from the thread id: kept live across the
  // sweeps they would occupy registers that the sweeps need (and spill).
  int t2 = threadIdx.x;
  asm volatile("" : "+v"(t2));
  const int r2 = t2 & 63, i2 = r2 & 3, j2 = (r2 >> 2) & 3, k2 = r2 >> 4;
  const int cell2 = blockIdx.x * (kThreads3 / kWave) + (t2 >> 6);
  // volume term with the weighted transposed derivative matrix, and Q*
  double Wx[4], Wy[4], Wz[4];
  rot_rows4(a.gtab + GTab::dw(n), i2, j2, k2, Wx, Wy, Wz);
  const double ih = 1.0 / h;
  if (cell2 < a.C) {
    double* Qsc = a.Qs + (size_t)cell2 * 5 * nd;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double vol = cx4(Wx, sF[v * nd + r2]) + cy4(Wy, sF[(5 + v) * nd + r2]) +
                         cz4(Wz, sF + (10 + v) * nd, r2 & 15);
      Qsc[v * nd + r2] = Q0[v] + dt * (vol * ih + (v == 3 ? Sb : 0.0));
    }
    face_data3<n>(tb, sq, sF, a.FD + (size_t)cell2 * 60 * 16, r2);
  }
}

// ---------------------------------------------------------------- corrector
// Per face node: the neighbour's face data (or the wall ghost), the largest
// wave and viscous speeds over both sides of the face, then the Rusanov flux
//   G = (F_L + F_R)/2 - (lambda + 2 eta lambda_v)/2 (Q_R - Q_L)
// with L the -axis side; per node: Q = Q* - dt/h (lifting of the six face
// fluxes), and the cell's CFL candidate from the new state.
template <int n>
__global__ __launch_bounds__(kThreads3) void k_corr3(Phys ph, Args3 a) {
  using G = Cfg3<n>;
  constexpr int nn = G::nn, nd = G::nd, NJ = 6 * nn, IT = (NJ + nd - 1) / nd;
  constexpr bool WL = G::WL;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, r = tid % nd;
  const bool mirror = G::spare && tid >= G::CB * nd;
  const int slot = mirror ? 0 : tid / nd;
  const int cell = blockIdx.x * G::CB + slot;
  const bool valid = !mirror && cell < a.C;
  const int c = cell < a.C ? cell : a.C - 1;
  double* sG = lds + slot * G::corr_slot;
  double* sl = sG + 30 * nn;
  double* sv = sl + 6 * nn;
  unsigned long long* smax = reinterpret_cast<unsigned long long*>(sv + 6 * nn);
  const int ci = c % a.nx, cj = (c / a.nx) % a.ny, ck = c / (a.nx * a.ny);
  const double h = a.h, dt = a.clock[1];
  const double zc = a.z0 + ck * h;
  if (r == 0) { smax[0] = 0ull; smax[1] = 0ull; }

  double qL[IT][5], qR[IT][5], fL[IT][5], fR[IT][5];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int q = r + it * nd;
    const bool act = q < NJ;
    const int qq = act ? q : 0;
    const int f = qq / nn, st = qq - f * nn, s = st / n;
    const int d = f >> 1, hi = f & 1;
    const double* own = a.FD + ((size_t)c * 6 + f) * 10 * nn + st;
    double Qo[5], Fo[5], Qn[5], Fn[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) { Qo[v] = own[v * nn]; Fo[v] = own[(5 + v) * nn]; }
    const int dim = d == 0 ? a.nx : (d == 1 ? a.ny : a.nz);
    const int pos = d == 0 ? ci : (d == 1 ? cj : ck);
    int np = pos + (hi ? 1 : -1);
    const bool outside = np < 0 || np >= dim;
    const bool wall = outside && ((a.wall >> f) & 1);
    if (outside && !wall) np = np < 0 ? np + dim : np - dim;
    const double zf = f == 4 ? zc : (f == 5 ? zc + h : zc + h * a.gtab[GTab::XI * n + s]);
    if (wall) {
      wall_ghost3(ph, d, zf, Qo, Fo, Qn, Fn);
    } else {
      const int o = d == 0 ? (ck * a.ny + cj) * a.nx + np
                           : (d == 1 ? (ck * a.ny + np) * a.nx + ci : (np * a.ny + cj) * a.nx + ci);
      const double* oth = a.FD + ((size_t)o * 6 + (f ^ 1)) * 10 * nn + st;
#pragma unroll
      for (int v = 0; v < 5; ++v) { Qn[v] = oth[v * nn]; Fn[v] = oth[(5 + v) * nn]; }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      qL[it][v] = hi ? Qo[v] : Qn[v]; qR[it][v] = hi ? Qn[v] : Qo[v];
      fL[it][v] = hi ? Fo[v] : Fn[v]; fR[it][v] = hi ? Fn[v] : Fo[v];
    }
    double l1, v1, l2, v2;
    eig3(ph, d, qL[it], zf, l1, v1);
    eig3(ph, d, qR[it], zf, l2, v2);
    if (act) { sl[q] = fmax(l1, l2); sv[q] = fmax(v1, v2); }
  }
  sync3<WL>();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int q = r + it * nd;
    if (q < NJ) {
      const int f = q / nn, st = q - f * nn;
      double lm = sl[f * nn], vm = sv[f * nn];
      for (int m = 1; m < nn; ++m) { lm = fmax(lm, sl[f * nn + m]); vm = fmax(vm, sv[f * nn + m]); }
      const double sp = lm + 2.0 * a.eta * vm;
#pragma unroll
      for (int v = 0; v < 5; ++v)
        sG[(f * 5 + v) * nn + st] = 0.5 * (fL[it][v] + fR[it][v]) - 0.5 * sp * (qR[it][v] - qL[it][v]);
    }
  }
  sync3<WL>();

  const int i = r % n, j = (r / n) % n, k = r / nn;
  const double L0i = a.gtab[GTab::L0 * n + i], L1i = a.gtab[GTab::L1 * n + i];
  const double L0j = a.gtab[GTab::L0 * n + j], L1j = a.gtab[GTab::L1 * n + j];
  const double L0k = a.gtab[GTab::L0 * n + k], L1k = a.gtab[GTab::L1 * n + k];
  const double* Qsc = a.Qs + (size_t)c * 5 * nd;
  const double sc = dt / h;
  double qn[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double* Gv = sG + v * nn;
    const double lx = L1i * Gv[5 * nn + k * n + j] - L0i * Gv[k * n + j];
    const double ly = L1j * Gv[15 * nn + k * n + i] - L0j * Gv[10 * nn + k * n + i];
    const double lz = L1k * Gv[25 * nn + j * n + i] - L0k * Gv[20 * nn + j * n + i];
    qn[v] = Qsc[v * nd + r] - sc * (lx + ly + lz);
  }
  if (valid) {
    double* Qo = a.Qout + (size_t)c * 5 * nd;
#pragma unroll
    for (int v = 0; v < 5; ++v) Qo[v * nd + r] = qn[v];
    // CFL candidate: max over the nodes of max(|u|,|v|,|w|) + c and of
    // lambda_v (non-negative doubles order like their bit patterns)
    const double z = zc + h * a.gtab[GTab::XI * n + k];
    const double ir = 1.0 / qn[0];
    const double p = pressure3(ph, qn, z);
    const double lam = fmax(fabs(qn[1]), fmax(fabs(qn[2]), fabs(qn[3]))) * ir + sqrt(ph.gamma * p * ir);
    const double lv = ph.lv_coef * ir;
    atomicMax(&smax[0], (unsigned long long)__double_as_longlong(lam));
    atomicMax(&smax[1], (unsigned long long)__double_as_longlong(lv));
  }
  sync3<WL>();
  if (valid && r == 0) {
    const double lam = __longlong_as_double((long long)smax[0]), lv = __longlong_as_double((long long)smax[1]);
    const double o = 2.0 * ph.N + 1.0;
    a.dtc[c] = ph.cfl * h / (3.0 * o * (lam + 2.0 * lv * o / h));
  }
}

// CFL candidate of every cell from the current state
template <int n>
__global__ __launch_bounds__(kThreads3) void k_dt3(Phys ph, Args3 a) {
  using G = Cfg3<n>;
  constexpr int nn = G::nn, nd = G::nd;
  __shared__ unsigned long long smax[G::CB][2];
  const int tid = threadIdx.x, slot = tid / nd, r = tid - slot * nd;
  const bool inslot = !G::spare || slot < G::CB;
  const int cell = blockIdx.x * G::CB + slot;
  const bool valid = inslot && cell < a.C;
  if (inslot && r == 0) { smax[slot][0] = 0ull; smax[slot][1] = 0ull; }
  sync3<G::WL>();
  if (valid) {
    const int ck = cell / (a.nx * a.ny), k = r / nn;
    const double* Qc = a.Q + (size_t)cell * 5 * nd;
    double q[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = Qc[v * nd + r];
    const double z = (a.z0 + ck * a.h) + a.h * a.gtab[GTab::XI * n + k];
    const double ir = 1.0 / q[0];
    const double p = pressure3(ph, q, z);
    const double lam = fmax(fabs(q[1]), fmax(fabs(q[2]), fabs(q[3]))) * ir + sqrt(ph.gamma * p * ir);
    atomicMax(&smax[slot][0], (unsigned long long)__double_as_longlong(lam));
    atomicMax(&smax[slot][1], (unsigned long long)__double_as_longlong(ph.lv_coef * ir));
  }
  sync3<G::WL>();
  if (valid && r == 0) {
    const double lam = __longlong_as_double((long long)smax[slot][0]);
    const double lv = __longlong_as_double((long long)smax[slot][1]);
    const double o = 2.0 * ph.N + 1.0;
    a.dtc[cell] = ph.cfl * a.h / (3.0 * o * (lam + 2.0 * lv * o / a.h));
  }
}

// ----------------------------------------------------------- initial states
// kind 0: hydrostatic background of constant potential temperature perturbed
// in theta at fixed pressure by the bubbles (eqs. cos-pertubation,
// bubbles-pertubation, with the distance in three dimensions), at rest;
// kind 1: the ABC flow (eq. abc-flow) at time t0
__global__ void k_init3(Phys ph, Args3 a, int n, int kind, Bubbles3 B, double t0, double* Q) {
  const int nd = n * n * n;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)a.C * nd) return;
  const int c = (int)(gid / nd), r = (int)(gid % nd);
  const int i = r % n, j = (r / n) % n, k = r / (n * n);
  const int ci = c % a.nx, cj = (c / a.nx) % a.ny, ck = c / (a.nx * a.ny);
  const double* xi = a.gtab + GTab::XI * n;
  const double x = a.x0 + a.h * (ci + xi[i]), y = a.y0 + a.h * (cj + xi[j]), z = a.z0 + a.h * (ck + xi[k]);
  double q[5];
  if (kind == 0) {
    double th = 0.0;
    for (int b = 0; b < B.nb; ++b) {
      const double* bb = B.b + 7 * b;
      const double dx = x - bb[4], dy = y - bb[5], dz = z - bb[6];
      const double rr = sqrt(dx * dx + dy * dy + dz * dz);
      if (bb[0] == 0.0) th += rr <= bb[2] ? 0.5 * bb[1] * (1.0 + cos(M_PI * rr / bb[2])) : 0.0;
      else th += rr <= bb[2] ? bb[1] : bb[1] * exp(-(rr - bb[2]) * (rr - bb[2]) / (bb[3] * bb[3]));
    }
    const double pi = 1.0 - ph.g * z / (ph.cp * ph.theta);
    const double pbg = ph.p0 * pow(pi, ph.cp_over_R);
    const double rho = pbg / (ph.R * (ph.theta + th) * pi);
    q[0] = rho; q[1] = 0.0; q[2] = 0.0; q[3] = 0.0;
    q[4] = pbg / ph.gm1 + rho * ph.g * z;
  } else {
    const double e1 = exp(-ph.mu * t0), e2 = exp(-2.0 * ph.mu * t0);
    const double u = e1 * (sin(z) + cos(y)), v = e1 * (sin(x) + cos(z)), w = e1 * (sin(y) + cos(x));
    const double p = 100.0 / ph.gamma - e2 * (cos(x) * sin(y) + sin(x) * cos(z) + sin(z) * cos(y));
    q[0] = 1.0; q[1] = u; q[2] = v; q[3] = w;
    q[4] = p / ph.gm1 + 0.5 * (u * u + v * v + w * w);
  }
  double* Qc = Q + (size_t)c * 5 * nd;
  for (int v = 0; v < 5; ++v) Qc[v * nd + r] = q[v];
}

// flag non-finite values and non-positive density or pressure
__global__ void k_health3(Phys ph, Args3 a, int n, int* flag) {
  const int nd = n * n * n;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)a.C * nd) return;
  const int c = (int)(gid / nd), r = (int)(gid % nd);
  const int ck = c / (a.nx * a.ny);
  const double* Qc = a.Q + (size_t)c * 5 * nd;
  double q[5];
  bool bad = false;
  for (int v = 0; v < 5; ++v) { q[v] = Qc[v * nd + r]; bad = bad || !isfinite(q[v]); }
  bad = bad || !(q[0] > 0.0);
  if (!bad) bad = !(pressure3(ph, q, (a.z0 + ck * a.h) + a.h * a.gtab[GTab::XI * n + r / (n * n)]) > 0.0);
  if (bad) atomicOr(flag, 1);
}

// --------------------------------------------------------------- launchers
template <int n>
static int pred3_n(const Phys& ph, const HostBasis& B, const Args3& a, hipStream_t s) {
  using G = Cfg3<n>;
  const int blocks = (a.C + G::CB - 1) / G::CB;
  const size_t lds = sizeof(double) * (size_t)G::CB * G::pred_slot;
  if constexpr (n == 4)
    hipLaunchKernelGGL(k_pred3_w64, dim3(blocks), dim3(kThreads3), lds, s, ph, tab_of<n>(B), a);
  else
    hipLaunchKernelGGL(k_pred3<n>, dim3(blocks), dim3(kThreads3), lds, s, ph, tab_of<n>(B), a);
  return check_launch("predictor3");
}
template <int n>
static int corr3_n(const Phys& ph, const Args3& a, hipStream_t s) {
  using G = Cfg3<n>;
  const int blocks = (a.C + G::CB - 1) / G::CB;
  const size_t lds = sizeof(double) * (size_t)G::CB * G::corr_slot;
  hipLaunchKernelGGL(k_corr3<n>, dim3(blocks), dim3(kThreads3), lds, s, ph, a);
  return check_launch("corrector3");
}
template <int n>
static int dt3_n(const Phys& ph, const Args3& a, hipStream_t s) {
  using G = Cfg3<n>;
  const int blocks = (a.C + G::CB - 1) / G::CB;
  hipLaunchKernelGGL(k_dt3<n>, dim3(blocks), dim3(kThreads3), 0, s, ph, a);
  return check_launch("cell_dt3");
}

#define ADG3_DISPATCH(fn, n, ...)                                        \
  switch (n) {                                                           \
    case 2: return fn<2>(__VA_ARGS__);                                   \
    case 3: return fn<3>(__VA_ARGS__);                                   \
    case 4: return fn<4>(__VA_ARGS__);                                   \
    case 5: return fn<5>(__VA_ARGS__);                                   \
    case 6: return fn<6>(__VA_ARGS__);                                   \
    default: return fail(ADG_EUNSUPPORTED, "order not supported in 3D"); \
  }

int launch_pred3(const Phys& ph, const HostBasis& B, const Args3& a, hipStream_t s) {
  if (a.C == 0) return ADG_OK;
  ADG3_DISPATCH(pred3_n, B.n, ph, B, a, s);
}
int launch_corr3(const Phys& ph, int n, const Args3& a, hipStream_t s) {
  if (a.C == 0) return ADG_OK;
  ADG3_DISPATCH(corr3_n, n, ph, a, s);
}
int launch_dt3(const Phys& ph, int n, const Args3& a, hipStream_t s) {
  if (a.C == 0) return ADG_OK;
  ADG3_DISPATCH(dt3_n, n, ph, a, s);
}
int launch_init3(const Phys& ph, int n, const Args3& a, int kind, const Bubbles3& B, double t0, double* Q,
                 hipStream_t s) {
  const long long tot = (long long)a.C * n * n * n;
  if (tot == 0) return ADG_OK;
  hipLaunchKernelGGL(k_init3, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ph, a, n, kind, B, t0, Q);
  return check_launch("init_state3");
}
int launch_health3(const Phys& ph, int n, const Args3& a, int* flag, hipStream_t s) {
  const long long tot = (long long)a.C * n * n * n;
  if (tot == 0) return ADG_OK;
  hipLaunchKernelGGL(k_health3, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ph, a, n, flag);
  return check_launch("health3");
}

}  // namespace adg
