// ADER-DG step kernels for gfx950: space-time predictor, corrector with the
// viscous Rusanov face flux, CFL time step.
//
// Work decomposition: one 64-lane wavefront per cell (n*n <= 64 spatial
// nodes).  Lane l < n*n owns spatial node (j, i) = (l / n, l % n) and keeps
// the whole time history of its node in registers; tensor-product
// contractions along x and z run as "line jobs" (one lane per (direction,
// variable, line), 8n jobs) through LDS slices of the current time level.
#include "adg_internal.h"

namespace adg {

template <int n>
struct LineJob {
  int dir, base, stride;
  bool active;
  __device__ LineJob(int lane) {
    constexpr int nn = n * n;
    active = lane < 8 * n;
    dir = lane / (4 * n);
    int v = (lane % (4 * n)) / n;
    int line = lane % n;
    base = v * nn + (dir == 0 ? line * n : line);
    stride = dir == 0 ? 1 : n;
  }
};

// Half tables: for Gauss-Legendre nodes (symmetric about 1/2) the derivative
// matrix is centro-antisymmetric, D[n-1-i][n-1-m] = -D[i][m], and so is the
// volume matrix Dw.  Only the first nh = ceil(n/2) rows are kept; row n-1-i is
// applied as minus row i on the reversed input line.
template <int n>
struct Half { static constexpr int nh = (n + 1) / 2; };

// out[i] = sum_m M[i][m] in[m] along this lane's line: src -> dst.  M holds
// the first nh rows in VGPRs (uniform values, loaded once per kernel).
template <int n>
__device__ inline void line_apply(const double (&M)[Half<n>::nh][n], const LineJob<n>& J, const double* src,
                                  double* dst) {
  constexpr int nh = Half<n>::nh;
  double in[n];
#pragma unroll
  for (int m = 0; m < n; ++m) in[m] = src[J.base + m * J.stride];
#pragma unroll
  for (int i = 0; i < nh; ++i) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) s = fma(M[i][m], in[m], s);
    dst[J.base + i * J.stride] = s;
  }
#pragma unroll
  for (int i = 0; i < n / 2; ++i) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) s = fma(M[i][m], in[n - 1 - m], s);
    dst[J.base + (n - 1 - i) * J.stride] = -s;
  }
}

// Load the first nh rows of an n x n table into VGPRs.  The empty asm marks
// every value as lane-varying, so the compiler keeps the table in vector
// registers instead of scalar registers (which cannot hold it and would
// spill into lanes).
template <int n>
__device__ inline void load_vtab(const double* g, double (&M)[Half<n>::nh][n]) {
#pragma unroll
  for (int i = 0; i < Half<n>::nh; ++i)
#pragma unroll
    for (int m = 0; m < n; ++m) {
      M[i][m] = g[i * n + m];
      asm volatile("" : "+v"(M[i][m]));
    }
}

struct StepArgs {
  const double* Qin;    // [C][4][n][n]
  double* Qout;         // corrector output (may alias Qin)
  double* Qs;           // [C][4][n][n]  Q* = Q^n + dt (volume + source)
  double* FD;           // [C][4 faces][2][4][n]
  double* dtc;          // [C] per-cell CFL candidates
  double* clock;        // t, dt, (unused), steps
  const double* geom;   // [C][4]
  const int* nbr;       // [C][4][4]
  const double* gtab;
  int C, iters;
  int* health;
};

// ------------------------------------------------------------------ predictor
// Per cell (one wavefront): the Picard iterate of all n time nodes lives in
// LDS (sq[b][v][j][i]).  Each sweep walks the time nodes in a runtime loop
// that is software-pipelined by one node: a line phase computes the
// divergence of the fluxes of node b and the gradients of node b+1, a node
// phase forms the residual R(b) (rank-1 update acc[a] += P[a][b] R(b), kept
// per node in registers) and the fluxes of node b+1.  Two barriers per node.

// flux and source of time node b at this lane's node: q from the iterate,
// gradients from sg; fluxes to sf
template <int n>
__device__ inline double node_flux(const Phys& ph, const double* qb, const double (*sg)[4 * n * n],
                                   double (*sf)[4 * n * n], int lane, double ih, double z, double rb, double pb,
                                   double q[4], double Fx[4], double Fz[4]) {
  constexpr int nn = n * n;
  double gx[4], gz[4], Sw;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    q[v] = qb[v * nn + lane];
    gx[v] = sg[0][v * nn + lane] * ih;
    gz[v] = sg[1][v * nn + lane] * ih;
  }
  flux_source(ph, q, gx, gz, z, rb, pb, Fx, Fz, Sw);
#pragma unroll
  for (int v = 0; v < 4; ++v) { sf[0][v * nn + lane] = Fx[v]; sf[1][v * nn + lane] = Fz[v]; }
  return Sw;
}

template <int n>
__global__ __launch_bounds__(kWave) void k_predictor(Phys ph, StepArgs a) {
  constexpr int nn = n * n, sl = 4 * nn;
  __shared__ double sq[n * sl];     // iterate at all time nodes; slot b takes R(b) once consumed
  __shared__ double sg[2][sl];      // gradients (x, z) of the next time node
  __shared__ double sf[2][sl];      // fluxes (x, z) of the current node, then their divergence

  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const bool node = lane < nn;
  const int ln = node ? lane : 0;
  const int jz = ln / n, ix = ln % n;
  const LineJob<n> J(lane);
  const double* gt = a.gtab;

  const double t0 = a.clock[0], dt = a.clock[1];
  const double x0 = a.geom[4 * c + 0], z0 = a.geom[4 * c + 1], h = a.geom[4 * c + 2];
  const double ih = 1.0 / h;
  const double x = x0 + h * gt[GTab::XI * n + ix];
  const double z = z0 + h * gt[GTab::XI * n + jz];
  double rb, pb;
  background(ph, z, rb, pb);

  double Dv[Half<n>::nh][n];
  load_vtab<n>(gt + GTab::d(n), Dv);

  const double* Qc = a.Qin + (size_t)c * sl;
  double Qn[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) Qn[v] = Qc[v * nn + ln];
  if (node) {
#pragma unroll
    for (int b = 0; b < n; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) sq[b * sl + v * nn + lane] = Qn[v];
  }
  __syncthreads();

  for (int it = 0; it < a.iters; ++it) {
    double acc[n][4];
#pragma unroll
    for (int b = 0; b < n; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[b][v] = 0.0;
#pragma unroll 1
    for (int b = 0; b < n; ++b) {
      double* qb = sq + b * sl;
      if (J.active) line_apply<n>(Dv, J, qb, sg[J.dir]);
      __syncthreads();
      double Sw = 0.0;
      if (node) {
        double q[4], Fx[4], Fz[4];
        Sw = node_flux<n>(ph, qb, sg, sf, lane, ih, z, rb, pb, q, Fx, Fz);
      }
      __syncthreads();
      if (J.active) line_apply<n>(Dv, J, sf[J.dir], sf[J.dir]);
      __syncthreads();
      if (node) {
        double R[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) R[v] = -(sf[0][v * nn + lane] + sf[1][v * nn + lane]) * ih;
        R[2] += Sw;
        if (ph.mms) R[3] += mms_source(ph, x, z, t0 + gt[GTab::XI * n + b] * dt);
        const double* pc = gt + GTab::pt(n) + b * n;
#pragma unroll
        for (int a2 = 0; a2 < n; ++a2) {
          const double p = pc[a2];
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[a2][v] = fma(p, R[v], acc[a2][v]);
        }
      }
      __syncthreads();
    }
    if (node) {
#pragma unroll
      for (int b = 0; b < n; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) sq[b * sl + v * nn + lane] = fma(dt, acc[b][v], Qn[v]);
    }
    __syncthreads();
  }

  // time averages of q, F and S on the last iterate
  double Qb[4] = {0, 0, 0, 0}, Fbx[4] = {0, 0, 0, 0}, Fbz[4] = {0, 0, 0, 0}, Sbw = 0.0, SbE = 0.0;
#pragma unroll 1
  for (int b = 0; b < n; ++b) {
    const double* qb = sq + b * sl;
    if (J.active) line_apply<n>(Dv, J, qb, sg[J.dir]);
    __syncthreads();
    if (node) {
      double q[4], Fx[4], Fz[4];
      const double Sw = node_flux<n>(ph, qb, sg, sf, lane, ih, z, rb, pb, q, Fx, Fz);
      const double wb = gt[GTab::W * n + b];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Qb[v] = fma(wb, q[v], Qb[v]);
        Fbx[v] = fma(wb, Fx[v], Fbx[v]);
        Fbz[v] = fma(wb, Fz[v], Fbz[v]);
      }
      Sbw = fma(wb, Sw, Sbw);
      if (ph.mms) SbE = fma(wb, mms_source(ph, x, z, t0 + gt[GTab::XI * n + b] * dt), SbE);
    }
    __syncthreads();
  }

  // volume term and face data
  if (node) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sq[v * nn + lane] = Qb[v];
      sf[0][v * nn + lane] = Fbx[v];
      sf[1][v * nn + lane] = Fbz[v];
    }
  }
  __syncthreads();
  if (J.active) {
    // Dw contraction of the averaged flux along the line; extrapolation of the
    // averaged state and flux to both ends of the line.
    double Wv[Half<n>::nh][n];
    load_vtab<n>(gt + GTab::dw(n), Wv);
    const double* src = sf[J.dir];
    line_apply<n>(Wv, J, src, sg[J.dir]);
    double inF[n], inQ[n];
#pragma unroll
    for (int m = 0; m < n; ++m) { inF[m] = src[J.base + m * J.stride]; inQ[m] = sq[J.base + m * J.stride]; }
    double q0 = 0, q1 = 0, f0 = 0, f1 = 0;
#pragma unroll
    for (int m = 0; m < n; ++m) {
      const double e0 = gt[GTab::E0 * n + m], e1 = gt[GTab::E1 * n + m];
      q0 = fma(e0, inQ[m], q0); q1 = fma(e1, inQ[m], q1);
      f0 = fma(e0, inF[m], f0); f1 = fma(e1, inF[m], f1);
    }
    const int v = (lane % (4 * n)) / n, line = lane % n;
    double* fd = a.FD + (size_t)c * 32 * n;
    const int fl = 2 * J.dir, fu = 2 * J.dir + 1;
    fd[((fl * 2 + 0) * 4 + v) * n + line] = q0;
    fd[((fl * 2 + 1) * 4 + v) * n + line] = f0;
    fd[((fu * 2 + 0) * 4 + v) * n + line] = q1;
    fd[((fu * 2 + 1) * 4 + v) * n + line] = f1;
  }
  __syncthreads();
  if (node) {
    double* qs = a.Qs + (size_t)c * sl;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double S = (v == 2) ? Sbw : (v == 3 ? SbE : 0.0);
      qs[v * nn + lane] = Qn[v] + dt * ((sg[0][v * nn + lane] + sg[1][v * nn + lane]) * ih + S);
    }
  }
}

// ------------------------------------------------------------------ corrector
// Ghost state and flux at a no-slip wall: mirrored velocity, background
// density and pressure (interior ones without gravity), mass flux mirrored,
// momentum flux copied, energy flux 2 q_bg - F with the background
// conductive flux q_bg = kappa g / cp through horizontal walls.
__device__ inline void wall_ghost(const Phys& ph, int d, double zf, const double Qi[4], const double Fi[4],
                                  double Qg[4], double Fg[4]) {
  const double u = Qi[1] / Qi[0], w = Qi[2] / Qi[0];
  double rb, pb;
  if (ph.gravity) background(ph, zf, rb, pb);
  else { rb = Qi[0]; pb = pressure(ph, Qi[0], Qi[1], Qi[2], Qi[3], zf); }
  const double geo = ph.gravity ? rb * (ph.g * zf) : 0.0;
  Qg[0] = rb;
  Qg[1] = -(rb * u);
  Qg[2] = -(rb * w);
  Qg[3] = pb / ph.gm1 + 0.5 * rb * (u * u + w * w) + geo;
  const double qbg = (ph.gravity && d == 1) ? ph.kappa * ph.g / ph.cp : 0.0;
  Fg[0] = -Fi[0];
  Fg[1] = Fi[1];
  Fg[2] = Fi[2];
  Fg[3] = 2.0 * qbg - Fi[3];
}

__device__ inline void eig(const Phys& ph, int d, const double q[4], double zf, double& lam, double& lv) {
  const double ir = 1.0 / q[0];
  const double p = pressure(ph, q[0], q[1], q[2], q[3], zf);
  lam = fabs(q[1 + d] * ir) + sqrt(ph.gamma * p * ir);
  lv = ph.lv_coef * ir;
}

template <int n>
__global__ __launch_bounds__(kWave) void k_corrector(Tab<n> T, Phys ph, StepArgs a) {
  constexpr int nn = n * n;
  __shared__ double sG[4][4][n];
  __shared__ double sL[4][n], sV[4][n];
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const double dt = a.clock[1];
  const double x0 = a.geom[4 * c + 0], z0 = a.geom[4 * c + 1], h = a.geom[4 * c + 2];
  (void)x0;
  const bool fl = lane < 4 * n;
  const int f = fl ? lane / n : 0, k = lane % n;
  const int d = f >> 1;
  const bool lower = (f & 1) == 0;   // face on the lower side: this cell is R
  double Qm[4], Fm[4], Qo[4], Fo[4];
  double zf = 0.0;
  if (fl) {
    const double* fd = a.FD + (size_t)c * 32 * n + f * 8 * n;
#pragma unroll
    for (int v = 0; v < 4; ++v) { Qm[v] = fd[v * n + k]; Fm[v] = fd[4 * n + v * n + k]; }
    zf = (d == 0) ? z0 + h * a.gtab[GTab::XI * n + k] : z0 + ((f & 1) ? h : 0.0);
    const int* nb = a.nbr + (size_t)c * 16 + f * 4;
    const int kind = nb[0];
    if (kind == kConforming) {
      const double* fo = a.FD + (size_t)nb[1] * 32 * n + (f ^ 1) * 8 * n;
#pragma unroll
      for (int v = 0; v < 4; ++v) { Qo[v] = fo[v * n + k]; Fo[v] = fo[4 * n + v * n + k]; }
    } else {
      wall_ghost(ph, d, zf, Qm, Fm, Qo, Fo);
    }
    double l1, v1, l2, v2;
    eig(ph, d, Qm, zf, l1, v1);
    eig(ph, d, Qo, zf, l2, v2);
    sL[f][k] = fmax(l1, l2);
    sV[f][k] = fmax(v1, v2);
  }
  __syncthreads();
  if (fl) {
    double lam = sL[f][0], lv = sV[f][0];
#pragma unroll
    for (int m = 1; m < n; ++m) { lam = fmax(lam, sL[f][m]); lv = fmax(lv, sV[f][m]); }
    const double eta = (2.0 * ph.N + 1.0) / (h * 1.2533141373155002512);  // h sqrt(pi/2)
    const double s = lam + 2.0 * eta * lv;
    const double* QL = lower ? Qo : Qm;
    const double* FL = lower ? Fo : Fm;
    const double* QR = lower ? Qm : Qo;
    const double* FR = lower ? Fm : Fo;
#pragma unroll
    for (int v = 0; v < 4; ++v) sG[f][v][k] = 0.5 * (FL[v] + FR[v]) - 0.5 * s * (QR[v] - QL[v]);
  }
  __syncthreads();
  const bool node = lane < nn;
  const int ln = node ? lane : 0;
  const int jz = ln / n, ix = ln % n;
  double lam = 0.0, lvm = 0.0;
  if (node) {
    const double L0i = a.gtab[GTab::L0 * n + ix], L1i = a.gtab[GTab::L1 * n + ix];
    const double L0j = a.gtab[GTab::L0 * n + jz], L1j = a.gtab[GTab::L1 * n + jz];
    const double* qs = a.Qs + (size_t)c * 4 * nn;
    double* qo = a.Qout + (size_t)c * 4 * nn;
    const double sc = dt / h;
    double q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double sx = L1i * sG[1][v][jz] - L0i * sG[0][v][jz];
      const double sz = L1j * sG[3][v][ix] - L0j * sG[2][v][ix];
      q[v] = qs[v * nn + lane] - sc * (sx + sz);
      qo[v * nn + lane] = q[v];
    }
    if (!ph.fixed_dt) {
      const double z = z0 + h * a.gtab[GTab::XI * n + jz];
      double l0, lv0, l1, lv1;
      eig(ph, 0, q, z, l0, lv0);
      eig(ph, 1, q, z, l1, lv1);
      lam = fmax(l0, l1);
      lvm = lv0;
    }
  }
  if (!ph.fixed_dt) {
    lam = wave_max(lam);
    lvm = wave_max(lvm);
    if (lane == 0) {
      const double o = 2.0 * ph.N + 1.0;
      a.dtc[c] = ph.cfl * h / (2.0 * o * (lam + 2.0 * lvm * o / h));
    }
  }
}

// per-cell CFL candidate from the current state (no update)
template <int n>
__global__ __launch_bounds__(kWave) void k_cell_dt(Phys ph, StepArgs a) {
  constexpr int nn = n * n;
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const double z0 = a.geom[4 * c + 1], h = a.geom[4 * c + 2];
  double lam = 0.0, lvm = 0.0;
  if (lane < nn) {
    const int jz = lane / n;
    const double* Qc = a.Qin + (size_t)c * 4 * nn;
    double q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = Qc[v * nn + lane];
    const double z = z0 + h * a.gtab[GTab::XI * n + jz];
    double l0, lv0, l1, lv1;
    eig(ph, 0, q, z, l0, lv0);
    eig(ph, 1, q, z, l1, lv1);
    lam = fmax(l0, l1);
    lvm = lv0;
  }
  lam = wave_max(lam);
  lvm = wave_max(lvm);
  if (lane == 0) {
    const double o = 2.0 * ph.N + 1.0;
    a.dtc[c] = ph.cfl * h / (2.0 * o * (lam + 2.0 * lvm * o / h));
  }
}

// Clock update by one workgroup: if advance, t += dt and steps += 1; if
// update, dt <- min over cells of the CFL candidates (a fixed reduction tree:
// min is exact, so the result does not depend on the order anyway).
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_clock(double* clock, const double* dtc, int C, int advance,
                                                           int update) {
  __shared__ double sm[kReduceThreads / kWave];
  const int t = threadIdx.x;
  double m = __builtin_inf();
  if (update)
    for (int c = t; c < C; c += kReduceThreads) m = fmin(m, dtc[c]);
  #pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmin(m, __shfl_xor(m, o, kWave));
  if ((t & (kWave - 1)) == 0) sm[t / kWave] = m;
  __syncthreads();
  if (t == 0) {
    double r = sm[0];
    for (int k = 1; k < kReduceThreads / kWave; ++k) r = fmin(r, sm[k]);
    if (advance) { clock[0] += clock[1]; clock[3] += 1.0; }
    if (update) clock[1] = r;
  }
}

// --------------------------------------------------------------- dispatchers
template <int n>
static Tab<n> make_tab(const adg_mesh* m) {
  Tab<n> T;
  for (int i = 0; i < n; ++i) {
    T.w[i] = m->w[i]; T.e0[i] = m->e0[i]; T.e1[i] = m->e1[i];
    for (int j = 0; j < n; ++j) {
      T.D[i][j] = m->D[i * n + j];
      T.P[i][j] = m->P[i * n + j];
      T.Dw[i][j] = m->Dw[i * n + j];
    }
  }
  return T;
}

StepArgs make_args(adg_mesh* m) {
  StepArgs a;
  char* ws = static_cast<char*>(m->ws);
  a.Qin = m->Q; a.Qout = m->Q;
  a.Qs = reinterpret_cast<double*>(ws + m->off_qs);
  a.FD = reinterpret_cast<double*>(ws + m->off_fd);
  a.dtc = reinterpret_cast<double*>(ws + m->off_dtc);
  a.health = reinterpret_cast<int*>(ws + m->off_health);
  a.clock = m->clock; a.geom = m->d_geom; a.nbr = m->d_nbr; a.gtab = m->d_gtab;
  a.C = m->C; a.iters = m->iters;
  return a;
}

template <int n>
static int launch_predictor_n(adg_mesh* m, hipStream_t s) {
  StepArgs a = make_args(m);
  hipLaunchKernelGGL(k_predictor<n>, dim3(m->C), dim3(kWave), 0, s, m->ph, a);
  return check_launch("predictor");
}
template <int n>
static int launch_corrector_n(adg_mesh* m, hipStream_t s) {
  StepArgs a = make_args(m);
  hipLaunchKernelGGL(k_corrector<n>, dim3(m->C), dim3(kWave), 0, s, make_tab<n>(m), m->ph, a);
  int rc = check_launch("corrector");
  if (rc) return rc;
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(kReduceThreads), 0, s, m->clock, a.dtc, m->C, 1,
                     m->ph.fixed_dt ? 0 : 1);
  return check_launch("clock");
}
template <int n>
static int launch_dt_n(adg_mesh* m, hipStream_t s) {
  StepArgs a = make_args(m);
  hipLaunchKernelGGL(k_cell_dt<n>, dim3(m->C), dim3(kWave), 0, s, m->ph, a);
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(kReduceThreads), 0, s, m->clock, a.dtc, m->C, 0, 1);
  return check_launch("compute_dt");
}

#define ADG_DISPATCH(fn, m, s)                         \
  switch ((m)->n) {                                    \
    case 2: return fn<2>(m, s);                        \
    case 3: return fn<3>(m, s);                        \
    case 4: return fn<4>(m, s);                        \
    case 5: return fn<5>(m, s);                        \
    case 6: return fn<6>(m, s);                        \
    case 7: return fn<7>(m, s);                        \
    case 8: return fn<8>(m, s);                        \
    default: return fail(ADG_EUNSUPPORTED, "order not supported"); \
  }

int launch_predictor(adg_mesh* m, hipStream_t s) { ADG_DISPATCH(launch_predictor_n, m, s); }
int launch_corrector(adg_mesh* m, hipStream_t s) { ADG_DISPATCH(launch_corrector_n, m, s); }
int launch_dt(adg_mesh* m, hipStream_t s) { ADG_DISPATCH(launch_dt_n, m, s); }

}  // namespace adg
