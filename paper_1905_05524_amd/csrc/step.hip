// ADER-DG step kernels for gfx950: space-time predictor, corrector with the
// viscous Rusanov face flux (conforming, wall and 1:3 non-conforming faces),
// CFL time step.
//
// Work decomposition.  A wavefront (64 lanes) owns CPW cells (CPW * n*n <=
// 64); a workgroup holds WPB independent wavefronts, each with its own LDS
// region, synchronised at wavefront level only.  In a cell, lane (slot, l)
// with l < n*n owns spatial node (j, i) = (l / n, l % n); tensor-product
// contractions along x and z run as "line jobs" (one lane per (direction,
// variable, line), 8n jobs per cell) on LDS slices of one time level.
// CPW and WPB are template parameters picked per order by the autotuner.
#include "adg_internal.h"

namespace adg {

// wavefront-scope barrier for LDS hand-offs between lanes of one wavefront:
// LDS operations of a wavefront execute in order, so a compiler fence and a
// wave barrier are enough.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int n>
struct Half { static constexpr int nh = (n + 1) / 2; };

template <int n, int CPW>
struct Lay {
  static constexpr int nn = n * n, sl = 4 * nn;
  static constexpr int jobs = 8 * n * CPW;                 // line jobs per wavefront
  static constexpr int rounds = (jobs + kWave - 1) / kWave;
  static constexpr int pred_cell = (n + 4) * sl;           // predictor LDS doubles per cell
  static constexpr int corr_cell = 16 * n + 24 * n + 48 * n;  // sG, sL/sV, sGs
};

// Line job of one lane in one round: direction, base offset and stride in a
// [4][n][n] slice, cell slot.
template <int n>
struct LineJob {
  int dir, base, stride, slot, v, line;
  bool active;
  __device__ LineJob(int job, int cpw) {
    constexpr int nn = n * n;
    slot = job / (8 * n);
    active = slot < cpw;
    const int jj = job % (8 * n);
    dir = jj / (4 * n);
    v = (jj % (4 * n)) / n;
    line = jj % n;
    base = v * nn + (dir == 0 ? line * n : line);
    stride = dir == 0 ? 1 : n;
  }
};

// Half tables: for Gauss-Legendre nodes (symmetric about 1/2) the derivative
// matrix is centro-antisymmetric, D[n-1-i][n-1-m] = -D[i][m], and so is the
// volume matrix Dw.  Only the first nh = ceil(n/2) rows are kept; row n-1-i is
// applied as minus row i on the reversed input line.
template <int n>
__device__ inline void line_apply(const double (&M)[Half<n>::nh][n], int base, int stride, const double* src,
                                  double* dst) {
  constexpr int nh = Half<n>::nh;
  double in[n];
#pragma unroll
  for (int m = 0; m < n; ++m) in[m] = src[base + m * stride];
#pragma unroll
  for (int i = 0; i < nh; ++i) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) s = fma(M[i][m], in[m], s);
    dst[base + i * stride] = s;
  }
#pragma unroll
  for (int i = 0; i < n / 2; ++i) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) s = fma(M[i][m], in[n - 1 - m], s);
    dst[base + (n - 1 - i) * stride] = -s;
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
  double* clock;        // [S][4]: t, dt, (unused), steps
  const int* scen;      // [C] scenario of each cell (NULL: scenario 0)
  const double* geom;   // [C][4]
  const int* nbr;       // [C][4][4]
  const double* gtab;
  double* iter_store;   // optional [C][iters][n][4][n][n]: Picard iterates q^1..q^I (adjoint)
  int C, iters;
};

// ------------------------------------------------------------------ predictor
// flux and source of one time node at this lane's node: q from the iterate
// slice qb, gradients from sg; fluxes to sf
template <int n>
__device__ inline double node_flux(const Phys& ph, const double* qb, const double* sg, double* sf, int l,
                                   double ih, double z, double rb, double pb, double q[4], double Fx[4],
                                   double Fz[4]) {
  constexpr int nn = n * n, sl = 4 * nn;
  double gx[4], gz[4], Sw;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    q[v] = qb[v * nn + l];
    gx[v] = sg[v * nn + l] * ih;
    gz[v] = sg[sl + v * nn + l] * ih;
  }
  flux_source(ph, q, gx, gz, z, rb, pb, Fx, Fz, Sw);
#pragma unroll
  for (int v = 0; v < 4; ++v) { sf[v * nn + l] = Fx[v]; sf[sl + v * nn + l] = Fz[v]; }
  return Sw;
}

// Per cell: the Picard iterate of all n time nodes lives in LDS
// (sq[b][v][j][i]); each sweep walks the time nodes b in a runtime loop:
// gradients by line jobs, flux and source per node, divergence by line jobs
// (in place), and the rank-1 update acc[a] += P[a][b] R(b) held per node in
// registers.  Then time averages, the volume term and the face data.
template <int n, int CPW, int WPB>
__global__ __launch_bounds__(kWave * WPB) void k_predictor(Phys ph, StepArgs a) {
  using L = Lay<n, CPW>;
  constexpr int nn = L::nn, sl = L::sl;
  extern __shared__ double lds[];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  double* wl = lds + (size_t)wave * CPW * L::pred_cell;
  const int cell0 = (blockIdx.x * WPB + wave) * CPW;

  // node role
  const int slot = lane / nn, l = lane % nn;
  const bool node = slot < CPW;
  const int c = cell0 + (node ? slot : 0);
  const bool valid = node && c < a.C;
  const int cc = valid ? c : 0;
  double* sq = wl + (node ? slot : 0) * L::pred_cell;
  double* sg = sq + n * sl;
  double* sf = sg + 2 * sl;
  const int jz = l / n, ix = l % n;
  const double* gt = a.gtab;

  const int s = a.scen ? a.scen[cc] : 0;
  const double t0 = a.clock[4 * s + 0], dt = a.clock[4 * s + 1];
  const double x0 = a.geom[4 * cc + 0], z0 = a.geom[4 * cc + 1], h = a.geom[4 * cc + 2];
  const double ih = 1.0 / h;
  const double x = x0 + h * gt[GTab::XI * n + ix];
  const double z = z0 + h * gt[GTab::XI * n + jz];
  double rb, pb;
  background(ph, z, rb, pb);

  double Dv[Half<n>::nh][n];
  load_vtab<n>(gt + GTab::d(n), Dv);

  double Qn[4];
  {
    const double* Qc = a.Qin + (size_t)cc * sl;
#pragma unroll
    for (int v = 0; v < 4; ++v) Qn[v] = valid ? Qc[v * nn + l] : (v == 0 || v == 3 ? 1.0 : 0.0);
  }
  if (node) {
#pragma unroll
    for (int b = 0; b < n; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) sq[b * sl + v * nn + l] = Qn[v];
  }
  wave_sync();

  // line-job roles (rounds of 64 jobs)
  const LineJob<n> J0(lane, CPW), J1(lane + kWave, CPW);
  double* jl0 = wl + (J0.active ? J0.slot : 0) * L::pred_cell;
  double* jl1 = wl + (J1.active ? J1.slot : 0) * L::pred_cell;
  // src/dst are offsets in a cell's region; direction d adds d * (dir stride)
  auto lines = [&](int src_off, int dst_off, int src_dir_stride, int dst_dir_stride) {
    if (J0.active)
      line_apply<n>(Dv, J0.base, J0.stride, jl0 + src_off + J0.dir * src_dir_stride,
                    jl0 + dst_off + J0.dir * dst_dir_stride);
    if (L::rounds > 1 && J1.active)
      line_apply<n>(Dv, J1.base, J1.stride, jl1 + src_off + J1.dir * src_dir_stride,
                    jl1 + dst_off + J1.dir * dst_dir_stride);
  };
  constexpr int OFF_G = n * sl, OFF_F = (n + 2) * sl;

  for (int it = 0; it < a.iters; ++it) {
    double acc[n][4];
#pragma unroll
    for (int b = 0; b < n; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[b][v] = 0.0;
#pragma unroll 1
    for (int b = 0; b < n; ++b) {
      lines(b * sl, OFF_G, 0, sl);           // gradients of time node b
      wave_sync();
      double Sw = 0.0;
      if (node) {
        double q[4], Fx[4], Fz[4];
        Sw = node_flux<n>(ph, sq + b * sl, sg, sf, l, ih, z, rb, pb, q, Fx, Fz);
      }
      wave_sync();
      lines(OFF_F, OFF_F, sl, sl);           // divergence parts, in place
      wave_sync();
      if (node) {
        double R[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) R[v] = -(sf[v * nn + l] + sf[sl + v * nn + l]) * ih;
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
      wave_sync();
    }
    if (node) {
#pragma unroll
      for (int b = 0; b < n; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) sq[b * sl + v * nn + l] = fma(dt, acc[b][v], Qn[v]);
      if (a.iter_store && valid) {
        double* st = a.iter_store + ((size_t)c * a.iters + it) * n * sl;
#pragma unroll
        for (int b = 0; b < n; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) st[b * sl + v * nn + l] = sq[b * sl + v * nn + l];
      }
    }
    wave_sync();
  }

  // time averages of q, F and S on the last iterate
  double Qb[4] = {0, 0, 0, 0}, Fbx[4] = {0, 0, 0, 0}, Fbz[4] = {0, 0, 0, 0}, Sbw = 0.0, SbE = 0.0;
#pragma unroll 1
  for (int b = 0; b < n; ++b) {
    lines(b * sl, OFF_G, 0, sl);
    wave_sync();
    if (node) {
      double q[4], Fx[4], Fz[4];
      const double Sw = node_flux<n>(ph, sq + b * sl, sg, sf, l, ih, z, rb, pb, q, Fx, Fz);
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
    wave_sync();
  }

  // volume term and face data: averaged state to slot 0, averaged fluxes to sf
  if (node) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sq[v * nn + l] = Qb[v];
      sf[v * nn + l] = Fbx[v];
      sf[sl + v * nn + l] = Fbz[v];
    }
  }
  wave_sync();
  {
    double Wv[Half<n>::nh][n];
    load_vtab<n>(gt + GTab::dw(n), Wv);
#pragma unroll
    for (int r = 0; r < L::rounds; ++r) {
      const LineJob<n>& J = r == 0 ? J0 : J1;
      double* jl = r == 0 ? jl0 : jl1;
      if (!J.active) continue;
      const int cj = cell0 + J.slot;
      const double* src = jl + OFF_F + J.dir * sl;
      line_apply<n>(Wv, J.base, J.stride, src, jl + OFF_G + J.dir * sl);
      if (cj >= a.C) continue;
      double q0 = 0, q1 = 0, f0 = 0, f1 = 0;
#pragma unroll
      for (int m = 0; m < n; ++m) {
        const double e0 = gt[GTab::E0 * n + m], e1 = gt[GTab::E1 * n + m];
        const double iq = jl[J.base + m * J.stride], iF = src[J.base + m * J.stride];
        q0 = fma(e0, iq, q0); q1 = fma(e1, iq, q1);
        f0 = fma(e0, iF, f0); f1 = fma(e1, iF, f1);
      }
      double* fd = a.FD + (size_t)cj * 32 * n;
      const int fl = 2 * J.dir, fu = 2 * J.dir + 1;
      fd[((fl * 2 + 0) * 4 + J.v) * n + J.line] = q0;
      fd[((fl * 2 + 1) * 4 + J.v) * n + J.line] = f0;
      fd[((fu * 2 + 0) * 4 + J.v) * n + J.line] = q1;
      fd[((fu * 2 + 1) * 4 + J.v) * n + J.line] = f1;
    }
  }
  wave_sync();
  if (valid) {
    double* qs = a.Qs + (size_t)c * sl;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double S = (v == 2) ? Sbw : (v == 3 ? SbE : 0.0);
      qs[v * nn + l] = Qn[v] + dt * ((sg[v * nn + l] + sg[sl + v * nn + l]) * ih + S);
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

// face data of cell cf, face f, node k: averaged state and normal flux
template <int n>
__device__ inline void load_face(const double* FD, int cf, int f, int k, double Q[4], double F[4]) {
  const double* fd = FD + (size_t)cf * 32 * n + f * 8 * n;
#pragma unroll
  for (int v = 0; v < 4; ++v) { Q[v] = fd[v * n + k]; F[v] = fd[4 * n + v * n + k]; }
}

// face polynomial of cell cf, face f, evaluated at node q of sub-face s
template <int n>
__device__ inline void prolong_face(const double* FD, const double* gt, int cf, int f, int s, int q, double Q[4],
                                    double F[4]) {
  const double* fd = FD + (size_t)cf * 32 * n + f * 8 * n;
  const double* P = gt + GTab::pk(n) + (s * n + q) * n;
#pragma unroll
  for (int v = 0; v < 4; ++v) { Q[v] = 0.0; F[v] = 0.0; }
#pragma unroll
  for (int m = 0; m < n; ++m) {
    const double p = P[m];
#pragma unroll
    for (int v = 0; v < 4; ++v) { Q[v] = fma(p, fd[v * n + m], Q[v]); F[v] = fma(p, fd[4 * n + v * n + m], F[v]); }
  }
}

__device__ inline void rusanov_flux(double s, const double QL[4], const double FL[4], const double QR[4],
                                    const double FR[4], double G[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) G[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * s * (QR[v] - QL[v]);
}

// Per cell: lanes (slot, f, k) handle face f at node k.  The Rusanov speed s
// is one value per (sub-)face: max over the face nodes of both sides of the
// normal eigenvalue bound, plus the viscous penalty 2 eta max lambda_v with
// eta = (2N+1)/(h sqrt(pi/2)), h the (finer) cell size at the face.
// Conforming: the neighbour's face data; wall: ghost data; fine side of a
// 1:3 face: the coarse neighbour's face polynomial at this sub-face; coarse
// side: the three sub-face fluxes restricted by L2 projection.  Both sides of
// a face evaluate the identical expressions, so the fluxes agree bitwise.
template <int n, int CPW, int WPB>
__global__ __launch_bounds__(kWave * WPB) void k_corrector(Phys ph, StepArgs a) {
  using L = Lay<n, CPW>;
  constexpr int nn = L::nn, sl = L::sl;
  extern __shared__ double lds[];
  __shared__ double slam[WPB][2][kWave];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  double* wl = lds + (size_t)wave * CPW * L::corr_cell;
  const int cell0 = (blockIdx.x * WPB + wave) * CPW;
  const double* gt = a.gtab;
  const double eta0 = (2.0 * ph.N + 1.0) / 1.2533141373155002512;   // (2N+1)/sqrt(pi/2)

  // face role
  const int fslot = lane / (4 * n);
  const int f = (lane % (4 * n)) / n, k = lane % n;
  const int fc = cell0 + fslot;
  const bool fl = fslot < CPW && fc < a.C;
  double* fw = wl + (fslot < CPW ? fslot : 0) * L::corr_cell;
  double* sG = fw;                 // [4 faces][4 vars][n]
  double* sL = fw + 16 * n;        // [4][3][n]
  double* sV = sL + 12 * n;        // [4][3][n]
  double* sGs = sV + 12 * n;       // [4][3][4][n]
  const int d = f >> 1;
  const bool lower = (f & 1) == 0;   // face on the lower side: this cell is R
  int kind = kWall, nb1 = 0, nb2 = 0, nb3 = 0;
  double hf = 1.0, z0f = 0.0;
  double Qm[4], Fm[4], Qo[4], Fo[4];
  if (fl) {
    const int* nb = a.nbr + (size_t)fc * 16 + f * 4;
    kind = nb[0]; nb1 = nb[1]; nb2 = nb[2]; nb3 = nb[3];
    hf = a.geom[4 * fc + 2]; z0f = a.geom[4 * fc + 1];
    if (kind != kCoarseSide) {
      const double zf = (d == 0) ? z0f + hf * gt[GTab::XI * n + k] : z0f + ((f & 1) ? hf : 0.0);
      load_face<n>(a.FD, fc, f, k, Qm, Fm);
      if (kind == kConforming) load_face<n>(a.FD, nb1, f ^ 1, k, Qo, Fo);
      else if (kind == kFineSide) prolong_face<n>(a.FD, gt, nb1, f ^ 1, nb2, k, Qo, Fo);
      else wall_ghost(ph, d, zf, Qm, Fm, Qo, Fo);
      double l1, v1, l2, v2;
      eig(ph, d, Qm, zf, l1, v1);
      eig(ph, d, Qo, zf, l2, v2);
      sL[(f * 3) * n + k] = fmax(l1, l2);
      sV[(f * 3) * n + k] = fmax(v1, v2);
    } else {
      for (int s = 0; s < 3; ++s) {
        const int fine = s == 0 ? nb1 : (s == 1 ? nb2 : nb3);
        const double zf = (d == 0) ? z0f + hf * (s + gt[GTab::XI * n + k]) / 3.0 : z0f + ((f & 1) ? hf : 0.0);
        double Qp[4], Fp[4], Qx[4], Fx[4];
        prolong_face<n>(a.FD, gt, fc, f, s, k, Qp, Fp);
        load_face<n>(a.FD, fine, f ^ 1, k, Qx, Fx);
        double l1, v1, l2, v2;
        eig(ph, d, Qp, zf, l1, v1);
        eig(ph, d, Qx, zf, l2, v2);
        sL[(f * 3 + s) * n + k] = fmax(l1, l2);
        sV[(f * 3 + s) * n + k] = fmax(v1, v2);
      }
    }
  }
  wave_sync();
  if (fl) {
    if (kind != kCoarseSide) {
      double lam = sL[(f * 3) * n], lv = sV[(f * 3) * n];
#pragma unroll
      for (int m = 1; m < n; ++m) { lam = fmax(lam, sL[(f * 3) * n + m]); lv = fmax(lv, sV[(f * 3) * n + m]); }
      const double s = lam + 2.0 * (eta0 / hf) * lv;
      double G[4];
      if (lower) rusanov_flux(s, Qo, Fo, Qm, Fm, G);
      else rusanov_flux(s, Qm, Fm, Qo, Fo, G);
#pragma unroll
      for (int v = 0; v < 4; ++v) sG[(f * 4 + v) * n + k] = G[v];
    } else {
      const double hfine = hf / 3.0;
      for (int s = 0; s < 3; ++s) {
        const int fine = s == 0 ? nb1 : (s == 1 ? nb2 : nb3);
        double lam = sL[(f * 3 + s) * n], lv = sV[(f * 3 + s) * n];
        for (int m = 1; m < n; ++m) { lam = fmax(lam, sL[(f * 3 + s) * n + m]); lv = fmax(lv, sV[(f * 3 + s) * n + m]); }
        const double sp = lam + 2.0 * (eta0 / hfine) * lv;
        double Qp[4], Fp[4], Qx[4], Fx[4], G[4];
        prolong_face<n>(a.FD, gt, fc, f, s, k, Qp, Fp);
        load_face<n>(a.FD, fine, f ^ 1, k, Qx, Fx);
        if (lower) rusanov_flux(sp, Qx, Fx, Qp, Fp, G);
        else rusanov_flux(sp, Qp, Fp, Qx, Fx, G);
#pragma unroll
        for (int v = 0; v < 4; ++v) sGs[((f * 3 + s) * 4 + v) * n + k] = G[v];
      }
    }
  }
  wave_sync();
  if (fl && kind == kCoarseSide) {
    // L2 restriction to the coarse face node m = k
    const double* Rk = gt + GTab::rk(n);
    double G[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int q = 0; q < n; ++q) {
        const double r = Rk[(s * n + k) * n + q];
#pragma unroll
        for (int v = 0; v < 4; ++v) G[v] = fma(r, sGs[((f * 3 + s) * 4 + v) * n + q], G[v]);
      }
#pragma unroll
    for (int v = 0; v < 4; ++v) sG[(f * 4 + v) * n + k] = G[v];
  }
  wave_sync();

  // node role: lifting and the next CFL candidate
  const int slot = lane / nn, l = lane % nn;
  const int c = cell0 + slot;
  const bool valid = slot < CPW && c < a.C;
  const double* sGc = wl + (slot < CPW ? slot : 0) * L::corr_cell;
  double lam_n = 0.0, lv_n = 0.0;
  if (valid) {
    const int jz = l / n, ix = l % n;
    const int sc = a.scen ? a.scen[c] : 0;
    const double dt = a.clock[4 * sc + 1];
    const double z0 = a.geom[4 * c + 1], h = a.geom[4 * c + 2];
    const double L0i = gt[GTab::L0 * n + ix], L1i = gt[GTab::L1 * n + ix];
    const double L0j = gt[GTab::L0 * n + jz], L1j = gt[GTab::L1 * n + jz];
    const double* qs = a.Qs + (size_t)c * sl;
    double* qo = a.Qout + (size_t)c * sl;
    const double scl = dt / h;
    double q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double sx = L1i * sGc[(1 * 4 + v) * n + jz] - L0i * sGc[(0 * 4 + v) * n + jz];
      const double sz = L1j * sGc[(3 * 4 + v) * n + ix] - L0j * sGc[(2 * 4 + v) * n + ix];
      q[v] = qs[v * nn + l] - scl * (sx + sz);
      qo[v * nn + l] = q[v];
    }
    if (!ph.fixed_dt) {
      const double zz = z0 + h * gt[GTab::XI * n + jz];
      double l0, lv0, l1, lv1;
      eig(ph, 0, q, zz, l0, lv0);
      eig(ph, 1, q, zz, l1, lv1);
      lam_n = fmax(l0, l1);
      lv_n = lv0;
    }
  }
  if (!ph.fixed_dt) {
    // maxima of lambda and lambda_v over the nodes of each cell slot (a
    // contiguous lane range), then the CFL rule on the cell maxima
    slam[wave][0][lane] = lam_n;
    slam[wave][1][lane] = lv_n;
    wave_sync();
    if (valid && l == 0) {
      double lm = lam_n, vm = lv_n;
      for (int j = 1; j < nn; ++j) { lm = fmax(lm, slam[wave][0][lane + j]); vm = fmax(vm, slam[wave][1][lane + j]); }
      const double h = a.geom[4 * c + 2];
      const double o = 2.0 * ph.N + 1.0;
      a.dtc[c] = ph.cfl * h / (2.0 * o * (lm + 2.0 * vm * o / h));
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

// Clock update, one workgroup per scenario: if advance, t += dt and
// steps += 1; if update, dt <- min of the CFL candidates of the scenario's
// cells [beg[s], end[s]) (min is exact, so the result is order independent).
constexpr int kReduceThreads = 256;
__global__ __launch_bounds__(kReduceThreads) void k_clock(double* clock, const double* dtc, const int* beg,
                                                           const int* end, int C, int advance, int update) {
  __shared__ double sm[kReduceThreads / kWave];
  const int s = blockIdx.x, t = threadIdx.x;
  const int b0 = beg ? beg[s] : 0, b1 = end ? end[s] : C;
  double m = __builtin_inf();
  if (update)
    for (int c = b0 + t; c < b1; c += kReduceThreads) m = fmin(m, dtc[c]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmin(m, __shfl_xor(m, o, kWave));
  if ((t & (kWave - 1)) == 0) sm[t / kWave] = m;
  __syncthreads();
  if (t == 0) {
    double r = sm[0];
    for (int k = 1; k < kReduceThreads / kWave; ++k) r = fmin(r, sm[k]);
    if (advance) { clock[4 * s + 0] += clock[4 * s + 1]; clock[4 * s + 3] += 1.0; }
    if (update) clock[4 * s + 1] = r;
  }
}

// --------------------------------------------------------------- dispatchers
StepArgs make_args(const Group& g) {
  StepArgs a;
  a.Qin = g.Q; a.Qout = g.Q; a.Qs = g.Qs; a.FD = g.FD; a.dtc = g.dtc;
  a.clock = g.clock; a.scen = g.d_scen; a.geom = g.d_geom; a.nbr = g.d_nbr; a.gtab = g.d_gtab;
  a.C = g.C; a.iters = g.iters;
  a.iter_store = nullptr;
  return a;
}

template <int n, int CPW, int WPB>
static int launch_pred_t(const Group& g, hipStream_t s) {
  using L = Lay<n, CPW>;
  const size_t lds = sizeof(double) * (size_t)WPB * CPW * L::pred_cell;
  const int per_block = CPW * WPB;
  const int blocks = (g.C + per_block - 1) / per_block;
  if (blocks == 0) return ADG_OK;
  hipLaunchKernelGGL((k_predictor<n, CPW, WPB>), dim3(blocks), dim3(kWave * WPB), lds, s, g.ph, make_args(g));
  return check_launch("predictor");
}
template <int n, int CPW, int WPB>
static int launch_corr_t(const Group& g, hipStream_t s) {
  using L = Lay<n, CPW>;
  const size_t lds = sizeof(double) * (size_t)WPB * CPW * L::corr_cell;
  const int per_block = CPW * WPB;
  const int blocks = (g.C + per_block - 1) / per_block;
  if (blocks == 0) return ADG_OK;
  hipLaunchKernelGGL((k_corrector<n, CPW, WPB>), dim3(blocks), dim3(kWave * WPB), lds, s, g.ph, make_args(g));
  return check_launch("corrector");
}

template <int n, int CPW>
static int pred_w(const Group& g, hipStream_t s) {
  switch (g.wpb) {
    case 1: return launch_pred_t<n, CPW, 1>(g, s);
    case 2: return launch_pred_t<n, CPW, 2>(g, s);
    case 4: return launch_pred_t<n, CPW, 4>(g, s);
    default: return fail(ADG_EINVAL, "waves per block must be 1, 2 or 4");
  }
}
template <int n, int CPW>
static int corr_w(const Group& g, hipStream_t s) {
  switch (g.wpb) {
    case 1: return launch_corr_t<n, CPW, 1>(g, s);
    case 2: return launch_corr_t<n, CPW, 2>(g, s);
    case 4: return launch_corr_t<n, CPW, 4>(g, s);
    default: return fail(ADG_EINVAL, "waves per block must be 1, 2 or 4");
  }
}
// cells per wavefront: 1, 2 or 4 (while CPW * n^2 <= 64)
template <int n>
static int pred_n(const Group& g, hipStream_t s) {
  constexpr int nn = n * n;
  if (g.cpw == 1) return pred_w<n, 1>(g, s);
  if constexpr (2 * nn <= kWave) { if (g.cpw == 2) return pred_w<n, 2>(g, s); }
  if constexpr (4 * nn <= kWave) { if (g.cpw == 4) return pred_w<n, 4>(g, s); }
  return fail(ADG_EINVAL, "cells per wavefront not supported for this order");
}
template <int n>
static int corr_n(const Group& g, hipStream_t s) {
  constexpr int nn = n * n;
  if (g.cpw == 1) return corr_w<n, 1>(g, s);
  if constexpr (2 * nn <= kWave) { if (g.cpw == 2) return corr_w<n, 2>(g, s); }
  if constexpr (4 * nn <= kWave) { if (g.cpw == 4) return corr_w<n, 4>(g, s); }
  return fail(ADG_EINVAL, "cells per wavefront not supported for this order");
}
template <int n>
static int dt_n(const Group& g, hipStream_t s) {
  if (g.C == 0) return ADG_OK;
  hipLaunchKernelGGL(k_cell_dt<n>, dim3(g.C), dim3(kWave), 0, s, g.ph, make_args(g));
  return check_launch("cell_dt");
}

#define ADG_DISPATCH_N(fn, g, s)                                   \
  switch ((g).n) {                                                 \
    case 2: return fn<2>(g, s);                                    \
    case 3: return fn<3>(g, s);                                    \
    case 4: return fn<4>(g, s);                                    \
    case 5: return fn<5>(g, s);                                    \
    case 6: return fn<6>(g, s);                                    \
    case 7: return fn<7>(g, s);                                    \
    case 8: return fn<8>(g, s);                                    \
    default: return fail(ADG_EUNSUPPORTED, "order not supported"); \
  }

int launch_predictor(const Group& g, hipStream_t s) { ADG_DISPATCH_N(pred_n, g, s); }

template <int n>
static int pred_store_n(const Group& g, double* store, hipStream_t s) {
  using L = Lay<n, 1>;
  if (g.C == 0) return ADG_OK;
  StepArgs a = make_args(g);
  a.iter_store = store;
  const size_t lds = sizeof(double) * (size_t)L::pred_cell;
  hipLaunchKernelGGL((k_predictor<n, 1, 1>), dim3(g.C), dim3(kWave), lds, s, g.ph, a);
  return check_launch("predictor(store)");
}
int launch_predictor_store(const Group& g, double* store, hipStream_t s) {
  switch (g.n) {
    case 2: return pred_store_n<2>(g, store, s);
    case 3: return pred_store_n<3>(g, store, s);
    case 4: return pred_store_n<4>(g, store, s);
    case 5: return pred_store_n<5>(g, store, s);
    case 6: return pred_store_n<6>(g, store, s);
    case 7: return pred_store_n<7>(g, store, s);
    case 8: return pred_store_n<8>(g, store, s);
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
}
int launch_corrector(const Group& g, hipStream_t s) { ADG_DISPATCH_N(corr_n, g, s); }
int launch_cell_dt(const Group& g, hipStream_t s) { ADG_DISPATCH_N(dt_n, g, s); }

int launch_clock(double* clock, const double* dtc, const int* beg, const int* end, int nscen, int C, int advance,
                 int update, hipStream_t s) {
  if (nscen <= 0) return ADG_OK;
  hipLaunchKernelGGL(k_clock, dim3(nscen), dim3(kReduceThreads), 0, s, clock, dtc, beg, end, C, advance, update);
  return check_launch("clock");
}

int max_cpw(int n) { return (4 * n * n <= kWave) ? 4 : ((2 * n * n <= kWave) ? 2 : 1); }

}  // namespace adg
