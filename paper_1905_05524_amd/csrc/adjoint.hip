// Hand-written adjoint (reverse mode) of one ADER-DG step, of the initial
// state map from the potential-temperature perturbation, and of the
// potential-temperature loss, for gfx950.
//
// The step is Q^{n+1} = Q*(Q^n) - (dt/h) lift(G(FD(Q^n))) with a frozen dt.
// Its adjoint maps lambda^{n+1} = dL/dQ^{n+1} to lambda^n = dL/dQ^n:
//   1. the forward predictor is recomputed from the checkpoint Q^n, storing
//      the Picard iterates (iterate store);
//   2. lifting adjoint: per cell and face, the face-flux adjoint of this
//      cell's half of the surface integral;
//   3. face adjoint: per face, both halves summed, then the reverse of the
//      Rusanov flux (and of a wall ghost) onto this cell's face data;
//      non-smooth points take the subgradient of the first maximum in the
//      scan order (side L nodes 0..n-1, then side R), and d|x|/dx = 0 at 0;
//   4. reverse predictor: face extrapolations, volume term and time
//      averages, then the Picard sweeps in reverse order (R = S - div F:
//      transposed derivative contractions and the reverse of the pointwise
//      flux), accumulating dL/dQ^n.
#include "adg_internal.h"

namespace adg {

__device__ inline void wave_sync_a() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// --------------------------------------------------------- pointwise VJP
// Reverse of flux_source: given adjoints aFx, aFz of the fluxes and aSw of
// the gravity source, returns the adjoints of the state and its gradients.
__device__ inline void flux_source_vjp(const Phys& ph, const double q[4], const double gx[4],
                                       const double gz[4], double z, double rb, const double aFx[4],
                                       const double aFz[4], double aSw, double aq[4], double agx[4],
                                       double agz[4]) {
  (void)rb;
  // forward intermediates
  const double rho = q[0], mx = q[1], mz = q[2], E = q[3];
  const double ir = 1.0 / rho;
  const double u = mx * ir, w = mz * ir;
  const double gzz = ph.gravity ? ph.g * z : 0.0;
  const double p = ph.gm1 * (E - 0.5 * (mx * u + mz * w) - rho * gzz);
  const double T = p * ir * ph.iR;
  const double dux = (gx[1] - u * gx[0]) * ir, duz = (gz[1] - u * gz[0]) * ir;
  const double dwx = (gx[2] - w * gx[0]) * ir, dwz = (gz[2] - w * gz[0]) * ir;
  const double hv2 = 0.5 * (u * u + w * w) + gzz;
  const double dpx = ph.gm1 * (gx[3] - hv2 * gx[0] - rho * (u * dux + w * dwx));
  double dpz = ph.gm1 * (gz[3] - hv2 * gz[0] - rho * (u * duz + w * dwz));
  if (ph.gravity) dpz -= ph.gm1 * rho * ph.g;
  const double div = dux + dwz;
  const double sxx = ph.mu * ((2.0 / 3.0) * div - 2.0 * dux);
  const double szz = ph.mu * ((2.0 / 3.0) * div - 2.0 * dwz);
  const double sxz = -ph.mu * (duz + dwx);
  const double H = E + p;
  // reverse sweep
  double brho = 0, bmx = 0, bmz = 0, bE = 0;
  double bu = 0, bw = 0, bH = 0, bpm = 0, bsxx = 0, bszz = 0, bsxz = 0, bdTx = 0, bdTz = 0;
  for (int v = 0; v < 4; ++v) { agx[v] = 0.0; agz[v] = 0.0; }
  if (ph.gravity) brho += -ph.g * aSw;
  // Fz3 = w H + u sxz + w szz - kappa dTz
  bw += aFz[3] * (H + szz); bH += aFz[3] * w; bu += aFz[3] * sxz; bsxz += aFz[3] * u; bszz += aFz[3] * w;
  bdTz += -ph.kappa * aFz[3];
  // Fz2 = mz w + pm + szz
  bmz += aFz[2] * w; bw += aFz[2] * mz; bpm += aFz[2]; bszz += aFz[2];
  // Fz1 = mx w + sxz
  bmx += aFz[1] * w; bw += aFz[1] * mx; bsxz += aFz[1];
  // Fz0 = mz
  bmz += aFz[0];
  // Fx3 = u H + u sxx + w sxz - kappa dTx
  bu += aFx[3] * (H + sxx); bH += aFx[3] * u; bsxx += aFx[3] * u; bw += aFx[3] * sxz; bsxz += aFx[3] * w;
  bdTx += -ph.kappa * aFx[3];
  // Fx2 = mz u + sxz
  bmz += aFx[2] * u; bu += aFx[2] * mz; bsxz += aFx[2];
  // Fx1 = mx u + pm + sxx
  bmx += aFx[1] * u; bu += aFx[1] * mx; bpm += aFx[1]; bsxx += aFx[1];
  // Fx0 = mx
  bmx += aFx[0];
  // H = E + p
  bE += bH;
  double bp = bH;
  // sxz = -mu (duz + dwx)
  double bduz = -ph.mu * bsxz, bdwx = -ph.mu * bsxz;
  // szz = mu (2/3 div - 2 dwz), sxx = mu (2/3 div - 2 dux)
  double bdiv = ph.mu * (2.0 / 3.0) * (bszz + bsxx);
  double bdwz = -2.0 * ph.mu * bszz, bdux = -2.0 * ph.mu * bsxx;
  // div = dux + dwz
  bdux += bdiv; bdwz += bdiv;
  // dTz = (dpz - R T gz0) ir iR ; dTx likewise
  const double c_ = ir * ph.iR;
  double bdpz = bdTz * c_, bdpx = bdTx * c_;
  double bT = -ph.R * (gz[0] * bdTz + gx[0] * bdTx) * c_;
  agz[0] += -ph.R * T * bdTz * c_;
  agx[0] += -ph.R * T * bdTx * c_;
  double bir = (bdTz * (dpz - ph.R * T * gz[0]) + bdTx * (dpx - ph.R * T * gx[0])) * ph.iR;
  // dpz = gm1 (gz3 - hv2 gz0 - rho (u duz + w dwz)) - [grav] gm1 rho g
  double t = bdpz * ph.gm1;
  agz[3] += t;
  double bhv2 = -t * gz[0];
  agz[0] += -t * hv2;
  brho += -t * (u * duz + w * dwz);
  bu += -t * rho * duz; bduz += -t * rho * u; bw += -t * rho * dwz; bdwz += -t * rho * w;
  if (ph.gravity) brho += -bdpz * ph.gm1 * ph.g;
  // dpx = gm1 (gx3 - hv2 gx0 - rho (u dux + w dwx))
  t = bdpx * ph.gm1;
  agx[3] += t;
  bhv2 += -t * gx[0];
  agx[0] += -t * hv2;
  brho += -t * (u * dux + w * dwx);
  bu += -t * rho * dux; bdux += -t * rho * u; bw += -t * rho * dwx; bdwx += -t * rho * w;
  // hv2 = 1/2 (u^2 + w^2) + gzz
  bu += bhv2 * u; bw += bhv2 * w;
  // dwz = (gz2 - w gz0) ir ; dwx ; duz ; dux
  agz[2] += bdwz * ir; bw += -bdwz * gz[0] * ir; agz[0] += -bdwz * w * ir; bir += bdwz * (gz[2] - w * gz[0]);
  agx[2] += bdwx * ir; bw += -bdwx * gx[0] * ir; agx[0] += -bdwx * w * ir; bir += bdwx * (gx[2] - w * gx[0]);
  agz[1] += bduz * ir; bu += -bduz * gz[0] * ir; agz[0] += -bduz * u * ir; bir += bduz * (gz[1] - u * gz[0]);
  agx[1] += bdux * ir; bu += -bdux * gx[0] * ir; agx[0] += -bdux * u * ir; bir += bdux * (gx[1] - u * gx[0]);
  // T = p ir iR
  bp += bT * ir * ph.iR; bir += bT * p * ph.iR;
  // pm = p - pb or p
  bp += bpm;
  // p = gm1 (E - 1/2 (mx u + mz w) - rho gzz)
  t = bp * ph.gm1;
  bE += t;
  bmx += -0.5 * t * u; bu += -0.5 * t * mx;
  bmz += -0.5 * t * w; bw += -0.5 * t * mz;
  brho += -t * gzz;
  // u = mx ir, w = mz ir
  bmx += bu * ir; bir += bu * mx;
  bmz += bw * ir; bir += bw * mz;
  // ir = 1/rho
  brho += -bir * ir * ir;
  aq[0] = brho; aq[1] = bmx; aq[2] = bmz; aq[3] = bE;
}

// ------------------------------------------------- line jobs (half tables)
template <int n>
struct HalfA { static constexpr int nh = (n + 1) / 2; };

template <int n>
__device__ inline void vtab_load(const double* g, double (&M)[HalfA<n>::nh][n]) {
#pragma unroll
  for (int i = 0; i < HalfA<n>::nh; ++i)
#pragma unroll
    for (int m = 0; m < n; ++m) {
      M[i][m] = g[i * n + m];
      asm volatile("" : "+v"(M[i][m]));
    }
}

// the same table left to the compiler: its entries are uniform, so they can
// live in scalar registers
template <int n>
__device__ inline void stab_load(const double* g, double (&M)[HalfA<n>::nh][n]) {
#pragma unroll
  for (int i = 0; i < HalfA<n>::nh; ++i)
#pragma unroll
    for (int m = 0; m < n; ++m) M[i][m] = g[i * n + m];
}

// out = M in along a line (M centro-antisymmetric, first nh rows stored)
template <int n>
__device__ inline void line_M(const double (&M)[HalfA<n>::nh][n], int base, int stride, const double* src,
                              double* dst, double scale) {
  constexpr int nh = HalfA<n>::nh;
  double in[n];
#pragma unroll
  for (int m = 0; m < n; ++m) in[m] = src[base + m * stride];
#pragma unroll
  for (int i = 0; i < nh; ++i) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) s = fma(M[i][m], in[m], s);
    dst[base + i * stride] = scale * s;
  }
#pragma unroll
  for (int i = 0; i < n / 2; ++i) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) s = fma(M[i][m], in[n - 1 - m], s);
    dst[base + (n - 1 - i) * stride] = -scale * s;
  }
}

// out = M^T in along a line: out[m] = sum_i M[i][m] in[i], with
// M[i][m] = -M[n-1-i][n-1-m] for the rows not stored
template <int n>
__device__ inline void line_MT(const double (&M)[HalfA<n>::nh][n], int base, int stride, const double* src,
                               double* dst, double scale) {
  constexpr int nh = HalfA<n>::nh;
  double in[n];
#pragma unroll
  for (int i = 0; i < n; ++i) in[i] = src[base + i * stride];
#pragma unroll
  for (int m = 0; m < n; ++m) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < nh; ++i) s = fma(M[i][m], in[i], s);
#pragma unroll
    for (int i = nh; i < n; ++i) s = fma(-M[n - 1 - i][n - 1 - m], in[i], s);
    dst[base + m * stride] = scale * s;
  }
}

struct AdjArgs {
  const double* Qn;      // checkpoint [C][4][n][n]
  const double* lam_in;  // dL/dQ^{n+1}
  double* lam_out;       // dL/dQ^n
  const double* FD;      // forward face data (recomputed)
  const double* store;   // iterates [C][I][n][4][n][n]
  double* lamFD;         // [C][4 faces][2][4][n]
  const double* clock;
  const double* geom;
  const int* nbr;
  const double* gtab;
  int C, iters;
};

// ---------------------------------------------------------- lifting adjoint
// The corrector's surface term of cell c, -(dt/h) (L1 G_{+} - L0 G_{-}) per
// row or column, transposed: cell c's half of the adjoint of face f's flux
// at face node k, variable v (L0 = e0/w, L1 = e1/w).
template <int n>
__device__ inline double lift_adj_half(const AdjArgs& a, int c, int f, int k, int v) {
  constexpr int nn = n * n;
  const double sc = a.clock[1] / a.geom[4 * c + 2];
  const double* lam = a.lam_in + (size_t)c * 4 * nn + v * nn;
  const double* Lt = a.gtab + (((f & 1) ? GTab::L1 : GTab::L0) * n);
  const double sgn = (f & 1) ? -sc : sc;   // +face: -(dt/h) L1, -face: +(dt/h) L0
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < n; ++m) {
    const int idx = (f < 2) ? (k * n + m) : (m * n + k);   // x-faces: row k; z-faces: column k
    s = fma(Lt[m], lam[idx], s);
  }
  return sgn * s;
}

// ------------------------------------------------------------ face adjoint
__device__ inline void eig_a(const Phys& ph, int d, const double q[4], double zf, double& lam, double& lv) {
  const double ir = 1.0 / q[0];
  const double p = pressure(ph, q[0], q[1], q[2], q[3], zf);
  lam = fabs((d == 0 ? q[1] : q[2]) * ir) + sqrt(ph.gamma * p * ir);
  lv = ph.lv_coef * ir;
}

// gradient of lambda = |v_d| + c and of lambda_v with respect to the state
__device__ inline void eig_grad(const Phys& ph, int d, const double q[4], double zf, double gl[4], double gv[4]) {
  const double rho = q[0], ir = 1.0 / rho;
  const double u = q[1] * ir, w = q[2] * ir;
  const double p = pressure(ph, q[0], q[1], q[2], q[3], zf);
  const double c = sqrt(ph.gamma * p * ir);
  const double vn = (d == 0 ? q[1] : q[2]) * ir;
  const double sg = vn > 0.0 ? 1.0 : (vn < 0.0 ? -1.0 : 0.0);
  const double geo = ph.gravity ? ph.g * zf : 0.0;
  // dp/dQ
  const double dp[4] = {ph.gm1 * (0.5 * (u * u + w * w) - geo), -ph.gm1 * u, -ph.gm1 * w, ph.gm1};
  // dc = gamma/(2c) (dp/rho - p drho/rho^2)
  const double k = ph.gamma / (2.0 * c);
  for (int v = 0; v < 4; ++v) gl[v] = k * dp[v] * ir;
  gl[0] += -k * p * ir * ir;
  gl[0] += sg * (-vn * ir);
  if (d == 0) gl[1] += sg * ir;
  else gl[2] += sg * ir;
  gv[0] = -ph.lv_coef * ir * ir; gv[1] = 0.0; gv[2] = 0.0; gv[3] = 0.0;
}

// wall ghost (as in the forward corrector) and its reverse
__device__ inline void ghost_fwd(const Phys& ph, int d, double zf, const double Qi[4], const double Fi[4], double Qg[4],
                                 double Fg[4]) {
  const double u = Qi[1] / Qi[0], w = Qi[2] / Qi[0];
  double rb, pb;
  if (ph.gravity) background(ph, zf, rb, pb);
  else { rb = Qi[0]; pb = pressure(ph, Qi[0], Qi[1], Qi[2], Qi[3], zf); }
  const double geo = ph.gravity ? rb * (ph.g * zf) : 0.0;
  Qg[0] = rb; Qg[1] = -(rb * u); Qg[2] = -(rb * w);
  Qg[3] = pb / ph.gm1 + 0.5 * rb * (u * u + w * w) + geo;
  const double qbg = (ph.gravity && d == 1) ? ph.kappa * ph.g / ph.cp : 0.0;
  Fg[0] = -Fi[0]; Fg[1] = Fi[1]; Fg[2] = Fi[2]; Fg[3] = 2.0 * qbg - Fi[3];
}

// adjoints of the ghost (aQg, aFg) -> adjoints of the interior data
__device__ inline void ghost_vjp(const Phys& ph, double zf, const double Qi[4], const double aQg[4],
                                 const double aFg[4], double aQi[4], double aFi[4]) {
  aFi[0] = -aFg[0]; aFi[1] = aFg[1]; aFi[2] = aFg[2]; aFi[3] = -aFg[3];
  const double rho = Qi[0], ir = 1.0 / rho;
  const double u = Qi[1] * ir, w = Qi[2] * ir;
  double rb, pb, brb = 0.0, bpb = 0.0, bu = 0.0, bw = 0.0;
  if (ph.gravity) background(ph, zf, rb, pb);
  else { rb = rho; pb = pressure(ph, Qi[0], Qi[1], Qi[2], Qi[3], zf); }
  // Qg0 = rb ; Qg1 = -rb u ; Qg2 = -rb w ; Qg3 = pb/gm1 + 1/2 rb (u^2+w^2) + rb g z
  brb += aQg[0] - aQg[1] * u - aQg[2] * w + aQg[3] * (0.5 * (u * u + w * w) + (ph.gravity ? ph.g * zf : 0.0));
  bu += -aQg[1] * rb + aQg[3] * rb * u;
  bw += -aQg[2] * rb + aQg[3] * rb * w;
  bpb += aQg[3] / ph.gm1;
  aQi[0] = 0.0; aQi[1] = 0.0; aQi[2] = 0.0; aQi[3] = 0.0;
  if (!ph.gravity) {
    aQi[0] += brb;
    // pb = gm1 (E - 1/2 (mx^2 + mz^2)/rho)
    aQi[3] += bpb * ph.gm1;
    aQi[1] += -bpb * ph.gm1 * u;
    aQi[2] += -bpb * ph.gm1 * w;
    aQi[0] += bpb * ph.gm1 * 0.5 * (u * u + w * w);
  }
  // u = mx/rho, w = mz/rho
  aQi[1] += bu * ir; aQi[2] += bw * ir;
  aQi[0] += -(bu * u + bw * w) * ir;
}

// Per cell, lanes (f, k): total flux adjoint of face f at node k (this
// cell's half plus the neighbour's, both from the lifting adjoint of the
// incoming adjoint state), then the reverse of the Rusanov flux
// onto this cell's own face data (and, at walls, through the ghost).
template <int n>
__global__ __launch_bounds__(kWave) void k_face_adj(Phys ph, AdjArgs a) {
  __shared__ double sLam[4][2][n], sLv[4][2][n], sQd[4][n];
  const int c = blockIdx.x, lane = threadIdx.x;
  const bool act = lane < 4 * n;
  const int f = act ? lane / n : 0, k = lane % n;
  const int d = f >> 1;
  const bool lower = (f & 1) == 0;     // this cell is side R
  const double* gt = a.gtab;
  const double h = a.geom[4 * c + 2], z0 = a.geom[4 * c + 1];
  const int* nb = a.nbr + (size_t)c * 16 + f * 4;
  const int kind = act ? nb[0] : kWall;
  double Qm[4], Fm[4], Qo[4], Fo[4], aG[4];
  const double zf = (d == 0) ? z0 + h * gt[GTab::XI * n + k] : z0 + ((f & 1) ? h : 0.0);
  if (act) {
    const double* fd = a.FD + (size_t)c * 32 * n + f * 8 * n;
    for (int v = 0; v < 4; ++v) {
      Qm[v] = fd[v * n + k]; Fm[v] = fd[4 * n + v * n + k];
      aG[v] = lift_adj_half<n>(a, c, f, k, v);
    }
    if (kind == kConforming) {
      const int o = nb[1];
      const double* fo = a.FD + (size_t)o * 32 * n + (f ^ 1) * 8 * n;
      for (int v = 0; v < 4; ++v) {
        Qo[v] = fo[v * n + k]; Fo[v] = fo[4 * n + v * n + k];
        aG[v] += lift_adj_half<n>(a, o, f ^ 1, k, v);
      }
    } else {
      ghost_fwd(ph, d, zf, Qm, Fm, Qo, Fo);
    }
    double QL[4], QR[4];
    for (int v = 0; v < 4; ++v) { QL[v] = lower ? Qo[v] : Qm[v]; QR[v] = lower ? Qm[v] : Qo[v]; }
    double l, lv;
    eig_a(ph, d, QL, zf, l, lv); sLam[f][0][k] = l; sLv[f][0][k] = lv;
    eig_a(ph, d, QR, zf, l, lv); sLam[f][1][k] = l; sLv[f][1][k] = lv;
    // this node's share of dL/ds = sum_v aG . (-1/2 (QR - QL))
    double ds = 0.0;
    for (int v = 0; v < 4; ++v) ds += aG[v] * (-0.5 * (QR[v] - QL[v]));
    sQd[f][k] = ds;
  }
  wave_sync_a();
  if (!act) return;
  // speed and its argmax: first maximum in the order L nodes 0..n-1, R nodes 0..n-1
  double lam = sLam[f][0][0], lvm = sLv[f][0][0];
  int al = 0, av = 0;
  for (int side = 0; side < 2; ++side)
    for (int m = 0; m < n; ++m) {
      const int id = side * n + m;
      if (id == 0) continue;
      if (sLam[f][side][m] > lam) { lam = sLam[f][side][m]; al = id; }
      if (sLv[f][side][m] > lvm) { lvm = sLv[f][side][m]; av = id; }
    }
  const double eta = (2.0 * ph.N + 1.0) / (h * 1.2533141373155002512);
  const double s = lam + 2.0 * eta * lvm;
  double bs = 0.0;
  for (int m = 0; m < n; ++m) bs += sQd[f][m];
  // G = 1/2 (FL + FR) - 1/2 s (QR - QL): adjoints of (QL, FL, QR, FR) at node k
  double aQL[4], aFL[4], aQR[4], aFR[4];
  for (int v = 0; v < 4; ++v) {
    aFL[v] = 0.5 * aG[v]; aFR[v] = 0.5 * aG[v];
    aQL[v] = 0.5 * s * aG[v]; aQR[v] = -0.5 * s * aG[v];
  }
  // speed terms at the argmax nodes (if they are this node)
  // speed terms at the argmax nodes (if they are this node)
  double gl[4], gv[4];
  if (al == k) {
    eig_grad(ph, d, lower ? Qo : Qm, zf, gl, gv);
    for (int v = 0; v < 4; ++v) aQL[v] += bs * gl[v];
  } else if (al == n + k) {
    eig_grad(ph, d, lower ? Qm : Qo, zf, gl, gv);
    for (int v = 0; v < 4; ++v) aQR[v] += bs * gl[v];
  }
  if (av == k) {
    eig_grad(ph, d, lower ? Qo : Qm, zf, gl, gv);
    for (int v = 0; v < 4; ++v) aQL[v] += bs * 2.0 * eta * gv[v];
  } else if (av == n + k) {
    eig_grad(ph, d, lower ? Qm : Qo, zf, gl, gv);
    for (int v = 0; v < 4; ++v) aQR[v] += bs * 2.0 * eta * gv[v];
  }
  double aQm[4], aFm[4], aQg[4], aFg[4];
  for (int v = 0; v < 4; ++v) {
    aQm[v] = lower ? aQR[v] : aQL[v];
    aFm[v] = lower ? aFR[v] : aFL[v];
    aQg[v] = lower ? aQL[v] : aQR[v];
    aFg[v] = lower ? aFL[v] : aFR[v];
  }
  if (kind == kWall) {
    double aQi[4], aFi[4];
    ghost_vjp(ph, zf, Qm, aQg, aFg, aQi, aFi);
    for (int v = 0; v < 4; ++v) { aQm[v] += aQi[v]; aFm[v] += aFi[v]; }
  }
  double* out = a.lamFD + (size_t)c * 32 * n + f * 8 * n;
  for (int v = 0; v < 4; ++v) { out[v * n + k] = aQm[v]; out[4 * n + v * n + k] = aFm[v]; }
}

// ------------------------------------------------------- reverse predictor
// One workgroup of NW wavefronts per cell; wavefront w owns the time levels
// b = w, w + NW, ... (NW = min(n, 4): at order 6, three cells' workgroups
// share a CU, so a 27x27 mesh runs in one round).  The reverse of every time
// level of a sweep (and of the final pass) is independent of the others once
// the sweep's residual adjoints are known, so the levels run side by side;
// the workgroup synchronises only where the levels meet (the time matrix
// mixes them).  Each wavefront has its own LDS slice buffers; the iterate
// adjoints Lq and the residual adjoints sR are shared.
template <int n>
constexpr int adj_waves() { return n < 4 ? n : 4; }

template <int n>
__global__ __launch_bounds__(kWave * adj_waves<n>()) void k_pred_adj(Phys ph, AdjArgs a) {
  constexpr int nn = n * n, sl = 4 * nn, NW = adj_waves<n>();
  __shared__ double Lq[n * sl];        // adjoint of the iterate at every time node
  __shared__ double sR[n * sl];        // residual adjoints of one reverse sweep
  __shared__ double sW[NW][3 * sl];    // per wavefront: state slice, then gradients / adjoint work
  const int c = blockIdx.x, w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  double* sq = sW[w];
  double* sg = sW[w] + sl;             // [2][sl]: gradients along x and z, reused for the adjoint work
  const bool node = lane < nn;
  const int l = node ? lane : 0;
  const int jz = l / n, ix = l % n;
  const bool job = lane < 8 * n;
  const int dir = lane / (4 * n), jv = (lane % (4 * n)) / n, line = lane % n;
  const int jbase = jv * nn + (dir == 0 ? line * n : line), jstride = dir == 0 ? 1 : n;
  const double* gt = a.gtab;
  const double dt = a.clock[1];
  const double z0 = a.geom[4 * c + 1], h = a.geom[4 * c + 2];
  const double ih = 1.0 / h;
  const double z = z0 + h * gt[GTab::XI * n + jz];
  double rb, pb;
  background(ph, z, rb, pb);
  (void)pb;
  double Dv[HalfA<n>::nh][n];
  stab_load<n>(gt + GTab::d(n), Dv);
  const double* Qc = a.Qn + (size_t)c * sl;
  const double* lin = a.lam_in + (size_t)c * sl;
  const double* lfd = a.lamFD + (size_t)c * 32 * n;
  const double* store = a.store + (size_t)c * a.iters * n * sl;
  const int I = a.iters;

  // (a) adjoints of Q*, of the averaged state, fluxes and source (every
  // wavefront computes them for its own use)
  double aQn[4], aQb[4], aFbx[4], aFbz[4], aSb = 0.0;
  double lq[4];
  for (int v = 0; v < 4; ++v) lq[v] = node ? lin[v * nn + l] : 0.0;
  for (int v = 0; v < 4; ++v) aQn[v] = w == 0 ? lq[v] : 0.0;   // direct part, counted once
  aSb = dt * lq[2];
  if (node)
    for (int v = 0; v < 4; ++v) sq[v * nn + l] = lq[v];
  wave_sync_a();
  {
    double Wv[HalfA<n>::nh][n];
    stab_load<n>(gt + GTab::dw(n), Wv);
    // lambda_Fbar = (dt/h) Dw^T lambda_Q* along x (rows) and z (columns)
    if (job) line_MT<n>(Wv, jbase, jstride, sq, sg + dir * sl, dt * ih);
  }
  wave_sync_a();
  if (node) {
    const double e0i = gt[GTab::E0 * n + ix], e1i = gt[GTab::E1 * n + ix];
    const double e0j = gt[GTab::E0 * n + jz], e1j = gt[GTab::E1 * n + jz];
    for (int v = 0; v < 4; ++v) {
      // face extrapolations: x faces use row jz, z faces column ix
      aQb[v] = e0i * lfd[(0 * 2 + 0) * 4 * n + v * n + jz] + e1i * lfd[(1 * 2 + 0) * 4 * n + v * n + jz] +
               e0j * lfd[(2 * 2 + 0) * 4 * n + v * n + ix] + e1j * lfd[(3 * 2 + 0) * 4 * n + v * n + ix];
      aFbx[v] = sg[v * nn + l] + e0i * lfd[(0 * 2 + 1) * 4 * n + v * n + jz] +
                e1i * lfd[(1 * 2 + 1) * 4 * n + v * n + jz];
      aFbz[v] = sg[sl + v * nn + l] + e0j * lfd[(2 * 2 + 1) * 4 * n + v * n + ix] +
                e1j * lfd[(3 * 2 + 1) * 4 * n + v * n + ix];
    }
  }
  wave_sync_a();

  // reverse of "flux/source at time level b": given aF (x, z) and aSw per
  // node, the state adjoint (direct + through the gradients) plus add[]
  // becomes Lq[b]
  auto slice_vjp = [&](int b, const double* qsrc, const double aFx[4], const double aFz[4], double aSw,
                       const double add[4]) {
    double q[4] = {0, 0, 0, 0};   // the node's state, kept for the flux adjoint
    if (node)
      for (int v = 0; v < 4; ++v) { q[v] = qsrc[v * nn + l]; sq[v * nn + l] = q[v]; }
    wave_sync_a();
    if (job) line_M<n>(Dv, jbase, jstride, sq, sg + dir * sl, ih);     // gradients
    wave_sync_a();
    double aq[4] = {0, 0, 0, 0};
    if (node) {
      double gx[4], gz[4], agx[4], agz[4];
      for (int v = 0; v < 4; ++v) { gx[v] = sg[v * nn + l]; gz[v] = sg[sl + v * nn + l]; }
      flux_source_vjp(ph, q, gx, gz, z, rb, aFx, aFz, aSw, aq, agx, agz);
      for (int v = 0; v < 4; ++v) { sg[v * nn + l] = agx[v]; sg[sl + v * nn + l] = agz[v]; }
    }
    wave_sync_a();
    // gradient adjoints back to the state: (1/h) D^T along each direction
    if (job) line_MT<n>(Dv, jbase, jstride, sg + dir * sl, sg + dir * sl, ih);
    wave_sync_a();
    if (node)
      for (int v = 0; v < 4; ++v) Lq[b * sl + v * nn + l] = aq[v] + sg[v * nn + l] + sg[sl + v * nn + l] + add[v];
    wave_sync_a();
  };

  // (b) final pass: F, S and q at the last iterate, averaged with w_b
  for (int b = w; b < n; b += NW) {
    const double wb = gt[GTab::W * n + b];
    double aFx[4], aFz[4], add[4];
    for (int v = 0; v < 4; ++v) { aFx[v] = wb * aFbx[v]; aFz[v] = wb * aFbz[v]; add[v] = wb * aQb[v]; }
    slice_vjp(b, store + ((size_t)(I - 1) * n + b) * sl, aFx, aFz, wb * aSb, add);
  }
  __syncthreads();

  // (c) Picard sweeps in reverse: q^{k+1}[a] = Q^n + dt sum_b P[a][b] R(q^k[b])
  for (int it = I - 1; it >= 0; --it) {
    for (int b = w; b < n; b += NW) {
      const double* prow = gt + GTab::pt(n) + b * n;   // P[a][b] over a
      if (node)
        for (int v = 0; v < 4; ++v) {
          aQn[v] += Lq[b * sl + v * nn + l];
          double s = 0.0;
          for (int a2 = 0; a2 < n; ++a2) s = fma(prow[a2], Lq[a2 * sl + v * nn + l], s);
          sR[b * sl + v * nn + l] = dt * s;
        }
    }
    __syncthreads();   // every level's Lq read before any is overwritten
    for (int b = w; b < n; b += NW) {
      // R = S - (1/h)(Dx Fx + Dz Fz): lambda_F = -(1/h) D^T lambda_R, lambda_Sw = lambda_R[2]
      if (job) line_MT<n>(Dv, jbase, jstride, sR + b * sl, sg + dir * sl, -ih);
      wave_sync_a();
      double aFx[4], aFz[4];
      for (int v = 0; v < 4; ++v) {
        aFx[v] = node ? sg[v * nn + l] : 0.0;
        aFz[v] = node ? sg[sl + v * nn + l] : 0.0;
      }
      const double aSw = node ? sR[b * sl + 2 * nn + l] : 0.0;
      wave_sync_a();
      const double zero[4] = {0, 0, 0, 0};
      slice_vjp(b, it > 0 ? store + ((size_t)(it - 1) * n + b) * sl : Qc, aFx, aFz, aSw, zero);
    }
    __syncthreads();   // every level's Lq written before the next sweep reads them
  }
  // q^0[b] = Q^n for every b; each wavefront's share (its accumulator and its
  // levels' last adjoints) summed through LDS
  if (node)
    for (int v = 0; v < 4; ++v) {
      double s = aQn[v];
      for (int b = w; b < n; b += NW) s += Lq[b * sl + v * nn + l];
      sR[w * sl + v * nn + l] = s;
    }
  __syncthreads();
  if (w == 0 && node) {
    double* out = a.lam_out + (size_t)c * sl;
    for (int v = 0; v < 4; ++v) {
      double s = 0.0;
      for (int k = 0; k < NW; ++k) s += sR[k * sl + v * nn + l];
      out[v * nn + l] = s;
    }
  }
}

// ----------------------------------------------- initial state from theta'
// rho = p_bar / (R pi (theta_bg + theta')), E = p_bar/(gamma-1) + rho g z, at rest.
__global__ void k_ic_theta(Phys ph, int n, int C, const double* geom, const double* gtab, const double* thp,
                           double* Q) {
  const int nn = n * n;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)C * nn) return;
  const int c = (int)(gid / nn), node = (int)(gid % nn);
  const double z = geom[4 * c + 1] + geom[4 * c + 2] * gtab[GTab::XI * n + node / n];
  const double pi = 1.0 - ph.ex_coef * z;
  const double pb = ph.p0 * pow(pi, ph.cp_over_R);
  const double rho = pb / (ph.R * pi * (ph.theta + thp[(size_t)c * nn + node]));
  double* Qc = Q + (size_t)c * 4 * nn;
  Qc[node] = rho; Qc[nn + node] = 0.0; Qc[2 * nn + node] = 0.0;
  Qc[3 * nn + node] = pb / ph.gm1 + rho * ph.g * z;
}

__global__ void k_ic_theta_adj(Phys ph, int n, int C, const double* geom, const double* gtab, const double* thp,
                               const double* lam, double* grad) {
  const int nn = n * n;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)C * nn) return;
  const int c = (int)(gid / nn), node = (int)(gid % nn);
  const double z = geom[4 * c + 1] + geom[4 * c + 2] * gtab[GTab::XI * n + node / n];
  const double pi = 1.0 - ph.ex_coef * z;
  const double pb = ph.p0 * pow(pi, ph.cp_over_R);
  const double th = ph.theta + thp[(size_t)c * nn + node];
  const double rho = pb / (ph.R * pi * th);
  const double drho = -rho / th;
  const double* lc = lam + (size_t)c * 4 * nn;
  grad[(size_t)c * nn + node] = drho * (lc[node] + ph.g * z * lc[3 * nn + node]);
}

// ------------------------------------------------- potential-temperature loss
// L = sqrt(sum_cells h^2 sum_ji w_i w_j (theta - theta_bg)^2), theta =
// T (p0/p)^(R/cp).  Per-cell partial sums, then one workgroup sums them in a
// fixed order and takes the root.
template <int n>
__global__ __launch_bounds__(kWave) void k_loss_part(Phys ph, const double* Q, const double* geom, const double* gtab,
                                                       double* part) {
  constexpr int nn = n * n;
  const int c = blockIdx.x, lane = threadIdx.x;
  double v = 0.0;
  if (lane < nn) {
    const int jz = lane / n, ix = lane % n;
    const double h = geom[4 * c + 2];
    const double z = geom[4 * c + 1] + h * gtab[GTab::XI * n + jz];
    const double* Qc = Q + (size_t)c * 4 * nn;
    const double rho = Qc[lane];
    const double p = pressure(ph, rho, Qc[nn + lane], Qc[2 * nn + lane], Qc[3 * nn + lane], z);
    const double th = p / (rho * ph.R) * pow(ph.p0 / p, ph.R_over_cp) - ph.theta;
    v = h * h * gtab[GTab::W * n + ix] * gtab[GTab::W * n + jz] * th * th;
  }
  v = wave_sum(v);
  if (lane == 0) part[c] = v;
}

__global__ __launch_bounds__(256) void k_loss_sum(const double* part, int C, double* out) {
  __shared__ double s[256];
  const int t = threadIdx.x;
  double v = 0.0;
  for (int c = t; c < C; c += 256) v += part[c];
  s[t] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) s[t] += s[t + w];
    __syncthreads();
  }
  if (t == 0) out[0] = sqrt(s[0]);
}

// lambda_Q = gL * dL/dQ = gL / L * h^2 w_i w_j (theta - theta_bg) dtheta/dQ
template <int n>
__global__ __launch_bounds__(kWave) void k_loss_adj(Phys ph, const double* Q, const double* geom, const double* gtab,
                                                      const double* L, const double* gL, double* lam) {
  constexpr int nn = n * n;
  const int c = blockIdx.x, lane = threadIdx.x;
  if (lane >= nn) return;
  const int jz = lane / n, ix = lane % n;
  const double h = geom[4 * c + 2];
  const double z = geom[4 * c + 1] + h * gtab[GTab::XI * n + jz];
  const double* Qc = Q + (size_t)c * 4 * nn;
  const double rho = Qc[lane], mx = Qc[nn + lane], mz = Qc[2 * nn + lane];
  const double p = pressure(ph, rho, mx, mz, Qc[3 * nn + lane], z);
  const double kap = ph.R_over_cp;
  const double th = p / (rho * ph.R) * pow(ph.p0 / p, kap);
  const double coef = gL[0] / L[0] * h * h * gtab[GTab::W * n + ix] * gtab[GTab::W * n + jz] * (th - ph.theta);
  // theta = (p0^kap / R) p^(1-kap) / rho
  const double dth_dp = (1.0 - kap) * th / p, dth_drho = -th / rho;
  const double u = mx / rho, w = mz / rho, geo = ph.gravity ? ph.g * z : 0.0;
  double* lc = lam + (size_t)c * 4 * nn;
  lc[lane] = coef * (dth_drho + dth_dp * ph.gm1 * (0.5 * (u * u + w * w) - geo));
  lc[nn + lane] = coef * dth_dp * (-ph.gm1 * u);
  lc[2 * nn + lane] = coef * dth_dp * (-ph.gm1 * w);
  lc[3 * nn + lane] = coef * dth_dp * ph.gm1;
}

// --------------------------------------------------------------- launchers
int launch_predictor_any(const Group& g, double* store, hipStream_t s);
int launch_corrector(const Group& g, hipStream_t s);

template <int n>
static int adj_n(const Group& g, AdjArgs a, hipStream_t s) {
  hipLaunchKernelGGL(k_face_adj<n>, dim3(g.C), dim3(kWave), 0, s, g.ph, a);
  hipLaunchKernelGGL(k_pred_adj<n>, dim3(g.C), dim3(kWave * adj_waves<n>()), 0, s, g.ph, a);
  return check_launch("step adjoint");
}

int launch_step_adjoint(const Group& g, const double* Qn, const double* lam_in, double* lam_out, double* store,
                        const double* fd, bool recompute, double* lamFD, hipStream_t s) {
  if (recompute) {
    // forward predictor from the checkpoint, keeping the iterates and the face data
    Group gf = g;
    gf.Q = const_cast<double*>(Qn);
    gf.FD = const_cast<double*>(fd);
    int rc = launch_predictor_any(gf, store, s);
    if (rc) return rc;
  }
  AdjArgs a;
  a.Qn = Qn; a.lam_in = lam_in; a.lam_out = lam_out; a.FD = fd; a.store = store;
  a.lamFD = lamFD; a.clock = g.clock; a.geom = g.d_geom; a.nbr = g.d_nbr; a.gtab = g.d_gtab;
  a.C = g.C; a.iters = g.iters;
  switch (g.n) {
    case 2: return adj_n<2>(g, a, s);
    case 3: return adj_n<3>(g, a, s);
    case 4: return adj_n<4>(g, a, s);
    case 5: return adj_n<5>(g, a, s);
    case 6: return adj_n<6>(g, a, s);
    case 7: return adj_n<7>(g, a, s);
    case 8: return adj_n<8>(g, a, s);
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
}

int launch_ic_theta(const Group& g, const double* thp, hipStream_t s) {
  const long long tot = (long long)g.C * g.n * g.n;
  if (!tot) return ADG_OK;
  hipLaunchKernelGGL(k_ic_theta, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g.ph, g.n, g.C, g.d_geom,
                     g.d_gtab, thp, g.Q);
  return check_launch("ic_theta");
}

int launch_ic_theta_adj(const Group& g, const double* thp, const double* lam, double* grad, hipStream_t s) {
  const long long tot = (long long)g.C * g.n * g.n;
  if (!tot) return ADG_OK;
  hipLaunchKernelGGL(k_ic_theta_adj, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g.ph, g.n, g.C,
                     g.d_geom, g.d_gtab, thp, lam, grad);
  return check_launch("ic_theta_adjoint");
}

template <int n>
static int loss_n(const Group& g, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_part<n>, dim3(g.C), dim3(kWave), 0, s, g.ph, g.Q, g.d_geom, g.d_gtab, part);
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, s, part, g.C, out);
  return check_launch("loss");
}
template <int n>
static int loss_adj_n(const Group& g, const double* L, const double* gL, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_adj<n>, dim3(g.C), dim3(kWave), 0, s, g.ph, g.Q, g.d_geom, g.d_gtab, L, gL, lam);
  return check_launch("loss adjoint");
}

int launch_loss(const Group& g, double* part, double* out, hipStream_t s) {
  switch (g.n) {
    case 2: return loss_n<2>(g, part, out, s);
    case 3: return loss_n<3>(g, part, out, s);
    case 4: return loss_n<4>(g, part, out, s);
    case 5: return loss_n<5>(g, part, out, s);
    case 6: return loss_n<6>(g, part, out, s);
    case 7: return loss_n<7>(g, part, out, s);
    case 8: return loss_n<8>(g, part, out, s);
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
}
int launch_loss_adj(const Group& g, const double* L, const double* gL, double* lam, hipStream_t s) {
  switch (g.n) {
    case 2: return loss_adj_n<2>(g, L, gL, lam, s);
    case 3: return loss_adj_n<3>(g, L, gL, lam, s);
    case 4: return loss_adj_n<4>(g, L, gL, lam, s);
    case 5: return loss_adj_n<5>(g, L, gL, lam, s);
    case 6: return loss_adj_n<6>(g, L, gL, lam, s);
    case 7: return loss_adj_n<7>(g, L, gL, lam, s);
    case 8: return loss_adj_n<8>(g, L, gL, lam, s);
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
}

}  // namespace adg
