// Space-time predictor for meshes too small to fill the chip with one
// wavefront per cell: one workgroup of n wavefronts per cell, wavefront b
// owning time level b.  The residuals of the n time levels of a Picard sweep
// are independent of each other; only the time matrix mixes them, through
// LDS and a workgroup barrier.  Same arithmetic as k_predictor (up to the
// order of the sums): strong-form residual with gradients in reference
// coordinates, X_b = Q + dt sum_a P[b][a] R_a, then the time averages, the
// volume term, Q* and the face data.
//
// Per level and node a lane holds 4 values of the iterate; contractions read
// n values of an LDS slice per output (state slice [4][n][n], fluxes
// [2][4][n][n] per level).  With n wavefronts per cell a 27x27 mesh of order
// 6 puts 5,103 wavefronts on the 1,024 SIMDs instead of 729.
#include "adg_internal.h"

namespace adg {

struct LvArgs {
  const double* Qin;   // [C][4][n][n]
  double* Qs;          // [C][4][n][n]
  double* FD;          // [C][4][2][4][n]
  const double* clock; // [S][4]
  const int* scen;     // [C] or null
  const double* geom;  // [C][4] x0, z0, h
  const double* gtab;
  double* iter_store;  // optional [C][iters][n][4][n][n]
  int C, iters;
};

template <int n>
__global__ __launch_bounds__(kWave * n) void k_predictor_lv(Phys ph, LvArgs a) {
  constexpr int nn = n * n, sl = 4 * nn;
  constexpr int nR = n > 3 ? n : 3;
  __shared__ double sR[nR * sl];        // scaled residuals of every level; level sums in the epilogue
  __shared__ double sW[n][3 * sl];      // per level: state slice [4][nn], fluxes [2][4][nn]
  const int c = blockIdx.x, b = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const bool node = lane < nn;
  const int l = node ? lane : 0;
  const int jz = l / n, ix = l % n;
  double* sq = sW[b];
  double* sF = sW[b] + sl;
  const double* gt = a.gtab;
  const int s = a.scen ? a.scen[c] : 0;
  const double t0 = a.clock[4 * s + 0], dt = a.clock[4 * s + 1];
  const double x0 = a.geom[4 * c + 0], z0 = a.geom[4 * c + 1], h = a.geom[4 * c + 2];
  const double ih = 1.0 / h, mu_h = ph.mu * ih, kappa_h = ph.kappa * ih, gh = ph.geff * h;
  const double sdt = -dt * ih;
  const double z = z0 + h * gt[GTab::XI * n + jz];
  double rb, pb;
  background(ph, z, rb, pb);
  double Di[n], Dj[n];
#pragma unroll
  for (int m = 0; m < n; ++m) {
    Di[m] = gt[GTab::d(n) + ix * n + m];
    Dj[m] = gt[GTab::d(n) + jz * n + m];
  }
  const double* Qc = a.Qin + (size_t)c * sl + l;
  double Q0[4], X[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) { Q0[v] = Qc[v * nn]; X[v] = Q0[v]; }
  // manufactured energy source at this level's time (it does not depend on the state)
  const double SE = ph.mms ? mms_source(ph, x0 + h * gt[GTab::XI * n + ix], z, t0 + gt[GTab::XI * n + b] * dt) : 0.0;

  // gradients (reference coordinates) of the slice in sq, then the flux
  auto grad_flux = [&](double Fx[4], double Fz[4]) {
    double gx[4], gz[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double ax = 0.0, az = 0.0;
#pragma unroll
      for (int m = 0; m < n; ++m) {
        ax = fma(Di[m], sq[v * nn + jz * n + m], ax);
        az = fma(Dj[m], sq[v * nn + m * n + ix], az);
      }
      gx[v] = ax; gz[v] = az;
    }
    double Sw;
    flux_source(ph, X, gx, gz, z, rb, pb, mu_h, kappa_h, gh, Fx, Fz, Sw);
    return Sw;
  };

  for (int it = 0; it < a.iters; ++it) {
    if (node)
#pragma unroll
      for (int v = 0; v < 4; ++v) sq[v * nn + l] = X[v];
    wave_sync();
    double Fx[4], Fz[4];
    const double Sw = grad_flux(Fx, Fz);
    if (node)
#pragma unroll
      for (int v = 0; v < 4; ++v) { sF[v * nn + l] = Fx[v]; sF[sl + v * nn + l] = Fz[v]; }
    wave_sync();
    if (node) {
      // scaled residual R' = div F - h S (reference divergence), R = -R'/h
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double d = 0.0;
#pragma unroll
        for (int m = 0; m < n; ++m) {
          d = fma(Di[m], sF[v * nn + jz * n + m], d);
          d = fma(Dj[m], sF[sl + v * nn + m * n + ix], d);
        }
        if (v == 2) d = fma(-h, Sw, d);
        if (v == 3 && ph.mms) d = fma(-h, SE, d);
        sR[b * sl + v * nn + l] = d;
      }
    }
    __syncthreads();
    // X_b = Q + dt sum_a P[b][a] R_a = Q - (dt/h) sum_a P[b][a] R'_a
    if (node) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < n; ++a2) acc = fma(gt[GTab::pt(n) + a2 * n + b], sR[a2 * sl + v * nn + l], acc);
        X[v] = fma(sdt, acc, Q0[v]);
      }
      if (a.iter_store) {
        double* st = a.iter_store + (((size_t)c * a.iters + it) * n + b) * sl;
#pragma unroll
        for (int v = 0; v < 4; ++v) st[v * nn + l] = X[v];
      }
    }
    __syncthreads();   // every level read the residuals before the next sweep writes them
  }

  // final pass: this level's weighted state, fluxes and sources
  if (node)
#pragma unroll
    for (int v = 0; v < 4; ++v) sq[v * nn + l] = X[v];
  wave_sync();
  double Fx[4], Fz[4];
  const double Sw = grad_flux(Fx, Fz);
  const double wb = gt[GTab::W * n + b];
  wave_sync();
  if (node) {
    // [state | x flux | z flux] of this level, weighted, in its own region;
    // the sources in the residual area
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sW[b][v * nn + l] = wb * X[v];
      sW[b][sl + v * nn + l] = wb * Fx[v];
      sW[b][2 * sl + v * nn + l] = wb * Fz[v];
    }
    sR[b * sl + l] = wb * Sw;
    sR[b * sl + nn + l] = wb * SE;
  }
  __syncthreads();
  if (b != 0) return;

  // level sums (fixed order), by the first wavefront: averaged state and
  // fluxes to the residual area as [state | x flux | z flux]
  double Qb[4], Sbw = 0.0, SbE = 0.0;
  double Fbx[4], Fbz[4];
  if (node) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double q = 0.0, fx = 0.0, fz = 0.0;
#pragma unroll
      for (int k = 0; k < n; ++k) {
        q += sW[k][v * nn + l];
        fx += sW[k][sl + v * nn + l];
        fz += sW[k][2 * sl + v * nn + l];
      }
      Qb[v] = q; Fbx[v] = fx; Fbz[v] = fz;
    }
#pragma unroll
    for (int k = 0; k < n; ++k) { Sbw += sR[k * sl + l]; SbE += sR[k * sl + nn + l]; }
  }
  wave_sync();
  double* sA = sR;   // [state | x flux | z flux], 3 sl
  if (node)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sA[v * nn + l] = Qb[v];
      sA[sl + v * nn + l] = Fbx[v];
      sA[2 * sl + v * nn + l] = Fbz[v];
    }
  wave_sync();
  if (node) {
    // volume term with Dw[i][m] = w_m D[m][i] / w_i along x and z, and Q*
    double* qs = a.Qs + (size_t)c * sl;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double vol = 0.0;
#pragma unroll
      for (int m = 0; m < n; ++m) {
        vol = fma(gt[GTab::dw(n) + ix * n + m], sA[sl + v * nn + jz * n + m], vol);
        vol = fma(gt[GTab::dw(n) + jz * n + m], sA[2 * sl + v * nn + m * n + ix], vol);
      }
      const double S = (v == 2) ? Sbw : (v == 3 ? SbE : 0.0);
      qs[v * nn + l] = Q0[v] + dt * (vol * ih + S);
    }
  }
  // face data: lane = (direction, variable, line) extrapolates the averaged
  // state and the normal flux of its line to both faces
  if (lane < 8 * n) {
    const int dir = lane / (4 * n), v = (lane % (4 * n)) / n, line = lane % n;
    const int base = v * nn + (dir == 0 ? line * n : line), stride = dir == 0 ? 1 : n;
    const double* fl = sA + (dir == 0 ? sl : 2 * sl);
    double q0 = 0, q1 = 0, f0 = 0, f1 = 0;
#pragma unroll
    for (int m = 0; m < n; ++m) {
      const double e0 = gt[GTab::E0 * n + m], e1 = gt[GTab::E1 * n + m];
      const double iq = sA[base + m * stride], iF = fl[base + m * stride];
      q0 = fma(e0, iq, q0); q1 = fma(e1, iq, q1);
      f0 = fma(e0, iF, f0); f1 = fma(e1, iF, f1);
    }
    double* fd = a.FD + (size_t)c * 32 * n;
    const int flo = 2 * dir, fhi = 2 * dir + 1;
    fd[((flo * 2 + 0) * 4 + v) * n + line] = q0;
    fd[((flo * 2 + 1) * 4 + v) * n + line] = f0;
    fd[((fhi * 2 + 0) * 4 + v) * n + line] = q1;
    fd[((fhi * 2 + 1) * 4 + v) * n + line] = f1;
  }
}

template <int n>
static int lv_n(const Phys& ph, const LvArgs& a, hipStream_t s) {
  if (a.C == 0) return ADG_OK;
  hipLaunchKernelGGL(k_predictor_lv<n>, dim3(a.C), dim3(kWave * n), 0, s, ph, a);
  return check_launch("predictor (levels)");
}

int launch_predictor_levels(const Group& g, double* store, hipStream_t s) {
  LvArgs a;
  a.Qin = g.Q; a.Qs = g.Qs; a.FD = g.FD; a.clock = g.clock; a.scen = g.d_scen; a.geom = g.d_geom;
  a.gtab = g.d_gtab; a.iter_store = store; a.C = g.C; a.iters = g.iters;
  switch (g.n) {
    case 2: return lv_n<2>(g.ph, a, s);
    case 3: return lv_n<3>(g.ph, a, s);
    case 4: return lv_n<4>(g.ph, a, s);
    case 5: return lv_n<5>(g.ph, a, s);
    case 6: return lv_n<6>(g.ph, a, s);
    case 7: return lv_n<7>(g.ph, a, s);
    case 8: return lv_n<8>(g.ph, a, s);
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
}

}  // namespace adg
