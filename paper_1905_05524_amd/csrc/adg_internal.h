// Internal definitions of the gfx950 ADER-DG library: constant tables,
// physics parameters in kernel-argument form, the mesh handle, and the
// pointwise physics as device functions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "adg.h"

namespace adg {

constexpr int kMaxN = 8;          // nodes per direction supported (order 7)
// the predictor runs a wavefront per time level while that puts at most this
// many wavefronts on the chip (three per SIMD): cells * n <= kLevelsWaves
constexpr int kLevelsWaves = 3072;
constexpr int kWave = 64;         // CDNA wavefront size

// Basis tables for n nodes, passed by value as a kernel argument so that every
// entry read with a compile-time index becomes a scalar (SGPR) operand.
template <int n>
struct Tab {
  double D[n][n];    // D[i][m] = phi_m'(xi_i)
  double P[n][n];    // time predictor matrix K1^{-1} W
  double Dw[n][n];   // volume term: Dw[i][m] = w_m D[m][i] / w_i
  double w[n];
  double e0[n], e1[n];
};

// Tables in global memory (one per handle), read with lane-dependent or
// runtime indices:
//   xi[n], w[n], L0[n] = e0/w, L1[n] = e1/w, e0[n], e1[n],
//   Pk[3][n][n]  sub-face k prolongation phi_m((k+xi_q)/3) at [k][q][m],
//   Rk[3][n][n]  restriction (w_q/3) phi_m((k+xi_q)/3)/w_m at [k][m][q],
//   D[n][n], Pt[n][n] (time matrix transposed: Pt[b][a] = P[a][b]), Dw[n][n],
//   even-odd forms of D and Dw (see EvenOdd below),
//   LU[n*n+n]: the time matrix K1 = L U (unit lower L, no pivoting: for
//   Gauss-Legendre nodes the factors stay bounded, |U_ii| >= 1 up to n = 8)
//   stored in the order the in-place solve of K1 y = W r reads it: for each
//   row i, w_i then L[i][0..i-1]; then for each row i from n-1 down to 0,
//   1/U_ii then U[i][i+1..n-1]/U_ii.
struct GTab {
  static constexpr int XI = 0, W = 1, L0 = 2, L1 = 3, E0 = 4, E1 = 5;
  static __host__ __device__ inline int pk(int n) { return 6 * n; }
  static __host__ __device__ inline int rk(int n) { return 6 * n + 3 * n * n; }
  static __host__ __device__ inline int d(int n) { return 6 * n + 6 * n * n; }
  static __host__ __device__ inline int pt(int n) { return 6 * n + 7 * n * n; }
  static __host__ __device__ inline int dw(int n) { return 6 * n + 8 * n * n; }
  static __host__ __device__ inline int eo_size(int n) { return 2 * (n / 2) * (n / 2) + 2 * (n / 2); }
  static __host__ __device__ inline int eo_d(int n) { return 6 * n + 9 * n * n; }
  static __host__ __device__ inline int eo_dw(int n) { return 6 * n + 9 * n * n + eo_size(n); }
  static __host__ __device__ inline int lu(int n) { return 6 * n + 9 * n * n + 2 * eo_size(n); }
  static __host__ __device__ inline int size(int n) { return 7 * n + 10 * n * n + 2 * eo_size(n); }
};

// Even-odd form of an n x n matrix T with T[n-1-i][n-1-m] = -T[i][m] (the
// Gauss-Legendre derivative matrix and the volume matrix are centro-
// antisymmetric), h = n/2, mid = (n-1)/2 for odd n:
//   A[i][m] = (T[i][m] - T[i][n-1-m]) / 2,  B[i][m] = (T[i][m] + T[i][n-1-m]) / 2
//   (i, m < h), C[i] = T[i][mid], M[m] = T[mid][m] (odd n only).
// With e_m = x_m + x_{n-1-m}, o_m = x_m - x_{n-1-m}: S_i = sum_m A[i][m] o_m,
// T_i = sum_m B[i][m] e_m + C[i] x_mid, (T x)_i = S_i + T_i,
// (T x)_{n-1-i} = S_i - T_i, (T x)_mid = sum_m M[m] o_m.  Stored as
// A[h][h], B[h][h], C[h], M[h].

struct Phys {
  double gamma, gm1, R, iR, cp, Pr, mu, kappa, g, p0, theta;
  double cp_over_R, R_over_cp, ex_coef;   // ex_coef = g/(cp theta)
  double lv_coef;                         // lambda_v = lv_coef / rho
  double mms_amp, mms_u, mms_w, mms_kx, mms_kz, mms_p;
  double cfl;
  double geff;                            // g with gravity on, 0 otherwise
  int gravity, mms, fixed_dt, N;
};

enum FaceKind { kConforming = 0, kWall = 1, kFineSide = 2, kCoarseSide = 3 };

// Everything a kernel launch needs for one set of cells of one order: the
// cells of one mesh, or of all scenarios of one order in a batch.
struct Group {
  int n = 0, N = 0, iters = 0, C = 0;
  Phys ph{};
  // handle-owned device tables
  double* d_geom = nullptr;   // [C][4] x0, z0, h, 0
  int* d_nbr = nullptr;       // [C][4 faces][4] kind, a, b, c (cell indices local to the group)
  double* d_gtab = nullptr;   // GTab layout
  int* d_scen = nullptr;      // [C] scenario index into clock (NULL: all 0)
  // caller-owned buffers bound by set_state
  double* Q = nullptr;        // [C][4][n][n]
  double* Qs = nullptr;       // [C][4][n][n]
  double* FD = nullptr;       // [C][4][2][4][n]
  double* dtc = nullptr;      // [C]
  double* clock = nullptr;    // [S][4]
  // launch shape: cells per wavefront, wavefronts per workgroup
  int cpw = 1, wpb = 1;
  // predictor kernel: -1 automatic (the time-level predictor while cells * n
  // <= kLevelsWaves, or over four wavefronts per cell while cells * 4 <=
  // kLevelsWaves), 0 one wavefront per cell, 1 the time-level predictor
  int lv = -1;
  // wavefronts per cell of the time-level predictor: 2 or 4 spread the n
  // time nodes over that many wavefronts (when fewer than n), else n
  int lw = 0;
  // handle-owned scratch of the TV statistics over many cells: per-workgroup
  // partials (count, mean, M2) and the thresholds (kTvPartDoubles doubles)
  double* d_part = nullptr;
  // corrector launches: a clock the corrector advances itself (frozen time
  // step, one mesh), or NULL
  double* advance = nullptr;
  int nc = 0;                 // the mesh has 1:3 non-conforming faces
};

// TV statistics over many cells: at most kStatParts per-workgroup partials
constexpr int kStatParts = 512;
constexpr int kTvPartDoubles = 3 * kStatParts + 3;

// wavefronts per cell the time-level predictor of g launches
inline int level_waves(const Group& g) { return (g.lw == 2 || g.lw == 4) && g.lw < g.n ? g.lw : g.n; }

// Host copies of the basis of one order.
struct HostBasis {
  int n = 0;
  std::vector<double> xi, w, D, P, Dw, e0, e1, gtab;
};

// Leaves by (level, i, j) on a mesh of nx x nz coarse cells with levels
// 0..L: one dense table per level while the boxes of all levels number at
// most kDenseBoxes (16 MB of ints), else a hash map keyed by the same box
// number (unique: nx * nz <= 2^26 coarse cells and L <= 8 give fewer than
// 2^62 boxes).  Lookups outside the grid of their level find nothing.
struct LeafIndex {
  static constexpr long long kDenseBoxes = 1LL << 22;
  int nx, nz, L;
  bool dense = false;
  std::vector<long long> off;   // per level: start of its table
  std::vector<int> tab;
  std::unordered_map<long long, int> map;
  LeafIndex(int nx_, int nz_, int L_, size_t n_leaves) : nx(nx_), nz(nz_), L(L_), off(L_ + 1, 0) {
    long long total = 0, s = 1;
    for (int l = 0; l <= L; ++l, s *= 3) {
      off[l] = total;
      total += (long long)nx * s * nz * s;
    }
    dense = total <= kDenseBoxes;
    if (dense) tab.assign((size_t)total, -1);
    else map.reserve(n_leaves * 2);
  }
  bool in_grid(int l, int i, int j) const {
    if (l < 0 || l > L || i < 0 || j < 0) return false;
    long long s = 1;
    for (int k = 0; k < l; ++k) s *= 3;
    return i < nx * s && j < nz * s;
  }
  long long slot(int l, int i, int j) const {
    long long s = 1;
    for (int k = 0; k < l; ++k) s *= 3;
    return off[l] + (long long)j * nx * s + i;
  }
  // records leaf c at (l, i, j); false if the box is outside the grid or
  // holds a leaf already
  bool insert(int l, int i, int j, int c) {
    if (!in_grid(l, i, j)) return false;
    if (!dense) return map.emplace(slot(l, i, j), c).second;
    int& t = tab[(size_t)slot(l, i, j)];
    if (t >= 0) return false;
    t = c;
    return true;
  }
  int find(int l, int i, int j) const {
    if (!in_grid(l, i, j)) return -1;
    if (!dense) {
      auto it = map.find(slot(l, i, j));
      return it == map.end() ? -1 : it->second;
    }
    return tab[(size_t)slot(l, i, j)];
  }
};

// Host mesh: leaves, geometry and face table.
struct HostMesh {
  int C = 0;
  std::vector<int> lev, ci, cj;
  std::vector<double> geom;   // [C][4]
  std::vector<int> nbr;       // [C][16]
};

}  // namespace adg

struct adg_mesh {
  adg_params prm;
  // device the handle's tables live on, and that device's static scratch
  // (device address, resolved at init; NULL if the lookup failed)
  int dev = 0;
  void* static_scratch = nullptr;
  int static_scratch_rc = 0;
  adg_mesh_desc desc{};
  adg::HostBasis basis;
  adg::HostMesh hm;
  adg::Group g;
  // bound (caller-owned)
  double* Q = nullptr;
  void* ws = nullptr;
  double* clock = nullptr;
  // workspace partition (byte offsets)
  size_t off_qs = 0, off_fd = 0, off_dtc = 0, off_health = 0, ws_bytes = 0;
  // pending regrid (from adg_regrid_plan): new leaves, transfer operations
  // and the new mesh tables
  bool plan_ready = false;
  std::vector<int> plan_lev, plan_ci, plan_cj, plan_ops;
  adg::HostMesh plan_mesh;
  // grow-only device buffers of the regrid: transfer operations (ints) and
  // the capacity, in cells, of the geometry and neighbour tables
  int* d_ops = nullptr;
  size_t ops_cap = 0;
  int cells_cap = 0;
  // pinned host staging of the regrid's uploads (grow-only, bytes)
  void* h_stage = nullptr;
  size_t stage_cap = 0;
};

namespace adg {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int check_launch(const char* what);

// Gauss-Legendre basis of n nodes and its device tables (computed in long
// double, stored in double).
void build_basis(int n, HostBasis& B);
// persistent predictor of one order group (k_predictor's body on work items
// from counter [2], nwaves resident wavefronts), and its resident
// wavefronts per CU
int launch_predictor_queue(const Group& g, unsigned* counter, int nwaves, hipStream_t s);
int predictor_queue_occupancy(int n, int* per_cu);
// device address of the allocation-free step's static scratch on device dev
// (the current device); looked up once per device
int static_scratch_address(int dev, void** ptr);
// parameter checks shared by the 2D and 3D handles
int validate_params(const adg_params* p);
Phys make_phys(const adg_params& p);

template <int n>
inline Tab<n> tab_of(const HostBasis& B) {
  Tab<n> T;
  for (int i = 0; i < n; ++i) {
    T.w[i] = B.w[i]; T.e0[i] = B.e0[i]; T.e1[i] = B.e1[i];
    for (int j = 0; j < n; ++j) {
      T.D[i][j] = B.D[i * n + j]; T.P[i][j] = B.P[i * n + j]; T.Dw[i][j] = B.Dw[i * n + j];
    }
  }
  return T;
}

// wavefront-scope barrier for LDS hand-offs between lanes of one wavefront:
// LDS operations of a wavefront execute in order, so a compiler fence and a
// wave barrier are enough.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- physics
// Hydrostatic background of constant potential temperature:
// Exner pi = 1 - g z/(cp theta), p = p0 pi^(cp/R), rho = p/(R theta pi).
__device__ inline void background(const Phys& ph, double z, double& rb, double& pb) {
  if (!ph.gravity) { rb = 0.0; pb = 0.0; return; }
  double pi = 1.0 - ph.ex_coef * z;
  pb = ph.p0 * pow(pi, ph.cp_over_R);
  rb = pb / (ph.R * ph.theta * pi);
}

__device__ inline double pressure(const Phys& ph, double rho, double mx, double mz, double E, double z) {
  const double geo = rho * (ph.geff * z);   // 0 without gravity
  return ph.gm1 * (E - 0.5 * (mx * mx + mz * mz) / rho - geo);
}

// Energy source of the manufactured advected density wave (T = p/(R rho),
// S_E = -kappa Lap T).
__device__ inline double mms_source(const Phys& ph, double x, double z, double t) {
  double X = x - ph.mms_u * t, Z = z - ph.mms_w * t;
  double sx, cx, sz, cz;
  sincos(ph.mms_kx * X, &sx, &cx);
  sincos(ph.mms_kz * Z, &sz, &cz);
  double rho = 1.0 + ph.mms_amp * sx * sz;
  double rx = ph.mms_amp * ph.mms_kx * cx * sz;
  double rz = ph.mms_amp * ph.mms_kz * sx * cz;
  double lap = -(ph.mms_kx * ph.mms_kx + ph.mms_kz * ph.mms_kz) * ph.mms_amp * sx * sz;
  double ir = 1.0 / rho;
  double lapT = ph.mms_p * ph.iR * (-lap * ir * ir + 2.0 * (rx * rx + rz * rz) * ir * ir * ir);
  return -ph.kappa * lapT;
}

// The paper's manufactured solution (CFD scenarios, eq.
// manufactured-solution): with phase xi = k (x + z) - om t, k = pi/5,
// om = 2 pi, the fields rho = 1 + sin(xi)/2, p = 1/gamma + cos(xi)/10,
// u = w = sin(xi)/4 depend on xi alone; d/dx = d/dz = k d/dxi and
// d/dt = -om d/dxi.
constexpr double kWaveK = 0.62831853071795864769;   // pi / 5
constexpr double kWaveOm = 6.28318530717958647693;  // 2 pi
__device__ inline void paper_wave_state(const Phys& ph, double x, double z, double t, double q[4]) {
  double sn, cs;
  sincos(kWaveK * (x + z) - kWaveOm * t, &sn, &cs);
  const double rho = 1.0 + 0.5 * sn, p = 1.0 / ph.gamma + 0.1 * cs, u = 0.25 * sn;
  q[0] = rho; q[1] = rho * u; q[2] = rho * u;
  q[3] = p / ph.gm1 + rho * u * u;
}
// Source that makes the wave solve the equation set without gravity,
// S = dQ/dt + div F, from the derivatives of the fields along xi (primes):
// the stress tensor gives sigma_xx = sigma_zz = -(2/3) mu k u',
// sigma_xz = -2 mu k u'; the heat flux -kappa k T' with T = p/(R rho), whose
// second derivative follows from differentiating R rho T = p twice.
__device__ inline void paper_wave_source(const Phys& ph, double x, double z, double t, double S[4]) {
  constexpr double k = kWaveK, om = kWaveOm;
  double sn, cs;
  sincos(k * (x + z) - om * t, &sn, &cs);
  const double rho = 1.0 + 0.5 * sn, r1 = 0.5 * cs, r2 = -0.5 * sn;
  const double p = 1.0 / ph.gamma + 0.1 * cs, p1 = -0.1 * sn, p2 = -0.1 * cs;
  const double u = 0.25 * sn, u1 = 0.25 * cs, u2 = -0.25 * sn;
  const double ir = 1.0 / rho;
  const double m1 = r1 * u + rho * u1;                 // (rho u)'
  const double mu1 = u * (r1 * u + 2.0 * rho * u1);    // (rho u^2)'
  const double E = p / ph.gm1 + rho * u * u, E1 = p1 / ph.gm1 + mu1;
  const double H1 = u1 * (E + p) + u * (E1 + p1);      // (u (E + p))'
  const double T = p * ir * ph.iR;
  const double T1 = (p1 * ph.iR - r1 * T) * ir;
  const double T2 = (p2 * ph.iR - r2 * T - 2.0 * r1 * T1) * ir;
  const double kk = k * k;
  S[0] = 2.0 * k * m1 - om * r1;
  S[1] = k * (2.0 * mu1 + p1) - om * m1 - (8.0 / 3.0) * ph.mu * kk * u2;
  S[2] = S[1];
  S[3] = 2.0 * k * H1 - om * E1 - (16.0 / 3.0) * ph.mu * kk * (u1 * u1 + u * u2) - 2.0 * ph.kappa * kk * T2;
}

// Reciprocal of a positive normal double: the hardware estimate refined by
// two Newton steps r <- r + r (1 - x r) (quadratic convergence; the result
// is within an ulp or so of 1/x, not necessarily correctly rounded).
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Flux (hyperbolic + viscous) in x and z and the gravity source of the
// vertical momentum at one node (eqs. equation-set, eos, temperature,
// stress-tensor, heat-conduction-coeff, momentum-equation-split).
// q: conserved state; gx, gz: its gradients in reference coordinates, i.e.
// h times the physical ones.  Every gradient enters the flux linearly through
// the stress and the heat flux, so the 1/h is carried by mu_h = mu / h and
// kappa_h = kappa / h, and the hydrostatic term of the vertical pressure
// gradient by gh = g h (0 without gravity).  rb, pb: background density and
// pressure at the node height z.
__device__ inline void flux_source(const Phys& ph, const double q[4], const double gx[4],
                                   const double gz[4], double z, double rb, double pb, double mu_h,
                                   double kappa_h, double gh, double Fx[4], double Fz[4], double& Sw) {
  const double rho = q[0], mx = q[1], mz = q[2], E = q[3];
  const double ir = recip(rho);
  const double u = mx * ir, w = mz * ir;
  // branch-free in the gravity switch: geff = gh = 0 and rb = pb = 0 without it
  const double gzz = ph.geff * z;
  const double p = ph.gm1 * (E - 0.5 * (mx * u + mz * w) - rho * gzz);
  const double pm = p - pb;
  const double T = p * ir * ph.iR;
  const double dux = (gx[1] - u * gx[0]) * ir, duz = (gz[1] - u * gz[0]) * ir;
  const double dwx = (gx[2] - w * gx[0]) * ir, dwz = (gz[2] - w * gz[0]) * ir;
  const double hv2 = 0.5 * (u * u + w * w) + gzz;
  const double dpx = ph.gm1 * (gx[3] - hv2 * gx[0] - rho * (u * dux + w * dwx));
  const double dpz = ph.gm1 * (gz[3] - hv2 * gz[0] - rho * (u * duz + w * dwz) - rho * gh);
  const double dTx = (dpx - ph.R * T * gx[0]) * ir * ph.iR;
  const double dTz = (dpz - ph.R * T * gz[0]) * ir * ph.iR;
  const double div = dux + dwz;
  const double sxx = mu_h * ((2.0 / 3.0) * div - 2.0 * dux);
  const double szz = mu_h * ((2.0 / 3.0) * div - 2.0 * dwz);
  const double sxz = -mu_h * (duz + dwx);
  const double H = E + p;
  Fx[0] = mx;
  Fx[1] = mx * u + pm + sxx;
  Fx[2] = mz * u + sxz;
  Fx[3] = u * H + u * sxx + w * sxz - kappa_h * dTx;
  Fz[0] = mz;
  Fz[1] = mx * w + sxz;
  Fz[2] = mz * w + pm + szz;
  Fz[3] = w * H + u * sxz + w * szz - kappa_h * dTz;
  Sw = -ph.geff * (rho - rb);
}

// max over the 64 lanes of a wavefront (butterfly, fixed order)
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

}  // namespace adg
