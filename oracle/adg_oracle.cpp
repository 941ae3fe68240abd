// Plain, slow FP64 CPU oracle for one ADER-DG step of 2D compressible
// Navier-Stokes with gravity, and for the total-variation refinement
// indicator.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
// CPU-baseline leg of the benchmark may load it; the product path never does.
//
// It shares no code with the GPU library: its own quadrature, its own
// matrices, its own mesh/face search, its own physics.  Every routine follows
// the paper (Krenz, Rannabauer, Bader, arXiv:1905.05524) or, where the paper
// delegates the scheme to cited works, the reading of the method stated next
// to it.  Loops are written in the order of the definitions, with no blocking
// or fusion.  Compiled with -O2 -ffp-contract=off and no fast-math.
//
// Scalar type is a template parameter so that the same code runs on doubles
// and on forward-mode dual numbers (used for exact directional derivatives of
// a multi-step rollout, the reference for the hand-written adjoint).
//
// Conventions
//   reference element [0,1]^2, Gauss-Legendre (GL) nodes xi_0..xi_N, n=N+1
//   Q[cell][var][jz][ix], var = (rho, rho*u, rho*w, rho*E)
//   node coordinates x = x0 + h*xi_ix, z = z0 + h*xi_jz
//   face f: 0 = -x side, 1 = +x side, 2 = -z side, 3 = +z side
//   face data FD[cell][f][0=Qbar,1=Fbar][var][k] (k: tangential node)
//   fluxes at faces are always the flux in the +axis direction
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <utility>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- dual numbers
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline Dual fabs(Dual a) { return a.v > 0 ? a : (a.v < 0 ? -a : Dual(0.0, 0.0)); }
inline Dual pow(Dual a, double e) {
  double p = std::pow(a.v, e);
  return Dual(p, e * std::pow(a.v, e - 1.0) * a.d);
}
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
using std::sqrt; using std::fabs; using std::pow;

// -------------------------------------------------------------------- params
// Flat parameter vector (indices shared with the Python wrapper of this file).
enum {
  P_N = 0, P_PICARD, P_GAMMA, P_PR, P_R, P_CP, P_MU, P_G, P_P0, P_THETA,
  P_GRAVITY, P_MMS, P_MMS_AMP, P_MMS_U, P_MMS_W, P_MMS_KX, P_MMS_KZ, P_MMS_P,
  P_CFL, P_COUNT
};

struct Params {
  int N, n, iters;
  double gamma, Pr, R, cp, mu, g, p0, theta_bg;
  bool gravity;
  int mms;   // manufactured source: 0 none, 1 advected density wave, 2 the paper's wave
  double mms_amp, mms_u, mms_w, mms_kx, mms_kz, mms_p;
  double cfl;
  double kappa;
};

Params read_params(const double* p) {
  Params P;
  P.N = (int)p[P_N]; P.n = P.N + 1;
  P.iters = (int)p[P_PICARD]; if (P.iters <= 0) P.iters = P.N + 1;
  P.gamma = p[P_GAMMA]; P.Pr = p[P_PR]; P.R = p[P_R]; P.cp = p[P_CP];
  P.mu = p[P_MU]; P.g = p[P_G]; P.p0 = p[P_P0]; P.theta_bg = p[P_THETA];
  P.gravity = p[P_GRAVITY] != 0.0; P.mms = (int)p[P_MMS];
  P.mms_amp = p[P_MMS_AMP]; P.mms_u = p[P_MMS_U]; P.mms_w = p[P_MMS_W];
  P.mms_kx = p[P_MMS_KX]; P.mms_kz = p[P_MMS_KZ]; P.mms_p = p[P_MMS_P];
  P.cfl = p[P_CFL];
  // heat conductivity kappa = mu*cp/Pr (paper, eq. heat-conduction-coeff)
  P.kappa = P.mu * P.cp / P.Pr;
  return P;
}

// --------------------------------------------------------------------- basis
// Gauss-Legendre nodes and weights on [0,1], Newton on the Legendre
// polynomial P_n in long double, then the Lagrange nodal basis on them.
struct Basis {
  int n;
  std::vector<double> xi, w, D, e0, e1, P;  // D[i*n+j] = phi_j'(xi_i)
};

void legendre(int n, long double x, long double& pn, long double& dpn) {
  long double p0 = 1.0L, p1 = x;
  if (n == 0) { pn = 1.0L; dpn = 0.0L; return; }
  for (int k = 2; k <= n; ++k) {
    long double pk = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
    p0 = p1; p1 = pk;
  }
  pn = p1;
  dpn = n * (x * p1 - p0) / (x * x - 1.0L);
}

long double lagrange(const std::vector<long double>& X, int j, long double x) {
  long double r = 1.0L;
  for (int m = 0; m < (int)X.size(); ++m)
    if (m != j) r *= (x - X[m]) / (X[j] - X[m]);
  return r;
}

Basis make_basis(int N) {
  Basis B; int n = N + 1; B.n = n;
  const long double PI = 3.141592653589793238462643383279502884L;
  std::vector<long double> X(n), W(n);
  for (int k = 0; k < n; ++k) {
    // k-th root of P_n on [-1,1] in decreasing order, mapped increasing below
    long double x = std::cos(PI * (k + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      long double pn, dpn; legendre(n, x, pn, dpn);
      long double dx = pn / dpn; x -= dx;
      if (std::fabs(dx) < 1e-30L) break;
    }
    long double pn, dpn; legendre(n, x, pn, dpn);
    long double wk = 2.0L / ((1.0L - x * x) * dpn * dpn);
    X[n - 1 - k] = (x + 1.0L) / 2.0L;
    W[n - 1 - k] = wk / 2.0L;
  }
  B.xi.resize(n); B.w.resize(n);
  for (int k = 0; k < n; ++k) { B.xi[k] = (double)X[k]; B.w[k] = (double)W[k]; }
  // derivative matrix D_ij = phi_j'(xi_i), from the product form of phi_j
  B.D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long double s = 0.0L;
      for (int m = 0; m < n; ++m) {
        if (m == j) continue;
        long double term = 1.0L / (X[j] - X[m]);
        for (int l = 0; l < n; ++l)
          if (l != j && l != m) term *= (X[i] - X[l]) / (X[j] - X[l]);
        s += term;
      }
      B.D[i * n + j] = (double)s;
    }
  B.e0.resize(n); B.e1.resize(n);
  for (int j = 0; j < n; ++j) {
    B.e0[j] = (double)lagrange(X, j, 0.0L);
    B.e1[j] = (double)lagrange(X, j, 1.0L);
  }
  // Space-time predictor matrices: the weak form of d/dtau on [0,1] with the
  // upwind value at tau=0 gives K1 q = e0 Q^n + dt W R, where
  //   K1_ab = phi_a(1) phi_b(1) - w_b phi_a'(tau_b).
  // Because K1 * 1 = e0, q = Q^n + dt K1^{-1} W R; P = K1^{-1} W.
  std::vector<long double> K(n * n), Pm(n * n);
  std::vector<long double> E0(n), E1(n), DD(n * n);
  for (int j = 0; j < n; ++j) { E0[j] = lagrange(X, j, 0.0L); E1[j] = lagrange(X, j, 1.0L); }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long double s = 0.0L;
      for (int m = 0; m < n; ++m) {
        if (m == j) continue;
        long double term = 1.0L / (X[j] - X[m]);
        for (int l = 0; l < n; ++l)
          if (l != j && l != m) term *= (X[i] - X[l]) / (X[j] - X[l]);
        s += term;
      }
      DD[i * n + j] = s;
    }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      K[a * n + b] = E1[a] * E1[b] - W[b] * DD[b * n + a];
  // Solve K * Pm = diag(W) by Gauss-Jordan with partial pivoting.
  std::vector<long double> A(K), Rhs(n * n, 0.0L);
  for (int a = 0; a < n; ++a) Rhs[a * n + a] = W[a];
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
    if (piv != col)
      for (int c = 0; c < n; ++c) {
        std::swap(A[piv * n + c], A[col * n + c]);
        std::swap(Rhs[piv * n + c], Rhs[col * n + c]);
      }
    long double d = A[col * n + col];
    for (int c = 0; c < n; ++c) { A[col * n + c] /= d; Rhs[col * n + c] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      long double f = A[r * n + col];
      if (f == 0.0L) continue;
      for (int c = 0; c < n; ++c) {
        A[r * n + c] -= f * A[col * n + c];
        Rhs[r * n + c] -= f * Rhs[col * n + c];
      }
    }
  }
  B.P.resize(n * n);
  for (int k = 0; k < n * n; ++k) B.P[k] = (double)Rhs[k];
  return B;
}

// Lagrange basis of B evaluated at an arbitrary point (long double product).
double phi_at(const Basis& B, int j, double x) {
  std::vector<long double> X(B.xi.begin(), B.xi.end());
  return (double)lagrange(X, j, (long double)x);
}

// ---------------------------------------------------------------- background
// Hydrostatic background of constant potential temperature theta_bg
// (paper eq. hydrostatic-balance, potential temperature definition):
//   Exner pi(z) = 1 - g z / (cp theta), p = p0 pi^(cp/R), T = theta pi,
//   rho = p / (R T).   d p/dz = -g rho holds exactly.
void background(const Params& P, double z, double& rho_b, double& p_b) {
  if (!P.gravity) { rho_b = 0.0; p_b = 0.0; return; }
  double pi = 1.0 - P.g * z / (P.cp * P.theta_bg);
  p_b = P.p0 * std::pow(pi, P.cp / P.R);
  rho_b = p_b / (P.R * P.theta_bg * pi);
}

// Manufactured energy source for the advected density wave
//   rho = 1 + A sin(kx X) sin(kz Z), X = x - u t, Z = z - w t, v = (u, w), p const:
// the Euler part is solved exactly, the heat flux -kappa grad T with
// T = p/(R rho) leaves S_E = -kappa Lap T.
double mms_source_E(const Params& P, double x, double z, double t) {
  double X = x - P.mms_u * t, Z = z - P.mms_w * t;
  double sx = std::sin(P.mms_kx * X), cx = std::cos(P.mms_kx * X);
  double sz = std::sin(P.mms_kz * Z), cz = std::cos(P.mms_kz * Z);
  double rho = 1.0 + P.mms_amp * sx * sz;
  double rx = P.mms_amp * P.mms_kx * cx * sz;
  double rz = P.mms_amp * P.mms_kz * sx * cz;
  double lap = -(P.mms_kx * P.mms_kx + P.mms_kz * P.mms_kz) * P.mms_amp * sx * sz;
  double lapT = (P.mms_p / P.R) * (-lap / (rho * rho) + 2.0 * (rx * rx + rz * rz) / (rho * rho * rho));
  return -P.kappa * lapT;
}

// Manufactured solution of the convergence test (paper, CFD scenarios, eq.
// manufactured-solution, with the CFD constants gamma = 1.4, Pr = 0.7,
// c_v = 1): every field depends on xi = k (x + z) - 2 pi t, k = pi/5,
//   p = 1/gamma + (1/10) cos xi,  rho = 1 + (1/2) sin xi,
//   (u, w) = (1/4, 1/4) sin xi,   E = p/(gamma-1) + rho (u^2 + w^2)/2,
// on the periodic square [0,10]^2 (one period along each axis).
void paper_mms_state(const Params& P, double x, double z, double t, double q[4]) {
  const double PI = 3.14159265358979323846;
  const double xi = (PI / 5.0) * (x + z) - 2.0 * PI * t;
  const double sn = std::sin(xi), cs = std::cos(xi);
  const double p = 1.0 / P.gamma + 0.1 * cs, rho = 1.0 + 0.5 * sn, u = 0.25 * sn;
  q[0] = rho; q[1] = rho * u; q[2] = rho * u;
  q[3] = p / (P.gamma - 1.0) + rho * u * u;
}

// Its source S = dQ/dt + div F(Q, grad Q) of the equation set without
// gravity (eq. equation-set with the stress tensor and the heat flux),
// worked out along xi: d/dx = d/dz = k d/dxi, d/dt = -omega d/dxi
// (omega = 2 pi), primes are d/dxi, s = sin xi, c = cos xi, a = 1/4:
//   rho' = c/2, p' = -s/10, u' = w' = a c, div v = 2 k a c,
//   sigma_xx = sigma_zz = -(2/3) mu k a c, sigma_xz = -2 mu k a c,
//   S_rho = -omega rho' + 2 k (rho u)'
//   S_mx = S_mz = -omega (rho u)' + k (2 (rho u^2)' + p') + (8/3) mu k^2 a s
//   S_E  = -omega E' + 2 k (u (E + p))' - (16/3) mu k^2 a^2 (c^2 - s^2)
//          - 2 kappa k^2 (p/rho)'' / R
// with (rho u)' = a c (1 + s), (rho u^2)' = a^2 c (2 s + 3 s^2 / 2).
void paper_mms_source(const Params& P, double x, double z, double t, double S[4]) {
  const double PI = 3.14159265358979323846;
  const double k = PI / 5.0, om = 2.0 * PI, a = 0.25, gm1 = P.gamma - 1.0;
  const double xi = k * (x + z) - om * t;
  const double sn = std::sin(xi), cs = std::cos(xi);
  const double rho = 1.0 + 0.5 * sn, p = 1.0 / P.gamma + 0.1 * cs, u = a * sn;
  const double E = p / gm1 + rho * u * u;
  const double d_rho = 0.5 * cs, dd_rho = -0.5 * sn;
  const double d_p = -0.1 * sn, dd_p = -0.1 * cs;
  const double d_ru = a * cs * (1.0 + sn);
  const double d_ruu = a * a * cs * (2.0 * sn + 1.5 * sn * sn);
  const double d_E = d_p / gm1 + d_ruu;
  const double d_uEp = a * cs * (E + p) + u * (d_E + d_p);
  // (p/rho)'' by the quotient rule
  const double f2 = dd_p / rho - 2.0 * d_p * d_rho / (rho * rho) - p * dd_rho / (rho * rho) +
                    2.0 * p * d_rho * d_rho / (rho * rho * rho);
  S[0] = -om * d_rho + 2.0 * k * d_ru;
  S[1] = -om * d_ru + k * (2.0 * d_ruu + d_p) + (8.0 / 3.0) * P.mu * k * k * a * sn;
  S[2] = S[1];
  S[3] = -om * d_E + 2.0 * k * d_uEp - (16.0 / 3.0) * P.mu * k * k * a * a * (cs * cs - sn * sn) -
         2.0 * P.kappa * k * k * f2 / P.R;
}

// ----------------------------------------------------------- pointwise physics
// Flux F = F^h(Q) + F^v(Q, grad Q) in x and z and source S at one point
// (paper eq. equation-set, eos, temperature, stress-tensor,
// heat-conduction-coeff, momentum-equation-split), 2D.
// Readings: the EOS geopotential term is rho*g*z; the momentum flux uses the
// perturbation pressure p - p_bar(z) and the source -g (rho - rho_bar(z));
// the energy flux uses the full pressure; gradients of primitive variables
// come from the gradients of the conserved variables by the chain rule.
template <class T>
void pointwise(const Params& P, const T q[4], const T gx[4], const T gz[4],
               double x, double z, double t, double rho_b, double p_b,
               T Fx[4], T Fz[4], T S[4]) {
  const double gm1 = P.gamma - 1.0;
  T rho = q[0], mx = q[1], mz = q[2], E = q[3];
  T u = mx / rho, w = mz / rho;
  T geo = P.gravity ? rho * (P.g * z) : T(0.0);
  T p = gm1 * (E - 0.5 * (mx * u + mz * w) - geo);
  T pm = P.gravity ? p - p_b : p;     // pressure in the momentum flux
  T Tm = p / (rho * P.R);             // temperature, p = rho R T
  // primitive gradients
  T dux = (gx[1] - u * gx[0]) / rho, duz = (gz[1] - u * gz[0]) / rho;
  T dwx = (gx[2] - w * gx[0]) / rho, dwz = (gz[2] - w * gz[0]) / rho;
  T v2 = u * u + w * w;
  T dpx = gm1 * (gx[3] - 0.5 * v2 * gx[0] - rho * (u * dux + w * dwx));
  T dpz = gm1 * (gz[3] - 0.5 * v2 * gz[0] - rho * (u * duz + w * dwz));
  if (P.gravity) {
    dpx = dpx - gm1 * (P.g * z) * gx[0];
    dpz = dpz - gm1 * ((P.g * z) * gz[0] + rho * P.g);
  }
  T dTx = (dpx - P.R * Tm * gx[0]) / (rho * P.R);
  T dTz = (dpz - P.R * Tm * gz[0]) / (rho * P.R);
  // stress tensor sigma = mu (2/3 div v I - (grad v + grad v^T))
  T div = dux + dwz;
  T sxx = P.mu * ((2.0 / 3.0) * div - 2.0 * dux);
  T szz = P.mu * ((2.0 / 3.0) * div - 2.0 * dwz);
  T sxz = -P.mu * (duz + dwx);
  Fx[0] = mx;
  Fx[1] = mx * u + pm + sxx;
  Fx[2] = mz * u + sxz;
  Fx[3] = u * (E + p) + (u * sxx + w * sxz) - P.kappa * dTx;
  Fz[0] = mz;
  Fz[1] = mx * w + sxz;
  Fz[2] = mz * w + pm + szz;
  Fz[3] = w * (E + p) + (u * sxz + w * szz) - P.kappa * dTz;
  S[0] = T(0.0); S[1] = T(0.0);
  S[2] = P.gravity ? -P.g * (rho - rho_b) : T(0.0);
  S[3] = P.mms == 1 ? T(mms_source_E(P, x, z, t)) : T(0.0);
  if (P.mms == 2) {
    double Sm[4];
    paper_mms_source(P, x, z, t, Sm);
    for (int v = 0; v < 4; ++v) S[v] = S[v] + Sm[v];
  }
}

// pressure and eigenvalue bounds at a state (used by the face flux and dt)
template <class T>
T pressure(const Params& P, const T q[4], double z) {
  T geo = P.gravity ? q[0] * (P.g * z) : T(0.0);
  return (P.gamma - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0] - geo);
}
// viscous eigenvalue bound lambda_v = max(4 mu / (3 rho), gamma mu / (Pr rho))
template <class T>
T lambda_visc(const Params& P, const T& rho) {
  T a = (4.0 * P.mu / 3.0) / rho, b = (P.gamma * P.mu / P.Pr) / rho;
  return val(a) >= val(b) ? a : b;
}

// ---------------------------------------------------------------------- mesh
// Cells are leaves (level, i, j) of a 3-way refined coarse grid nx x nz; the
// oracle finds face neighbours through a dense map at the finest level.
struct Cell { int level, i, j; double x0, z0, h; };
enum { BC_PERIODIC = 0, BC_WALL = 1 };

struct Neighbor {
  // kind: 0 conforming, 1 wall, 2 this cell is fine (nb coarse, sub-face k),
  //       3 this cell is coarse (nb[0..2] fine, in sub-face order)
  int kind; int nb[3]; int k;
};

struct Mesh {
  int nx, nz, L, bc[4];
  double x0, z0, Lx, Lz;
  std::vector<Cell> cells;
  std::vector<Neighbor> nbr;  // [cell*4 + face]
  bool ok = true;
};

int ipow3(int e) { int r = 1; while (e-- > 0) r *= 3; return r; }

Mesh build_mesh(const int* mi, const double* md, const int* lev, const int* ci, const int* cj) {
  Mesh M;
  M.nx = mi[0]; M.nz = mi[1]; M.L = mi[2];
  for (int s = 0; s < 4; ++s) M.bc[s] = mi[3 + s];
  int C = mi[7];
  M.x0 = md[0]; M.z0 = md[1]; M.Lx = md[2]; M.Lz = md[3];
  double hc = M.Lx / M.nx;
  M.cells.resize(C);
  for (int c = 0; c < C; ++c) {
    Cell& k = M.cells[c];
    if (lev) { k.level = lev[c]; k.i = ci[c]; k.j = cj[c]; }
    else { k.level = 0; k.i = c % M.nx; k.j = c / M.nx; }
    k.h = hc / ipow3(k.level);
    k.x0 = M.x0 + k.i * k.h; k.z0 = M.z0 + k.j * k.h;
  }
  int F = ipow3(M.L), NXf = M.nx * F, NZf = M.nz * F;
  std::vector<int> owner((size_t)NXf * NZf, -1);
  for (int c = 0; c < C; ++c) {
    const Cell& k = M.cells[c]; int sz = ipow3(M.L - k.level);
    for (int a = 0; a < sz; ++a)
      for (int b = 0; b < sz; ++b) {
        int X = k.i * sz + a, Z = k.j * sz + b;
        if (X < 0 || X >= NXf || Z < 0 || Z >= NZf || owner[(size_t)Z * NXf + X] != -1) { M.ok = false; continue; }
        owner[(size_t)Z * NXf + X] = c;
      }
  }
  for (size_t q = 0; q < owner.size(); ++q) if (owner[q] < 0) M.ok = false;
  if (!M.ok) return M;
  M.nbr.resize((size_t)C * 4);
  for (int c = 0; c < C; ++c) {
    const Cell& k = M.cells[c]; int sz = ipow3(M.L - k.level);
    for (int f = 0; f < 4; ++f) {
      Neighbor& nb = M.nbr[c * 4 + f];
      nb.kind = 1; nb.k = 0; nb.nb[0] = nb.nb[1] = nb.nb[2] = -1;
      // fine-unit cells just outside face f
      std::vector<int> outs;
      bool outside = false;
      for (int t = 0; t < sz; ++t) {
        int X, Z;
        if (f == 0) { X = k.i * sz - 1; Z = k.j * sz + t; }
        else if (f == 1) { X = (k.i + 1) * sz; Z = k.j * sz + t; }
        else if (f == 2) { X = k.i * sz + t; Z = k.j * sz - 1; }
        else { X = k.i * sz + t; Z = (k.j + 1) * sz; }
        if (X < 0 || X >= NXf || Z < 0 || Z >= NZf) {
          if (M.bc[f] != BC_PERIODIC) { outside = true; break; }
          X = (X + NXf) % NXf; Z = (Z + NZf) % NZf;
        }
        int o = owner[(size_t)Z * NXf + X];
        if (outs.empty() || outs.back() != o) outs.push_back(o);
      }
      if (outside) { nb.kind = 1; continue; }
      if (outs.size() == 1) {
        const Cell& o = M.cells[outs[0]];
        if (o.level == k.level) { nb.kind = 0; nb.nb[0] = outs[0]; }
        else if (o.level == k.level - 1) {
          nb.kind = 2; nb.nb[0] = outs[0];
          // sub-face index along the tangential direction
          int tk = (f < 2) ? k.j : k.i, to = (f < 2) ? o.j : o.i;
          nb.k = tk - 3 * to;
          if (nb.k < 0 || nb.k > 2) M.ok = false;
        } else M.ok = false;
      } else if (outs.size() == 3) {
        nb.kind = 3;
        for (int s = 0; s < 3; ++s) {
          nb.nb[s] = outs[s];
          if (M.cells[outs[s]].level != k.level + 1) M.ok = false;
        }
      } else M.ok = false;
    }
  }
  return M;
}

// ------------------------------------------------------------------ predictor
// Element-local space-time predictor (ADER-DG, Dumbser et al. 2008), read as:
// initial guess q^0 = Q^n at every time node; a fixed number of Picard sweeps
//   q^{k+1}[a] = Q^n + dt sum_b P_ab R(q^k)[b],
//   R = S - (1/h)(D_x F_x + D_z F_z)   (strong form, no face terms);
// then F, S on the last iterate and their GL time averages.
template <class T>
struct CellPred {
  std::vector<T> Qbar, Fbx, Fbz, Sbar;   // [4][n][n] each, time averages
};

template <class T>
void residual_slice(const Params& P, const Basis& B, const Cell& c, const T* q /*[4][n][n]*/,
                    double t, T* Fx, T* Fz, T* S, T* R /*nullable*/) {
  const int n = P.n;
  std::vector<T> gx(4 * n * n), gz(4 * n * n);
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        T sx = 0.0, sz = 0.0;
        for (int m = 0; m < n; ++m) {
          sx += B.D[i * n + m] * q[(v * n + j) * n + m];
          sz += B.D[j * n + m] * q[(v * n + m) * n + i];
        }
        gx[(v * n + j) * n + i] = sx / c.h;
        gz[(v * n + j) * n + i] = sz / c.h;
      }
  for (int j = 0; j < n; ++j) {
    double z = c.z0 + c.h * B.xi[j];
    double rb, pb; background(P, z, rb, pb);
    for (int i = 0; i < n; ++i) {
      double x = c.x0 + c.h * B.xi[i];
      T qq[4], a[4], b[4], fx[4], fz[4], s[4];
      for (int v = 0; v < 4; ++v) {
        int id = (v * n + j) * n + i;
        qq[v] = q[id]; a[v] = gx[id]; b[v] = gz[id];
      }
      pointwise(P, qq, a, b, x, z, t, rb, pb, fx, fz, s);
      for (int v = 0; v < 4; ++v) {
        int id = (v * n + j) * n + i;
        Fx[id] = fx[v]; Fz[id] = fz[v]; S[id] = s[v];
      }
    }
  }
  if (!R) return;
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        T dx = 0.0, dz = 0.0;
        for (int m = 0; m < n; ++m) {
          dx += B.D[i * n + m] * Fx[(v * n + j) * n + m];
          dz += B.D[j * n + m] * Fz[(v * n + m) * n + i];
        }
        int id = (v * n + j) * n + i;
        R[id] = S[id] - (dx + dz) / c.h;
      }
}

template <class T>
void predictor_cell(const Params& P, const Basis& B, const Cell& c, const T* Qn,
                    double tn, double dt, CellPred<T>& out) {
  const int n = P.n, sl = 4 * n * n;
  std::vector<T> q((size_t)n * sl), qn((size_t)n * sl), R((size_t)n * sl);
  std::vector<T> Fx(sl), Fz(sl), S(sl);
  for (int a = 0; a < n; ++a)
    for (int k = 0; k < sl; ++k) q[(size_t)a * sl + k] = Qn[k];
  for (int it = 0; it < P.iters; ++it) {
    for (int b = 0; b < n; ++b)
      residual_slice(P, B, c, &q[(size_t)b * sl], tn + B.xi[b] * dt, Fx.data(), Fz.data(), S.data(),
                     &R[(size_t)b * sl]);
    for (int a = 0; a < n; ++a)
      for (int k = 0; k < sl; ++k) {
        T acc = 0.0;
        for (int b = 0; b < n; ++b) acc += B.P[a * n + b] * R[(size_t)b * sl + k];
        qn[(size_t)a * sl + k] = Qn[k] + dt * acc;
      }
    std::swap(q, qn);
  }
  out.Qbar.assign(sl, T(0.0)); out.Fbx.assign(sl, T(0.0));
  out.Fbz.assign(sl, T(0.0)); out.Sbar.assign(sl, T(0.0));
  for (int a = 0; a < n; ++a) {
    residual_slice(P, B, c, &q[(size_t)a * sl], tn + B.xi[a] * dt, Fx.data(), Fz.data(), S.data(),
                   (T*)nullptr);
    for (int k = 0; k < sl; ++k) {
      out.Qbar[k] += B.w[a] * q[(size_t)a * sl + k];
      out.Fbx[k] += B.w[a] * Fx[k];
      out.Fbz[k] += B.w[a] * Fz[k];
      out.Sbar[k] += B.w[a] * S[k];
    }
  }
}

// Volume integral of the time-averaged flux plus the averaged source (the
// weak-form corrector without its face terms), GL collocation mass matrix:
//   Q*_ji = Q^n_ji + dt[(1/h)((1/w_i) sum_m w_m D_mi Fx_jm + (1/w_j) sum_m w_m D_mj Fz_mi) + S_ji]
template <class T>
void volume_update(const Params& P, const Basis& B, const Cell& c, const T* Qn, const CellPred<T>& pr,
                   double dt, T* Qs) {
  const int n = P.n;
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        T ax = 0.0, az = 0.0;
        for (int m = 0; m < n; ++m) {
          ax += B.w[m] * B.D[m * n + i] * pr.Fbx[(v * n + j) * n + m];
          az += B.w[m] * B.D[m * n + j] * pr.Fbz[(v * n + m) * n + i];
        }
        int id = (v * n + j) * n + i;
        Qs[id] = Qn[id] + dt * ((ax / B.w[i] + az / B.w[j]) / c.h + pr.Sbar[id]);
      }
}

// Face data: the time-averaged state and normal flux (flux along the face's
// axis, +axis direction) extrapolated to face f by the basis values at 0 or 1.
template <class T>
void face_data(const Params& P, const Basis& B, const CellPred<T>& pr, T* FD /*[4][2][4][n]*/) {
  const int n = P.n;
  for (int f = 0; f < 4; ++f)
    for (int v = 0; v < 4; ++v)
      for (int k = 0; k < n; ++k) {
        const std::vector<double>& e = (f == 0 || f == 2) ? B.e0 : B.e1;
        T sq = 0.0, sf = 0.0;
        for (int m = 0; m < n; ++m) {
          int id = (f < 2) ? (v * n + k) * n + m : (v * n + m) * n + k;
          sq += e[m] * pr.Qbar[id];
          sf += e[m] * ((f < 2) ? pr.Fbx[id] : pr.Fbz[id]);
        }
        FD[((f * 2 + 0) * 4 + v) * n + k] = sq;
        FD[((f * 2 + 1) * 4 + v) * n + k] = sf;
      }
}

// ---------------------------------------------------------------- face flux
// Rusanov-type flux with a viscous penalty (Gassner et al. 2008, used in
// ADER-DG by Dumbser 2010 / Fambri 2017), read as
//   G = 1/2 (Fn_L + Fn_R) - 1/2 s (Q_R - Q_L),
//   s = max_nodes(|v_d| + c) + 2 eta max_nodes(lambda_v), eta = (2N+1)/(h sqrt(pi/2)),
// maxima over the face nodes of both sides; L is the lower-coordinate side.
template <class T>
void rusanov(const Params& P, int d, double h, const double* zf /*[n]*/, const T* QL, const T* FL,
             const T* QR, const T* FR, T* G /*[4][n]*/) {
  const int n = P.n;
  const double PI = 3.14159265358979323846;
  T lam = 0.0, lv = 0.0; bool first = true;
  for (int side = 0; side < 2; ++side) {
    const T* Q = side ? QR : QL;
    for (int k = 0; k < n; ++k) {
      T q[4] = {Q[0 * n + k], Q[1 * n + k], Q[2 * n + k], Q[3 * n + k]};
      T p = pressure(P, q, zf[k]);
      T c = sqrt(P.gamma * p / q[0]);
      T vn = q[1 + d] / q[0];
      T l = fabs(vn) + c;
      T lvk = lambda_visc(P, q[0]);
      if (first || val(l) > val(lam)) lam = l;
      if (first || val(lvk) > val(lv)) lv = lvk;
      first = false;
    }
  }
  double eta = (2.0 * P.N + 1.0) / (h * std::sqrt(PI / 2.0));
  T s = lam + 2.0 * eta * lv;
  for (int v = 0; v < 4; ++v)
    for (int k = 0; k < n; ++k)
      G[v * n + k] = 0.5 * (FL[v * n + k] + FR[v * n + k]) - 0.5 * s * (QR[v * n + k] - QL[v * n + k]);
}

// Ghost data at a no-slip wall (paper: background density and energy at the
// boundary, background heat flux imposed): velocity mirrored, density and
// pressure from the background (from the interior state without gravity),
// mass flux mirrored, momentum flux copied, energy flux 2 q_bg - F.
template <class T>
void wall_ghost(const Params& P, int d, const double* zf, const T* Qi, const T* Fi, T* Qg, T* Fg) {
  const int n = P.n;
  for (int k = 0; k < n; ++k) {
    T q[4] = {Qi[0 * n + k], Qi[1 * n + k], Qi[2 * n + k], Qi[3 * n + k]};
    T u = q[1] / q[0], w = q[2] / q[0];
    T rb, pb;
    if (P.gravity) { double r, p; background(P, zf[k], r, p); rb = r; pb = p; }
    else { rb = q[0]; pb = pressure(P, q, zf[k]); }
    T geo = P.gravity ? rb * (P.g * zf[k]) : T(0.0);
    Qg[0 * n + k] = rb;
    Qg[1 * n + k] = -(rb * u);
    Qg[2 * n + k] = -(rb * w);
    Qg[3 * n + k] = pb / (P.gamma - 1.0) + 0.5 * rb * (u * u + w * w) + geo;
    double qbg = (P.gravity && d == 1) ? P.kappa * P.g / P.cp : 0.0;
    Fg[0 * n + k] = -Fi[0 * n + k];
    Fg[1 * n + k] = Fi[1 * n + k];
    Fg[2 * n + k] = Fi[2 * n + k];
    Fg[3 * n + k] = 2.0 * qbg - Fi[3 * n + k];
  }
}

// z coordinates of the nodes of face f of cell c (fine sub-face: own nodes)
void face_z(const Basis& B, const Cell& c, int f, double* zf) {
  for (int k = 0; k < B.n; ++k) {
    if (f < 2) zf[k] = c.z0 + c.h * B.xi[k];
    else zf[k] = c.z0 + (f == 3 ? c.h : 0.0);
  }
}

// Numerical flux on face f of cell c, at c's own face nodes.
template <class T>
void face_flux(const Params& P, const Basis& B, const Mesh& M, int c, int f,
               const std::vector<T>& FD /*[C][4][2][4][n]*/, T* G /*[4][n]*/) {
  const int n = P.n, fs = 2 * 4 * n;   // per-face stride
  const int d = f / 2;
  const bool lower = (f == 0 || f == 2);   // face on the lower side: c is the R side
  const Cell& cc = M.cells[c];
  const Neighbor& nb = M.nbr[c * 4 + f];
  const int opp = f ^ 1;
  const T* Qm = &FD[((size_t)c * 4 + f) * fs];
  const T* Fm = Qm + 4 * n;
  double zf[16]; face_z(B, cc, f, zf);
  std::vector<T> Qo(4 * n), Fo(4 * n);
  if (nb.kind == 0) {
    const T* Qx = &FD[((size_t)nb.nb[0] * 4 + opp) * fs];
    for (int k = 0; k < 4 * n; ++k) { Qo[k] = Qx[k]; Fo[k] = Qx[4 * n + k]; }
  } else if (nb.kind == 1) {
    wall_ghost(P, d, zf, Qm, Fm, Qo.data(), Fo.data());
  } else if (nb.kind == 2) {
    // coarse neighbour: prolong its face polynomial to sub-face k
    const T* Qx = &FD[((size_t)nb.nb[0] * 4 + opp) * fs];
    for (int v = 0; v < 4; ++v)
      for (int q = 0; q < n; ++q) {
        T sq = 0.0, sf = 0.0;
        for (int m = 0; m < n; ++m) {
          double ph = phi_at(B, m, (nb.k + B.xi[q]) / 3.0);
          sq += ph * Qx[v * n + m]; sf += ph * Qx[4 * n + v * n + m];
        }
        Qo[v * n + q] = sq; Fo[v * n + q] = sf;
      }
  } else {
    // coarse cell: three fine sub-faces; prolong own data, solve, restrict
    std::vector<T> Gc(4 * n, T(0.0));
    for (int s = 0; s < 3; ++s) {
      const int fc = nb.nb[s];
      const Cell& fcell = M.cells[fc];
      const T* Qx = &FD[((size_t)fc * 4 + opp) * fs];
      std::vector<T> Qp(4 * n), Fp(4 * n), Gk(4 * n);
      for (int v = 0; v < 4; ++v)
        for (int q = 0; q < n; ++q) {
          T sq = 0.0, sf = 0.0;
          for (int m = 0; m < n; ++m) {
            double ph = phi_at(B, m, (s + B.xi[q]) / 3.0);
            sq += ph * Qm[v * n + m]; sf += ph * Fm[v * n + m];
          }
          Qp[v * n + q] = sq; Fp[v * n + q] = sf;
        }
      double zs[16]; face_z(B, fcell, opp, zs);
      if (lower) rusanov(P, d, fcell.h, zs, Qx, Qx + 4 * n, Qp.data(), Fp.data(), Gk.data());
      else rusanov(P, d, fcell.h, zs, Qp.data(), Fp.data(), Qx, Qx + 4 * n, Gk.data());
      // L2 restriction to the coarse face: G_C[m] = (1/w_m) sum_q (w_q/3) phi_m((s+xi_q)/3) G_s[q]
      for (int v = 0; v < 4; ++v)
        for (int m = 0; m < n; ++m) {
          T acc = 0.0;
          for (int q = 0; q < n; ++q)
            acc += (B.w[q] / 3.0) * phi_at(B, m, (s + B.xi[q]) / 3.0) * Gk[v * n + q];
          Gc[v * n + m] += acc / B.w[m];
        }
    }
    for (int k = 0; k < 4 * n; ++k) G[k] = Gc[k];
    return;
  }
  if (lower) rusanov(P, d, cc.h, zf, Qo.data(), Fo.data(), Qm, Fm, G);
  else rusanov(P, d, cc.h, zf, Qm, Fm, Qo.data(), Fo.data(), G);
}

// Surface part of the corrector (GL collocation mass matrix):
//   Q^{n+1}_ji = Q*_ji - (dt/h)[(e1_i G1_j - e0_i G0_j)/w_i + (e1_j G3_i - e0_j G2_i)/w_j]
template <class T>
void lift(const Params& P, const Basis& B, const Cell& c, double dt, const T* G /*[4][4][n]*/, T* Q) {
  const int n = P.n;
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        T sx = (B.e1[i] * G[(1 * 4 + v) * n + j] - B.e0[i] * G[(0 * 4 + v) * n + j]) / B.w[i];
        T sz = (B.e1[j] * G[(3 * 4 + v) * n + i] - B.e0[j] * G[(2 * 4 + v) * n + i]) / B.w[j];
        Q[(v * n + j) * n + i] = Q[(v * n + j) * n + i] - (dt / c.h) * (sx + sz);
      }
}

// One full step: predictor on every cell, face fluxes, corrector.
template <class T>
void step(const Params& P, const Basis& B, const Mesh& M, const T* Q, double t, double dt, T* Qout,
          T* Qstar_out, T* FD_out) {
  const int C = (int)M.cells.size(), n = P.n, sl = 4 * n * n, fsz = 4 * 2 * 4 * n;
  std::vector<T> Qs((size_t)C * sl), FD((size_t)C * fsz);
#pragma omp parallel for schedule(dynamic, 4)
  for (int c = 0; c < C; ++c) {
    CellPred<T> pr;
    predictor_cell(P, B, M.cells[c], Q + (size_t)c * sl, t, dt, pr);
    volume_update(P, B, M.cells[c], Q + (size_t)c * sl, pr, dt, &Qs[(size_t)c * sl]);
    face_data(P, B, pr, &FD[(size_t)c * fsz]);
  }
  if (Qstar_out) for (size_t k = 0; k < Qs.size(); ++k) Qstar_out[k] = Qs[k];
  if (FD_out) for (size_t k = 0; k < FD.size(); ++k) FD_out[k] = FD[k];
  if (!Qout) return;
#pragma omp parallel for schedule(dynamic, 4)
  for (int c = 0; c < C; ++c) {
    std::vector<T> G(4 * 4 * n);
    for (int f = 0; f < 4; ++f) face_flux(P, B, M, c, f, FD, &G[(size_t)f * 4 * n]);
    for (int k = 0; k < sl; ++k) Qout[(size_t)c * sl + k] = Qs[(size_t)c * sl + k];
    lift(P, B, M.cells[c], dt, G.data(), Qout + (size_t)c * sl);
  }
}

// ---------------------------------------------------------------------- CFL
// dt = cfl * min_cells h / (d (2N+1) (lambda + 2 lambda_v (2N+1)/h)), d = 2,
// lambda = max over nodes of max(|u|,|w|) + c, lambda_v as in the face flux.
double compute_dt(const Params& P, const Basis& B, const Mesh& M, const double* Q) {
  const int n = P.n, sl = 4 * n * n;
  double dt = 1e300;
  for (size_t c = 0; c < M.cells.size(); ++c) {
    const Cell& cc = M.cells[c];
    double lam = 0.0, lv = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double q[4];
        for (int v = 0; v < 4; ++v) q[v] = Q[c * sl + (v * n + j) * n + i];
        double z = cc.z0 + cc.h * B.xi[j];
        double p = pressure(P, q, z);
        double cs = std::sqrt(P.gamma * p / q[0]);
        double l = std::max(std::fabs(q[1] / q[0]), std::fabs(q[2] / q[0])) + cs;
        lam = std::max(lam, l);
        lv = std::max(lv, lambda_visc(P, q[0]));
      }
    double o = 2.0 * P.N + 1.0;
    double dtc = P.cfl * cc.h / (2.0 * o * (lam + 2.0 * lv * o / cc.h));
    dt = std::min(dt, dtc);
  }
  return dt;
}

// ------------------------------------------------------------- TV indicator
// Potential temperature theta = T (p0/p)^(R/cp) (paper, stratified flows).
template <class T>
T theta_of(const Params& P, const T q[4], double z) {
  T p = pressure(P, q, z);
  T Tm = p / (q[0] * P.R);
  return Tm * pow(P.p0 / p, P.R / P.cp);
}

// TV of f over a cell (paper eq. tv): the l1 norm of grad f integrated by
// GL quadrature on the collocated nodes with the weights of the reference
// element (they sum to one), physical derivatives (1/h) D; that is the mean
// of |df/dx| + |df/dz| over the cell:
//   TV = (1/h) sum_ji w_i w_j (|sum_m D_im f_jm| + |sum_m D_jm f_mi|)
// (reading: a cell-size-independent indicator; with the h^2 Jacobian of the
// physical cell, children would carry a ninth of their parent's TV)
template <class T>
T cell_tv(const Params& P, const Basis& B, const Cell& c, const T* Qc, int var) {
  const int n = P.n;
  std::vector<T> f(n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      T q[4];
      for (int v = 0; v < 4; ++v) q[v] = Qc[(v * n + j) * n + i];
      f[j * n + i] = (var == 0) ? theta_of(P, q, c.z0 + c.h * B.xi[j]) : q[0];
    }
  T tv = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      T dx = 0.0, dz = 0.0;
      for (int m = 0; m < n; ++m) {
        dx += B.D[i * n + m] * f[j * n + m];
        dz += B.D[j * n + m] * f[m * n + i];
      }
      tv += B.w[i] * B.w[j] * (fabs(dx) + fabs(dz));
    }
  return tv / c.h;
}

// Initial state from a nodal potential-temperature perturbation theta' at
// fixed background pressure (paper, Section 4.2): theta = theta_bg + theta',
// T = theta * Exner, rho = p_bar/(R T), at rest, E = p_bar/(gamma-1) + rho g z.
template <class T>
void ic_theta(const Params& P, const Basis& B, const Mesh& M, const T* thp, T* Q) {
  const int n = P.n, sl = 4 * n * n;
  for (size_t c = 0; c < M.cells.size(); ++c) {
    const Cell& cc = M.cells[c];
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double z = cc.z0 + cc.h * B.xi[j];
        double pi = 1.0 - P.g * z / (P.cp * P.theta_bg);
        double pb = P.p0 * std::pow(pi, P.cp / P.R);
        T th = P.theta_bg + thp[c * n * n + j * n + i];
        T rho = pb / (P.R * (th * pi));
        T* q = Q + c * sl;
        q[(0 * n + j) * n + i] = rho;
        q[(1 * n + j) * n + i] = T(0.0);
        q[(2 * n + j) * n + i] = T(0.0);
        q[(3 * n + j) * n + i] = pb / (P.gamma - 1.0) + rho * (P.g * z);
      }
  }
}

// L = sqrt(sum_cells h^2 sum_ji w_i w_j (theta - theta_bg)^2)
template <class T>
T loss_theta(const Params& P, const Basis& B, const Mesh& M, const T* Q) {
  const int n = P.n, sl = 4 * n * n;
  T acc = 0.0;
  for (size_t c = 0; c < M.cells.size(); ++c) {
    const Cell& cc = M.cells[c];
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        T q[4];
        for (int v = 0; v < 4; ++v) q[v] = Q[c * sl + (v * n + j) * n + i];
        T d = theta_of(P, q, cc.z0 + cc.h * B.xi[j]) - P.theta_bg;
        acc += (cc.h * cc.h * B.w[i] * B.w[j]) * (d * d);
      }
  }
  return sqrt(acc);
}

// Potential-temperature perturbation of a list of bubbles at (x, z) (paper,
// stratified flows: eqs. cos-pertubation, read with cos(pi r / a) so that it
// vanishes at r = a, and bubbles-pertubation), r = |(x, z) - (xc, zc)|_2;
// bubbles[b] = (shape, A, a, s, xc, zc): shape 0 = cosine
// A/2 (1 + cos(pi r / a)) for r <= a, else 0; shape 1 = plateau A for r <= a
// and A exp(-(r - a)^2 / s^2) beyond.  Perturbations of several bubbles add.
double bubble_theta(int nb, const double* bubbles, double x, double z) {
  const double PI = 3.14159265358979323846;
  double th = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double* bb = bubbles + 6 * b;
    double r = std::sqrt((x - bb[4]) * (x - bb[4]) + (z - bb[5]) * (z - bb[5]));
    if ((int)bb[0] == 0) { if (r <= bb[2]) th += 0.5 * bb[1] * (1.0 + std::cos(PI * r / bb[2])); }
    else th += (r <= bb[2]) ? bb[1] : bb[1] * std::exp(-(r - bb[2]) * (r - bb[2]) / (bb[3] * bb[3]));
  }
  return th;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int oracle_set_threads(int nt) {
#ifdef _OPENMP
  if (nt > 0) omp_set_num_threads(nt);
  return omp_get_max_threads();
#else
  (void)nt; return 1;
#endif
}

int oracle_param_count(void) { return P_COUNT; }

int oracle_basis(int N, double* xi, double* w, double* D, double* e0, double* e1, double* P) {
  if (N < 0 || N > 15) return -1;
  Basis B = make_basis(N);
  int n = N + 1;
  for (int k = 0; k < n; ++k) { xi[k] = B.xi[k]; w[k] = B.w[k]; e0[k] = B.e0[k]; e1[k] = B.e1[k]; }
  for (int k = 0; k < n * n; ++k) { D[k] = B.D[k]; P[k] = B.P[k]; }
  return 0;
}

int oracle_lagrange(int N, int j, double x, double* out) {
  Basis B = make_basis(N);
  *out = phi_at(B, j, x);
  return 0;
}

int oracle_background(const double* prm, double z, double* rho_b, double* p_b) {
  Params P = read_params(prm);
  background(P, z, *rho_b, *p_b);
  return 0;
}

int oracle_pointwise(const double* prm, const double* q, const double* gx, const double* gz,
                     double x, double z, double t, double* Fx, double* Fz, double* S) {
  Params P = read_params(prm);
  double rb, pb; background(P, z, rb, pb);
  pointwise(P, q, gx, gz, x, z, t, rb, pb, Fx, Fz, S);
  return 0;
}

int oracle_mesh_check(const int* mi, const double* md, const int* lev, const int* ci, const int* cj,
                      int* kinds /*[C][4] or NULL*/) {
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  if (kinds)
    for (size_t k = 0; k < M.nbr.size(); ++k) kinds[k] = M.nbr[k].kind;
  return 0;
}

// Predictor outputs: Q* [C][4][n][n] and face data [C][4][2][4][n].
int oracle_predictor(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
                     const int* cj, const double* Q, double t, double dt, double* Qstar, double* FD) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  step<double>(P, B, M, Q, t, dt, nullptr, Qstar, FD);
  return 0;
}

int oracle_step(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
                const int* cj, const double* Q, double t, double dt, double* Qout) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  step<double>(P, B, M, Q, t, dt, Qout, nullptr, nullptr);
  return 0;
}

// nsteps steps in place; dt fixed if dt > 0 else recomputed by the CFL rule
// before every step.  t is advanced.
int oracle_run(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
               const int* cj, double* Q, double* t, double dt, int nsteps) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  size_t tot = M.cells.size() * 4 * P.n * P.n;
  std::vector<double> Qn(tot);
  for (int s = 0; s < nsteps; ++s) {
    double h = dt > 0 ? dt : compute_dt(P, B, M, Q);
    step<double>(P, B, M, Q, *t, h, Qn.data(), nullptr, nullptr);
    std::memcpy(Q, Qn.data(), tot * sizeof(double));
    *t += h;
  }
  return 0;
}

int oracle_dt(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
              const int* cj, const double* Q, double* dt) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  *dt = compute_dt(P, B, M, Q);
  return 0;
}

// Perturbation theta' of a bubble list at one point (the routine the
// initial state interpolates at the nodes).
int oracle_bubble_theta(int nb, const double* bubbles, double x, double z, double* th) {
  *th = bubble_theta(nb, bubbles, x, z);
  return 0;
}

// Numerical flux across one face along direction d (0 = x, 1 = z) of cells
// of size h from the two sides' face data (time-averaged state and normal
// flux at the n face nodes, [4][n] each, L the lower-coordinate side), the
// face nodes at heights zf[n]; G [4][n].
int oracle_face_flux(const double* prm, int d, double h, const double* zf, const double* QL, const double* FL,
                     const double* QR, const double* FR, double* G) {
  Params P = read_params(prm);
  rusanov<double>(P, d, h, zf, QL, FL, QR, FR, G);
  return 0;
}

// Potential-temperature loss of a state.
int oracle_loss_theta(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
                      const int* cj, const double* Q, double* L) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  *L = loss_theta<double>(P, B, M, Q);
  return 0;
}

// TV per cell, mean/std over cells merged pairwise with the update formulas of
// Chan, Golub & LeVeque (paper, refinement criterion), and flags
//   +1 refine if TV >= mu + Tr sigma, -1 coarsen if TV < mu + Tc sigma, else 0;
// sigma == 0 keeps every cell.  stats = (count, mean, population sigma).
int oracle_tv(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
              const int* cj, const double* Q, int var, double Tr, double Tc, double* tv,
              int8_t* flags, double* stats) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  const int C = (int)M.cells.size(), sl = 4 * P.n * P.n;
  for (int c = 0; c < C; ++c) tv[c] = cell_tv(P, B, M.cells[c], Q + (size_t)c * sl, var);
  // Chan et al. pairwise merge: singletons (1, x, 0) merged bottom-up in a
  // balanced binary tree over the cell order.
  std::vector<double> cn(C), mu(C), m2(C);
  for (int c = 0; c < C; ++c) { cn[c] = 1.0; mu[c] = tv[c]; m2[c] = 0.0; }
  for (int width = 1; width < C; width *= 2)
    for (int a = 0; a + width < C; a += 2 * width) {
      int b = a + width;
      double n = cn[a] + cn[b], delta = mu[b] - mu[a];
      double m = mu[a] + delta * cn[b] / n;
      double M2 = m2[a] + m2[b] + delta * delta * cn[a] * cn[b] / n;
      cn[a] = n; mu[a] = m; m2[a] = M2;
    }
  double mean = C ? mu[0] : 0.0, sigma = C ? std::sqrt(m2[0] / cn[0]) : 0.0;
  stats[0] = C; stats[1] = mean; stats[2] = sigma;
  for (int c = 0; c < C; ++c) {
    if (sigma == 0.0) { flags[c] = 0; continue; }
    if (tv[c] >= mean + Tr * sigma) flags[c] = 1;
    else if (tv[c] < mean + Tc * sigma) flags[c] = -1;
    else flags[c] = 0;
  }
  return 0;
}

// Initial conditions by nodal interpolation.
// kind 0: hydrostatic background of constant potential temperature perturbed
//   by bubbles; bubbles[b] = (shape, A, a, s, xc, zc), shape 0 = cosine
//   theta' = A/2 (1 + cos(pi r / a)) for r <= a, shape 1 = A for r <= a and
//   A exp(-(r-a)^2/s^2) beyond; theta' of several bubbles add; the pressure
//   stays the background one, rho = p/(R T), T = theta * Exner, at rest.
// kind 1: the advected density wave of the manufactured solution at time t0.
// kind 2: the paper's manufactured solution at time t0.
int oracle_ic(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
              const int* cj, int kind, int nb, const double* bubbles, double t0, double* Q) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  const int n = P.n, sl = 4 * n * n;
  for (size_t c = 0; c < M.cells.size(); ++c) {
    const Cell& cc = M.cells[c];
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double x = cc.x0 + cc.h * B.xi[i], z = cc.z0 + cc.h * B.xi[j];
        double q[4];
        if (kind == 2) {
          paper_mms_state(P, x, z, t0, q);
        } else if (kind == 1) {
          double X = x - P.mms_u * t0, Z = z - P.mms_w * t0;
          double rho = 1.0 + P.mms_amp * std::sin(P.mms_kx * X) * std::sin(P.mms_kz * Z);
          q[0] = rho; q[1] = rho * P.mms_u; q[2] = rho * P.mms_w;
          q[3] = P.mms_p / (P.gamma - 1.0) + 0.5 * rho * (P.mms_u * P.mms_u + P.mms_w * P.mms_w);
        } else {
          double th = bubble_theta(nb, bubbles, x, z);
          double pi = 1.0 - P.g * z / (P.cp * P.theta_bg);
          double pb = P.p0 * std::pow(pi, P.cp / P.R);
          double T = (P.theta_bg + th) * pi;
          double rho = pb / (P.R * T);
          q[0] = rho; q[1] = 0.0; q[2] = 0.0;
          q[3] = pb / (P.gamma - 1.0) + rho * P.g * z;
        }
        for (int v = 0; v < 4; ++v) Q[c * sl + (v * n + j) * n + i] = q[v];
      }
  }
  return 0;
}

// Directional derivative of one step (frozen dt) by forward-mode dual
// numbers: Qout = step(Q), dQout = step'(Q) dQ.
int oracle_step_jvp(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
                    const int* cj, const double* Q, const double* dQ, double t, double dt, double* Qout,
                    double* dQout) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  const size_t tot = M.cells.size() * 4 * P.n * P.n;
  std::vector<Dual> Qd(tot), Od(tot);
  for (size_t k = 0; k < tot; ++k) Qd[k] = Dual(Q[k], dQ[k]);
  step<Dual>(P, B, M, Qd.data(), t, dt, Od.data(), nullptr, nullptr);
  for (size_t k = 0; k < tot; ++k) { Qout[k] = Od[k].v; dQout[k] = Od[k].d; }
  return 0;
}

// Loss after K steps (frozen dt) from the initial perturbation theta', and
// its directional derivative along dtheta (forward-mode dual numbers).
int oracle_rollout_jvp(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
                       const int* cj, const double* thp, const double* dthp, double t0, double dt, int K,
                       double* L, double* dL) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  const size_t nodes = M.cells.size() * P.n * P.n, tot = 4 * nodes;
  std::vector<Dual> th(nodes), Q(tot), Qn(tot);
  for (size_t k = 0; k < nodes; ++k) th[k] = Dual(thp[k], dthp ? dthp[k] : 0.0);
  ic_theta<Dual>(P, B, M, th.data(), Q.data());
  double t = t0;
  for (int s = 0; s < K; ++s) {
    step<Dual>(P, B, M, Q.data(), t, dt, Qn.data(), nullptr, nullptr);
    std::swap(Q, Qn);
    t += dt;
  }
  Dual l = loss_theta<Dual>(P, B, M, Q.data());
  *L = l.v;
  *dL = l.d;
  return 0;
}

// Regrid after the refinement criterion (paper, Section 3): a flag +1 splits
// a leaf into its 3x3 children (not beyond the finest level), -1 marks it for
// coarsening; the nine children of a parent are merged into the parent only
// when all nine are leaves and all are marked (and never below level 0).
// Leaves are emitted in old order: children row by row in place of a split
// leaf, a merged parent at the position of its first child.  States: a child
// takes the parent polynomial at its nodes; a merged parent takes the L2
// projection of its children (GL quadrature on each child).  Outputs are
// sized for 9*C leaves; *C_new is set.
}  // extern "C"

namespace {

// Regrid decisions with 2:1 balance (neighbouring leaves differ by at most
// one level after the regrid).  Reading of the paper's rule (refine wins;
// a family coarsens only if all nine siblings are leaves flagged coarsen)
// extended by the balance the 1:3 face coupling needs:
//   1. clamp: refine at the finest level and coarsen at level 0 become keep;
//   2. refinement closure: a leaf that is not refined but touches, across a
//      face, a leaf whose new level exceeds its own level by two, is refined;
//      repeated until nothing changes;
//   3. coarsening: every complete family of leaves flagged coarsen (none of
//      them refined by step 2) is a candidate; a candidate whose parent would
//      touch, across one of its faces, a leaf of new level above the parent's
//      level + 1 keeps its children; repeated until nothing changes.
// Returns per leaf: 1 refine, -1 coarsen (with its family), 0 keep.
// Brute force on the finest grid: the leaves across a face are read from an
// owner map of the finest cells.
std::vector<int> balanced_decisions(const Mesh& M, const int8_t* flags) {
  const int C = (int)M.cells.size(), L = M.L;
  const int F = ipow3(L), NXf = M.nx * F, NZf = M.nz * F;
  std::vector<int> owner((size_t)NXf * NZf, -1);
  for (int c = 0; c < C; ++c) {
    const Cell& k = M.cells[c];
    const int sz = ipow3(L - k.level);
    for (int b = 0; b < sz; ++b)
      for (int a = 0; a < sz; ++a) owner[(size_t)(k.j * sz + b) * NXf + (k.i * sz + a)] = c;
  }
  std::vector<int> f(C), nl(C);
  for (int c = 0; c < C; ++c) {
    int v = flags[c];
    if (v == 1 && M.cells[c].level == L) v = 0;
    if (v == -1 && M.cells[c].level == 0) v = 0;
    f[c] = v;
  }
  auto newlevel = [&](int c) { return M.cells[c].level + (f[c] == 1 ? 1 : 0) - (f[c] == -2 ? 1 : 0); };
  // highest new level among the leaves across face fc of the box (level l, i, j); -1 at a wall
  auto across = [&](int l, int i, int j, int fc) {
    const int sz = ipow3(L - l);
    int best = -1;
    for (int t = 0; t < sz; ++t) {
      int X, Z;
      if (fc == 0) { X = i * sz - 1; Z = j * sz + t; }
      else if (fc == 1) { X = (i + 1) * sz; Z = j * sz + t; }
      else if (fc == 2) { X = i * sz + t; Z = j * sz - 1; }
      else { X = i * sz + t; Z = (j + 1) * sz; }
      if (X < 0 || X >= NXf || Z < 0 || Z >= NZf) {
        if (M.bc[fc] != BC_PERIODIC) return -1;
        X = (X + NXf) % NXf; Z = (Z + NZf) % NZf;
      }
      best = std::max(best, newlevel(owner[(size_t)Z * NXf + X]));
    }
    return best;
  };
  // 2. refinement closure
  for (bool changed = true; changed;) {
    changed = false;
    for (int c = 0; c < C; ++c) {
      const Cell& k = M.cells[c];
      if (f[c] == 1) continue;
      for (int fc = 0; fc < 4; ++fc)
        if (across(k.level, k.i, k.j, fc) > k.level + 1) { f[c] = 1; changed = true; break; }
    }
  }
  // 3. coarsening candidates: complete families flagged -1 (marked -2)
  for (int c = 0; c < C; ++c) {
    const Cell& k = M.cells[c];
    if (f[c] != -1) continue;
    int found = 0;
    bool all = true;
    for (int c2 = 0; c2 < C; ++c2) {
      const Cell& s2 = M.cells[c2];
      if (s2.level == k.level && s2.i / 3 == k.i / 3 && s2.j / 3 == k.j / 3) {
        ++found;
        if (f[c2] != -1 && f[c2] != -2) all = false;
      }
    }
    if (found == 9 && all) {
      for (int c2 = 0; c2 < C; ++c2) {
        const Cell& s2 = M.cells[c2];
        if (s2.level == k.level && s2.i / 3 == k.i / 3 && s2.j / 3 == k.j / 3) f[c2] = -2;
      }
    }
  }
  for (int c = 0; c < C; ++c)
    if (f[c] == -1) f[c] = 0;
  for (bool changed = true; changed;) {
    changed = false;
    for (int c = 0; c < C; ++c) {
      const Cell& k = M.cells[c];
      if (f[c] != -2) continue;
      const int pl = k.level - 1, pi = k.i / 3, pj = k.j / 3;
      bool ok = true;
      for (int fc = 0; fc < 4 && ok; ++fc)
        if (across(pl, pi, pj, fc) > pl + 1) ok = false;
      if (!ok) {
        for (int c2 = 0; c2 < C; ++c2) {
          const Cell& s2 = M.cells[c2];
          if (s2.level == k.level && s2.i / 3 == pi && s2.j / 3 == pj) f[c2] = 0;
        }
        changed = true;
      }
    }
  }
  for (int c = 0; c < C; ++c) nl[c] = f[c] == -2 ? -1 : f[c];
  return nl;
}

}  // namespace

extern "C" {

int oracle_regrid(const double* prm, const int* mi, const double* md, const int* lev, const int* ci,
                  const int* cj, const double* Q, const int8_t* flags, int* nlev, int* nci, int* ncj,
                  double* Qn, int* C_new) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh M = build_mesh(mi, md, lev, ci, cj);
  if (!M.ok) return -1;
  const int C = (int)M.cells.size(), n = P.n, sl = 4 * n * n, L = M.L;
  for (int c = 0; c < C; ++c)
    if (flags[c] < -1 || flags[c] > 1) return -1;
  const std::vector<int> dec = balanced_decisions(M, flags);
  (void)L;
  std::vector<int> done;   // parents already emitted, as (l, i, j) triples
  int out = 0;
  for (int c = 0; c < C; ++c) {
    const Cell& k = M.cells[c];
    if (dec[c] == -1) {   // the family merges; emitted at its first leaf
      int pl = k.level - 1, pi = k.i / 3, pj = k.j / 3;
      bool seen = false;
      for (size_t q = 0; q < done.size(); q += 3)
        if (done[q] == pl && done[q + 1] == pi && done[q + 2] == pj) seen = true;
      if (seen) continue;
      done.push_back(pl); done.push_back(pi); done.push_back(pj);
      nlev[out] = pl; nci[out] = pi; ncj[out] = pj;
      double* dst = Qn + (size_t)out * sl;
      for (int t = 0; t < sl; ++t) dst[t] = 0.0;
      for (int c2 = 0; c2 < C; ++c2) {
        const Cell& ch = M.cells[c2];
        if (ch.level != k.level || ch.i / 3 != pi || ch.j / 3 != pj) continue;
        int a = ch.i - 3 * pi, b = ch.j - 3 * pj;
        for (int v = 0; v < 4; ++v)
          for (int jj = 0; jj < n; ++jj)
            for (int ii = 0; ii < n; ++ii) {
              double s = 0.0;
              for (int l2 = 0; l2 < n; ++l2)
                for (int m2 = 0; m2 < n; ++m2)
                  s += (B.w[m2] * B.w[l2] / 9.0) * phi_at(B, ii, (a + B.xi[m2]) / 3.0) *
                       phi_at(B, jj, (b + B.xi[l2]) / 3.0) * Q[(size_t)c2 * sl + (v * n + l2) * n + m2];
              dst[(v * n + jj) * n + ii] += s / (B.w[ii] * B.w[jj]);
            }
      }
      ++out;
    } else if (dec[c] == 1) {
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
          nlev[out] = k.level + 1; nci[out] = 3 * k.i + a; ncj[out] = 3 * k.j + b;
          double* dst = Qn + (size_t)out * sl;
          for (int v = 0; v < 4; ++v)
            for (int jj = 0; jj < n; ++jj)
              for (int ii = 0; ii < n; ++ii) {
                double s = 0.0;
                for (int l2 = 0; l2 < n; ++l2)
                  for (int m2 = 0; m2 < n; ++m2)
                    s += phi_at(B, m2, (a + B.xi[ii]) / 3.0) * phi_at(B, l2, (b + B.xi[jj]) / 3.0) *
                         Q[(size_t)c * sl + (v * n + l2) * n + m2];
                dst[(v * n + jj) * n + ii] = s;
              }
          ++out;
        }
    } else {
      nlev[out] = k.level; nci[out] = k.i; ncj[out] = k.j;
      for (int t = 0; t < sl; ++t) Qn[(size_t)out * sl + t] = Q[(size_t)c * sl + t];
      ++out;
    }
  }
  *C_new = out;
  return 0;
}

}  // extern "C"

// ========================================================================= 3D
// The same scheme in three space dimensions on uniform grids of cubes
// (periodic or wall boundaries, no adaptivity): conserved variables
// (rho, rho u, rho v, rho w, rho E), gravity along -z.  Every definition is
// the 2D one with the third direction added: the flux and source of the
// equation set, the element-local predictor, time averages, face
// extrapolation, the viscous Rusanov flux with the wall ghost state, the
// corrector, and the time step with d = 3 in the Courant rule.
// Layout: Q[cell][var][k][j][i] (z, y, x nodes; x fastest), cells
// c = (k * ny + j) * nx + i; faces 0/1: -x/+x, 2/3: -y/+y, 4/5: -z/+z; face
// nodes ordered by the two tangential directions in (z, y, x) order.
namespace {

struct Mesh3 {
  int nx, ny, nz, bc[6];
  double x0, y0, z0, h;
  int C() const { return nx * ny * nz; }
};

Mesh3 read_mesh3(const int* mi, const double* md) {
  Mesh3 M;
  M.nx = mi[0]; M.ny = mi[1]; M.nz = mi[2];
  for (int f = 0; f < 6; ++f) M.bc[f] = mi[3 + f];
  M.x0 = md[0]; M.y0 = md[1]; M.z0 = md[2]; M.h = md[3];
  return M;
}

// flux F[d][v] (d = x, y, z) and source S[v] at one point; g[d][v] are the
// physical gradients of the conserved variables
void pointwise3(const Params& P, const double q[5], const double g[3][5], double z, double rho_b, double p_b,
                double F[3][5], double S[5]) {
  const double gm1 = P.gamma - 1.0;
  const double rho = q[0], E = q[4];
  const double m[3] = {q[1], q[2], q[3]};
  const double u[3] = {m[0] / rho, m[1] / rho, m[2] / rho};
  const double geo = P.gravity ? rho * (P.g * z) : 0.0;
  const double p = gm1 * (E - 0.5 * (m[0] * u[0] + m[1] * u[1] + m[2] * u[2]) - geo);
  const double pm = P.gravity ? p - p_b : p;
  const double Tm = p / (rho * P.R);
  double du[3][3];   // du[a][d] = d u_a / d x_d
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) du[a][d] = (g[d][1 + a] - u[a] * g[d][0]) / rho;
  const double v2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double dT[3];
  for (int d = 0; d < 3; ++d) {
    double dp = gm1 * (g[d][4] - 0.5 * v2 * g[d][0] - rho * (u[0] * du[0][d] + u[1] * du[1][d] + u[2] * du[2][d]));
    if (P.gravity) {
      dp = dp - gm1 * (P.g * z) * g[d][0];
      if (d == 2) dp = dp - gm1 * rho * P.g;
    }
    dT[d] = (dp - P.R * Tm * g[d][0]) / (rho * P.R);
  }
  const double div = du[0][0] + du[1][1] + du[2][2];
  double sig[3][3];   // sigma = mu (2/3 div I - (grad v + grad v^T))
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) sig[a][b] = P.mu * ((a == b ? (2.0 / 3.0) * div : 0.0) - (du[a][b] + du[b][a]));
  for (int d = 0; d < 3; ++d) {
    F[d][0] = m[d];
    for (int a = 0; a < 3; ++a) F[d][1 + a] = m[a] * u[d] + (a == d ? pm : 0.0) + sig[a][d];
    F[d][4] = u[d] * (E + p) + (u[0] * sig[0][d] + u[1] * sig[1][d] + u[2] * sig[2][d]) - P.kappa * dT[d];
  }
  for (int v = 0; v < 5; ++v) S[v] = 0.0;
  S[3] = P.gravity ? -P.g * (rho - rho_b) : 0.0;
}

double pressure3(const Params& P, const double q[5], double z) {
  const double geo = P.gravity ? q[0] * (P.g * z) : 0.0;
  return (P.gamma - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0] - geo);
}

inline size_t at3(int n, int v, int k, int j, int i) { return (((size_t)v * n + k) * n + j) * n + i; }

// Predictor of one cell (cell origin x0, y0, z0): time averages Qb, Fb[d],
// Sb, then the partial update Qs = Q + dt ((1/h) sum_d volume_d(Fb_d) + Sb)
// and the face data FD[6][2][5][n][n] (averaged state, averaged normal flux).
void predictor3_cell(const Params& P, const Basis& B, double x0, double y0, double z0, double h,
                     const double* Q, double dt, double* Qs, double* FD) {
  const int n = P.n, nd = 5 * n * n * n;
  std::vector<double> q((size_t)n * nd), qn((size_t)n * nd), R((size_t)n * nd);
  for (int a = 0; a < n; ++a)
    for (int t = 0; t < nd; ++t) q[(size_t)a * nd + t] = Q[t];
  auto residual = [&](const double* qa, double* Fout /*[3][nd] or null*/, double* Sout, double* Ra) {
    std::vector<double> g(3 * (size_t)nd), F(3 * (size_t)nd), S(nd);
    for (int v = 0; v < 5; ++v)
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int m = 0; m < n; ++m) {
              sx += B.D[i * n + m] * qa[at3(n, v, k, j, m)];
              sy += B.D[j * n + m] * qa[at3(n, v, k, m, i)];
              sz += B.D[k * n + m] * qa[at3(n, v, m, j, i)];
            }
            g[0 * (size_t)nd + at3(n, v, k, j, i)] = sx / h;
            g[1 * (size_t)nd + at3(n, v, k, j, i)] = sy / h;
            g[2 * (size_t)nd + at3(n, v, k, j, i)] = sz / h;
          }
    for (int k = 0; k < n; ++k) {
      const double z = z0 + h * B.xi[k];
      double rb, pb;
      background(P, z, rb, pb);
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double qq[5], gg[3][5], FF[3][5], SS[5];
          for (int v = 0; v < 5; ++v) {
            qq[v] = qa[at3(n, v, k, j, i)];
            for (int d = 0; d < 3; ++d) gg[d][v] = g[d * (size_t)nd + at3(n, v, k, j, i)];
          }
          pointwise3(P, qq, gg, z, rb, pb, FF, SS);
          for (int v = 0; v < 5; ++v) {
            for (int d = 0; d < 3; ++d) F[d * (size_t)nd + at3(n, v, k, j, i)] = FF[d][v];
            S[at3(n, v, k, j, i)] = SS[v];
          }
        }
    }
    if (Fout) for (size_t t = 0; t < 3 * (size_t)nd; ++t) Fout[t] = F[t];
    if (Sout) for (int t = 0; t < nd; ++t) Sout[t] = S[t];
    if (Ra)
      for (int v = 0; v < 5; ++v)
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              double dv = 0.0;
              for (int m = 0; m < n; ++m) {
                dv += B.D[i * n + m] * F[0 * (size_t)nd + at3(n, v, k, j, m)];
                dv += B.D[j * n + m] * F[1 * (size_t)nd + at3(n, v, k, m, i)];
                dv += B.D[k * n + m] * F[2 * (size_t)nd + at3(n, v, m, j, i)];
              }
              Ra[at3(n, v, k, j, i)] = S[at3(n, v, k, j, i)] - dv / h;
            }
  };
  for (int it = 0; it < P.iters; ++it) {
    for (int b = 0; b < n; ++b) residual(&q[(size_t)b * nd], nullptr, nullptr, &R[(size_t)b * nd]);
    for (int a = 0; a < n; ++a)
      for (int t = 0; t < nd; ++t) {
        double s = 0.0;
        for (int b = 0; b < n; ++b) s += B.P[a * n + b] * R[(size_t)b * nd + t];
        qn[(size_t)a * nd + t] = Q[t] + dt * s;
      }
    q.swap(qn);
  }
  std::vector<double> Qb(nd, 0.0), Fb(3 * (size_t)nd, 0.0), Sb(nd, 0.0), Fa(3 * (size_t)nd), Sa(nd);
  for (int b = 0; b < n; ++b) {
    residual(&q[(size_t)b * nd], Fa.data(), Sa.data(), nullptr);
    for (int t = 0; t < nd; ++t) {
      Qb[t] += B.w[b] * q[(size_t)b * nd + t];
      Sb[t] += B.w[b] * Sa[t];
    }
    for (size_t t = 0; t < 3 * (size_t)nd; ++t) Fb[t] += B.w[b] * Fa[t];
  }
  // partial update: volume term (1/w_i) sum_m w_m D_mi Fb[..m..] along each direction
  for (int v = 0; v < 5; ++v)
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double vx = 0.0, vy = 0.0, vz = 0.0;
          for (int m = 0; m < n; ++m) {
            vx += B.w[m] * B.D[m * n + i] * Fb[0 * (size_t)nd + at3(n, v, k, j, m)];
            vy += B.w[m] * B.D[m * n + j] * Fb[1 * (size_t)nd + at3(n, v, k, m, i)];
            vz += B.w[m] * B.D[m * n + k] * Fb[2 * (size_t)nd + at3(n, v, m, j, i)];
          }
          const double vol = vx / B.w[i] + vy / B.w[j] + vz / B.w[k];
          Qs[at3(n, v, k, j, i)] = Q[at3(n, v, k, j, i)] + dt * (vol / h + Sb[at3(n, v, k, j, i)]);
        }
  // face data: extrapolation along the normal of the averaged state and normal flux
  const int fs = 2 * 5 * n * n;
  for (int f = 0; f < 6; ++f) {
    const int d = f / 2;
    const std::vector<double>& e = (f % 2) ? B.e1 : B.e0;
    for (int v = 0; v < 5; ++v)
      for (int s = 0; s < n; ++s)
        for (int t = 0; t < n; ++t) {
          double aq = 0.0, af = 0.0;
          for (int m = 0; m < n; ++m) {
            size_t idx;
            if (d == 0) idx = at3(n, v, s, t, m);        // (k, j) face node, x along m
            else if (d == 1) idx = at3(n, v, s, m, t);   // (k, i)
            else idx = at3(n, v, m, s, t);               // (j, i)
            aq += e[m] * Qb[idx];
            af += e[m] * Fb[d * (size_t)nd + idx];
          }
          FD[(size_t)f * fs + ((0 * 5 + v) * n + s) * n + t] = aq;
          FD[(size_t)f * fs + ((1 * 5 + v) * n + s) * n + t] = af;
        }
  }
}

// z coordinate of face node (s, t) of face f of a cell at height z0
double face_z3(const Basis& B, int f, double z0, double h, int s, int t) {
  (void)t;
  if (f == 4) return z0;
  if (f == 5) return z0 + h;
  return z0 + h * B.xi[s];   // x and y faces: s runs along z
}

// ghost state and flux at a no-slip wall with normal direction d
void wall_ghost3(const Params& P, int d, double zf, const double Qi[5], const double Fi[5], double Qg[5],
                 double Fg[5]) {
  const double u[3] = {Qi[1] / Qi[0], Qi[2] / Qi[0], Qi[3] / Qi[0]};
  double rb, pb;
  if (P.gravity) background(P, zf, rb, pb);
  else { rb = Qi[0]; pb = pressure3(P, Qi, zf); }
  const double geo = P.gravity ? rb * (P.g * zf) : 0.0;
  Qg[0] = rb;
  for (int a = 0; a < 3; ++a) Qg[1 + a] = -(rb * u[a]);
  Qg[4] = pb / (P.gamma - 1.0) + 0.5 * rb * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + geo;
  const double qbg = (P.gravity && d == 2) ? P.kappa * P.g / P.cp : 0.0;
  Fg[0] = -Fi[0];
  for (int a = 0; a < 3; ++a) Fg[1 + a] = Fi[1 + a];
  Fg[4] = 2.0 * qbg - Fi[4];
}

int cell3(const Mesh3& M, int i, int j, int k) { return (k * M.ny + j) * M.nx + i; }

// one step: predictor of every cell, then per face the Rusanov flux and the
// corrector (lifting of the six face fluxes)
void step3(const Params& P, const Basis& B, const Mesh3& M, const double* Q, double t, double dt, double* out) {
  (void)t;
  const int n = P.n, nd = 5 * n * n * n, C = M.C(), fs = 2 * 5 * n * n;
  std::vector<double> Qs((size_t)C * nd), FD((size_t)C * 6 * fs);
#pragma omp parallel for schedule(dynamic)
  for (int c = 0; c < C; ++c) {
    const int i = c % M.nx, j = (c / M.nx) % M.ny, k = c / (M.nx * M.ny);
    predictor3_cell(P, B, M.x0 + i * M.h, M.y0 + j * M.h, M.z0 + k * M.h, M.h, Q + (size_t)c * nd, dt,
                    &Qs[(size_t)c * nd], &FD[(size_t)c * 6 * fs]);
  }
  const double PI = 3.14159265358979323846;
  const double eta = (2.0 * P.N + 1.0) / (M.h * std::sqrt(PI / 2.0));
#pragma omp parallel for schedule(dynamic)
  for (int c = 0; c < C; ++c) {
    const int ci = c % M.nx, cj = (c / M.nx) % M.ny, ck = c / (M.nx * M.ny);
    const double z0 = M.z0 + ck * M.h;
    std::vector<double> G((size_t)6 * 5 * n * n);
    for (int f = 0; f < 6; ++f) {
      const int d = f / 2, hi = f % 2;
      int ni = ci + (d == 0 ? (hi ? 1 : -1) : 0), nj = cj + (d == 1 ? (hi ? 1 : -1) : 0),
          nk = ck + (d == 2 ? (hi ? 1 : -1) : 0);
      const int dims[3] = {M.nx, M.ny, M.nz};
      int* nn3[3] = {&ni, &nj, &nk};
      bool wall = false;
      if (*nn3[d] < 0 || *nn3[d] >= dims[d]) {
        if (M.bc[f] == BC_WALL) wall = true;
        else *nn3[d] = (*nn3[d] + dims[d]) % dims[d];
      }
      const double* own = &FD[((size_t)c * 6 + f) * fs];
      std::vector<double> other(fs);
      if (wall) {
        for (int s = 0; s < n; ++s)
          for (int tt = 0; tt < n; ++tt) {
            double Qi[5], Fi[5], Qg[5], Fg[5];
            for (int v = 0; v < 5; ++v) {
              Qi[v] = own[((0 * 5 + v) * n + s) * n + tt];
              Fi[v] = own[((1 * 5 + v) * n + s) * n + tt];
            }
            wall_ghost3(P, d, face_z3(B, f, z0, M.h, s, tt), Qi, Fi, Qg, Fg);
            for (int v = 0; v < 5; ++v) {
              other[((0 * 5 + v) * n + s) * n + tt] = Qg[v];
              other[((1 * 5 + v) * n + s) * n + tt] = Fg[v];
            }
          }
      } else {
        const int o = cell3(M, ni, nj, nk);
        const double* src = &FD[((size_t)o * 6 + (f ^ 1)) * fs];
        for (int q = 0; q < fs; ++q) other[q] = src[q];
      }
      // L = lower side (-axis), R = upper side
      const double* QL = hi ? own : other.data();
      const double* QR = hi ? other.data() : own;
      double lam = 0.0, lv = 0.0;
      bool first = true;
      for (int side = 0; side < 2; ++side) {
        const double* Qx = side ? QR : QL;
        for (int s = 0; s < n; ++s)
          for (int tt = 0; tt < n; ++tt) {
            double q[5];
            for (int v = 0; v < 5; ++v) q[v] = Qx[((0 * 5 + v) * n + s) * n + tt];
            const double p = pressure3(P, q, face_z3(B, f, z0, M.h, s, tt));
            const double l = std::fabs(q[1 + d] / q[0]) + std::sqrt(P.gamma * p / q[0]);
            const double lvk = lambda_visc(P, q[0]);
            if (first || l > lam) lam = l;
            if (first || lvk > lv) lv = lvk;
            first = false;
          }
      }
      const double sp = lam + 2.0 * eta * lv;
      for (int v = 0; v < 5; ++v)
        for (int q = 0; q < n * n; ++q) {
          const double qL = QL[(0 * 5 + v) * n * n + q], qR = QR[(0 * 5 + v) * n * n + q];
          const double fL = QL[(1 * 5 + v) * n * n + q], fR = QR[(1 * 5 + v) * n * n + q];
          G[((size_t)f * 5 + v) * n * n + q] = 0.5 * (fL + fR) - 0.5 * sp * (qR - qL);
        }
    }
    for (int v = 0; v < 5; ++v)
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            auto g = [&](int f, int s, int tt) { return G[((size_t)f * 5 + v) * n * n + s * n + tt]; };
            const double lx = (B.e1[i] * g(1, k, j) - B.e0[i] * g(0, k, j)) / B.w[i];
            const double ly = (B.e1[j] * g(3, k, i) - B.e0[j] * g(2, k, i)) / B.w[j];
            const double lz = (B.e1[k] * g(5, j, i) - B.e0[k] * g(4, j, i)) / B.w[k];
            out[(size_t)c * nd + at3(n, v, k, j, i)] = Qs[(size_t)c * nd + at3(n, v, k, j, i)] - dt / M.h * (lx + ly + lz);
          }
  }
}

double dt3(const Params& P, const Basis& B, const Mesh3& M, const double* Q) {
  const int n = P.n, nd = 5 * n * n * n;
  double dt = 1e300;
  for (int c = 0; c < M.C(); ++c) {
    const int ck = c / (M.nx * M.ny);
    double lam = 0.0, lv = 0.0;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double q[5];
          for (int v = 0; v < 5; ++v) q[v] = Q[(size_t)c * nd + at3(n, v, k, j, i)];
          const double z = M.z0 + ck * M.h + M.h * B.xi[k];
          const double cs = std::sqrt(P.gamma * pressure3(P, q, z) / q[0]);
          const double l = std::max(std::fabs(q[1]), std::max(std::fabs(q[2]), std::fabs(q[3]))) / q[0] + cs;
          lam = std::max(lam, l);
          lv = std::max(lv, lambda_visc(P, q[0]));
        }
    const double o = 2.0 * P.N + 1.0;
    dt = std::min(dt, P.cfl * M.h / (3.0 * o * (lam + 2.0 * lv * o / M.h)));
  }
  return dt;
}

}  // namespace

extern "C" {

int oracle3_step(const double* prm, const int* mi, const double* md, const double* Q, double t, double dt,
                 double* out) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  step3(P, B, read_mesh3(mi, md), Q, t, dt, out);
  return 0;
}

int oracle3_predictor(const double* prm, const int* mi, const double* md, const double* Q, double dt, double* Qs,
                      double* FD) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh3 M = read_mesh3(mi, md);
  const int n = P.n, nd = 5 * n * n * n, fs = 2 * 5 * n * n;
#pragma omp parallel for schedule(dynamic)
  for (int c = 0; c < M.C(); ++c) {
    const int i = c % M.nx, j = (c / M.nx) % M.ny, k = c / (M.nx * M.ny);
    predictor3_cell(P, B, M.x0 + i * M.h, M.y0 + j * M.h, M.z0 + k * M.h, M.h, Q + (size_t)c * nd, dt,
                    Qs + (size_t)c * nd, FD + (size_t)c * 6 * fs);
  }
  return 0;
}

int oracle3_dt(const double* prm, const int* mi, const double* md, const double* Q, double* out) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  *out = dt3(P, B, read_mesh3(mi, md), Q);
  return 0;
}

int oracle3_run(const double* prm, const int* mi, const double* md, double* Q, double* t, double dt, int nsteps) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh3 M = read_mesh3(mi, md);
  const size_t tot = (size_t)M.C() * 5 * P.n * P.n * P.n;
  std::vector<double> Qn(tot);
  for (int s = 0; s < nsteps; ++s) {
    const double h = dt > 0 ? dt : dt3(P, B, M, Q);
    step3(P, B, M, Q, *t, h, Qn.data());
    std::memcpy(Q, Qn.data(), tot * sizeof(double));
    *t += h;
  }
  return 0;
}

// Initial states by nodal interpolation.  kind 0: background atmosphere
// perturbed in theta by bubbles [shape, A, a, s, xc, yc, zc] (shape 0:
// cosine (A/2)(1 + cos(pi r / a)) for r <= a; 1: A for r <= a, else
// A exp(-(r - a)^2 / s^2)), at rest, pressure unperturbed; kind 1: the ABC
// flow at time t0 (rho = 1, velocity exp(-mu t) (sin z + cos y,
// sin x + cos z, sin y + cos x), p = 100/gamma - exp(-2 mu t)(cos x sin y +
// sin x cos z + sin z cos y)).
int oracle3_ic(const double* prm, const int* mi, const double* md, int kind, int nb, const double* bub, double t0,
               double* Q) {
  Params P = read_params(prm);
  Basis B = make_basis(P.N);
  Mesh3 M = read_mesh3(mi, md);
  const int n = P.n, nd = 5 * n * n * n;
  const double PI = 3.14159265358979323846;
  for (int c = 0; c < M.C(); ++c) {
    const int ci = c % M.nx, cj = (c / M.nx) % M.ny, ck = c / (M.nx * M.ny);
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          const double x = M.x0 + M.h * (ci + B.xi[i]), y = M.y0 + M.h * (cj + B.xi[j]),
                       z = M.z0 + M.h * (ck + B.xi[k]);
          double q[5];
          if (kind == 0) {
            double th = 0.0;
            for (int b = 0; b < nb; ++b) {
              const double* bb = bub + 7 * b;
              const double dx = x - bb[4], dy = y - bb[5], dz = z - bb[6];
              const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
              if ((int)bb[0] == 0) th += r <= bb[2] ? 0.5 * bb[1] * (1.0 + std::cos(PI * r / bb[2])) : 0.0;
              else th += r <= bb[2] ? bb[1] : bb[1] * std::exp(-(r - bb[2]) * (r - bb[2]) / (bb[3] * bb[3]));
            }
            const double pi = 1.0 - P.g * z / (P.cp * P.theta_bg);
            const double pb = P.p0 * std::pow(pi, P.cp / P.R);
            const double rho = pb / (P.R * (P.theta_bg + th) * pi);
            q[0] = rho; q[1] = q[2] = q[3] = 0.0;
            q[4] = pb / (P.gamma - 1.0) + rho * P.g * z;
          } else {
            const double a = std::exp(-P.mu * t0), a2 = std::exp(-2.0 * P.mu * t0);
            const double u = a * (std::sin(z) + std::cos(y)), v = a * (std::sin(x) + std::cos(z)),
                         w = a * (std::sin(y) + std::cos(x));
            const double p = 100.0 / P.gamma - a2 * (std::cos(x) * std::sin(y) + std::sin(x) * std::cos(z) +
                                                     std::sin(z) * std::cos(y));
            q[0] = 1.0; q[1] = u; q[2] = v; q[3] = w;
            q[4] = p / (P.gamma - 1.0) + 0.5 * (u * u + v * v + w * w);
          }
          for (int vv = 0; vv < 5; ++vv) Q[(size_t)c * nd + at3(n, vv, k, j, i)] = q[vv];
        }
  }
  return 0;
}

}  // extern "C"

// ============================================================ finite volume
// The engine's second scheme (Numerics): MUSCL-Hancock finite volumes
// stabilised with the van Albada limiter, run without viscosity for the
// colliding bubbles (stratified-flow section).  Uniform grid of nx x nz
// square cells of edge h, one value per cell, Q[c][4], c = j * nx + i, the
// value standing for the cell centre.  The pointwise physics, the Rusanov
// flux and the wall ghost are those of the DG scheme at one node (N = 0,
// mu = 0).  One step:
//   1. slopes of the conserved variables per direction, limited with van
//      Albada (at a wall, the neighbour is the wall ghost state at the ghost
//      cell's centre);
//   2. Hancock half step: the four face values Q -+ slope/2 all move by
//      dt/(2h) times the flux differences across the cell (each flux at its
//      face height) plus dt/2 times the source of the cell value;
//   3. Rusanov flux of the evolved face values of the two cells of a face
//      (the wall ghost of the evolved value at a wall);
//   4. Q <- Q - dt/h (flux differences) + dt * source of the half-step cell
//      value (Q plus the half-step increment).
// Time step: the Courant rule of the DG scheme at N = 0 without viscosity,
// dt = cfl h / (2 lambda), lambda = max over cells of max(|u|,|w|) + c.
namespace {

struct FVMesh {
  int nx, nz, bc[4];   // bc: west, east, south, north
  double x0, z0, h;
  int C() const { return nx * nz; }
};

FVMesh read_fv_mesh(const int* mi, const double* md) {
  FVMesh M;
  M.nx = mi[0]; M.nz = mi[1];
  for (int f = 0; f < 4; ++f) M.bc[f] = mi[2 + f];
  M.x0 = md[0]; M.z0 = md[1]; M.h = md[2];
  return M;
}

// the parameters of the scheme at one node without viscosity
Params fv_params(const double* prm) {
  Params P = read_params(prm);
  P.N = 0; P.n = 1; P.iters = 1;
  P.mu = 0.0; P.kappa = 0.0; P.mms = 0;
  return P;
}

// van Albada limited slope from the backward and forward differences a, b:
// a b (a + b) / (a^2 + b^2) when a b > 0, else 0; that is b phi(a / b) with
// phi(r) = (r^2 + r) / (r^2 + 1) on r > 0.
double van_albada(double a, double b) {
  if (!(a * b > 0.0)) return 0.0;
  return a * b * (a + b) / (a * a + b * b);
}

// inviscid flux along d (0: x, 1: z) and the vertical-momentum source at height z
void fv_flux(const Params& P, const double q[4], double z, int d, double F[4], double* Sw) {
  double rb, pb;
  background(P, z, rb, pb);
  const double zero[4] = {0.0, 0.0, 0.0, 0.0};
  double Fx[4], Fz[4], S[4];
  pointwise<double>(P, q, zero, zero, 0.0, z, 0.0, rb, pb, Fx, Fz, S);
  for (int v = 0; v < 4; ++v) F[v] = d == 0 ? Fx[v] : Fz[v];
  if (Sw) *Sw = S[2];
}

// ghost state at a wall for a state q at height z (the DG wall ghost)
void fv_ghost_state(const Params& P, int d, const double q[4], double z, double g[4]) {
  double F0[4] = {0.0, 0.0, 0.0, 0.0}, Fg[4];
  wall_ghost<double>(P, d, &z, q, F0, g, Fg);
}

double fv_zc(const FVMesh& M, int j) { return M.z0 + (j + 0.5) * M.h; }

// Hancock half step of every cell: evolved face values E[c][4 faces][4]
// (faces: west, east, south, north) and the half-step increment inc[c][4].
void fv_predict(const Params& P, const FVMesh& M, const double* Q, double dt, double* E, double* inc) {
  const double h = M.h;
  for (int j = 0; j < M.nz; ++j)
    for (int i = 0; i < M.nx; ++i) {
      const int c = j * M.nx + i;
      const double* q = Q + 4 * c;
      const double zc = fv_zc(M, j);
      double slope[2][4];
      for (int d = 0; d < 2; ++d) {
        double lo[4], hi[4];
        for (int side = 0; side < 2; ++side) {
          double* nb = side ? hi : lo;
          const int f = 2 * d + side;
          int ni = i + (d == 0 ? (side ? 1 : -1) : 0), nj = j + (d == 1 ? (side ? 1 : -1) : 0);
          const bool out = ni < 0 || ni >= M.nx || nj < 0 || nj >= M.nz;
          if (out && M.bc[f] == BC_WALL) {
            // ghost cell centre: mirror of the cell centre across the face
            const double zg = d == 1 ? zc + (side ? h : -h) : zc;
            fv_ghost_state(P, d, q, zg, nb);
          } else {
            ni = (ni + M.nx) % M.nx; nj = (nj + M.nz) % M.nz;
            for (int v = 0; v < 4; ++v) nb[v] = Q[4 * (nj * M.nx + ni) + v];
          }
        }
        for (int v = 0; v < 4; ++v) slope[d][v] = van_albada(q[v] - lo[v], hi[v] - q[v]);
      }
      double fv[4][4];   // face values: west, east, south, north
      for (int v = 0; v < 4; ++v) {
        fv[0][v] = q[v] - 0.5 * slope[0][v];
        fv[1][v] = q[v] + 0.5 * slope[0][v];
        fv[2][v] = q[v] - 0.5 * slope[1][v];
        fv[3][v] = q[v] + 0.5 * slope[1][v];
      }
      const double zf[4] = {zc, zc, zc - 0.5 * h, zc + 0.5 * h};
      double F[4][4], Sw;
      for (int f = 0; f < 4; ++f) fv_flux(P, fv[f], zf[f], f / 2, F[f], nullptr);
      double Fc[4];
      fv_flux(P, q, zc, 0, Fc, &Sw);
      double* ic = inc + 4 * c;
      for (int v = 0; v < 4; ++v) {
        ic[v] = dt / (2.0 * h) * ((F[0][v] - F[1][v]) + (F[2][v] - F[3][v]));
        if (v == 2) ic[v] += 0.5 * dt * Sw;
      }
      for (int f = 0; f < 4; ++f)
        for (int v = 0; v < 4; ++v) E[(4 * c + f) * 4 + v] = fv[f][v] + ic[v];
    }
}

void fv_step(const Params& P, const FVMesh& M, const double* Q, double dt, double* out) {
  const int C = M.C();
  const double h = M.h;
  std::vector<double> E((size_t)C * 16), inc((size_t)C * 4);
  fv_predict(P, M, Q, dt, E.data(), inc.data());
  for (int j = 0; j < M.nz; ++j)
    for (int i = 0; i < M.nx; ++i) {
      const int c = j * M.nx + i;
      const double zc = fv_zc(M, j);
      double G[4][4];
      for (int f = 0; f < 4; ++f) {
        const int d = f / 2, hi = f % 2;
        const double zf = d == 0 ? zc : zc + (hi ? 0.5 * h : -0.5 * h);
        const double* own = &E[(4 * c + f) * 4];
        double Fo[4];
        fv_flux(P, own, zf, d, Fo, nullptr);
        double Qn[4], Fn[4];
        int ni = i + (d == 0 ? (hi ? 1 : -1) : 0), nj = j + (d == 1 ? (hi ? 1 : -1) : 0);
        const bool out = ni < 0 || ni >= M.nx || nj < 0 || nj >= M.nz;
        if (out && M.bc[f] == BC_WALL) {
          wall_ghost<double>(P, d, &zf, own, Fo, Qn, Fn);
        } else {
          ni = (ni + M.nx) % M.nx; nj = (nj + M.nz) % M.nz;
          const double* oth = &E[(4 * (nj * M.nx + ni) + (f ^ 1)) * 4];
          for (int v = 0; v < 4; ++v) Qn[v] = oth[v];
          fv_flux(P, Qn, zf, d, Fn, nullptr);
        }
        const double zz[1] = {zf};
        if (hi) rusanov<double>(P, d, h, zz, own, Fo, Qn, Fn, G[f]);
        else rusanov<double>(P, d, h, zz, Qn, Fn, own, Fo, G[f]);
      }
      double qh[4], F0[4], Sh;
      for (int v = 0; v < 4; ++v) qh[v] = Q[4 * c + v] + inc[4 * c + v];
      fv_flux(P, qh, zc, 0, F0, &Sh);
      for (int v = 0; v < 4; ++v) {
        double val = Q[4 * c + v] - dt / h * ((G[1][v] - G[0][v]) + (G[3][v] - G[2][v]));
        if (v == 2) val += dt * Sh;
        out[4 * c + v] = val;
      }
    }
}

double fv_dt(const Params& P, const FVMesh& M, const double* Q) {
  double lam = 0.0;
  for (int j = 0; j < M.nz; ++j)
    for (int i = 0; i < M.nx; ++i) {
      const double* q = Q + 4 * (j * M.nx + i);
      const double c = std::sqrt(P.gamma * pressure(P, q, fv_zc(M, j)) / q[0]);
      lam = std::max(lam, std::max(std::fabs(q[1]), std::fabs(q[2])) / q[0] + c);
    }
  return P.cfl * M.h / (2.0 * lam);
}

}  // namespace

extern "C" {

double oracle_van_albada(double a, double b) { return van_albada(a, b); }

int oracle_fv_predict(const double* prm, const int* mi, const double* md, const double* Q, double dt, double* E,
                      double* inc) {
  fv_predict(fv_params(prm), read_fv_mesh(mi, md), Q, dt, E, inc);
  return 0;
}

int oracle_fv_step(const double* prm, const int* mi, const double* md, const double* Q, double dt, double* out) {
  fv_step(fv_params(prm), read_fv_mesh(mi, md), Q, dt, out);
  return 0;
}

int oracle_fv_dt(const double* prm, const int* mi, const double* md, const double* Q, double* out) {
  *out = fv_dt(fv_params(prm), read_fv_mesh(mi, md), Q);
  return 0;
}

int oracle_fv_run(const double* prm, const int* mi, const double* md, double* Q, double* t, double dt, int nsteps) {
  const Params P = fv_params(prm);
  const FVMesh M = read_fv_mesh(mi, md);
  std::vector<double> Qn((size_t)M.C() * 4);
  for (int s = 0; s < nsteps; ++s) {
    const double h = dt > 0 ? dt : fv_dt(P, M, Q);
    fv_step(P, M, Q, h, Qn.data());
    std::memcpy(Q, Qn.data(), Qn.size() * sizeof(double));
    *t += h;
  }
  return 0;
}

// Cell values at the centres: kind 0 the background perturbed by bubbles
// [shape, A, a, s, xc, zc] (as the DG initial state), kind 1 the advected
// density wave of the manufactured solution at time t0 (without its source).
int oracle_fv_ic(const double* prm, const int* mi, const double* md, int kind, int nb, const double* bub, double t0,
                 double* Q) {
  const Params P = read_params(prm);
  const FVMesh M = read_fv_mesh(mi, md);
  const double PI = 3.14159265358979323846;
  for (int j = 0; j < M.nz; ++j)
    for (int i = 0; i < M.nx; ++i) {
      const double x = M.x0 + (i + 0.5) * M.h, z = M.z0 + (j + 0.5) * M.h;
      double* q = Q + 4 * (j * M.nx + i);
      if (kind == 1) {
        const double X = x - P.mms_u * t0, Z = z - P.mms_w * t0;
        const double rho = 1.0 + P.mms_amp * std::sin(P.mms_kx * X) * std::sin(P.mms_kz * Z);
        q[0] = rho; q[1] = rho * P.mms_u; q[2] = rho * P.mms_w;
        q[3] = P.mms_p / (P.gamma - 1.0) + 0.5 * rho * (P.mms_u * P.mms_u + P.mms_w * P.mms_w);
        continue;
      }
      double th = 0.0;
      for (int b = 0; b < nb; ++b) {
        const double* bb = bub + 6 * b;
        const double r = std::sqrt((x - bb[4]) * (x - bb[4]) + (z - bb[5]) * (z - bb[5]));
        if ((int)bb[0] == 0) { if (r <= bb[2]) th += 0.5 * bb[1] * (1.0 + std::cos(PI * r / bb[2])); }
        else th += (r <= bb[2]) ? bb[1] : bb[1] * std::exp(-(r - bb[2]) * (r - bb[2]) / (bb[3] * bb[3]));
      }
      const double pi = 1.0 - P.g * z / (P.cp * P.theta_bg);
      const double pb = P.p0 * std::pow(pi, P.cp / P.R);
      const double rho = pb / (P.R * (P.theta_bg + th) * pi);
      q[0] = rho; q[1] = 0.0; q[2] = 0.0;
      q[3] = pb / (P.gamma - 1.0) + rho * P.g * z;
    }
  return 0;
}

}  // extern "C"
