// Host side of the C ABI: parameter validation, Gauss-Legendre basis, leaf
// list and face tables, handle lifetime, workspace layout, dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "adg_internal.h"

namespace adg {

int launch_predictor(const Group& g, hipStream_t s);
int launch_corrector(const Group& g, hipStream_t s);
int launch_cell_dt(const Group& g, hipStream_t s);
int launch_clock(double* clock, const double* dtc, const int* beg, const int* end, int nscen, int C, int advance,
                 int update, hipStream_t s);
int max_cpw(int n);
int launch_init_state(const Group& g, int c0, int count, int kind, int nbub, const double* d_bub, double t0,
                      hipStream_t s);
int launch_tv(const Group& g, int var, double Tr, double Tc, double* tv, int8_t* flags,
              double* stats, hipStream_t s);
int launch_health(const Group& g, int* flag, hipStream_t s);
int launch_regrid(int n, int C, const int* ops, const double* Qold, double* Qnew, const double* gtab,
                  hipStream_t s);
int launch_step_adjoint(const Group& g, const double* Qn, const double* lam_in, double* lam_out, double* store,
                        const double* fd, bool recompute, double* lamFD, hipStream_t s);
int launch_predictor_store(const Group& g, double* store, hipStream_t s);
int launch_predictor_levels(const Group& g, double* store, hipStream_t s);
int launch_ic_theta(const Group& g, const double* thp, hipStream_t s);
int launch_ic_theta_adj(const Group& g, const double* thp, const double* lam, double* grad, hipStream_t s);
int launch_loss(const Group& g, double* part, double* out, hipStream_t s);
int launch_loss_adj(const Group& g, const double* L, const double* gL, double* lam, hipStream_t s);
int regrid_plan(const std::vector<int>& lev, const std::vector<int>& ci, const std::vector<int>& cj,
                const int8_t* flags, int L, int nx, int nz, const int* bc, std::vector<int>& nlev,
                std::vector<int>& nci, std::vector<int>& ncj, std::vector<int>& ops);

static thread_local std::string g_err;

// Predictor of a group with the kernel its launch mode selects: the
// time-level predictor (lv = 1 with the group's wavefronts per cell), or
// automatically one wavefront per time level while cells * n <= kLevelsWaves,
// the levels over four wavefronts per cell while cells * 4 <= kLevelsWaves
// (n > 4), else one wavefront per cell with the group's launch shape; with a
// store, the Picard iterates are kept (adjoint).
int launch_predictor_any(const Group& g, double* store, hipStream_t s) {
  if (g.lv == 1) return launch_predictor_levels(g, store, s);
  if (g.lv < 0) {
    const long cn = (long)g.C * g.n;
    if (cn <= kLevelsWaves || (g.n > 4 && 4L * g.C <= kLevelsWaves)) {
      Group t = g;
      t.lw = cn <= kLevelsWaves ? 0 : 4;
      return launch_predictor_levels(t, store, s);
    }
  }
  return store ? launch_predictor_store(g, store, s) : launch_predictor(g, s);
}

// Corrector of one mesh, then its clock: with a frozen time step the
// corrector's first workgroup advances t and the step count itself (no clock
// kernel); otherwise the clock kernel reduces the per-cell bounds into dt.
int launch_corrector_clock(Group g, double* clock, hipStream_t s) {
  if (g.ph.fixed_dt) {
    g.advance = clock;
    return launch_corrector(g, s);
  }
  int rc = launch_corrector(g, s);
  if (rc) return rc;
  return launch_clock(clock, g.dtc, nullptr, nullptr, 1, g.C, 1, 1, s);
}

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) { g_err = msg; return code; }
int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ADG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return ADG_OK;
}

// ------------------------------------------------------------------ basis
// Gauss-Legendre nodes on [0,1]: Newton's method on the Legendre polynomial
// of degree n (three-term recurrence), long double; weights from P_n'.
static void gauss_legendre(int n, std::vector<long double>& x, std::vector<long double>& w) {
  x.assign(n, 0.0L); w.assign(n, 0.0L);
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int k = 0; k < (n + 1) / 2; ++k) {
    long double r = cosl(pi * (4.0L * k + 3.0L) / (4.0L * n + 2.0L));
    long double dp = 0.0L;
    for (int it = 0; it < 64; ++it) {
      long double pm1 = 1.0L, p = r;
      for (int l = 2; l <= n; ++l) {
        long double pn = ((2 * l - 1) * r * p - (l - 1) * pm1) / l;
        pm1 = p; p = pn;
      }
      if (n == 1) { p = r; pm1 = 1.0L; }
      dp = n * (r * p - pm1) / (r * r - 1.0L);
      long double step = p / dp;
      r -= step;
      if (fabsl(step) <= 1e-24L) {
        // refresh the derivative at the converged root
        pm1 = 1.0L; p = r;
        for (int l = 2; l <= n; ++l) {
          long double pn = ((2 * l - 1) * r * p - (l - 1) * pm1) / l;
          pm1 = p; p = pn;
        }
        if (n == 1) { p = r; pm1 = 1.0L; }
        dp = n * (r * p - pm1) / (r * r - 1.0L);
        break;
      }
    }
    long double wk = 2.0L / ((1.0L - r * r) * dp * dp);
    // r is in (0,1] descending with k: map +-r to [0,1]
    x[n - 1 - k] = 0.5L * (1.0L + r); w[n - 1 - k] = 0.5L * wk;
    x[k] = 0.5L * (1.0L - r); w[k] = 0.5L * wk;
  }
  if (n % 2 == 1) x[n / 2] = 0.5L;
}

// Lagrange basis on nodes x through barycentric weights lam.
static long double bary_phi(const std::vector<long double>& x, const std::vector<long double>& lam, int j,
                            long double t) {
  for (size_t m = 0; m < x.size(); ++m)
    if (t == x[m]) return (int)m == j ? 1.0L : 0.0L;
  long double num = lam[j] / (t - x[j]), den = 0.0L;
  for (size_t m = 0; m < x.size(); ++m) den += lam[m] / (t - x[m]);
  return num / den;
}

void build_basis(int n, HostBasis& B) {
  B.n = n;
  std::vector<long double> x, w;
  gauss_legendre(n, x, w);
  std::vector<long double> lam(n, 1.0L);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (x[j] - x[k]);
  std::vector<long double> D(n * n, 0.0L);
  for (int i = 0; i < n; ++i) {
    long double diag = 0.0L;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      D[i * n + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
      diag -= D[i * n + j];
    }
    D[i * n + i] = diag;
  }
  std::vector<long double> e0(n), e1(n);
  for (int j = 0; j < n; ++j) { e0[j] = bary_phi(x, lam, j, 0.0L); e1[j] = bary_phi(x, lam, j, 1.0L); }
  // K1_ab = e1_a e1_b - w_b D_ba; P = K1^{-1} diag(w) by LU with pivoting
  std::vector<long double> A(n * n), X(n * n, 0.0L);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) A[a * n + b] = e1[a] * e1[b] - w[b] * D[b * n + a];
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) piv[k] = k;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (fabsl(A[r * n + k]) > fabsl(A[p * n + k])) p = r;
    if (p != k) { for (int c = 0; c < n; ++c) std::swap(A[p * n + c], A[k * n + c]); std::swap(piv[p], piv[k]); }
    for (int r = k + 1; r < n; ++r) {
      A[r * n + k] /= A[k * n + k];
      for (int c = k + 1; c < n; ++c) A[r * n + c] -= A[r * n + k] * A[k * n + c];
    }
  }
  for (int col = 0; col < n; ++col) {
    std::vector<long double> y(n);
    for (int r = 0; r < n; ++r) y[r] = (piv[r] == col) ? w[col] : 0.0L;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < r; ++c) y[r] -= A[r * n + c] * y[c];
    for (int r = n - 1; r >= 0; --r) {
      for (int c = r + 1; c < n; ++c) y[r] -= A[r * n + c] * y[c];
      y[r] /= A[r * n + r];
    }
    for (int r = 0; r < n; ++r) X[r * n + col] = y[r];
  }
  B.xi.resize(n); B.w.resize(n); B.e0.resize(n); B.e1.resize(n);
  B.D.resize(n * n); B.P.resize(n * n); B.Dw.resize(n * n);
  for (int k = 0; k < n; ++k) {
    B.xi[k] = (double)x[k]; B.w[k] = (double)w[k];
    B.e0[k] = (double)e0[k]; B.e1[k] = (double)e1[k];
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      B.D[i * n + j] = (double)D[i * n + j];
      B.P[i * n + j] = (double)X[i * n + j];
      B.Dw[i * n + j] = (double)(w[j] * D[j * n + i] / w[i]);
    }
  B.gtab.assign(GTab::size(n), 0.0);
  for (int k = 0; k < n; ++k) {
    B.gtab[GTab::XI * n + k] = (double)x[k];
    B.gtab[GTab::W * n + k] = (double)w[k];
    B.gtab[GTab::L0 * n + k] = (double)(e0[k] / w[k]);
    B.gtab[GTab::L1 * n + k] = (double)(e1[k] / w[k]);
    B.gtab[GTab::E0 * n + k] = (double)e0[k];
    B.gtab[GTab::E1 * n + k] = (double)e1[k];
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      B.gtab[GTab::d(n) + i * n + j] = B.D[i * n + j];
      B.gtab[GTab::pt(n) + j * n + i] = B.P[i * n + j];
      B.gtab[GTab::dw(n) + i * n + j] = B.Dw[i * n + j];
    }
  // unpivoted LU of K1 for the in-place time solve (layout with GTab::lu)
  {
    std::vector<long double> Lm(n * n, 0.0L), Um(n * n, 0.0L);
    for (int k = 0; k < n; ++k) {
      for (int c = k; c < n; ++c) {
        long double acc = e1[k] * e1[c] - w[c] * D[c * n + k];
        for (int j = 0; j < k; ++j) acc -= Lm[k * n + j] * Um[j * n + c];
        Um[k * n + c] = acc;
      }
      for (int r = k + 1; r < n; ++r) {
        long double acc = e1[r] * e1[k] - w[k] * D[k * n + r];
        for (int j = 0; j < k; ++j) acc -= Lm[r * n + j] * Um[j * n + k];
        Lm[r * n + k] = acc / Um[k * n + k];
      }
    }
    double* t = B.gtab.data() + GTab::lu(n);
    int o = 0;
    for (int i = 0; i < n; ++i) {
      t[o++] = (double)w[i];
      for (int j = 0; j < i; ++j) t[o++] = (double)Lm[i * n + j];
    }
    for (int i = n - 1; i >= 0; --i) {
      t[o++] = (double)(1.0L / Um[i * n + i]);
      for (int j = i + 1; j < n; ++j) t[o++] = (double)(Um[i * n + j] / Um[i * n + i]);
    }
  }
  // even-odd forms of D and Dw
  const int hh = n / 2, mid = (n - 1) / 2;
  for (int which = 0; which < 2; ++which) {
    auto T = [&](int i, int j) -> long double {
      return which == 0 ? D[i * n + j] : w[j] * D[j * n + i] / w[i];
    };
    double* e = B.gtab.data() + (which == 0 ? GTab::eo_d(n) : GTab::eo_dw(n));
    for (int i = 0; i < hh; ++i) {
      for (int m = 0; m < hh; ++m) {
        e[i * hh + m] = (double)((T(i, m) - T(i, n - 1 - m)) / 2.0L);
        e[hh * hh + i * hh + m] = (double)((T(i, m) + T(i, n - 1 - m)) / 2.0L);
      }
      if (n % 2) {
        e[2 * hh * hh + i] = (double)T(i, mid);
        e[2 * hh * hh + hh + i] = (double)T(mid, i);
      }
    }
  }
  for (int s = 0; s < 3; ++s)
    for (int q = 0; q < n; ++q)
      for (int mm = 0; mm < n; ++mm) {
        long double ph = bary_phi(x, lam, mm, (s + x[q]) / 3.0L);
        B.gtab[GTab::pk(n) + (s * n + q) * n + mm] = (double)ph;
        B.gtab[GTab::rk(n) + (s * n + mm) * n + q] = (double)((w[q] / 3.0L) * ph / w[mm]);
      }
}

// ------------------------------------------------------------------- mesh
static int pow3(int e) { int r = 1; while (e-- > 0) r *= 3; return r; }

static int build_mesh(const adg_mesh_desc& d, HostMesh& H) {
  const bool uniform = d.leaf_level == nullptr;
  const int C = uniform ? d.nx * d.nz : d.n_leaves;
  H.C = C;
  H.lev.resize(C); H.ci.resize(C); H.cj.resize(C);
  for (int c = 0; c < C; ++c) {
    if (uniform) { H.lev[c] = 0; H.ci[c] = c % d.nx; H.cj[c] = c / d.nx; }
    else { H.lev[c] = d.leaf_level[c]; H.ci[c] = d.leaf_i[c]; H.cj[c] = d.leaf_j[c]; }
    const int l = H.lev[c];
    if (l < 0 || l > d.max_level) return fail(ADG_EINVAL, "leaf level out of range");
    const int s = pow3(l);
    if (H.ci[c] < 0 || H.ci[c] >= d.nx * s || H.cj[c] < 0 || H.cj[c] >= d.nz * s)
      return fail(ADG_EINVAL, "leaf index out of range");
  }
  const int L = d.max_level;
  LeafIndex idx(d.nx, d.nz, L, (size_t)C);
  long long area = 0;
  for (int c = 0; c < C; ++c) {
    if (!idx.insert(H.lev[c], H.ci[c], H.cj[c], c)) return fail(ADG_EINVAL, "duplicate leaf");
    const long long s = pow3(L - H.lev[c]);
    area += s * s;
  }
  const long long full = (long long)d.nx * pow3(L) * (long long)d.nz * pow3(L);
  if (area != full) return fail(ADG_EINVAL, "leaves do not tile the domain");
  for (int c = 0; c < C; ++c) {   // no leaf may have an ancestor among the leaves
    int l = H.lev[c], i = H.ci[c], j = H.cj[c];
    while (l > 0) {
      l -= 1; i /= 3; j /= 3;
      if (idx.find(l, i, j) >= 0) return fail(ADG_EINVAL, "leaf overlaps an ancestor");
    }
  }
  const double hc = d.Lx / d.nx;
  H.geom.assign((size_t)C * 4, 0.0);
  H.nbr.assign((size_t)C * 16, -1);
  for (int c = 0; c < C; ++c) {
    const int l = H.lev[c];
    const double h = hc / pow3(l);
    H.geom[4 * c + 0] = d.x0 + H.ci[c] * h;
    H.geom[4 * c + 1] = d.z0 + H.cj[c] * h;
    H.geom[4 * c + 2] = h;
  }
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  for (int c = 0; c < C; ++c) {
    const int l = H.lev[c];
    const int NX = d.nx * pow3(l), NZ = d.nz * pow3(l);
    for (int f = 0; f < 4; ++f) {
      int* nb = &H.nbr[(size_t)c * 16 + f * 4];
      int i = H.ci[c] + di[f], j = H.cj[c] + dj[f];
      if (i < 0 || i >= NX || j < 0 || j >= NZ) {
        if (d.bc[f] == ADG_BC_WALL) { nb[0] = kWall; continue; }
        i = (i + NX) % NX; j = (j + NZ) % NZ;
      }
      const int same = idx.find(l, i, j);
      if (same >= 0) { nb[0] = kConforming; nb[1] = same; continue; }
      if (l > 0) {
        const int pc = idx.find(l - 1, i / 3, j / 3);
        if (pc >= 0) {
          nb[0] = kFineSide; nb[1] = pc;
          nb[2] = (f < 2) ? (H.cj[c] % 3) : (H.ci[c] % 3);
          continue;
        }
      }
      if (l < L) {
        int kids[3];
        bool ok = true;
        for (int s = 0; s < 3; ++s) {
          // children of (l, i, j) touching face f of this cell, in tangential order
          int ci2 = (f == 0) ? 3 * i + 2 : (f == 1) ? 3 * i : 3 * i + s;
          int cj2 = (f == 2) ? 3 * j + 2 : (f == 3) ? 3 * j : 3 * j + s;
          const int kc = idx.find(l + 1, ci2, cj2);
          if (kc < 0) { ok = false; break; }
          kids[s] = kc;
        }
        if (ok) { nb[0] = kCoarseSide; nb[1] = kids[0]; nb[2] = kids[1]; nb[3] = kids[2]; continue; }
      }
      return fail(ADG_EINVAL, "neighbouring leaves differ by more than one level");
    }
  }
  return ADG_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int validate_params(const adg_params* p) {
  if (!p) return fail(ADG_EINVAL, "null params");
  if (p->order < 1 || p->order > kMaxN - 1) return fail(ADG_EINVAL, "order must be in 1..7");
  if (p->picard_iters < 0) return fail(ADG_EINVAL, "picard_iters < 0");
  if (!(p->gamma > 1.0) || !(p->R > 0.0) || !(p->cp > 0.0) || !(p->Pr > 0.0) || !(p->mu >= 0.0))
    return fail(ADG_EINVAL, "invalid gas constants");
  if (p->gravity && (!(p->theta_bg > 0.0) || !(p->p0 > 0.0) || !(p->g >= 0.0)))
    return fail(ADG_EINVAL, "invalid background atmosphere");
  if (!(p->cfl > 0.0)) return fail(ADG_EINVAL, "cfl must be > 0");
  if (p->mms < 0 || p->mms > 2) return fail(ADG_EINVAL, "mms must be 0, 1 or 2");
  if (p->mms == 2 && p->gravity)
    return fail(ADG_EINVAL, "the paper's manufactured solution solves the equations without gravity");
  return ADG_OK;
}

static int validate_mesh(const adg_mesh_desc* d) {
  if (!d) return fail(ADG_EINVAL, "null mesh");
  if (d->nx < 1 || d->nz < 1 || !(d->Lx > 0.0) || !(d->Lz > 0.0)) return fail(ADG_EINVAL, "invalid domain");
  if (std::fabs(d->Lx / d->nx - d->Lz / d->nz) > 1e-12 * (d->Lx / d->nx))
    return fail(ADG_EINVAL, "cells must be square (Lx/nx == Lz/nz)");
  if (d->max_level < 0 || d->max_level > 8) return fail(ADG_EINVAL, "max_level must be in 0..8");
  for (int f = 0; f < 4; ++f)
    if (d->bc[f] != ADG_BC_PERIODIC && d->bc[f] != ADG_BC_WALL) return fail(ADG_EINVAL, "invalid bc");
  if ((d->bc[0] == ADG_BC_PERIODIC) != (d->bc[1] == ADG_BC_PERIODIC) ||
      (d->bc[2] == ADG_BC_PERIODIC) != (d->bc[3] == ADG_BC_PERIODIC))
    return fail(ADG_EINVAL, "periodic boundaries must come in pairs");
  const bool any = d->leaf_level || d->leaf_i || d->leaf_j;
  const bool all = d->leaf_level && d->leaf_i && d->leaf_j;
  if (any && !all) return fail(ADG_EINVAL, "leaf arrays must be all set or all NULL");
  if (all && d->n_leaves < 1) return fail(ADG_EINVAL, "n_leaves < 1");
  if (!all && d->max_level != 0) return fail(ADG_EINVAL, "uniform grid requires max_level 0");
  long long cells = all ? d->n_leaves : (long long)d->nx * d->nz;
  if (cells > (1LL << 26)) return fail(ADG_EINVAL, "too many cells");
  // the coarse grid, and each direction of the finest level, must index in
  // 32-bit ints (leaf indices, box products in the face search and regrid)
  if ((long long)d->nx * d->nz > (1LL << 26)) return fail(ADG_EINVAL, "too many coarse cells");
  long long s = 1;
  for (int l = 0; l < d->max_level; ++l) s *= 3;
  if ((long long)d->nx * s > INT32_MAX || (long long)d->nz * s > INT32_MAX)
    return fail(ADG_EINVAL, "finest level exceeds 32-bit indices (nx or nz times 3^max_level)");
  return ADG_OK;
}

Phys make_phys(const adg_params& p) {
  Phys ph{};
  ph.gamma = p.gamma; ph.gm1 = p.gamma - 1.0; ph.R = p.R; ph.iR = 1.0 / p.R; ph.cp = p.cp; ph.Pr = p.Pr;
  ph.mu = p.mu; ph.kappa = p.mu * p.cp / p.Pr; ph.g = p.g; ph.p0 = p.p0; ph.theta = p.theta_bg;
  ph.cp_over_R = p.cp / p.R; ph.R_over_cp = p.R / p.cp;
  ph.ex_coef = p.gravity ? p.g / (p.cp * p.theta_bg) : 0.0;
  ph.lv_coef = std::max(4.0 * p.mu / 3.0, p.gamma * p.mu / p.Pr);
  ph.mms_amp = p.mms_amp; ph.mms_u = p.mms_u; ph.mms_w = p.mms_w;
  ph.mms_kx = p.mms_kx; ph.mms_kz = p.mms_kz; ph.mms_p = p.mms_p;
  ph.cfl = p.cfl; ph.geff = p.gravity ? p.g : 0.0; ph.gravity = p.gravity ? 1 : 0; ph.mms = p.mms; ph.fixed_dt = p.fixed_dt ? 1 : 0;
  ph.N = p.order;
  return ph;
}

static void free_group(Group& g) {
  if (g.d_geom) (void)hipFree(g.d_geom);
  if (g.d_nbr) (void)hipFree(g.d_nbr);
  if (g.d_gtab) (void)hipFree(g.d_gtab);
  if (g.d_scen) (void)hipFree(g.d_scen);
  if (g.d_part) (void)hipFree(g.d_part);
  g.d_geom = nullptr; g.d_nbr = nullptr; g.d_gtab = nullptr; g.d_scen = nullptr; g.d_part = nullptr;
}

// Allocate and upload a group's tables.
static int upload_group(Group& g, const std::vector<double>& geom, const std::vector<int>& nbr,
                        const std::vector<double>& gtab, const std::vector<int>* scen) {
  const size_t C = (size_t)g.C;
  g.nc = 0;
  for (size_t k = 0; k < 4 * C; ++k)
    if (nbr[4 * k] == kFineSide || nbr[4 * k] == kCoarseSide) { g.nc = 1; break; }
  hipError_t e = hipSuccess;
  if (C) {
    e = hipMalloc(&g.d_geom, sizeof(double) * 4 * C);
    if (e == hipSuccess) e = hipMalloc(&g.d_nbr, sizeof(int) * 16 * C);
    if (e == hipSuccess && scen) e = hipMalloc(&g.d_scen, sizeof(int) * C);
  }
  if (e == hipSuccess) e = hipMalloc(&g.d_gtab, sizeof(double) * gtab.size());
  if (e == hipSuccess) e = hipMalloc(&g.d_part, sizeof(double) * kTvPartDoubles);
  if (e != hipSuccess) { free_group(g); return fail(ADG_ENOMEM, "device allocation failed"); }
  if (C) {
    e = hipMemcpy(g.d_geom, geom.data(), sizeof(double) * 4 * C, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g.d_nbr, nbr.data(), sizeof(int) * 16 * C, hipMemcpyHostToDevice);
    if (e == hipSuccess && scen) e = hipMemcpy(g.d_scen, scen->data(), sizeof(int) * C, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(g.d_gtab, gtab.data(), sizeof(double) * gtab.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { free_group(g); return fail(ADG_EHIP, "upload failed"); }
  return ADG_OK;
}

static int need_state(adg_mesh* m) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (!m->Q || !m->ws || !m->clock) return fail(ADG_ESTATE, "no state bound (adg_set_state)");
  return ADG_OK;
}

static int check_bubbles(int kind, int gravity, int n_bubbles, const double* bubbles) {
  if (kind < 0 || kind > 2)
    return fail(ADG_EINVAL, "kind must be 0 (bubbles), 1 (manufactured density wave) or 2 (the paper's wave)");
  if (kind == 0 && !gravity) return fail(ADG_EINVAL, "bubble states need gravity (background)");
  if (n_bubbles < 0 || n_bubbles > 16 || (n_bubbles > 0 && !bubbles)) return fail(ADG_EINVAL, "bad bubble list");
  for (int b = 0; b < n_bubbles; ++b) {
    const double* bb = bubbles + 6 * b;
    if (bb[0] != ADG_SHAPE_COSINE && bb[0] != ADG_SHAPE_PLATEAU_GAUSS) return fail(ADG_EINVAL, "bad bubble shape");
    if (bb[0] == ADG_SHAPE_COSINE && !(bb[2] > 0.0)) return fail(ADG_EINVAL, "cosine bubble radius must be > 0");
    if (bb[0] == ADG_SHAPE_PLATEAU_GAUSS && !(bb[3] > 0.0)) return fail(ADG_EINVAL, "decay s must be > 0");
  }
  return ADG_OK;
}

// init_state on cells [c0, c0+count) of a group (synchronous: the bubble list
// travels through a temporary device copy).
static int init_state_range(const Group& g, int c0, int count, int kind, int n_bubbles, const double* bubbles,
                            double t0, hipStream_t s) {
  double* d_bub = nullptr;
  if (n_bubbles > 0) {
    if (hipMalloc(&d_bub, sizeof(double) * 6 * n_bubbles) != hipSuccess) return fail(ADG_ENOMEM, "alloc");
    if (hipMemcpy(d_bub, bubbles, sizeof(double) * 6 * n_bubbles, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d_bub);
      return fail(ADG_EHIP, "upload bubbles");
    }
  }
  int rc = launch_init_state(g, c0, count, kind, n_bubbles, d_bub, t0, s);
  if (d_bub) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(d_bub);
  }
  return rc;
}

// Time pred + corr (corrector writing into Q*, so the state is untouched) for
// every launch shape and keep the fastest.
static int autotune_group(Group& g, hipStream_t s, int reps, float* best_ms) {
  if (g.C == 0) return ADG_OK;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(ADG_EHIP, "event");
  // candidates: (lv, lw, cpw, wpb); lv = 1 is the time-level predictor with
  // lw = n, 2 or 4 wavefronts per cell (its corrector shape is the default one)
  const int cpws[3] = {1, 2, 4}, wpbs[3] = {1, 2, 4}, lws[3] = {0, 2, 4};
  int bl = g.lv, blw = g.lw, bc = g.cpw, bw = g.wpb;
  float best = 1e30f;
  for (int k = -3; k < 9; ++k) {
    Group t = g;
    if (k < 0) {
      t.lv = 1; t.lw = lws[k + 3]; t.cpw = 1; t.wpb = 1;
      if (t.lw && t.lw >= g.n) continue;   // the same kernel as lw = n
    } else {
      t.lv = 0; t.cpw = cpws[k / 3]; t.wpb = wpbs[k % 3];
      if (t.cpw > max_cpw(g.n)) continue;
    }
    Group tc = t;
    tc.Q = t.Qs;   // corrector reads Q*, writes in place: state untouched
    int rc = launch_predictor_any(t, nullptr, s);   // warm-up
    if (!rc) rc = launch_corrector(tc, s);
    if (rc) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return rc; }
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) {
      launch_predictor_any(t, nullptr, s);
      launch_corrector(tc, s);
    }
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) { best = ms; bl = t.lv; blw = t.lw; bc = t.cpw; bw = t.wpb; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g.lv = bl; g.lw = blw; g.cpw = bc; g.wpb = bw;
  if (best_ms) *best_ms = best / reps;
  return check_launch("autotune");
}

// workspace: Q* [C][4][n][n], face data [C][4][2][4][n], CFL candidates, health flag
static size_t workspace_size(int C_, int n, size_t* off_qs, size_t* off_fd, size_t* off_dtc, size_t* off_h) {
  const size_t C = (size_t)C_;
  size_t off = 0;
  *off_qs = off; off = align256(off + sizeof(double) * C * 4 * n * n);
  *off_fd = off; off = align256(off + sizeof(double) * C * 32 * n);
  *off_dtc = off; off = align256(off + sizeof(double) * C);
  *off_h = off; off = align256(off + sizeof(int));
  return off;
}

static void layout_workspace(adg_mesh* m) {
  m->ws_bytes = workspace_size(m->g.C, m->g.n, &m->off_qs, &m->off_fd, &m->off_dtc, &m->off_health);
}

}  // namespace adg

using namespace adg;

// ================================================================ single mesh
extern "C" {

const char* adg_last_error(void) { return g_err.c_str(); }

int adg_init_mesh(const adg_params* prm, const adg_mesh_desc* mesh, adg_mesh** out) {
  if (!out) return fail(ADG_EINVAL, "null out");
  int rc = validate_params(prm);
  if (!rc) rc = validate_mesh(mesh);
  if (rc) return rc;
  adg_mesh* m = new (std::nothrow) adg_mesh();
  if (!m) return fail(ADG_ENOMEM, "out of host memory");
  m->prm = *prm;
  rc = build_mesh(*mesh, m->hm);
  m->desc = *mesh;
  m->desc.leaf_level = m->desc.leaf_i = m->desc.leaf_j = nullptr;   // not retained
  if (rc) { delete m; return rc; }
  const int n = prm->order + 1;
  build_basis(n, m->basis);
  Group& g = m->g;
  g.n = n; g.N = prm->order; g.iters = prm->picard_iters > 0 ? prm->picard_iters : n;
  g.C = m->hm.C; g.ph = make_phys(*prm);
  rc = upload_group(g, m->hm.geom, m->hm.nbr, m->basis.gtab, nullptr);
  if (rc) { delete m; return rc; }
  m->cells_cap = g.C;
  layout_workspace(m);
  // the allocation-free step's scratch on this device (a failed lookup only
  // disables adg_step_static, which then reports it)
  if (hipGetDevice(&m->dev) != hipSuccess) m->static_scratch_rc = fail(ADG_EHIP, "no current device");
  else m->static_scratch_rc = static_scratch_address(m->dev, &m->static_scratch);
  *out = m;
  return ADG_OK;
}

int adg_destroy(adg_mesh* m) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  free_group(m->g);
  if (m->d_ops) (void)hipFree(m->d_ops);
  if (m->h_stage) (void)hipHostFree(m->h_stage);
  delete m;
  return ADG_OK;
}

int adg_mesh_info(const adg_mesh* m, int* n_cells, int* n_nodes) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (n_cells) *n_cells = m->g.C;
  if (n_nodes) *n_nodes = m->g.n;
  return ADG_OK;
}

int adg_workspace_bytes(const adg_mesh* m, size_t* bytes) {
  if (!m || !bytes) return fail(ADG_EINVAL, "null argument");
  *bytes = m->ws_bytes;
  return ADG_OK;
}

int adg_set_state(adg_mesh* m, double* Q, void* workspace, double* clock) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (!Q || !workspace || !clock) return fail(ADG_EINVAL, "null buffer");
  if (((uintptr_t)workspace & 255) != 0) return fail(ADG_EINVAL, "workspace must be 256-byte aligned");
  if (((uintptr_t)Q & 7) != 0 || ((uintptr_t)clock & 7) != 0) return fail(ADG_EINVAL, "misaligned buffer");
  m->Q = Q; m->ws = workspace; m->clock = clock;
  char* ws = static_cast<char*>(workspace);
  m->g.Q = Q;
  m->g.Qs = reinterpret_cast<double*>(ws + m->off_qs);
  m->g.FD = reinterpret_cast<double*>(ws + m->off_fd);
  m->g.dtc = reinterpret_cast<double*>(ws + m->off_dtc);
  m->g.clock = clock;
  return ADG_OK;
}

int adg_init_state(adg_mesh* m, int kind, int n_bubbles, const double* bubbles, double t0, void* stream) {
  int rc = need_state(m);
  if (!rc) rc = check_bubbles(kind, m->prm.gravity, n_bubbles, bubbles);
  if (rc) return rc;
  return init_state_range(m->g, 0, m->g.C, kind, n_bubbles, bubbles, t0, (hipStream_t)stream);
}

int adg_compute_dt(adg_mesh* m, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  rc = launch_cell_dt(m->g, s);
  if (rc) return rc;
  return launch_clock(m->clock, m->g.dtc, nullptr, nullptr, 1, m->g.C, 0, 1, s);
}

int adg_predictor(adg_mesh* m, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  return launch_predictor_any(m->g, nullptr, (hipStream_t)stream);
}

int adg_corrector(adg_mesh* m, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  return launch_corrector_clock(m->g, m->clock, (hipStream_t)stream);
}

int adg_step(adg_mesh* m, void* stream) {
  int rc = adg_predictor(m, stream);
  if (rc) return rc;
  return adg_corrector(m, stream);
}

int adg_tv_indicator(adg_mesh* m, int var, double T_refine, double T_coarsen, double* tv, int8_t* flags,
                     double* stats, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  if (var != ADG_VAR_THETA && var != ADG_VAR_RHO) return fail(ADG_EINVAL, "var must be THETA or RHO");
  if (var == ADG_VAR_THETA && !(m->prm.p0 > 0.0)) return fail(ADG_EINVAL, "theta needs p0 > 0");
  if (!tv || !flags || !stats) return fail(ADG_EINVAL, "null output");
  if (!(T_refine > T_coarsen)) return fail(ADG_EINVAL, "T_refine must exceed T_coarsen");
  return launch_tv(m->g, var, T_refine, T_coarsen, tv, flags, stats, (hipStream_t)stream);
}

int adg_check_health(adg_mesh* m, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  int* flag = reinterpret_cast<int*>(static_cast<char*>(m->ws) + m->off_health);
  if (hipMemsetAsync(flag, 0, sizeof(int), s) != hipSuccess) return fail(ADG_EHIP, "memset");
  rc = launch_health(m->g, flag, s);
  if (rc) return rc;
  int h = 0;
  if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return fail(ADG_EHIP, "copy");
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ADG_EHIP, "sync");
  if (h) return fail(ADG_ESTATE, "state has non-finite values or non-positive density/pressure");
  return ADG_OK;
}

int adg_basis(const adg_mesh* m, double* xi, double* w, double* D, double* P) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  const int n = m->g.n;
  if (xi) std::memcpy(xi, m->basis.xi.data(), sizeof(double) * n);
  if (w) std::memcpy(w, m->basis.w.data(), sizeof(double) * n);
  if (D) std::memcpy(D, m->basis.D.data(), sizeof(double) * n * n);
  if (P) std::memcpy(P, m->basis.P.data(), sizeof(double) * n * n);
  return ADG_OK;
}

int adg_get_leaves(const adg_mesh* m, int32_t* level, int32_t* i, int32_t* j) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  for (int c = 0; c < m->hm.C; ++c) {
    if (level) level[c] = m->hm.lev[c];
    if (i) i[c] = m->hm.ci[c];
    if (j) j[c] = m->hm.cj[c];
  }
  return ADG_OK;
}

int adg_regrid_plan(adg_mesh* m, const int8_t* flags_host, int* n_cells_new, size_t* ws_bytes_new) {
  if (!m || !flags_host) return fail(ADG_EINVAL, "null argument");
  m->plan_ready = false;
  int rc = regrid_plan(m->hm.lev, m->hm.ci, m->hm.cj, flags_host, m->desc.max_level, m->desc.nx, m->desc.nz,
                       m->desc.bc, m->plan_lev, m->plan_ci,
                       m->plan_cj, m->plan_ops);
  if (rc) return rc;
  // the new leaves must form a valid mesh (at most one level between neighbours)
  adg_mesh_desc d = m->desc;
  d.n_leaves = (int)m->plan_lev.size();
  d.leaf_level = m->plan_lev.data(); d.leaf_i = m->plan_ci.data(); d.leaf_j = m->plan_cj.data();
  rc = build_mesh(d, m->plan_mesh);   // kept for adg_regrid_apply
  if (rc) return fail(ADG_EUNSUPPORTED, std::string("regrid result is not a valid mesh: ") + g_err);
  size_t a, b, c, e;
  if (n_cells_new) *n_cells_new = d.n_leaves;
  if (ws_bytes_new) *ws_bytes_new = workspace_size(d.n_leaves, m->g.n, &a, &b, &c, &e);
  m->plan_ready = true;
  return ADG_OK;
}

int adg_regrid_apply(adg_mesh* m, double* Q_new, void* workspace_new, double* clock, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  if (!m->plan_ready) return fail(ADG_ESTATE, "no regrid plan (adg_regrid_plan)");
  if (!Q_new || !workspace_new || !clock) return fail(ADG_EINVAL, "null buffer");
  if (Q_new == m->Q) return fail(ADG_EINVAL, "Q_new must not alias the current state");
  hipStream_t s = (hipStream_t)stream;
  const int Cn = (int)m->plan_lev.size();
  const size_t nops = m->plan_ops.size();
  HostMesh& H = m->plan_mesh;
  Group& g = m->g;
  // transfer operations through a grow-only device buffer
  if (nops > m->ops_cap) {
    if (m->d_ops) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(m->d_ops);
      m->d_ops = nullptr;
      m->ops_cap = 0;
    }
    if (hipMalloc(&m->d_ops, sizeof(int) * nops) != hipSuccess) {
      m->d_ops = nullptr;
      return fail(ADG_ENOMEM, "alloc ops");
    }
    m->ops_cap = nops;
  }
  // the uploads go through a grow-only pinned staging buffer: operations,
  // geometry, neighbours (an apply ends with a stream synchronisation, so no
  // earlier copy from it is in flight)
  const size_t b_ops = sizeof(int) * nops, b_geom = sizeof(double) * 4 * (size_t)H.C,
               b_nbr = sizeof(int) * 16 * (size_t)H.C;
  const size_t o_geom = align256(b_ops), o_nbr = o_geom + align256(b_geom), need = o_nbr + align256(b_nbr);
  if (need > m->stage_cap) {
    if (m->h_stage) {
      (void)hipDeviceSynchronize();   // no copy from the old buffer is in flight
      (void)hipHostFree(m->h_stage);
    }
    m->h_stage = nullptr;
    m->stage_cap = 0;
    if (hipHostMalloc(&m->h_stage, need + need / 4) != hipSuccess) {
      m->h_stage = nullptr;
      return fail(ADG_ENOMEM, "pinned staging allocation failed");
    }
    m->stage_cap = need + need / 4;
  }
  char* st = static_cast<char*>(m->h_stage);
  if (nops) {
    std::memcpy(st, m->plan_ops.data(), b_ops);
    if (hipMemcpyAsync(m->d_ops, st, b_ops, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(ADG_EHIP, "upload ops");
  }
  rc = launch_regrid(m->g.n, Cn, m->d_ops, m->Q, Q_new, m->g.d_gtab, s);
  if (rc) return rc;
  std::memcpy(st + o_geom, H.geom.data(), b_geom);   // staged while the transfer kernel runs
  std::memcpy(st + o_nbr, H.nbr.data(), b_nbr);
  // every kernel that reads the old tables (on any stream) is done before
  // they are overwritten or freed
  if (hipDeviceSynchronize() != hipSuccess) return fail(ADG_EHIP, "synchronize failed");
  // the new geometry and neighbour tables (built by the plan): in place when
  // they fit, else in new buffers with some headroom; the basis table stays
  if (H.C > m->cells_cap) {
    if (g.d_geom) (void)hipFree(g.d_geom);
    if (g.d_nbr) (void)hipFree(g.d_nbr);
    g.d_geom = nullptr; g.d_nbr = nullptr; m->cells_cap = 0;
    const int cap = H.C + H.C / 4 + 16;
    if (hipMalloc(&g.d_geom, sizeof(double) * 4 * (size_t)cap) != hipSuccess ||
        hipMalloc(&g.d_nbr, sizeof(int) * 16 * (size_t)cap) != hipSuccess) {
      if (g.d_geom) (void)hipFree(g.d_geom);
      g.d_geom = nullptr; g.C = 0;
      return fail(ADG_ENOMEM, "device allocation failed");
    }
    m->cells_cap = cap;
  }
  if (H.C && (hipMemcpyAsync(g.d_geom, st + o_geom, b_geom, hipMemcpyHostToDevice, s) != hipSuccess ||
              hipMemcpyAsync(g.d_nbr, st + o_nbr, b_nbr, hipMemcpyHostToDevice, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess)) {
    g.C = 0;
    return fail(ADG_EHIP, "upload failed");
  }
  g.C = H.C;
  g.nc = 0;
  for (size_t k = 0; k < 4 * (size_t)H.C; ++k)
    if (H.nbr[4 * k] == kFineSide || H.nbr[4 * k] == kCoarseSide) { g.nc = 1; break; }
  m->hm = std::move(H);
  m->plan_mesh = HostMesh();
  m->plan_ready = false;
  layout_workspace(m);
  return adg_set_state(m, Q_new, workspace_new, clock);
}

// adjoint workspace: iterate store [C][I][n][4][n][n], face-data adjoints
// [C][4][2][4][n], loss partials [C]
static void adj_layout(const adg_mesh* m, size_t* off_store, size_t* off_fd, size_t* off_part, size_t* total) {
  const size_t C = (size_t)m->g.C, n = (size_t)m->g.n, I = (size_t)m->g.iters;
  size_t off = 0;
  *off_store = off; off = align256(off + sizeof(double) * C * I * n * 4 * n * n);
  *off_fd = off; off = align256(off + sizeof(double) * C * 32 * n);
  *off_part = off; off = align256(off + sizeof(double) * C);
  *total = off;
}

static int adjoint_supported(const adg_mesh* m) {
  for (size_t k = 0; k < m->hm.nbr.size(); k += 4)
    if (m->hm.nbr[k] == kFineSide || m->hm.nbr[k] == kCoarseSide)
      return fail(ADG_EUNSUPPORTED, "the adjoint supports conforming meshes only");
  return ADG_OK;
}

int adg_adjoint_workspace_bytes(const adg_mesh* m, size_t* bytes) {
  if (!m || !bytes) return fail(ADG_EINVAL, "null argument");
  size_t a, c, d;
  adj_layout(m, &a, &c, &d, bytes);
  return ADG_OK;
}

int adg_step_adjoint(adg_mesh* m, const double* Q_n, const double* lam_np1, double* lam_n, void* adj_ws,
                     void* stream) {
  int rc = need_state(m);
  if (!rc) rc = adjoint_supported(m);
  if (rc) return rc;
  if (!Q_n || !lam_np1 || !lam_n || !adj_ws) return fail(ADG_EINVAL, "null buffer");
  if (lam_n == lam_np1) return fail(ADG_EINVAL, "lam_n must not alias lam_np1");
  if (((uintptr_t)adj_ws & 255) != 0) return fail(ADG_EINVAL, "adjoint workspace must be 256-byte aligned");
  size_t os, ofd, op, tot;
  adj_layout(m, &os, &ofd, &op, &tot);
  char* w = static_cast<char*>(adj_ws);
  return launch_step_adjoint(m->g, Q_n, lam_np1, lam_n, reinterpret_cast<double*>(w + os), m->g.FD, true,
                             reinterpret_cast<double*>(w + ofd),
                             (hipStream_t)stream);
}

int adg_keep_bytes(const adg_mesh* m, size_t* store_bytes, size_t* fd_bytes) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  const size_t C = (size_t)m->g.C, n = (size_t)m->g.n, I = (size_t)m->g.iters;
  if (store_bytes) *store_bytes = sizeof(double) * C * I * n * 4 * n * n;
  if (fd_bytes) *fd_bytes = sizeof(double) * C * 32 * n;
  return ADG_OK;
}

int adg_step_keep(adg_mesh* m, double* store, double* fd, void* stream) {
  int rc = need_state(m);
  if (!rc) rc = adjoint_supported(m);
  if (rc) return rc;
  if (!store || !fd) return fail(ADG_EINVAL, "null buffer");
  hipStream_t s = (hipStream_t)stream;
  Group gf = m->g;
  gf.FD = fd;   // the corrector reads the kept face data
  rc = launch_predictor_any(gf, store, s);
  if (rc) return rc;
  return launch_corrector_clock(gf, m->clock, s);
}

int adg_step_to(adg_mesh* m, double* Q_out, double* store, double* fd, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  if (!Q_out) return fail(ADG_EINVAL, "null buffer");
  if (((uintptr_t)Q_out & 7) != 0) return fail(ADG_EINVAL, "misaligned buffer");
  if ((store == nullptr) != (fd == nullptr)) return fail(ADG_EINVAL, "store and fd must both be given or both be NULL");
  if (store) {
    rc = adjoint_supported(m);
    if (rc) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  Group gp = m->g;
  if (fd) gp.FD = fd;   // the corrector reads the kept face data
  rc = launch_predictor_any(gp, store, s);
  if (rc) return rc;
  Group gc = gp;
  gc.Q = Q_out;         // the corrector writes Q^{n+1} here; it reads only Q* and the face data
  return launch_corrector_clock(gc, m->clock, s);
}

int adg_step_adjoint_kept(adg_mesh* m, const double* Q_n, const double* store, const double* fd,
                          const double* lam_np1, double* lam_n, void* adj_ws, void* stream) {
  int rc = need_state(m);
  if (!rc) rc = adjoint_supported(m);
  if (rc) return rc;
  if (!Q_n || !store || !fd || !lam_np1 || !lam_n || !adj_ws) return fail(ADG_EINVAL, "null buffer");
  if (lam_n == lam_np1) return fail(ADG_EINVAL, "lam_n must not alias lam_np1");
  if (((uintptr_t)adj_ws & 255) != 0) return fail(ADG_EINVAL, "adjoint workspace must be 256-byte aligned");
  size_t os, ofd, op, tot;
  adj_layout(m, &os, &ofd, &op, &tot);
  char* w = static_cast<char*>(adj_ws);
  return launch_step_adjoint(m->g, Q_n, lam_np1, lam_n, const_cast<double*>(store), fd, false,
                             reinterpret_cast<double*>(w + ofd),
                             (hipStream_t)stream);
}

int adg_ic_theta(adg_mesh* m, const double* theta_prime, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  if (!m->prm.gravity) return fail(ADG_EINVAL, "the theta' initial state needs gravity (background)");
  if (!theta_prime) return fail(ADG_EINVAL, "null buffer");
  return launch_ic_theta(m->g, theta_prime, (hipStream_t)stream);
}

int adg_ic_theta_adjoint(adg_mesh* m, const double* theta_prime, const double* lam, double* grad, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  if (!m->prm.gravity) return fail(ADG_EINVAL, "the theta' initial state needs gravity (background)");
  if (!theta_prime || !lam || !grad) return fail(ADG_EINVAL, "null buffer");
  return launch_ic_theta_adj(m->g, theta_prime, lam, grad, (hipStream_t)stream);
}

int adg_loss_theta(adg_mesh* m, double* loss, void* adj_ws, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  if (!loss || !adj_ws) return fail(ADG_EINVAL, "null buffer");
  size_t os, ofd, op, tot;
  adj_layout(m, &os, &ofd, &op, &tot);
  return launch_loss(m->g, reinterpret_cast<double*>(static_cast<char*>(adj_ws) + op), loss, (hipStream_t)stream);
}

int adg_loss_theta_adjoint(adg_mesh* m, const double* loss, const double* grad_loss, double* lam, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  if (!loss || !grad_loss || !lam) return fail(ADG_EINVAL, "null buffer");
  return launch_loss_adj(m->g, loss, grad_loss, lam, (hipStream_t)stream);
}

int adg_set_launch(adg_mesh* m, int cells_per_wave, int waves_per_block) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (cells_per_wave == 0) {   // time-level predictor: n (1), 2 or 4 wavefronts per cell
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
      return fail(ADG_EINVAL, "waves_per_block must be 1, 2 or 4 with cells_per_wave 0");
    m->g.lv = 1; m->g.lw = waves_per_block == 1 ? 0 : waves_per_block; m->g.cpw = 1; m->g.wpb = 1;
    return ADG_OK;
  }
  if ((cells_per_wave != 1 && cells_per_wave != 2 && cells_per_wave != 4) || cells_per_wave > max_cpw(m->g.n))
    return fail(ADG_EINVAL, "cells_per_wave must be 0, 1, 2 or 4 with cells_per_wave * n^2 <= 64");
  if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
    return fail(ADG_EINVAL, "waves_per_block must be 1, 2 or 4");
  m->g.lv = 0; m->g.cpw = cells_per_wave; m->g.wpb = waves_per_block;
  return ADG_OK;
}

int adg_autotune(adg_mesh* m, int reps, void* stream, int* cells_per_wave, int* waves_per_block) {
  int rc = need_state(m);
  if (rc) return rc;
  if (reps < 1) return fail(ADG_EINVAL, "reps < 1");
  rc = autotune_group(m->g, (hipStream_t)stream, reps, nullptr);
  if (rc) return rc;
  if (cells_per_wave) *cells_per_wave = m->g.lv == 1 ? 0 : m->g.cpw;
  if (waves_per_block) *waves_per_block = m->g.lv == 1 ? (level_waves(m->g) == m->g.n ? 1 : m->g.lw) : m->g.wpb;
  return ADG_OK;
}

}  // extern "C"

// ===================================================================== batch
struct adg_batch {
  int S = 0;
  adg_params prm0;                       // physical parameters shared by all scenarios
  std::vector<adg::Group> groups;        // one per distinct order
  std::vector<adg::HostBasis> bases;
  std::vector<int> scen_group, scen_c0, scen_C, scen_n;   // scenario -> group, first cell, cells, nodes
  std::vector<int> group_c0;             // first global cell of each group
  std::vector<size_t> group_q0;          // first double of each group's state
  size_t q_doubles = 0, ws_bytes = 0;
  std::vector<size_t> off_qs, off_fd;    // per group, bytes into the workspace
  size_t off_dtc = 0;
  int* d_beg = nullptr;                  // [S] global first cell
  int* d_end = nullptr;                  // [S] global end cell
  int C_total = 0;
  // bound
  double* Q = nullptr;
  void* ws = nullptr;
  double* clock = nullptr;
  double* dtc = nullptr;
  // concurrency and graph
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;        // [0] fork, [1+g] join
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t graph_stream = nullptr;
  // predictor mode: 0 one launch per order group, 1 one persistent launch per
  // order group on a work counter, resident grids sized by modelled work
  int mode = 0;
  unsigned* d_queue = nullptr;           // [2 per group]
  std::vector<int> queue_waves;          // resident wavefronts per group
};

namespace adg {

static void batch_free(adg_batch* b) {
  for (auto& g : b->groups) free_group(g);
  if (b->d_beg) (void)hipFree(b->d_beg);
  if (b->d_end) (void)hipFree(b->d_end);
  for (auto s : b->streams) (void)hipStreamDestroy(s);
  for (auto e : b->events) (void)hipEventDestroy(e);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->d_queue) (void)hipFree(b->d_queue);
  b->d_queue = nullptr;
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->streams.clear(); b->events.clear();
  b->exec = nullptr; b->graph = nullptr;
}

static int batch_need_state(adg_batch* b) {
  if (!b) return fail(ADG_EINVAL, "null batch");
  if (!b->Q || !b->ws || !b->clock) return fail(ADG_ESTATE, "no state bound (adg_batch_set_state)");
  return ADG_OK;
}

// one step of every scenario: fork one stream per order group (predictor,
// corrector), join, then one clock update for all scenarios
static int batch_enqueue_step(adg_batch* b, hipStream_t s) {
  const int G = (int)b->groups.size();
  if (hipEventRecord(b->events[0], s) != hipSuccess) return fail(ADG_EHIP, "event record");
  for (int g = 0; g < G; ++g) {
    hipStream_t gs = b->streams[g];
    if (hipStreamWaitEvent(gs, b->events[0], 0) != hipSuccess) return fail(ADG_EHIP, "stream wait");
    int rc = b->mode == 1 ? launch_predictor_queue(b->groups[g], b->d_queue + 2 * g, b->queue_waves[g], gs)
                          : launch_predictor_any(b->groups[g], nullptr, gs);
    if (!rc) rc = launch_corrector(b->groups[g], gs);
    if (rc) return rc;
    if (hipEventRecord(b->events[1 + g], gs) != hipSuccess) return fail(ADG_EHIP, "event record");
    if (hipStreamWaitEvent(s, b->events[1 + g], 0) != hipSuccess) return fail(ADG_EHIP, "stream wait");
  }
  return launch_clock(b->clock, b->dtc, b->d_beg, b->d_end, b->S, b->C_total, 1, b->prm0.fixed_dt ? 0 : 1, s);
}

}  // namespace adg

extern "C" {

int adg_batch_create(const adg_params* prm, const adg_mesh_desc* mesh, int n_scen, adg_batch** out) {
  if (!out || !prm || !mesh) return fail(ADG_EINVAL, "null argument");
  if (n_scen < 1 || n_scen > 4096) return fail(ADG_EINVAL, "n_scen must be in 1..4096");
  for (int s = 0; s < n_scen; ++s) {
    int rc = validate_params(&prm[s]);
    if (!rc) rc = validate_mesh(&mesh[s]);
    if (rc) return fail(rc, "scenario " + std::to_string(s) + ": " + g_err);
    const adg_params& a = prm[0], &c = prm[s];
    if (a.gamma != c.gamma || a.Pr != c.Pr || a.R != c.R || a.cp != c.cp || a.mu != c.mu || a.g != c.g ||
        a.p0 != c.p0 || a.theta_bg != c.theta_bg || a.gravity != c.gravity || a.mms != c.mms || a.cfl != c.cfl ||
        a.fixed_dt != c.fixed_dt || a.picard_iters != c.picard_iters)
      return fail(ADG_EINVAL, "scenarios of a batch must share all parameters except the order");
  }
  adg_batch* b = new (std::nothrow) adg_batch();
  if (!b) return fail(ADG_ENOMEM, "out of host memory");
  b->S = n_scen;
  b->prm0 = prm[0];
  std::vector<HostMesh> hms(n_scen);
  for (int s = 0; s < n_scen; ++s) {
    int rc = build_mesh(mesh[s], hms[s]);
    if (rc) { delete b; return fail(rc, "scenario " + std::to_string(s) + ": " + g_err); }
  }
  // group by order (ascending)
  std::vector<int> orders;
  for (int s = 0; s < n_scen; ++s) orders.push_back(prm[s].order);
  std::sort(orders.begin(), orders.end());
  orders.erase(std::unique(orders.begin(), orders.end()), orders.end());
  const int G = (int)orders.size();
  b->groups.resize(G); b->bases.resize(G);
  b->scen_group.resize(n_scen); b->scen_c0.resize(n_scen); b->scen_C.resize(n_scen); b->scen_n.resize(n_scen);
  b->group_c0.resize(G); b->group_q0.resize(G); b->off_qs.resize(G); b->off_fd.resize(G);
  std::vector<int> beg(n_scen), end(n_scen);
  int cglob = 0;
  size_t q0 = 0;
  for (int gi = 0; gi < G; ++gi) {
    const int N = orders[gi], n = N + 1;
    build_basis(n, b->bases[gi]);
    std::vector<double> geom;
    std::vector<int> nbr, scen;
    int C = 0;
    for (int s = 0; s < n_scen; ++s) {
      if (prm[s].order != N) continue;
      const HostMesh& H = hms[s];
      b->scen_group[s] = gi; b->scen_c0[s] = C; b->scen_C[s] = H.C; b->scen_n[s] = n;
      beg[s] = cglob + C; end[s] = cglob + C + H.C;
      geom.insert(geom.end(), H.geom.begin(), H.geom.end());
      for (int k = 0; k < H.C * 16; ++k) {
        const int f = (k % 16) / 4, slot = k % 4;
        (void)f;
        int v = H.nbr[k];
        const int kind = H.nbr[k - slot];
        // cell references are local to the scenario: shift into the group
        if (slot > 0 && v >= 0) {
          const bool is_cell = (kind == kConforming && slot == 1) || (kind == kFineSide && slot == 1) ||
                               (kind == kCoarseSide);
          if (is_cell) v += C;
        }
        nbr.push_back(v);
      }
      for (int c = 0; c < H.C; ++c) scen.push_back(s);
      C += H.C;
    }
    Group& g = b->groups[gi];
    g.n = n; g.N = N; g.iters = prm[0].picard_iters > 0 ? prm[0].picard_iters : n; g.C = C;
    adg_params pg = prm[0];
    pg.order = N;
    g.ph = make_phys(pg);
    g.cpw = max_cpw(n); g.wpb = 1;
    int rc = upload_group(g, geom, nbr, b->bases[gi].gtab, &scen);
    if (rc) { batch_free(b); delete b; return rc; }
    b->group_c0[gi] = cglob;
    b->group_q0[gi] = q0;
    q0 += (size_t)C * 4 * n * n;
    cglob += C;
  }
  b->C_total = cglob;
  b->q_doubles = q0;
  size_t off = 0;
  for (int gi = 0; gi < G; ++gi) {
    const size_t C = b->groups[gi].C, n = b->groups[gi].n;
    b->off_qs[gi] = off; off = align256(off + sizeof(double) * C * 4 * n * n);
    b->off_fd[gi] = off; off = align256(off + sizeof(double) * C * 32 * n);
  }
  b->off_dtc = off; off = align256(off + sizeof(double) * (size_t)cglob);
  b->ws_bytes = off;
  if (hipMalloc(&b->d_beg, sizeof(int) * n_scen) != hipSuccess ||
      hipMalloc(&b->d_end, sizeof(int) * n_scen) != hipSuccess ||
      hipMemcpy(b->d_beg, beg.data(), sizeof(int) * n_scen, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_end, end.data(), sizeof(int) * n_scen, hipMemcpyHostToDevice) != hipSuccess) {
    batch_free(b); delete b;
    return fail(ADG_ENOMEM, "device allocation failed");
  }
  b->streams.resize(G, nullptr);
  b->events.resize(G + 1, nullptr);
  for (int gi = 0; gi < G; ++gi)
    if (hipStreamCreateWithFlags(&b->streams[gi], hipStreamNonBlocking) != hipSuccess) {
      batch_free(b); delete b;
      return fail(ADG_EHIP, "stream creation failed");
    }
  for (int k = 0; k <= G; ++k)
    if (hipEventCreateWithFlags(&b->events[k], hipEventDisableTiming) != hipSuccess) {
      batch_free(b); delete b;
      return fail(ADG_EHIP, "event creation failed");
    }
  *out = b;
  return ADG_OK;
}

int adg_batch_destroy(adg_batch* b) {
  if (!b) return fail(ADG_EINVAL, "null batch");
  batch_free(b);
  delete b;
  return ADG_OK;
}

int adg_batch_info(const adg_batch* b, int* n_groups, int* total_cells, size_t* q_doubles, size_t* ws_bytes) {
  if (!b) return fail(ADG_EINVAL, "null batch");
  if (n_groups) *n_groups = (int)b->groups.size();
  if (total_cells) *total_cells = b->C_total;
  if (q_doubles) *q_doubles = b->q_doubles;
  if (ws_bytes) *ws_bytes = b->ws_bytes;
  return ADG_OK;
}

int adg_batch_scenario(const adg_batch* b, int s, size_t* q_offset, int* n_cells, int* n_nodes) {
  if (!b) return fail(ADG_EINVAL, "null batch");
  if (s < 0 || s >= b->S) return fail(ADG_EINVAL, "scenario out of range");
  const int gi = b->scen_group[s], n = b->scen_n[s];
  if (q_offset) *q_offset = b->group_q0[gi] + (size_t)b->scen_c0[s] * 4 * n * n;
  if (n_cells) *n_cells = b->scen_C[s];
  if (n_nodes) *n_nodes = n;
  return ADG_OK;
}

int adg_batch_set_state(adg_batch* b, double* Q, void* workspace, double* clocks) {
  if (!b) return fail(ADG_EINVAL, "null batch");
  if (!Q || !workspace || !clocks) return fail(ADG_EINVAL, "null buffer");
  if (((uintptr_t)workspace & 255) != 0) return fail(ADG_EINVAL, "workspace must be 256-byte aligned");
  if (((uintptr_t)Q & 7) != 0 || ((uintptr_t)clocks & 7) != 0) return fail(ADG_EINVAL, "misaligned buffer");
  b->Q = Q; b->ws = workspace; b->clock = clocks;
  char* ws = static_cast<char*>(workspace);
  b->dtc = reinterpret_cast<double*>(ws + b->off_dtc);
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    Group& g = b->groups[gi];
    g.Q = Q + b->group_q0[gi];
    g.Qs = reinterpret_cast<double*>(ws + b->off_qs[gi]);
    g.FD = reinterpret_cast<double*>(ws + b->off_fd[gi]);
    g.dtc = b->dtc + b->group_c0[gi];
    g.clock = clocks;
  }
  // a captured graph holds the old pointers
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return ADG_OK;
}

int adg_batch_init_state(adg_batch* b, int s, int kind, int n_bubbles, const double* bubbles, double t0,
                         void* stream) {
  int rc = batch_need_state(b);
  if (rc) return rc;
  if (s < 0 || s >= b->S) return fail(ADG_EINVAL, "scenario out of range");
  rc = check_bubbles(kind, b->prm0.gravity, n_bubbles, bubbles);
  if (rc) return rc;
  return init_state_range(b->groups[b->scen_group[s]], b->scen_c0[s], b->scen_C[s], kind, n_bubbles, bubbles, t0,
                          (hipStream_t)stream);
}

int adg_batch_compute_dt(adg_batch* b, void* stream) {
  int rc = batch_need_state(b);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (auto& g : b->groups) {
    rc = launch_cell_dt(g, s);
    if (rc) return rc;
  }
  return launch_clock(b->clock, b->dtc, b->d_beg, b->d_end, b->S, b->C_total, 0, 1, s);
}

int adg_batch_step(adg_batch* b, void* stream) {
  int rc = batch_need_state(b);
  if (rc) return rc;
  return batch_enqueue_step(b, (hipStream_t)stream);
}

int adg_batch_step_graph(adg_batch* b, void* stream) {
  int rc = batch_need_state(b);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(ADG_EINVAL, "graph steps need a non-default stream");
  if (b->exec && b->graph_stream != s) {
    (void)hipGraphExecDestroy(b->exec); b->exec = nullptr;
    (void)hipGraphDestroy(b->graph); b->graph = nullptr;
  }
  if (!b->exec) {
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail(ADG_EHIP, "begin capture failed");
    rc = batch_enqueue_step(b, s);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess || !graph) return fail(ADG_EHIP, "end capture failed");
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(ADG_EHIP, "graph instantiation failed");
    }
    b->graph = graph; b->exec = exec; b->graph_stream = s;
  }
  if (hipGraphLaunch(b->exec, s) != hipSuccess) return fail(ADG_EHIP, "graph launch failed");
  return ADG_OK;
}

int adg_batch_autotune(adg_batch* b, int reps, void* stream, int* cells_per_wave, int* waves_per_block) {
  int rc = batch_need_state(b);
  if (rc) return rc;
  if (reps < 1) return fail(ADG_EINVAL, "reps < 1");
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    rc = autotune_group(b->groups[gi], (hipStream_t)stream, reps, nullptr);
    if (rc) return rc;
    if (cells_per_wave) cells_per_wave[gi] = b->groups[gi].lv == 1 ? 0 : b->groups[gi].cpw;
    if (waves_per_block) {
      const Group& gg = b->groups[gi];
      waves_per_block[gi] = gg.lv == 1 ? (level_waves(gg) == gg.n ? 1 : gg.lw) : gg.wpb;
    }
  }
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return ADG_OK;
}

int adg_batch_set_mode(adg_batch* b, int mode) {
  if (!b) return fail(ADG_EINVAL, "null batch");
  if (mode != 0 && mode != 1) return fail(ADG_EINVAL, "mode must be 0 (launch per order) or 1 (persistent)");
  if (mode == 1 && b->prm0.mms == 2)
    return fail(ADG_EUNSUPPORTED, "the persistent batch predictor has no manufactured-solution source");
  if (mode == 1 && !b->d_queue) {
    const int G = (int)b->groups.size();
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      return fail(ADG_EHIP, "device query failed");
    // resident wavefronts: every group's share of the chip, by modelled
    // predictor work (cells x (N+1)^4), of the slots its own occupancy allows
    double tot = 0.0;
    std::vector<double> w(G);
    for (int g = 0; g < G; ++g) {
      const double n = b->groups[g].n;
      w[g] = b->groups[g].C * n * n * n * n;
      tot += w[g];
    }
    b->queue_waves.assign(G, 1);
    for (int g = 0; g < G; ++g) {
      int per_cu = 0;
      int rc = predictor_queue_occupancy(b->groups[g].n, &per_cu);
      if (rc) return rc;
      b->queue_waves[g] = std::max(1, (int)(cus * per_cu * (w[g] / tot) + 0.5));
    }
    if (hipMalloc(&b->d_queue, sizeof(unsigned) * 2 * (size_t)G) != hipSuccess ||
        hipMemset(b->d_queue, 0, sizeof(unsigned) * 2 * (size_t)G) != hipSuccess)
      return fail(ADG_ENOMEM, "work counter allocation failed");
  }
  b->mode = mode;
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return ADG_OK;
}

int adg_batch_set_launch(adg_batch* b, int group, int cells_per_wave, int waves_per_block) {
  if (!b) return fail(ADG_EINVAL, "null batch");
  if (group < 0 || group >= (int)b->groups.size()) return fail(ADG_EINVAL, "group out of range");
  Group& g = b->groups[group];
  if (cells_per_wave == 0) {   // time-level predictor: n (1), 2 or 4 wavefronts per cell
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
      return fail(ADG_EINVAL, "waves_per_block must be 1, 2 or 4 with cells_per_wave 0");
    g.lv = 1; g.lw = waves_per_block == 1 ? 0 : waves_per_block; g.cpw = 1; g.wpb = 1;
  } else {
    if ((cells_per_wave != 1 && cells_per_wave != 2 && cells_per_wave != 4) || cells_per_wave > max_cpw(g.n))
      return fail(ADG_EINVAL, "cells_per_wave must be 0, 1, 2 or 4 with cells_per_wave * n^2 <= 64");
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
      return fail(ADG_EINVAL, "waves_per_block must be 1, 2 or 4");
    g.lv = 0; g.cpw = cells_per_wave; g.wpb = waves_per_block;
  }
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return ADG_OK;
}

}  // extern "C"
