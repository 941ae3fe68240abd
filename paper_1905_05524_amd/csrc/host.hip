// Host side of the C ABI: parameter validation, Gauss-Legendre basis, leaf
// list and face tables, handle lifetime, workspace layout, dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "adg_internal.h"

namespace adg {

int launch_predictor(adg_mesh* m, hipStream_t s);
int launch_corrector(adg_mesh* m, hipStream_t s);
int launch_dt(adg_mesh* m, hipStream_t s);
int launch_init_state(adg_mesh* m, int kind, int nbub, const double* d_bub, double t0, hipStream_t s);
int launch_tv(adg_mesh* m, int var, double Tr, double Tc, double* tv, int8_t* flags, double* stats,
              hipStream_t s);
int launch_health(adg_mesh* m, int* flag, hipStream_t s);

static thread_local std::string g_err;

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

static void build_basis(adg_mesh* m) {
  const int n = m->n;
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
  m->xi.resize(n); m->w.resize(n); m->e0.resize(n); m->e1.resize(n);
  m->D.resize(n * n); m->P.resize(n * n); m->Dw.resize(n * n);
  for (int k = 0; k < n; ++k) {
    m->xi[k] = (double)x[k]; m->w[k] = (double)w[k];
    m->e0[k] = (double)e0[k]; m->e1[k] = (double)e1[k];
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      m->D[i * n + j] = (double)D[i * n + j];
      m->P[i * n + j] = (double)X[i * n + j];
      m->Dw[i * n + j] = (double)(w[j] * D[j * n + i] / w[i]);
    }
  m->gtab_h.assign(GTab::size(n), 0.0);
  for (int k = 0; k < n; ++k) {
    m->gtab_h[GTab::XI * n + k] = (double)x[k];
    m->gtab_h[GTab::W * n + k] = (double)w[k];
    m->gtab_h[GTab::L0 * n + k] = (double)(e0[k] / w[k]);
    m->gtab_h[GTab::L1 * n + k] = (double)(e1[k] / w[k]);
    m->gtab_h[GTab::E0 * n + k] = (double)e0[k];
    m->gtab_h[GTab::E1 * n + k] = (double)e1[k];
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      m->gtab_h[GTab::d(n) + i * n + j] = m->D[i * n + j];
      m->gtab_h[GTab::pt(n) + j * n + i] = m->P[i * n + j];
      m->gtab_h[GTab::dw(n) + i * n + j] = m->Dw[i * n + j];
    }
  for (int s = 0; s < 3; ++s)
    for (int q = 0; q < n; ++q)
      for (int mm = 0; mm < n; ++mm) {
        long double ph = bary_phi(x, lam, mm, (s + x[q]) / 3.0L);
        m->gtab_h[GTab::pk(n) + (s * n + q) * n + mm] = (double)ph;
        m->gtab_h[GTab::rk(n) + (s * n + mm) * n + q] = (double)((w[q] / 3.0L) * ph / w[mm]);
      }
}

// ------------------------------------------------------------------- mesh
static long long key3(int l, int i, int j) { return ((long long)l << 52) ^ ((long long)i << 26) ^ (long long)j; }
static int pow3(int e) { int r = 1; while (e-- > 0) r *= 3; return r; }

static int build_mesh(adg_mesh* m) {
  const adg_mesh_desc& d = m->desc;
  const bool uniform = d.leaf_level == nullptr;
  const int C = uniform ? d.nx * d.nz : d.n_leaves;
  m->C = C;
  m->lev.resize(C); m->ci.resize(C); m->cj.resize(C);
  for (int c = 0; c < C; ++c) {
    if (uniform) { m->lev[c] = 0; m->ci[c] = c % d.nx; m->cj[c] = c / d.nx; }
    else { m->lev[c] = d.leaf_level[c]; m->ci[c] = d.leaf_i[c]; m->cj[c] = d.leaf_j[c]; }
    const int l = m->lev[c];
    if (l < 0 || l > d.max_level) return fail(ADG_EINVAL, "leaf level out of range");
    const int s = pow3(l);
    if (m->ci[c] < 0 || m->ci[c] >= d.nx * s || m->cj[c] < 0 || m->cj[c] >= d.nz * s)
      return fail(ADG_EINVAL, "leaf index out of range");
  }
  std::unordered_map<long long, int> idx;
  idx.reserve((size_t)C * 2);
  long long area = 0;
  const int L = d.max_level;
  for (int c = 0; c < C; ++c) {
    if (!idx.emplace(key3(m->lev[c], m->ci[c], m->cj[c]), c).second) return fail(ADG_EINVAL, "duplicate leaf");
    const long long s = pow3(L - m->lev[c]);
    area += s * s;
  }
  const long long full = (long long)d.nx * pow3(L) * (long long)d.nz * pow3(L);
  if (area != full) return fail(ADG_EINVAL, "leaves do not tile the domain");
  for (int c = 0; c < C; ++c) {   // no leaf may have an ancestor among the leaves
    int l = m->lev[c], i = m->ci[c], j = m->cj[c];
    while (l > 0) {
      l -= 1; i /= 3; j /= 3;
      if (idx.count(key3(l, i, j))) return fail(ADG_EINVAL, "leaf overlaps an ancestor");
    }
  }
  const double hc = d.Lx / d.nx;
  m->geom_h.assign((size_t)C * 4, 0.0);
  m->nbr_h.assign((size_t)C * 16, -1);
  for (int c = 0; c < C; ++c) {
    const int l = m->lev[c];
    const double h = hc / pow3(l);
    m->geom_h[4 * c + 0] = d.x0 + m->ci[c] * h;
    m->geom_h[4 * c + 1] = d.z0 + m->cj[c] * h;
    m->geom_h[4 * c + 2] = h;
  }
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  for (int c = 0; c < C; ++c) {
    const int l = m->lev[c];
    const int NX = d.nx * pow3(l), NZ = d.nz * pow3(l);
    for (int f = 0; f < 4; ++f) {
      int* nb = &m->nbr_h[(size_t)c * 16 + f * 4];
      int i = m->ci[c] + di[f], j = m->cj[c] + dj[f];
      if (i < 0 || i >= NX || j < 0 || j >= NZ) {
        if (d.bc[f] == ADG_BC_WALL) { nb[0] = kWall; continue; }
        i = (i + NX) % NX; j = (j + NZ) % NZ;
      }
      auto it = idx.find(key3(l, i, j));
      if (it != idx.end()) { nb[0] = kConforming; nb[1] = it->second; continue; }
      if (l > 0) {
        auto pc = idx.find(key3(l - 1, i / 3, j / 3));
        if (pc != idx.end()) {
          nb[0] = kFineSide; nb[1] = pc->second;
          nb[2] = (f < 2) ? (m->cj[c] % 3) : (m->ci[c] % 3);
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
          auto kc = idx.find(key3(l + 1, ci2, cj2));
          if (kc == idx.end()) { ok = false; break; }
          kids[s] = kc->second;
        }
        if (ok) { nb[0] = kCoarseSide; nb[1] = kids[0]; nb[2] = kids[1]; nb[3] = kids[2]; continue; }
      }
      return fail(ADG_EINVAL, "neighbouring leaves differ by more than one level");
    }
  }
  return ADG_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int validate(const adg_params* p, const adg_mesh_desc* d) {
  if (!p || !d) return fail(ADG_EINVAL, "null params or mesh");
  if (p->order < 1 || p->order > kMaxN - 1) return fail(ADG_EINVAL, "order must be in 1..7");
  if (p->picard_iters < 0) return fail(ADG_EINVAL, "picard_iters < 0");
  if (!(p->gamma > 1.0) || !(p->R > 0.0) || !(p->cp > 0.0) || !(p->Pr > 0.0) || !(p->mu >= 0.0))
    return fail(ADG_EINVAL, "invalid gas constants");
  if (p->gravity && (!(p->theta_bg > 0.0) || !(p->p0 > 0.0) || !(p->g >= 0.0)))
    return fail(ADG_EINVAL, "invalid background atmosphere");
  if (!(p->cfl > 0.0)) return fail(ADG_EINVAL, "cfl must be > 0");
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
  return ADG_OK;
}

static void set_phys(adg_mesh* m) {
  const adg_params& p = m->prm;
  Phys& ph = m->ph;
  ph.gamma = p.gamma; ph.gm1 = p.gamma - 1.0; ph.R = p.R; ph.iR = 1.0 / p.R; ph.cp = p.cp; ph.Pr = p.Pr;
  ph.mu = p.mu; ph.kappa = p.mu * p.cp / p.Pr; ph.g = p.g; ph.p0 = p.p0; ph.theta = p.theta_bg;
  ph.cp_over_R = p.cp / p.R; ph.R_over_cp = p.R / p.cp;
  ph.ex_coef = p.gravity ? p.g / (p.cp * p.theta_bg) : 0.0;
  ph.lv_coef = std::max(4.0 * p.mu / 3.0, p.gamma * p.mu / p.Pr);
  ph.mms_amp = p.mms_amp; ph.mms_u = p.mms_u; ph.mms_w = p.mms_w;
  ph.mms_kx = p.mms_kx; ph.mms_kz = p.mms_kz; ph.mms_p = p.mms_p;
  ph.cfl = p.cfl; ph.gravity = p.gravity ? 1 : 0; ph.mms = p.mms ? 1 : 0; ph.fixed_dt = p.fixed_dt ? 1 : 0;
  ph.N = p.order;
}

static void free_dev(adg_mesh* m) {
  if (m->d_geom) (void)hipFree(m->d_geom);
  if (m->d_nbr) (void)hipFree(m->d_nbr);
  if (m->d_gtab) (void)hipFree(m->d_gtab);
  m->d_geom = nullptr; m->d_nbr = nullptr; m->d_gtab = nullptr;
}

static int need_state(adg_mesh* m) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (!m->Q || !m->ws || !m->clock) return fail(ADG_ESTATE, "no state bound (adg_set_state)");
  return ADG_OK;
}

}  // namespace adg

using namespace adg;

extern "C" {

const char* adg_last_error(void) { return g_err.c_str(); }

int adg_init_mesh(const adg_params* prm, const adg_mesh_desc* mesh, adg_mesh** out) {
  if (!out) return fail(ADG_EINVAL, "null out");
  int rc = validate(prm, mesh);
  if (rc) return rc;
  adg_mesh* m = new (std::nothrow) adg_mesh();
  if (!m) return fail(ADG_ENOMEM, "out of host memory");
  m->prm = *prm;
  m->desc = *mesh;
  m->desc.leaf_level = m->desc.leaf_i = m->desc.leaf_j = nullptr;
  m->N = prm->order; m->n = prm->order + 1;
  m->iters = prm->picard_iters > 0 ? prm->picard_iters : prm->order + 1;
  set_phys(m);
  // build the mesh from the caller's leaf arrays (not retained)
  adg_mesh_desc d = *mesh;
  m->desc = d;
  rc = build_mesh(m);
  m->desc.leaf_level = m->desc.leaf_i = m->desc.leaf_j = nullptr;
  if (rc) { delete m; return rc; }
  for (size_t k = 0; k < m->nbr_h.size(); k += 4)
    if (m->nbr_h[k] == kFineSide || m->nbr_h[k] == kCoarseSide) {
      delete m;
      return fail(ADG_EUNSUPPORTED, "non-conforming faces are not supported by this build");
    }
  build_basis(m);
  const int C = m->C, n = m->n;
  hipError_t e = hipMalloc(&m->d_geom, sizeof(double) * 4 * C);
  if (e == hipSuccess) e = hipMalloc(&m->d_nbr, sizeof(int) * 16 * C);
  if (e == hipSuccess) e = hipMalloc(&m->d_gtab, sizeof(double) * m->gtab_h.size());
  if (e != hipSuccess) { free_dev(m); delete m; return fail(ADG_ENOMEM, "device allocation failed"); }
  e = hipMemcpy(m->d_geom, m->geom_h.data(), sizeof(double) * 4 * C, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->d_nbr, m->nbr_h.data(), sizeof(int) * 16 * C, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m->d_gtab, m->gtab_h.data(), sizeof(double) * m->gtab_h.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { free_dev(m); delete m; return fail(ADG_EHIP, "upload failed"); }
  // workspace: Q* [C][4][n][n], face data [C][4][2][4][n], health flag
  size_t off = 0;
  m->off_qs = off; off = align256(off + sizeof(double) * (size_t)C * 4 * n * n);
  m->off_fd = off; off = align256(off + sizeof(double) * (size_t)C * 32 * n);
  m->off_dtc = off; off = align256(off + sizeof(double) * (size_t)C);
  m->off_health = off; off = align256(off + sizeof(int));
  m->ws_bytes = off;
  *out = m;
  return ADG_OK;
}

int adg_destroy(adg_mesh* m) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  free_dev(m);
  delete m;
  return ADG_OK;
}

int adg_mesh_info(const adg_mesh* m, int* n_cells, int* n_nodes) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (n_cells) *n_cells = m->C;
  if (n_nodes) *n_nodes = m->n;
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
  return ADG_OK;
}

int adg_init_state(adg_mesh* m, int kind, int n_bubbles, const double* bubbles, double t0, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  if (kind != 0 && kind != 1) return fail(ADG_EINVAL, "kind must be 0 (bubbles) or 1 (manufactured)");
  if (kind == 0 && !m->prm.gravity) return fail(ADG_EINVAL, "bubble states need gravity (background)");
  if (n_bubbles < 0 || n_bubbles > 16 || (n_bubbles > 0 && !bubbles)) return fail(ADG_EINVAL, "bad bubble list");
  for (int b = 0; b < n_bubbles; ++b) {
    const double* bb = bubbles + 6 * b;
    if (bb[0] != ADG_SHAPE_COSINE && bb[0] != ADG_SHAPE_PLATEAU_GAUSS) return fail(ADG_EINVAL, "bad bubble shape");
    if (bb[0] == ADG_SHAPE_COSINE && !(bb[2] > 0.0)) return fail(ADG_EINVAL, "cosine bubble radius must be > 0");
    if (bb[0] == ADG_SHAPE_PLATEAU_GAUSS && !(bb[3] > 0.0)) return fail(ADG_EINVAL, "decay s must be > 0");
  }
  // the bubble list travels through a small device copy owned by the call's stream order
  double* d_bub = nullptr;
  if (n_bubbles > 0) {
    if (hipMalloc(&d_bub, sizeof(double) * 6 * n_bubbles) != hipSuccess) return fail(ADG_ENOMEM, "alloc");
    if (hipMemcpy(d_bub, bubbles, sizeof(double) * 6 * n_bubbles, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d_bub);
      return fail(ADG_EHIP, "upload bubbles");
    }
  }
  rc = launch_init_state(m, kind, n_bubbles, d_bub, t0, (hipStream_t)stream);
  if (d_bub) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(d_bub);
  }
  return rc;
}

int adg_compute_dt(adg_mesh* m, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  return launch_dt(m, (hipStream_t)stream);
}

int adg_predictor(adg_mesh* m, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  return launch_predictor(m, (hipStream_t)stream);
}

int adg_corrector(adg_mesh* m, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  return launch_corrector(m, (hipStream_t)stream);
}

int adg_step(adg_mesh* m, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  rc = launch_predictor(m, (hipStream_t)stream);
  if (rc) return rc;
  return launch_corrector(m, (hipStream_t)stream);
}

int adg_tv_indicator(adg_mesh* m, int var, double T_refine, double T_coarsen, double* tv, int8_t* flags,
                     double* stats, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  if (var != ADG_VAR_THETA && var != ADG_VAR_RHO) return fail(ADG_EINVAL, "var must be THETA or RHO");
  if (var == ADG_VAR_THETA && !(m->prm.p0 > 0.0)) return fail(ADG_EINVAL, "theta needs p0 > 0");
  if (!tv || !flags || !stats) return fail(ADG_EINVAL, "null output");
  if (!(T_refine > T_coarsen)) return fail(ADG_EINVAL, "T_refine must exceed T_coarsen");
  return launch_tv(m, var, T_refine, T_coarsen, tv, flags, stats, (hipStream_t)stream);
}

int adg_check_health(adg_mesh* m, void* stream) {
  int rc = need_state(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  int* flag = reinterpret_cast<int*>(static_cast<char*>(m->ws) + m->off_health);
  if (hipMemsetAsync(flag, 0, sizeof(int), s) != hipSuccess) return fail(ADG_EHIP, "memset");
  rc = launch_health(m, flag, s);
  if (rc) return rc;
  int h = 0;
  if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return fail(ADG_EHIP, "copy");
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ADG_EHIP, "sync");
  if (h) return fail(ADG_ESTATE, "state has non-finite values or non-positive density/pressure");
  return ADG_OK;
}

int adg_basis(const adg_mesh* m, double* xi, double* w, double* D, double* P) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  const int n = m->n;
  if (xi) std::memcpy(xi, m->xi.data(), sizeof(double) * n);
  if (w) std::memcpy(w, m->w.data(), sizeof(double) * n);
  if (D) std::memcpy(D, m->D.data(), sizeof(double) * n * n);
  if (P) std::memcpy(P, m->P.data(), sizeof(double) * n * n);
  return ADG_OK;
}

}  // extern "C"
