// Host side of the three-dimensional C ABI: validation, handle lifetime,
// workspace layout and dispatch of the kernels in step3.hip.
#include <cmath>
#include <new>

#include "adg3_internal.h"

namespace adg {

static size_t align256_3(size_t x) { return (x + 255) & ~(size_t)255; }

static int validate_mesh3(const adg3_mesh_desc* d) {
  if (!d) return fail(ADG_EINVAL, "null mesh");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1 || !(d->h > 0.0) || !std::isfinite(d->h))
    return fail(ADG_EINVAL, "invalid domain");
  if (!std::isfinite(d->x0) || !std::isfinite(d->y0) || !std::isfinite(d->z0))
    return fail(ADG_EINVAL, "invalid domain");
  for (int f = 0; f < 6; ++f)
    if (d->bc[f] != ADG_BC_PERIODIC && d->bc[f] != ADG_BC_WALL) return fail(ADG_EINVAL, "invalid bc");
  for (int a = 0; a < 3; ++a)
    if ((d->bc[2 * a] == ADG_BC_PERIODIC) != (d->bc[2 * a + 1] == ADG_BC_PERIODIC))
      return fail(ADG_EINVAL, "periodic boundaries must come in pairs");
  const long long cells = (long long)d->nx * d->ny * d->nz;
  if (cells > (1LL << 24)) return fail(ADG_EINVAL, "too many cells");
  return ADG_OK;
}

static Args3 args_of(const adg3_mesh* m) {
  Args3 a{};
  char* ws = static_cast<char*>(m->ws);
  a.Q = m->Q; a.Qout = m->Q;
  a.Qs = ws ? reinterpret_cast<double*>(ws + m->off_qs) : nullptr;
  a.FD = ws ? reinterpret_cast<double*>(ws + m->off_fd) : nullptr;
  a.dtc = ws ? reinterpret_cast<double*>(ws + m->off_dtc) : nullptr;
  a.clock = m->clock; a.gtab = m->d_gtab;
  a.nx = m->desc.nx; a.ny = m->desc.ny; a.nz = m->desc.nz; a.C = m->C; a.iters = m->iters;
  a.wall = 0;
  for (int f = 0; f < 6; ++f)
    if (m->desc.bc[f] == ADG_BC_WALL) a.wall |= 1 << f;
  a.x0 = m->desc.x0; a.y0 = m->desc.y0; a.z0 = m->desc.z0; a.h = m->desc.h;
  a.eta = (2.0 * m->prm.order + 1.0) / (m->desc.h * std::sqrt(M_PI / 2.0));
  return a;
}

static int need_state3(adg3_mesh* m) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (!m->Q || !m->ws || !m->clock) return fail(ADG_ESTATE, "no state bound (adg3_set_state)");
  return ADG_OK;
}

}  // namespace adg

using namespace adg;

extern "C" {

int adg3_init_mesh(const adg_params* prm, const adg3_mesh_desc* mesh, adg3_mesh** out) {
  if (!out) return fail(ADG_EINVAL, "null out");
  int rc = validate_params(prm);
  if (!rc) rc = validate_mesh3(mesh);
  if (rc) return rc;
  if (prm->order > 5) return fail(ADG_EINVAL, "order must be in 1..5 in 3D");
  if (prm->mms) return fail(ADG_EUNSUPPORTED, "the manufactured source is two-dimensional");
  adg3_mesh* m = new (std::nothrow) adg3_mesh();
  if (!m) return fail(ADG_ENOMEM, "out of host memory");
  m->prm = *prm;
  m->desc = *mesh;
  m->n = prm->order + 1;
  m->C = mesh->nx * mesh->ny * mesh->nz;
  m->iters = prm->picard_iters > 0 ? prm->picard_iters : m->n;
  m->ph = make_phys(*prm);
  build_basis(m->n, m->basis);
  const size_t tb = sizeof(double) * m->basis.gtab.size();
  if (hipMalloc(&m->d_gtab, tb) != hipSuccess) { delete m; return fail(ADG_ENOMEM, "device allocation failed"); }
  if (hipMemcpy(m->d_gtab, m->basis.gtab.data(), tb, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(m->d_gtab);
    delete m;
    return fail(ADG_EHIP, "upload failed");
  }
  const size_t C = (size_t)m->C, nd = (size_t)m->n * m->n * m->n, nn = (size_t)m->n * m->n;
  size_t off = 0;
  m->off_qs = off; off = align256_3(off + sizeof(double) * C * 5 * nd);
  m->off_fd = off; off = align256_3(off + sizeof(double) * C * 60 * nn);
  m->off_dtc = off; off = align256_3(off + sizeof(double) * C);
  m->off_health = off; off = align256_3(off + sizeof(int));
  m->ws_bytes = off;
  *out = m;
  return ADG_OK;
}

int adg3_destroy(adg3_mesh* m) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (m->d_gtab) (void)hipFree(m->d_gtab);
  delete m;
  return ADG_OK;
}

int adg3_mesh_info(const adg3_mesh* m, int* n_cells, int* n_nodes) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (n_cells) *n_cells = m->C;
  if (n_nodes) *n_nodes = m->n;
  return ADG_OK;
}

int adg3_workspace_bytes(const adg3_mesh* m, size_t* bytes) {
  if (!m || !bytes) return fail(ADG_EINVAL, "null argument");
  *bytes = m->ws_bytes;
  return ADG_OK;
}

int adg3_set_state(adg3_mesh* m, double* Q, void* workspace, double* clock) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (!Q || !workspace || !clock) return fail(ADG_EINVAL, "null buffer");
  if (((uintptr_t)workspace & 255) != 0) return fail(ADG_EINVAL, "workspace must be 256-byte aligned");
  if (((uintptr_t)Q & 7) != 0 || ((uintptr_t)clock & 7) != 0) return fail(ADG_EINVAL, "misaligned buffer");
  m->Q = Q; m->ws = workspace; m->clock = clock;
  return ADG_OK;
}

int adg3_init_state(adg3_mesh* m, int kind, int n_bubbles, const double* bubbles, double t0, void* stream) {
  int rc = need_state3(m);
  if (rc) return rc;
  if (kind != 0 && kind != 1) return fail(ADG_EINVAL, "kind must be 0 (bubbles) or 1 (ABC flow)");
  if (kind == 0 && !m->prm.gravity) return fail(ADG_EINVAL, "bubble states need gravity (background)");
  if (n_bubbles < 0 || n_bubbles > kMaxBubbles3 || (n_bubbles > 0 && !bubbles))
    return fail(ADG_EINVAL, "bad bubble list");
  Bubbles3 B{};
  B.nb = kind == 0 ? n_bubbles : 0;
  for (int b = 0; b < B.nb; ++b) {
    const double* bb = bubbles + 7 * b;
    if (bb[0] != ADG_SHAPE_COSINE && bb[0] != ADG_SHAPE_PLATEAU_GAUSS) return fail(ADG_EINVAL, "bad bubble shape");
    if (bb[0] == ADG_SHAPE_COSINE && !(bb[2] > 0.0)) return fail(ADG_EINVAL, "cosine bubble radius must be > 0");
    if (bb[0] == ADG_SHAPE_PLATEAU_GAUSS && !(bb[3] > 0.0)) return fail(ADG_EINVAL, "decay s must be > 0");
    for (int q = 0; q < 7; ++q) B.b[7 * b + q] = bb[q];
  }
  return launch_init3(m->ph, m->n, args_of(m), kind, B, t0, m->Q, (hipStream_t)stream);
}

int adg3_compute_dt(adg3_mesh* m, void* stream) {
  int rc = need_state3(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const Args3 a = args_of(m);
  rc = launch_dt3(m->ph, m->n, a, s);
  if (rc) return rc;
  return launch_clock(m->clock, a.dtc, nullptr, nullptr, 1, m->C, 0, 1, s);
}

int adg3_predictor(adg3_mesh* m, void* stream) {
  int rc = need_state3(m);
  if (rc) return rc;
  return launch_pred3(m->ph, m->basis, args_of(m), (hipStream_t)stream);
}

int adg3_corrector(adg3_mesh* m, void* stream) {
  int rc = need_state3(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const Args3 a = args_of(m);
  rc = launch_corr3(m->ph, m->n, a, s);
  if (rc) return rc;
  return launch_clock(m->clock, a.dtc, nullptr, nullptr, 1, m->C, 1, m->ph.fixed_dt ? 0 : 1, s);
}

int adg3_step(adg3_mesh* m, void* stream) {
  int rc = adg3_predictor(m, stream);
  if (rc) return rc;
  return adg3_corrector(m, stream);
}

int adg3_check_health(adg3_mesh* m, void* stream) {
  int rc = need_state3(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  int* flag = reinterpret_cast<int*>(static_cast<char*>(m->ws) + m->off_health);
  if (hipMemsetAsync(flag, 0, sizeof(int), s) != hipSuccess) return fail(ADG_EHIP, "memset");
  rc = launch_health3(m->ph, m->n, args_of(m), flag, s);
  if (rc) return rc;
  int h = 0;
  if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return fail(ADG_EHIP, "copy");
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ADG_EHIP, "sync");
  if (h) return fail(ADG_ESTATE, "state has non-finite values or non-positive density/pressure");
  return ADG_OK;
}

}  // extern "C"
