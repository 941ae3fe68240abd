// Auxiliary kernels for gfx950: initial state, total-variation indicator with
// Chan-merged statistics and refinement flags, state health check.
#include <algorithm>

#include "adg_internal.h"

namespace adg {

// --------------------------------------------------------- initial state
// One thread per node.  kind 0: hydrostatic background of constant potential
// temperature perturbed in theta at fixed pressure (rho from p = rho R T,
// T = theta * Exner, at rest); kind 1: the manufactured density wave at t0;
// kind 2: the paper's manufactured solution at t0.
__global__ void k_init_state(Phys ph, int n, int C, const double* geom, const double* gtab, int kind,
                             int nbub, const double* bub, double t0, double* Q) {
  // geom and Q point at the first cell of the range
  const int nn = n * n;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)C * nn) return;
  const int c = (int)(gid / nn), node = (int)(gid % nn);
  const int jz = node / n, ix = node % n;
  const double h = geom[4 * c + 2];
  const double x = geom[4 * c + 0] + h * gtab[GTab::XI * n + ix];
  const double z = geom[4 * c + 1] + h * gtab[GTab::XI * n + jz];
  double q[4];
  if (kind == 2) {
    paper_wave_state(ph, x, z, t0, q);
  } else if (kind == 1) {
    const double rho = 1.0 + ph.mms_amp * sin(ph.mms_kx * (x - ph.mms_u * t0)) * sin(ph.mms_kz * (z - ph.mms_w * t0));
    q[0] = rho; q[1] = rho * ph.mms_u; q[2] = rho * ph.mms_w;
    q[3] = ph.mms_p / ph.gm1 + 0.5 * rho * (ph.mms_u * ph.mms_u + ph.mms_w * ph.mms_w);
  } else {
    double dth = 0.0;
    for (int b = 0; b < nbub; ++b) {
      const double* bb = bub + 6 * b;
      const double dx = x - bb[4], dz = z - bb[5];
      const double r = sqrt(dx * dx + dz * dz);
      if ((int)bb[0] == ADG_SHAPE_COSINE) {
        if (r <= bb[2]) dth += 0.5 * bb[1] * (1.0 + cos(M_PI * r / bb[2]));
      } else {
        const double e = (r - bb[2]) / bb[3];
        dth += (r <= bb[2]) ? bb[1] : bb[1] * exp(-e * e);
      }
    }
    const double pi = 1.0 - ph.ex_coef * z;
    const double pb = ph.p0 * pow(pi, ph.cp_over_R);
    const double T = (ph.theta + dth) * pi;
    const double rho = pb / (ph.R * T);
    q[0] = rho; q[1] = 0.0; q[2] = 0.0;
    q[3] = pb / ph.gm1 + rho * ph.g * z;
  }
  for (int v = 0; v < 4; ++v) Q[(size_t)c * 4 * nn + v * nn + node] = q[v];
}

// ------------------------------------------------------------- TV per cell
// TV = (1/h) sum_ji w_i w_j (|sum_m D_im f_jm| + |sum_m D_jm f_mi|), f =
// theta or rho at the nodes: the mean of |df/dx| + |df/dz| over the cell
// (eq. tv by GL quadrature with the reference element's weights, which sum
// to one, of the physical gradient).  A wavefront holds 64 / P cells, P the
// power of two >= n^2, one lane per node: the lane forms f, then both
// derivatives at its node from the cell's values in LDS; the cell's P lanes
// sum the weighted node terms in a butterfly.
constexpr int kTvThreads = 256;
constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }
// cells per workgroup of k_tv
template <int n>
constexpr int tv_cells_per_block() { return (kTvThreads / kWave) * (kWave / pow2_at_least(n * n)); }
template <int n>
__global__ __launch_bounds__(kTvThreads) void k_tv(Phys ph, int C, const double* Q, const double* geom,
                                                    const double* gtab, int var, double* tv) {
  constexpr int nn = n * n, P = pow2_at_least(nn), K = kWave / P, CB = tv_cells_per_block<n>();
  __shared__ double sf[CB * nn];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int slot = lane / P, node = lane % P;
  const int cs = wave * K + slot;                           // cell within the workgroup
  const int c = blockIdx.x * CB + cs;
  const bool valid = node < nn && c < C;
  const int jz = node / n, ix = node % n;
  double h = 1.0;
  if (valid) {
    const double z0 = geom[4 * c + 1];
    h = geom[4 * c + 2];
    const double* Qc = Q + (size_t)c * 4 * nn;
    const double rho = Qc[node];
    double f = rho;
    if (var == ADG_VAR_THETA) {
      const double z = z0 + h * gtab[GTab::XI * n + jz];
      const double p = pressure(ph, rho, Qc[nn + node], Qc[2 * nn + node], Qc[3 * nn + node], z);
      const double Tm = p / (rho * ph.R);
      f = Tm * pow(ph.p0 / p, ph.R_over_cp);
    }
    sf[cs * nn + node] = f;
  }
  __syncthreads();
  double part = 0.0;
  if (valid) {
    const double* Di = gtab + GTab::d(n) + ix * n;   // row i of D
    const double* Dj = gtab + GTab::d(n) + jz * n;   // row j of D
    const double* fc = sf + cs * nn;
    double dx = 0.0, dz = 0.0;
#pragma unroll
    for (int m = 0; m < n; ++m) {
      dx = fma(Di[m], fc[jz * n + m], dx);
      dz = fma(Dj[m], fc[m * n + ix], dz);
    }
    part = gtab[GTab::W * n + ix] * gtab[GTab::W * n + jz] * (fabs(dx) + fabs(dz));
  }
#pragma unroll
  for (int o = 1; o < P; o <<= 1) part += __shfl_xor(part, o, kWave);
  if (node == 0 && c < C) tv[c] = part / h;
}

// ---------------------------------------------------- statistics and flags
// Single workgroup: each thread folds a contiguous chunk of cells with the
// one-element updates of Chan, Golub & LeVeque (count, mean, M2); partials are
// then merged pairwise in a fixed tree.  Deterministic for a given C.
// stats = (count, mean, population sigma); flags as in the refinement rule.
constexpr int kStatThreads = 1024;

__device__ inline void chan_merge(double& na, double& ma, double& qa, double nb, double mb, double qb) {
  const double nt = na + nb;
  if (nb == 0.0) return;
  if (na == 0.0) { na = nb; ma = mb; qa = qb; return; }
  const double d = mb - ma;
  ma = ma + d * nb / nt;
  qa = qa + qb + d * d * na * nb / nt;
  na = nt;
}

__device__ inline void chan_shfl(double& na, double& ma, double& qa, int o) {
  const double nb = __shfl_xor(na, o, kWave), mb = __shfl_xor(ma, o, kWave), qb = __shfl_xor(qa, o, kWave);
  // both partners merge (lower lane's partial first) so they hold the same result
  const bool low = (threadIdx.x & o) == 0;
  double n1 = low ? na : nb, m1 = low ? ma : mb, q1 = low ? qa : qb;
  chan_merge(n1, m1, q1, low ? nb : na, low ? mb : ma, low ? qb : qa);
  na = n1; ma = m1; qa = q1;
}

// One workgroup: each thread folds the cells t, t + 1024, ... in one at a
// time (Welford's update, the Chan merge of a single value: exact for equal
// values, so a constant field keeps sigma = 0); partials are merged by Chan's
// formulas in a fixed butterfly within each wavefront, then across the 16
// wavefronts in order.
__global__ __launch_bounds__(kStatThreads) void k_stats_flags(const double* tv, int C, double Tr, double Tc,
                                                                 int8_t* flags, double* stats) {
  constexpr int nw = kStatThreads / kWave;
  __shared__ double sn[nw], sm[nw], sq[nw], sres[2];
  const int t = threadIdx.x;
  double na = 0.0, ma = 0.0, qa = 0.0;
  for (int c = t; c < C; c += kStatThreads) {
    const double x = tv[c];
    const double nt = na + 1.0;
    const double d = x - ma;
    const double r = 1.0 / nt;
    ma = fma(d, r, ma);
    qa = fma(d * d, na * r, qa);
    na = nt;
  }
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) chan_shfl(na, ma, qa, o);
  if ((t & (kWave - 1)) == 0) { sn[t / kWave] = na; sm[t / kWave] = ma; sq[t / kWave] = qa; }
  __syncthreads();
  if (t == 0) {
    double cn = sn[0], cm = sm[0], cq = sq[0];
    for (int w = 1; w < nw; ++w) chan_merge(cn, cm, cq, sn[w], sm[w], sq[w]);
    const double sigma = cn > 0.0 ? sqrt(cq / cn) : 0.0;
    stats[0] = cn; stats[1] = cm; stats[2] = sigma;
    sres[0] = cm; sres[1] = sigma;
  }
  __syncthreads();
  const double mean = sres[0], sigma = sres[1];
  const double thr_r = mean + Tr * sigma, thr_c = mean + Tc * sigma;
  for (int c = t; c < C; c += kStatThreads) {
    int8_t f = 0;
    if (sigma != 0.0) {
      const double v = tv[c];
      if (v >= thr_r) f = 1;
      else if (v < thr_c) f = -1;
    }
    flags[c] = f;
  }
}

// Many cells: each workgroup folds a contiguous range of cells into (count,
// mean, M2) as above and writes its partial; one workgroup merges the
// partials in workgroup order (Chan), writes the statistics and keeps the
// threshold pair; a grid then writes the flags.  Deterministic for a given C.
constexpr int kStatSingle = 65536;   // up to this many cells: the single-workgroup kernel

__global__ __launch_bounds__(kStatThreads) void k_stats_part(const double* tv, int C, int per_block, double* part) {
  constexpr int nw = kStatThreads / kWave;
  __shared__ double sn[nw], sm[nw], sq[nw];
  const int t = threadIdx.x;
  const int beg = blockIdx.x * per_block, end = min(C, beg + per_block);
  double na = 0.0, ma = 0.0, qa = 0.0;
  for (int c = beg + t; c < end; c += kStatThreads) {
    const double x = tv[c];
    const double nt = na + 1.0;
    const double d = x - ma;
    const double r = 1.0 / nt;
    ma = fma(d, r, ma);
    qa = fma(d * d, na * r, qa);
    na = nt;
  }
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) chan_shfl(na, ma, qa, o);
  if ((t & (kWave - 1)) == 0) { sn[t / kWave] = na; sm[t / kWave] = ma; sq[t / kWave] = qa; }
  __syncthreads();
  if (t == 0) {
    double cn = sn[0], cm = sm[0], cq = sq[0];
    for (int w = 1; w < nw; ++w) chan_merge(cn, cm, cq, sn[w], sm[w], sq[w]);
    part[3 * blockIdx.x + 0] = cn;
    part[3 * blockIdx.x + 1] = cm;
    part[3 * blockIdx.x + 2] = cq;
  }
}

// merge of the nparts partials (one wavefront: a Chan butterfly over lanes
// holding parts k, k + 64, ..., folded in order first); stats as above, and
// (mean + Tr sigma, mean + Tc sigma, sigma) to thr for the flag pass
__global__ __launch_bounds__(kWave) void k_stats_merge(const double* part, int nparts, double Tr, double Tc,
                                                      double* stats, double* thr) {
  const int t = threadIdx.x;
  double na = 0.0, ma = 0.0, qa = 0.0;
  for (int k = t; k < nparts; k += kWave) chan_merge(na, ma, qa, part[3 * k], part[3 * k + 1], part[3 * k + 2]);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) chan_shfl(na, ma, qa, o);
  if (t == 0) {
    const double sigma = na > 0.0 ? sqrt(qa / na) : 0.0;
    stats[0] = na; stats[1] = ma; stats[2] = sigma;
    thr[0] = ma + Tr * sigma; thr[1] = ma + Tc * sigma; thr[2] = sigma;
  }
}

__global__ void k_flags(const double* tv, int C, const double* thr, int8_t* flags) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const double sigma = thr[2];
  int8_t f = 0;
  if (sigma != 0.0) {
    const double v = tv[c];
    if (v >= thr[0]) f = 1;
    else if (v < thr[1]) f = -1;
  }
  flags[c] = f;
}

// ------------------------------------------------------------------ health
__global__ void k_health(Phys ph, int n, int C, const double* Q, const double* geom, const double* gtab,
                         int* flag) {
  const int nn = n * n;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)C * nn) return;
  const int c = (int)(gid / nn), node = (int)(gid % nn);
  const double* Qc = Q + (size_t)c * 4 * nn;
  const double rho = Qc[node], mx = Qc[nn + node], mz = Qc[2 * nn + node], E = Qc[3 * nn + node];
  const double z = geom[4 * c + 1] + geom[4 * c + 2] * gtab[GTab::XI * n + node / n];
  bool bad = !(isfinite(rho) && isfinite(mx) && isfinite(mz) && isfinite(E)) || !(rho > 0.0);
  if (!bad) bad = !(pressure(ph, rho, mx, mz, E, z) > 0.0);
  if (bad) atomicOr(flag, 1);
}

// --------------------------------------------------------------- launchers
int launch_init_state(const Group& g, int c0, int count, int kind, int nbub, const double* d_bub, double t0,
                      hipStream_t s) {
  const long long tot = (long long)count * g.n * g.n;
  if (tot == 0) return ADG_OK;
  const int bs = 256;
  const long long nb = (tot + bs - 1) / bs;
  hipLaunchKernelGGL(k_init_state, dim3((unsigned)nb), dim3(bs), 0, s, g.ph, g.n, count, g.d_geom + 4 * (size_t)c0,
                     g.d_gtab, kind, nbub, d_bub, t0, g.Q + (size_t)c0 * 4 * g.n * g.n);
  return check_launch("init_state");
}

template <int n>
static int launch_tv_n(const Group& g, int var, double* tv, hipStream_t s) {
  constexpr int CB = tv_cells_per_block<n>();
  hipLaunchKernelGGL(k_tv<n>, dim3((g.C + CB - 1) / CB), dim3(kTvThreads), 0, s, g.ph, g.C, g.Q, g.d_geom, g.d_gtab,
                     var, tv);
  return check_launch("tv");
}

int launch_tv(const Group& g, int var, double Tr, double Tc, double* tv, int8_t* flags,
              double* stats, hipStream_t s) {
  int rc;
  if (g.C == 0) return fail(ADG_EINVAL, "empty mesh");
  switch (g.n) {
    case 2: rc = launch_tv_n<2>(g, var, tv, s); break;
    case 3: rc = launch_tv_n<3>(g, var, tv, s); break;
    case 4: rc = launch_tv_n<4>(g, var, tv, s); break;
    case 5: rc = launch_tv_n<5>(g, var, tv, s); break;
    case 6: rc = launch_tv_n<6>(g, var, tv, s); break;
    case 7: rc = launch_tv_n<7>(g, var, tv, s); break;
    case 8: rc = launch_tv_n<8>(g, var, tv, s); break;
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
  if (rc) return rc;
  if (g.C <= kStatSingle || !g.d_part) {
    hipLaunchKernelGGL(k_stats_flags, dim3(1), dim3(kStatThreads), 0, s, tv, g.C, Tr, Tc, flags, stats);
    return check_launch("stats_flags");
  }
  // contiguous ranges of at least kStatThreads cells, at most kStatParts of them
  const int per = std::max(kStatThreads, (g.C + kStatParts - 1) / kStatParts);
  const int nparts = (g.C + per - 1) / per;
  double* part = g.d_part;
  double* thr = g.d_part + 3 * kStatParts;
  hipLaunchKernelGGL(k_stats_part, dim3(nparts), dim3(kStatThreads), 0, s, tv, g.C, per, part);
  hipLaunchKernelGGL(k_stats_merge, dim3(1), dim3(kWave), 0, s, part, nparts, Tr, Tc, stats, thr);
  hipLaunchKernelGGL(k_flags, dim3((g.C + 255) / 256), dim3(256), 0, s, tv, g.C, thr, flags);
  return check_launch("stats_flags");
}

int launch_health(const Group& g, int* flag, hipStream_t s) {
  const long long tot = (long long)g.C * g.n * g.n;
  if (tot == 0) return ADG_OK;
  const int bs = 256;
  hipLaunchKernelGGL(k_health, dim3((unsigned)((tot + bs - 1) / bs)), dim3(bs), 0, s, g.ph, g.n, g.C, g.Q,
                     g.d_geom, g.d_gtab, flag);
  return check_launch("health");
}

}  // namespace adg
