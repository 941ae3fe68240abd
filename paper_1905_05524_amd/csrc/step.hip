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

template <int n>
struct Half { static constexpr int nh = (n + 1) / 2; };

// Two-layout LDS regions (the predictor with several cells per wavefront;
// the corrector's sizes).  Each time slice is kept twice: as [4 vars][z][x]
// and transposed as [4 vars][x][z], so that every line job (one lane per
// direction, variable and line: x lines in the first layout, z lines in the
// second) reads and writes n consecutive values.  Gradients, fluxes and
// divergences follow the same pairing: the x parts in the first layout, the
// z parts in the transposed one.  Lines that start n doubles apart (n odd)
// measured no LDS bank conflicts in the job order used here.  With one cell
// per wavefront the slice is kept once (PLay below).
template <int n, int CPW>
struct Lay {
  static constexpr int nn = n * n, sl = 4 * nn;
  static constexpr int T = sl;                             // transposed copy of a region
  static constexpr int F0 = 2 * sl;                        // gradients / fluxes region
  static constexpr int jobs = 8 * n * CPW;                 // line jobs per wavefront
  static constexpr int rounds = (jobs + kWave - 1) / kWave;
  static constexpr int corr_cell = 16 * n + 24 * n + 48 * n;  // sG, sL/sV, sGs
};

// most cells per wavefront for n nodes per direction (at most four)
constexpr int max_cpw_c(int n) { return (4 * n * n <= kWave) ? 4 : ((2 * n * n <= kWave) ? 2 : 1); }

// Line job of one lane in one round: direction, variable, line, cell slot and
// the offset of its first value within a region (x lines in the first
// layout, z lines in the transposed one; unit stride in both).
template <int n>
struct LineJob {
  int dir, base, slot, v, line;
  bool active;
  __device__ LineJob(int job, int cpw) {
    constexpr int nn = n * n;
    slot = job / (8 * n);
    active = slot < cpw;
    const int jj = job % (8 * n);
    dir = jj / (4 * n);
    v = (jj % (4 * n)) / n;
    line = jj % n;
    base = (dir ? 4 * nn : 0) + v * nn + line * n;
  }
};

// LDS layout of the per-cell predictor (k_predictor, the persistent batch
// predictor).  The slice is written once, as [4 vars][z][x], and the z line
// jobs of the gradient pass read it with stride n; the gradients, fluxes and
// divergences keep their two parts (x part [v][z][x], z part [v][x][z]), so
// every other line access has unit stride.  Writing the slice once removes
// a quarter of the LDS writes of a time level.  Jobs are variable-major as in
// LineJob.  With one cell per wavefront the x jobs start at lane 0 and the z
// jobs at the first 16-lane boundary after them (at n = 7 that measured half
// the LDS bank-conflict cycles of z jobs packed right after the x jobs, and
// fewer than variables padded to other strides or line-major job orders).
// With several cells per wavefront, two rounds of line jobs and odd n, the
// first round runs every x job and the second every z job, so that each
// round has one stride (3 % faster at n = 3 and 5; at n = 4 the stride-4 z
// reads measured 2.5 % slower).  Otherwise, with several cells per
// wavefront, the slice is kept in both layouts (Lay).
template <int n, int CPW>
struct PLay {
  static constexpr int nn = n * n;
  static constexpr bool one = CPW == 1;
  static constexpr bool split = CPW > 1 && Lay<n, CPW>::rounds == 2 && n % 2 == 1;   // x round, z round
  static constexpr bool single = one || split;       // the slice in one layout
  static constexpr int ST = 4 * nn;                  // transposed slice (two-layout case)
  static constexpr int GX = single ? 4 * nn : 8 * nn;   // x part of gradients / fluxes
  static constexpr int GZ = GX + 4 * nn;             // z part
  static constexpr int SM = GZ + 4 * nn;             // manufactured source, staging of the averages
  static constexpr int cell = SM + (n > 5 ? n : 5) * nn;   // doubles per cell
  static constexpr int Z0 = ((4 * n + 15) / 16) * 16;      // first z job's lane (one cell per wavefront)
  static constexpr int rounds = one ? 1 : Lay<n, CPW>::rounds;
  static_assert(!one || Z0 + 4 * n <= kWave, "one round of line jobs");
  static_assert(!split || 4 * n * CPW <= kWave, "the x jobs fit one round");
};

// Line job of one lane in one round of the per-cell predictor: direction,
// variable, line, cell slot; the gradient pass reads n values from src with
// stride sst() and writes them to dst (unit stride), where the divergence
// pass and the face extrapolation of the fluxes also work; the face
// extrapolation of the state reads the src line.
template <int n, int CPW>
struct PJob {
  int dir, slot, v, line, src, dst;
  bool active;
  // the stride of the src line; with one cell per wavefront it is derived
  // from src and dst alone (z jobs: dst - src > 4 n^2), so that it need not
  // be kept in a register through the sweeps
  __device__ int sst() const {
    using P = PLay<n, CPW>;
    if constexpr (P::one) {
      int d = dst;
      asm volatile("" : "+v"(d));
      return d - src > 4 * n * n ? n : 1;
    } else if constexpr (P::split) {
      return dir ? n : 1;
    } else {
      return 1;
    }
  }
  __device__ PJob(int job) {
    using P = PLay<n, CPW>;
    constexpr int nn = n * n;
    if constexpr (P::one) {
      dir = job >= P::Z0;
      const int j = dir ? job - P::Z0 : job;
      active = j < 4 * n;
      const int jj = active ? j : 0;
      slot = 0;
      v = jj / n;
      line = jj % n;
      src = dir ? v * nn + line : v * nn + line * n;
      dst = (dir ? P::GZ : P::GX) + v * nn + line * n;
    } else if constexpr (P::split) {
      dir = job >= kWave;
      const int j = dir ? job - kWave : job;
      slot = j / (4 * n);
      active = slot < CPW;
      const int jj = active ? j % (4 * n) : 0;
      if (!active) slot = 0;
      v = jj / n;
      line = jj % n;
      src = dir ? v * nn + line : v * nn + line * n;
      dst = (dir ? P::GZ : P::GX) + v * nn + line * n;
    } else {
      const LineJob<n> J(job, CPW);
      dir = J.dir; slot = J.slot; v = J.v; line = J.line; active = J.active;
      src = J.base;
      dst = P::GX + J.base;
    }
  }
};

// Even-odd tables of a centro-antisymmetric n x n matrix in VGPRs (layout
// and formulas with GTab).  The empty asm marks every value as lane-varying
// so the compiler keeps the tables in vector registers.
template <int n>
struct EOTab {
  static constexpr int h = n / 2;
  double A[h][h], B[h][h], C[h], M[h];
};
template <int n>
__device__ inline void load_eo(const double* g, EOTab<n>& T) {
  constexpr int h = n / 2;
#pragma unroll
  for (int i = 0; i < h; ++i) {
#pragma unroll
    for (int m = 0; m < h; ++m) {
      T.A[i][m] = g[i * h + m];
      T.B[i][m] = g[h * h + i * h + m];
      asm volatile("" : "+v"(T.A[i][m]), "+v"(T.B[i][m]));
    }
    if constexpr (n % 2) {   // the short middle column and row may live in scalar registers
      T.C[i] = g[2 * h * h + i];
      T.M[i] = g[2 * h * h + h + i];
    }
  }
}

// dst line = T * src line (n consecutive values at base); src may equal dst.
template <int n>
__device__ inline void line_eo(const EOTab<n>& T, int base, const double* src, double* dst) {
  constexpr int stride = 1;
  constexpr int h = n / 2, mid = (n - 1) / 2;
  double in[n];
#pragma unroll
  for (int m = 0; m < n; ++m) in[m] = src[base + m * stride];
  double e[h], o[h];
#pragma unroll
  for (int m = 0; m < h; ++m) { e[m] = in[m] + in[n - 1 - m]; o[m] = in[m] - in[n - 1 - m]; }
#pragma unroll
  for (int i = 0; i < h; ++i) {
    double S = T.A[i][0] * o[0], U = T.B[i][0] * e[0];
#pragma unroll
    for (int m = 1; m < h; ++m) { S = fma(T.A[i][m], o[m], S); U = fma(T.B[i][m], e[m], U); }
    if constexpr (n % 2) U = fma(T.C[i], in[mid], U);
    dst[base + i * stride] = S + U;
    dst[base + (n - 1 - i) * stride] = S - U;
  }
  if constexpr (n % 2) {
    double S = T.M[0] * o[0];
#pragma unroll
    for (int m = 1; m < h; ++m) S = fma(T.M[m], o[m], S);
    dst[base + mid * stride] = S;
  }
}

// d line = T * (n values of s with stride ss); d has unit stride.  SS > 0:
// the stride is SS, known at compile time (immediate offsets).
template <int n, int SS = 0>
__device__ inline void line_eo_s(const EOTab<n>& T, const double* s, int ss, double* d) {
  constexpr int h = n / 2, mid = (n - 1) / 2;
  // a run-time stride is opaque to the compiler at each call, so that the n
  // read addresses are formed here rather than hoisted and held in registers
  if constexpr (SS > 0) ss = SS;
  else asm volatile("" : "+v"(ss));
  double in[n];
#pragma unroll
  for (int m = 0; m < n; ++m) in[m] = s[m * ss];
  double e[h], o[h];
#pragma unroll
  for (int m = 0; m < h; ++m) { e[m] = in[m] + in[n - 1 - m]; o[m] = in[m] - in[n - 1 - m]; }
#pragma unroll
  for (int i = 0; i < h; ++i) {
    double S = T.A[i][0] * o[0], U = T.B[i][0] * e[0];
#pragma unroll
    for (int m = 1; m < h; ++m) { S = fma(T.A[i][m], o[m], S); U = fma(T.B[i][m], e[m], U); }
    if constexpr (n % 2) U = fma(T.C[i], in[mid], U);
    d[i] = S + U;
    d[n - 1 - i] = S - U;
  }
  if constexpr (n % 2) {
    double S = T.M[0] * o[0];
#pragma unroll
    for (int m = 1; m < h; ++m) S = fma(T.M[m], o[m], S);
    d[mid] = S;
  }
}

// A wave-uniform double moved to scalar registers.
__device__ inline double uniform(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
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
  double* advance;      // optional clock [4] the corrector advances (t += dt, steps += 1)
  int C, iters;
};

// ------------------------------------------------------------------ predictor
// Flux and source of one time node at this lane's node: state q (registers),
// reference-coordinate gradients from the gradient region (x parts at node offset l of the first
// layout, z parts at offset tl of the transposed one); the fluxes overwrite
// the gradients in place (each lane reads and writes only its own node)
// unless store is false.
template <int n>
__device__ inline double node_flux(const Phys& ph, const double q[4], double* sf, int l, int tl, double mu_h,
                                   double kappa_h, double gh, double z, double rb, double pb, double Fx[4],
                                   double Fz[4], bool store) {
  constexpr int nn = n * n, T = 4 * nn;
  double gx[4], gz[4], Sw;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    gx[v] = sf[v * nn + l];
    gz[v] = sf[T + v * nn + tl];
  }
  flux_source(ph, q, gx, gz, z, rb, pb, mu_h, kappa_h, gh, Fx, Fz, Sw);
  if (store) {
#pragma unroll
    for (int v = 0; v < 4; ++v) { sf[v * nn + l] = Fx[v]; sf[T + v * nn + tl] = Fz[v]; }
  }
  return Sw;
}

// Up to n = 7 the kernel is held to 168 VGPRs, three wavefronts per SIMD.
// Per cell: lane l < n*n owns spatial node l = (j, i) and holds, in
// registers, the Picard iterate at all n time nodes, X[b][v] (the time-node
// loop is unrolled so the array is statically indexed).  Per sweep and time
// node b: the slice X[b] goes to LDS, gradients by line jobs,
// flux and source per node (fluxes over the gradients), divergence by line
// jobs in place, and the residual R(b) replaces X[b] (the old iterate at b is
// no longer needed).  At the end of the sweep the time solve
// X[a] = Q^n + dt sum_b P[a][b] R(b) runs per node in registers.  Then time
// averages, the volume term and the face data.  PW: the variant with the
// source of the paper's manufactured solution (a separate instantiation, so
// that the source's temporaries do not add to the register pressure of the
// other workloads).
//
// predictor_wave is the work of wavefront `wave` of a workgroup on CPW cells
// starting at cell0, in that wavefront's LDS region; k_predictor runs it on
// consecutive cells, the persistent batch predictor on cells handed out by a
// work counter.
template <int n, int CPW, bool PW>
__device__ __forceinline__ void predictor_wave(Phys ph, StepArgs a, int wave, int cell0) {
  using P = PLay<n, CPW>;
  constexpr int nn = P::nn, sl = 4 * nn, ZO = 4 * nn;   // z part of gradients / fluxes
  extern __shared__ double lds[];
  const int lane = threadIdx.x % kWave;
  double* wl = lds + (size_t)wave * CPW * P::cell;

  // node role
  const int slot = lane / nn, l = lane % nn;
  const bool node = slot < CPW;
  // (with one cell per wavefront the cell index is wave-uniform)
  const int c = CPW == 1 ? cell0 : cell0 + (node ? slot : 0);
  const bool valid = node && c < a.C;
  const int cc = CPW == 1 ? (cell0 < a.C ? cell0 : 0) : (valid ? c : 0);
  const int jz = l / n, ix = l % n;
  const int tl = ix * n + jz;                           // node offset in the transposed layout
  double* sq = wl + (node ? slot : 0) * P::cell;       // slice
  double* sf = sq + P::GX;                              // gradients / fluxes: x part, z part at ZO
  double* sm = sq + P::SM;                              // [n][n*n] manufactured source (if any)
  const double* gt = a.gtab;

  // cell-level values: with one cell per wavefront they are read through a
  // wave-uniform index (scalar registers)
  const int cu = (CPW == 1) ? (cell0 < a.C ? cell0 : a.C - 1) : cc;
  const int s = a.scen ? a.scen[cu] : 0;
  const double t0 = a.clock[4 * s + 0], dt = a.clock[4 * s + 1];
  const double x0 = a.geom[4 * cu + 0], z0 = a.geom[4 * cu + 1], h = a.geom[4 * cu + 2];
  double ih = 1.0 / h, mu_h = ph.mu * ih, kappa_h = ph.kappa * ih, gh = ph.geff * h;
  if constexpr (CPW == 1) { ih = uniform(ih); mu_h = uniform(mu_h); kappa_h = uniform(kappa_h); gh = uniform(gh); }
  const double z = z0 + h * gt[GTab::XI * n + jz];
  double rb, pb;
  background(ph, z, rb, pb);

  EOTab<n> Dt;
  load_eo<n>(gt + GTab::eo_d(n), Dt);

  // Q^n of this node (lanes past the last cell read cell 0 and store nothing);
  // it is re-read from memory where needed rather than held in registers
  const double* Qc = a.Qin + (size_t)cc * sl + l;
  double X[n][4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double q = Qc[v * nn];
#pragma unroll
    for (int b = 0; b < n; ++b) X[b][v] = q;
  }

  // manufactured energy source of the density wave at the n time nodes (it
  // does not depend on the state), evaluated once
  if ((!PW && ph.mms) && node) {
    const double x = x0 + h * gt[GTab::XI * n + ix];
#pragma unroll 1
    for (int b = 0; b < n; ++b) sm[b * nn + l] = mms_source(ph, x, z, t0 + gt[GTab::XI * n + b] * dt);
  }

  // line-job roles (rounds of 64 jobs)
  const PJob<n, CPW> J0(lane), J1(lane + kWave);
  double* jl0 = wl + (J0.active ? J0.slot : 0) * P::cell;
  double* jl1 = wl + (J1.active ? J1.slot : 0) * P::cell;
  // the gradient pass (slice to gradients) and the divergence pass (fluxes,
  // in place)
  // with one cell per wavefront the job's two offsets are kept packed in one
  // register through the sweeps (opaque to the compiler, so that it does not
  // keep the unpacked values instead)
  int jp0 = J0.src | (J0.dst << 16);
  if constexpr (P::one) asm volatile("" : "+v"(jp0));
  auto grad_lines = [&]() {
    if constexpr (P::split) {   // x jobs in the first round, z jobs in the second
      if (J0.active) line_eo_s<n, 1>(Dt, jl0 + J0.src, 1, jl0 + J0.dst);
      if (J1.active) line_eo_s<n, n>(Dt, jl1 + J1.src, n, jl1 + J1.dst);
    } else if constexpr (P::one) {
      const int s0 = jp0 & 0xffff, d0 = jp0 >> 16;
      if (J0.active) line_eo_s<n>(Dt, jl0 + s0, d0 - s0 > 4 * nn ? n : 1, jl0 + d0);
    } else {
      if (J0.active) line_eo_s<n>(Dt, jl0 + J0.src, J0.sst(), jl0 + J0.dst);
      if (P::rounds > 1 && J1.active) line_eo_s<n>(Dt, jl1 + J1.src, J1.sst(), jl1 + J1.dst);
    }
  };
  auto div_lines = [&]() {
    if constexpr (P::one) {
      if (J0.active) line_eo<n>(Dt, jp0 >> 16, jl0, jl0);
    } else {
      if (J0.active) line_eo<n>(Dt, J0.dst, jl0, jl0);
      if (P::rounds > 1 && J1.active) line_eo<n>(Dt, J1.dst, jl1, jl1);
    }
  };
  auto put_slice = [&](const double q[4]) {
    if (node) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sq[v * nn + l] = q[v];
        if constexpr (!P::single) sq[P::ST + v * nn + tl] = q[v];
      }
    }
  };

#pragma unroll 1
  for (int it = 0; it < a.iters; ++it) {
#pragma unroll
    for (int b = 0; b < n; ++b) {
      if (b > 0 && it == 0 && !PW) {
        // the first sweep starts from Q^n at every time node, so every node
        // has the residual of node 0 (bit for bit); only the manufactured
        // source depends on the time node: node 0's divergence of the energy
        // flux is still in LDS.  (With the paper's wave, whose source acts
        // on every variable, the first sweep evaluates every time node.)
        if (node) {
          X[b][0] = X[0][0];
          X[b][1] = X[0][1];
          X[b][2] = X[0][2];
          X[b][3] = ph.mms ? fma(-h, sm[b * nn + l], sf[3 * nn + l] + sf[ZO + 3 * nn + tl]) : X[0][3];
        }
        continue;
      }
      put_slice(X[b]);
      wave_sync();
      grad_lines();                          // gradients of time node b
      wave_sync();
      double Sw = 0.0;
      if (node) {
        double Fx[4], Fz[4];
        Sw = node_flux<n>(ph, X[b], sf, l, tl, mu_h, kappa_h, gh, z, rb, pb, Fx, Fz, true);
      }
      wave_sync();
      div_lines();                           // divergence parts, in place
      wave_sync();
      if (node) {   // scaled residual R' = div F - h S, with R = -R' / h
#pragma unroll
        for (int v = 0; v < 4; ++v) X[b][v] = sf[v * nn + l] + sf[ZO + v * nn + tl];
        X[b][2] = fma(-h, Sw, X[b][2]);
        if ((!PW && ph.mms)) X[b][3] = fma(-h, sm[b * nn + l], X[b][3]);
        if constexpr (PW) {
          double Sm[4];
          paper_wave_source(ph, x0 + h * gt[GTab::XI * n + ix], z, t0 + gt[GTab::XI * n + b] * dt, Sm);
#pragma unroll
          for (int v = 0; v < 4; ++v) X[b][v] = fma(-h, Sm[v], X[b][v]);
        }
      }
    }
    // time solve per node, in place: X[a] = Q^n + dt (K1^{-1} W R)[a] by
    // forward and back substitution with the unpivoted LU factors of K1
    // (equal to applying P = K1^{-1} W).  The table is read in order through
    // scalar loads; each entry serves the four variables.
    {
      const double* lu0 = gt + GTab::lu(n);
      asm volatile("" : "+s"(lu0));
      typedef const __attribute__((address_space(4))) double* cptr;
      cptr t = (cptr)lu0;
      int o = 0;
#pragma unroll
      for (int i = 0; i < n; ++i) {             // z_i = w_i R_i - sum_{j<i} L_ij z_j
        const double wi = t[o++];
#pragma unroll
        for (int v = 0; v < 4; ++v) X[i][v] *= wi;
#pragma unroll
        for (int j = 0; j < i; ++j) {
          const double Lij = t[o++];
#pragma unroll
          for (int v = 0; v < 4; ++v) X[i][v] = fma(-Lij, X[j][v], X[i][v]);
        }
      }
#pragma unroll
      for (int i = n - 1; i >= 0; --i) {       // y_i = z_i / U_ii - sum_{j>i} (U_ij / U_ii) y_j
        const double iu = t[o++];
#pragma unroll
        for (int v = 0; v < 4; ++v) X[i][v] *= iu;
#pragma unroll
        for (int j = i + 1; j < n; ++j) {
          const double Uij = t[o++];
#pragma unroll
          for (int v = 0; v < 4; ++v) X[i][v] = fma(-Uij, X[j][v], X[i][v]);
        }
      }
      const double sdt = (CPW == 1) ? uniform(-dt * ih) : -dt * ih;   // R = -R' / h
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double qn = Qc[v * nn];
#pragma unroll
        for (int i = 0; i < n; ++i) X[i][v] = fma(sdt, X[i][v], qn);
      }
    }
    if (a.iter_store && valid) {
      double* st = a.iter_store + ((size_t)c * a.iters + it) * n * sl;
#pragma unroll
      for (int b = 0; b < n; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) st[b * sl + v * nn + l] = X[b][v];
    }
  }

  // time averages on the last iterate.  The averaged state and the averaged
  // manufactured source do not need the fluxes: they go to the (now unused)
  // source region first, so that only the flux averages are carried in
  // registers through the final pass.
  if (node) {
    double SbE = 0.0;
    if ((!PW && ph.mms)) {
#pragma unroll
      for (int b = 0; b < n; ++b) SbE = fma(gt[GTab::W * n + b], sm[b * nn + l], SbE);
    }
    double Qb[4] = {0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < n; ++b) {
      const double wb = gt[GTab::W * n + b];
#pragma unroll
      for (int v = 0; v < 4; ++v) Qb[v] = fma(wb, X[b][v], Qb[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sm[v * nn + l] = Qb[v];
    sm[4 * nn + l] = SbE;
  }
  // flux averages accumulate in registers; they go to LDS once, in the
  // layouts the line jobs of the volume term read: x fluxes in the first, z
  // fluxes in the transposed one
  double Sbw = 0.0, Fxa[4], Fza[4];
#pragma unroll
  for (int b = 0; b < n; ++b) {
    put_slice(X[b]);
    wave_sync();
    grad_lines();
    wave_sync();
    if (node) {
      double Fx[4], Fz[4];
      const double Sw = node_flux<n>(ph, X[b], sf, l, tl, mu_h, kappa_h, gh, z, rb, pb, Fx, Fz, false);
      const double wb = gt[GTab::W * n + b];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Fxa[v] = b == 0 ? wb * Fx[v] : fma(wb, Fx[v], Fxa[v]);
        Fza[v] = b == 0 ? wb * Fz[v] : fma(wb, Fz[v], Fza[v]);
      }
      Sbw = fma(wb, Sw, Sbw);
    }
  }
  wave_sync();

  // face data and volume term: averaged state to the slice region, averaged
  // fluxes to the flux region; each line job extrapolates its line to both
  // faces, then replaces the flux line by its volume contraction (in place:
  // lines are disjoint).
  double SbE = 0.0;
  if (node) {
    double Qb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) Qb[v] = sm[v * nn + l];
    SbE = sm[4 * nn + l];
    put_slice(Qb);
#pragma unroll
    for (int v = 0; v < 4; ++v) { sf[v * nn + l] = Fxa[v]; sf[ZO + v * nn + tl] = Fza[v]; }
  }
  wave_sync();
  {
    EOTab<n> Wt;
    load_eo<n>(gt + GTab::eo_dw(n), Wt);
    // the line-job roles are derived again from the lane (hidden from the
    // compiler) instead of being held in registers through the sweeps
    int lane_r = lane;
    asm volatile("" : "+v"(lane_r));
#pragma unroll
    for (int r = 0; r < P::rounds; ++r) {
      const PJob<n, CPW> J(lane_r + r * kWave);
      double* jl = wl + (J.active ? J.slot : 0) * P::cell;
      if (!J.active) continue;
      const int cj = cell0 + J.slot;
      double q0 = 0, q1 = 0, f0 = 0, f1 = 0;
#pragma unroll
      for (int m = 0; m < n; ++m) {
        const double e0 = gt[GTab::E0 * n + m], e1 = gt[GTab::E1 * n + m];
        const double iq = jl[J.src + m * J.sst()], iF = jl[J.dst + m];
        q0 = fma(e0, iq, q0); q1 = fma(e1, iq, q1);
        f0 = fma(e0, iF, f0); f1 = fma(e1, iF, f1);
      }
      line_eo<n>(Wt, J.dst, jl, jl);
      if (cj >= a.C) continue;
      double* fd = a.FD + (size_t)cj * 32 * n;
      const int fl0 = 2 * J.dir, fu = 2 * J.dir + 1;
      fd[((fl0 * 2 + 0) * 4 + J.v) * n + J.line] = q0;
      fd[((fl0 * 2 + 1) * 4 + J.v) * n + J.line] = f0;
      fd[((fu * 2 + 0) * 4 + J.v) * n + J.line] = q1;
      fd[((fu * 2 + 1) * 4 + J.v) * n + J.line] = f1;
    }
  }
  wave_sync();
  if (valid) {
    double* qs = a.Qs + (size_t)c * sl;
    if constexpr (PW) {
      // time average of the paper's manufactured source (state-independent)
      double Sp[4] = {0.0, 0.0, 0.0, 0.0};
      const double xn = x0 + h * gt[GTab::XI * n + ix];
#pragma unroll 1
      for (int b = 0; b < n; ++b) {
        double Sm[4];
        paper_wave_source(ph, xn, z, t0 + gt[GTab::XI * n + b] * dt, Sm);
        const double wb = gt[GTab::W * n + b];
#pragma unroll
        for (int v = 0; v < 4; ++v) Sp[v] = fma(wb, Sm[v], Sp[v]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double S = ((v == 2) ? Sbw : (v == 3 ? SbE : 0.0)) + Sp[v];
        qs[v * nn + l] = Qc[v * nn] + dt * ((sf[v * nn + l] + sf[ZO + v * nn + tl]) * ih + S);
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double S = (v == 2) ? Sbw : (v == 3 ? SbE : 0.0);
        qs[v * nn + l] = Qc[v * nn] + dt * ((sf[v * nn + l] + sf[ZO + v * nn + tl]) * ih + S);
      }
    }
  }
}

template <int n, int CPW, int WPB, bool PW = false>
__global__ __launch_bounds__(kWave * WPB, (n <= 7 ? 3 : 1)) void k_predictor(Phys ph, StepArgs a) {
  // with several wavefronts per workgroup the index is made wave-uniform
  // (scalar), which keeps the cell-level values out of vector registers
  const int wave = WPB == 1 ? (int)(threadIdx.x / kWave) : __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  predictor_wave<n, CPW, PW>(ph, a, wave, (blockIdx.x * WPB + wave) * CPW);
}

// ------------------------------------------- predictor, wavefronts per level
// For meshes too small to fill the chip with one wavefront per cell: one
// workgroup of W wavefronts per cell, wavefront w owning the time nodes
// w, w + W, ... (W = n: one wavefront per time node).  Each wavefront runs
// the slice machinery of k_predictor with one cell per wavefront (the slice
// in one LDS layout, line jobs, even-odd contractions) on its time nodes one
// after the other, in its own LDS region of 4 slices.  Within a Picard
// sweep the n residuals are independent; they meet in a shared LDS area,
// where the time matrix mixes them: X_b = Q + dt sum_a P[b][a] R_a (with one
// wavefront per node each residual sits in its wavefront's region, else in
// an area of its own).  The first sweep evaluates one residual (every node
// starts from Q^n).  In the final pass every wavefront leaves the weighted
// sum of its nodes' state, fluxes and sources in its region; the first
// wavefront sums the W regions in order and runs the
// epilogue of k_predictor (volume term, Q*, face data).  Same arithmetic as
// k_predictor up to the order of the sums.
template <int n, int W, bool PW>
__device__ __forceinline__ void predictor_levels(Phys ph, StepArgs a, int c) {
  using P = PLay<n, 1>;
  constexpr int nn = n * n, sl = 4 * nn, ZO = 4 * nn, WR = 4 * sl;
  static_assert(P::GZ + 4 * nn + sl <= WR, "slice, gradients and a residual fit a region");
  constexpr int NL = (n + W - 1) / W;             // time nodes per wavefront (the last may own fewer)
  extern __shared__ double lds[];                 // W regions of WR doubles, then (W < n) the residuals [n][sl]
  // the wavefront index is wave-uniform: scalar, so are its time-node tables
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  double* wl = lds + (size_t)w * WR;
  // residual of time node b: the last slice of its region (W = n), or [b][sl] after the regions
  auto res = [&](int b) { return W == n ? lds + (size_t)b * WR + (WR - sl) : lds + (size_t)W * WR + (size_t)b * sl; };
  const bool node = lane < nn;
  const int l = node ? lane : 0;
  const int jz = l / n, ix = l % n, tl = ix * n + jz;
  double* sq = wl;           // slice
  double* sf = wl + P::GX;   // gradients / fluxes: x part, z part at ZO
  const double* gt = a.gtab;
  const int s = a.scen ? a.scen[c] : 0;
  const double t0 = a.clock[4 * s + 0], dt = a.clock[4 * s + 1];
  const double x0 = a.geom[4 * c + 0], z0 = a.geom[4 * c + 1], h = a.geom[4 * c + 2];
  const double ih = 1.0 / h, mu_h = ph.mu * ih, kappa_h = ph.kappa * ih, gh = ph.geff * h;
  const double sdt = -dt * ih;   // R = -R' / h
  const double z = z0 + h * gt[GTab::XI * n + jz];
  double rb, pb;
  background(ph, z, rb, pb);
  EOTab<n> Dt;
  load_eo<n>(gt + GTab::eo_d(n), Dt);
  const double* Qc = a.Qin + (size_t)c * sl + l;
  double X[NL][4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double q = Qc[v * nn];
#pragma unroll
    for (int k = 0; k < NL; ++k) X[k][v] = q;
  }
  // manufactured source at this node and each owned level's time (it does
  // not depend on the state): the density wave's energy source, or the
  // paper's wave's source of every variable
  double SE[NL], Sm[NL][4];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int b = w + k * W;
    SE[k] = (!PW && ph.mms && node && b < n) ? mms_source(ph, x0 + h * gt[GTab::XI * n + ix], z,
                                                          t0 + gt[GTab::XI * n + b] * dt) : 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) Sm[k][v] = 0.0;
    if constexpr (PW) {
      if (node && b < n) paper_wave_source(ph, x0 + h * gt[GTab::XI * n + ix], z, t0 + gt[GTab::XI * n + b] * dt, Sm[k]);
    }
  }

  const PJob<n, 1> J(lane);
  auto grad_lines = [&]() {
    if (J.active) line_eo_s<n>(Dt, wl + J.src, J.sst(), wl + J.dst);
  };
  auto div_lines = [&]() {
    if (J.active) line_eo<n>(Dt, J.dst, wl, wl);
  };
  auto put_slice = [&](const double q[4]) {
    if (node) {
#pragma unroll
      for (int v = 0; v < 4; ++v) sq[v * nn + l] = q[v];
    }
  };
  // scaled residual R' = div F - h S of the slice q (without the manufactured source)
  auto residual = [&](const double q[4], double R[4]) {
    put_slice(q);
    wave_sync();
    grad_lines();
    wave_sync();
    double Sw = 0.0;
    if (node) {
      double Fx[4], Fz[4];
      Sw = node_flux<n>(ph, q, sf, l, tl, mu_h, kappa_h, gh, z, rb, pb, Fx, Fz, true);
    }
    wave_sync();
    div_lines();
    wave_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) R[v] = node ? sf[v * nn + l] + sf[ZO + v * nn + tl] : 0.0;
    R[2] = fma(-h, Sw, R[2]);
  };
  // the manufactured source of owned level k added, to the shared area
  auto put_residual = [&](int k, double R[4]) {
    const int b = w + k * W;
    if (node) {
      if (!PW && ph.mms) R[3] = fma(-h, SE[k], R[3]);
      if constexpr (PW) {
#pragma unroll
        for (int v = 0; v < 4; ++v) R[v] = fma(-h, Sm[k][v], R[v]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) res(b)[v * nn + l] = R[v];
    }
  };

#pragma unroll 1
  for (int it = 0; it < a.iters; ++it) {
    if (it == 0) {
      // every node starts from Q^n: the first wavefront's residual serves all
      if (w == 0) {
        double R[4];
        residual(X[0], R);
        if (node)
#pragma unroll
          for (int v = 0; v < 4; ++v) sq[v * nn + l] = R[v];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        if (w + k * W >= n) break;
        double R[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) R[v] = node ? lds[v * nn + l] : 0.0;
        put_residual(k, R);
      }
    } else {
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        if (w + k * W >= n) break;
        double R[4];
        residual(X[k], R);
        put_residual(k, R);
        wave_sync();
      }
    }
    __syncthreads();   // every node's residual in LDS
    if (node) {
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        const int b = w + k * W;
        if (b >= n) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double acc = 0.0;
#pragma unroll
          for (int a2 = 0; a2 < n; ++a2) acc = fma(gt[GTab::pt(n) + a2 * n + b], res(a2)[v * nn + l], acc);
          X[k][v] = fma(sdt, acc, Qc[v * nn]);
        }
        if (a.iter_store) {
          double* st = a.iter_store + (((size_t)c * a.iters + it) * n + b) * sl;
#pragma unroll
          for (int v = 0; v < 4; ++v) st[v * nn + l] = X[k][v];
        }
      }
    }
    __syncthreads();   // every residual read (and the first sweep's shared one) before the next sweep
  }

  // final pass: the owned nodes' fluxes and sources at the last iterate,
  // weighted and summed, to this wavefront's region as [state | x flux |
  // z flux | vertical-momentum source | energy source | mass source |
  // horizontal-momentum source]
  double Qw[4], Fxw[4], Fzw[4], Sww = 0.0, SEw = 0.0, S0w = 0.0, S1w = 0.0;
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int b = w + k * W;
    if (b >= n) break;
    put_slice(X[k]);
    wave_sync();
    grad_lines();
    wave_sync();
    double Fx[4], Fz[4], Sw = 0.0;
    if (node) Sw = node_flux<n>(ph, X[k], sf, l, tl, mu_h, kappa_h, gh, z, rb, pb, Fx, Fz, false);
    wave_sync();
    const double wb = gt[GTab::W * n + b];
    const double s2 = PW ? Sw + Sm[k][2] : Sw, s3 = PW ? Sm[k][3] : SE[k];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Qw[v] = k == 0 ? wb * X[k][v] : fma(wb, X[k][v], Qw[v]);
      Fxw[v] = k == 0 ? wb * Fx[v] : fma(wb, Fx[v], Fxw[v]);
      Fzw[v] = k == 0 ? wb * Fz[v] : fma(wb, Fz[v], Fzw[v]);
    }
    Sww = k == 0 ? wb * s2 : fma(wb, s2, Sww);
    SEw = k == 0 ? wb * s3 : fma(wb, s3, SEw);
    if constexpr (PW) {
      S0w = k == 0 ? wb * Sm[k][0] : fma(wb, Sm[k][0], S0w);
      S1w = k == 0 ? wb * Sm[k][1] : fma(wb, Sm[k][1], S1w);
    }
  }
  if (node) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      wl[v * nn + l] = Qw[v];
      wl[(4 + v) * nn + l] = Fxw[v];
      wl[(8 + v) * nn + l] = Fzw[v];
    }
    wl[12 * nn + l] = Sww;
    wl[13 * nn + l] = SEw;
    if constexpr (PW) {
      wl[14 * nn + l] = S0w;
      wl[15 * nn + l] = S1w;
    }
  }
  __syncthreads();
  if (w != 0) return;

  // sums over the wavefronts in a fixed order, then the epilogue of k_predictor
  double Qb[4] = {0, 0, 0, 0}, Fbx[4] = {0, 0, 0, 0}, Fbz[4] = {0, 0, 0, 0}, Sbw = 0.0, SbE = 0.0;
  double Sb0 = 0.0, Sb1 = 0.0;   // paper's wave only
  if (node) {
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const double* r = lds + (size_t)k * WR;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Qb[v] += r[v * nn + l];
        Fbx[v] += r[(4 + v) * nn + l];
        Fbz[v] += r[(8 + v) * nn + l];
      }
      Sbw += r[12 * nn + l];
      SbE += r[13 * nn + l];
      if constexpr (PW) {
        Sb0 += r[14 * nn + l];
        Sb1 += r[15 * nn + l];
      }
    }
  }
  wave_sync();
  if (node) {
    put_slice(Qb);
#pragma unroll
    for (int v = 0; v < 4; ++v) { sf[v * nn + l] = Fbx[v]; sf[ZO + v * nn + tl] = Fbz[v]; }
  }
  wave_sync();
  {
    EOTab<n> Wt;
    load_eo<n>(gt + GTab::eo_dw(n), Wt);
    if (J.active) {
      double q0 = 0, q1 = 0, f0 = 0, f1 = 0;
#pragma unroll
      for (int m = 0; m < n; ++m) {
        const double e0 = gt[GTab::E0 * n + m], e1 = gt[GTab::E1 * n + m];
        const double iq = wl[J.src + m * J.sst()], iF = wl[J.dst + m];
        q0 = fma(e0, iq, q0); q1 = fma(e1, iq, q1);
        f0 = fma(e0, iF, f0); f1 = fma(e1, iF, f1);
      }
      line_eo<n>(Wt, J.dst, wl, wl);
      double* fd = a.FD + (size_t)c * 32 * n;
      const int fl0 = 2 * J.dir, fu = 2 * J.dir + 1;
      fd[((fl0 * 2 + 0) * 4 + J.v) * n + J.line] = q0;
      fd[((fl0 * 2 + 1) * 4 + J.v) * n + J.line] = f0;
      fd[((fu * 2 + 0) * 4 + J.v) * n + J.line] = q1;
      fd[((fu * 2 + 1) * 4 + J.v) * n + J.line] = f1;
    }
  }
  wave_sync();
  if (node) {
    double* qs = a.Qs + (size_t)c * sl;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double S = (v == 2) ? Sbw : (v == 3 ? SbE : (v == 0 ? Sb0 : Sb1));
      qs[v * nn + l] = Qc[v * nn] + dt * ((sf[v * nn + l] + sf[ZO + v * nn + tl]) * ih + S);
    }
  }
}

template <int n, int W, bool PW = false>
__global__ __launch_bounds__(kWave * W, (W < n && n <= 7 ? 3 : 1)) void k_predictor_lv(Phys ph, StepArgs a) {
  predictor_levels<n, W, PW>(ph, a, blockIdx.x);
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
template <int n, int CPW, int WPB, bool NC>
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

  // Q* of this lane's node, loaded first so that its latency overlaps the
  // face phase
  const int slot = lane / nn, l = lane % nn;
  const int c = cell0 + slot;
  const bool valid = slot < CPW && c < a.C;
  double qsv[4] = {0.0, 0.0, 0.0, 0.0};
  if (valid) {
    const double* qs = a.Qs + (size_t)c * sl;
#pragma unroll
    for (int v = 0; v < 4; ++v) qsv[v] = qs[v * nn + l];
  }

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
    if (!NC || kind != kCoarseSide) {
      const double zf = (d == 0) ? z0f + hf * gt[GTab::XI * n + k] : z0f + ((f & 1) ? hf : 0.0);
      load_face<n>(a.FD, fc, f, k, Qm, Fm);
      if (kind == kConforming) load_face<n>(a.FD, nb1, f ^ 1, k, Qo, Fo);
      else if (NC && kind == kFineSide) prolong_face<n>(a.FD, gt, nb1, f ^ 1, nb2, k, Qo, Fo);
      else wall_ghost(ph, d, zf, Qm, Fm, Qo, Fo);
      double l1, v1, l2, v2;
      eig(ph, d, Qm, zf, l1, v1);
      eig(ph, d, Qo, zf, l2, v2);
      sL[(f * 3) * n + k] = fmax(l1, l2);
      sV[(f * 3) * n + k] = fmax(v1, v2);
    } else if constexpr (NC) {
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
    if (!NC || kind != kCoarseSide) {
      double lam = sL[(f * 3) * n], lv = sV[(f * 3) * n];
#pragma unroll
      for (int m = 1; m < n; ++m) { lam = fmax(lam, sL[(f * 3) * n + m]); lv = fmax(lv, sV[(f * 3) * n + m]); }
      const double s = lam + 2.0 * (eta0 / hf) * lv;
      double G[4];
      if (lower) rusanov_flux(s, Qo, Fo, Qm, Fm, G);
      else rusanov_flux(s, Qm, Fm, Qo, Fo, G);
#pragma unroll
      for (int v = 0; v < 4; ++v) sG[(f * 4 + v) * n + k] = G[v];
    } else if constexpr (NC) {
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
  if (NC && fl && kind == kCoarseSide) {
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
  const double* sGc = wl + (slot < CPW ? slot : 0) * L::corr_cell;
  double lam_n = 0.0, lv_n = 0.0;
  if (valid) {
    const int jz = l / n, ix = l % n;
    const int sc = a.scen ? a.scen[c] : 0;
    const double dt = a.clock[4 * sc + 1];
    const double z0 = a.geom[4 * c + 1], h = a.geom[4 * c + 2];
    const double L0i = gt[GTab::L0 * n + ix], L1i = gt[GTab::L1 * n + ix];
    const double L0j = gt[GTab::L0 * n + jz], L1j = gt[GTab::L1 * n + jz];
    double* qo = a.Qout + (size_t)c * sl;
    const double scl = dt / h;
    double q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double sx = L1i * sGc[(1 * 4 + v) * n + jz] - L0i * sGc[(0 * 4 + v) * n + jz];
      const double sz = L1j * sGc[(3 * 4 + v) * n + ix] - L0j * sGc[(2 * 4 + v) * n + ix];
      q[v] = qsv[v] - scl * (sx + sz);
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
    double lm, vm;
    if constexpr (CPW == 1) {
      lm = wave_max(lam_n);   // lanes without a node hold 0
      vm = wave_max(lv_n);
    } else {
      slam[wave][0][lane] = lam_n;
      slam[wave][1][lane] = lv_n;
      wave_sync();
      lm = lam_n; vm = lv_n;
      if (valid && l == 0)
        for (int j = 1; j < nn; ++j) { lm = fmax(lm, slam[wave][0][lane + j]); vm = fmax(vm, slam[wave][1][lane + j]); }
    }
    if (valid && l == 0) {
      const double h = a.geom[4 * c + 2];
      const double o = 2.0 * ph.N + 1.0;
      a.dtc[c] = ph.cfl * h / (2.0 * o * (lm + 2.0 * vm * o / h));
    }
  }
  // a frozen time step: the clock advances here, with no reduction to wait
  // for (the corrector reads only dt, which does not change)
  if (a.advance && blockIdx.x == 0 && threadIdx.x == 0) {
    a.advance[0] += a.advance[1];
    a.advance[3] += 1.0;
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
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_clock(double* clock, const double* dtc, const int* beg,
                                                           const int* end, int C, int advance, int update) {
  __shared__ double sm[kReduceThreads / kWave];
  const int s = blockIdx.x, t = threadIdx.x;
  const int b0 = beg ? beg[s] : 0, b1 = end ? end[s] : C;
  // the clock is read before the reduction so that its latency overlaps it
  double t_old = 0.0, dt_old = 0.0, n_old = 0.0;
  if (t == 0) { t_old = clock[4 * s + 0]; dt_old = clock[4 * s + 1]; n_old = clock[4 * s + 3]; }
  double m = __builtin_inf();
  if (update) {
    // four independent loads in flight per thread
    int c = b0 + t;
    for (; c + 3 * kReduceThreads < b1; c += 4 * kReduceThreads) {
      const double a0 = dtc[c], a1 = dtc[c + kReduceThreads], a2 = dtc[c + 2 * kReduceThreads],
                   a3 = dtc[c + 3 * kReduceThreads];
      m = fmin(m, fmin(fmin(a0, a1), fmin(a2, a3)));
    }
    for (; c < b1; c += kReduceThreads) m = fmin(m, dtc[c]);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmin(m, __shfl_xor(m, o, kWave));
  if ((t & (kWave - 1)) == 0) sm[t / kWave] = m;
  __syncthreads();
  if (t == 0) {
    double r = sm[0];
    for (int k = 1; k < kReduceThreads / kWave; ++k) r = fmin(r, sm[k]);
    if (advance) { clock[4 * s + 0] = t_old + dt_old; clock[4 * s + 3] = n_old + 1.0; }
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
  a.advance = g.advance;
  return a;
}

// ------------------------------------------------- persistent batch predictor
// One persistent launch per order group: a grid of resident wavefronts that
// take work items (one wavefront's cells) from the group's device counter
// until none are left, each running the per-wavefront body of k_predictor.
// The last wavefront to finish resets the counter pair for the next launch
// (every wavefront of the grid reaches that point: the loop ends when the
// counter passes the last item).  The batch sizes each order's grid by its
// share of the modelled work, so that the orders, launched side by side,
// finish together.
template <int n, int CPW>
__global__ __launch_bounds__(kWave, (n <= 7 ? 3 : 1)) void k_predictor_queue(Phys ph, StepArgs a, unsigned* counter,
                                                                              unsigned nwaves) {
  const unsigned items = (unsigned)((a.C + CPW - 1) / CPW);
  for (;;) {
    unsigned item = 0;
    if (threadIdx.x == 0) item = atomicAdd(&counter[0], 1u);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= items) break;
    // an opaque copy of the buffer pointers per item, so that the body's
    // table and state loads stay inside the loop (hoisted, they would stay
    // live across the whole body)
    StepArgs ai = a;
    asm volatile("" : "+s"(ai.gtab), "+s"(ai.geom), "+s"(ai.Qin), "+s"(ai.clock));
    predictor_wave<n, CPW, false>(ph, ai, 0, (int)item * CPW);
  }
  if (threadIdx.x == 0) {
    const unsigned done = atomicAdd(&counter[1], 1u);
    if (done + 1 == nwaves) {
      atomicExch(&counter[0], 0u);
      atomicExch(&counter[1], 0u);
    }
  }
}

template <int n>
static int queue_n(const Group& g, unsigned* counter, int nwaves, hipStream_t s) {
  constexpr int CPW = max_cpw_c(n);
  const size_t lds = sizeof(double) * (size_t)CPW * PLay<n, CPW>::cell;
  hipLaunchKernelGGL((k_predictor_queue<n, CPW>), dim3(nwaves), dim3(kWave), lds, s, g.ph, make_args(g), counter,
                     (unsigned)nwaves);
  return check_launch("persistent predictor");
}

int launch_predictor_queue(const Group& g, unsigned* counter, int nwaves, hipStream_t s) {
  if (g.C == 0 || nwaves < 1) return ADG_OK;
  if (g.ph.mms == 2) return fail(ADG_EUNSUPPORTED, "the persistent batch predictor has no manufactured-solution source");
  switch (g.n) {
    case 2: return queue_n<2>(g, counter, nwaves, s);
    case 3: return queue_n<3>(g, counter, nwaves, s);
    case 4: return queue_n<4>(g, counter, nwaves, s);
    case 5: return queue_n<5>(g, counter, nwaves, s);
    case 6: return queue_n<6>(g, counter, nwaves, s);
    case 7: return queue_n<7>(g, counter, nwaves, s);
    case 8: return queue_n<8>(g, counter, nwaves, s);
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
}

// resident wavefronts per CU of the persistent predictor of order n-1
template <int n>
static int queue_occ(int* per_cu) {
  constexpr int CPW = max_cpw_c(n);
  const size_t lds = sizeof(double) * (size_t)CPW * PLay<n, CPW>::cell;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_predictor_queue<n, CPW>, kWave, lds) == hipSuccess
             ? ADG_OK
             : fail(ADG_EHIP, "occupancy query failed");
}
int predictor_queue_occupancy(int n, int* per_cu) {
  switch (n) {
    case 2: return queue_occ<2>(per_cu);
    case 3: return queue_occ<3>(per_cu);
    case 4: return queue_occ<4>(per_cu);
    case 5: return queue_occ<5>(per_cu);
    case 6: return queue_occ<6>(per_cu);
    case 7: return queue_occ<7>(per_cu);
    case 8: return queue_occ<8>(per_cu);
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
}

template <int n, int CPW, int WPB, bool PW = false>
static int launch_pred_t(const Group& g, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)WPB * CPW * PLay<n, CPW>::cell;
  const int per_block = CPW * WPB;
  const int blocks = (g.C + per_block - 1) / per_block;
  if (blocks == 0) return ADG_OK;
  hipLaunchKernelGGL((k_predictor<n, CPW, WPB, PW>), dim3(blocks), dim3(kWave * WPB), lds, s, g.ph,
                     make_args(g));
  return check_launch("predictor");
}
template <int n, int CPW, int WPB>
static int launch_corr_t(const Group& g, hipStream_t s) {
  using L = Lay<n, CPW>;
  const size_t lds = sizeof(double) * (size_t)WPB * CPW * L::corr_cell;
  const int per_block = CPW * WPB;
  const int blocks = (g.C + per_block - 1) / per_block;
  if (blocks == 0) return ADG_OK;
  // meshes without 1:3 faces take the variant without their code paths
  if (g.nc)
    hipLaunchKernelGGL((k_corrector<n, CPW, WPB, true>), dim3(blocks), dim3(kWave * WPB), lds, s, g.ph,
                       make_args(g));
  else
    hipLaunchKernelGGL((k_corrector<n, CPW, WPB, false>), dim3(blocks), dim3(kWave * WPB), lds, s, g.ph,
                       make_args(g));
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
  // the paper's manufactured solution runs one cell per wavefront (the
  // launch shape does not change results)
  if (g.ph.mms == 2) return launch_pred_t<n, 1, 1, true>(g, s);
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

template <int n, int W>
static void pred_lv_w(const Group& g, const StepArgs& a, hipStream_t s) {
  using L = Lay<n, 1>;
  const size_t lds = sizeof(double) * ((size_t)W * 4 * L::sl + (W < n ? (size_t)n * L::sl : 0));
  if (g.ph.mms == 2)
    hipLaunchKernelGGL((k_predictor_lv<n, W, true>), dim3(g.C), dim3(kWave * W), lds, s, g.ph, a);
  else
    hipLaunchKernelGGL((k_predictor_lv<n, W>), dim3(g.C), dim3(kWave * W), lds, s, g.ph, a);
}
template <int n>
static int pred_lv_n(const Group& g, double* store, hipStream_t s) {
  if (g.C == 0) return ADG_OK;
  StepArgs a = make_args(g);
  a.iter_store = store;
  const int W = level_waves(g);
  if constexpr (n > 2) { if (W == 2) { pred_lv_w<n, 2>(g, a, s); return check_launch("predictor (levels)"); } }
  if constexpr (n > 4) { if (W == 4) { pred_lv_w<n, 4>(g, a, s); return check_launch("predictor (levels)"); } }
  pred_lv_w<n, n>(g, a, s);
  return check_launch("predictor (levels)");
}
int launch_predictor_levels(const Group& g, double* store, hipStream_t s) {
  switch (g.n) {
    case 2: return pred_lv_n<2>(g, store, s);
    case 3: return pred_lv_n<3>(g, store, s);
    case 4: return pred_lv_n<4>(g, store, s);
    case 5: return pred_lv_n<5>(g, store, s);
    case 6: return pred_lv_n<6>(g, store, s);
    case 7: return pred_lv_n<7>(g, store, s);
    case 8: return pred_lv_n<8>(g, store, s);
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
}

template <int n>
static int pred_store_n(const Group& g, double* store, hipStream_t s) {
  if (g.C == 0) return ADG_OK;
  StepArgs a = make_args(g);
  a.iter_store = store;
  const size_t lds = sizeof(double) * (size_t)PLay<n, 1>::cell;
  if (g.ph.mms == 2)
    hipLaunchKernelGGL((k_predictor<n, 1, 1, true>), dim3(g.C), dim3(kWave), lds, s, g.ph, a);
  else
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

int max_cpw(int n) { return max_cpw_c(n); }

}  // namespace adg
