// Internal definitions of the three-dimensional step: kernel arguments, the
// handle, and the launchers of the kernels in step3.hip.
#pragma once

#include "adg3.h"
#include "adg_internal.h"

namespace adg {

constexpr int kMaxBubbles3 = 16;

// Everything the 3D kernels read: bound buffers, the grid and the tables.
struct Args3 {
  const double* Q;      // [C][5][nd] state
  double* Qout;         // corrector output (equal to Q: updated in place)
  double* Qs;           // [C][5][nd] Q*
  double* FD;           // [C][6][2][5][nn] face data
  double* dtc;          // [C] CFL candidates
  const double* clock;  // (t, dt, -, steps)
  const double* gtab;   // GTab layout
  int nx, ny, nz, C, iters;
  int wall;             // bit f set: domain face f is a wall
  double x0, y0, z0, h;
  double eta;           // (2N+1) / (h sqrt(pi/2)), penalty of the viscous speed
};

// Bubble list passed by value to the initial-state kernel.
struct Bubbles3 {
  int nb;
  double b[kMaxBubbles3 * 7];   // (shape, A, a, s, xc, yc, zc) per bubble
};

int launch_pred3(const Phys& ph, const HostBasis& B, const Args3& a, hipStream_t s);
int launch_corr3(const Phys& ph, int n, const Args3& a, hipStream_t s);
int launch_dt3(const Phys& ph, int n, const Args3& a, hipStream_t s);
int launch_init3(const Phys& ph, int n, const Args3& a, int kind, const Bubbles3& B, double t0, double* Q,
                 hipStream_t s);
int launch_health3(const Phys& ph, int n, const Args3& a, int* flag, hipStream_t s);
int launch_clock(double* clock, const double* dtc, const int* beg, const int* end, int nscen, int C, int advance,
                 int update, hipStream_t s);

}  // namespace adg

struct adg3_mesh {
  adg_params prm{};
  adg3_mesh_desc desc{};
  adg::HostBasis basis;
  adg::Phys ph{};
  int n = 0, C = 0, iters = 0;
  double* d_gtab = nullptr;
  // bound (caller-owned)
  double* Q = nullptr;
  void* ws = nullptr;
  double* clock = nullptr;
  // workspace partition (byte offsets)
  size_t off_qs = 0, off_fd = 0, off_dtc = 0, off_health = 0, ws_bytes = 0;
};
