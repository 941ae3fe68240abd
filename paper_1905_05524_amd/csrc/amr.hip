// Adaptive mesh refinement: the regrid plan (host) and the state transfer
// kernel (gfx950).
//
// Plan (Numerics, refinement criterion: subcells are coarsened only when all
// of them are marked): flags +1 refine, -1 coarsen, 0 keep; refine is dropped
// at the finest level, coarsen at the coarsest; a family of nine siblings is
// replaced by its parent only if all nine are leaves flagged coarsen; with
// several levels, refinements and coarsenings are adjusted to keep
// neighbouring leaves within one level (regrid_plan).  New leaf order: old leaves in order; a refined leaf is replaced
// by its children (row by row), a coarsened family by its parent at the
// position of its first sibling.
// Transfer: copy; prolongation to a child by exact interpolation of the
// parent polynomial; restriction of nine children by L2 projection.
#include <algorithm>
#include <map>
#include <set>
#include <tuple>
#include <unordered_map>

#include "adg_internal.h"

namespace adg {

enum RegridOp { kCopy = 0, kProlong = 1, kRestrict = 2 };

// ops[c][12] = op, a, b, src[9]
template <int n>
__global__ __launch_bounds__(kWave) void k_regrid(const int* ops, const double* Qold, double* Qnew,
                                                   const double* gtab) {
  constexpr int nn = n * n;
  const int c = blockIdx.x, lane = threadIdx.x;
  const int* op = ops + 12 * c;
  if (lane >= nn) return;
  const int j = lane / n, i = lane % n;
  double* dst = Qnew + (size_t)c * 4 * nn;
  if (op[0] == kCopy) {
    const double* src = Qold + (size_t)op[3] * 4 * nn;
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[v * nn + lane] = src[v * nn + lane];
  } else if (op[0] == kProlong) {
    const int a = op[1], b = op[2];
    const double* src = Qold + (size_t)op[3] * 4 * nn;
    const double* Pa = gtab + GTab::pk(n) + (a * n + i) * n;   // phi_m((a + xi_i)/3)
    const double* Pb = gtab + GTab::pk(n) + (b * n + j) * n;   // phi_l((b + xi_j)/3)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double s = 0.0;
      for (int l = 0; l < n; ++l) {
        double r = 0.0;
#pragma unroll
        for (int m = 0; m < n; ++m) r = fma(Pa[m], src[v * nn + l * n + m], r);
        s = fma(Pb[l], r, s);
      }
      dst[v * nn + lane] = s;
    }
  } else {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) {
        const double* src = Qold + (size_t)op[3 + 3 * b + a] * 4 * nn;
        const double* Ra = gtab + GTab::rk(n) + (a * n + i) * n;   // (w_m/3) phi_i((a+xi_m)/3) / w_i
        const double* Rb = gtab + GTab::rk(n) + (b * n + j) * n;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double s = 0.0;
          for (int l = 0; l < n; ++l) {
            double r = 0.0;
#pragma unroll
            for (int m = 0; m < n; ++m) r = fma(Ra[m], src[v * nn + l * n + m], r);
            s = fma(Rb[l], r, s);
          }
          acc[v] += s;
        }
      }
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[v * nn + lane] = acc[v];
  }
}

template <int n>
static int launch_regrid_n(int C, const int* ops, const double* Qold, double* Qnew, const double* gtab,
                           hipStream_t s) {
  if (C == 0) return ADG_OK;
  hipLaunchKernelGGL(k_regrid<n>, dim3(C), dim3(kWave), 0, s, ops, Qold, Qnew, gtab);
  return check_launch("regrid");
}

int launch_regrid(int n, int C, const int* ops, const double* Qold, double* Qnew, const double* gtab,
                  hipStream_t s) {
  switch (n) {
    case 2: return launch_regrid_n<2>(C, ops, Qold, Qnew, gtab, s);
    case 3: return launch_regrid_n<3>(C, ops, Qold, Qnew, gtab, s);
    case 4: return launch_regrid_n<4>(C, ops, Qold, Qnew, gtab, s);
    case 5: return launch_regrid_n<5>(C, ops, Qold, Qnew, gtab, s);
    case 6: return launch_regrid_n<6>(C, ops, Qold, Qnew, gtab, s);
    case 7: return launch_regrid_n<7>(C, ops, Qold, Qnew, gtab, s);
    case 8: return launch_regrid_n<8>(C, ops, Qold, Qnew, gtab, s);
    default: return fail(ADG_EUNSUPPORTED, "order not supported");
  }
}

using Box = std::tuple<int, int, int>;   // level, i, j

// Regrid decisions with 2:1 balance, so that neighbouring leaves differ by
// at most one level after the regrid (the 1:3 face coupling needs it):
//   1. refine is dropped at the finest level, coarsen at level 0;
//   2. refinement closure: a leaf not refined that would touch, across a
//      face, a leaf two or more levels finer after the regrid is refined;
//      repeated to a fixed point;
//   3. coarsening: a complete family of nine leaves flagged coarsen (none
//      refined by step 2) is a candidate; a candidate whose parent would
//      touch, across a face, a leaf more than one level finer keeps its
//      children; repeated to a fixed point (cancelling only raises levels).
// Leaves across a face are found through the leaf map: the neighbouring box
// at the same level, then its ancestors (a coarser leaf covers it), else its
// descendants along the shared face.
namespace {

struct LeafMap {
  LeafIndex idx;
  const std::vector<int>& lev;
  const std::vector<int>& ci;
  const std::vector<int>& cj;
  int nx, nz;
  const int* bc;
  LeafMap(const std::vector<int>& l, const std::vector<int>& i, const std::vector<int>& j, int nx_, int nz_,
          const int* bc_, int L)
      : idx(nx_, nz_, L, l.size()), lev(l), ci(i), cj(j), nx(nx_), nz(nz_), bc(bc_) {
    for (size_t c = 0; c < l.size(); ++c) idx.insert(l[c], i[c], j[c], (int)c);
  }
  int find(int l, int i, int j) const { return idx.find(l, i, j); }
};

int pow3i(int e) { int r = 1; while (e-- > 0) r *= 3; return r; }

// highest new level over the leaves inside box (l, i, j) that touch its side
// `side` (0: low x, 1: high x, 2: low z, 3: high z)
template <class NL>
int max_on_side(const LeafMap& M, const NL& nl, int l, int i, int j, int side, int L) {
  const int c = M.find(l, i, j);
  if (c >= 0) return nl(c);
  if (l >= L) return -1;   // not a leaf and cannot be split further: covered by an ancestor
  int best = -1;
  for (int t = 0; t < 3; ++t) {
    const int a = side == 0 ? 0 : side == 1 ? 2 : t;
    const int b = side == 2 ? 0 : side == 3 ? 2 : t;
    best = std::max(best, max_on_side(M, nl, l + 1, 3 * i + a, 3 * j + b, side, L));
  }
  return best;
}

// highest new level over the leaves across face f of box (l, i, j); -1 at a wall
template <class NL>
int across_face(const LeafMap& M, const NL& nl, int l, int i, int j, int f, int L) {
  const int NX = M.nx * pow3i(l), NZ = M.nz * pow3i(l);
  int i2 = i + (f == 0 ? -1 : f == 1 ? 1 : 0), j2 = j + (f == 2 ? -1 : f == 3 ? 1 : 0);
  if (i2 < 0 || i2 >= NX || j2 < 0 || j2 >= NZ) {
    if (M.bc[f] == ADG_BC_WALL) return -1;
    i2 = (i2 + NX) % NX; j2 = (j2 + NZ) % NZ;
  }
  // a coarser (or equal) leaf covering the neighbouring box
  for (int la = l, ia = i2, ja = j2; la >= 0; --la, ia /= 3, ja /= 3) {
    const int c = M.find(la, ia, ja);
    if (c >= 0) return nl(c);
  }
  // finer leaves: those of the neighbouring box on the side facing this box
  const int side = f == 0 ? 1 : f == 1 ? 0 : f == 2 ? 3 : 2;
  return max_on_side(M, nl, l, i2, j2, side, L);
}

}  // namespace

// New leaf list and transfer ops from the old leaves and flags.
int regrid_plan(const std::vector<int>& lev, const std::vector<int>& ci, const std::vector<int>& cj,
                const int8_t* flags, int L, int nx, int nz, const int* bc, std::vector<int>& nlev,
                std::vector<int>& nci, std::vector<int>& ncj, std::vector<int>& ops) {
  const int C = (int)lev.size();
  std::vector<int> eff(C);
  for (int c = 0; c < C; ++c) {
    int f = flags[c];
    if (f != -1 && f != 0 && f != 1) return fail(ADG_EINVAL, "flags must be -1, 0 or +1");
    if (f == 1 && lev[c] >= L) f = 0;
    if (f == -1 && lev[c] == 0) f = 0;
    eff[c] = f;
  }
  const LeafMap M(lev, ci, cj, nx, nz, bc, L);
  // new level: +1 refine, -1 accepted coarsening (coded 2 below)
  std::vector<int> coarsen(C, 0);
  auto nl = [&](int c) { return lev[c] + (eff[c] == 1 ? 1 : 0) - coarsen[c]; };
  // refinement closure
  for (bool changed = true; changed;) {
    changed = false;
    for (int c = 0; c < C; ++c) {
      if (eff[c] == 1) continue;
      for (int f = 0; f < 4; ++f)
        if (across_face(M, nl, lev[c], ci[c], cj[c], f, L) > lev[c] + 1) {
          eff[c] = 1;
          changed = true;
          break;
        }
    }
  }
  // coarsening candidates: families whose nine children are leaves flagged coarsen
  // (parents in (level, i, j) order)
  std::map<Box, int> cnt;
  for (int c = 0; c < C; ++c)
    if (lev[c] > 0 && eff[c] == -1) cnt[Box(lev[c] - 1, ci[c] / 3, cj[c] / 3)] += 1;
  std::vector<Box> fams;
  for (const auto& kv : cnt)
    if (kv.second == 9) fams.push_back(kv.first);
  auto family = [&](const Box& pk, int* out) {
    // the nine children (row by row) of parent box pk, as leaf indices
    const auto [pl, pi, pj] = pk;
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) out[3 * b + a] = M.find(pl + 1, 3 * pi + a, 3 * pj + b);
    return pk;
  };
  for (const Box& pk : fams) {
    int kids[9];
    family(pk, kids);
    for (int k = 0; k < 9; ++k) coarsen[kids[k]] = 1;
  }
  for (bool changed = true; changed;) {
    changed = false;
    for (const Box& pk : fams) {
      int kids[9];
      auto [pl, pi, pj] = family(pk, kids);
      if (!coarsen[kids[0]]) continue;
      bool ok = true;
      for (int f = 0; f < 4 && ok; ++f)
        if (across_face(M, nl, pl, pi, pj, f, L) > pl + 1) ok = false;
      if (!ok) {
        for (int k = 0; k < 9; ++k) coarsen[kids[k]] = 0;
        changed = true;
      }
    }
  }
  std::set<Box> emitted;
  nlev.clear(); nci.clear(); ncj.clear(); ops.clear();
  auto emit = [&](int l, int i, int j, int op, int a, int b, const int* src, int ns) {
    nlev.push_back(l); nci.push_back(i); ncj.push_back(j);
    int rec[12] = {op, a, b, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    for (int k = 0; k < ns; ++k) rec[3 + k] = src[k];
    ops.insert(ops.end(), rec, rec + 12);
  };
  for (int c = 0; c < C; ++c) {
    const int l = lev[c], i = ci[c], j = cj[c];
    if (coarsen[c]) {
      const Box pk(l - 1, i / 3, j / 3);
      if (!emitted.insert(pk).second) continue;
      int src[9];
      family(pk, src);
      emit(l - 1, i / 3, j / 3, kRestrict, 0, 0, src, 9);
      continue;
    }
    if (eff[c] == 1) {
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) emit(l + 1, 3 * i + a, 3 * j + b, kProlong, a, b, &c, 1);
    } else {
      emit(l, i, j, kCopy, 0, 0, &c, 1);
    }
  }
  return ADG_OK;
}

}  // namespace adg
