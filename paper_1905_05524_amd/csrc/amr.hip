// Adaptive mesh refinement: the regrid plan (host) and the state transfer
// kernel (gfx950).
//
// Plan (paper, Section 3: refinement criterion, subcells are coarsened only
// when all of them are marked): flags +1 refine, -1 coarsen, 0 keep; refine
// is dropped at the finest level, coarsen at the coarsest; a family of nine
// siblings is replaced by its parent only if all nine are leaves flagged
// coarsen.  New leaf order: old leaves in order; a refined leaf is replaced
// by its children (row by row), a coarsened family by its parent at the
// position of its first sibling.
// Transfer: copy; prolongation to a child by exact interpolation of the
// parent polynomial; restriction of nine children by L2 projection.
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

static long long fkey(int l, int i, int j) { return ((long long)l << 52) ^ ((long long)i << 26) ^ (long long)j; }

// New leaf list and transfer ops from the old leaves and flags.
int regrid_plan(const std::vector<int>& lev, const std::vector<int>& ci, const std::vector<int>& cj,
                const int8_t* flags, int L, std::vector<int>& nlev, std::vector<int>& nci, std::vector<int>& ncj,
                std::vector<int>& ops) {
  const int C = (int)lev.size();
  std::vector<int> eff(C);
  for (int c = 0; c < C; ++c) {
    int f = flags[c];
    if (f != -1 && f != 0 && f != 1) return fail(ADG_EINVAL, "flags must be -1, 0 or +1");
    if (f == 1 && lev[c] >= L) f = 0;
    if (f == -1 && lev[c] == 0) f = 0;
    eff[c] = f;
  }
  // families whose nine children are all leaves flagged coarsen
  std::unordered_map<long long, int> cnt;
  std::unordered_map<long long, int> child_of;   // child key -> old index
  for (int c = 0; c < C; ++c)
    if (lev[c] > 0) {
      child_of[fkey(lev[c], ci[c], cj[c])] = c;
      if (eff[c] == -1) cnt[fkey(lev[c] - 1, ci[c] / 3, cj[c] / 3)] += 1;
    }
  std::unordered_map<long long, int> emitted;
  nlev.clear(); nci.clear(); ncj.clear(); ops.clear();
  auto emit = [&](int l, int i, int j, int op, int a, int b, const int* src, int ns) {
    nlev.push_back(l); nci.push_back(i); ncj.push_back(j);
    int rec[12] = {op, a, b, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    for (int k = 0; k < ns; ++k) rec[3 + k] = src[k];
    ops.insert(ops.end(), rec, rec + 12);
  };
  for (int c = 0; c < C; ++c) {
    const int l = lev[c], i = ci[c], j = cj[c];
    if (l > 0) {
      const long long pk = fkey(l - 1, i / 3, j / 3);
      auto it = cnt.find(pk);
      if (it != cnt.end() && it->second == 9) {
        if (emitted.count(pk)) continue;
        emitted[pk] = 1;
        int src[9];
        for (int b = 0; b < 3; ++b)
          for (int a = 0; a < 3; ++a)
            src[3 * b + a] = child_of.at(fkey(l, 3 * (i / 3) + a, 3 * (j / 3) + b));
        emit(l - 1, i / 3, j / 3, kRestrict, 0, 0, src, 9);
        continue;
      }
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
