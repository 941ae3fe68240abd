// Measured device peaks (include/adg_peaks.h): FP64 vector FMA loop, FP64
// matrix-core loop, stream copy.  Each compute loop keeps several independent
// dependency chains per wavefront so that issue, not latency, bounds it.
#include <cmath>

#include "adg_peaks.h"
#include "adg_internal.h"

namespace adg {

constexpr int kPeakThreads = 256;
constexpr int kPeakBlocks = 256 * 8;   // eight workgroups per CU
constexpr int kFmaChains = 8, kFmaIters = 4096;
constexpr int kMfmaChains = 4, kMfmaIters = 2048;
typedef double v4d __attribute__((ext_vector_type(4)));

// x <- x y + z in kFmaChains independent chains (|y| < 1: values stay bounded)
__global__ __launch_bounds__(kPeakThreads) void k_peak_fma(double* sink, double y, double z) {
  double x[kFmaChains];
#pragma unroll
  for (int c = 0; c < kFmaChains; ++c) x[c] = z * (c + 1 + threadIdx.x % 7);
  for (int i = 0; i < kFmaIters; ++i) {
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) x[c] = fma(x[c], y, z);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kFmaChains; ++c) s += x[c];
  sink[(size_t)blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// acc += A B on 16x16x4 tiles in kMfmaChains independent accumulators
__global__ __launch_bounds__(kPeakThreads) void k_peak_mfma(double* sink, double a, double b) {
  v4d acc[kMfmaChains];
#pragma unroll
  for (int c = 0; c < kMfmaChains; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
  const double av = a * (1 + threadIdx.x % 4), bv = b * (1 + threadIdx.x % 3);
  for (int i = 0; i < kMfmaIters; ++i) {
#pragma unroll
    for (int c = 0; c < kMfmaChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kMfmaChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  sink[(size_t)blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// FP64 matrix cores beside the FP64 vector units: the waves of a workgroup
// below mfma_waves run chains of v_mfma_f64_4x4x4 (512 flops each), the
// others chains of vector FMAs: four MFMA chains of kMfmaIters steps (2,048
// flops per wavefront and step), eight FMA chains of 4 kMfmaIters steps
// (twice the flops of the MFMA side).
__global__ __launch_bounds__(kPeakThreads) void k_peak_share(double* sink, double a, double b, int mfma_waves) {
  const int wave = threadIdx.x / kWave;
  double s = 0.0;
  if (wave < mfma_waves) {
    double acc[kMfmaChains];
#pragma unroll
    for (int c = 0; c < kMfmaChains; ++c) acc[c] = 0.0;
    const double av = a * (1 + threadIdx.x % 4), bv = b * (1 + threadIdx.x % 3);
    for (int i = 0; i < kMfmaIters; ++i) {
#pragma unroll
      for (int c = 0; c < kMfmaChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bv, acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < kMfmaChains; ++c) s += acc[c];
  } else {
    double x[kFmaChains];
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) x[c] = a * (c + 1 + threadIdx.x % 7);
    for (int i = 0; i < 4 * kMfmaIters; ++i) {
#pragma unroll
      for (int c = 0; c < kFmaChains; ++c) x[c] = fma(x[c], 0.999999, b);
    }
#pragma unroll
    for (int c = 0; c < kFmaChains; ++c) s += x[c];
  }
  sink[(size_t)blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// dst <- src, 16-byte words, four per thread and round with the loads issued together
__global__ __launch_bounds__(kPeakThreads) void k_peak_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                            size_t n2) {
  const size_t stride = (size_t)gridDim.x * kPeakThreads;
  for (size_t k = (size_t)blockIdx.x * kPeakThreads + threadIdx.x; k < n2; k += 4 * stride) {
    if (k + 3 * stride < n2) {
      const double2 v0 = src[k], v1 = src[k + stride], v2 = src[k + 2 * stride], v3 = src[k + 3 * stride];
      dst[k] = v0; dst[k + stride] = v1; dst[k + 2 * stride] = v2; dst[k + 3 * stride] = v3;
    } else {
      for (int u = 0; u < 4; ++u)
        if (k + u * stride < n2) dst[k + u * stride] = src[k + u * stride];
    }
  }
}

}  // namespace adg

using namespace adg;

namespace {

// fastest of three timed launches (after one untimed), in milliseconds
template <class Launch>
int best_ms(hipStream_t s, Launch launch, double& best) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(ADG_EHIP, "event create failed");
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(ADG_EHIP, "event create failed"); }
  int rc = ADG_OK;
  best = INFINITY;
  launch();
  rc = check_launch("peak loop");
  for (int r = 0; r < 3 && rc == ADG_OK; ++r) {
    (void)hipEventRecord(e0, s);
    launch();
    (void)hipEventRecord(e1, s);
    rc = check_launch("peak loop");
    if (rc == ADG_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(ADG_EHIP, "event synchronize failed");
    float ms = 0.0f;
    if (rc == ADG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(ADG_EHIP, "event time failed");
    if (rc == ADG_OK && ms < best) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

extern "C" {

int adg_peaks_sink_bytes(size_t* bytes) {
  if (!bytes) return fail(ADG_EINVAL, "null argument");
  *bytes = sizeof(double) * (size_t)kPeakBlocks * kPeakThreads;
  return ADG_OK;
}

int adg_measure_fp64_sharing(void* sink, double* out, void* stream) {
  if (!sink || !out) return fail(ADG_EINVAL, "null argument");
  if (((uintptr_t)sink & 7) != 0) return fail(ADG_EINVAL, "misaligned sink");
  hipStream_t s = (hipStream_t)stream;
  double* sk = static_cast<double*>(sink);
  const int waves_per_block = kPeakThreads / kWave;
  const double blocks = kPeakBlocks;
  const double mfma_flops = 512.0 * kMfmaChains * kMfmaIters;                   // per wave
  const double fma_flops = 2.0 * kFmaChains * 4.0 * kMfmaIters * kWave;         // per wave
  double ms = 0.0;
  // MFMA on every wave, then FMA on every wave, then half and half
  const int split[3] = {waves_per_block, 0, waves_per_block / 2};
  for (int k = 0; k < 3; ++k) {
    int rc = best_ms(s, [&] {
      hipLaunchKernelGGL(k_peak_share, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, sk, 1e-3, 2e-3, split[k]);
    }, ms);
    if (rc) return rc;
    const double mw = blocks * split[k], vw = blocks * (waves_per_block - split[k]);
    const double secs = ms * 1e-3;
    if (k == 0) out[0] = mfma_flops * mw / secs / 1e12;
    if (k == 1) out[1] = fma_flops * vw / secs / 1e12;
    if (k == 2) { out[3] = mfma_flops * mw / secs / 1e12; out[4] = fma_flops * vw / secs / 1e12; out[2] = out[3] + out[4]; }
  }
  return ADG_OK;
}

int adg_measure_peaks(void* sink, const void* src, void* dst, size_t copy_bytes, double* out, void* stream) {
  if (!sink || !out) return fail(ADG_EINVAL, "null argument");
  if (((uintptr_t)sink & 7) != 0) return fail(ADG_EINVAL, "misaligned sink");
  if (copy_bytes) {
    if (!src || !dst) return fail(ADG_EINVAL, "null copy buffer");
    if ((copy_bytes & 15) != 0 || ((uintptr_t)src & 15) != 0 || ((uintptr_t)dst & 15) != 0)
      return fail(ADG_EINVAL, "copy buffers and size must be 16-byte aligned");
  }
  hipStream_t s = (hipStream_t)stream;
  double* sk = static_cast<double*>(sink);
  double ms = 0.0;
  int rc = best_ms(s, [&] {
    hipLaunchKernelGGL(k_peak_fma, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, sk, 0.999999, 1e-3);
  }, ms);
  if (rc) return rc;
  out[0] = 2.0 * kFmaChains * kFmaIters * (double)kPeakBlocks * kPeakThreads / (ms * 1e-3) / 1e12;
  rc = best_ms(s, [&] {
    hipLaunchKernelGGL(k_peak_mfma, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, sk, 1e-3, 2e-3);
  }, ms);
  if (rc) return rc;
  const double waves = (double)kPeakBlocks * (kPeakThreads / kWave);
  out[1] = 2048.0 * kMfmaChains * kMfmaIters * waves / (ms * 1e-3) / 1e12;
  out[2] = NAN;
  if (copy_bytes) {
    const size_t n2 = copy_bytes / 16;
    const unsigned blocks = (unsigned)std::min<size_t>((n2 + kPeakThreads - 1) / kPeakThreads, 256 * 64);
    rc = best_ms(s, [&] {
      hipLaunchKernelGGL(k_peak_copy, dim3(blocks), dim3(kPeakThreads), 0, s, static_cast<const double2*>(src),
                         static_cast<double2*>(dst), n2);
    }, ms);
    if (rc) return rc;
    out[2] = 2.0 * (double)copy_bytes / (ms * 1e-3) / 1e9;
  }
  return ADG_OK;
}

}  // extern "C"
