// The allocation-free step: adg_step with its workspace (the predictor's
// partial update Q*, the face data and the per-cell time-step bounds) in a
// file-scope device array instead of a caller-supplied buffer, for callers
// that cannot allocate device memory.
//
// The array is a device symbol: in host code its name is a host-side stand-in,
// never a device address.  Its address on a device comes from
// hipGetSymbolAddress with that device current, looked up once per device
// (at handle creation) and kept per device; every launch receives that
// address.  Each GPU holds its own copy until the process ends, and every
// call on one GPU shares it.
#include <mutex>

#include "adg_internal.h"

namespace adg {

constexpr size_t kStaticScratchBytes = ADG_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

int static_scratch_address(int dev, void** ptr) {
  *ptr = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return fail(ADG_EUNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ADG_EHIP, std::string("static scratch lookup failed: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return ADG_OK;
}

int launch_predictor_any(const Group& g, double* store, hipStream_t s);
int launch_corrector(const Group& g, hipStream_t s);
int launch_corrector_clock(Group g, double* clock, hipStream_t s);

}  // namespace adg

using namespace adg;

extern "C" int adg_step_static(adg_mesh* m, double* Q, double* clock, void* stream) {
  if (!m) return fail(ADG_EINVAL, "null handle");
  if (!Q || !clock) return fail(ADG_EINVAL, "null buffer");
  if (((uintptr_t)Q & 7) != 0 || ((uintptr_t)clock & 7) != 0) return fail(ADG_EINVAL, "misaligned buffer");
  if (m->g.C == 0) return fail(ADG_ESTATE, "mesh has no cells");
  if (m->ws_bytes > kStaticScratchBytes)
    return fail(ADG_EINVAL, "mesh needs " + std::to_string(m->ws_bytes) + " bytes of workspace; the static scratch holds " +
                                std::to_string(kStaticScratchBytes));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(ADG_EHIP, "no current device");
  if (dev != m->dev) return fail(ADG_EINVAL, "current device is not the handle's device");
  if (m->static_scratch_rc != ADG_OK || !m->static_scratch)
    return fail(ADG_EHIP, "static scratch unavailable on this device");
  // the handle's group with the step's buffers: the caller's Q and clock,
  // the workspace sections at the same offsets as in a bound workspace
  Group g = m->g;
  char* ws = static_cast<char*>(m->static_scratch);
  g.Q = Q;
  g.Qs = reinterpret_cast<double*>(ws + m->off_qs);
  g.FD = reinterpret_cast<double*>(ws + m->off_fd);
  g.dtc = reinterpret_cast<double*>(ws + m->off_dtc);
  g.clock = clock;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = launch_predictor_any(g, nullptr, s);
  if (rc) return rc;
  return launch_corrector_clock(g, clock, s);
}
