// The fused q-space loss head for callers that cannot allocate (code under
// graph capture, tight serving loops, harnesses that forbid allocation):
// the same kernels as dlm_sh2signal_mse_fwd_bwd, with the per-wave partial
// sums and the two-pass reduction's chunk sums in a static device array
// instead of a caller workspace.
//
// `scratch` is one array per device, held until the process ends.  In host
// code its name is only a host-side stand-in, so its device address is
// looked up once per device (that device current) and cached; every launch
// takes the cached pointer.  The kernels write every partial they later
// read, so nothing needs clearing between calls.  All calls on one device
// share the array: calls that overlap on one device (different streams,
// or host threads without ordering between them) race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace {

// 4 MiB: per-wave partials for up to (kScratchFloats - kSumBlocks) waves of
// 16 voxels x one shell, e.g. 5.59 M voxels of a three-shell table.
constexpr size_t kScratchFloats = size_t(1) << 20;
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float *g_scratch[kMaxDevices] = {};

// Device address of the current device's `scratch`, looked up on the first
// call on that device.
dlm_status scratch_for_current_device(float **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0)
    return dlm::report(DLM_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(hipGetLastError()));
  if (dev >= kMaxDevices) return dlm::report(DLM_EDEVICE, "device %d is beyond the %d devices supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !ptr)
      return dlm::report(DLM_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                         hipGetErrorString(rc));
    g_scratch[dev] = static_cast<float *>(ptr);
  }
  *out = g_scratch[dev];
  return DLM_OK;
}

}  // namespace

extern "C" {

size_t dlm_sh2signal_mse_static_scratch_bytes(void) { return kScratchFloats * sizeof(float); }

dlm_status dlm_sh2signal_mse_fwd_bwd_noalloc(const dlm_sh_plan *plan, const float *c, const float *target, int64_t V,
                                             float *loss, float *dc, float *xhat, dlm_precision prec, void *stream) {
  if (!plan) return dlm::report(DLM_EINVAL, "plan is NULL");
  if (V <= 0) return dlm::report(DLM_EINVAL, "V must be > 0");
  const size_t need = dlm_sh2signal_mse_workspace_bytes(plan, V);
  const size_t have = kScratchFloats * sizeof(float);
  if (need > have)
    return dlm::report(DLM_EWORKSPACE,
                       "%lld voxels need %zu bytes of partial sums; the static scratch holds %zu "
                       "(use dlm_sh2signal_mse_fwd_bwd with a workspace)",
                       (long long)V, need, have);
  float *ptr = nullptr;
  const dlm_status s = scratch_for_current_device(&ptr);
  if (s != DLM_OK) return s;
  return dlm_sh2signal_mse_fwd_bwd(plan, c, target, V, loss, dc, xhat, ptr, have, prec, stream);
}

}  // extern "C"
