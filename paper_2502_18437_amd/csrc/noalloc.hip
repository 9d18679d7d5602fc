// Entry point that allocates nothing: mpm_eval_stress_noalloc, the stress
// evaluation of mpm_eval_stress (the fixed-corotated Kirchhoff stress of the
// substep's constitutive step) for callers that cannot allocate device
// memory. Host inputs and outputs are staged through `scratch`, a fixed
// device array of this translation unit, instead of the device buffers that
// mpm_eval_stress allocates per call; device inputs and outputs need no
// staging.
//
// `scratch` lives on every GPU the library runs on until the process ends.
// Host code never passes its name to a kernel or a copy: that name is a host
// stand-in, not a device address. The first call on a device looks up the
// device's own address of the array once (hipGetSymbolAddress, with that
// device current) and keeps it per device.
#include <mutex>

#include "mpm.h"
#include "mpm_internal.h"

namespace mpm {

// Per particle: F (9 floats), E (1) and tau (9).
constexpr int64_t kStageFloats = 19;
static_assert(MPM_NOALLOC_MAX_PARTICLES > 0, "the staging limit must be positive");
static __device__ __align__(256) float scratch[kStageFloats * MPM_NOALLOC_MAX_PARTICLES];

constexpr int kMaxDevices = 64;

namespace {

std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

thread_local const char* g_noalloc_error = nullptr;

int noalloc_fail(int code, const char* msg) {
  g_noalloc_error = msg;
  return code;
}

// Device address of `scratch` on the current device, looked up on the first
// call per device; nullptr on failure.
float* scratch_on_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

const char* noalloc_last_error() { return g_noalloc_error; }
void noalloc_clear_error() { g_noalloc_error = nullptr; }

}  // namespace mpm

using namespace mpm;

extern "C" int mpm_eval_stress_noalloc(int64_t n, const float* F, const float* E, float nu, float* tau,
                                       int32_t where) {
  g_noalloc_error = nullptr;
  if (n < 0 || (n > 0 && (!F || !E || !tau)) || !(nu >= 0.0f && nu < 0.5f) ||
      (where != MPM_HOST && where != MPM_DEVICE))
    return noalloc_fail(MPM_EINVAL, "mpm_eval_stress_noalloc: bad argument");
  if (n > MPM_NOALLOC_MAX_PARTICLES)
    return noalloc_fail(MPM_ETOOBIG, "mpm_eval_stress_noalloc: n exceeds MPM_NOALLOC_MAX_PARTICLES");
  if (n == 0) return MPM_OK;
  if (where == MPM_DEVICE) {
    launch_eval_stress(n, F, E, nu, tau, nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e == hipSuccess ? MPM_OK : noalloc_fail(MPM_EHIP, "mpm_eval_stress_noalloc: HIP error");
  }
  float* base = scratch_on_current_device();
  if (!base) return noalloc_fail(MPM_EHIP, "mpm_eval_stress_noalloc: hipGetSymbolAddress failed");
  float* dF = base;
  float* dE = base + 9 * n;
  float* dT = base + 10 * n;
  hipError_t e = hipMemcpy(dF, F, sizeof(float) * 9 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dE, E, sizeof(float) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_eval_stress(n, dF, dE, nu, dT, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(tau, dT, sizeof(float) * 9 * n, hipMemcpyDeviceToHost);
  return e == hipSuccess ? MPM_OK : noalloc_fail(MPM_EHIP, "mpm_eval_stress_noalloc: HIP error");
}
