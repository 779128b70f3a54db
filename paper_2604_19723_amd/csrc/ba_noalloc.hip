// Allocation-free variant of the whole path (covariance -> spectrum -> peaks):
// the workspace is a fixed device array of this library instead of a caller
// buffer, so the call makes no allocation of any kind.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ba_internal.h"

namespace {

constexpr size_t kScratchBytes = BA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends. Host code never uses this
// name as an address: it is only the symbol handed to hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

// Device address of the current device's copy, looked up once per device.
hipError_t scratch_for_current_device(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

ba_status ba_run_noalloc(ba_plan p, int32_t n_trials, int32_t n_snap, const void* Y, int32_t k,
                         float* P, int32_t* idx, float* val, double* refined, void* stream) {
  static const char* fn = "ba_run_noalloc";
  if (!p) {
    ba::set_error(std::string(fn) + ": plan is NULL");
    return BA_ERR_ARG;
  }
  size_t need = 0;
  ba_status st = ba_workspace_size(p, n_trials, n_snap, P != nullptr, &need);
  if (st != BA_OK) {
    ba::set_error(std::string(fn) + ": n_trials >= 0 and n_snap >= 1 required");
    return st;
  }
  if (need > kScratchBytes) {
    ba::set_error(std::string(fn) + ": the batch needs " + std::to_string(need) +
                  " bytes of workspace, the fixed scratch array holds " + std::to_string(kScratchBytes) +
                  "; split the batch or pass P");
    return BA_ERR_ARG;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && dev != p->device) {
    ba::set_error(std::string(fn) + ": the plan's device must be the current device");
    return BA_ERR_ARG;
  }
  void* ws = nullptr;
  if (e == hipSuccess) e = scratch_for_current_device(dev, &ws);
  if (e != hipSuccess) {
    ba::set_error(std::string(fn) + ": scratch lookup failed: " + hipGetErrorName(e));
    return BA_ERR_DEVICE;
  }
  // every kernel of the path writes its part of the workspace before reading
  // it (R, the streamed Q, the staged spectrum), so nothing needs clearing
  return ba_run(p, n_trials, n_snap, Y, k, P, idx, val, refined, ws, kScratchBytes, stream);
}

}  // extern "C"
