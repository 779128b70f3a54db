// Host side of the learned-proposal path: pack -> network -> windows ->
// full-grid fallback for the trials whose windows are not conclusive.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "mlp.h"
#include "propose.h"

using namespace ba;

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t x, u, list, count, rc, pc, ic, vc, refc, total;
};

Layout layout(const Plan& p, int B, int dout, int K) {
  Layout L;
  size_t o = 0;
  L.x = o; o += al(size_t(B) * p.M * p.M * 4);
  L.u = o; o += al(size_t(B) * dout * 4);
  L.list = o; o += al(size_t(B) * 4);
  L.count = o; o += 256;
  L.rc = o; o += al(size_t(B) * p.M * p.M * 8);
  L.pc = o; o += al(size_t(B) * p.G * 4);
  L.ic = o; o += al(size_t(B) * K * 4);
  L.vc = o; o += al(size_t(B) * K * 4);
  L.refc = o; o += al(size_t(B) * K * 8);
  L.total = o;
  return L;
}

ba_status p_arg(const char* fn, const std::string& w) {
  set_error(std::string(fn) + ": " + w);
  return BA_ERR_ARG;
}

ba_status p_dev(const char* fn, hipError_t e) {
  set_error(std::string(fn) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
  return BA_ERR_DEVICE;
}

}  // namespace

// the network handle's layer sizes (defined in mlp.cpp)
extern "C" ba_status ba_mlp_dims(ba_mlp n, int32_t* d_in, int32_t* d_out);

extern "C" {

ba_status ba_propose_workspace_size(ba_plan plan, int32_t n_trials, int32_t d_out, int32_t k, size_t* bytes) {
  if (!plan || !bytes || n_trials < 0 || d_out < 1 || k < 1) return p_arg("ba_propose_workspace_size", "bad argument");
  *bytes = layout(*static_cast<const Plan*>(plan), n_trials, d_out, k).total;
  return BA_OK;
}

ba_status ba_propose_refine(ba_plan plan, ba_mlp net, int32_t n_trials, const void* R, int32_t k,
                            int32_t half_window, float tau, int32_t* idx, float* val, double* refined,
                            uint8_t* fell_back, int32_t* n_fallback, void* workspace, size_t workspace_bytes,
                            void* stream) {
  static const char* fn = "ba_propose_refine";
  if (!plan || !net) return p_arg(fn, "plan and network are required");
  const Plan& p = *static_cast<const Plan*>(plan);
  int32_t din = 0, dout = 0;
  ba_mlp_dims(net, &din, &dout);
  if (p.precision != BA_PREC_F32 || p.Mp > 64 || p.kind != BA_GRID_ULA_DEG || p.shape1 != 1 || p.wrap0)
    return p_arg(fn, "needs an FP32 plan of at most 64 elements on a 1-D angle grid");
  if (din != p.M * p.M) return p_arg(fn, "the network input must be M^2 (packed covariance)");
  if (k < 1 || k > kMaxProp || k > dout) return p_arg(fn, "k must be in [1, min(8, network outputs)]");
  if (half_window < 1 || half_window > kMaxHalfWindow) return p_arg(fn, "half_window must be in [1, 100]");
  if (!(tau >= 0.f && tau <= 1.f)) return p_arg(fn, "tau must be in [0, 1]");
  if (n_trials < 0) return p_arg(fn, "n_trials >= 0 required");
  if (n_trials == 0) {
    const hipError_t e0 = n_fallback ? launch_zero_count(n_fallback, static_cast<hipStream_t>(stream)) : hipSuccess;
    return e0 == hipSuccess ? BA_OK : p_dev(fn, e0);
  }
  if (!R || !idx || !val || !refined || !fell_back) return p_arg(fn, "null buffer");
  const Layout L = layout(p, n_trials, dout, k);
  if (!workspace || workspace_bytes < L.total) return p_arg(fn, "workspace smaller than ba_propose_workspace_size");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return p_arg(fn, "workspace must be 256-byte aligned");
  // uniform grid in degrees
  const double th0 = p.coords[0];
  const double step = p.G > 1 ? (p.coords[p.G - 1] - p.coords[0]) / double(p.G - 1) : 1.0;
  for (int64_t g = 0; g < p.G; ++g)
    if (std::fabs(p.coords[g] - (th0 + double(g) * step)) > 1e-9 * std::fabs(step) + 1e-12)
      return p_arg(fn, "the angle grid must be uniform");

  char* ws = static_cast<char*>(workspace);
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* X = reinterpret_cast<float*>(ws + L.x);
  float* U = reinterpret_cast<float*>(ws + L.u);
  int* list = reinterpret_cast<int*>(ws + L.list);
  int* count = reinterpret_cast<int*>(ws + L.count);
  hipError_t e = ba_pack_covariance(p.M, n_trials, R, X, stream) == BA_OK ? hipSuccess : hipErrorLaunchFailure;
  if (e == hipSuccess && ba_mlp_forward(net, n_trials, X, U, stream) != BA_OK) e = hipErrorLaunchFailure;
  if (e == hipSuccess) e = launch_zero_count(count, s);
  if (e == hipSuccess) {
    WindowArgs a{static_cast<const float2*>(R), reinterpret_cast<const float4*>(p.d_X), U, p.M, p.G, dout, k,
                 half_window, th0, step, tau, idx, val, refined, fell_back, list, count};
    e = launch_window(a, p.Mp, n_trials, s);
  }
  // full-grid fallback for the trials the window kernel listed: every launch
  // is sized for the whole batch and reads the list's length on the device,
  // so nothing here waits for the device
  if (e == hipSuccess) {
    float2* Rc = reinterpret_cast<float2*>(ws + L.rc);
    float* Pc = reinterpret_cast<float*>(ws + L.pc);
    int* ic = reinterpret_cast<int*>(ws + L.ic);
    float* vc = reinterpret_cast<float*>(ws + L.vc);
    double* rc = reinterpret_cast<double*>(ws + L.refc);
    e = launch_gather_r(list, count, n_trials, static_cast<const float2*>(R), Rc, p.M, s);
    // the projection's launch is shaped for a fallback batch of up to 1024
    // trials at a time (larger ones loop)
    if (e == hipSuccess) e = launch_spectrum_mfma_counted(p, n_trials, count, 1024, Rc, Pc, s);
    if (e == hipSuccess) e = launch_peaks(p, n_trials, Pc, k, ic, vc, rc, s, count);
    if (e == hipSuccess) e = launch_scatter(list, count, n_trials, k, ic, vc, rc, idx, val, refined, s);
    if (e == hipSuccess && n_fallback) e = hipMemcpyAsync(n_fallback, count, sizeof(int), hipMemcpyDeviceToDevice, s);
  }
  if (e != hipSuccess) return p_dev(fn, e);
  return BA_OK;
}

}  // extern "C"
