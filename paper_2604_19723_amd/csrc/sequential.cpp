// Host side of the residual projector (Sec. IV-D.2) and of project-out-and-
// rescan detection built on it.
#include <hip/hip_runtime.h>

#include <string>

#include "ba_internal.h"

using namespace ba;

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct SeqLayout {
  size_t rt, p, i1, v1, r1, spec, total;
};

// Each pass's spectrum is staged in the workspace, except on plans whose
// projection emits peak candidates: there the workspace holds the candidate
// records of one pass (k = 1) instead.
SeqLayout seq_layout(const Plan& p, int B) {
  SeqLayout L;
  size_t o = 0;
  L.rt = o; o += al(size_t(B) * p.M * p.M * 8);
  L.p = o; o += al(candidates_supported(p) ? candidate_bytes(p, B, 1) : size_t(B) * p.G * 4);
  L.i1 = o; o += al(size_t(B) * 4);
  L.v1 = o; o += al(size_t(B) * 4);
  L.r1 = o; o += al(size_t(B) * p.ndim * 8);
  L.spec = o; o += al(spectrum_ws_bytes(p, B));
  L.total = o;
  return L;
}

ba_status s_arg(const char* fn, const std::string& w) {
  set_error(std::string(fn) + ": " + w);
  return BA_ERR_ARG;
}

ba_status s_dev(const char* fn, hipError_t e) {
  set_error(std::string(fn) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
  return BA_ERR_DEVICE;
}

}  // namespace

extern "C" {

ba_status ba_residual_covariance(ba_plan plan, int32_t n_trials, const void* R, int32_t S, const void* Psi,
                                 void* R_out, void* stream) {
  static const char* fn = "ba_residual_covariance";
  if (!plan) return s_arg(fn, "plan is NULL");
  if (n_trials < 0) return s_arg(fn, "n_trials >= 0 required");
  if (S < 0 || S > kMaxPeaks) return s_arg(fn, "S must be in [0, 16]");
  if (n_trials == 0) return BA_OK;
  if (!R || !R_out || (S > 0 && !Psi)) return s_arg(fn, "null buffer");
  const Plan& p = *static_cast<const Plan*>(plan);
  const hipError_t e = launch_residual(p, n_trials, static_cast<const float2*>(R), S,
                                       static_cast<const float2*>(Psi), nullptr, 0, static_cast<float2*>(R_out),
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : s_dev(fn, e);
}

ba_status ba_sequential_workspace_size(ba_plan plan, int32_t n_trials, size_t* bytes) {
  if (!plan || !bytes || n_trials < 0) return s_arg("ba_sequential_workspace_size", "bad argument");
  *bytes = seq_layout(*static_cast<const Plan*>(plan), n_trials).total;
  return BA_OK;
}

ba_status ba_sequential_peaks(ba_plan plan, int32_t n_trials, const void* R, int32_t k, int32_t* idx, float* val,
                              double* refined, void* workspace, size_t workspace_bytes, void* stream) {
  static const char* fn = "ba_sequential_peaks";
  if (!plan) return s_arg(fn, "plan is NULL");
  if (n_trials < 0) return s_arg(fn, "n_trials >= 0 required");
  if (k < 1 || k > kMaxPeaks) return s_arg(fn, "k must be in [1, 16]");
  if (n_trials == 0) return BA_OK;
  if (!R || !idx || !val) return s_arg(fn, "null buffer");
  const Plan& p = *static_cast<const Plan*>(plan);
  const SeqLayout L = seq_layout(p, n_trials);
  if (!workspace || workspace_bytes < L.total)
    return s_arg(fn, "workspace missing or smaller than ba_sequential_workspace_size");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return s_arg(fn, "workspace must be 256-byte aligned");
  char* w = static_cast<char*>(workspace);
  float2* Rt = reinterpret_cast<float2*>(w + L.rt);
  float* P = reinterpret_cast<float*>(w + L.p);
  int* i1 = reinterpret_cast<int*>(w + L.i1);
  float* v1 = reinterpret_cast<float*>(w + L.v1);
  double* r1 = reinterpret_cast<double*>(w + L.r1);
  void* spec = w + L.spec;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const float2* R0 = static_cast<const float2*>(R);
  hipError_t e = hipSuccess;
  for (int pass = 0; pass < k && e == hipSuccess; ++pass) {
    const float2* src = R0;
    if (pass > 0) {
      // the first `pass` columns of idx hold the points found so far
      e = launch_residual(p, n_trials, R0, pass, nullptr, idx, k, Rt, s);
      src = Rt;
    }
    if (candidates_supported(p)) {
      float4* rec = reinterpret_cast<float4*>(P);
      if (e == hipSuccess) e = launch_spectrum_candidates(p, n_trials, src, nullptr, 1, rec, s);
      if (e == hipSuccess) e = launch_peaks_merge(p, n_trials, 1, rec, i1, v1, r1, s);
    } else {
      if (e == hipSuccess) e = launch_spectrum(p, n_trials, src, P, spec, s);
      if (e == hipSuccess) e = launch_peaks(p, n_trials, P, 1, i1, v1, r1, s);
    }
    if (e == hipSuccess) e = launch_put_column(n_trials, pass, k, p.ndim, i1, v1, r1, idx, val, refined, s);
  }
  return e == hipSuccess ? BA_OK : s_dev(fn, e);
}

}  // extern "C"
