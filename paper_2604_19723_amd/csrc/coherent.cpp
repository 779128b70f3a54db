// Host side of the coherent multi-array cost over SFV position candidates
// (the paper's own birth-proposal workload, Sec. IV-D.2 with the geometry of
// Sec. II-A and the array response of Sec. II-B).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ba_internal.h"
#include "coherent.h"

using namespace ba;

struct ba_coherent_s {
  int J = 0, nf = 0, ny = 0, nz = 0, Nz = 0, JNz = 0, Kp = 0;
  double fc = 0.0;
  int64_t G = 0, ctiles = 0;
  double* d_geom = nullptr;  // pa [J][3], rot [J][9], mt [3], freq [nf], py [ny], pz [nz]
  double* d_cand = nullptr;  // [G][3]
  double box_lo[3] = {0.0, 0.0, 0.0}, box_hi[3] = {0.0, 0.0, 0.0};  // the candidates' bounding box (m)
  float* d_X = nullptr;      // [ctiles * 8 blocks][Kp * 16] in MFMA B-fragment order
  CohGeom geo{};
};

namespace {

constexpr double kCLight = 299792458.0;

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

ba_status c_arg(const char* fn, const std::string& w) {
  set_error(std::string(fn) + ": " + w);
  return BA_ERR_ARG;
}

ba_status c_dev(const char* fn, hipError_t e) {
  set_error(std::string(fn) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
  return e == hipErrorOutOfMemory ? BA_ERR_NOMEM : BA_ERR_DEVICE;
}

void free_all(ba_coherent_s* h) {
  if (h->d_geom) (void)hipFree(h->d_geom);
  if (h->d_cand) (void)hipFree(h->d_cand);
  if (h->d_X) (void)hipFree(h->d_X);
  delete h;
}

}  // namespace

extern "C" {

ba_status ba_coherent_create(ba_coherent* out, int32_t n_arrays, const double* pa_pos, const double* pa_rot,
                             int32_t n_y, int32_t n_z, int32_t n_f, double fc, double bandwidth,
                             const double* p_mt, int64_t n_cand, const double* candidates) {
  static const char* fn = "ba_coherent_create";
  if (!out) return c_arg(fn, "out is NULL");
  *out = nullptr;
  if (n_arrays < 1 || n_arrays > 16) return c_arg(fn, "n_arrays must be in [1, 16]");
  if (n_y < 1 || n_y > 16 || n_z < 1 || n_z > 16) return c_arg(fn, "n_y and n_z must be in [1, 16]");
  if (n_f < 1 || n_f > 64) return c_arg(fn, "n_f must be in [1, 64]");
  if (!(fc > 0.0) || !(bandwidth >= 0.0) || !std::isfinite(fc) || !std::isfinite(bandwidth))
    return c_arg(fn, "fc > 0 and bandwidth >= 0 required");
  if (n_cand < 1 || n_cand > (int64_t(1) << 26)) return c_arg(fn, "n_cand must be in [1, 2^26]");
  if (!pa_pos || !pa_rot || !p_mt || !candidates) return c_arg(fn, "null host array");
  const int Nz = n_f * n_y * n_z;
  if (n_arrays * Nz > 2048) return c_arg(fn, "n_arrays * n_f * n_y * n_z must be <= 2048");
  for (int64_t g = 0; g < n_cand; ++g) {
    const double* s = candidates + 3 * g;
    const double n2 = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
    if (!(n2 > 0.0) || !std::isfinite(n2)) return c_arg(fn, "candidate SFV positions must be finite and nonzero");
  }
  auto* h = new ba_coherent_s;
  h->J = n_arrays;
  h->nf = n_f;
  h->ny = n_y;
  h->nz = n_z;
  h->Nz = Nz;
  h->JNz = n_arrays * Nz;
  h->Kp = (2 * h->JNz + 31) / 32 * 32;
  h->fc = fc;
  h->G = n_cand;
  h->ctiles = (n_cand + 127) / 128;
  for (int a = 0; a < 3; ++a) h->box_lo[a] = h->box_hi[a] = candidates[a];
  for (int64_t g = 1; g < n_cand; ++g)
    for (int a = 0; a < 3; ++a) {
      h->box_lo[a] = std::min(h->box_lo[a], candidates[3 * g + a]);
      h->box_hi[a] = std::max(h->box_hi[a], candidates[3 * g + a]);
    }
  // geometry: element positions at half a wavelength, centred; baseband
  // frequencies equally spaced over the bandwidth and centred on zero
  const double lam = kCLight / fc;
  std::vector<double> geom;
  geom.insert(geom.end(), pa_pos, pa_pos + 3 * n_arrays);
  geom.insert(geom.end(), pa_rot, pa_rot + 9 * n_arrays);
  geom.insert(geom.end(), p_mt, p_mt + 3);
  for (int f = 0; f < n_f; ++f)
    geom.push_back(n_f == 1 ? 0.0 : (f - (n_f - 1) / 2.0) * (bandwidth / (n_f - 1)));
  for (int i = 0; i < n_y; ++i) geom.push_back((i - (n_y - 1) / 2.0) * lam / 2.0);
  for (int i = 0; i < n_z; ++i) geom.push_back((i - (n_z - 1) / 2.0) * lam / 2.0);
  hipError_t e = hipMalloc(&h->d_geom, geom.size() * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(h->d_geom, geom.data(), geom.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&h->d_cand, size_t(n_cand) * 3 * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpy(h->d_cand, candidates, size_t(n_cand) * 3 * sizeof(double), hipMemcpyHostToDevice);
  const size_t xbytes = size_t(h->ctiles) * 8 * size_t(h->Kp) * 16 * sizeof(float);
  if (e == hipSuccess) e = hipMalloc(&h->d_X, xbytes);
  if (e == hipSuccess) e = hipMemset(h->d_X, 0, xbytes);  // padding rows and columns stay zero
  if (e != hipSuccess) {
    free_all(h);
    return c_dev(fn, e);
  }
  const double* d = h->d_geom;
  h->geo.J = n_arrays;
  h->geo.nf = n_f;
  h->geo.ny = n_y;
  h->geo.nz = n_z;
  h->geo.fc = fc;
  h->geo.pa = d;
  h->geo.rot = d + 3 * n_arrays;
  h->geo.mt = d + 12 * n_arrays;
  h->geo.freq = d + 12 * n_arrays + 3;
  h->geo.py = h->geo.freq + n_f;
  h->geo.pz = h->geo.py + n_y;
  e = launch_coh_table(h->geo, h->d_cand, n_cand, h->Kp, h->d_X, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_all(h);
    return c_dev(fn, e);
  }
  *out = h;
  return BA_OK;
}

ba_status ba_coherent_destroy(ba_coherent h) {
  if (!h) return c_arg("ba_coherent_destroy", "handle is NULL");
  (void)hipDeviceSynchronize();
  free_all(h);
  return BA_OK;
}

ba_status ba_coherent_info(ba_coherent h, int32_t* n_obs, int64_t* n_cand) {
  if (!h) return c_arg("ba_coherent_info", "handle is NULL");
  if (n_obs) *n_obs = h->JNz;
  if (n_cand) *n_cand = h->G;
  return BA_OK;
}

ba_status ba_coherent_workspace_size(ba_coherent h, int32_t n_trials, size_t* bytes) {
  if (!h || !bytes || n_trials < 0) return c_arg("ba_coherent_workspace_size", "bad argument");
  // the trial rows of the spectrum, or the slice partials of the moments (used one after the other)
  const size_t rows = al(size_t(coh_row_blocks(n_trials)) * (h->Kp / 16) * 256 * sizeof(float));
  const size_t mom = al(point_moments_ws_bytes(n_trials, h->G));
  *bytes = rows > mom ? rows : mom;
  return BA_OK;
}

ba_status ba_coherent_spectrum(ba_coherent h, int32_t n_trials, const void* Z, float* P, void* workspace,
                               size_t workspace_bytes, void* stream) {
  static const char* fn = "ba_coherent_spectrum";
  if (!h) return c_arg(fn, "handle is NULL");
  if (n_trials < 0) return c_arg(fn, "n_trials >= 0 required");
  if (n_trials == 0) return BA_OK;
  if (!Z || !P) return c_arg(fn, "null buffer");
  size_t need = 0;
  (void)ba_coherent_workspace_size(h, n_trials, &need);
  if (!workspace || workspace_bytes < need) return c_arg(fn, "workspace missing or smaller than ba_coherent_workspace_size");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return c_arg(fn, "workspace must be 256-byte aligned");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  float* A = static_cast<float*>(workspace);
  hipError_t e = launch_coh_rows(static_cast<const float2*>(Z), n_trials, h->JNz, h->Kp, A, s);
  if (e == hipSuccess)
    e = launch_coh_gemm(A, h->d_X, P, n_trials, h->G, h->ctiles, h->Kp, float(1.0 / (double(h->Nz) * h->Nz)), s);
  return e == hipSuccess ? BA_OK : c_dev(fn, e);
}

ba_status ba_coherent_moments(ba_coherent h, int32_t n_trials, const float* P, double* mu_cov, void* workspace,
                              size_t workspace_bytes, void* stream) {
  static const char* fn = "ba_coherent_moments";
  if (!h) return c_arg(fn, "handle is NULL");
  if (n_trials < 0) return c_arg(fn, "n_trials >= 0 required");
  if (n_trials == 0) return BA_OK;
  if (!P || !mu_cov) return c_arg(fn, "null buffer");
  size_t need = 0;
  (void)ba_coherent_workspace_size(h, n_trials, &need);
  if (!workspace || workspace_bytes < need) return c_arg(fn, "workspace missing or smaller than ba_coherent_workspace_size");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return c_arg(fn, "workspace must be 256-byte aligned");
  const hipError_t e = launch_point_moments(n_trials, P, h->G, h->d_cand, mu_cov, workspace,
                                            static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : c_dev(fn, e);
}

ba_status ba_coherent_sample(ba_coherent h, int32_t n_trials, const double* mu_cov, int32_t n_particles,
                             const double* z, double* particles, double* weights, void* stream) {
  static const char* fn = "ba_coherent_sample";
  if (!h) return c_arg(fn, "handle is NULL");
  if (n_trials < 0 || n_particles < 0) return c_arg(fn, "n_trials >= 0 and n_particles >= 0 required");
  if (n_trials == 0 || n_particles == 0) return BA_OK;
  if (!mu_cov || !z || !particles || !weights) return c_arg(fn, "null buffer");
  ProposalRegion reg{};
  for (int a = 0; a < 3; ++a) {
    reg.lo[a] = h->box_lo[a];
    reg.hi[a] = h->box_hi[a];
    reg.period[a] = 0.0;
  }
  const hipError_t e = launch_proposal_sample(n_trials, mu_cov, 3, n_particles, z, reg, particles, weights,
                                              static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : c_dev(fn, e);
}

}  // extern "C"
