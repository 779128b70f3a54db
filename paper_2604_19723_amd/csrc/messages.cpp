// Host side of the particle update messages (Sec. IV-C; Supplementary Sec. S-V).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "ba_internal.h"
#include "messages.h"

using namespace ba;

struct ba_msgs_s {
  MsgGeom geo{};
  double* d_geom = nullptr;  // pa [J][3], rot [J][9]
};

namespace {

ba_status m_arg(const char* fn, const std::string& w) {
  set_error(std::string(fn) + ": " + w);
  return BA_ERR_ARG;
}

ba_status m_dev(const char* fn, hipError_t e) {
  set_error(std::string(fn) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
  return e == hipErrorOutOfMemory ? BA_ERR_NOMEM : BA_ERR_DEVICE;
}

}  // namespace

extern "C" {

ba_status ba_msgs_create(ba_msgs* out, int32_t n_arrays, const double* pa_pos, const double* pa_rot, int32_t n_y,
                         int32_t n_z, int32_t n_f, double fc, double bandwidth) {
  static const char* fn = "ba_msgs_create";
  if (!out) return m_arg(fn, "out is NULL");
  *out = nullptr;
  if (n_arrays < 1 || n_arrays > 16) return m_arg(fn, "n_arrays must be in [1, 16]");
  if (n_y < 1 || n_y > 16 || n_z < 1 || n_z > 16) return m_arg(fn, "n_y and n_z must be in [1, 16]");
  if (n_f < 1 || n_f > 64) return m_arg(fn, "n_f must be in [1, 64]");
  if (n_f * n_y * n_z > 1024) return m_arg(fn, "n_f * n_y * n_z must be <= 1024");
  if (!(fc > 0.0) || !(bandwidth >= 0.0) || !std::isfinite(fc) || !std::isfinite(bandwidth))
    return m_arg(fn, "fc > 0 and bandwidth >= 0 required");
  if (!pa_pos || !pa_rot) return m_arg(fn, "null host array");
  auto* h = new ba_msgs_s;
  std::vector<double> geom(pa_pos, pa_pos + 3 * n_arrays);
  geom.insert(geom.end(), pa_rot, pa_rot + 9 * n_arrays);
  hipError_t e = hipMalloc(&h->d_geom, geom.size() * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(h->d_geom, geom.data(), geom.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (h->d_geom) (void)hipFree(h->d_geom);
    delete h;
    return m_dev(fn, e);
  }
  h->geo.J = n_arrays;
  h->geo.nf = n_f;
  h->geo.ny = n_y;
  h->geo.nz = n_z;
  h->geo.fc = fc;
  h->geo.df = n_f > 1 ? bandwidth / (n_f - 1) : 0.0;
  h->geo.pa = h->d_geom;
  h->geo.rot = h->d_geom + 3 * n_arrays;
  *out = h;
  return BA_OK;
}

ba_status ba_msgs_destroy(ba_msgs h) {
  if (!h) return m_arg("ba_msgs_destroy", "handle is NULL");
  (void)hipDeviceSynchronize();
  (void)hipFree(h->d_geom);
  delete h;
  return BA_OK;
}

ba_status ba_msgs_workspace_size(ba_msgs h, int32_t n_feat, int32_t n_part, size_t* bytes) {
  static const char* fn = "ba_msgs_workspace_size";
  if (!h || !bytes) return m_arg(fn, "null argument");
  if (n_feat < 1 || n_feat > 16) return m_arg(fn, "n_feat must be in [1, 16]");
  if (n_part < 1 || n_part > (1 << 26)) return m_arg(fn, "n_part must be in [1, 2^26]");
  *bytes = msg_workspace_bytes(h->geo, n_feat, n_part);
  return BA_OK;
}

ba_status ba_update_messages(ba_msgs h, const ba_msg_inputs* in, const ba_msg_outputs* out, void* workspace,
                             size_t workspace_bytes, void* stream) {
  static const char* fn = "ba_update_messages";
  if (!h || !in || !out) return m_arg(fn, "null handle, inputs or outputs");
  const int S = in->n_feat, P = in->n_part;
  if (S < 1 || S > 16) return m_arg(fn, "n_feat must be in [1, 16]");
  if (P < 1 || P > (1 << 26)) return m_arg(fn, "n_part must be in [1, 2^26]");
  if (!in->z || !in->mt_pos || !in->w_beta || !in->sfv || !in->gamma || !in->mu || !in->w_alpha || !in->zeta ||
      !in->eta || !in->w_xi)
    return m_arg(fn, "null input buffer");
  const size_t need = msg_workspace_bytes(h->geo, S, P);
  if (!workspace || workspace_bytes < need) return m_arg(fn, "workspace missing or smaller than ba_msgs_workspace_size");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return m_arg(fn, "workspace must be 256-byte aligned");
  MsgIn mi;
  mi.S = S;
  mi.P = P;
  mi.z = static_cast<const double2*>(in->z);
  mi.mt = in->mt_pos;
  mi.wb = in->w_beta;
  mi.sfv = in->sfv;
  mi.gamma = in->gamma;
  mi.mu = static_cast<const double2*>(in->mu);
  mi.wa = in->w_alpha;
  mi.zeta = in->zeta;
  mi.eta = in->eta;
  mi.wxi = in->w_xi;
  MsgOut mo{out->log_iota, out->log_nu, out->log_kappa, out->log_kappa0, out->log_omega};
  const hipError_t e = launch_messages(h->geo, mi, mo, workspace, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : m_dev(fn, e);
}

}  // extern "C"
