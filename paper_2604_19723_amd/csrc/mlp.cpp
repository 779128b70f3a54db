// Host side of the proposal network: parameter and activation buffers
// (allocated once, for a maximum batch), forward, gradients, Adam steps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "mlp.h"

namespace ba {
namespace {

struct Mlp {
  int device = 0;
  int prec = BA_PREC_BF16;
  int L = 0;                 // affine layers
  std::vector<int> dims;     // d_in, hidden..., d_out
  std::vector<int64_t> woff, boff;
  int64_t nparams = 0;
  int max_batch = 0;
  float* params = nullptr;   // FP32 master weights [W1 b1 W2 b2 ...]
  float* grads = nullptr;
  float* am = nullptr;
  float* av = nullptr;
  std::vector<float*> Z, H;  // per hidden layer [max_batch][d]
  float* Yb = nullptr;       // [max_batch][d_out]
  float* dA = nullptr;       // ping-pong [max_batch][dmax]
  float* dB = nullptr;
  float* loss = nullptr;
  int64_t t = 0;             // Adam steps taken
};

hipError_t gemm(const Mlp& n, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                int64_t sbn, float* C, int64_t ldc, int M, int N, int K, int mode, const float* bias, float* Z,
                hipStream_t s) {
  GemmArgs g{A, B, C, M, N, K, sam, sak, sbk, sbn, ldc, mode, bias, Z};
  return launch_gemm(g, n.prec, s);
}

// forward over B <= max_batch rows; the output goes to Y (ldc d_out)
hipError_t forward_rows(const Mlp& n, int B, const float* X, float* Y, hipStream_t s) {
  const float* Hin = X;
  hipError_t e = hipSuccess;
  for (int l = 0; l < n.L && e == hipSuccess; ++l) {
    const int din = n.dims[l], dout = n.dims[l + 1];
    const float* W = n.params + n.woff[l];
    const float* b = n.params + n.boff[l];
    if (l < n.L - 1) {
      e = gemm(n, Hin, din, 1, W, 1, din, n.H[l], dout, B, dout, din, kGemmHidden, b, n.Z[l], s);
      Hin = n.H[l];
    } else {
      e = gemm(n, Hin, din, 1, W, 1, din, Y, dout, B, dout, din, kGemmBias, b, nullptr, s);
    }
  }
  return e;
}

// forward + loss + backward into n.grads (B <= max_batch)
hipError_t gradients(Mlp& n, int B, const float* X, const float* T, const float* mask, float* loss,
                     hipStream_t s) {
  hipError_t e = forward_rows(n, B, X, n.Yb, s);
  const int dout = n.dims[n.L];
  float* dZ = n.dA;
  float* dZn = n.dB;
  if (e == hipSuccess) e = launch_mse(n.Yb, T, mask, dZ, loss ? loss : n.loss, B * dout, s);
  for (int l = n.L - 1; l >= 0 && e == hipSuccess; --l) {
    const int din = n.dims[l], dl = n.dims[l + 1];
    const float* Hin = l == 0 ? X : n.H[l - 1];
    // dW = dZ^T Hin  [dl][din], K = B
    e = gemm(n, dZ, 1, dl, Hin, din, 1, n.grads + n.woff[l], din, dl, din, B, kGemmPlain, nullptr, nullptr, s);
    if (e == hipSuccess) e = launch_colsum(dZ, n.grads + n.boff[l], B, dl, s);
    if (l > 0 && e == hipSuccess) {
      // dZ_{l-1} = (dZ W) * gelu'(Z_{l-1})  [B][din], K = dl
      e = gemm(n, dZ, dl, 1, n.params + n.woff[l], din, 1, dZn, din, B, din, dl, kGemmGeluGrad, nullptr,
               n.Z[l - 1], s);
      std::swap(dZ, dZn);
    }
  }
  return e;
}

void free_mlp(Mlp* n) {
  if (!n) return;
  for (float* p : {n->params, n->grads, n->am, n->av, n->Yb, n->dA, n->dB, n->loss})
    if (p) (void)hipFree(p);
  for (float* p : n->Z)
    if (p) (void)hipFree(p);
  for (float* p : n->H)
    if (p) (void)hipFree(p);
  delete n;
}

}  // namespace
}  // namespace ba

using namespace ba;

struct ba_mlp_s : public ba::Mlp {};

static ba_status m_arg(const char* fn, const std::string& w) {
  set_error(std::string(fn) + ": " + w);
  return BA_ERR_ARG;
}

static ba_status m_dev(const char* fn, hipError_t e) {
  set_error(std::string(fn) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
  return e == hipErrorOutOfMemory ? BA_ERR_NOMEM : BA_ERR_DEVICE;
}

extern "C" {

ba_status ba_mlp_create(ba_mlp* out, int32_t d_in, int32_t d_hidden, int32_t n_hidden, int32_t d_out,
                        int32_t max_batch, int32_t precision, uint64_t seed) {
  static const char* fn = "ba_mlp_create";
  if (!out) return m_arg(fn, "out is NULL");
  *out = nullptr;
  if (d_in < 1 || d_hidden < 1 || n_hidden < 0 || d_out < 1 || d_in > (1 << 20) || d_hidden > (1 << 16) ||
      n_hidden > 16 || d_out > 1024)
    return m_arg(fn, "layer sizes out of range");
  if (max_batch < 1 || max_batch > (1 << 20)) return m_arg(fn, "max_batch out of range");
  if (precision != BA_PREC_F32 && precision != BA_PREC_BF16) return m_arg(fn, "precision must be F32 or BF16");
  ba_mlp n = new (std::nothrow) ba_mlp_s();
  if (!n) return m_arg(fn, "host allocation failed");
  n->prec = precision;
  n->max_batch = max_batch;
  n->dims.push_back(d_in);
  for (int i = 0; i < n_hidden; ++i) n->dims.push_back(d_hidden);
  n->dims.push_back(d_out);
  n->L = int(n->dims.size()) - 1;
  int64_t off = 0;
  int dmax = 0;
  for (int l = 0; l < n->L; ++l) {
    n->woff.push_back(off);
    off += int64_t(n->dims[l + 1]) * n->dims[l];
    n->boff.push_back(off);
    off += n->dims[l + 1];
    dmax = std::max(dmax, n->dims[l + 1]);
  }
  dmax = std::max(dmax, d_hidden);
  n->nparams = off;
  hipError_t e = hipGetDevice(&n->device);
  const size_t pb = size_t(off) * sizeof(float);
  if (e == hipSuccess) e = hipMalloc(&n->params, pb);
  if (e == hipSuccess) e = hipMalloc(&n->grads, pb);
  if (e == hipSuccess) e = hipMalloc(&n->am, pb);
  if (e == hipSuccess) e = hipMalloc(&n->av, pb);
  if (e == hipSuccess) e = hipMemset(n->am, 0, pb);
  if (e == hipSuccess) e = hipMemset(n->av, 0, pb);
  for (int l = 0; l < n->L - 1 && e == hipSuccess; ++l) {
    float *z = nullptr, *h = nullptr;
    e = hipMalloc(&z, size_t(max_batch) * n->dims[l + 1] * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&h, size_t(max_batch) * n->dims[l + 1] * sizeof(float));
    n->Z.push_back(z);
    n->H.push_back(h);
  }
  if (e == hipSuccess) e = hipMalloc(&n->Yb, size_t(max_batch) * d_out * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&n->dA, size_t(max_batch) * dmax * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&n->dB, size_t(max_batch) * dmax * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&n->loss, 256);
  if (e == hipSuccess) {
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases
    std::vector<float> w(off);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < n->L; ++l) {
      const double bound = 1.0 / std::sqrt(double(n->dims[l]));
      std::uniform_real_distribution<double> U(-bound, bound);
      for (int64_t i = n->woff[l]; i < n->boff[l] + n->dims[l + 1]; ++i) w[i] = float(U(rng));
    }
    e = hipMemcpy(n->params, w.data(), pb, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    ba_status st = m_dev(fn, e);
    free_mlp(n);
    return st;
  }
  *out = n;
  return BA_OK;
}

ba_status ba_mlp_destroy(ba_mlp n) {
  if (!n) return BA_OK;
  (void)hipDeviceSynchronize();
  free_mlp(n);
  return BA_OK;
}

ba_status ba_mlp_dims(ba_mlp n, int32_t* d_in, int32_t* d_out) {
  if (!n) return m_arg("ba_mlp_dims", "handle is NULL");
  if (d_in) *d_in = n->dims[0];
  if (d_out) *d_out = n->dims[n->L];
  return BA_OK;
}

ba_status ba_mlp_num_params(ba_mlp n, int64_t* count) {
  if (!n || !count) return m_arg("ba_mlp_num_params", "null argument");
  *count = n->nparams;
  return BA_OK;
}

ba_status ba_mlp_get_weights(ba_mlp n, float* host, int64_t count) {
  static const char* fn = "ba_mlp_get_weights";
  if (!n || !host) return m_arg(fn, "null argument");
  if (count != n->nparams) return m_arg(fn, "count must equal ba_mlp_num_params");
  hipError_t e = hipMemcpy(host, n->params, size_t(count) * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? BA_OK : m_dev(fn, e);
}

ba_status ba_mlp_set_weights(ba_mlp n, const float* host, int64_t count) {
  static const char* fn = "ba_mlp_set_weights";
  if (!n || !host) return m_arg(fn, "null argument");
  if (count != n->nparams) return m_arg(fn, "count must equal ba_mlp_num_params");
  hipError_t e = hipMemcpy(n->params, host, size_t(count) * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(n->am, 0, size_t(count) * sizeof(float));
  if (e == hipSuccess) e = hipMemset(n->av, 0, size_t(count) * sizeof(float));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  n->t = 0;
  return e == hipSuccess ? BA_OK : m_dev(fn, e);
}

ba_status ba_mlp_forward(ba_mlp n, int32_t B, const float* X, float* Y, void* stream) {
  static const char* fn = "ba_mlp_forward";
  if (!n) return m_arg(fn, "handle is NULL");
  if (B < 0) return m_arg(fn, "B >= 0 required");
  if (B == 0) return BA_OK;
  if (!X || !Y) return m_arg(fn, "null buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int din = n->dims[0], dout = n->dims[n->L];
  hipError_t e = hipSuccess;
  for (int b0 = 0; b0 < B && e == hipSuccess; b0 += n->max_batch) {
    const int nb = std::min(n->max_batch, B - b0);
    e = forward_rows(*n, nb, X + int64_t(b0) * din, Y + int64_t(b0) * dout, s);
  }
  return e == hipSuccess ? BA_OK : m_dev(fn, e);
}

ba_status ba_mlp_gradients(ba_mlp n, int32_t B, const float* X, const float* T, const float* mask,
                           float* grads_out, float* loss_out, void* stream) {
  static const char* fn = "ba_mlp_gradients";
  if (!n) return m_arg(fn, "handle is NULL");
  if (B < 1 || B > n->max_batch) return m_arg(fn, "1 <= B <= max_batch required");
  if (!X || !T || !grads_out) return m_arg(fn, "null buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = gradients(*n, B, X, T, mask, loss_out, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(grads_out, n->grads, size_t(n->nparams) * sizeof(float), hipMemcpyDeviceToDevice, s);
  return e == hipSuccess ? BA_OK : m_dev(fn, e);
}

ba_status ba_mlp_train_step(ba_mlp n, int32_t B, const float* X, const float* T, const float* mask,
                            float lr, float* loss_out, void* stream) {
  static const char* fn = "ba_mlp_train_step";
  if (!n) return m_arg(fn, "handle is NULL");
  if (B < 1 || B > n->max_batch) return m_arg(fn, "1 <= B <= max_batch required");
  if (!X || !T) return m_arg(fn, "null buffer");
  if (!(lr > 0.f) || !std::isfinite(lr)) return m_arg(fn, "lr must be positive");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = gradients(*n, B, X, T, mask, loss_out, s);
  n->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = float(1.0 - std::pow(b1, double(n->t)));
  const float c2 = float(1.0 - std::pow(b2, double(n->t)));
  if (e == hipSuccess) e = launch_adam(n->params, n->grads, n->am, n->av, n->nparams, lr, float(b1), float(b2), 1e-8f, c1, c2, s);
  return e == hipSuccess ? BA_OK : m_dev(fn, e);
}

ba_status ba_pack_covariance(int32_t n_elem, int32_t n_trials, const void* R, float* X, void* stream) {
  static const char* fn = "ba_pack_covariance";
  if (n_elem < 2 || n_elem > kMaxElem) return m_arg(fn, "n_elem must be in [2, 256]");
  if (n_trials < 0) return m_arg(fn, "n_trials >= 0 required");
  if (n_trials == 0) return BA_OK;
  if (!R || !X) return m_arg(fn, "null buffer");
  hipError_t e = launch_pack(static_cast<const float2*>(R), X, n_elem, n_trials, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : m_dev(fn, e);
}

}  // extern "C"
