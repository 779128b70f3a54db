// C-ABI entry points: argument validation, plan lifetime, host-side steering
// tables, and dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ba_internal.h"

namespace ba {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

static ba_status arg_error(const char* fn, const std::string& what) {
  set_error(std::string(fn) + ": " + what);
  return BA_ERR_ARG;
}

static ba_status dev_error(const char* fn, hipError_t e) {
  set_error(std::string(fn) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
  return e == hipErrorOutOfMemory ? BA_ERR_NOMEM : BA_ERR_DEVICE;
}

// Unit propagation direction of grid point g (directional cosines, Suppl. S-II).
static void grid_direction(int kind, const double* grid, int64_t g, double u[3]) {
  constexpr double d2r = M_PI / 180.0;
  if (kind == BA_GRID_ULA_DEG) {
    const double t = grid[g] * d2r;
    u[0] = std::cos(t);
    u[1] = std::sin(t);
    u[2] = 0.0;
  } else if (kind == BA_GRID_AZEL_DEG) {
    const double az = grid[2 * g] * d2r, el = grid[2 * g + 1] * d2r;
    u[0] = std::cos(el) * std::cos(az);
    u[1] = std::cos(el) * std::sin(az);
    u[2] = std::sin(el);
  } else {
    u[0] = grid[3 * g];
    u[1] = grid[3 * g + 1];
    u[2] = grid[3 * g + 2];
  }
}

// Which projection kernel a plan uses. Up to 64 elements Q stays in registers
// (k_proj_q in FP32, k_proj_qb for the BF16 passes); larger arrays use the
// streaming kernel, which first writes Q to the workspace in fragment order.
static bool uses_stream(const Plan& p) { return p.precision != BA_PREC_F32_VALU && p.Mp > 64; }

size_t spectrum_ws_bytes(const Plan& p, int B) { return uses_stream(p) ? qprep_bytes(p, B) : 0; }

hipError_t launch_spectrum(const Plan& p, int B, const float2* R, float* P, void* ws, hipStream_t s) {
  if (p.precision == BA_PREC_F32_VALU) return launch_spectrum_valu(p, B, R, P, s);
  if (!uses_stream(p))
    return p.precision == BA_PREC_F32 ? launch_spectrum_mfma(p, B, R, P, s) : launch_spectrum_qb(p, B, R, P, s);
  return launch_spectrum_stream(p, B, R, ws, P, s);
}

// Steering value a_g[m] = exp(+j 2 pi p_m . u_g) in FP64, the phase in cycles
// reduced to [-1/2, 1/2] before the complex exponential.
struct Steer {
  const std::vector<double>& pos;
  const std::vector<double>& u;  // [G][3]
  void operator()(int m, int64_t g, double* re, double* im) const {
    double ph = pos[3 * m] * u[3 * g] + pos[3 * m + 1] * u[3 * g + 1] + pos[3 * m + 2] * u[3 * g + 2];
    ph -= std::rint(ph);
    const double w = 2.0 * M_PI * ph;
    *re = std::cos(w);
    *im = std::sin(w);
  }
};

static uint16_t bf16_rne_host(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

static float bf16_to_float_host(uint16_t h) {
  const uint32_t u = uint32_t(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Real-equivalent steering x_g = [Re a_g; Im a_g] (rows padded to 2 Mp with
// zeros) in the MFMA B-fragment order shared by the projection kernels:
// column g of block jb = g / 16 sits at lane (k % 4) * 16 + g % 16 of k-step
// k / 4, and four consecutive k-steps of one lane share a 16-byte word.
static std::vector<float> build_x_table(const Steer& st, int M, int64_t G, int Mp, int64_t nblocks) {
  const int K = 2 * Mp;
  std::vector<float> x(size_t(nblocks) * K * 16, 0.f);
  auto place = [&](int64_t g, int k, float v) {
    const int64_t jb = g / 16;
    const int j = int(g % 16), s = k / 4, l = (k % 4) * 16 + j;
    x[size_t(jb) * K * 16 + size_t(((s / 4) * 64 + l) * 4 + (s % 4))] = v;
  };
  for (int m = 0; m < M; ++m)
    for (int64_t g = 0; g < G; ++g) {
      double re, im;
      st(m, g, &re, &im);
      place(g, m, float(re));
      place(g, Mp + m, float(im));
    }
  return x;
}

// The same steering split into BF16 hi = bf16(x), lo = bf16(x - hi) from the
// FP64 value, in the B-fragment order of v_mfma_f32_16x16x32_bf16:
// [block][k-chunk of 32][hi, lo][lane][8], lane l element e holding
// x[32 kc + 8 (l / 16) + e] of column 16 block + l % 16.
static std::vector<uint16_t> build_xb_table(const Steer& st, int M, int64_t G, int Mp,
                                            int64_t nblocks) {
  const int K = 2 * Mp, nkc = K / 32;
  std::vector<uint16_t> x(size_t(nblocks) * K * 16 * 2, 0);
  auto place = [&](int64_t g, int k, double v) {
    const int64_t jb = g / 16;
    const int j = int(g % 16), kc = k / 32, kk = k % 32;
    const int l = (kk / 8) * 16 + j, e = kk % 8;
    const uint16_t hi = bf16_rne_host(float(v));
    const uint16_t lo = bf16_rne_host(float(v - double(bf16_to_float_host(hi))));
    const size_t base = ((size_t(jb) * nkc + kc) * 2) * 512;
    x[base + size_t(l) * 8 + e] = hi;
    x[base + 512 + size_t(l) * 8 + e] = lo;
  };
  for (int m = 0; m < M; ++m)
    for (int64_t g = 0; g < G; ++g) {
      double re, im;
      st(m, g, &re, &im);
      place(g, m, re);
      place(g, Mp + m, im);
    }
  return x;
}

static void free_plan(Plan* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  if (p->d_A) (void)hipFree(p->d_A);
  if (p->d_X) (void)hipFree(p->d_X);
  if (p->d_Xb) (void)hipFree(p->d_Xb);
  if (p->d_coords) (void)hipFree(p->d_coords);
  (void)hipSetDevice(cur);
  delete p;
}

// FP32 fragment-order table of the first Mrows elements of a plan, padded to Mp
// element rows and nblocks column blocks (used by the ragged path per size class).
std::vector<float> plan_x_table(const Plan& p, int Mrows, int Mp, int64_t nblocks) {
  std::vector<double> u(size_t(p.G) * 3);
  for (int64_t g = 0; g < p.G; ++g) grid_direction(p.kind, p.coords.data(), g, &u[3 * g]);
  const Steer st{p.pos, u};
  return build_x_table(st, Mrows, p.G, Mp, nblocks);
}

}  // namespace ba

using namespace ba;

static inline Plan* P_(ba_plan p) { return static_cast<Plan*>(p); }

extern "C" {

const char* ba_status_string(ba_status s) {
  switch (s) {
    case BA_OK: return "ok";
    case BA_ERR_ARG: return "invalid argument";
    case BA_ERR_DEVICE: return "device error";
    case BA_ERR_NOMEM: return "out of device memory";
    case BA_ERR_UNSUPPORTED: return "unsupported";
    case BA_ERR_STATE: return "invalid state";
    default: return "unknown status";
  }
}

const char* ba_last_error(void) { return g_last_error.c_str(); }

const char* ba_version(void) { return "bartlett-mi355x 0.1 (gfx950)"; }

ba_status ba_plan_create(ba_plan* out, int32_t n_elem, const double* elem_pos_wl,
                         int32_t grid_kind, int64_t n_grid, const double* grid,
                         int32_t grid_shape0, int32_t grid_shape1, int32_t wrap0,
                         int32_t precision) {
  static const char* fn = "ba_plan_create";
  if (!out) return arg_error(fn, "out is NULL");
  *out = nullptr;
  if (n_elem < 1 || n_elem > kMaxElem) return arg_error(fn, "n_elem must be in [1, 256]");
  if (!elem_pos_wl) return arg_error(fn, "elem_pos_wl is NULL");
  if (grid_kind != BA_GRID_DIRS && grid_kind != BA_GRID_ULA_DEG && grid_kind != BA_GRID_AZEL_DEG)
    return arg_error(fn, "unknown grid_kind");
  if (n_grid < 1 || n_grid > (int64_t(1) << 30)) return arg_error(fn, "n_grid out of range");
  if (!grid) return arg_error(fn, "grid is NULL");
  const int s1 = grid_shape1 <= 1 ? 1 : grid_shape1;
  if (grid_shape0 < 1 || int64_t(grid_shape0) * s1 != n_grid)
    return arg_error(fn, "grid_shape0 * grid_shape1 must equal n_grid");
  if (wrap0 < 0 || wrap0 > 2) return arg_error(fn, "wrap0 must be 0, 1 or 2");
  if (wrap0 && (wrap0 == 2 ? grid_shape0 - 1 : grid_shape0) < 3)
    return arg_error(fn, "a wrapping dimension needs a period of at least 3");
  if (precision != BA_PREC_F32 && precision != BA_PREC_BF16X3 && precision != BA_PREC_BF16 &&
      precision != BA_PREC_F32_VALU)
    return arg_error(fn, "unknown precision");
  for (int64_t i = 0; i < int64_t(n_elem) * 3; ++i)
    if (!std::isfinite(elem_pos_wl[i])) return arg_error(fn, "non-finite element position");
  const int64_t gvals = n_grid * (grid_kind == BA_GRID_ULA_DEG ? 1 : grid_kind == BA_GRID_AZEL_DEG ? 2 : 3);
  for (int64_t i = 0; i < gvals; ++i)
    if (!std::isfinite(grid[i])) return arg_error(fn, "non-finite grid value");

  ba_plan_s* p = new (std::nothrow) ba_plan_s();
  if (!p) return arg_error(fn, "host allocation failed");
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { delete p; return dev_error(fn, e); }
  p->M = n_elem;
  p->G = n_grid;
  p->kind = grid_kind;
  p->shape0 = grid_shape0;
  p->shape1 = s1;
  p->wrap0 = wrap0;
  p->rows = wrap0 == 2 ? grid_shape0 - 1 : grid_shape0;
  p->ndim = s1 == 1 ? 1 : 2;
  p->coord_dim = grid_kind == BA_GRID_ULA_DEG ? 1 : grid_kind == BA_GRID_AZEL_DEG ? 2 : 3;
  p->precision = precision;
  p->pos.assign(elem_pos_wl, elem_pos_wl + 3 * n_elem);
  p->coords.assign(grid, grid + gvals);

  // Steering tables, all from FP64 values: the complex [M][G] table of the
  // vector-ALU kernels, the FP32 real-equivalent table in MFMA fragment order,
  // and (split precisions) its BF16 hi/lo split.
  const int M = n_elem;
  std::vector<double> u(size_t(n_grid) * 3);
  for (int64_t g = 0; g < n_grid; ++g) grid_direction(grid_kind, grid, g, &u[3 * g]);
  const Steer st{p->pos, u};
  std::vector<float2> at(size_t(n_grid) * M);  // [M][G]
  for (int m = 0; m < M; ++m)
    for (int64_t g = 0; g < n_grid; ++g) {
      double re, im;
      st(m, g, &re, &im);
      at[size_t(m) * n_grid + g] = make_float2(float(re), float(im));
    }
  const bool split = precision == BA_PREC_BF16X3 || precision == BA_PREC_BF16;
  p->Mp = M <= 8 ? 8 : M <= 16 ? 16 : M <= 32 ? 32 : M <= 64 ? 64 : M <= 128 ? 128 : 256;
  if (split && p->Mp < 64) p->Mp = 64;
  p->Gb = (n_grid + 15) / 16;
  p->Xblocks = (p->Gb + 31) / 32 * 32;
  e = hipMalloc(&p->d_A, at.size() * sizeof(float2));
  if (e == hipSuccess) e = hipMemcpy(p->d_A, at.data(), at.size() * sizeof(float2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&p->d_coords, p->coords.size() * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_coords, p->coords.data(), p->coords.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    std::vector<float> x = build_x_table(st, M, n_grid, p->Mp, p->Xblocks);
    e = hipMalloc(&p->d_X, x.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(p->d_X, x.data(), x.size() * sizeof(float), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && split) {
    std::vector<uint16_t> xb = build_xb_table(st, M, n_grid, p->Mp, p->Xblocks);
    e = hipMalloc(&p->d_Xb, xb.size() * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemcpy(p->d_Xb, xb.data(), xb.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    ba_status st = dev_error(fn, e);
    free_plan(p);
    return st;
  }
  *out = p;
  return BA_OK;
}

ba_status ba_plan_destroy(ba_plan p) {
  if (!p) return BA_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(P_(p)->device);
  (void)hipDeviceSynchronize();
  (void)hipSetDevice(cur);
  free_plan(P_(p));
  return BA_OK;
}

ba_status ba_plan_info(ba_plan p, int32_t* n_elem, int64_t* n_grid, int32_t* ndim) {
  if (!p) return arg_error("ba_plan_info", "plan is NULL");
  if (n_elem) *n_elem = P_(p)->M;
  if (n_grid) *n_grid = P_(p)->G;
  if (ndim) *ndim = P_(p)->ndim;
  return BA_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

ba_status ba_workspace_size(ba_plan p, int32_t n_trials, int32_t n_snap, int32_t with_spectrum_out,
                            size_t* bytes) {
  static const char* fn = "ba_workspace_size";
  if (!p) return arg_error(fn, "plan is NULL");
  if (!bytes) return arg_error(fn, "bytes is NULL");
  if (n_trials < 0 || n_snap < 1) return arg_error(fn, "n_trials >= 0 and n_snap >= 1 required");
  const Plan& q = *P_(p);
  size_t b = align256(size_t(n_trials) * q.M * q.M * sizeof(float2));
  if (candidates_supported(q)) {
    b += align256(candidate_bytes(q, n_trials, kMaxPeaks));
  } else {
    b += align256(spectrum_ws_bytes(q, n_trials));
    if (!with_spectrum_out) b += align256(size_t(n_trials) * q.G * sizeof(float));
  }
  *bytes = b;
  return BA_OK;
}

ba_status ba_spectrum_workspace_size(ba_plan p, int32_t n_trials, size_t* bytes) {
  static const char* fn = "ba_spectrum_workspace_size";
  if (!p) return arg_error(fn, "plan is NULL");
  if (!bytes) return arg_error(fn, "bytes is NULL");
  if (n_trials < 0) return arg_error(fn, "n_trials >= 0 required");
  *bytes = spectrum_ws_bytes(*P_(p), n_trials);
  return BA_OK;
}

#define CHECK_PLAN(fn)                                   \
  if (!p) return arg_error(fn, "plan is NULL");          \
  const Plan& q = *P_(p);                                \
  (void)q;

ba_status ba_covariance(ba_plan p, int32_t n_trials, int32_t n_snap, const void* Y, void* R,
                        void* stream) {
  static const char* fn = "ba_covariance";
  CHECK_PLAN(fn);
  if (n_trials < 0 || n_snap < 1) return arg_error(fn, "n_trials >= 0 and n_snap >= 1 required");
  if (n_trials == 0) return BA_OK;
  if (!Y || !R) return arg_error(fn, "null buffer");
  hipError_t e = launch_covariance(q, n_trials, n_snap, static_cast<const float2*>(Y),
                                   static_cast<float2*>(R), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : dev_error(fn, e);
}

ba_status ba_spectrum(ba_plan p, int32_t n_trials, const void* R, float* P, void* workspace,
                      size_t workspace_bytes, void* stream) {
  static const char* fn = "ba_spectrum";
  CHECK_PLAN(fn);
  if (n_trials < 0) return arg_error(fn, "n_trials >= 0 required");
  if (n_trials == 0) return BA_OK;
  if (!R || !P) return arg_error(fn, "null buffer");
  const size_t need = spectrum_ws_bytes(q, n_trials);
  if (need && (!workspace || workspace_bytes < need))
    return arg_error(fn, "workspace missing or smaller than ba_spectrum_workspace_size");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return arg_error(fn, "workspace must be 256-byte aligned");
  hipError_t e = launch_spectrum(q, n_trials, static_cast<const float2*>(R), P, workspace,
                                 static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : dev_error(fn, e);
}

ba_status ba_spectrum_snapshots(ba_plan p, int32_t n_trials, int32_t n_snap, const void* Y,
                                float* P, void* stream) {
  static const char* fn = "ba_spectrum_snapshots";
  CHECK_PLAN(fn);
  if (n_trials < 0 || n_snap < 1) return arg_error(fn, "n_trials >= 0 and n_snap >= 1 required");
  if (n_trials == 0) return BA_OK;
  if (!Y || !P) return arg_error(fn, "null buffer");
  hipError_t e = launch_spectrum_snapshots(q, n_trials, n_snap, static_cast<const float2*>(Y), P,
                                           static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : dev_error(fn, e);
}

ba_status ba_peaks(ba_plan p, int32_t n_trials, const float* P, int32_t k, int32_t* idx,
                   float* val, double* refined, void* stream) {
  static const char* fn = "ba_peaks";
  CHECK_PLAN(fn);
  if (n_trials < 0) return arg_error(fn, "n_trials >= 0 required");
  if (k < 1 || k > kMaxPeaks) return arg_error(fn, "k must be in [1, 16]");
  if (n_trials == 0) return BA_OK;
  if (!P || !idx || !val) return arg_error(fn, "null buffer");
  hipError_t e = launch_peaks(q, n_trials, P, k, idx, val, refined, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : dev_error(fn, e);
}

ba_status ba_proposal_moments(ba_plan p, int32_t n_trials, const float* P, double* mu_cov,
                              void* stream) {
  static const char* fn = "ba_proposal_moments";
  CHECK_PLAN(fn);
  if (n_trials < 0) return arg_error(fn, "n_trials >= 0 required");
  if (n_trials == 0) return BA_OK;
  if (!P || !mu_cov) return arg_error(fn, "null buffer");
  hipError_t e = launch_moments(q, n_trials, P, mu_cov, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : dev_error(fn, e);
}

ba_status ba_proposal_sample(ba_plan p, int32_t n_trials, const double* mu_cov, int32_t n_particles,
                             const double* z, double* particles, double* weights, void* stream) {
  static const char* fn = "ba_proposal_sample";
  CHECK_PLAN(fn);
  if (n_trials < 0 || n_particles < 0) return arg_error(fn, "n_trials >= 0 and n_particles >= 0 required");
  if (q.kind == BA_GRID_DIRS) {
    set_error(std::string(fn) + ": direction-vector grids have no angle region");
    return BA_ERR_UNSUPPORTED;
  }
  if (n_trials == 0 || n_particles == 0) return BA_OK;
  if (!mu_cov || !z || !particles || !weights) return arg_error(fn, "null buffer");
  // the region spanned by the grid's coordinates (degrees)
  ProposalRegion reg{};
  const int d = q.coord_dim;
  const int64_t G = q.G;
  for (int a = 0; a < d; ++a) {
    double lo = q.coords[a], hi = q.coords[a];
    for (int64_t g = 0; g < G; ++g) {
      lo = std::min(lo, q.coords[g * d + a]);
      hi = std::max(hi, q.coords[g * d + a]);
    }
    reg.lo[a] = lo;
    reg.hi[a] = hi;
    reg.period[a] = 0.0;
  }
  if (q.kind == BA_GRID_AZEL_DEG && q.wrap0) {
    // azimuth runs along the first grid axis (rows of shape1 points)
    const int s1 = q.shape1;
    reg.lo[0] = q.coords[0];
    reg.period[0] = q.wrap0 == 2 ? q.coords[int64_t(q.shape0 - 1) * s1 * d] - q.coords[0]
                                 : double(q.shape0) * (q.coords[int64_t(s1) * d] - q.coords[0]);
    reg.hi[0] = reg.lo[0] + reg.period[0];
    if (!(reg.period[0] > 0.0)) return arg_error(fn, "azimuth grid without a positive period");
  }
  hipError_t e = launch_proposal_sample(n_trials, mu_cov, d, n_particles, z, reg, particles, weights,
                                        static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : dev_error(fn, e);
}

// An error reported by the entry point `from` on behalf of `fn`: the message
// names fn.
static ba_status renamed_error(const char* fn, const char* from, ba_status st) {
  std::string m = g_last_error;
  const size_t n = std::strlen(from);
  if (m.compare(0, n, from) == 0) m = fn + m.substr(n);
  set_error(m);
  return st;
}

ba_status ba_candidates_size(ba_plan p, int32_t n_trials, int32_t k, size_t* bytes) {
  static const char* fn = "ba_candidates_size";
  CHECK_PLAN(fn);
  if (!bytes) return arg_error(fn, "bytes is NULL");
  if (n_trials < 0) return arg_error(fn, "n_trials >= 0 required");
  if (k < 1 || k > kMaxPeaks) return arg_error(fn, "k must be in [1, 16]");
  if (!candidates_supported(q)) {
    set_error(std::string(fn) + ": plans of up to 64 elements on 1-D grids in FP32, BF16x3 or BF16 only");
    return BA_ERR_UNSUPPORTED;
  }
  *bytes = candidate_bytes(q, n_trials, k);
  return BA_OK;
}

ba_status ba_spectrum_candidates(ba_plan p, int32_t n_trials, const void* R, int32_t k, float* P, void* cand,
                                 size_t cand_bytes, void* stream) {
  static const char* fn = "ba_spectrum_candidates";
  size_t need = 0;
  const ba_status st = ba_candidates_size(p, n_trials, k, &need);
  if (st != BA_OK) return renamed_error(fn, "ba_candidates_size", st);
  if (n_trials == 0) return BA_OK;
  if (!R || !cand) return arg_error(fn, "null buffer");
  if (cand_bytes < need) return arg_error(fn, "cand smaller than ba_candidates_size");
  if (reinterpret_cast<uintptr_t>(cand) & 15) return arg_error(fn, "cand must be 16-byte aligned");
  hipError_t e = launch_spectrum_candidates(*P_(p), n_trials, static_cast<const float2*>(R), P, k,
                                            static_cast<float4*>(cand), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : dev_error(fn, e);
}

ba_status ba_peaks_merge(ba_plan p, int32_t n_trials, int32_t k, const void* cand, int32_t* idx, float* val,
                         double* refined, void* stream) {
  static const char* fn = "ba_peaks_merge";
  size_t need = 0;
  const ba_status st = ba_candidates_size(p, n_trials, k, &need);
  if (st != BA_OK) return renamed_error(fn, "ba_candidates_size", st);
  if (n_trials == 0) return BA_OK;
  if (!cand || !idx || !val) return arg_error(fn, "null buffer");
  hipError_t e = launch_peaks_merge(*P_(p), n_trials, k, static_cast<const float4*>(cand), idx, val, refined,
                                    static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BA_OK : dev_error(fn, e);
}

ba_status ba_run(ba_plan p, int32_t n_trials, int32_t n_snap, const void* Y, int32_t k, float* P,
                 int32_t* idx, float* val, double* refined, void* workspace, size_t workspace_bytes,
                 void* stream) {
  static const char* fn = "ba_run";
  CHECK_PLAN(fn);
  if (n_trials < 0 || n_snap < 1) return arg_error(fn, "n_trials >= 0 and n_snap >= 1 required");
  if (k < 1 || k > kMaxPeaks) return arg_error(fn, "k must be in [1, 16]");
  if (n_trials == 0) return BA_OK;
  if (!Y || !idx || !val) return arg_error(fn, "null buffer");
  size_t need = 0;
  ba_workspace_size(p, n_trials, n_snap, P != nullptr, &need);
  if (!workspace || workspace_bytes < need)
    return arg_error(fn, "workspace missing or smaller than ba_workspace_size");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return arg_error(fn, "workspace must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  float2* R = reinterpret_cast<float2*>(ws);
  char* Qws = ws + align256(size_t(n_trials) * q.M * q.M * sizeof(float2));
  if (candidates_supported(q)) {
    float4* rec = reinterpret_cast<float4*>(Qws);
    hipError_t e = launch_covariance(q, n_trials, n_snap, static_cast<const float2*>(Y), R, s);
    if (e == hipSuccess) e = launch_spectrum_candidates(q, n_trials, R, P, k, rec, s);
    if (e == hipSuccess) e = launch_peaks_merge(q, n_trials, k, rec, idx, val, refined, s);
    return e == hipSuccess ? BA_OK : dev_error(fn, e);
  }
  float* Pw = P;
  if (!Pw) Pw = reinterpret_cast<float*>(Qws + align256(spectrum_ws_bytes(q, n_trials)));
  hipError_t e = launch_covariance(q, n_trials, n_snap, static_cast<const float2*>(Y), R, s);
  if (e == hipSuccess) e = launch_spectrum(q, n_trials, R, Pw, Qws, s);
  if (e == hipSuccess) e = launch_peaks(q, n_trials, Pw, k, idx, val, refined, s);
  return e == hipSuccess ? BA_OK : dev_error(fn, e);
}

}  // extern "C"
