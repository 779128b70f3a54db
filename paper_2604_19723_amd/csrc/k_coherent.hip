// The paper's own birth-proposal cost (Sec. IV-D.2): the coherent Bartlett
// spectrum over J arrays for candidate SFV positions,
//   P(s) = | sum_j (1/N_z) z_j^H psi_j(s) |^2,
// with psi_j the path-loss compensated wideband URA response of the path
// that a surface with SFV s creates between the terminal and array j
// (virtual anchor, Householder mirror and array rotation of Sec. II-A; array
// response of Sec. II-B).
//
// Stacking the arrays, z^H psi(s) is one complex inner product of length
// J N_z; with x_s = [Re psi; Im psi], u = [Re z; Im z] and v = [-Im z; Re z],
// Re = u^T x_s and Im = v^T x_s. A batch of trials that share the geometry is
// therefore a real GEMM [u_b; v_b] x X over K = 2 J N_z with |.|^2 fused into
// the epilogue, on v_mfma_f32_16x16x4f32.
//
//  k_coh_table: X in the MFMA B-fragment order of the projection kernels,
//    built once per plan from FP64 geometry and phases, rounded to FP32;
//  k_coh_rows: the trial rows in A-fragment order;
//  k_coh_gemm: 128 rows (64 trials) x 128 candidates per workgroup, 4 waves
//    of 32 rows; steering chunks of 32 k by LDS DMA, double-buffered; trial
//    fragments from L2 one chunk ahead; XCD-aware tile order so that the
//    row tiles of one candidate tile run together on one XCD.
#include <hip/hip_runtime.h>

#include "coherent.h"
#include "proj_common.h"

namespace ba {
namespace {

constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846;

// One thread per (candidate, array): geometry once, then its N_z elements.
// Element (k, j) of the table lies at block k/16... in the layout of the
// projection kernels: ((s / 4) * 64 + (k % 4) * 16 + col) * 4 + s % 4 within
// the 16-column block of the candidate, s = k / 4, for row k of x.
__global__ __launch_bounds__(256) void k_coh_table(CohGeom geo, const double* __restrict__ cand, int64_t G,
                                                   int Kp, float* __restrict__ X) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= G * geo.J) return;
  const int64_t g = t / geo.J;
  const int j = int(t - g * geo.J);
  const double s0 = cand[3 * g], s1 = cand[3 * g + 1], s2 = cand[3 * g + 2];
  const double ss = s0 * s0 + s1 * s1 + s2 * s2;
  const double* pa = geo.pa + 3 * j;
  const double* R = geo.rot + 9 * j;
  // virtual anchor p_va = p_pa - (2 p_pa.s / |s|^2 - 1) s; w = H (p_mt - p_va)
  const double k1 = 2.0 * (pa[0] * s0 + pa[1] * s1 + pa[2] * s2) / ss - 1.0;
  const double d0 = geo.mt[0] - (pa[0] - k1 * s0), d1 = geo.mt[1] - (pa[1] - k1 * s1),
               d2 = geo.mt[2] - (pa[2] - k1 * s2);
  const double k2 = 2.0 * (d0 * s0 + d1 * s1 + d2 * s2) / ss;
  const double w0 = d0 - k2 * s0, w1 = d1 - k2 * s1, w2 = d2 - k2 * s2;
  // local frame: r = R^T w (rotation stored row-major)
  const double r0 = R[0] * w0 + R[3] * w1 + R[6] * w2;
  const double r1 = R[1] * w0 + R[4] * w1 + R[7] * w2;
  const double r2 = R[2] * w0 + R[5] * w1 + R[8] * w2;
  const double d = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
  const double lam = kC / geo.fc;
  const double amp = lam / (4.0 * kPi * d);
  // sin(el) sin(az) = r_y / d and cos(el) = r_z / d
  const double uy = r1 / d, uz = r2 / d;
  const double ph0 = -2.0 * kPi * geo.fc * d / kC;
  const int Nz = geo.nf * geo.ny * geo.nz;
  const int half = geo.J * Nz;
  const int64_t blk = g / 16;
  const int col = int(g % 16);
  float* Xb = X + blk * int64_t(Kp) * 16;
  for (int f = 0; f < geo.nf; ++f) {
    const double phf = ph0 - 2.0 * kPi * geo.freq[f] * d / kC;
    for (int iy = 0; iy < geo.ny; ++iy) {
      const double phy = phf + 2.0 * kPi / lam * geo.py[iy] * uy;
      for (int iz = 0; iz < geo.nz; ++iz) {
        const double ph = phy + 2.0 * kPi / lam * geo.pz[iz] * uz;
        double sn, cs;
        sincos(ph, &sn, &cs);
        const int e = (f * geo.ny + iy) * geo.nz + iz;
        const int kr = j * Nz + e, ki = half + j * Nz + e;
        const int sr = kr / 4, si = ki / 4;
        Xb[((sr / 4) * 64 + (kr % 4) * 16 + col) * 4 + sr % 4] = float(amp * cs);
        Xb[((si / 4) * 64 + (ki % 4) * 16 + col) * 4 + si % 4] = float(amp * sn);
      }
    }
  }
}

// Trial rows in A-fragment order: A[rb][kg][lane][4], lane = i%16 + 16 (k%4),
// element s%4 for k-step s = k/4 and k-group kg = s/4; row 2b is u_b, row
// 2b+1 is v_b. Rows past 2B and k past 2 J N_z are zero.
__global__ __launch_bounds__(256) void k_coh_rows(const float2* __restrict__ Z, int B, int JNz, int Kp,
                                                  int64_t nrb, float* __restrict__ A) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int nkg = Kp / 16;
  const int64_t total = nrb * nkg * 256;
  if (t >= total) return;
  const int e = int(t % 4);
  const int lane = int((t / 4) % 64);
  const int64_t q = t / 256;
  const int kg = int(q % nkg);
  const int64_t rb = q / nkg;
  const int64_t i = rb * 16 + (lane & 15);
  const int k = (kg * 4 + e) * 4 + (lane >> 4);
  const int64_t b = i / 2;
  float v = 0.f;
  if (b < B && k < 2 * JNz) {
    const bool second = k >= JNz;
    const float2 z = Z[b * JNz + (second ? k - JNz : k)];
    v = (i & 1) == 0 ? (second ? z.y : z.x) : (second ? z.x : -z.y);
  }
  A[t] = v;
}

constexpr int kRB = 2;   // row blocks per wave
constexpr int kCBc = 8;  // 16-column blocks per tile

__global__ __launch_bounds__(256, 2) void k_coh_gemm(const float4* __restrict__ A, const float4* __restrict__ X,
                                                     float* __restrict__ P, int B, int64_t G, int Kp, int nrow,
                                                     int64_t nlogical, float scale) {
  extern __shared__ __attribute__((aligned(16))) float4 sB[];  // [2][kCBc blocks][2 k-groups][64]
  constexpr int CH = kCBc * 2 * 64;                             // float4 per chunk (16 KB)
  const int64_t nphys = int64_t(gridDim.x);
  const int64_t ib = blockIdx.x;
  const int64_t L = (ib % 8) * (nphys / 8) + ib / 8;
  if (L >= nlogical) return;
  const int64_t ctile = L / nrow;
  const int rtile = int(L % nrow);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nkg = Kp / 16, nch = Kp / 32;
  const int64_t rb0 = int64_t(rtile) * 8 + wave * kRB;  // 16-row blocks

  floatx4 acc[kRB][kCBc];
#pragma unroll
  for (int r = 0; r < kRB; ++r)
#pragma unroll
    for (int c = 0; c < kCBc; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};

  // chunk ch = k-groups 2ch, 2ch+1 of the tile's 8 column blocks: 16 DMAs of 1 KB, 4 per wave
#define BA_FETCH_C(ch, buf)                                                                   \
  do {                                                                                        \
    _Pragma("unroll") for (int d_ = 0; d_ < 4; ++d_) {                                        \
      const int q_ = wave * 4 + d_; /* block q_/2, k-group q_%2 */                            \
      const int64_t blk_ = ctile * kCBc + (q_ >> 1);                                          \
      lds_dma16(X + (blk_ * nkg + 2 * (ch) + (q_ & 1)) * 64 + lane, sB + (buf) * CH + q_ * 64); \
    }                                                                                         \
  } while (0)

  BA_FETCH_C(0, 0);
  float4 a[kRB][2], an[kRB][2];
#pragma unroll
  for (int r = 0; r < kRB; ++r)
#pragma unroll
    for (int h = 0; h < 2; ++h) a[r][h] = A[((rb0 + r) * nkg + h) * 64 + lane];
  lds_dma_wait();
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    if (more) {
      BA_FETCH_C(ch + 1, buf ^ 1);
#pragma unroll
      for (int r = 0; r < kRB; ++r)
#pragma unroll
        for (int h = 0; h < 2; ++h) an[r][h] = A[((rb0 + r) * nkg + 2 * (ch + 1) + h) * 64 + lane];
    }
    const float4* sb = sB + buf * CH;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int c = 0; c < kCBc; ++c) {
        const float4 bv = lds_frag(sb, (c * 2 + h) * 64 + lane);
#pragma unroll
        for (int r = 0; r < kRB; ++r) {
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].x, bv.x, acc[r][c], 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].y, bv.y, acc[r][c], 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].z, bv.z, acc[r][c], 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].w, bv.w, acc[r][c], 0, 0, 0);
        }
      }
    }
    if (more) {
#pragma unroll
      for (int r = 0; r < kRB; ++r)
#pragma unroll
        for (int h = 0; h < 2; ++h) a[r][h] = an[r][h];
    }
    lds_dma_wait();
    __syncthreads();
  }
#undef BA_FETCH_C
  // rows 16 rb + 4 (lane/16) + e: (e, e+1) = (u, v) of one trial; column 16 c + lane%16
#pragma unroll
  for (int r = 0; r < kRB; ++r) {
    const int64_t row0 = (rb0 + r) * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int c = 0; c < kCBc; ++c) {
      const int64_t g = (ctile * kCBc + c) * 16 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int64_t b = row0 / 2 + q;
        if (b < B && g < G) {
          const float re = acc[r][c][2 * q], im = acc[r][c][2 * q + 1];
          P[b * G + g] = (re * re + im * im) * scale;
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_coh_table(const CohGeom& geo, const double* cand, int64_t G, int Kp, float* X, hipStream_t s) {
  const int64_t n = G * geo.J;
  hipLaunchKernelGGL(k_coh_table, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, geo, cand, G, Kp, X);
  return hipGetLastError();
}

// rows padded to whole 128-row tiles of the GEMM
int64_t coh_row_blocks(int B) { return int64_t((2 * B + 127) / 128) * 8; }

hipError_t launch_coh_rows(const float2* Z, int B, int JNz, int Kp, float* A, hipStream_t s) {
  const int64_t nrb = coh_row_blocks(B);
  const int64_t total = nrb * (Kp / 16) * 256;
  hipLaunchKernelGGL(k_coh_rows, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, Z, B, JNz, Kp, nrb, A);
  return hipGetLastError();
}

hipError_t launch_coh_gemm(const float* A, const float* X, float* P, int B, int64_t G, int64_t ctiles, int Kp,
                           float scale, hipStream_t s) {
  const int nrow = (2 * B + 127) / 128;
  const int64_t nlog = int64_t(nrow) * ctiles;
  const int64_t nphys = (nlog + 7) / 8 * 8;
  if (nphys > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = 2 * kCBc * 2 * 64 * sizeof(float4);
  hipLaunchKernelGGL(k_coh_gemm, dim3(unsigned(nphys)), dim3(256), lds, s, reinterpret_cast<const float4*>(A),
                     reinterpret_cast<const float4*>(X), P, B, G, Kp, nrow, nlog, scale);
  return hipGetLastError();
}

}  // namespace ba
