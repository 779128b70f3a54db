// Sample covariance R = (1/T) sum_t y_t y_t^H per trial (the R of the Bartlett
// cost in its covariance form, Sec. IV-D.2 read for T snapshots).
//
// One workgroup computes a 32x32 tile of R for one trial from the upper
// triangle of tile pairs (mt <= nt). Snapshot blocks of 32 x 32 complex values
// are staged in LDS with coalesced loads (each snapshot is a contiguous
// M-vector in HBM) and accumulated in FP32. The lower triangle is written as
// the conjugate of the upper one, so R is exactly Hermitian with a real
// diagonal.
#include "ba_internal.h"

namespace ba {
namespace {

constexpr int kTile = 32;   // output tile edge
constexpr int kChunk = 32;  // snapshots per LDS stage

__global__ __launch_bounds__(256) void k_cov_tiles(const float2* __restrict__ Y,
                                                   float2* __restrict__ R, int M, int T,
                                                   int ntile, int npairs) {
  const int64_t b = blockIdx.x / npairs;
  int rem = blockIdx.x % npairs;
  int mt = 0;
  while (rem >= ntile - mt) {
    rem -= ntile - mt;
    ++mt;
  }
  const int nt = mt + rem;
  const float2* Yb = Y + b * int64_t(T) * M;

  __shared__ float2 sm[kChunk][kTile + 1];
  __shared__ float2 sn[kChunk][kTile + 1];
  const int tx = threadIdx.x & 31;
  const int ty = threadIdx.x >> 5;  // 0..7
  float accr[4] = {0.f, 0.f, 0.f, 0.f};
  float acci[4] = {0.f, 0.f, 0.f, 0.f};

  for (int t0 = 0; t0 < T; t0 += kChunk) {
    for (int i = threadIdx.x; i < kChunk * kTile; i += 256) {
      const int tt = i / kTile, mm = i % kTile;
      const int t = t0 + tt;
      const int gm = mt * kTile + mm, gn = nt * kTile + mm;
      const bool tok = t < T;
      sm[tt][mm] = (tok && gm < M) ? Yb[int64_t(t) * M + gm] : make_float2(0.f, 0.f);
      sn[tt][mm] = (tok && gn < M) ? Yb[int64_t(t) * M + gn] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll 8
    for (int tt = 0; tt < kChunk; ++tt) {
      const float2 yn = sn[tt][tx];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float2 ym = sm[tt][ty + 8 * i];
        // ym * conj(yn)
        accr[i] += ym.x * yn.x + ym.y * yn.y;
        acci[i] += ym.y * yn.x - ym.x * yn.y;
      }
    }
    __syncthreads();
  }

  const float invT = 1.0f / float(T);
  float2* Rb = R + b * int64_t(M) * M;
  const int n = nt * kTile + tx;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = mt * kTile + ty + 8 * i;
    if (m < M && n < M && m <= n) {
      const float re = accr[i] * invT;
      const float im = (m == n) ? 0.f : acci[i] * invT;
      Rb[int64_t(m) * M + n] = make_float2(re, im);
      Rb[int64_t(n) * M + m] = make_float2(re, -im);
    }
  }
}

}  // namespace

hipError_t launch_covariance(const Plan& p, int B, int T, const float2* Y, float2* R,
                             hipStream_t s) {
  const int ntile = (p.M + kTile - 1) / kTile;
  const int npairs = ntile * (ntile + 1) / 2;
  const int64_t nblk = int64_t(B) * npairs;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cov_tiles, dim3(unsigned(nblk)), dim3(256), 0, s, Y, R, p.M, T, ntile, npairs);
  return hipGetLastError();
}

}  // namespace ba
