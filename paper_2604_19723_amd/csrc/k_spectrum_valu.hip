// Bartlett spectrum on the vector ALUs (reference path of the library; the
// MFMA projection replaces it for the covariance route at scale).
//
//   covariance route: P[g] = Re(a_g^H R a_g) / M^2
//   snapshot route:   P[g] = (1/T) sum_t |a_g^H y_t|^2 / M^2
//
// One workgroup takes a tile of GT grid points of one trial. The steering
// tile A[:, g0:g0+GT] is staged in LDS; each wave owns a residue class of rows
// (or snapshots) so the R row (or the snapshot) it reads is wave-uniform and
// comes through the scalar cache. Partial sums of the waves meet in LDS.
#include "ba_internal.h"

namespace ba {
namespace {

template <int GT>
__global__ __launch_bounds__(256) void k_spec_cov_valu(const float2* __restrict__ R,
                                                       const float2* __restrict__ A,
                                                       float* __restrict__ P, int M, int64_t G,
                                                       int ntile) {
  constexpr int RG = 256 / GT;
  extern __shared__ float2 sA[];  // [M][GT]
  __shared__ float part[RG][GT];
  const int64_t b = blockIdx.x / ntile;
  const int64_t g0 = int64_t(blockIdx.x % ntile) * GT;
  const int gl = threadIdx.x % GT;
  // with GT >= 64 the row group is wave-uniform, so its loads go through the scalar cache
  const int rg = GT >= 64 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x / GT)) : int(threadIdx.x / GT);
  for (int i = threadIdx.x; i < M * GT; i += 256) {
    const int n = i / GT, c = i % GT;
    const int64_t g = g0 + c;
    sA[i] = g < G ? A[int64_t(n) * G + g] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const float2* Rb = R + b * int64_t(M) * M;
  float acc = 0.f;
  for (int m = rg; m < M; m += RG) {
    float cr = 0.f, ci = 0.f;
    const float2* Rm = Rb + int64_t(m) * M;
    for (int n = 0; n < M; ++n) {
      const float2 r = Rm[n];
      const float2 a = sA[n * GT + gl];
      cr += r.x * a.x - r.y * a.y;
      ci += r.x * a.y + r.y * a.x;
    }
    const float2 am = sA[m * GT + gl];
    acc += am.x * cr + am.y * ci;  // Re(conj(a_m) c_m)
  }
  part[rg][gl] = acc;
  __syncthreads();
  if (threadIdx.x < GT) {
    const int64_t g = g0 + gl;
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < RG; ++r) s += part[r][gl];
    if (g < G) P[b * G + g] = s / float(M * M);
  }
}

template <int GT>
__global__ __launch_bounds__(256) void k_spec_snap_valu(const float2* __restrict__ Y,
                                                        const float2* __restrict__ A,
                                                        float* __restrict__ P, int M, int T,
                                                        int64_t G, int ntile) {
  constexpr int RG = 256 / GT;
  extern __shared__ float2 sA[];  // [M][GT]
  __shared__ float part[RG][GT];
  const int64_t b = blockIdx.x / ntile;
  const int64_t g0 = int64_t(blockIdx.x % ntile) * GT;
  const int gl = threadIdx.x % GT;
  // with GT >= 64 the row group is wave-uniform, so its loads go through the scalar cache
  const int rg = GT >= 64 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x / GT)) : int(threadIdx.x / GT);
  for (int i = threadIdx.x; i < M * GT; i += 256) {
    const int n = i / GT, c = i % GT;
    const int64_t g = g0 + c;
    sA[i] = g < G ? A[int64_t(n) * G + g] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const float2* Yb = Y + b * int64_t(T) * M;
  float acc = 0.f;
  for (int t = rg; t < T; t += RG) {
    const float2* yt = Yb + int64_t(t) * M;
    float zr = 0.f, zi = 0.f;
    for (int m = 0; m < M; ++m) {
      const float2 y = yt[m];
      const float2 a = sA[m * GT + gl];
      // conj(a) * y
      zr += a.x * y.x + a.y * y.y;
      zi += a.x * y.y - a.y * y.x;
    }
    acc += zr * zr + zi * zi;
  }
  part[rg][gl] = acc;
  __syncthreads();
  if (threadIdx.x < GT) {
    const int64_t g = g0 + gl;
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < RG; ++r) s += part[r][gl];
    if (g < G) P[b * G + g] = s / float(T) / float(M * M);
  }
}

}  // namespace

hipError_t launch_spectrum_valu(const Plan& p, int B, const float2* R, float* P, hipStream_t s) {
  const int GT = p.M <= 128 ? 64 : 32;
  const int ntile = int((p.G + GT - 1) / GT);
  const int64_t nblk = int64_t(B) * ntile;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = size_t(p.M) * GT * sizeof(float2);
  if (GT == 32)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_spec_cov_valu<32>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (GT == 64)
    hipLaunchKernelGGL(k_spec_cov_valu<64>, dim3(unsigned(nblk)), dim3(256), lds, s, R, p.d_A, P,
                       p.M, p.G, ntile);
  else
    hipLaunchKernelGGL(k_spec_cov_valu<32>, dim3(unsigned(nblk)), dim3(256), lds, s, R, p.d_A, P,
                       p.M, p.G, ntile);
  return hipGetLastError();
}

hipError_t launch_spectrum_snapshots(const Plan& p, int B, int T, const float2* Y, float* P,
                                     hipStream_t s) {
  const int GT = p.M <= 128 ? 64 : 32;
  const int ntile = int((p.G + GT - 1) / GT);
  const int64_t nblk = int64_t(B) * ntile;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = size_t(p.M) * GT * sizeof(float2);
  if (GT == 32)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_spec_snap_valu<32>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (GT == 64)
    hipLaunchKernelGGL(k_spec_snap_valu<64>, dim3(unsigned(nblk)), dim3(256), lds, s, Y, p.d_A, P,
                       p.M, T, p.G, ntile);
  else
    hipLaunchKernelGGL(k_spec_snap_valu<32>, dim3(unsigned(nblk)), dim3(256), lds, s, Y, p.d_A, P,
                       p.M, T, p.G, ntile);
  return hipGetLastError();
}

}  // namespace ba
