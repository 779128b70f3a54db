// Gaussian birth proposal (Sec. IV-D.2): particles drawn from N(mu, C) built
// from the Bartlett moments, with importance weights proportional to the
// indicator of the search region over the proposal density (a target that is
// uniform on the region), normalised per trial.
//
// One workgroup per trial, FP64 throughout. With C = L L^T and a particle
// p = mu + L z, the proposal density is exp(-|z|^2 / 2) / ((2 pi)^(d/2) det L);
// det L and the constant are common to every particle of a trial and cancel in
// the normalisation, so the unnormalised log-weight is |z|^2 / 2 inside the
// region and -inf outside. A periodic coordinate (azimuth) is always inside
// and is reported wrapped into [lo, lo + period); its density is the Gaussian
// at the unwrapped draw. A covariance that is not positive definite gives a
// degenerate proposal: every particle is mu with equal weights. A trial
// without a particle inside the region gets NaN weights.
#include <hip/hip_runtime.h>

#include "ba_internal.h"

namespace ba {
namespace {

__device__ double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__device__ double block_add(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_proposal_sample(const double* __restrict__ mu_cov, int d, int N,
                                                         const double* __restrict__ z, ProposalRegion reg,
                                                         double* __restrict__ part, double* __restrict__ w) {
  __shared__ double red[4];
  const int64_t b = blockIdx.x;
  const double* mc = mu_cov + b * (d + d * d);
  double mu[3] = {0.0, 0.0, 0.0}, L[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int a = 0; a < d; ++a) mu[a] = mc[a];
  // Cholesky of C (d <= 3); any non-positive or non-finite pivot: degenerate
  bool pd = true;
  for (int j = 0; j < d && pd; ++j) {
    double s = mc[d + j * d + j];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    if (!(s > 0.0) || !isfinite(s)) {
      pd = false;
      break;
    }
    L[j][j] = sqrt(s);
    for (int i = j + 1; i < d; ++i) {
      double t = mc[d + i * d + j];
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  const double* zb = z + b * int64_t(N) * d;
  double* pb = part + b * int64_t(N) * d;
  double* wb = w + b * int64_t(N);
  if (!pd) {
    for (int n = threadIdx.x; n < N; n += 256) {
      for (int a = 0; a < d; ++a) pb[int64_t(n) * d + a] = mu[a];
      wb[n] = 1.0 / double(N);
    }
    return;
  }
  double lmax = -INFINITY;
  for (int n = threadIdx.x; n < N; n += 256) {
    double zz[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) zz[a] = zb[int64_t(n) * d + a];
    bool inside = true;
    double q = 0.0;
    for (int i = 0; i < d; ++i) {
      double p = mu[i];
      for (int k = 0; k <= i; ++k) p += L[i][k] * zz[k];
      q += zz[i] * zz[i];
      if (reg.period[i] > 0.0) {
        double r = fmod(p - reg.lo[i], reg.period[i]);
        if (r < 0.0) r += reg.period[i];
        p = reg.lo[i] + r;
      } else if (!(p >= reg.lo[i] && p <= reg.hi[i])) {
        inside = false;
      }
      pb[int64_t(n) * d + i] = p;
    }
    const double lw = inside ? 0.5 * q : -INFINITY;
    wb[n] = lw;  // unnormalised log-weight, rewritten below by the same thread
    lmax = fmax(lmax, lw);
  }
  lmax = block_max(lmax, red);
  double s = 0.0;
  if (lmax > -INFINITY)
    for (int n = threadIdx.x; n < N; n += 256) s += exp(wb[n] - lmax);
  s = block_add(s, red);
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  for (int n = threadIdx.x; n < N; n += 256) wb[n] = lmax > -INFINITY ? exp(wb[n] - lmax) / s : nan;
}

}  // namespace

hipError_t launch_proposal_sample(int B, const double* mu_cov, int d, int N, const double* z,
                                  const ProposalRegion& reg, double* particles, double* weights, hipStream_t s) {
  if (B == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_proposal_sample, dim3(unsigned(B)), dim3(256), 0, s, mu_cov, d, N, z, reg, particles,
                     weights);
  return hipGetLastError();
}

}  // namespace ba
