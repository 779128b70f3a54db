// Residual covariance (Sec. IV-D.2): R~ = Pi R Pi with Pi = I - Psi Psi^+, the
// projector onto the complement of the span of the known steering vectors.
//
// One workgroup per trial, one thread per element row (M <= 256), all the
// small algebra in FP64 and R~ rounded to FP32 once at the end:
//   1. Psi [M][S] into LDS (given vectors, or columns of the plan's steering
//      table picked by grid index; index -1 gives a zero column);
//   2. Gram Gm = Psi^H Psi by wave reductions;
//   3. Cholesky Gm = L L^H on one thread; a column whose pivot (the squared
//      norm of its part orthogonal to the earlier kept columns) is at most
//      kRankEps times its squared norm is dependent and dropped;
//   4. orthonormal basis Q = Psi L^-H, each thread solving for its own row;
//   5. U = R Q, each thread its own row (R read by columns: R is Hermitian);
//   6. V = Q^H U by wave reductions, W = U - Q V;
//   7. R~ = R - Q U^H - W Q^H, which equals Pi R Pi for Pi = I - Q Q^H; the
//      upper triangle is evaluated and mirrored, so R~ is exactly Hermitian.
// Every element of R~[m][n] with m <= n is read from R and written by the
// same thread, and the lower triangle of R is only read before step 7, so R~
// may overwrite R.
#include <hip/hip_runtime.h>

#include "ba_internal.h"

namespace ba {
namespace {

constexpr double kRankEps = 1e-10;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int SMAX>
__global__ __launch_bounds__(256) void k_residual(const float2* __restrict__ R, int M, int S,
                                                  const float2* __restrict__ Psi, const int* __restrict__ gidx,
                                                  int ld, const float2* __restrict__ A, int64_t G,
                                                  float2* __restrict__ Rout) {
  extern __shared__ __attribute__((aligned(16))) double2 sm[];
  double2* sQ = sm;              // [SMAX][M]: Psi, then Q
  double2* sW = sm + SMAX * M;   // [SMAX][M]: U, then W
  __shared__ double2 sG[SMAX][SMAX];
  __shared__ double2 sL[SMAX][SMAX];
  __shared__ int keep[SMAX];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t b = blockIdx.x;
  const float2* Rb = R + b * int64_t(M) * M;
  float2* Ob = Rout + b * int64_t(M) * M;

  // 1. Psi
  for (int v = tid; v < SMAX * M; v += 256) {
    const int s = v / M, m = v - s * M;
    double2 z = make_double2(0.0, 0.0);
    if (s < S) {
      if (Psi) {
        const float2 f = Psi[(b * S + s) * M + m];
        z = make_double2(f.x, f.y);
      } else {
        const int g = gidx[b * ld + s];
        if (g >= 0 && g < G) {
          const float2 f = A[int64_t(m) * G + g];
          z = make_double2(f.x, f.y);
        }
      }
    }
    sQ[v] = z;
  }
  __syncthreads();

  // 2. Gram, upper triangle by waves, mirrored
  const int npairs = S * (S + 1) / 2;
  for (int e = wave; e < npairs; e += 4) {
    int i = 0, r = e;
    while (r >= S - i) {
      r -= S - i;
      ++i;
    }
    const int j = i + r;
    double re = 0.0, im = 0.0;
    for (int m = lane; m < M; m += 64) {
      const double2 c = cmulc(sQ[i * M + m], sQ[j * M + m]);
      re += c.x;
      im += c.y;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
      sG[i][j] = make_double2(re, im);
      sG[j][i] = make_double2(re, -im);
    }
  }
  __syncthreads();

  // 3. Cholesky with rank drop: Gm[i][j] = sum_k L[i][k] conj(L[j][k])
  if (tid == 0) {
    for (int i = 0; i < SMAX; ++i)
      for (int j = 0; j < SMAX; ++j) sL[i][j] = make_double2(0.0, 0.0);
    for (int j = 0; j < S; ++j) {
      double d = sG[j][j].x;
      for (int k = 0; k < j; ++k) d -= sL[j][k].x * sL[j][k].x + sL[j][k].y * sL[j][k].y;
      keep[j] = d > kRankEps * sG[j][j].x ? 1 : 0;
      if (!keep[j]) continue;  // column j of L stays zero
      const double ljj = sqrt(d);
      sL[j][j] = make_double2(ljj, 0.0);
      for (int i = j + 1; i < S; ++i) {
        double2 v = sG[i][j];
        for (int k = 0; k < j; ++k) v = csub(v, cmul(sL[i][k], make_double2(sL[j][k].x, -sL[j][k].y)));
        sL[i][j] = make_double2(v.x / ljj, v.y / ljj);
      }
    }
  }
  __syncthreads();

  // 4. own row of Q: q L^H = psi
  const int m = tid;
  const bool row = m < M;
  double2 q[SMAX], u[SMAX];
#pragma unroll
  for (int j = 0; j < SMAX; ++j) {
    q[j] = make_double2(0.0, 0.0);
    if (row && j < S && keep[j]) {
      double2 v = sQ[j * M + m];
#pragma unroll
      for (int k = 0; k < j; ++k) v = csub(v, cmul(q[k], make_double2(sL[j][k].x, -sL[j][k].y)));
      q[j] = make_double2(v.x / sL[j][j].x, v.y / sL[j][j].x);
    }
  }
  if (row) {
#pragma unroll
    for (int j = 0; j < SMAX; ++j) sQ[j * M + m] = q[j];
  }
  __syncthreads();

  // 5. own row of U = R Q; R[m][n] = conj(R[n][m]) read down column m
#pragma unroll
  for (int j = 0; j < SMAX; ++j) u[j] = make_double2(0.0, 0.0);
  if (row) {
    for (int n = 0; n < M; ++n) {
      const float2 f = Rb[int64_t(n) * M + m];
      const double2 r = make_double2(f.x, -f.y);
#pragma unroll
      for (int j = 0; j < SMAX; ++j) u[j] = cadd(u[j], cmul(r, sQ[j * M + n]));
    }
#pragma unroll
    for (int j = 0; j < SMAX; ++j) sW[j * M + m] = u[j];
  }
  __syncthreads();

  // 6. V = Q^H U (S x S) by waves, then W = U - Q V
  for (int e = wave; e < S * S; e += 4) {
    const int i = e / S, j = e - i * S;
    double re = 0.0, im = 0.0;
    for (int mm = lane; mm < M; mm += 64) {
      const double2 c = cmulc(sQ[i * M + mm], sW[j * M + mm]);
      re += c.x;
      im += c.y;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) sG[i][j] = make_double2(re, im);
  }
  __syncthreads();
  double2 w[SMAX];
#pragma unroll
  for (int j = 0; j < SMAX; ++j) {
    w[j] = u[j];
#pragma unroll
    for (int k = 0; k < SMAX; ++k)
      if (k < S && j < S) w[j] = csub(w[j], cmul(q[k], sG[k][j]));
  }
  __syncthreads();  // U no longer read from LDS
  if (row) {
#pragma unroll
    for (int j = 0; j < SMAX; ++j) sW[j * M + m] = w[j];
  }
  __syncthreads();

  // 7. column n = tid: R~[i][n] = R[i][n] - Q[i] U[n]^H - W[i] Q[n]^H for i <= n
  if (row) {
    const int n = m;
    for (int i = 0; i <= n; ++i) {
      const float2 f = Rb[int64_t(i) * M + n];
      double2 v = make_double2(f.x, f.y);
#pragma unroll
      for (int j = 0; j < SMAX; ++j) {
        v = csub(v, cmul(sQ[j * M + i], make_double2(u[j].x, -u[j].y)));
        v = csub(v, cmul(sW[j * M + i], make_double2(q[j].x, -q[j].y)));
      }
      if (i == n) v.y = 0.0;
      Ob[int64_t(i) * M + n] = make_float2(float(v.x), float(v.y));
      if (i < n) Ob[int64_t(n) * M + i] = make_float2(float(v.x), float(-v.y));
    }
  }
}

// one thread per trial: copy a single-peak result into column c of [B][K]
__global__ void k_put_column(int B, int c, int K, int ndim, const int* __restrict__ i1, const float* __restrict__ v1,
                             const double* __restrict__ r1, int* __restrict__ idx, float* __restrict__ val,
                             double* __restrict__ ref) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  idx[int64_t(b) * K + c] = i1[b];
  val[int64_t(b) * K + c] = v1[b];
  if (ref)
    for (int d = 0; d < ndim; ++d) ref[(int64_t(b) * K + c) * ndim + d] = r1[int64_t(b) * ndim + d];
}

template <int SMAX>
hipError_t launch_res(int B, const float2* R, int M, int S, const float2* Psi, const int* gidx, int ld,
                      const float2* A, int64_t G, float2* Rout, hipStream_t s) {
  const size_t lds = size_t(2) * SMAX * M * sizeof(double2);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_residual<SMAX>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual<SMAX>, dim3(unsigned(B)), dim3(256), lds, s, R, M, S, Psi, gidx, ld, A, G, Rout);
  return hipGetLastError();
}

}  // namespace

size_t residual_lds_bytes(int M, int S) {
  const int smax = S <= 4 ? 4 : S <= 8 ? 8 : 16;
  return size_t(2) * smax * M * sizeof(double2);
}

hipError_t launch_residual(const Plan& p, int B, const float2* R, int S, const float2* Psi, const int* gidx,
                           int ld, float2* Rout, hipStream_t s) {
  if (B == 0) return hipSuccess;
  if (p.M > 256 || S < 0 || S > 16) return hipErrorInvalidValue;
  if (S <= 4) return launch_res<4>(B, R, p.M, S, Psi, gidx, ld, p.d_A, p.G, Rout, s);
  if (S <= 8) return launch_res<8>(B, R, p.M, S, Psi, gidx, ld, p.d_A, p.G, Rout, s);
  return launch_res<16>(B, R, p.M, S, Psi, gidx, ld, p.d_A, p.G, Rout, s);
}

hipError_t launch_put_column(int B, int c, int K, int ndim, const int* i1, const float* v1, const double* r1,
                             int* idx, float* val, double* ref, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_put_column, dim3(unsigned((B + 255) / 256)), dim3(256), 0, s, B, c, K, ndim, i1, v1, r1,
                     idx, val, ref);
  return hipGetLastError();
}

}  // namespace ba
