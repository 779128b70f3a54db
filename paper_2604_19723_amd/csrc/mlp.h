// Internal declarations of the proposal network.
#pragma once

#include "ba_internal.h"

namespace ba {

enum { kGemmPlain = 0, kGemmBias = 1, kGemmHidden = 2, kGemmGeluGrad = 3 };

// C[m][n] = sum_k A[m sam + k sak] B[k sbk + n sbn], then the epilogue of `mode`:
//   plain:     C = acc
//   bias:      C = acc + bias[n]
//   hidden:    Z = acc + bias[n];  C = gelu(Z)
//   gelu-grad: C = acc * gelu'(Z)   (Z read at the same [m][n])
struct GemmArgs {
  const float* A;
  const float* B;
  float* C;
  int M, N, K;
  int64_t sam, sak, sbk, sbn, ldc;
  int mode;
  const float* bias;
  float* Z;
};

hipError_t launch_gemm(const GemmArgs& g, int prec, hipStream_t s);
hipError_t launch_colsum(const float* dZ, float* db, int M, int N, hipStream_t s);
hipError_t launch_mse(const float* Y, const float* T, const float* mask, float* dY, float* loss, int n,
                      hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_pack(const float2* R, float* X, int M, int B, hipStream_t s);

}  // namespace ba
