// Internal declarations of the coherent multi-array cost (SFV candidates).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ba {

// geometry of one plan, in device memory (FP64)
struct CohGeom {
  int J, nf, ny, nz;
  double fc;
  const double* pa;    // [J][3] array positions (m)
  const double* rot;   // [J][3][3] array rotations, row-major (local -> global)
  const double* mt;    // [3] terminal position (m)
  const double* freq;  // [nf] baseband frequencies (Hz)
  const double* py;    // [ny] horizontal element positions (m)
  const double* pz;    // [nz] vertical element positions (m)
};

hipError_t launch_coh_table(const CohGeom& geo, const double* cand, int64_t G, int Kp, float* X, hipStream_t s);
int64_t coh_row_blocks(int B);
hipError_t launch_coh_rows(const float2* Z, int B, int JNz, int Kp, float* A, hipStream_t s);
hipError_t launch_coh_gemm(const float* A, const float* X, float* P, int B, int64_t G, int64_t ctiles, int Kp,
                           float scale, hipStream_t s);
size_t point_moments_ws_bytes(int B, int64_t G);
hipError_t launch_point_moments(int B, const float* P, int64_t G, const double* X, double* mu_cov, void* ws,
                                hipStream_t s);

}  // namespace ba
