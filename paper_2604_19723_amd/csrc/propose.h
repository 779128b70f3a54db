// Internal declarations of the learned-proposal refinement.
#pragma once

#include "ba_internal.h"

namespace ba {

constexpr int kMaxProp = 8;         // proposals (peaks) per trial
constexpr int kMaxWinBlocks = 16;   // 16-column blocks covering one window (half width <= 100)
constexpr int kMaxHalfWindow = 100;

struct WindowArgs {
  const float2* R;      // [B][M][M]
  const float4* X;      // plan steering table, fragment order
  const float* U;       // [B][dout] network outputs (sin of the direction)
  int M;
  int64_t G;
  int dout, K, hw;
  double theta0, step;  // uniform angle grid, degrees
  float tau;
  int* idx;
  float* val;
  double* refined;
  unsigned char* fell;
  int* fb_list;
  int* fb_count;
};

// 16-column blocks one window of half width hw can touch
__host__ __device__ inline int window_blocks(int hw) { return (2 * hw) / 16 + 2; }
size_t window_lds_bytes(int Mp, int hw);
hipError_t launch_window(const WindowArgs& a, int Mp, int B, hipStream_t s);
hipError_t launch_zero_count(int* count, hipStream_t s);
// n: the most trials the list can hold; *count (on the device) of them are used
hipError_t launch_gather_r(const int* list, const int* count, int n, const float2* R, float2* Rc, int M,
                           hipStream_t s);
hipError_t launch_scatter(const int* list, const int* count, int n, int K, const int* idx_c, const float* val_c,
                          const double* ref_c, int* idx, float* val, double* ref, hipStream_t s);

}  // namespace ba
