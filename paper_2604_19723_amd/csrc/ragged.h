// Internal declarations of the ragged (uneven) batch path.
#pragma once

#include <cstdint>

#include "ba_internal.h"

namespace ba {

constexpr int kRaggedClasses = 5;      // padded element counts 8, 16, 32, 64, 128
constexpr int kRaggedMaxPeaks = 8;
constexpr int kRaggedMaxGrid = 16384;  // the spectrum row of one trial lives in LDS
constexpr int kRaggedLds = 152 * 1024;   // dynamic LDS of the persistent kernel
constexpr int kRaggedPackWaves = 8;      // packed trials per workgroup ticket (one per wave)
constexpr int kRaggedPackClasses = 3;    // classes that can run packed (up to 32 elements)

enum { kRouteCov = 0, kRouteSnap = 1 };

// One trial of the batch, in processing order (longest first).
struct RItem {
  int64_t y_off;  // complex offset of the [T][M] block in the pool
  int32_t trial;  // index of the trial in the caller's order (output row)
  int32_t M, T, K;
  int32_t cls;    // Mp = 8 << cls
  int32_t route;  // kRouteCov or kRouteSnap
};

struct RArgs {
  const RItem* items;      // whole-workgroup items first, then the packed ones
  int32_t n_items;
  int32_t n_wg_items;      // items taken one per ticket by a whole workgroup
  int32_t n_units;         // tickets: n_wg_items + ceil(packed / waves per workgroup)
  const float2* Y;
  const float4* X[kRaggedClasses];   // per-class steering tables (fragment order)
  int32_t nchunk[kRaggedClasses];    // 32 KB chunks per class table that hold grid points
  int32_t wr[kRaggedClasses];        // waves along rows per class (tuned)
  int64_t G;
  int32_t s1, rows, wrap0, ndim, kmax;
  float* P;         // [B][G] or null
  int32_t* idx;     // [B][kmax]
  float* val;       // [B][kmax]
  double* refined;  // [B][kmax][ndim] or null
  int32_t* counter;
};

// valid waves-along-rows choices per class
inline int ragged_wr_options(int cls, int* out) {
  switch (cls) {
    case 0: out[0] = 1; return 1;
    case 1: out[0] = 1; out[1] = 2; return 2;
    case 2: out[0] = 2; out[1] = 4; return 2;
    case 3: out[0] = 4; out[1] = 8; return 2;
    default: out[0] = 8; return 1;
  }
}

int ragged_blocks_per_chunk(int cls);
hipError_t ragged_prepare();
hipError_t launch_ragged(const RArgs* d_args, int n_wg, hipStream_t s);
hipError_t launch_ragged_reset(int32_t* counter, hipStream_t s);
// rewrite the buffer fields of the device-side arguments (stream-ordered)
hipError_t launch_ragged_bind(RArgs* d_args, const float2* Y, float* P, int32_t* idx, float* val, double* refined,
                              hipStream_t s);

}  // namespace ba
