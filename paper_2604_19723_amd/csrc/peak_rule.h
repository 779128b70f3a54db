// The peak rule shared by the full-spectrum pick (k_peaks) and the candidates
// the projection epilogue gathers per column range: order of candidates and
// the parabolic vertex of a maximum (Sec. IV-D.2: the candidate of largest
// cost is the estimate; refinement between grid points is this build's).
#pragma once

#include <hip/hip_runtime.h>

namespace ba {

// Strict total order on (value, grid index): larger value first, ties to the
// lower index. Every comparison with NaN is false, so a NaN never wins.
__device__ __forceinline__ bool peak_better(float va, int ia, float vb, int ib) {
  return va > vb || (va == vb && ia < ib);
}

// Vertex offset of the parabola through (-1, pm), (0, p0), (1, pp), clipped to
// half a grid step; 0 when the three points are collinear or not finite.
__device__ __forceinline__ double peak_parabolic(double pm, double p0, double pp) {
#pragma clang fp contract(off)
  const double den = pm - 2.0 * p0 + pp;
  if (den == 0.0 || !isfinite(den)) return 0.0;
  const double d = 0.5 * (pm - pp) / den;
  return d > 0.5 ? 0.5 : (d < -0.5 ? -0.5 : d);
}

}  // namespace ba
