// Shared device pieces of the register-resident MFMA projection (Q in
// registers, steering blocks in B-fragment order); see k_proj_mfma.hip.
#pragma once

#include "ba_internal.h"

namespace ba {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int MP, int WRO = 0>
struct QCfg {
  static constexpr int K = 2 * MP;                 // GEMM depth = rows of Q
  static constexpr int KS = K / 4;                 // MFMA k-steps
  static constexpr int RBLK = K / 16;              // 16-row blocks of Q
  // waves along rows (WRO > 0 overrides the default split)
  static constexpr int WR = WRO > 0 ? WRO : (RBLK >= 8 ? 4 : (RBLK >= 4 ? 2 : 1));
  static constexpr int RB = RBLK / WR;             // row blocks per wave
  static constexpr int WC = 4 / WR;                // waves along columns
  static constexpr int BLK = K * 16;               // floats per 16-column block
  static constexpr int NB = 8192 / BLK;            // blocks per 32 KB chunk
  static constexpr int CH4 = 8192 / 4;             // float4 per chunk
  static constexpr int F4 = CH4 / 256;             // float4 per thread per chunk
};

// Row split of the register-resident projection at each padded size: for
// MP = 64 two waves along rows (four row blocks each, the 16-column blocks
// shared out between the two wave pairs) halves the B-fragment LDS reads and
// gives each wave four independent accumulators. The full-grid kernel and the
// refinement-window kernel use the same split, so window values equal the
// full-grid values bit for bit.
template <int MP>
constexpr int kProjWR = MP == 64 ? 2 : 0;

// Direct global -> LDS copy of 16 bytes per lane (global_load_lds_dwordx4):
// lane i's word lands at lds_wave + 16 i. lds_wave must be wave-uniform and
// point into dynamic shared memory. Completion is tracked by vmcnt; callers
// wait with lds_dma_wait() before the barrier that publishes the data.
__device__ __forceinline__ void lds_dma16(const void* gsrc_lane, void* lds_wave) {
  __builtin_amdgcn_global_load_lds(gsrc_lane, reinterpret_cast<__attribute__((address_space(3))) void*>(
                                                  reinterpret_cast<uintptr_t>(lds_wave)),
                                   16, 0, 0);
}

__device__ __forceinline__ void lds_dma_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0) */ }

// Read of a fragment from an LDS chunk that an earlier lds_dma_wait() and
// barrier have published. The restrict-qualified base gives the load alias
// scope information; without it the compiler cannot tell the chunk being
// read from the chunk still in flight and waits for every outstanding LDS
// DMA before the read, which serialises the prefetch with the MFMAs.
template <typename T>
__device__ __forceinline__ T lds_frag(const T* __restrict__ base, int i) {
  return base[i];
}

// Q = [[Rr, -Ri], [Ri, Rr]] element (i, k) for an element count padded to MP
__device__ __forceinline__ float qval(const float2* __restrict__ Rb, int M, int MP, int i, int k) {
  const bool iim = i >= MP, kim = k >= MP;
  const int ir = iim ? i - MP : i, kr = kim ? k - MP : k;
  if (ir >= M || kr >= M) return 0.f;
  const float2 r = Rb[ir * M + kr];
  return (iim == kim) ? r.x : (iim ? r.y : -r.y);
}

// A operand of the waves' rows: rows i = wr*RB*16 + rb*16 + lane%16, k = 4s + lane/16
template <int MP, int WRO = 0>
__device__ __forceinline__ void load_q_fragments(const float2* __restrict__ Rb, int M, int wr, int lane,
                                                 float (&a)[QCfg<MP, WRO>::RB][QCfg<MP, WRO>::KS]) {
  using C = QCfg<MP, WRO>;
#pragma unroll
  for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
    for (int s = 0; s < C::KS; ++s)
      a[rb][s] = qval(Rb, M, MP, wr * C::RB * 16 + rb * 16 + (lane & 15), 4 * s + (lane >> 4));
}

// One 16-column block: returns, in lanes 0..15, this wave's partial
// sum over its rows of x_g[i] (Q x_g)[i] for the block's columns.
template <int MP, int WRO = 0>
__device__ __forceinline__ float block_quadratic(const float (&a)[QCfg<MP, WRO>::RB][QCfg<MP, WRO>::KS],
                                                 const float4* __restrict__ bx, const float* __restrict__ xf,
                                                 int wr, int lane) {
  using C = QCfg<MP, WRO>;
  floatx4 acc[C::RB];
#pragma unroll
  for (int rb = 0; rb < C::RB; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s4 = 0; s4 < C::KS / 4; ++s4) {
    const float4 bv = bx[s4 * 64 + lane];
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb) {
      acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 0], bv.x, acc[rb], 0, 0, 0);
      acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 1], bv.y, acc[rb], 0, 0, 0);
      acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 2], bv.z, acc[rb], 0, 0, 0);
      acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 3], bv.w, acc[rb], 0, 0, 0);
    }
  }
  float part = 0.f;
#pragma unroll
  for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = wr * C::RB * 16 + rb * 16 + 4 * (lane >> 4) + r;
      const int s = i >> 2;
      part += xf[((s >> 2) * 64 + r * 16 + (lane & 15)) * 4 + (s & 3)] * acc[rb][r];
    }
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  return part;
}

}  // namespace ba
