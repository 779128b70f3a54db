// Shared device pieces of the register-resident MFMA projection (Q in
// registers, steering blocks in B-fragment order); see k_proj_mfma.hip.
#pragma once

#include "ba_internal.h"

namespace ba {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Register-resident projection in its symmetric form. Q is symmetric, so
//   x^T Q x = 2 x^T U x,  U = the upper triangle of Q with its diagonal halved,
// and the 16-row block rb of U is zero left of its diagonal block: it needs
// only the k-steps s >= 4 rb. Each wave takes the pair of row blocks
// (p, RBLK - 1 - p), whose k ranges together always span KS + 4 steps, so the
// waves carry equal work and about half the MFMAs of the full Q x.
template <int MP>
struct QCfg {
  static constexpr int K = 2 * MP;                 // GEMM depth = rows of Q
  static constexpr int KS = K / 4;                 // MFMA k-steps
  static constexpr int RBLK = K / 16;              // 16-row blocks of Q
  static constexpr bool PAIRS = RBLK >= 2;         // a single block (MP = 8) has no partner
  static constexpr int WR = PAIRS ? RBLK / 2 : 1;  // waves along rows, one pair each
  static constexpr int WC = 4 / WR;                // waves along columns
  static constexpr int VL = PAIRS ? KS + 4 : KS;   // A-fragment registers per wave
  // steering chunks of 8 KB (one 16-column block at M = 64): with the small
  // register footprint of the symmetric form, short chunks let six
  // workgroups share a CU and hide each other's barrier and DMA waits
  static constexpr int BLK = K * 16;               // floats per 16-column block
  static constexpr int NB = 2048 / BLK;            // blocks per chunk
  static constexpr int CH4 = 2048 / 4;             // float4 per chunk
  static_assert(WR >= 1 && WR <= 4, "at most four row waves");
};

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

// U(i, k) for the symmetric form: Q(i, k) right of the diagonal, half the
// diagonal, zero left of it
__device__ __forceinline__ float uval(const float2* __restrict__ Rb, int M, int MP, int i, int k) {
  if (k < i) return 0.f;
  const float q = qval(Rb, M, MP, i, k);
  return k == i ? 0.5f * q : q;
}

// A operand of wave wr's row-block pair, in its virtual step order: steps
// v < KS - 4 wr hold row block wr at k-step 4 wr + v; the 4 (wr + 1) steps
// after them hold row block RBLK - 1 - wr at k-step v - 4. Row i = 16 rb +
// lane % 16, k = 4 s + lane / 16.
template <int MP>
__device__ __forceinline__ void load_q_fragments(const float2* __restrict__ Rb, int M, int wr, int lane,
                                                 float (&a)[QCfg<MP>::VL]) {
  using C = QCfg<MP>;
  const int nlo = C::KS - 4 * wr;
#pragma unroll
  for (int v = 0; v < C::VL; ++v) {
    const bool lo = v < nlo;
    const int rb = lo ? wr : C::RBLK - 1 - wr;
    const int s = lo ? 4 * wr + v : v - 4;
    a[v] = uval(Rb, M, MP, rb * 16 + (lane & 15), 4 * s + (lane >> 4));
  }
}

// x_i (U x)_i summed over the 16 rows of row block RB and the four values each
// lane holds of it
template <int RB>
__device__ __forceinline__ float row_block_dot(const floatx4& acc, const float* __restrict__ xf, int lane) {
  float part = 0.f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = RB * 16 + 4 * (lane >> 4) + r;
    const int s = i >> 2;
    part += xf[((s >> 2) * 64 + r * 16 + (lane & 15)) * 4 + (s & 3)] * acc[r];
  }
  return part;
}

template <int MP, int PP>
__device__ __forceinline__ float pair_quadratic(const float (&a)[QCfg<MP>::VL], const float4* __restrict__ bx,
                                                const float* __restrict__ xf, int lane) {
  using C = QCfg<MP>;
  constexpr int LO = PP, HI = C::RBLK - 1 - PP;  // HI >= LO; equal only without pairs
  constexpr int NLO = C::KS - 4 * LO;
  floatx4 alo = floatx4{0.f, 0.f, 0.f, 0.f}, ahi = alo;
#pragma unroll
  for (int s4 = LO; s4 < C::RBLK; ++s4) {
    const float4 bv = bx[s4 * 64 + lane];
    const int vl = 4 * (s4 - LO);
    alo = __builtin_amdgcn_mfma_f32_16x16x4f32(a[vl + 0], bv.x, alo, 0, 0, 0);
    alo = __builtin_amdgcn_mfma_f32_16x16x4f32(a[vl + 1], bv.y, alo, 0, 0, 0);
    alo = __builtin_amdgcn_mfma_f32_16x16x4f32(a[vl + 2], bv.z, alo, 0, 0, 0);
    alo = __builtin_amdgcn_mfma_f32_16x16x4f32(a[vl + 3], bv.w, alo, 0, 0, 0);
    if (C::PAIRS && s4 >= HI) {
      const int vh = NLO + 4 * (s4 - HI);
      ahi = __builtin_amdgcn_mfma_f32_16x16x4f32(a[vh + 0], bv.x, ahi, 0, 0, 0);
      ahi = __builtin_amdgcn_mfma_f32_16x16x4f32(a[vh + 1], bv.y, ahi, 0, 0, 0);
      ahi = __builtin_amdgcn_mfma_f32_16x16x4f32(a[vh + 2], bv.z, ahi, 0, 0, 0);
      ahi = __builtin_amdgcn_mfma_f32_16x16x4f32(a[vh + 3], bv.w, ahi, 0, 0, 0);
    }
  }
  float part = row_block_dot<LO>(alo, xf, lane);
  if (C::PAIRS) part += row_block_dot<HI>(ahi, xf, lane);
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  return part;
}

// One 16-column block: returns, in lanes 0..15, this wave's partial sum
// x^T U x over its row-block pair for the block's columns (half the wave's
// share of the spectrum value times M^2).
template <int MP>
__device__ __forceinline__ float block_quadratic(const float (&a)[QCfg<MP>::VL], const float4* __restrict__ bx,
                                                 const float* __restrict__ xf, int wr, int lane) {
  using C = QCfg<MP>;
  if constexpr (C::WR == 1) {
    return pair_quadratic<MP, 0>(a, bx, xf, lane);
  } else if constexpr (C::WR == 2) {
    return wr == 0 ? pair_quadratic<MP, 0>(a, bx, xf, lane) : pair_quadratic<MP, 1>(a, bx, xf, lane);
  } else {
    switch (wr) {
      case 0: return pair_quadratic<MP, 0>(a, bx, xf, lane);
      case 1: return pair_quadratic<MP, 1>(a, bx, xf, lane);
      case 2: return pair_quadratic<MP, 2>(a, bx, xf, lane);
      default: return pair_quadratic<MP, 3>(a, bx, xf, lane);
    }
  }
}

}  // namespace ba
