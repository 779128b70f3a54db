// Bartlett spectrum as one real GEMM on the matrix cores, with the quadratic
// form fused into the epilogue.
//
// For a steering vector a = ar + j ai and a Hermitian R = Rr + j Ri,
//   Re(a^H R a) = x^T Q x,   x = [ar; ai],   Q = [[Rr, -Ri], [Ri, Rr]]  (2M x 2M, symmetric),
// so the spectrum of one trial over the grid is P_g = sum_k X[k][g] (Q X)[k][g] / M^2
// with X the 2M x G real-equivalent steering table: a GEMM with K = 2M whose
// output never leaves the registers (Sec. IV-D.2 cost, written as a dense
// contraction over the candidate set).
//
// MI355X mapping (v_mfma_f32_16x16x4f32, FP32 in and out):
//  * one workgroup = one trial x a range of grid columns; 4 waves;
//  * Q is built from R once per workgroup straight into MFMA A-operand
//    registers (each wave owns RB row blocks of 16 rows, all K);
//  * the steering table is stored in HBM already in B-fragment order (16
//    columns per block, 4 k-steps per lane per 16-byte word), so one chunk of
//    32 KB is a straight coalesced copy into LDS and every fragment read is a
//    conflict-free ds_read_b128; chunks are double-buffered through registers;
//  * epilogue: the accumulator tile is multiplied by the matching rows of the
//    same LDS tile, reduced across the 4 row-groups of a wave by two lane
//    shuffles and across waves through LDS, then scaled by 1/M^2.
// Element counts up to 64 are padded to MP in {8, 16, 32, 64} with zero rows.
#include "ba_internal.h"

namespace ba {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int MP>
struct QCfg {
  static constexpr int K = 2 * MP;                 // GEMM depth = rows of Q
  static constexpr int KS = K / 4;                 // MFMA k-steps
  static constexpr int RBLK = K / 16;              // 16-row blocks of Q
  static constexpr int WR = RBLK >= 8 ? 4 : (RBLK >= 4 ? 2 : 1);  // waves along rows
  static constexpr int RB = RBLK / WR;             // row blocks per wave
  static constexpr int WC = 4 / WR;                // waves along columns
  static constexpr int BLK = K * 16;               // floats per 16-column block
  static constexpr int NB = 8192 / BLK;            // blocks per 32 KB chunk
  static constexpr int CH4 = 8192 / 4;             // float4 per chunk
  static constexpr int F4 = CH4 / 256;             // float4 per thread per chunk
};

__device__ __forceinline__ float qval(const float2* __restrict__ Rb, int M, int MP, int i, int k) {
  const bool iim = i >= MP, kim = k >= MP;
  const int ir = iim ? i - MP : i, kr = kim ? k - MP : k;
  if (ir >= M || kr >= M) return 0.f;
  const float2 r = Rb[ir * M + kr];
  // Q = [[Rr, -Ri], [Ri, Rr]]
  return (iim == kim) ? r.x : (iim ? r.y : -r.y);
}

template <int MP>
__global__ __launch_bounds__(256, 2) void k_proj_q(const float2* __restrict__ R,
                                                   const float4* __restrict__ Xg,
                                                   float* __restrict__ P, int M, int64_t G,
                                                   int nchunk, int chunks_per_wg, int nsplit) {
  using C = QCfg<MP>;
  __shared__ float4 sX[2][C::CH4];
  __shared__ float red[2][C::WR][C::NB * 16];

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave % C::WR, wc = wave / C::WR;
  const int64_t b = blockIdx.x / nsplit;
  const int c0 = (blockIdx.x % nsplit) * chunks_per_wg;
  const int c1 = min(c0 + chunks_per_wg, nchunk);
  if (c0 >= c1) return;  // uniform across the workgroup

  // A operand: rows i = wr*RB*16 + rb*16 + lane%16, k = 4s + lane/16
  float a[C::RB][C::KS];
  const float2* Rb = R + b * int64_t(M) * M;
#pragma unroll
  for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
    for (int s = 0; s < C::KS; ++s)
      a[rb][s] = qval(Rb, M, MP, wr * C::RB * 16 + rb * 16 + (lane & 15), 4 * s + (lane >> 4));

  float4 pre[C::F4];
#pragma unroll
  for (int f = 0; f < C::F4; ++f) pre[f] = Xg[int64_t(c0) * C::CH4 + f * 256 + threadIdx.x];
#pragma unroll
  for (int f = 0; f < C::F4; ++f) sX[0][f * 256 + threadIdx.x] = pre[f];
  __syncthreads();

  const float invM2 = 1.0f / float(M * M);
  for (int c = c0; c < c1; ++c) {
    const int buf = (c - c0) & 1;
    const bool more = c + 1 < c1;
    if (more) {
#pragma unroll
      for (int f = 0; f < C::F4; ++f) pre[f] = Xg[int64_t(c + 1) * C::CH4 + f * 256 + threadIdx.x];
    }
    const float* sx = reinterpret_cast<const float*>(sX[buf]);
    for (int jb = wc; jb < C::NB; jb += C::WC) {
      floatx4 acc[C::RB];
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
      const float4* bx = sX[buf] + jb * (C::BLK / 4);
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
      // epilogue: acc[rb][r] = (Q X)[i][g0 + lane%16] with i = row(rb) + 4*(lane/16) + r
      float part = 0.f;
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = wr * C::RB * 16 + rb * 16 + 4 * (lane >> 4) + r;
          const int s = i >> 2;
          const float xv = sx[jb * C::BLK + ((s >> 2) * 64 + r * 16 + (lane & 15)) * 4 + (s & 3)];
          part += xv * acc[rb][r];
        }
      part += __shfl_xor(part, 16, 64);
      part += __shfl_xor(part, 32, 64);
      if (C::WR == 1) {
        const int64_t g = int64_t(c) * C::NB * 16 + jb * 16 + lane;
        if (lane < 16 && g < G) P[b * G + g] = part * invM2;
      } else if (lane < 16) {
        red[buf][wr][jb * 16 + lane] = part;
      }
    }
    if (more) {
#pragma unroll
      for (int f = 0; f < C::F4; ++f) sX[buf ^ 1][f * 256 + threadIdx.x] = pre[f];
    }
    __syncthreads();
    if (C::WR > 1) {
      for (int t = threadIdx.x; t < C::NB * 16; t += 256) {
        float s = 0.f;
#pragma unroll
        for (int w = 0; w < C::WR; ++w) s += red[buf][w][t];
        const int64_t g = int64_t(c) * C::NB * 16 + t;
        if (g < G) P[b * G + g] = s * invM2;
      }
    }
  }
}

template <int MP>
hipError_t launch_q(const Plan& p, int B, const float2* R, float* P, hipStream_t s) {
  using C = QCfg<MP>;
  const int nchunk = int((p.Gb + C::NB - 1) / C::NB);  // the table holds Xblocks >= nchunk * NB
  // split the grid columns over several workgroups when there are few trials
  int nsplit = 1;
  while (int64_t(B) * nsplit < 2048 && nsplit < nchunk) nsplit *= 2;
  const int per = (nchunk + nsplit - 1) / nsplit;
  nsplit = (nchunk + per - 1) / per;
  const int64_t nblk = int64_t(B) * nsplit;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_proj_q<MP>, dim3(unsigned(nblk)), dim3(256), 0, s, R,
                     reinterpret_cast<const float4*>(p.d_X), P, p.M, p.G, nchunk, per, nsplit);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_spectrum_mfma(const Plan& p, int B, const float2* R, float* P, hipStream_t s) {
  switch (p.Mp) {
    case 8: return launch_q<8>(p, B, R, P, s);
    case 16: return launch_q<16>(p, B, R, P, s);
    case 32: return launch_q<32>(p, B, R, P, s);
    case 64: return launch_q<64>(p, B, R, P, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ba
