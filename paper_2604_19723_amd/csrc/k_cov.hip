// Sample covariance R = (1/T) sum_t y_t y_t^H per trial (the R of the Bartlett
// cost in its covariance form, Sec. IV-D.2 read for T snapshots).
//
// One workgroup computes a 32x32 tile of R for one trial from the upper
// triangle of tile pairs (mt <= nt). Snapshot blocks of 32 x 32 complex values
// are staged in LDS with coalesced loads (each snapshot is a contiguous
// M-vector in HBM) and accumulated in FP32. The lower triangle is written as
// the conjugate of the upper one, so R is exactly Hermitian with a real
// diagonal.
#include "ba_internal.h"

namespace ba {
namespace {

constexpr int kTile = 32;   // output tile edge
constexpr int kChunk = 32;  // snapshots per LDS stage

__global__ __launch_bounds__(256) void k_cov_tiles(const float2* __restrict__ Y,
                                                   float2* __restrict__ R, int M, int T,
                                                   int ntile, int npairs) {
  const int64_t b = blockIdx.x / npairs;
  int rem = blockIdx.x % npairs;
  int mt = 0;
  while (rem >= ntile - mt) {
    rem -= ntile - mt;
    ++mt;
  }
  const int nt = mt + rem;
  const float2* Yb = Y + b * int64_t(T) * M;

  __shared__ float2 sm[kChunk][kTile + 1];
  __shared__ float2 sn[kChunk][kTile + 1];
  const int tx = threadIdx.x & 31;
  const int ty = threadIdx.x >> 5;  // 0..7
  float accr[4] = {0.f, 0.f, 0.f, 0.f};
  float acci[4] = {0.f, 0.f, 0.f, 0.f};

  for (int t0 = 0; t0 < T; t0 += kChunk) {
    for (int i = threadIdx.x; i < kChunk * kTile; i += 256) {
      const int tt = i / kTile, mm = i % kTile;
      const int t = t0 + tt;
      const int gm = mt * kTile + mm, gn = nt * kTile + mm;
      const bool tok = t < T;
      sm[tt][mm] = (tok && gm < M) ? Yb[int64_t(t) * M + gm] : make_float2(0.f, 0.f);
      sn[tt][mm] = (tok && gn < M) ? Yb[int64_t(t) * M + gn] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll 8
    for (int tt = 0; tt < kChunk; ++tt) {
      const float2 yn = sn[tt][tx];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float2 ym = sm[tt][ty + 8 * i];
        // ym * conj(yn)
        accr[i] += ym.x * yn.x + ym.y * yn.y;
        acci[i] += ym.y * yn.x - ym.x * yn.y;
      }
    }
    __syncthreads();
  }

  const float invT = 1.0f / float(T);
  float2* Rb = R + b * int64_t(M) * M;
  const int n = nt * kTile + tx;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = mt * kTile + ty + 8 * i;
    if (m < M && n < M && m <= n) {
      const float re = accr[i] * invT;
      const float im = (m == n) ? 0.f : acci[i] * invT;
      Rb[int64_t(m) * M + n] = make_float2(re, im);
      Rb[int64_t(n) * M + m] = make_float2(re, -im);
    }
  }
}

// Arrays of up to 64 elements: the covariance as a real Gram matrix on the
// matrix cores. With z_t the 2M floats of snapshot t (re, im interleaved),
// G = sum_t z_t z_t^T and
//   Re R[m][n] = G[2m][2n] + G[2m+1][2n+1],  Im R[m][n] = G[2m+1][2n] - G[2m][2n+1].
// One workgroup per trial; 64-snapshot chunks staged row-major in LDS; the
// 16x16 tiles of G on or above the diagonal (each holds 8x8 elements of R)
// are split over the waves by pairs of tile rows (w, MT-1-w), so every wave
// carries MT+1 tiles. A k-step of v_mfma_f32_16x16x4f32 reads each 16-column
// fragment once (lane (i, k) holds z_{t+k}[16c + i]) and uses it as the B
// operand of both rows' tiles.
typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int kGramChunk = 64;

// One wave's share of a trial's Gram matrix: tile rows (RA, MT - 1 - RA) as a
// compile-time case, so the MFMA sequence has no per-tile branch and the wave
// holds only its own tiles; RA < 0: a wave without tiles (it stages
// snapshots and keeps the barriers). Rows of the snapshot chunk are staged
// through registers two complex values per 16-byte load when every row
// starts on 16 bytes (M even, the block aligned), else one per 8-byte load.
template <int MT, int RA>
__device__ __forceinline__ void cov_gram_wave(const float2* __restrict__ Yb, float2* __restrict__ Rb, int M, int T,
                                              float* sZ, int lane) {
  constexpr int W = 16 * MT;   // Gram columns, 2M padded
  constexpr int LD = W + 16;   // LDS row stride: rows k and k+1 fall on different bank halves
  constexpr bool ACT = RA >= 0;
  constexpr int RB = ACT ? MT - 1 - RA : 0;
  constexpr bool TWO = ACT && RB != RA;
  floatx4 accA[MT], accB[MT];
#pragma unroll
  for (int c = 0; c < MT; ++c) {
    accA[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    accB[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  const int fi = lane & 15, fk = lane >> 4;
  // the next chunk is loaded into registers while the current one is multiplied
  constexpr int kPer = kGramChunk * (W / 2) / 256;  // float2 per thread and chunk
  static_assert(kGramChunk * (W / 2) % 512 == 0, "staging split");
  const bool wide = (M & 1) == 0 && (reinterpret_cast<uintptr_t>(Yb) & 15) == 0;
  float2 yv[kPer];
  auto load_chunk = [&](int t0) {
    if (wide) {
      const float4* Y4 = reinterpret_cast<const float4*>(Yb);
#pragma unroll
      for (int q = 0; q < kPer / 2; ++q) {
        const int v = threadIdx.x + q * 256;  // pair of columns 2 (v % (W / 4)), row v / (W / 4)
        const int tt = v / (W / 4), m = 2 * (v - tt * (W / 4));
        const int t = t0 + tt;
        const float4 w = (t < T && m < M) ? Y4[(int64_t(t) * M + m) >> 1] : make_float4(0.f, 0.f, 0.f, 0.f);
        yv[2 * q] = make_float2(w.x, w.y);
        yv[2 * q + 1] = make_float2(w.z, w.w);
      }
    } else {
#pragma unroll
      for (int q = 0; q < kPer / 2; ++q) {
        const int v = threadIdx.x + q * 256;
        const int tt = v / (W / 4), m = 2 * (v - tt * (W / 4));
        const int t = t0 + tt;
        yv[2 * q] = (t < T && m < M) ? Yb[int64_t(t) * M + m] : make_float2(0.f, 0.f);
        yv[2 * q + 1] = (t < T && m + 1 < M) ? Yb[int64_t(t) * M + m + 1] : make_float2(0.f, 0.f);
      }
    }
  };
  load_chunk(0);
  for (int t0 = 0; t0 < T; t0 += kGramChunk) {
#pragma unroll
    for (int q = 0; q < kPer / 2; ++q) {
      const int v = threadIdx.x + q * 256;
      const int tt = v / (W / 4), m = 2 * (v - tt * (W / 4));
      *reinterpret_cast<float4*>(&sZ[tt * LD + 2 * m]) =
          make_float4(yv[2 * q].x, yv[2 * q].y, yv[2 * q + 1].x, yv[2 * q + 1].y);
    }
    __syncthreads();
    if (t0 + kGramChunk < T) load_chunk(t0 + kGramChunk);
    if constexpr (ACT) {
#pragma unroll 2
      for (int s = 0; s < kGramChunk / 4; ++s) {
        const float* row = sZ + (4 * s + fk) * LD + fi;
        float f[MT];
#pragma unroll
        for (int c = RA; c < MT; ++c) f[c] = row[16 * c];
#pragma unroll
        for (int c = RA; c < MT; ++c) {
          accA[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[RA], f[c], accA[c], 0, 0, 0);
          if (TWO && c >= RB) accB[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[RB], f[c], accB[c], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  if constexpr (ACT) {
    // D[i][j] of a tile sits in lane j + 16 (i / 4), register i % 4; the odd
    // column 2n+1 is in the neighbouring lane
    const float invT = 1.0f / float(T);
    const bool even = (lane & 1) == 0;
#pragma unroll
    for (int h = 0; h < (TWO ? 2 : 1); ++h) {
      const int r = h == 0 ? RA : RB;
#pragma unroll
      for (int c = 0; c < MT; ++c) {
        if (c < r) continue;
        const floatx4 a = h == 0 ? accA[c] : accB[c];
        floatx4 x;
#pragma unroll
        for (int e = 0; e < 4; ++e) x[e] = __shfl_xor(a[e], 1, 64);
        if (!even) continue;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int m = 8 * r + 2 * (lane >> 4) + q;
          const int n = 8 * c + (fi >> 1);
          if (m >= M || n >= M || m > n) continue;
          const float re = (a[2 * q] + x[2 * q + 1]) * invT;
          const float im = m == n ? 0.f : (a[2 * q + 1] - x[2 * q]) * invT;
          Rb[int64_t(m) * M + n] = make_float2(re, im);
          if (m != n) Rb[int64_t(n) * M + m] = make_float2(re, -im);
        }
      }
    }
  }
}

template <int MT>
__global__ __launch_bounds__(256) void k_cov_mfma(const float2* __restrict__ Y, float2* __restrict__ R, int M,
                                                  int T) {
  constexpr int W = 16 * MT;
  constexpr int LD = W + 16;
  __shared__ __attribute__((aligned(16))) float sZ[kGramChunk * LD];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t b = blockIdx.x;
  const float2* Yb = Y + b * int64_t(T) * M;
  float2* Rb = R + b * int64_t(M) * M;
  constexpr int NP = (MT + 1) / 2;  // tile-row pairs, one per wave
  switch (wave) {
    case 0: cov_gram_wave<MT, 0>(Yb, Rb, M, T, sZ, lane); break;
    case 1:
      if constexpr (NP > 1) cov_gram_wave<MT, 1>(Yb, Rb, M, T, sZ, lane);
      else cov_gram_wave<MT, -1>(Yb, Rb, M, T, sZ, lane);
      break;
    case 2:
      if constexpr (NP > 2) cov_gram_wave<MT, 2>(Yb, Rb, M, T, sZ, lane);
      else cov_gram_wave<MT, -1>(Yb, Rb, M, T, sZ, lane);
      break;
    default:
      if constexpr (NP > 3) cov_gram_wave<MT, 3>(Yb, Rb, M, T, sZ, lane);
      else cov_gram_wave<MT, -1>(Yb, Rb, M, T, sZ, lane);
      break;
  }
}

}  // namespace

hipError_t launch_covariance(const Plan& p, int B, int T, const float2* Y, float2* R,
                             hipStream_t s) {
  if (p.M <= 64) {
    const dim3 grid{static_cast<uint32_t>(B)}, block{256u};
    switch ((p.M + 7) / 8) {
      case 1: hipLaunchKernelGGL(k_cov_mfma<1>, grid, block, 0, s, Y, R, p.M, T); break;
      case 2: hipLaunchKernelGGL(k_cov_mfma<2>, grid, block, 0, s, Y, R, p.M, T); break;
      case 3: hipLaunchKernelGGL(k_cov_mfma<3>, grid, block, 0, s, Y, R, p.M, T); break;
      case 4: hipLaunchKernelGGL(k_cov_mfma<4>, grid, block, 0, s, Y, R, p.M, T); break;
      case 5: hipLaunchKernelGGL(k_cov_mfma<5>, grid, block, 0, s, Y, R, p.M, T); break;
      case 6: hipLaunchKernelGGL(k_cov_mfma<6>, grid, block, 0, s, Y, R, p.M, T); break;
      case 7: hipLaunchKernelGGL(k_cov_mfma<7>, grid, block, 0, s, Y, R, p.M, T); break;
      default: hipLaunchKernelGGL(k_cov_mfma<8>, grid, block, 0, s, Y, R, p.M, T); break;
    }
    return hipGetLastError();
  }
  const int ntile = (p.M + kTile - 1) / kTile;
  const int npairs = ntile * (ntile + 1) / 2;
  const int64_t nblk = int64_t(B) * npairs;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cov_tiles, dim3(unsigned(nblk)), dim3(256), 0, s, Y, R, p.M, T, ntile, npairs);
  return hipGetLastError();
}

}  // namespace ba
