// Sample covariance R = (1/T) sum_t y_t y_t^H per trial (the R of the Bartlett
// cost in its covariance form, Sec. IV-D.2 read for T snapshots), on the
// matrix cores in FP32. Only the upper triangle is formed; the lower one is
// written as its conjugate, so R is exactly Hermitian with a real diagonal.
#include "ba_internal.h"

namespace ba {
namespace {

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

// Arrays of more than 64 elements: R in blocks of 64 x 64 elements, one
// workgroup per pair of element blocks (mb <= nb) of one trial. The pair's
// share of the real Gram, G over the float rows of block mb and the float
// columns of block nb, is a 128 x 128 array of 8 x 8 tiles of 16. On a
// diagonal pair only the tiles on or above the diagonal are formed, split
// over waves 0-3 by tile-row pairs (w, 7 - w) as above; off the diagonal
// each of the eight waves takes one tile row across all eight tile columns.
// Chunks of 32 snapshots of both blocks are staged row-major in LDS by all
// eight waves, the next one held in registers while the current one is
// multiplied.
constexpr int kBlkE = 64;              // elements per block
constexpr int kBlkW = 2 * kBlkE;       // floats per block row
constexpr int kBlkLD = kBlkW + 16;     // LDS row stride (as kGramChunk's)
constexpr int kBlkChunk = 32;          // snapshots per stage
constexpr int kBlkWaves = 8;           // waves per workgroup
constexpr int kBlkThreads = 64 * kBlkWaves;
constexpr int kBlkWide = kBlkChunk * kBlkE / 2 / kBlkThreads;  // float4 per thread per block
static_assert(kBlkWide >= 1 && kBlkChunk * kBlkE / 2 % kBlkThreads == 0, "staging split");

// Tile rows RA and RB (RB == RA: one row; RA < 0: no tiles, the wave only
// stages snapshots and keeps the barriers); columns from RA (resp. RB) on
// when UPPER, else all eight. Ym, Yn: the snapshots' first element of each
// block (row stride M); cm, cn: elements in each block; Rb: the trial's R.
template <int RA, int RB, bool UPPER>
__device__ __forceinline__ void cov_block_wave(const float2* __restrict__ Ym, const float2* __restrict__ Yn,
                                               float2* __restrict__ Rb, int M, int T, int cm, int cn, int m0,
                                               int n0, bool wide, float* sM, float* sN, int lane) {
  constexpr bool ACT = RA >= 0;
  constexpr bool TWO = ACT && RB != RA;
  constexpr int CA = !ACT ? 0 : (UPPER ? RA : 0), CB = !ACT ? 0 : (UPPER ? RB : 0);
  constexpr bool SAME = UPPER;  // a diagonal pair stages one block
  floatx4 accA[8], accB[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    accA[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    accB[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  const int fi = lane & 15, fk = lane >> 4;
  float4 ym[kBlkWide], yn[kBlkWide];
  // thread v of a block's chunk: row v / 32, elements 2 (v % 32) and 2 (v % 32) + 1
  auto load_block = [&](const float2* __restrict__ Yb, int cnt, int t0, float4 (&y)[kBlkWide]) {
#pragma unroll
    for (int q = 0; q < kBlkWide; ++q) {
      const int v = threadIdx.x + q * kBlkThreads;
      const int tt = v >> 5, m = 2 * (v & 31);
      const int t = t0 + tt;
      if (wide) {
        y[q] = (t < T && m < cnt) ? *reinterpret_cast<const float4*>(Yb + int64_t(t) * M + m)
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        const float2 a = (t < T && m < cnt) ? Yb[int64_t(t) * M + m] : make_float2(0.f, 0.f);
        const float2 b = (t < T && m + 1 < cnt) ? Yb[int64_t(t) * M + m + 1] : make_float2(0.f, 0.f);
        y[q] = make_float4(a.x, a.y, b.x, b.y);
      }
    }
  };
  auto store_block = [&](float* s, const float4 (&y)[kBlkWide]) {
#pragma unroll
    for (int q = 0; q < kBlkWide; ++q) {
      const int v = threadIdx.x + q * kBlkThreads;
      *reinterpret_cast<float4*>(&s[(v >> 5) * kBlkLD + 4 * (v & 31)]) = y[q];
    }
  };
  load_block(Ym, cm, 0, ym);
  if constexpr (!SAME) load_block(Yn, cn, 0, yn);
  const float* sB = SAME ? sM : sN;
  for (int t0 = 0; t0 < T; t0 += kBlkChunk) {
    store_block(sM, ym);
    if constexpr (!SAME) store_block(sN, yn);
    __syncthreads();
    if (t0 + kBlkChunk < T) {
      load_block(Ym, cm, t0 + kBlkChunk, ym);
      if constexpr (!SAME) load_block(Yn, cn, t0 + kBlkChunk, yn);
    }
    if constexpr (ACT) {
#pragma unroll 2
    for (int s = 0; s < kBlkChunk / 4; ++s) {
      const int row = (4 * s + fk) * kBlkLD + fi;
      const float fa = sM[row + 16 * RA];
      const float fb = TWO ? sM[row + 16 * RB] : 0.f;
      float f[8];
#pragma unroll
      for (int c = CA < CB ? CA : CB; c < 8; ++c) f[c] = sB[row + 16 * c];
#pragma unroll
      for (int c = CA; c < 8; ++c) accA[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa, f[c], accA[c], 0, 0, 0);
      if constexpr (TWO) {
#pragma unroll
        for (int c = CB; c < 8; ++c) accB[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb, f[c], accB[c], 0, 0, 0);
      }
    }
    }
    __syncthreads();
  }
  if constexpr (!ACT) return;
  // D[i][j] of a tile sits in lane j + 16 (i / 4), register i % 4; the odd
  // column 2n+1 is in the neighbouring lane
  const float invT = 1.0f / float(T);
  const bool even = (lane & 1) == 0;
#pragma unroll
  for (int h = 0; h < (TWO ? 2 : 1); ++h) {
    const int r = h == 0 ? RA : RB;
    const int c0 = h == 0 ? CA : CB;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c < c0) continue;
      const floatx4 a = h == 0 ? accA[c] : accB[c];
      floatx4 x;
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = __shfl_xor(a[e], 1, 64);
      if (!even) continue;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ml = 8 * r + 2 * (lane >> 4) + q, nl = 8 * c + (fi >> 1);
        const int m = m0 + ml, n = n0 + nl;
        if (ml >= cm || nl >= cn || m > n) continue;
        const float re = (a[2 * q] + x[2 * q + 1]) * invT;
        const float im = m == n ? 0.f : (a[2 * q + 1] - x[2 * q]) * invT;
        Rb[int64_t(m) * M + n] = make_float2(re, im);
        if (m != n) Rb[int64_t(n) * M + m] = make_float2(re, -im);
      }
    }
  }
}

// nbk = ceil(M / 64) element blocks, npair = nbk (nbk + 1) / 2 pairs per
// trial, total = B npair logical workgroups. The launch is padded to a
// multiple of 8; workgroup i runs on XCD i mod 8, so logical workgroup
// (i mod 8) (n / 8) + i / 8 gives every XCD a contiguous run and a trial's
// pairs read its snapshots through one L2.
__global__ __launch_bounds__(kBlkThreads) void k_cov_blocks(const float2* __restrict__ Y, float2* __restrict__ R,
                                                            int M, int T, int nbk, int npair, int64_t total) {
  __shared__ __attribute__((aligned(16))) float sM[kBlkChunk * kBlkLD];
  __shared__ __attribute__((aligned(16))) float sN[kBlkChunk * kBlkLD];
  const int64_t nphys = int64_t(gridDim.x);
  const int64_t l = int64_t(blockIdx.x % 8) * (nphys / 8) + blockIdx.x / 8;
  if (l >= total) return;  // padding: the whole workgroup leaves before any barrier
  const int64_t b = l / npair;
  int rem = int(l - b * npair), mb = 0;
  while (rem >= nbk - mb) {
    rem -= nbk - mb;
    ++mb;
  }
  const int nb = mb + rem;
  const int m0 = kBlkE * mb, n0 = kBlkE * nb;
  const int cm = min(kBlkE, M - m0), cn = min(kBlkE, M - n0);
  const float2* Yb = Y + b * int64_t(T) * M;
  float2* Rb = R + b * int64_t(M) * M;
  const float2* Ym = Yb + m0;
  const float2* Yn = Yb + n0;
  // 16-byte loads when every block row starts on 16 bytes
  const bool wide = (M & 1) == 0 && (reinterpret_cast<uintptr_t>(Yb) & 15) == 0;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // off the diagonal wave w forms tile row w across all eight tile columns;
  // on it waves 0-3 form the tile-row pairs (w, 7 - w) and waves 4-7 only stage
#define BA_COV_BLOCK_CASE(w, RA, RB)                                                       \
  case w:                                                                                  \
    if (mb == nb)                                                                          \
      cov_block_wave<RA, RB, true>(Ym, Yn, Rb, M, T, cm, cn, m0, n0, wide, sM, sN, lane);  \
    else                                                                                   \
      cov_block_wave<w, w, false>(Ym, Yn, Rb, M, T, cm, cn, m0, n0, wide, sM, sN, lane);   \
    break;
  switch (wave) {
    BA_COV_BLOCK_CASE(0, 0, 7)
    BA_COV_BLOCK_CASE(1, 1, 6)
    BA_COV_BLOCK_CASE(2, 2, 5)
    BA_COV_BLOCK_CASE(3, 3, 4)
    BA_COV_BLOCK_CASE(4, -1, -1)
    BA_COV_BLOCK_CASE(5, -1, -1)
    BA_COV_BLOCK_CASE(6, -1, -1)
    default:
      if (mb == nb)
        cov_block_wave<-1, -1, true>(Ym, Yn, Rb, M, T, cm, cn, m0, n0, wide, sM, sN, lane);
      else
        cov_block_wave<7, 7, false>(Ym, Yn, Rb, M, T, cm, cn, m0, n0, wide, sM, sN, lane);
      break;
  }
#undef BA_COV_BLOCK_CASE
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
  const int nbk = (p.M + kBlkE - 1) / kBlkE;
  const int npair = nbk * (nbk + 1) / 2;
  const int64_t total = int64_t(B) * npair;
  const int64_t nphys = (total + 7) / 8 * 8;
  if (nphys > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cov_blocks, dim3(unsigned(nphys)), dim3(kBlkThreads), 0, s, Y, R, p.M, T, nbk, npair, total);
  return hipGetLastError();
}

}  // namespace ba
