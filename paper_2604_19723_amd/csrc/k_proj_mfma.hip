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
// Q is symmetric, so x^T Q x = 2 x^T U x with U its upper triangle (diagonal
// halved): the GEMM runs over U only, about half the MFMAs of Q X.
//
// MI355X mapping (v_mfma_f32_16x16x4f32, FP32 in and out):
//  * one workgroup = one trial x a range of grid columns; 4 waves;
//  * U is built from R once per workgroup straight into MFMA A-operand
//    registers; each wave owns the pair of 16-row blocks (p, 2M/16 - 1 - p),
//    whose k ranges right of the diagonal add up to the same length for every
//    p (at M = 64 the four waves take the four pairs and share all columns;
//    smaller arrays split the 16-column blocks of a chunk between waves);
//  * the steering table is stored in HBM already in B-fragment order (16
//    columns per block, 4 k-steps per lane per 16-byte word), so one chunk of
//    8 KB is a straight copy into LDS, done by the gfx950 LDS DMA
//    (global_load_lds_dwordx4, no registers involved) one chunk ahead, and
//    every fragment read is a conflict-free ds_read_b128;
//  * epilogue: the accumulator tiles are multiplied by the matching rows of
//    the same LDS tile, reduced across the 4 row-groups of a wave by two lane
//    shuffles and across waves through LDS in a fixed order, then scaled by
//    2/M^2.
// Element counts up to 64 are padded to MP in {8, 16, 32, 64} with zero rows.
//
// Candidate variant (1-D grids): wave 0 also runs the peak rule over the
// column range while the spectrum passes through it, once per window of 64
// columns (four chunks at M = 64) gathered in its lanes. Each column whose two
// neighbours lie inside the range is tested once both are known (the last
// column of a window waits for the next window's first), and the maxima enter
// a sorted top-k list held across the wave's lanes (entry j in lane j) with
// both neighbour values for the refinement. The range's first and last
// columns, whose neighbours belong to other ranges, are left to the merge
// kernel, which gets the two values at each end of every range. The spectrum
// itself is written only when the caller asks for it.
#include <algorithm>
#include <climits>

#include "cand_window.h"
#include "proj_common.h"

namespace ba {
namespace {

// One trial's spectrum over the chunks [c0, c1) of the steering table; with
// CAND, also the peak candidates of the range (rc, wave 0), and P written only
// when Pb is not null.
template <int MP, bool CAND = false>
__device__ __forceinline__ void proj_q_trial(const float2* __restrict__ Rb, const float4* __restrict__ Xg,
                                             float* __restrict__ Pb, int M, int64_t G, int c0, int c1,
                                             float4* sX, float (*red)[QCfg<MP>::WR][QCfg<MP>::NB * 16],
                                             RangeCands* rc = nullptr) {
  using C = QCfg<MP>;
  // Candidate epilogue: wave 0 gathers the spectrum of CPW consecutive chunks
  // (a window of WIN >= 64 columns, NPL per lane) and runs the peak rule once
  // per window
  constexpr int CW = C::NB * 16;                // columns per chunk
  constexpr int WIN = CW > 64 ? CW : 64;
  constexpr int CPW = WIN / CW;
  constexpr int NPL = WIN / 64;
  static_assert(!CAND || NPL <= 2, "at most two columns per lane");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave % C::WR, wc = wave / C::WR;
  float vwin[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) vwin[i] = 0.f;

  // each wave copies its quarter of a chunk, 64 lanes x 16 bytes per DMA
  auto fetch = [&](int c, int buf) {
#pragma unroll
    for (int f = 0; f < C::CH4 / 4 / 64; ++f) {
      const int o = wave * (C::CH4 / 4) + f * 64;
      lds_dma16(Xg + int64_t(c) * C::CH4 + o + lane, sX + buf * C::CH4 + o);
    }
  };

  float a[C::VL];
  load_q_fragments<MP>(Rb, M, wr, lane, a);
  fetch(c0, 0);
  lds_dma_wait();
  __syncthreads();

  const float scale = 2.0f / float(M * M);  // P = 2 x^T U x / M^2
  for (int c = c0; c < c1; ++c) {
    const int buf = (c - c0) & 1;
    const bool more = c + 1 < c1;
    if (more) fetch(c + 1, buf ^ 1);  // the other buffer was last read before the previous barrier
    const float4* sxb = sX + buf * C::CH4;
    const float* sx = reinterpret_cast<const float*>(sxb);
    for (int jb = wc; jb < C::NB; jb += C::WC) {
      const float part = block_quadratic<MP>(a, sxb + jb * (C::BLK / 4), sx + jb * C::BLK, wr, lane);
      if (C::WR == 1 && !CAND) {
        const int64_t g = int64_t(c) * C::NB * 16 + jb * 16 + lane;
        if (lane < 16 && g < G) Pb[g] = part * scale;
      } else if (lane < 16) {
        red[buf][wr][jb * 16 + lane] = part;
      }
    }
    lds_dma_wait();
    __syncthreads();
    if constexpr (CAND) {
      // same sums and scaling as below, so P is bit-identical to the plain launch
      if (wave == 0) {
        const int q = c % CPW;  // this chunk's slot in the window
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
          const int t = lane * NPL + i - q * CW;  // column within the chunk
          if (t >= 0 && t < CW) {
            float sum;
            if (C::WR == 1) {
              sum = red[buf][0][t];
            } else {
              sum = 0.f;
#pragma unroll
              for (int w = 0; w < C::WR; ++w) sum += red[buf][w][t];
            }
            vwin[i] = sum * scale;
            const int64_t g = int64_t(c) * CW + t;
            if (Pb && g < G) Pb[g] = vwin[i];
          }
        }
        if (q == CPW - 1 || c == c1 - 1)
          window_candidates<WIN, NPL>(*rc, vwin, (c / CPW) * WIN, c / CPW == c0 / CPW, lane);
      }
    } else if (C::WR > 1) {
      for (int t = threadIdx.x; t < C::NB * 16; t += 256) {
        float s = 0.f;
#pragma unroll
        for (int w = 0; w < C::WR; ++w) s += red[buf][w][t];
        const int64_t g = int64_t(c) * C::NB * 16 + t;
        if (g < G) Pb[g] = s * scale;
      }
    }
  }
}

template <int MP>
__global__ __launch_bounds__(256, 2) void k_proj_q(const float2* __restrict__ R,
                                                   const float4* __restrict__ Xg,
                                                   float* __restrict__ P, int M, int64_t G,
                                                   int nchunk, int chunks_per_wg, int nsplit) {
  using C = QCfg<MP>;
  extern __shared__ __attribute__((aligned(16))) float4 sX[];   // [2][CH4], dynamic: filled by LDS DMA
  __shared__ float red[2][C::WR][C::NB * 16];
  const int64_t b = blockIdx.x / nsplit;
  const int c0 = (blockIdx.x % nsplit) * chunks_per_wg;
  const int c1 = min(c0 + chunks_per_wg, nchunk);
  if (c0 >= c1) return;  // uniform across the workgroup
  proj_q_trial<MP>(R + b * int64_t(M) * M, Xg, P + b * G, M, G, c0, c1, sX, red);
}

// The same over a batch whose size is only known on the device (*count
// trials, count <= the launch's capacity): the workgroups of one column range
// step through the trials with a stride of the number of trial slots in the
// grid, so the host sizes the launch without reading the count.
template <int MP>
__global__ __launch_bounds__(256, 2) void k_proj_q_counted(const float2* __restrict__ R,
                                                           const float4* __restrict__ Xg,
                                                           float* __restrict__ P, int M, int64_t G,
                                                           int nchunk, int chunks_per_wg, int nsplit,
                                                           const int* __restrict__ count) {
  using C = QCfg<MP>;
  extern __shared__ __attribute__((aligned(16))) float4 sX[];
  __shared__ float red[2][C::WR][C::NB * 16];
  const int c0 = (blockIdx.x % nsplit) * chunks_per_wg;
  const int c1 = min(c0 + chunks_per_wg, nchunk);
  if (c0 >= c1) return;
  const int64_t n = *count;
  const int64_t stride = gridDim.x / nsplit;
  for (int64_t b = blockIdx.x / nsplit; b < n; b += stride) {
    proj_q_trial<MP>(R + b * int64_t(M) * M, Xg, P + b * G, M, G, c0, c1, sX, red);
    __syncthreads();  // the next trial's first chunk reuses both LDS buffers
  }
}

// Spectrum of one trial's column range with its peak candidates: record
// (b, range) holds k list entries {value, index bits, left, right} (index
// INT_MAX: empty) and then {P[g0], P[g0 + 1], P[gl - 1], P[gl]}.
template <int MP>
__global__ __launch_bounds__(256, 6) void k_proj_qc(const float2* __restrict__ R, const float4* __restrict__ Xg,
                                                    float* __restrict__ P, int M, int64_t G, int nchunk,
                                                    int chunks_per_wg, int nsplit, int rows, int k,
                                                    float4* __restrict__ rec) {
  using C = QCfg<MP>;
  constexpr int CW = C::NB * 16;
  extern __shared__ __attribute__((aligned(16))) float4 sX[];
  __shared__ float red[2][C::WR][C::NB * 16];
  const int64_t b = blockIdx.x / nsplit;
  const int sp = int(blockIdx.x % nsplit);
  const int c0 = sp * chunks_per_wg;
  const int c1 = min(c0 + chunks_per_wg, nchunk);
  RangeCands rc;
  rc.init(c0 * CW, min(c1 * CW, rows), k);
  if (c0 < c1)  // always: the host sets nsplit = ceil(nchunk / chunks_per_wg)
    proj_q_trial<MP, true>(R + b * int64_t(M) * M, Xg, P ? P + b * G : nullptr, M, G, c0, c1, sX, red, &rc);
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    float4* o = rec + (b * nsplit + sp) * (k + 1);
    if (lane < k) o[lane] = make_float4(rc.lv, __int_as_float(rc.li), rc.ll, rc.lr);
    if (lane == 0) o[k] = make_float4(rc.e[0], rc.e[1], rc.e[2], rc.e[3]);
  }
}

// Split the grid columns over several workgroups per trial until there are
// enough of them for the last round of workgroups on the CUs to be a small
// tail (10 000 trials: two column halves, 10.58 -> 10.42 ms), keeping at
// least 32 chunks per workgroup to pay for building U in its registers, and
// at most max_split ranges.
void split_columns(int nchunk, int Bs, int max_split, int* nsplit_out, int* per_out) {
  int nsplit = 1;
  while (int64_t(Bs) * nsplit < 16384 && 2 * nsplit * 32 <= nchunk && 2 * nsplit <= max_split) nsplit *= 2;
  const int per = (nchunk + nsplit - 1) / nsplit;
  *per_out = per;
  *nsplit_out = (nchunk + per - 1) / per;
}

template <int MP>
hipError_t launch_q(const Plan& p, int B, const float2* R, float* P, hipStream_t s, const int* count = nullptr,
                    int expect = 0) {
  using C = QCfg<MP>;
  const int nchunk = int((p.Gb + C::NB - 1) / C::NB);  // the table holds Xblocks >= nchunk * NB
  // a device-counted batch is split for the size the caller expects
  const int Bs = count ? std::max(1, std::min(expect, B)) : B;
  int nsplit = 1, per = nchunk;
  split_columns(nchunk, Bs, INT_MAX, &nsplit, &per);
  const int64_t nblk = int64_t(count ? Bs : B) * nsplit;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = 2 * C::CH4 * sizeof(float4);
  if (count)
    hipLaunchKernelGGL((k_proj_q_counted<MP>), dim3(unsigned(nblk)), dim3(256), lds, s, R,
                       reinterpret_cast<const float4*>(p.d_X), P, p.M, p.G, nchunk, per, nsplit, count);
  else
    hipLaunchKernelGGL((k_proj_q<MP>), dim3(unsigned(nblk)), dim3(256), lds, s, R,
                       reinterpret_cast<const float4*>(p.d_X), P, p.M, p.G, nchunk, per, nsplit);
  return hipGetLastError();
}

template <int MP>
hipError_t launch_qc(const Plan& p, int B, const float2* R, float* P, int k, float4* rec, hipStream_t s) {
  using C = QCfg<MP>;
  const CandLayout L = candidate_layout(p, B);
  const int nchunk = int((p.Gb + C::NB - 1) / C::NB);
  const int64_t nblk = int64_t(B) * L.nsplit;
  if (nblk > 0x7fffffff || L.span != int64_t(L.per) * C::NB * 16) return hipErrorInvalidValue;
  const size_t lds = 2 * C::CH4 * sizeof(float4);
  hipLaunchKernelGGL((k_proj_qc<MP>), dim3(unsigned(nblk)), dim3(256), lds, s, R,
                     reinterpret_cast<const float4*>(p.d_X), P, p.M, p.G, nchunk, L.per, L.nsplit, p.rows, k,
                     rec);
  return hipGetLastError();
}

}  // namespace

bool candidates_supported(const Plan& p) {
  if (p.shape1 != 1) return false;
  if (p.precision == BA_PREC_F32) return p.Mp <= 64;
  return (p.precision == BA_PREC_BF16X3 || p.precision == BA_PREC_BF16) && p.Mp == 64 && p.d_Xb;
}

CandLayout candidate_layout(const Plan& p, int B) {
  CandLayout L{};
  if (p.precision != BA_PREC_F32) {  // k_proj_qb: 64-column chunks, ranges per trial pair
    qb_split(p, B, kMaxCandRanges, &L.nsplit, &L.per);
    L.span = int64_t(L.per) * 64;
    return L;
  }
  const int nb = 64 / p.Mp;  // 16-column blocks per chunk (8 KB of steering)
  const int nchunk = int((p.Gb + nb - 1) / nb);
  split_columns(nchunk, std::max(B, 1), kMaxCandRanges, &L.nsplit, &L.per);
  L.span = int64_t(L.per) * nb * 16;
  return L;
}

size_t candidate_bytes(const Plan& p, int B, int k) {
  return size_t(B) * candidate_layout(p, B).nsplit * size_t(k + 1) * sizeof(float4);
}

hipError_t launch_spectrum_candidates(const Plan& p, int B, const float2* R, float* P, int k, float4* rec,
                                      hipStream_t s) {
  if (p.precision != BA_PREC_F32) return launch_spectrum_qb_candidates(p, B, R, P, k, rec, s);
  switch (p.Mp) {
    case 8: return launch_qc<8>(p, B, R, P, k, rec, s);
    case 16: return launch_qc<16>(p, B, R, P, k, rec, s);
    case 32: return launch_qc<32>(p, B, R, P, k, rec, s);
    case 64: return launch_qc<64>(p, B, R, P, k, rec, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spectrum_mfma(const Plan& p, int B, const float2* R, float* P, hipStream_t s) {
  switch (p.Mp) {
    case 8: return launch_q<8>(p, B, R, P, s);
    case 16: return launch_q<16>(p, B, R, P, s);
    case 32: return launch_q<32>(p, B, R, P, s);
    case 64: return launch_q<64>(p, B, R, P, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spectrum_mfma_counted(const Plan& p, int cap, const int* count, int expect, const float2* R,
                                        float* P, hipStream_t s) {
  switch (p.Mp) {
    case 8: return launch_q<8>(p, cap, R, P, s, count, expect);
    case 16: return launch_q<16>(p, cap, R, P, s, count, expect);
    case 32: return launch_q<32>(p, cap, R, P, s, count, expect);
    case 64: return launch_q<64>(p, cap, R, P, s, count, expect);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ba
