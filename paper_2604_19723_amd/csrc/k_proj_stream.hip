// Bartlett spectrum for large arrays (2*Mp = 256 or 512 real rows) and the
// BF16 split-precision projection, as a trial-batched GEMM with the quadratic
// form fused into the epilogue: P_g = 2 x_g^T L x_g / M^2, L the lower
// triangle of the symmetric Q with its diagonal halved (Q symmetric, so
// x^T Q x = 2 x^T L x; see k_proj_mfma.hip).
//
// Stage 1, k_qprep: builds L per trial from R and writes it in MFMA
// A-fragment order: FP32 for v_mfma_f32_16x16x4f32, or the BF16 hi/lo split
// (hi = bf16(l), lo = bf16(l - hi), round to nearest even) for
// v_mfma_f32_16x16x32_bf16.
//
// Stage 2, k_proj_s: one workgroup of 8 waves computes a tile of 128 grid
// columns of one trial over all 2*Mp rows. Wave w owns the row blocks
// w, w + 8, w + 16, ...; row block rb takes part in the k-chunks of 32 up to
// its diagonal chunk rb / 2, so at every chunk the active row blocks are
// spread evenly over the four SIMDs (waves w and w + 4 share one), and a row
// block's sums are final in the very chunk whose steering rows it needs for
// the quadratic form: the epilogue of each row block reads x from the LDS
// chunk at that point and no steering value is fetched twice. Each wave
// streams its own A fragments straight from L2, one chunk ahead; the
// steering fragments of the tile go through LDS in chunks of 32 k values,
// double-buffered by the LDS DMA. The per-wave sums are reduced over rows by
// lane shuffles, then across waves through LDS. Tiles are ordered so that
// each XCD walks through whole trials: the workgroups resident on one XCD
// share one trial's L in that XCD's L2.
//
// BF16X3: L X ~= Lh Xh + Lh Xl + Ll Xh (the lo*lo term dropped), FP32
// accumulate; the epilogue takes x = xh + xl (16 significant bits, below the
// error of the dropped term). BF16 (one pass, Lh Xh) is a precision ablation.
#include "proj_common.h"

namespace ba {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));

constexpr int kCB = 8;     // 16-column blocks per tile (128 columns)

// waves per workgroup (2 per SIMD, up to 256 registers each)
template <int PREC>
constexpr int waves_for() { return 8; }

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float(unsigned(h) << 16); }

// L(i, k): Q left of the diagonal, half the diagonal, zero right of it
__device__ __forceinline__ float lval(const float2* __restrict__ Rb, int M, int MP, int i, int k) {
  if (k > i) return 0.f;
  const float q = qval(Rb, M, MP, i, k);
  return k == i ? 0.5f * q : q;
}

// FP32 layout: Lf[b][kc][rbg][h][lane][4]: k-chunk kc of 32, row block rbg,
//   lane l, word h, element e holds L[16 rbg + l%16][32 kc + 4 (4h + e) + l/16].
// BF16 layout: Lb[b][kc][rbg][hl][lane][8]: lane l, element e holds
//   (hi or lo of) L[16 rbg + l%16][32 kc + 8 (l/16) + e].
// Chunks right of a row block's diagonal (kc > rbg / 2) would hold zeros; they
// are neither loaded nor multiplied, so they are not written either.
template <int PREC>
__global__ __launch_bounds__(256) void k_qprep(const float2* __restrict__ R, void* __restrict__ Qout,
                                               int M, int MP) {
  // one workgroup per (row block, trial), walking the row block's k-chunks
  // up to its diagonal chunk
  const int K = 2 * MP, nrb = K / 16;
  const int64_t b = blockIdx.y;
  const int rbg = blockIdx.x;
  const float2* Rb = R + b * int64_t(M) * M;
  const int64_t per_trial = int64_t(K) * K;
  const int t = threadIdx.x;  // 256 threads
  for (int kc = 0; kc <= (rbg >> 1); ++kc) {
    if (PREC == BA_PREC_F32) {
      // 16 rows x 32 k = 512 values, 2 per thread
      float* Q = static_cast<float*>(Qout) + b * per_trial + (int64_t(kc) * nrb + rbg) * 512;
      for (int v = t; v < 512; v += 256) {
        const int h = v >> 8, l = (v >> 2) & 63, e = v & 3;
        const int i = 16 * rbg + (l & 15);
        const int k = 32 * kc + 4 * (4 * h + e) + (l >> 4);
        Q[v] = lval(Rb, M, MP, i, k);
      }
    } else {
      unsigned short* Q =
          static_cast<unsigned short*>(Qout) + 2 * (b * per_trial + (int64_t(kc) * nrb + rbg) * 512);
      for (int v = t; v < 512; v += 256) {
        const int l = v >> 3, e = v & 7;
        const int i = 16 * rbg + (l & 15);
        const int k = 32 * kc + 8 * (l >> 4) + e;
        const float q = lval(Rb, M, MP, i, k);
        const unsigned short hi = bf16_rne(q);
        const unsigned short lo = bf16_rne(q - bf16_to_f(hi));
        Q[v] = hi;
        Q[512 + v] = lo;
      }
    }
  }
}

// One k-chunk of the FP32 kernel for the last N row-block slots of a wave
// (the ones not yet past their diagonal chunk); after each half of the A
// fragments is used, the same half of the next chunk's fragments is loaded
// for the slots still active there (first_next on).
template <int N, int RBW, int NRB, int WS>
__device__ __forceinline__ void chunk_f32(floatx4 (&acc)[RBW][kCB], float4 (&a)[RBW][2],
                                          const float4* __restrict__ sb, const float4* __restrict__ Qw,
                                          int kc_next, bool more, int first_next, int wave, int lane) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      const float4 bv = lds_frag(sb, c * 128 + h * 64 + lane);
#pragma unroll
      for (int r = RBW - N; r < RBW; ++r) {
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].x, bv.x, acc[r][c], 0, 0, 0);
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].y, bv.y, acc[r][c], 0, 0, 0);
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].z, bv.z, acc[r][c], 0, 0, 0);
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].w, bv.w, acc[r][c], 0, 0, 0);
      }
    }
    if (more) {
#pragma unroll
      for (int r = 0; r < RBW; ++r) {
        if (r < first_next) continue;  // past its diagonal chunk: nothing to load
        a[r][h] = Qw[(int64_t(kc_next) * NRB + wave + WS * r) * 128 + h * 64 + lane];
      }
    }
  }
}

// Quadratic-form sums of a finished row block rbg (rows 16 rbg + 4 (lane/16)
// + e, column 16 c + lane%16 of the tile) against the steering rows of the
// LDS chunk that holds them: FP32 chunk words [c][h][lane'][4] hold
// x[32 kc + 4 (4 h + e') + lane'/16][16 c + lane'%16]
__device__ __forceinline__ void fold_rows_f32(float (&part)[kCB], const floatx4 (&acc)[kCB],
                                              const float* __restrict__ sbf, int rbg, int lane) {
#pragma unroll
  for (int c = 0; c < kCB; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      part[c] += sbf[(c * 128 + (rbg & 1) * 64 + 16 * e + (lane & 15)) * 4 + (lane >> 4)] * acc[c][e];
}

__device__ __forceinline__ float bf_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// the same from a BF16 chunk, words [c][hi, lo][lane'][8] holding
// x[32 kc + 8 (lane'/16) + e'][16 c + lane'%16]: the four rows of a lane are
// four consecutive values of one word, x = xh + xl
__device__ __forceinline__ void fold_rows_bf16(float (&part)[kCB], const floatx4 (&acc)[kCB],
                                               const uint4* __restrict__ sb, int rbg, int lane) {
  const int w = (rbg & 1) * 32 + (lane >> 5) * 16 + (lane & 15), eh = (lane >> 4) & 1;
#pragma unroll
  for (int c = 0; c < kCB; ++c) {
    const uint2 xh = lds_frag(reinterpret_cast<const uint2*>(sb + c * 128 + w), eh);
    const uint2 xl = lds_frag(reinterpret_cast<const uint2*>(sb + c * 128 + 64 + w), eh);
    part[c] += (bf_lo(xh.x) + bf_lo(xl.x)) * acc[c][0];
    part[c] += (bf_hi(xh.x) + bf_hi(xl.x)) * acc[c][1];
    part[c] += (bf_lo(xh.y) + bf_lo(xl.y)) * acc[c][2];
    part[c] += (bf_hi(xh.y) + bf_hi(xl.y)) * acc[c][3];
  }
}

// One k-chunk of the split-precision kernel for the last N row-block slots
// of a wave (those not past their diagonal chunk). For each column block the
// passes go over all N slots in turn (hi x hi for every slot, then hi x lo,
// then lo x hi), so consecutive MFMAs write different accumulators; the
// fragments of column block c + 1 are read from LDS while block c is
// multiplied.
template <int N, int RBW, int PREC>
__device__ __forceinline__ void chunk_bf16(floatx4 (&acc)[RBW][kCB], const uint4 (&ah)[RBW], const uint4 (&al)[RBW],
                                           const uint4* __restrict__ sb, int lane) {
  // column blocks in pairs: every pass goes over both blocks of the pair and
  // all N slots, so even a single active slot has two independent chains
  uint4 bh0 = lds_frag(sb, lane), bl0 = lds_frag(sb, 64 + lane);
  uint4 bh1 = lds_frag(sb, 128 + lane), bl1 = lds_frag(sb, 192 + lane);
#pragma unroll
  for (int cp = 0; cp < kCB / 2; ++cp) {
    const int c0 = 2 * cp, c1 = c0 + 1;
    uint4 nh0 = bh0, nl0 = bl0, nh1 = bh1, nl1 = bl1;
    if (cp + 1 < kCB / 2) {
      nh0 = lds_frag(sb, (c0 + 2) * 128 + lane);
      nl0 = lds_frag(sb, (c0 + 2) * 128 + 64 + lane);
      nh1 = lds_frag(sb, (c1 + 2) * 128 + lane);
      nl1 = lds_frag(sb, (c1 + 2) * 128 + 64 + lane);
    }
    const bf16x8 vh0 = __builtin_bit_cast(bf16x8, bh0), vl0 = __builtin_bit_cast(bf16x8, bl0);
    const bf16x8 vh1 = __builtin_bit_cast(bf16x8, bh1), vl1 = __builtin_bit_cast(bf16x8, bl1);
#pragma unroll
    for (int r = RBW - N; r < RBW; ++r) {
      acc[r][c0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah[r]), vh0, acc[r][c0], 0, 0, 0);
      acc[r][c1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah[r]), vh1, acc[r][c1], 0, 0, 0);
    }
    if (PREC == BA_PREC_BF16X3) {
#pragma unroll
      for (int r = RBW - N; r < RBW; ++r) {
        acc[r][c0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah[r]), vl0, acc[r][c0], 0, 0, 0);
        acc[r][c1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah[r]), vl1, acc[r][c1], 0, 0, 0);
      }
#pragma unroll
      for (int r = RBW - N; r < RBW; ++r) {
        acc[r][c0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al[r]), vh0, acc[r][c0], 0, 0, 0);
        acc[r][c1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al[r]), vh1, acc[r][c1], 0, 0, 0);
      }
    }
    bh0 = nh0;
    bl0 = nl0;
    bh1 = nh1;
    bl1 = nl1;
  }
}

template <int MP, int PREC>
__global__ __launch_bounds__(64 * waves_for<PREC>(), 1) void k_proj_s(const void* __restrict__ Qin,
                                                const float4* __restrict__ Xf,   // FP32 table (fragment order)
                                                const uint4* __restrict__ Xb,    // BF16 hi/lo table
                                                float* __restrict__ P, int M, int64_t G, int ntile,
                                                int64_t nlogical) {
  constexpr int kWaves = waves_for<PREC>();
  constexpr int K = 2 * MP;
  constexpr int NKC = K / 32;            // k-chunks
  constexpr int NRB = K / 16;            // row blocks
  constexpr int RBW = NRB / kWaves;      // row blocks per wave
  constexpr int CHUNK16 = kCB * 64 * 2;  // 16-byte words of B per chunk (16 KB)
  static_assert(RBW >= 1, "rows per wave");

  extern __shared__ __attribute__((aligned(16))) uint4 sBd[];  // [2][CHUNK16], filled by LDS DMA
  __shared__ float red[kWaves][kCB * 16];

  // XCD-aware order: hardware places workgroup i on XCD i % 8, so logical tile
  // L = (i % 8) * (n / 8) + i / 8 gives each XCD a contiguous run of tiles.
  const int64_t nphys = int64_t(gridDim.x);
  const int64_t i = blockIdx.x;
  const int64_t L = (i % 8) * (nphys / 8) + i / 8;
  if (L >= nlogical) return;
  const int64_t b = L / ntile;
  const int tile = int(L % ntile);

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // slot r holds row block wave + kWaves r, which takes part up to its
  // diagonal k-chunk (wave + kWaves r) / 2: slots drop out in order, every 4
  // chunks, each right after the chunk that finishes it
  static_assert(kWaves == 8, "last chunk of slot r = wave / 2 + 4 r");
  const int kc00 = wave >> 1;
  auto first_active = [&](int kc) { return kc <= kc00 ? 0 : (kc - kc00 + 3) / 4; };
  float part[kCB];
#pragma unroll
  for (int c = 0; c < kCB; ++c) part[c] = 0.f;

  floatx4 acc[RBW][kCB];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int c = 0; c < kCB; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};

  // B chunk kc: 8 column blocks x 2 KB = 16 DMAs of 64 lanes x 16 bytes, spread over the waves
  const uint4* Xsrc = PREC == BA_PREC_F32 ? reinterpret_cast<const uint4*>(Xf) : Xb;
  constexpr int DPW = 16 / kWaves;  // DMAs per wave
#define BA_FETCH_B(kc, buf)                                                                     \
  do {                                                                                          \
    _Pragma("unroll") for (int d_ = 0; d_ < DPW; ++d_) {                                        \
      const int q_ = wave * DPW + d_;                /* 0..15: block q_/2, half q_%2 */        \
      const int64_t blk_ = int64_t(tile) * kCB + (q_ >> 1);                                     \
      lds_dma16(Xsrc + (blk_ * NKC + (kc)) * 128 + (q_ & 1) * 64 + lane,                        \
                sBd + (buf) * CHUNK16 + q_ * 64);                                               \
    }                                                                                           \
  } while (0)

  BA_FETCH_B(0, 0);

  if (PREC == BA_PREC_F32) {
    // A fragments of a chunk come as two halves (k-steps 0..3 and 4..7); the
    // next chunk's half h is loaded as soon as this chunk is done with it, so
    // each load has half a chunk of MFMA work to land in, with no extra registers
    const float4* Qw = static_cast<const float4*>(Qin) + b * (int64_t(K) * K / 4);
    float4 a[RBW][2];
#pragma unroll
    for (int r = 0; r < RBW; ++r)
#pragma unroll
      for (int h = 0; h < 2; ++h) a[r][h] = Qw[int64_t(wave + kWaves * r) * 128 + h * 64 + lane];
    lds_dma_wait();
    __syncthreads();
    for (int kc = 0; kc < NKC; ++kc) {
      const int buf = kc & 1;
      const bool more = kc + 1 < NKC;
      if (more) BA_FETCH_B(kc + 1, buf ^ 1);
      const float4* sb = reinterpret_cast<const float4*>(sBd + buf * CHUNK16);
      const int fnext = more ? first_active(kc + 1) : RBW;
      switch (RBW - min(RBW, first_active(kc))) {
        case 0:
          chunk_f32<0, RBW, NRB, kWaves>(acc, a, sb, Qw, kc + 1, more, fnext, wave, lane);
          break;
        case 1:
          chunk_f32<1, RBW, NRB, kWaves>(acc, a, sb, Qw, kc + 1, more, fnext, wave, lane);
          break;
        case 2:
          if constexpr (RBW >= 2) chunk_f32<2, RBW, NRB, kWaves>(acc, a, sb, Qw, kc + 1, more, fnext, wave, lane);
          break;
        case 3:
          if constexpr (RBW >= 3) chunk_f32<3, RBW, NRB, kWaves>(acc, a, sb, Qw, kc + 1, more, fnext, wave, lane);
          break;
        default:
          if constexpr (RBW >= 4) chunk_f32<4, RBW, NRB, kWaves>(acc, a, sb, Qw, kc + 1, more, fnext, wave, lane);
          break;
      }
      // the slot whose diagonal chunk this is: its rows' sums are final
#pragma unroll
      for (int r = 0; r < RBW; ++r)
        if (kc == kc00 + 4 * r) fold_rows_f32(part, acc[r], reinterpret_cast<const float*>(sb),
                                                       wave + kWaves * r, lane);
      lds_dma_wait();
      __syncthreads();
    }
  } else {
    const uint4* Qw = static_cast<const uint4*>(Qin) + b * (int64_t(K) * K / 4);
    uint4 ah[RBW], al[RBW], anh[RBW], anl[RBW];
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
      ah[r] = Qw[int64_t(wave + kWaves * r) * 128 + lane];
      al[r] = Qw[int64_t(wave + kWaves * r) * 128 + 64 + lane];
      anh[r] = anl[r] = make_uint4(0u, 0u, 0u, 0u);
    }
    lds_dma_wait();
    __syncthreads();
    for (int kc = 0; kc < NKC; ++kc) {
      const int buf = kc & 1;
      const bool more = kc + 1 < NKC;
      if (more) {
        BA_FETCH_B(kc + 1, buf ^ 1);
        // slots past their diagonal chunk load nothing (their registers keep
        // stale values that no MFMA reads)
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          if (r < first_active(kc + 1)) continue;
          anh[r] = Qw[(int64_t(kc + 1) * NRB + wave + kWaves * r) * 128 + lane];
          anl[r] = Qw[(int64_t(kc + 1) * NRB + wave + kWaves * r) * 128 + 64 + lane];
        }
      }
      // slots r < first are past their diagonal chunk: the active ones are a
      // suffix of the wave's slots, one code path per count (scalar switch)
      const int first = first_active(kc);
      const uint4* sb = sBd + buf * CHUNK16;
      switch (RBW - min(RBW, first)) {
        case 0: break;
        case 1: chunk_bf16<1, RBW, PREC>(acc, ah, al, sb, lane); break;
        case 2:
          if constexpr (RBW >= 2) chunk_bf16<2, RBW, PREC>(acc, ah, al, sb, lane);
          break;
        case 3:
          if constexpr (RBW >= 3) chunk_bf16<3, RBW, PREC>(acc, ah, al, sb, lane);
          break;
        default:
          if constexpr (RBW >= 4) chunk_bf16<4, RBW, PREC>(acc, ah, al, sb, lane);
          break;
      }
#pragma unroll
      for (int r = 0; r < RBW; ++r)
        if (kc == kc00 + 4 * r) fold_rows_bf16(part, acc[r], sb, wave + kWaves * r, lane);
      if (more) {
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          ah[r] = anh[r];
          al[r] = anl[r];
        }
      }
      lds_dma_wait();
      __syncthreads();
    }
  }

#undef BA_FETCH_B
#pragma unroll
  for (int c = 0; c < kCB; ++c) {
    float v = part[c];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lane < 16) red[wave][c * 16 + lane] = v;
  }
  __syncthreads();
  if (threadIdx.x < kCB * 16) {
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += red[w][threadIdx.x];
    const int64_t g = int64_t(tile) * kCB * 16 + threadIdx.x;
    if (g < G) P[b * G + g] = s * (2.0f / float(M * M));  // P = 2 x^T L x / M^2
  }
}

template <int MP, int PREC>
hipError_t launch_s(const Plan& p, int B, const void* Q, float* P, hipStream_t s) {
  constexpr int kWaves = waves_for<PREC>();
  const int ntile = int((p.Gb + kCB - 1) / kCB);  // <= Xblocks / kCB
  const int64_t nlog = int64_t(B) * ntile;
  const int64_t nphys = (nlog + 7) / 8 * 8;
  if (nphys > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_proj_s<MP, PREC>), dim3(unsigned(nphys)), dim3(64 * kWaves), 2 * 1024 * sizeof(uint4), s, Q,
                     reinterpret_cast<const float4*>(p.d_X), reinterpret_cast<const uint4*>(p.d_Xb),
                     P, p.M, p.G, ntile, nlog);
  return hipGetLastError();
}

}  // namespace

size_t qprep_bytes(const Plan& p, int B) {
  const int K = 2 * p.Mp;
  return size_t(B) * K * K * 4;  // FP32, or BF16 hi + lo
}

hipError_t launch_spectrum_stream(const Plan& p, int B, const float2* R, void* Qws, float* P,
                                  hipStream_t s) {
  const int K = 2 * p.Mp;
  const dim3 g1(unsigned(K / 16), unsigned(B));
  const bool f32 = p.precision == BA_PREC_F32;
  if (f32)
    hipLaunchKernelGGL(k_qprep<BA_PREC_F32>, g1, dim3(256), 0, s, R, Qws, p.M, p.Mp);
  else
    hipLaunchKernelGGL(k_qprep<BA_PREC_BF16X3>, g1, dim3(256), 0, s, R, Qws, p.M, p.Mp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define BA_S(MPV)                                                                           \
  if (p.Mp == MPV) {                                                                         \
    if (p.precision == BA_PREC_F32) return launch_s<MPV, BA_PREC_F32>(p, B, Qws, P, s);     \
    if (p.precision == BA_PREC_BF16X3) return launch_s<MPV, BA_PREC_BF16X3>(p, B, Qws, P, s); \
    return launch_s<MPV, BA_PREC_BF16>(p, B, Qws, P, s);                                   \
  }
  // plans of up to 64 elements use the register-resident kernels instead
  BA_S(128)
  BA_S(256)
#undef BA_S
  return hipErrorInvalidValue;
}

}  // namespace ba
