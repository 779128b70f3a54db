// Bartlett spectrum for large arrays (2*Mp = 256 or 512 real rows) and the
// BF16 split-precision projection, as a trial-batched GEMM with the quadratic
// form fused into the epilogue: P_g = x_g^T Q x_g / M^2 (see k_proj_mfma.hip).
//
// Stage 1, k_qprep: builds Q = [[Rr, -Ri], [Ri, Rr]] per trial from R and
// writes it in MFMA A-fragment order: FP32 for v_mfma_f32_16x16x4f32, or the
// BF16 hi/lo split (hi = bf16(q), lo = bf16(q - hi), round to nearest even)
// for v_mfma_f32_16x16x32_bf16.
//
// Stage 2, k_proj_s: one workgroup of 8 waves computes a
// tile of 128 grid columns of one trial over all 2*Mp rows. Each wave owns
// 2*Mp/waves rows and streams its own A fragments straight from L2, one
// chunk ahead; the steering fragments of the tile go through LDS in chunks
// of 32 k values, double-buffered by the LDS DMA. The
// accumulators never leave the registers: the epilogue multiplies them by the
// FP32 steering rows of the same tile and reduces over rows (lane shuffles,
// then LDS across waves). Tiles are ordered so that each XCD walks through
// whole trials: the workgroups resident on one XCD share one trial's Q in
// that XCD's L2.
//
// BF16X3: Q X ~= Qh Xh + Qh Xl + Ql Xh (the lo*lo term dropped), FP32 accumulate.
// BF16 (one pass, Qh Xh) exists as a precision ablation only.
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

__device__ __forceinline__ float qval(const float2* __restrict__ Rb, int M, int MP, int i, int k) {
  const bool iim = i >= MP, kim = k >= MP;
  const int ir = iim ? i - MP : i, kr = kim ? k - MP : k;
  if (ir >= M || kr >= M) return 0.f;
  const float2 r = Rb[ir * M + kr];
  return (iim == kim) ? r.x : (iim ? r.y : -r.y);
}

// FP32 layout: Qf[b][kc][rbg][h][lane][4]: k-chunk kc of 32, row block rbg,
//   lane l, word h, element e holds Q[16 rbg + l%16][32 kc + 4 (4h + e) + l/16].
// BF16 layout: Qb[b][kc][rbg][hl][lane][8]: lane l, element e holds
//   (hi or lo of) Q[16 rbg + l%16][32 kc + 8 (l/16) + e].
template <int PREC>
__global__ __launch_bounds__(256) void k_qprep(const float2* __restrict__ R, void* __restrict__ Qout,
                                               int M, int MP) {
  const int K = 2 * MP, nkc = K / 32, nrb = K / 16;
  const int64_t b = blockIdx.y;
  const int kc = blockIdx.x / nrb, rbg = blockIdx.x % nrb;
  const float2* Rb = R + b * int64_t(M) * M;
  const int64_t per_trial = int64_t(K) * K;
  const int t = threadIdx.x;  // 256 threads
  if (PREC == BA_PREC_F32) {
    // 16 rows x 32 k = 512 values, 2 per thread
    float* Q = static_cast<float*>(Qout) + b * per_trial + (int64_t(kc) * nrb + rbg) * 512;
    for (int v = t; v < 512; v += 256) {
      const int h = v >> 8, l = (v >> 2) & 63, e = v & 3;
      const int i = 16 * rbg + (l & 15);
      const int k = 32 * kc + 4 * (4 * h + e) + (l >> 4);
      Q[v] = qval(Rb, M, MP, i, k);
    }
  } else {
    unsigned short* Q = static_cast<unsigned short*>(Qout) + 2 * (b * per_trial + (int64_t(kc) * nrb + rbg) * 512);
    for (int v = t; v < 512; v += 256) {
      const int l = v >> 3, e = v & 7;
      const int i = 16 * rbg + (l & 15);
      const int k = 32 * kc + 8 * (l >> 4) + e;
      const float q = qval(Rb, M, MP, i, k);
      const unsigned short hi = bf16_rne(q);
      const unsigned short lo = bf16_rne(q - bf16_to_f(hi));
      Q[v] = hi;
      Q[512 + v] = lo;
    }
  }
  (void)nkc;
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
  const int rb0 = wave * RBW;

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
      for (int h = 0; h < 2; ++h) a[r][h] = Qw[(int64_t(0) * NRB + rb0 + r) * 128 + h * 64 + lane];
    lds_dma_wait();
    __syncthreads();
    for (int kc = 0; kc < NKC; ++kc) {
      const int buf = kc & 1;
      const bool more = kc + 1 < NKC;
      if (more) BA_FETCH_B(kc + 1, buf ^ 1);
      const float4* sb = reinterpret_cast<const float4*>(sBd + buf * CHUNK16);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int c = 0; c < kCB; ++c) {
          const float4 bv = lds_frag(sb, c * 128 + h * 64 + lane);
#pragma unroll
          for (int r = 0; r < RBW; ++r) {
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].x, bv.x, acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].y, bv.y, acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].z, bv.z, acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][h].w, bv.w, acc[r][c], 0, 0, 0);
          }
        }
        if (more) {
#pragma unroll
          for (int r = 0; r < RBW; ++r) a[r][h] = Qw[(int64_t(kc + 1) * NRB + rb0 + r) * 128 + h * 64 + lane];
        }
      }
      lds_dma_wait();
      __syncthreads();
    }
  } else {
    const uint4* Qw = static_cast<const uint4*>(Qin) + b * (int64_t(K) * K / 4);
    uint4 ah[RBW], al[RBW], anh[RBW], anl[RBW];
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
      ah[r] = Qw[(int64_t(0) * NRB + rb0 + r) * 128 + lane];
      al[r] = Qw[(int64_t(0) * NRB + rb0 + r) * 128 + 64 + lane];
    }
    lds_dma_wait();
    __syncthreads();
    for (int kc = 0; kc < NKC; ++kc) {
      const int buf = kc & 1;
      const bool more = kc + 1 < NKC;
      if (more) {
        BA_FETCH_B(kc + 1, buf ^ 1);
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          anh[r] = Qw[(int64_t(kc + 1) * NRB + rb0 + r) * 128 + lane];
          anl[r] = Qw[(int64_t(kc + 1) * NRB + rb0 + r) * 128 + 64 + lane];
        }
      }
      // fragments of column block c + 1 are read while block c is multiplied
      uint4 bh = lds_frag(sBd + buf * CHUNK16, lane);
      uint4 bl = lds_frag(sBd + buf * CHUNK16, 64 + lane);
#pragma unroll
      for (int c = 0; c < kCB; ++c) {
        uint4 nh = bh, nl = bl;
        if (c + 1 < kCB) {
          nh = lds_frag(sBd + buf * CHUNK16, (c + 1) * 128 + lane);
          nl = lds_frag(sBd + buf * CHUNK16, (c + 1) * 128 + 64 + lane);
        }
        const bf16x8 vbh = __builtin_bit_cast(bf16x8, bh);
        const bf16x8 vbl = __builtin_bit_cast(bf16x8, bl);
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          const bf16x8 vah = __builtin_bit_cast(bf16x8, ah[r]);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, vbh, acc[r][c], 0, 0, 0);
          if (PREC == BA_PREC_BF16X3) {
            const bf16x8 val = __builtin_bit_cast(bf16x8, al[r]);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vah, vbl, acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(val, vbh, acc[r][c], 0, 0, 0);
          }
        }
        bh = nh;
        bl = nl;
      }
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
  // epilogue: rows i = 16 (rb0 + r) + 4 (lane/16) + e, column 16 c + lane%16
  float part[kCB];
#pragma unroll
  for (int c = 0; c < kCB; ++c) part[c] = 0.f;
  const float* xf = reinterpret_cast<const float*>(Xf);
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rbg = rb0 + r;  // 16 rows = k-steps 4 rbg .. 4 rbg + 3, one 16-k group
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      const int64_t blk = int64_t(tile) * kCB + c;
      const float* xb = xf + blk * (int64_t(K) * 16) + int64_t(rbg) * 256;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // k = 16 rbg + 4 (lane/16) + e -> s = 4 rbg + lane/16, lane' = e*16 + lane%16
        const float xv = xb[(e * 16 + (lane & 15)) * 4 + (lane >> 4)];
        part[c] += xv * acc[r][c][e];
      }
    }
  }
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
    if (g < G) P[b * G + g] = s / float(M * M);
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
  const dim3 g1(unsigned((K / 32) * (K / 16)), unsigned(B));
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
  // FP32 plans of up to 64 elements use the register-resident kernel instead
  if (p.Mp == 64 && p.precision == BA_PREC_BF16X3) return launch_s<64, BA_PREC_BF16X3>(p, B, Qws, P, s);
  if (p.Mp == 64 && p.precision == BA_PREC_BF16) return launch_s<64, BA_PREC_BF16>(p, B, Qws, P, s);
  BA_S(128)
  BA_S(256)
#undef BA_S
  return hipErrorInvalidValue;
}

}  // namespace ba
