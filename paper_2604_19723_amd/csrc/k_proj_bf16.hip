// Split-precision Bartlett projection for arrays of up to 64 elements with Q
// resident in registers (the BF16 counterpart of k_proj_q).
//
// U X ~= Uh Xh + Uh Xl + Ul Xh on v_mfma_f32_16x16x32_bf16, FP32 accumulate
// (hi = bf16(u), lo = bf16(u - hi), round to nearest even; the lo*lo term is
// dropped), with U the upper triangle of the symmetric Q (diagonal halved), so
// x^T Q x = 2 x^T U x. Row block rb of U needs the k-steps of 32 from rb / 2
// on; the pairs of row blocks (p, 7 - p) a wave holds need 5 of the 8 k-steps
// of the full Q. U's hi/lo fragments are built from R once per workgroup;
// the BF16 steering chunks (hi and lo interleaved per k-step) arrive by LDS
// DMA one chunk ahead. The quadratic-form epilogue takes x = xh + xl from the
// same LDS chunk (16 significant bits, below the error of the dropped term).
//
// A workgroup serves two trials, and each wave carries both: every steering
// chunk brought on chip and every B fragment and epilogue row read from LDS
// serves the two trials. 4 waves = 2 row waves x 2 column halves of the
// chunk. Row wave w holds the row blocks {w, 7 - w, 2 + w, 5 - w}, whose
// first k-steps are {0, 3, 1, 2} for either w, so both run the same code. Per
// 16-column block a wave issues 2 x 10 x 3 = 60 MFMAs against 8
// conflict-free 16-byte LDS reads and 8 8-byte epilogue reads. The 160
// registers of hi/lo fragments leave room for two waves per SIMD; the
// workgroup builds them in LDS first, so no wave holds conversion
// temporaries beside them (no spills).
//
// Candidate variant (1-D grids): after each chunk's barrier wave t holds trial
// t's 64 new spectrum values, one per lane, which is one window of the peak
// rule of k_proj_qc (cand_window.h); the spectrum is written only when the
// caller asks for it.
#include <algorithm>
#include <climits>

#include "cand_window.h"
#include "proj_common.h"

namespace ba {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int MPB = 64;             // padded element count
constexpr int KB = 2 * MPB;         // 128 rows of Q
constexpr int NKC = KB / 32;        // 4 k-steps of 32
constexpr int WRB = 2;              // row waves per trial
constexpr int NSLOT = 4;            // row blocks per wave
constexpr int NFRAG = 10;           // k-steps held per wave: 4 + 1 + 3 + 2
constexpr int NTW = 2;              // trials per workgroup
constexpr int BLKW = NKC * 2 * 64;  // 16-byte words per 16-column block (8 KB)
constexpr int NBB = 4;              // blocks per 32 KB chunk
constexpr int CHW = NBB * BLKW;     // 16-byte words per chunk

// row block of slot j for row wave w, its first k-step, and its first register
__device__ __forceinline__ constexpr int slot_rb(int j, int w) {
  return j == 0 ? w : (j == 1 ? 7 - w : (j == 2 ? 2 + w : 5 - w));
}
__device__ __forceinline__ constexpr int slot_kc0(int j) { return j == 0 ? 0 : (j == 1 ? 3 : (j == 2 ? 1 : 2)); }
__device__ __forceinline__ constexpr int slot_off(int j) { return j == 0 ? 0 : (j == 1 ? 4 : (j == 2 ? 5 : 8)); }
static_assert(slot_off(3) + NKC - slot_kc0(3) == NFRAG, "fragment count");

__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float lo_half(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_half(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// CAND: P may be null; rows = candidate rows of the grid; rec = candidate
// records [B][nsplit][k + 1] as k_proj_qc writes them
template <int PREC, bool CAND = false>
__global__ __launch_bounds__(256, 2) void k_proj_qb(const float2* __restrict__ R, const uint4* __restrict__ Xb,
                                                    float* __restrict__ P, int B, int M, int64_t G, int nchunk,
                                                    int chunks_per_wg, int nsplit, int rows = 0, int k = 0,
                                                    float4* __restrict__ rec = nullptr) {
  extern __shared__ __attribute__((aligned(16))) uint4 sXb[];  // [2][CHW], LDS DMA
  __shared__ float red[2][NTW][WRB][NBB * 16];

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave % WRB, wc = wave / WRB;  // row wave, column half
  const int64_t pair = blockIdx.x / nsplit;
  const int sp = int(blockIdx.x % nsplit);
  const int c0 = sp * chunks_per_wg;
  const int c1 = min(c0 + chunks_per_wg, nchunk);
  static_assert(NBB * 16 == 64, "a chunk is one 64-column window");
  RangeCands rc;  // wave t < NTW: trial t's candidates over this column range
  if (CAND) rc.init(c0 * 64, min(c1 * 64, rows), k);
  if (c0 >= c1) return;  // never: the host sets nsplit = ceil(nchunk / chunks_per_wg)

  // A operand hi/lo of U for both trials: slot j, k-step kc >= slot_kc0(j):
  // rows i = 16 slot_rb(j, wr) + lane%16, k = 32 kc + 8 (lane/16) + e. The
  // workgroup builds one trial's fragments at a time in LDS (the steering
  // buffers, not in use yet: [row block][k-step][hi, lo][lane] words, 64 KB),
  // all 256 threads converting R in turn, and each wave then reads its own.
  // An odd batch leaves the last pair with one trial: its second copy repeats
  // the first and stores nothing.
  uint4 ah[NTW][NFRAG], al[NTW][NFRAG];
  static_assert(8 * NKC * 2 * 64 <= 2 * CHW, "a trial's fragments fit the steering buffers");
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    const int64_t bq = pair * NTW + t < B ? pair * NTW + t : pair * NTW;
    const float2* Rb = R + bq * int64_t(M) * M;
    if (t > 0) __syncthreads();  // the previous trial's fragments have been read
    for (int it = threadIdx.x; it < 8 * NKC * 64; it += 256) {
      const int ln = it & 63, rk = it >> 6, rbg = rk / NKC, kc = rk % NKC;
      const int i = 16 * rbg + (ln & 15);
      unsigned short h[8], l[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * kc + 8 * (ln >> 4) + e;
        const float q = k < i ? 0.f : (k == i ? 0.5f : 1.f) * qval(Rb, M, MPB, i, k);
        h[e] = bf16_bits(q);
        l[e] = bf16_bits(q - __uint_as_float(unsigned(h[e]) << 16));
      }
      sXb[(rk * 2 + 0) * 64 + ln] = make_uint4(h[0] | (unsigned(h[1]) << 16), h[2] | (unsigned(h[3]) << 16),
                                               h[4] | (unsigned(h[5]) << 16), h[6] | (unsigned(h[7]) << 16));
      sXb[(rk * 2 + 1) * 64 + ln] = make_uint4(l[0] | (unsigned(l[1]) << 16), l[2] | (unsigned(l[3]) << 16),
                                               l[4] | (unsigned(l[5]) << 16), l[6] | (unsigned(l[7]) << 16));
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NSLOT; ++j)
#pragma unroll
      for (int kc = slot_kc0(j); kc < NKC; ++kc) {
        const int f = slot_off(j) + kc - slot_kc0(j), rk = slot_rb(j, wr) * NKC + kc;
        ah[t][f] = sXb[(rk * 2 + 0) * 64 + lane];
        al[t][f] = sXb[(rk * 2 + 1) * 64 + lane];
      }
  }
  __syncthreads();  // every wave holds its fragments before the steering DMA reuses the buffers

#define BA_FETCH(c, buf)                                                                  \
  do {                                                                                    \
    _Pragma("unroll") for (int f_ = 0; f_ < CHW / 4 / 64; ++f_) {                         \
      const int o_ = wave * (CHW / 4) + f_ * 64;                                          \
      lds_dma16(Xb + int64_t(c) * CHW + o_ + lane, sXb + (buf) * CHW + o_);               \
    }                                                                                     \
  } while (0)

  BA_FETCH(c0, 0);
  lds_dma_wait();
  __syncthreads();
  const float scale = 2.0f / float(M * M);  // P = 2 x^T U x / M^2
  // epilogue: lane holds D rows 16 rbg + 4 (lane/16) + e, column lane%16; in the
  // B layout those are 4 consecutive values of one 16-byte word
  const int ew = (lane >> 5) * 16 + (lane & 15), eh = (lane >> 4) & 1;
  for (int c = c0; c < c1; ++c) {
    const int buf = (c - c0) & 1;
    if (c + 1 < c1) BA_FETCH(c + 1, buf ^ 1);
    // each B fragment and epilogue row read from LDS serves both trials
#pragma unroll
    for (int jj = 0; jj < NBB / 2; ++jj) {
      const int jb = 2 * jj + wc;
      const uint4* bx = sXb + buf * CHW + jb * BLKW;
      floatx4 acc[NTW][NSLOT];
#pragma unroll
      for (int t = 0; t < NTW; ++t)
#pragma unroll
        for (int j = 0; j < NSLOT; ++j) acc[t][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc) {
        const bf16x8 bh = __builtin_bit_cast(bf16x8, lds_frag(bx, (2 * kc) * 64 + lane));
        const bf16x8 bl = __builtin_bit_cast(bf16x8, lds_frag(bx, (2 * kc + 1) * 64 + lane));
        // pass-major over the (trial, slot) accumulators: consecutive MFMAs
        // write different accumulators
#pragma unroll
        for (int pass = 0; pass < (PREC == BA_PREC_BF16X3 ? 3 : 1); ++pass)
#pragma unroll
          for (int t = 0; t < NTW; ++t)
#pragma unroll
            for (int j = 0; j < NSLOT; ++j) {
              if (kc < slot_kc0(j)) continue;
              const int f = slot_off(j) + kc - slot_kc0(j);
              const bf16x8 va = __builtin_bit_cast(bf16x8, pass == 2 ? al[t][f] : ah[t][f]);
              acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, pass == 1 ? bl : bh, acc[t][j], 0, 0, 0);
            }
      }
      float part[NTW];
#pragma unroll
      for (int t = 0; t < NTW; ++t) part[t] = 0.f;
#pragma unroll
      for (int j = 0; j < NSLOT; ++j) {
        const int rbg = slot_rb(j, wr), kc = rbg >> 1;
        const int w = (rbg & 1) * 32 + ew;
        const uint2 xh = lds_frag(reinterpret_cast<const uint2*>(bx + (kc * 2) * 64 + w), eh);
        const uint2 xl = lds_frag(reinterpret_cast<const uint2*>(bx + (kc * 2 + 1) * 64 + w), eh);
        const float x0 = lo_half(xh.x) + lo_half(xl.x), x1 = hi_half(xh.x) + hi_half(xl.x);
        const float x2 = lo_half(xh.y) + lo_half(xl.y), x3 = hi_half(xh.y) + hi_half(xl.y);
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
          part[t] += x0 * acc[t][j][0];
          part[t] += x1 * acc[t][j][1];
          part[t] += x2 * acc[t][j][2];
          part[t] += x3 * acc[t][j][3];
        }
      }
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        float v = part[t];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (lane < 16) red[buf][t][wr][jb * 16 + lane] = v;
      }
    }
    lds_dma_wait();
    __syncthreads();
    if (threadIdx.x < NTW * NBB * 16) {
      const int t = threadIdx.x % (NBB * 16), tw = threadIdx.x / (NBB * 16);
      const int64_t bo = pair * NTW + tw;
      const int64_t g = int64_t(c) * NBB * 16 + t;
      const float v = (red[buf][tw][0][t] + red[buf][tw][1][t]) * scale;
      if (CAND) {
        float vw[1] = {v};
        if (P && bo < B && g < G) P[bo * G + g] = v;
        window_candidates<64, 1>(rc, vw, c * 64, c == c0, lane);  // wave tw, trial tw
      } else if (bo < B && g < G) {
        P[bo * G + g] = v;
      }
    }
  }
#undef BA_FETCH
  if (CAND && wave < NTW) {
    const int64_t bo = pair * NTW + wave;
    if (bo < B) {
      float4* o = rec + (bo * nsplit + sp) * (k + 1);
      if (lane < k) o[lane] = make_float4(rc.lv, __int_as_float(rc.li), rc.ll, rc.lr);
      if (lane == 0) o[k] = make_float4(rc.e[0], rc.e[1], rc.e[2], rc.e[3]);
    }
  }
}

}  // namespace

// column ranges per trial pair: split until there are 2048 workgroups, at
// most max_split ranges
void qb_split(const Plan& p, int B, int max_split, int* nsplit_out, int* per_out) {
  const int nchunk = int((p.Gb + NBB - 1) / NBB);
  const int64_t pairs = (int64_t(std::max(B, 1)) + NTW - 1) / NTW;
  int nsplit = 1;
  while (pairs * nsplit < 2048 && nsplit < nchunk && 2 * nsplit <= max_split) nsplit *= 2;
  const int per = (nchunk + nsplit - 1) / nsplit;
  *per_out = per;
  *nsplit_out = (nchunk + per - 1) / per;
}

hipError_t launch_spectrum_qb_candidates(const Plan& p, int B, const float2* R, float* P, int k, float4* rec,
                                         hipStream_t s) {
  if (p.Mp != MPB || !p.d_Xb) return hipErrorInvalidValue;
  if (B == 0) return hipSuccess;
  const int nchunk = int((p.Gb + NBB - 1) / NBB);
  if (int64_t(nchunk) * NBB > p.Xblocks) return hipErrorInvalidValue;
  const CandLayout L = candidate_layout(p, B);
  if (L.span != int64_t(L.per) * NBB * 16) return hipErrorInvalidValue;
  const int64_t nblk = (int64_t(B) + NTW - 1) / NTW * L.nsplit;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = 2 * CHW * sizeof(uint4);
  const uint4* Xb = reinterpret_cast<const uint4*>(p.d_Xb);
  if (p.precision == BA_PREC_BF16X3)
    hipLaunchKernelGGL((k_proj_qb<BA_PREC_BF16X3, true>), dim3(unsigned(nblk)), dim3(256), lds, s, R, Xb, P, B, p.M,
                       p.G, nchunk, L.per, L.nsplit, p.rows, k, rec);
  else
    hipLaunchKernelGGL((k_proj_qb<BA_PREC_BF16, true>), dim3(unsigned(nblk)), dim3(256), lds, s, R, Xb, P, B, p.M,
                       p.G, nchunk, L.per, L.nsplit, p.rows, k, rec);
  return hipGetLastError();
}

hipError_t launch_spectrum_qb(const Plan& p, int B, const float2* R, float* P, hipStream_t s) {
  if (p.Mp != MPB || !p.d_Xb) return hipErrorInvalidValue;
  if (B == 0) return hipSuccess;
  // chunks stay inside the table: it holds a whole number of 32-block groups
  const int nchunk = int((p.Gb + NBB - 1) / NBB);
  if (int64_t(nchunk) * NBB > p.Xblocks) return hipErrorInvalidValue;
  const int64_t pairs = (int64_t(B) + NTW - 1) / NTW;
  int nsplit = 1, per = nchunk;
  qb_split(p, B, INT_MAX, &nsplit, &per);
  const int64_t nblk = pairs * nsplit;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = 2 * CHW * sizeof(uint4);
  const uint4* Xb = reinterpret_cast<const uint4*>(p.d_Xb);
  if (p.precision == BA_PREC_BF16X3)
    hipLaunchKernelGGL(k_proj_qb<BA_PREC_BF16X3>, dim3(unsigned(nblk)), dim3(256), lds, s, R, Xb, P, B, p.M, p.G,
                       nchunk, per, nsplit);
  else
    hipLaunchKernelGGL(k_proj_qb<BA_PREC_BF16>, dim3(unsigned(nblk)), dim3(256), lds, s, R, Xb, P, B, p.M, p.G,
                       nchunk, per, nsplit);
  return hipGetLastError();
}

}  // namespace ba
