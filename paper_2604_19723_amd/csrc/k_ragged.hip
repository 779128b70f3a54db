// Uneven batches in one persistent launch: covariance -> Bartlett spectrum ->
// peaks, trial by trial, for trials of different element counts, snapshot
// counts and source counts (the Sec. IV-D.2 grid search run for many
// heterogeneous realisations at once).
//
// Each workgroup (8 waves, 160 KB LDS) takes the next trial from an atomic
// ticket; trials are ordered longest first on the host, so the tail of the
// launch is made of short trials. Per trial, everything stays on the CU:
//  1. covariance route: R = (1/T) sum_t y_t y_t^H into LDS on the vector ALUs
//     (snapshot chunks staged in LDS, 4 x BN register blocks over the upper
//     triangle, the snapshot range split over thread groups when the matrix
//     is small, partial sums combined in a fixed order; the matrix-core
//     Gram form for the 64- and 128-element classes); the upper triangle U
//     of Q = [[Rr, -Ri], [Ri, Rr]] (diagonal halved, x^T Q x = 2 x^T U x)
//     then goes into MFMA A-operand registers;
//     snapshot route (few snapshots): the A operand is S = [[Yr, Yi],
//     [Yi, -Yr]] read straight from the snapshots, rows 2T instead of 2M;
//  2. projection on v_mfma_f32_16x16x4f32 against the steering table of the
//     trial's size class (the first Mp elements of the plan's geometry:
//     exact, a per-point phase common to all elements cancels in |a^H y|^2),
//     the epilogue forming 2 x^T (U x) or sum |S x|^2 into an LDS spectrum row;
//  3. peak pick and FP64 refinement from that LDS row.
//
// Packed small trials: a trial of at most 32 elements on a 1-D grid (when the
// host packs its class) runs inside one wave, and a workgroup takes eight of
// them per ticket. Each wave has 16 KB of LDS of its own and never waits for
// the other waves: the covariance as the real Gram matrix of the snapshots on
// the matrix cores, U into A-operand registers, the projection against the
// class table streamed into its LDS by DMA (waits on its own counters only),
// and the peaks gathered from the spectrum as it is produced (64-column
// windows across the lanes, a top-k list, the end columns with the row's
// wrap), so no spectrum row is kept.
#include <climits>

#include "cand_window.h"
#include "proj_common.h"
#include "ragged.h"

namespace ba {
namespace {

constexpr int kThreads = 512;
constexpr int kOffP = 64 * 1024;      // spectrum row (<= 64 KB)
constexpr int kOffRed = 128 * 1024;   // cross-wave partial sums (<= 32 KB)
constexpr int kOffY = 128 * 1024;     // snapshot staging during the covariance (24 KB)
constexpr int kStageBytes = 24 * 1024;

template <int MP>
struct RC {
  static constexpr int K = 2 * MP;
  static constexpr int KS = K / 4;
  static constexpr int NRB = K / 16;
  static constexpr int BLK = K * 16;
  static constexpr int NB = 8192 / BLK;
  static constexpr int CH4 = 2048;
  static constexpr int F4 = CH4 / kThreads;
};

__device__ __forceinline__ bool better(float va, int ia, float vb, int ib) {
  return va > vb || (va == vb && ia < ib);
}

__device__ __forceinline__ int wrap_row(int j0, int rows) {
  return j0 < 0 ? j0 + rows : (j0 >= rows ? j0 - rows : j0);
}

__device__ double parabolic(double pm, double p0, double pp) {
#pragma clang fp contract(off)
  const double den = pm - 2.0 * p0 + pp;
  if (den == 0.0 || !isfinite(den)) return 0.0;
  const double d = 0.5 * (pm - pp) / den;
  return d > 0.5 ? 0.5 : (d < -0.5 ? -0.5 : d);
}

// ---------------------------------------------------------------- covariance

template <int BN>
__device__ __forceinline__ void covariance_lds(const float2* __restrict__ Yb, int M, int T, unsigned char* smem) {
  constexpr int BM = 4;
  float2* sR = reinterpret_cast<float2*>(smem);
  float2* sPart = sR + M * M;
  float2* sY = reinterpret_cast<float2*>(smem + kOffY);
  const int tid = threadIdx.x;
  const int nbm = (M + BM - 1) / BM, nbn = (M + BN - 1) / BN;
  int n_bp = 0;
  for (int bn = 0; bn < nbn; ++bn) n_bp += min(nbm - 1, (BN * bn + BN - 1) / BM) + 1;
  // thread groups split the snapshots when the matrix is small (at most 32
  // groups, and no more than there are snapshots); every group's partial sums
  // go to LDS between R and the snapshot staging area, and the combine is
  // spread over all threads, one output value each, summed in group order
  // (deterministic)
  const int part_bytes = n_bp * BM * BN * 8;
  const int room = (kOffY - M * M * 8) / part_bytes;
  const int n_tg = max(1, min(min(kThreads / n_bp, room), min(32, T)));
  const int bp = tid % n_bp, tg = tid / n_bp;
  const bool active = tg < n_tg && tid < n_bp * n_tg;
  auto block_of = [&](int pair, int& bm_out, int& bn_out) {
    int r = pair, c = 0;
    for (bn_out = 0; bn_out < nbn; ++bn_out) {
      c = min(nbm - 1, (BN * bn_out + BN - 1) / BM) + 1;
      if (r < c) break;
      r -= c;
    }
    bm_out = r;
  };
  int bm = 0, bn = 0;
  block_of(bp, bm, bn);
  float ar[BM][BN], ai[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) ar[i][j] = ai[i][j] = 0.f;

  const int TC = kStageBytes / (M * 8);
  for (int t0 = 0; t0 < T; t0 += TC) {
    const int nt = min(TC, T - t0);
    for (int v = tid; v < TC * M; v += kThreads) {
      const int tt = v / M;
      sY[v] = tt < nt ? Yb[int64_t(t0) * M + v] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    if (active) {
      for (int tt = tg; tt < nt; tt += n_tg) {
        const float2* yt = sY + tt * M;
        float2 ym[BM], yn[BN];
#pragma unroll
        for (int i = 0; i < BM; ++i) {
          const int m = BM * bm + i;
          ym[i] = m < M ? yt[m] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int n = BN * bn + j;
          yn[j] = n < M ? yt[n] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
          for (int j = 0; j < BN; ++j) {
            // ym * conj(yn)
            ar[i][j] += ym[i].x * yn[j].x + ym[i].y * yn[j].y;
            ai[i][j] += ym[i].y * yn[j].x - ym[i].x * yn[j].y;
          }
      }
    }
    __syncthreads();
  }
  if (active) {
    float2* dst = sPart + (int64_t(tg) * n_bp + bp) * (BM * BN);
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) dst[i * BN + j] = make_float2(ar[i][j], ai[i][j]);
  }
  __syncthreads();
  const float invT = 1.0f / float(T);
  for (int pe = tid; pe < n_bp * BM * BN; pe += kThreads) {
    const int pr = pe / (BM * BN), e = pe % (BM * BN);
    float2 acc = make_float2(0.f, 0.f);
    for (int g2 = 0; g2 < n_tg; ++g2) {
      const float2 v = sPart[(int64_t(g2) * n_bp + pr) * (BM * BN) + e];
      acc.x += v.x;
      acc.y += v.y;
    }
    int pbm = 0, pbn = 0;
    block_of(pr, pbm, pbn);
    const int m = BM * pbm + e / BN, n = BN * pbn + e % BN;
    if (m < M && n < M && m <= n) {
      const float re = acc.x * invT;
      const float im = (m == n) ? 0.f : acc.y * invT;
      sR[m * M + n] = make_float2(re, im);
      sR[n * M + m] = make_float2(re, -im);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- one trial
//
// The projection of each size class is inlined into the kernel body, where
// the compiler sees every LDS access against the kernel's own LDS block and
// can tell the chunk being read from the chunk in flight; the covariance and
// the peak pick stay out of line (their registers do not add to the
// projection's, and the peak pick is one routine for every class).

template <int BN>
__device__ __attribute__((noinline)) void stage_covariance(const float2* __restrict__ Yb, int M, int T,
                                                           unsigned char* smem) {
  covariance_lds<BN>(Yb, M, T, smem);
}

// Direct global -> LDS copy of 4 bytes per lane (global_load_lds_dword): lane
// i's word lands at lds_wave + 4 i (lds_wave wave-uniform); completion is
// tracked by vmcnt like lds_dma16.
__device__ __forceinline__ void lds_dma4(const void* gsrc_lane, void* lds_wave) {
  __builtin_amdgcn_global_load_lds(gsrc_lane, reinterpret_cast<__attribute__((address_space(3))) void*>(
                                                  reinterpret_cast<uintptr_t>(lds_wave)),
                                   4, 0, 0);
}

// Covariance of the larger classes on the matrix cores: the real Gram matrix
// G = sum_t z_t z_t^T of the snapshots' float views (re, im interleaved), with
//   Re R[m][n] = G[2m][2n] + G[2m+1][2n+1],  Im R[m][n] = G[2m+1][2n] - G[2m][2n+1],
// written to the LDS matrix R (exactly Hermitian). The 16x16 Gram tiles on or
// above the diagonal go to the waves as tile-row pairs (RA, MT-1-RA), RA a
// compile-time case per wave, so the MFMA sequence has no per-tile branch and
// a wave holds only its own accumulator tiles (MT + 1; at 64 elements, with
// four pairs for eight waves, each pair's tile columns are split by parity
// over two waves, 4 and 5 tiles). R is written only after
// the last snapshot, so the snapshot stages use all of the LDS: two buffers
// of TC rows (68 snapshots at 128 elements, 132 at 64; row stride 2 MP + 16
// floats, so the four k-rows of a fragment fall on different bank quarters),
// the next stage streamed in by LDS DMA while the current one is multiplied
// (one 16-byte DMA per row when the rows are 16-byte aligned, 4-byte words
// otherwise: a row of 2M floats is copied exactly, nothing past the trial's
// block is read), one barrier per stage; within a stage the next k-step's
// fragments are read while the current one is multiplied. Columns past 2M
// keep stale values: a Gram entry reads only its own two columns, and those
// entries are never used. Rows past T up to the next multiple of 4 are zeroed.
template <int MT>
struct GramCfg {
  static constexpr int W = 16 * MT;                               // Gram columns = 2 MP
  static constexpr int LD = W + 16;
  static constexpr int TC = ((kRaggedLds / 2) / (LD * 4)) & ~3;   // snapshots per stage buffer
  static_assert(2 * TC * LD * 4 <= kRaggedLds && TC >= 4, "two stage buffers fit the LDS");
};

// Tile rows (RA, MT - 1 - RA), the tile columns c with c % NH == H of them
// (NH = 2 splits a pair over two waves when there are fewer pairs than
// waves); RA < 0: a wave without Gram tiles (it streams snapshots and keeps
// the barriers).
template <int MT, int RA, int H, int NH>
__device__ __forceinline__ void gram_rows(const float* __restrict__ Yf, int M, int T, unsigned char* smem,
                                          int wave, int lane) {
  using C = GramCfg<MT>;
  constexpr int W = C::W, LD = C::LD, TC = C::TC;
  constexpr bool ACT = RA >= 0;
  constexpr int RB = ACT ? MT - 1 - RA : 0;
  constexpr bool TWO = ACT && RB != RA;
  float* sZ = reinterpret_cast<float*>(smem);  // [2][TC][LD] until R is written
  float2* sR = reinterpret_cast<float2*>(smem);
  const int fi = lane & 15, fk = lane >> 4;
  const int nst = (T + TC - 1) / TC;
  floatx4 accA[MT], accB[MT];
#pragma unroll
  for (int c = 0; c < MT; ++c) {
    accA[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    accB[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  }

  // rows t0 .. t0 + nrow - 1 of stage st into buffer buf, spread over the
  // waves: a whole row per 16-byte DMA when every row starts on 16 bytes (M
  // even, the block 16-byte aligned), else 64 floats of a row per 4-byte DMA;
  // the rows up to the next multiple of 4 past T are zeroed with plain stores
  const bool wide = (M & 1) == 0 && (reinterpret_cast<uintptr_t>(Yf) & 15) == 0;
  auto fetch = [&](int st, int buf) {
    const int t0 = st * TC;
    const int nrow = min(TC, T - t0);
    float* dst = sZ + buf * (TC * LD);
    if (wide) {
      for (int r = wave; r < nrow; r += kThreads / 64)
        if (lane < M / 2) lds_dma16(Yf + (int64_t(t0 + r) * M) * 2 + 4 * lane, dst + r * LD);
    } else {
      for (int it = wave; it < nrow * (W / 64); it += kThreads / 64) {
        const int r = it / (W / 64), part = it - r * (W / 64);
        const int f = part * 64 + lane;
        if (f < 2 * M) lds_dma4(Yf + (int64_t(t0 + r) * M) * 2 + f, dst + r * LD + part * 64);
      }
    }
    const int nz = ((nrow + 3) & ~3) - nrow;
    for (int e = threadIdx.x; e < nz * W; e += kThreads) dst[(nrow + e / W) * LD + e % W] = 0.f;
  };

  fetch(0, 0);
  lds_dma_wait();
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) fetch(st + 1, buf ^ 1);  // that buffer was last read before the previous barrier
    if constexpr (ACT) {
      const int nks = (min(TC, T - st * TC) + 3) >> 2;
      const float* __restrict__ zb = sZ + buf * (TC * LD);
      auto load = [&](float (&dst)[MT], int s) {
        const float* row = zb + (4 * s + fk) * LD + fi;
#pragma unroll
        for (int c = RA; c < MT; ++c)
          if (c % NH == H || c == RA || c == RB) dst[c] = lds_frag(row, 16 * c);
      };
      auto step = [&](const float (&src)[MT]) {
#pragma unroll
        for (int c = RA; c < MT; ++c) {
          if (c % NH != H) continue;
          accA[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(src[RA], src[c], accA[c], 0, 0, 0);
          if (TWO && c >= RB) accB[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(src[RB], src[c], accB[c], 0, 0, 0);
        }
      };
      float f[MT], g[MT];
      load(f, 0);
      int s = 0;
      for (; s + 2 <= nks; s += 2) {
        load(g, s + 1);
        step(f);
        if (s + 2 < nks) load(f, s + 2);
        step(g);
      }
      if (s < nks) step(f);
    }
    lds_dma_wait();
    __syncthreads();
  }
  // every stage is consumed: R overwrites the stage buffers
  if constexpr (ACT) {
    const float invT = 1.0f / float(T);
    const bool even = (lane & 1) == 0;
#pragma unroll
    for (int h = 0; h < (TWO ? 2 : 1); ++h) {
      const int r = h == 0 ? RA : RB;
#pragma unroll
      for (int c = 0; c < MT; ++c) {
        if (c < r || c % NH != H) continue;
        const floatx4 a = h == 0 ? accA[c] : accB[c];
        floatx4 x;
#pragma unroll
        for (int e = 0; e < 4; ++e) x[e] = __shfl_xor(a[e], 1, 64);
        if (!even) continue;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int m = 8 * r + 2 * fk + q;
          const int n = 8 * c + (fi >> 1);
          if (m >= M || n >= M || m > n) continue;
          const float re = (a[2 * q] + x[2 * q + 1]) * invT;
          const float im = m == n ? 0.f : (a[2 * q + 1] - x[2 * q]) * invT;
          sR[m * M + n] = make_float2(re, im);
          if (m != n) sR[n * M + m] = make_float2(re, -im);
        }
      }
    }
  }
  __syncthreads();
}

template <int MT>
__device__ __attribute__((noinline)) void stage_covariance_gram(const float2* __restrict__ Yb, int M_arg, int T_arg,
                                                                unsigned char* smem) {
  // the sizes and the wave index are the same in every lane: scalar loop control
  const int M = __builtin_amdgcn_readfirstlane(M_arg), T = __builtin_amdgcn_readfirstlane(T_arg);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const float* Yf = reinterpret_cast<const float*>(Yb);
  static_assert(kThreads / 64 == 8 && MT <= 16, "eight waves cover the tile-row pairs");
  // MT / 2 pairs: one per wave at 16 tile rows; at 8 each pair's columns are
  // split by parity over waves w and w + 4 (9 tiles -> 4 and 5)
  constexpr int NH = MT >= 16 ? 1 : 2;
  constexpr int NP = (MT + 1) / 2;  // tile-row pairs
#define BA_GRAM_WAVE(w)                                                                            \
  case w:                                                                                          \
    if constexpr (w < NP * NH)                                                                     \
      gram_rows<MT, (w % NP), (w / NP), NH>(Yf, M, T, smem, wave, lane);                           \
    else                                                                                           \
      gram_rows<MT, -1, 0, NH>(Yf, M, T, smem, wave, lane);                                        \
    break;
  switch (wave) {
    BA_GRAM_WAVE(0)
    BA_GRAM_WAVE(1)
    BA_GRAM_WAVE(2)
    BA_GRAM_WAVE(3)
    BA_GRAM_WAVE(4)
    BA_GRAM_WAVE(5)
    BA_GRAM_WAVE(6)
    BA_GRAM_WAVE(7)
  }
#undef BA_GRAM_WAVE
}

// MFMAs of one 16-column block for a wave's two row blocks: W0 >= 0 is the
// covariance route's pair (W0, NRB - 1 - W0), whose blocks skip the k-steps
// left of their diagonal (compile-time, no branch per step); W0 < 0 takes
// every k-step for both (snapshot route).
template <int MP, int W0>
__device__ __forceinline__ void pair_chunk_mfma(floatx4 (&acc)[2], const float (&a)[2][RC<MP>::KS],
                                                const float4* __restrict__ bx, int lane) {
  using C = RC<MP>;
  constexpr int S0 = W0 >= 0 ? W0 : 0, S1 = W0 >= 0 ? C::NRB - 1 - W0 : 0;
#pragma unroll
  for (int s4 = S0 < S1 ? S0 : S1; s4 < C::KS / 4; ++s4) {
    const float4 bv = bx[s4 * 64 + lane];
    if (s4 >= S0) {
      acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][4 * s4 + 0], bv.x, acc[0], 0, 0, 0);
      acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][4 * s4 + 1], bv.y, acc[0], 0, 0, 0);
      acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][4 * s4 + 2], bv.z, acc[0], 0, 0, 0);
      acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][4 * s4 + 3], bv.w, acc[0], 0, 0, 0);
    }
    if (s4 >= S1) {
      acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1][4 * s4 + 0], bv.x, acc[1], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1][4 * s4 + 1], bv.y, acc[1], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1][4 * s4 + 2], bv.z, acc[1], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1][4 * s4 + 3], bv.w, acc[1], 0, 0, 0);
    }
  }
}

// the chunk loop for NACT active row blocks per wave (a prefix of its RB,
// row blocks rbg[0] < rbg[1]); on the covariance route the A operand is the
// upper triangle U of Q, and row block rbg skips the k-steps left of its
// diagonal block (uniform branches: cov and rbg are scalar)
template <int MP, int WR, int NACT, int RB>
__device__ __forceinline__ void project_chunks(const RArgs& A, const float4* __restrict__ Xg, int nchunk,
                                               const float (&a)[RB][RC<MP>::KS], bool cov, float scale,
                                               const int (&rbg)[RB], float* __restrict__ Pout,
                                               unsigned char* smem) {
  using C = RC<MP>;
  constexpr int WC = (kThreads / 64) / WR;
  // the wave index through a scalar register: the pair switch below is uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int wr = wave % WR, wc = wave / WR;
  float4* sX = reinterpret_cast<float4*>(smem);
  float* sP = reinterpret_cast<float*>(smem + kOffP);
  float* red = reinterpret_cast<float*>(smem + kOffRed);  // [2][WR][NB*16]

  // table chunks (32 KB) arrive by LDS DMA, one chunk ahead: 8 waves x 4 x 64 lanes x 16 bytes
#define BA_FETCH_X(c, buf)                                                                    \
  do {                                                                                        \
    _Pragma("unroll") for (int f_ = 0; f_ < C::CH4 / kThreads; ++f_) {                        \
      const int o_ = wave * (C::CH4 / 8) + f_ * 64;                                           \
      lds_dma16(Xg + int64_t(c) * C::CH4 + o_ + lane, sX + (buf) * C::CH4 + o_);              \
    }                                                                                         \
  } while (0)
  BA_FETCH_X(0, 0);
  lds_dma_wait();
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) BA_FETCH_X(c + 1, buf ^ 1);
    const float4* xb4 = sX + buf * C::CH4;
    const float* xbf = reinterpret_cast<const float*>(xb4);
    for (int jb = wc; jb < C::NB; jb += WC) {
      floatx4 acc[NACT > 0 ? NACT : 1];
#pragma unroll
      for (int rb = 0; rb < NACT; ++rb) acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
      const float4* bx = xb4 + jb * (C::BLK / 4);
      if constexpr (NACT == 2 && RB == 2) {
        if (cov) {
          // the covariance route's pair (wr, NRB - 1 - wr) as a compile-time
          // case: the k-steps left of each block's diagonal are dropped
          // without a branch per step
          static_assert(WR <= 8, "pair cases");
          switch (wr) {
            case 0: pair_chunk_mfma<MP, 0>(acc, a, bx, lane); break;
            case 1: if constexpr (WR > 1) pair_chunk_mfma<MP, 1>(acc, a, bx, lane); break;
            case 2: if constexpr (WR > 2) pair_chunk_mfma<MP, 2>(acc, a, bx, lane); break;
            case 3: if constexpr (WR > 3) pair_chunk_mfma<MP, 3>(acc, a, bx, lane); break;
            case 4: if constexpr (WR > 4) pair_chunk_mfma<MP, 4>(acc, a, bx, lane); break;
            case 5: if constexpr (WR > 5) pair_chunk_mfma<MP, 5>(acc, a, bx, lane); break;
            case 6: if constexpr (WR > 6) pair_chunk_mfma<MP, 6>(acc, a, bx, lane); break;
            default: if constexpr (WR > 7) pair_chunk_mfma<MP, 7>(acc, a, bx, lane); break;
          }
        } else {
          pair_chunk_mfma<MP, -1>(acc, a, bx, lane);
        }
      } else {
#pragma unroll
        for (int s4 = 0; s4 < C::KS / 4; ++s4) {
          if (NACT == 0) break;
          if (cov && s4 < rbg[0]) continue;
          const float4 bv = bx[s4 * 64 + lane];
#pragma unroll
          for (int rb = 0; rb < NACT; ++rb) {
            if (cov && s4 < rbg[rb]) continue;
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 0], bv.x, acc[rb], 0, 0, 0);
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 1], bv.y, acc[rb], 0, 0, 0);
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 2], bv.z, acc[rb], 0, 0, 0);
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 3], bv.w, acc[rb], 0, 0, 0);
          }
        }
      }
      float part = 0.f;
#pragma unroll
      for (int rb = 0; rb < NACT; ++rb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (cov) {
            const int i = 16 * rbg[rb] + 4 * (lane >> 4) + r;
            const int s = i >> 2;
            const float xv = xbf[jb * C::BLK + ((s >> 2) * 64 + r * 16 + (lane & 15)) * 4 + (s & 3)];
            part += xv * acc[rb][r];
          } else {
            part += acc[rb][r] * acc[rb][r];
          }
        }
      }
      part += __shfl_xor(part, 16, 64);
      part += __shfl_xor(part, 32, 64);
      if (lane < 16) red[(buf * WR + wr) * (C::NB * 16) + jb * 16 + lane] = part;
    }
    lds_dma_wait();
    __syncthreads();
    for (int t = threadIdx.x; t < C::NB * 16; t += kThreads) {
      float sum = 0.f;
#pragma unroll
      for (int w = 0; w < WR; ++w) sum += red[(buf * WR + w) * (C::NB * 16) + t];
      const int64_t g = int64_t(c) * C::NB * 16 + t;
      if (g < A.G) {
        const float p = sum * scale;
        sP[g] = p;
        if (Pout) Pout[g] = p;
      }
    }
  }
#undef BA_FETCH_X
  __syncthreads();  // spectrum row complete
}

template <int MP, int WR>
__device__ __forceinline__ void trial_project(const RArgs& A, const RItem& it, const float4* __restrict__ Xg,
                                              int nchunk, unsigned char* smem) {
  using C = RC<MP>;
  constexpr int RB = (C::NRB + WR - 1) / WR;  // row blocks per wave (round-robin)
  const int lane = threadIdx.x & 63;
  // the wave index is uniform: taking it through a scalar register keeps the
  // active-block count below in scalar registers too
  const int wr = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) % WR;
  const int M = it.M, T = it.T;
  const float2* Yb = A.Y + it.y_off;
  const bool cov = __builtin_amdgcn_readfirstlane(it.route) == kRouteCov;
  // row blocks of this wave: with two per wave the pair (wr, NRB - 1 - wr),
  // whose spans right of the diagonal add up to NRB + 1 blocks for every wr
  static_assert(RB == 1 || RB * WR == C::NRB, "pairs cover the row blocks");
  int rbg[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) rbg[rb] = rb == 0 ? wr : C::NRB - 1 - wr;
  const int Tp = (T + 7) & ~7;
  const int nrb_act = cov ? C::NRB : min(C::NRB, Tp / 8);

  // 1. A operand
  float a[RB][C::KS];
  if (cov) {
    if constexpr (MP >= 64)
      stage_covariance_gram<MP / 8>(Yb, M, T, smem);
    else
      stage_covariance<4>(Yb, M, T, smem);
    const float2* sR = reinterpret_cast<const float2*>(smem);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int s = 0; s < C::KS; ++s) {
        // U: Q right of the diagonal, half the diagonal, zero left of it
        const int i = 16 * rbg[rb] + (lane & 15);
        const int k = 4 * s + (lane >> 4);
        const bool iim = i >= MP, kim = k >= MP;
        const int ir = iim ? i - MP : i, kr = kim ? k - MP : k;
        float q = 0.f;
        if (k >= i && i < C::K && ir < M && kr < M) {
          const float2 r = sR[ir * M + kr];
          q = (iim == kim) ? r.x : (iim ? r.y : -r.y);
          if (k == i) q *= 0.5f;
        }
        a[rb][s] = q;
      }
  } else {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int s = 0; s < C::KS; ++s) {
        const int i = 16 * rbg[rb] + (lane & 15);
        const int k = 4 * s + (lane >> 4);
        const bool second = i >= Tp;
        const int t = second ? i - Tp : i;
        const bool kim = k >= MP;
        const int m = kim ? k - MP : k;
        float q = 0.f;
        if (i < 2 * Tp && t < T && m < M) {
          const float2 y = Yb[int64_t(t) * M + m];
          // rows t: [Yr, Yi]; rows Tp + t: [Yi, -Yr]
          q = second ? (kim ? -y.x : y.y) : (kim ? y.y : y.x);
        }
        a[rb][s] = q;
      }
  }
  __syncthreads();  // LDS covariance consumed

  // 2. projection over the active row blocks of this wave (rbg[rb] < nrb_act);
  // the covariance route's sums are x^T U x = (x^T Q x) / 2
  const float scale = cov ? 2.0f / float(M * M) : 1.0f / (float(T) * float(M * M));
  float* Pout = A.P ? A.P + int64_t(it.trial) * A.G : nullptr;
  int nact = 0;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) nact += (rbg[rb] < nrb_act) ? 1 : 0;
  static_assert(RB <= 2, "row blocks per wave");
  if (nact == RB)
    project_chunks<MP, WR, RB, RB>(A, Xg, nchunk, a, cov, scale, rbg, Pout, smem);
  else if (RB == 2 && nact == 1)
    project_chunks<MP, WR, (RB == 2 ? 1 : 0), RB>(A, Xg, nchunk, a, cov, scale, rbg, Pout, smem);
  else
    project_chunks<MP, WR, 0, RB>(A, Xg, nchunk, a, cov, scale, rbg, Pout, smem);
}

// 3. peaks from the LDS row (same rule as the standalone peak kernel). Grid
// indices fit 32 bits (rows x s1 <= 16384); a 1-D row needs no division.
// Each thread keeps a sorted list of its best KC maxima; each wave then
// selects its own best K by K butterfly rounds over its lanes' list heads (no
// barriers), and wave 0 selects the trial's best K from the eight wave lists.
// Every list holds at least K entries, so the result is the top K of the row
// under the same total order.
__device__ __forceinline__ void offer_local(float p, int g, float (&lv)[kRaggedMaxPeaks],
                                            int (&li)[kRaggedMaxPeaks]) {
#pragma unroll
  for (int j = kRaggedMaxPeaks - 1; j >= 0; --j) {
    if (j > 0 && better(p, g, lv[j - 1], li[j - 1])) {
      lv[j] = lv[j - 1];
      li[j] = li[j - 1];
    } else if (better(p, g, lv[j], li[j])) {
      lv[j] = p;
      li[j] = g;
    }
  }
}

__device__ __forceinline__ void wave_best(float& v, int& i) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(v, off, 64);
    const int oi = __shfl_xor(i, off, 64);
    if (better(ov, oi, v, i)) {
      v = ov;
      i = oi;
    }
  }
}

__device__ __attribute__((noinline)) void trial_peaks(const RArgs& A, const RItem& it, unsigned char* smem) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float* sP = reinterpret_cast<const float*>(smem + kOffP);
  constexpr int KC = kRaggedMaxPeaks;
  float lv[KC];
  int li[KC];
#pragma unroll
  for (int j = 0; j < KC; ++j) {
    lv[j] = -INFINITY;
    li[j] = INT_MAX;
  }
  const int s1 = A.s1, rows = A.rows, wrap0 = A.wrap0;
  if (s1 == 1) {
    for (int g = threadIdx.x; g < rows; g += kThreads) {
      const float p = sP[g];
      if (p != p) continue;
      bool ok = true;
      if (wrap0 || g > 0) ok = p > sP[wrap_row(g - 1, rows)];
      if (wrap0 || g + 1 < rows) ok = ok && p >= sP[wrap_row(g + 1, rows)];
      if (ok) offer_local(p, g, lv, li);
    }
  } else {
    const int ncand = rows * s1;
    for (int g = threadIdx.x; g < ncand; g += kThreads) {
      const float p = sP[g];
      if (p != p) continue;
      const int i0 = g / s1, i1 = g - i0 * s1;
      bool ok = true;
      for (int di = -1; di <= 1; ++di) {
        int j0 = i0 + di;
        if (wrap0)
          j0 = wrap_row(j0, rows);
        else if (j0 < 0 || j0 >= rows)
          continue;
        for (int dj = -1; dj <= 1; ++dj) {
          if (di == 0 && dj == 0) continue;
          const int j1 = i1 + dj;
          if (j1 < 0 || j1 >= s1) continue;
          const float q = sP[j0 * s1 + j1];
          const bool earlier = di < 0 || (di == 0 && dj < 0);
          ok = ok && (earlier ? (p > q) : (p >= q));
        }
      }
      if (ok) offer_local(p, g, lv, li);
    }
  }
  // each wave's best K: round r takes the best list head of the wave
  float* wv = reinterpret_cast<float*>(smem + kOffRed);              // [8][KC]
  int* wi = reinterpret_cast<int*>(smem + kOffRed + 8 * KC * 4);     // [8][KC]
  const int K = it.K;
  int head = 0;
  for (int r = 0; r < K; ++r) {
    float v = -INFINITY;
    int i = INT_MAX;
#pragma unroll
    for (int j = 0; j < KC; ++j)
      if (j == head) {
        v = lv[j];
        i = li[j];
      }
    const int hi = i;
    wave_best(v, i);
    if (i != INT_MAX && hi == i) ++head;  // grid indices are unique: this lane's head won
    if (lane == 0) {
      wv[wave * KC + r] = v;
      wi[wave * KC + r] = i;
    }
  }
  __syncthreads();
  if (wave == 0) {
    // lane l holds entry l % K of wave l / K's list (K <= 8: all 64 fit)
    float cv = -INFINITY;
    int ci = INT_MAX;
    if (lane < (kThreads / 64) * K) {
      cv = wv[(lane / K) * KC + lane % K];
      ci = wi[(lane / K) * KC + lane % K];
    }
    float selv = -INFINITY;
    int seli = INT_MAX;
    for (int r = 0; r < K; ++r) {
      float v = cv;
      int i = ci;
      wave_best(v, i);
      if (i != INT_MAX && ci == i) {
        cv = -INFINITY;
        ci = INT_MAX;
      }
      if (lane == r) {
        selv = v;
        seli = i;
      }
    }
    if (lane < A.kmax) {
      const int j = lane;
      const int64_t o = int64_t(it.trial) * A.kmax + j;
      const int g = j < K ? seli : INT_MAX;
      const double nan = __longlong_as_double(0x7ff8000000000000LL);
      if (g == INT_MAX) {
        A.idx[o] = -1;
        A.val[o] = __int_as_float(0x7fc00000);
        if (A.refined)
          for (int d = 0; d < A.ndim; ++d) A.refined[o * A.ndim + d] = nan;
      } else {
        A.idx[o] = g;
        A.val[o] = selv;
        if (A.refined) {
          const int i0 = g / s1, i1 = g - i0 * s1;
          const double p0 = double(sP[g]);
          double d0 = 0.0;
          if (wrap0 || (i0 > 0 && i0 < rows - 1)) {
            const int jm = wrap_row(i0 - 1, rows), jp = wrap_row(i0 + 1, rows);
            d0 = parabolic(double(sP[jm * s1 + i1]), p0, double(sP[jp * s1 + i1]));
          }
          A.refined[o * A.ndim] = double(i0) + d0;
          if (A.ndim == 2) {
            double d1 = 0.0;
            if (i1 > 0 && i1 < s1 - 1) d1 = parabolic(double(sP[i0 * s1 + i1 - 1]), p0, double(sP[i0 * s1 + i1 + 1]));
            A.refined[o * A.ndim + 1] = double(i1) + d1;
          }
        }
      }
    }
  }
  __syncthreads();  // LDS reused by the next trial
}

// ---------------------------------------------------------------- packed small trials

constexpr int kWaveLds = 16 * 1024;  // LDS of one wave in packed mode

// Orders this wave's LDS accesses: writes before the point are seen by reads
// after it from any lane of the wave (the LDS runs one wave's accesses in
// order), and the compiler moves no LDS access across it.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// R = (1/T) sum_t y_t y_t^H of one trial (M <= MP <= 32) into wR [M][M], by one
// wave: the real Gram matrix of the snapshots' float views (re, im
// interleaved, zero-padded to 2 MP) on v_mfma_f32_16x16x4f32, snapshot stages
// in the wave's LDS (rows of 48 or 80 floats: the four rows a fragment reads
// fall on different bank quarters), then Re R[m][n] = G[2m][2n] +
// G[2m+1][2n+1], Im R[m][n] = G[2m+1][2n] - G[2m][2n+1] (exactly Hermitian).
template <int MP>
__device__ __forceinline__ void wave_covariance(const float2* __restrict__ Yb, int M, int T, float* wz,
                                                float2* wR, int lane) {
  constexpr int W = 2 * MP;
  constexpr int MT = W / 16;  // Gram tiles per side
  constexpr int NT = MT * (MT + 1) / 2;
  constexpr int LD = W <= 32 ? 48 : 80;
  constexpr int TC = ((kWaveLds / 4) / LD) & ~3;  // snapshots per stage
  static_assert(W <= LD && TC >= 4, "stage layout");
  floatx4 acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int fi = lane & 15, fk = lane >> 4;
  for (int t0 = 0; t0 < T; t0 += TC) {
    const int nt = min(TC, T - t0);
    for (int v = lane; v < TC * MP; v += 64) {
      const int tt = v / MP, m = v - tt * MP;
      float2 y = make_float2(0.f, 0.f);
      if (tt < nt && m < M) y = Yb[int64_t(t0 + tt) * M + m];
      *reinterpret_cast<float2*>(&wz[tt * LD + 2 * m]) = y;
    }
    wave_lds_sync();
    for (int s = 0; s < (nt + 3) / 4; ++s) {  // staged rows past nt are zero
      const float* row = wz + (4 * s + fk) * LD + fi;
      float f[MT];
#pragma unroll
      for (int c = 0; c < MT; ++c) f[c] = row[16 * c];
      int q = 0;
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = a; b < MT; ++b, ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[a], f[b], acc[q], 0, 0, 0);
    }
    wave_lds_sync();
  }
  const float invT = 1.0f / float(T);
  const bool even = (lane & 1) == 0;
  int q = 0;
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = a; b < MT; ++b, ++q) {
      const floatx4 g = acc[q];
      floatx4 x;
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = __shfl_xor(g[e], 1, 64);  // the neighbouring (odd) Gram column
      if (!even) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = 8 * a + 2 * fk + h, n = 8 * b + (fi >> 1);
        if (m >= M || n >= M || m > n) continue;
        const float re = (g[2 * h] + x[2 * h + 1]) * invT;
        const float im = m == n ? 0.f : (g[2 * h + 1] - x[2 * h]) * invT;
        wR[m * M + n] = make_float2(re, im);
        if (m != n) wR[n * M + m] = make_float2(re, -im);
      }
    }
  wave_lds_sync();
}

// One packed trial (covariance route, 1-D grid) by the calling wave, in its
// LDS region wsm.
template <int MP>
__device__ __forceinline__ void wave_trial(const RArgs& A, const RItem& it, const float4* __restrict__ Xg,
                                           unsigned char* wsm, int lane) {
  using C = RC<MP>;
  constexpr int NBW = 8192 / (C::BLK * 4);  // column blocks per 8 KB chunk
  constexpr int CH4 = 512;                   // float4 per chunk
  const int M = it.M, T = it.T;
  const float2* Yb = A.Y + it.y_off;

  // 1. covariance, then U (Q right of the diagonal, half the diagonal) into
  // the A operand of both row blocks
  float2* wR = reinterpret_cast<float2*>(wsm);
  wave_covariance<MP>(Yb, M, T, reinterpret_cast<float*>(wsm), wR, lane);
  float a[C::NRB][C::KS];
#pragma unroll
  for (int rb = 0; rb < C::NRB; ++rb)
#pragma unroll
    for (int s = 0; s < C::KS; ++s) {
      const int i = 16 * rb + (lane & 15);
      const int k = 4 * s + (lane >> 4);
      const bool iim = i >= MP, kim = k >= MP;
      const int ir = iim ? i - MP : i, kr = kim ? k - MP : k;
      float q = 0.f;
      if (k >= i && ir < M && kr < M) {
        const float2 r = wR[ir * M + kr];
        q = (iim == kim) ? r.x : (iim ? r.y : -r.y);
        if (k == i) q *= 0.5f;
      }
      a[rb][s] = q;
    }
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): R is read before the DMA overwrites it
  wave_lds_sync();

  // 2. projection chunk by chunk (8 KB of the class table, the next one in
  // flight by LDS DMA), 3. peaks gathered on the way
  const int G = int(A.G), rows = A.rows;
  const int nblk = (G + 15) / 16;
  const int nch = (nblk + NBW - 1) / NBW;
  const float scale = 2.0f / float(M * M);
  float* Pout = A.P ? A.P + int64_t(it.trial) * A.G : nullptr;
  float4* sx = reinterpret_cast<float4*>(wsm);  // [2][CH4]
  auto fetch = [&](int c, int buf) {
#pragma unroll
    for (int f = 0; f < CH4 / 64; ++f) lds_dma16(Xg + int64_t(c) * CH4 + f * 64 + lane, sx + buf * CH4 + f * 64);
  };
  RangeCands rc;
  rc.init(0, rows, it.K);
  float vwin[1] = {0.f};
  fetch(0, 0);
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) {
      fetch(c + 1, buf ^ 1);  // that buffer's reads finished at the end of chunk c - 1
      __builtin_amdgcn_s_waitcnt(0x0F70 | (CH4 / 64));  // vmcnt(8): all but the chunk just issued
    } else {
      lds_dma_wait();
    }
    wave_lds_sync();
    const float4* xb4 = sx + buf * CH4;
    for (int jb = 0; jb < NBW; ++jb) {
      const int blk = c * NBW + jb;
      if (blk >= nblk) break;
      const float4* bx = xb4 + jb * (C::BLK / 4);
      const float* xf = reinterpret_cast<const float*>(bx);
      float part = 0.f;
#pragma unroll
      for (int rb = 0; rb < C::NRB; ++rb) {
        floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s4 = rb; s4 < C::KS / 4; ++s4) {  // U is zero left of the diagonal block
          const float4 bv = lds_frag(bx, s4 * 64 + lane);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 0], bv.x, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 1], bv.y, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 2], bv.z, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][4 * s4 + 3], bv.w, acc, 0, 0, 0);
        }
        // x_i (U x)_i over the row block's rows, from the same LDS block
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rb * 16 + 4 * (lane >> 4) + r;
          const int sidx = i >> 2;
          part += lds_frag(xf, ((sidx >> 2) * 64 + r * 16 + (lane & 15)) * 4 + (sidx & 3)) * acc[r];
        }
      }
      part += __shfl_xor(part, 16, 64);
      part += __shfl_xor(part, 32, 64);
      const float p = part * scale;  // every lane: column blk * 16 + lane % 16
      const int g = blk * 16 + lane;
      if (Pout && lane < 16 && g < G) Pout[g] = p;
      const int qslot = blk & 3;  // this block's quarter of its 64-column window
      if ((lane >> 4) == qslot) vwin[0] = p;
      if (qslot == 3 || blk == nblk - 1) window_candidates<64, 1>(rc, vwin, (blk >> 2) * 64, blk < 4, lane);
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this buffer's reads are done before it is refilled
    wave_lds_sync();
  }
  finish_whole_row(rc, rows, A.wrap0, lane);

  if (lane < A.kmax) {
    const int64_t o = int64_t(it.trial) * A.kmax + lane;
    if (rc.li == INT_MAX) {
      A.idx[o] = -1;
      A.val[o] = __int_as_float(0x7fc00000);
      if (A.refined) A.refined[o * A.ndim] = __longlong_as_double(0x7ff8000000000000LL);
    } else {
      A.idx[o] = rc.li;
      A.val[o] = rc.lv;
      if (A.refined) {
        double d0 = 0.0;
        if (A.wrap0 || (rc.li > 0 && rc.li < rows - 1))
          d0 = peak_parabolic(double(rc.ll), double(rc.lv), double(rc.lr));
        A.refined[o * A.ndim] = double(rc.li) + d0;
      }
    }
  }
}

// The arguments live in device memory (a pointer, not a by-value struct):
// the per-trial routine takes them by reference, which would otherwise force
// a private copy of the whole struct.
__global__ __launch_bounds__(kThreads, 1) void k_ragged(const RArgs* __restrict__ pargs) {
  const RArgs& A = *pargs;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int s_ticket;
  for (;;) {
    if (threadIdx.x == 0) s_ticket = atomicAdd(A.counter, 1);
    __syncthreads();
    const int t = s_ticket;
    __syncthreads();
    if (t >= A.n_units) break;  // uniform: every wave leaves
    if (t >= A.n_wg_items) {
      // eight packed trials, one per wave
      const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
      const int i = A.n_wg_items + (t - A.n_wg_items) * (kThreads / 64) + wave;
      if (i < A.n_items) {
        const RItem it = A.items[i];
        unsigned char* wsm = smem + wave * kWaveLds;
        switch (__builtin_amdgcn_readfirstlane(it.cls)) {
          case 0: wave_trial<8>(A, it, A.X[0], wsm, lane); break;
          case 1: wave_trial<16>(A, it, A.X[1], wsm, lane); break;
          default: wave_trial<32>(A, it, A.X[2], wsm, lane); break;
        }
      }
      __syncthreads();  // the next ticket may use the LDS as a whole
      continue;
    }
    const RItem it = A.items[t];
    // class parameters picked with constant indices (no local copy of the arguments)
    switch (it.cls) {
      case 0: trial_project<8, 1>(A, it, A.X[0], A.nchunk[0], smem); break;
      case 1:
        if (A.wr[1] == 1) trial_project<16, 1>(A, it, A.X[1], A.nchunk[1], smem);
        else trial_project<16, 2>(A, it, A.X[1], A.nchunk[1], smem);
        break;
      case 2:
        if (A.wr[2] == 2) trial_project<32, 2>(A, it, A.X[2], A.nchunk[2], smem);
        else trial_project<32, 4>(A, it, A.X[2], A.nchunk[2], smem);
        break;
      case 3:
        if (A.wr[3] == 4) trial_project<64, 4>(A, it, A.X[3], A.nchunk[3], smem);
        else trial_project<64, 8>(A, it, A.X[3], A.nchunk[3], smem);
        break;
      default: trial_project<128, 8>(A, it, A.X[4], A.nchunk[4], smem); break;
    }
    trial_peaks(A, it, smem);
  }
}

__global__ void k_ragged_reset(int32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

__global__ void k_ragged_bind(RArgs* args, const float2* Y, float* P, int32_t* idx, float* val, double* refined) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    args->Y = Y;
    args->P = P;
    args->idx = idx;
    args->val = val;
    args->refined = refined;
  }
}

}  // namespace

int ragged_blocks_per_chunk(int cls) {
  switch (cls) {
    case 0: return RC<8>::NB;
    case 1: return RC<16>::NB;
    case 2: return RC<32>::NB;
    case 3: return RC<64>::NB;
    default: return RC<128>::NB;
  }
}

hipError_t ragged_prepare() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_ragged),
                             hipFuncAttributeMaxDynamicSharedMemorySize, kRaggedLds);
}

hipError_t launch_ragged(const RArgs* d_args, int n_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_ragged, dim3(unsigned(n_wg)), dim3(kThreads), kRaggedLds, s, d_args);
  return hipGetLastError();
}

hipError_t launch_ragged_bind(RArgs* d_args, const float2* Y, float* P, int32_t* idx, float* val, double* refined,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_ragged_bind, dim3(1), dim3(64), 0, s, d_args, Y, P, idx, val, refined);
  return hipGetLastError();
}

hipError_t launch_ragged_reset(int32_t* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_ragged_reset, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

}  // namespace ba
