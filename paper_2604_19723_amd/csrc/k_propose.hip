// Learned-proposal refinement: the Bartlett spectrum (Sec. IV-D.2) evaluated
// only in narrow windows of the full grid around the network's coarse
// directions, the window maxima taken as the peaks, and a per-trial verdict
// on whether the full grid search must be run instead.
//
// One workgroup per trial. Q goes into MFMA registers as in the full-grid
// kernel; each window is covered by the consecutive 16-column blocks of the
// plan's steering table that contain it (a contiguous slice of the table, so
// window points are exactly full-grid points). The maximum of each window
// (ties to the lower index) is a local maximum of the full spectrum when it
// lies strictly inside the window, and its parabolic refinement uses the
// same neighbours as on the full grid. A trial falls back when a proposal or
// any spectrum value inside a window is NaN, when a window maximum sits on a
// window edge that is not a grid edge, when two windows find the same point,
// or when the normalised cost P M / tr(R) = a^H R a / (M tr R) of a peak is
// not at least the threshold tau.
#include <climits>

#include "proj_common.h"
#include <algorithm>

#include "propose.h"

namespace ba {
namespace {

__device__ __forceinline__ bool better(float va, int ia, float vb, int ib) {
  return va > vb || (va == vb && ia < ib);
}

__device__ double parabolic(double pm, double p0, double pp) {
#pragma clang fp contract(off)
  const double den = pm - 2.0 * p0 + pp;
  if (den == 0.0 || !isfinite(den)) return 0.0;
  const double d = 0.5 * (pm - pp) / den;
  return d > 0.5 ? 0.5 : (d < -0.5 ? -0.5 : d);
}

template <int MP>
__global__ __launch_bounds__(256, 6) void k_window(WindowArgs A) {
  using C = QCfg<MP>;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  // LDS: two steering chunks (one in flight by LDS DMA), then the spectrum
  // rows of the K windows, sized for the windows of this launch
  const int nbmax = window_blocks(A.hw);
  float4* sX = reinterpret_cast<float4*>(smem);                                   // [2][CH4]
  float* sP = reinterpret_cast<float*>(smem + size_t(2) * C::CH4 * 16);          // [kMaxProp][nbmax*16]
  __shared__ float red[2][C::WR][16 * C::NB];
  __shared__ int s_lo[kMaxProp], s_hi[kMaxProp], s_jb0[kMaxProp];
  __shared__ float s_tr;
  __shared__ int s_nan;  // a NaN proposal or window value was seen
  __shared__ float wv[4];
  __shared__ int wi[4];
  __shared__ float s_pv[kMaxProp];
  __shared__ int s_pi[kMaxProp];

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave % C::WR, wc = wave / C::WR;
  const int64_t b = blockIdx.x;
  const int M = A.M, K = A.K;
  const float2* Rb = A.R + b * int64_t(M) * M;

  float a[C::VL];
  load_q_fragments<MP>(Rb, M, wr, lane, a);

  if (threadIdx.x == 0) {
    float tr = 0.f;
    for (int m = 0; m < M; ++m) tr += Rb[m * M + m].x;
    s_tr = tr;
    // proposals sorted ascending, mapped to the nearest full-grid index
    float u[kMaxProp];
    int nanp = 0;
    for (int k = 0; k < K; ++k) {
      u[k] = A.U[b * A.dout + k];
      if (u[k] != u[k]) nanp = 1;
    }
    s_nan = nanp;
    for (int i = 1; i < K; ++i)
      for (int j = i; j > 0 && u[j] < u[j - 1]; --j) {
        const float t = u[j];
        u[j] = u[j - 1];
        u[j - 1] = t;
      }
    for (int k = 0; k < K; ++k) {
      float uk = u[k];
      uk = uk != uk ? 0.f : fminf(1.f, fmaxf(-1.f, uk));  // a NaN proposal (the trial falls back) still gets a window
      const double th = asin(double(uk)) * (180.0 / M_PI);
      long long c = llrint((th - A.theta0) / A.step);
      c = c < 0 ? 0 : (c > A.G - 1 ? A.G - 1 : c);
      const int lo = int(c - A.hw < 0 ? 0 : c - A.hw);
      const int hi = int(c + A.hw > A.G - 1 ? A.G - 1 : c + A.hw);
      s_lo[k] = lo;
      s_hi[k] = hi;
      s_jb0[k] = lo / 16;
    }
  }
  __syncthreads();

  // The windows' 16-column blocks are contiguous slices of the table; they
  // are taken in chunks of NB blocks (8 KB, the full-grid kernel's chunk), over
  // all windows in turn, the next chunk in flight by LDS DMA while the current
  // one is multiplied. Values and reduction order are those of k_proj_q.
  const float scale = 2.0f / float(M * M);  // as the full-grid kernel: P = 2 x^T U x / M^2
  auto nbw = [&](int k) { return s_hi[k] / 16 - s_jb0[k] + 1; };
  auto fetch = [&](int k, int c, int buf) {
    const int nvalid = min(C::NB, nbw(k) - c * C::NB);
    const float4* src = A.X + int64_t(s_jb0[k] + c * C::NB) * (C::BLK / 4);
#pragma unroll
    for (int f = 0; f < C::CH4 / 4 / 64; ++f) {
      const int o = wave * (C::CH4 / 4) + f * 64;  // one DMA lies inside one block
      if (o / (C::BLK / 4) < nvalid) lds_dma16(src + o + lane, sX + buf * C::CH4 + o);
    }
  };
  int k = 0, c = 0;
  fetch(0, 0, 0);
  lds_dma_wait();
  __syncthreads();
  for (int t = 0;; ++t) {
    int kn = k, cn = c + 1;
    if (cn * C::NB >= nbw(k)) {
      kn = k + 1;
      cn = 0;
    }
    const bool more = kn < K;
    const int buf = t & 1;
    if (more) fetch(kn, cn, buf ^ 1);  // the other buffer was last read before the previous barrier
    const float4* sxb = sX + buf * C::CH4;
    const float* sx = reinterpret_cast<const float*>(sxb);
    const int nvalid = min(C::NB, nbw(k) - c * C::NB);
    for (int jb = wc; jb < nvalid; jb += C::WC) {
      const float part = block_quadratic<MP>(a, sxb + jb * (C::BLK / 4), sx + jb * C::BLK, wr, lane);
      if (lane < 16) red[buf][wr][jb * 16 + lane] = part;
    }
    lds_dma_wait();
    __syncthreads();
    for (int q = threadIdx.x; q < nvalid * 16; q += 256) {
      float s = 0.f;
#pragma unroll
      for (int w = 0; w < C::WR; ++w) s += red[buf][w][q];
      sP[k * (16 * nbmax) + c * C::NB * 16 + q] = s * scale;
    }
    if (!more) break;
    k = kn;
    c = cn;
  }
  __syncthreads();

  // window maxima
  for (int k = 0; k < K; ++k) {
    const int lo = s_lo[k], hi = s_hi[k], base = s_jb0[k] * 16;
    float bv = -INFINITY;
    int bi = INT_MAX;
    for (int g = lo + int(threadIdx.x); g <= hi; g += 256) {
      const float p = sP[k * (16 * nbmax) + (g - base)];
      if (p != p) {
        s_nan = 1;  // every writer stores the same value
      } else if (better(p, g, bv, bi)) {
        bv = p;
        bi = g;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (better(ov, oi, bv, bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      wv[wave] = bv;
      wi[wave] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < 4; ++w)
        if (better(wv[w], wi[w], bv, bi)) {
          bv = wv[w];
          bi = wi[w];
        }
      s_pv[k] = bv;
      s_pi[k] = bi;
    }
    __syncthreads();
  }

  if (threadIdx.x == 0) {
    bool fail = s_nan != 0;
    for (int k = 0; k < K; ++k) {
      const int g = s_pi[k];
      if (g == INT_MAX) {
        fail = true;
        continue;
      }
      if ((g == s_lo[k] && g > 0) || (g == s_hi[k] && g < A.G - 1)) fail = true;
      if (!(s_pv[k] * float(M) / s_tr >= A.tau)) fail = true;
      for (int j = 0; j < k; ++j)
        if (s_pi[j] == g) fail = true;
    }
    A.fell[b] = fail ? 1 : 0;
    if (fail) {
      const int slot = atomicAdd(A.fb_count, 1);
      A.fb_list[slot] = int(b);
    } else {
      // order by value (ties to the lower index), refine on the window row
      int ord[kMaxProp];
      for (int k = 0; k < K; ++k) ord[k] = k;
      for (int i = 1; i < K; ++i)
        for (int j = i; j > 0 && better(s_pv[ord[j]], s_pi[ord[j]], s_pv[ord[j - 1]], s_pi[ord[j - 1]]); --j) {
          const int t = ord[j];
          ord[j] = ord[j - 1];
          ord[j - 1] = t;
        }
      for (int r = 0; r < K; ++r) {
        const int k = ord[r], g = s_pi[k], base = s_jb0[k] * 16;
        const float* row = sP + k * (16 * nbmax) - base;
        A.idx[b * K + r] = g;
        A.val[b * K + r] = s_pv[k];
        double d = 0.0;
        if (g > 0 && g < A.G - 1) d = parabolic(double(row[g - 1]), double(row[g]), double(row[g + 1]));
        A.refined[b * K + r] = double(g) + d;
      }
    }
  }
}

// scatter the full-grid results of the fallback trials into the outputs
__global__ void k_scatter(const int* __restrict__ list, const int* __restrict__ count, int K,
                          const int* __restrict__ idx_c, const float* __restrict__ val_c,
                          const double* __restrict__ ref_c, int* __restrict__ idx, float* __restrict__ val,
                          double* __restrict__ ref) {
  const int i = blockIdx.x * 64 + (threadIdx.x >> 3);
  const int k = threadIdx.x & 7;
  if (i >= *count || k >= K) return;
  const int64_t b = list[i];
  idx[b * K + k] = idx_c[int64_t(i) * K + k];
  val[b * K + k] = val_c[int64_t(i) * K + k];
  ref[b * K + k] = ref_c[int64_t(i) * K + k];
}

// gather the covariances of the *count fallback trials into a compact batch
// (workgroups step through the list with the grid's stride)
__global__ void k_gather_r(const int* __restrict__ list, const int* __restrict__ count,
                           const float2* __restrict__ R, float2* __restrict__ Rc, int M) {
  const int n = *count;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t b = list[i];
    for (int e = threadIdx.x; e < M * M; e += 256) Rc[int64_t(i) * M * M + e] = R[b * M * M + e];
  }
}

__global__ void k_zero_count(int* count) {
  if (threadIdx.x == 0) *count = 0;
}

}  // namespace

size_t window_lds_bytes(int Mp, int hw) {
  (void)Mp;  // two 8 KB steering chunks at every element count
  const size_t nb = size_t(window_blocks(hw));
  return size_t(2) * 8192 + size_t(kMaxProp) * 16 * nb * 4;
}

hipError_t launch_window(const WindowArgs& a, int Mp, int B, hipStream_t s) {
  const size_t lds = window_lds_bytes(Mp, a.hw);
  hipError_t e = hipSuccess;
#define BA_W(MPV)                                                                                    \
  case MPV:                                                                                          \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_window<MPV>),                            \
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));                   \
    if (e != hipSuccess) return e;                                                                   \
    hipLaunchKernelGGL(k_window<MPV>, dim3(unsigned(B)), dim3(256), lds, s, a);                      \
    break;
  switch (Mp) {
    BA_W(8)
    BA_W(16)
    BA_W(32)
    BA_W(64)
    default: return hipErrorInvalidValue;
  }
#undef BA_W
  return hipGetLastError();
}

hipError_t launch_zero_count(int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, s, count);
  return hipGetLastError();
}

hipError_t launch_gather_r(const int* list, const int* count, int n, const float2* R, float2* Rc, int M,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_gather_r, dim3(unsigned(std::min(n, 2048))), dim3(256), 0, s, list, count, R, Rc, M);
  return hipGetLastError();
}

hipError_t launch_scatter(const int* list, const int* count, int n, int K, const int* idx_c, const float* val_c,
                          const double* ref_c, int* idx, float* val, double* ref, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(unsigned((n + 63) / 64)), dim3(512), 0, s, list, count, K, idx_c, val_c,
                     ref_c, idx, val, ref);
  return hipGetLastError();
}

}  // namespace ba
