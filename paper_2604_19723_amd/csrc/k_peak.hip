// Peak pick, parabolic refinement and proposal moments per trial.
//
// The paper takes the candidate of maximum Bartlett cost as the proposal mean
// and the cost-weighted second central moment as its covariance (Sec.
// IV-D.2). Here the argmax is generalised to the K largest local maxima:
// a point is a maximum when it is strictly greater than every neighbour
// before it in raster order and >= every neighbour after it (8-neighbourhood
// on 2-D grids, optional wrap of dim0); missing neighbours are not compared,
// and every comparison with NaN is false. Ties in value go to the lower index.
//
// One workgroup per trial. Each lane scans a strided slice of the grid
// (coalesced; a 1-D row is staged in LDS first, other grids in bands of rows)
// and keeps a sorted top-KC list in registers; the lists meet in LDS and K
// rounds of a wave-shuffle argmax pick the winners in order.
#include <climits>

#include <algorithm>

#include "ba_internal.h"
#include "coherent.h"
#include "peak_rule.h"

namespace ba {
namespace {

// 1-D candidate rows staged in LDS: 30 KB, which with the 32 KB of merge lists
// (16 per lane) stays within the 64 KB a workgroup gets without opting in
constexpr int kPeakRowMax = 7680;

__device__ __forceinline__ bool better(float va, int ia, float vb, int ib) { return peak_better(va, ia, vb, ib); }

__device__ __forceinline__ int wrap_row(int j0, int rows) {
  return j0 < 0 ? j0 + rows : (j0 >= rows ? j0 - rows : j0);
}

__device__ bool is_local_max(const float* __restrict__ Pb, int i0, int i1, float p, int s1,
                             int rows, int wrap0) {
  if (p != p) return false;
  bool ok = true;
  for (int di = -1; di <= 1; ++di) {
    int j0 = i0 + di;
    if (wrap0)
      j0 = wrap_row(j0, rows);
    else if (j0 < 0 || j0 >= rows)
      continue;
    for (int dj = -1; dj <= 1; ++dj) {
      if (di == 0 && dj == 0) continue;
      if (s1 == 1 && dj != 0) continue;
      const int j1 = i1 + dj;
      if (j1 < 0 || j1 >= s1) continue;
      const float q = Pb[int64_t(j0) * s1 + j1];
      const bool earlier = di < 0 || (di == 0 && dj < 0);
      ok = ok && (earlier ? (p > q) : (p >= q));
    }
  }
  return ok;
}

// Insert (v, g) into a sorted list of compile-time capacity; the unrolled form
// keeps the list in registers.
template <int KC>
__device__ __forceinline__ void insert(float (&lv)[KC], int (&li)[KC], float v, int g) {
#pragma unroll
  for (int j = KC - 1; j >= 0; --j) {
    if (j > 0 && better(v, g, lv[j - 1], li[j - 1])) {
      lv[j] = lv[j - 1];
      li[j] = li[j - 1];
    } else if (better(v, g, lv[j], li[j])) {
      lv[j] = v;
      li[j] = g;
    }
  }
}

__device__ double parabolic(double pm, double p0, double pp) { return peak_parabolic(pm, p0, pp); }

// Where the candidates meet their neighbours:
//  kPeakGlobal: in global memory (is_local_max), for rows too wide for LDS;
//  kPeakOneD:   a 1-D grid (s1 == 1) whose candidate row fits in LDS is staged
//               there with coalesced loads first, and each point meets its two
//               neighbours in LDS (the earlier neighbour strictly, the later
//               one with >=, wrap of the row when wrap0, every comparison
//               with NaN false);
//  kPeakBand:   any other grid is walked in bands of whole dim-0 rows, each
//               staged in LDS with the row before and the row after it
//               (wrapped when wrap0), and tested by the same rule as
//               is_local_max against the staged rows.
// Every lane keeps its own sorted top-KC list, so the result does not
// depend on which lane meets which point.
constexpr int kPeakGlobal = 0, kPeakOneD = 1, kPeakBand = 2;

// columns one lane tests per step in a band
constexpr int kPeakRun = 8;

// rows of a band of a grid with s1 points per dim-0 row (0: too wide)
__host__ __device__ __forceinline__ int peak_band_rows(int s1) { return kPeakRowMax / s1 - 2; }

// is_local_max against staged rows: sR + L s1 is the point's own row, the
// rows before and after it sit at L - 1 and L + 1
__device__ __forceinline__ bool is_local_max_band(const float* sR, int L, int i0, int i1, float p, int s1,
                                                  int rows, int wrap0) {
  if (p != p) return false;
  bool ok = true;
#pragma unroll
  for (int di = -1; di <= 1; ++di) {
    if (!wrap0 && (i0 + di < 0 || i0 + di >= rows)) continue;
    const float* q = sR + (L + di) * s1;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      if (di == 0 && dj == 0) continue;
      if (s1 == 1 && dj != 0) continue;
      const int j1 = i1 + dj;
      if (j1 < 0 || j1 >= s1) continue;
      const bool earlier = di < 0 || (di == 0 && dj < 0);
      ok = ok && (earlier ? (p > q[j1]) : (p >= q[j1]));
    }
  }
  return ok;
}

template <int KC, int MODE>
__device__ __forceinline__ void peaks_trial(int64_t b, const float* __restrict__ P, int64_t G, int s1,
                                            int rows, int wrap0, int k, int* __restrict__ idx,
                                            float* __restrict__ val,
                                            double* __restrict__ refined, int ndim) {
  const float* Pb = P + b * G;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  float lv[KC];
  int li[KC];
#pragma unroll
  for (int j = 0; j < KC; ++j) {
    lv[j] = -INFINITY;
    li[j] = INT_MAX;
  }
  const int64_t ncand = int64_t(rows) * s1;
  if constexpr (MODE == kPeakOneD) {
    extern __shared__ float sRow[];  // [rows]
    // eight loads in flight per lane before their values are stored
    for (int g0 = 0; g0 < rows; g0 += 8 * 256) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int g = g0 + j * 256 + tid;
        v[j] = g < rows ? Pb[g] : 0.f;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int g = g0 + j * 256 + tid;
        if (g < rows) sRow[g] = v[j];
      }
    }
    __syncthreads();
    for (int g = tid; g < rows; g += 256) {
      const float p = sRow[g];
      bool ok = p == p;
      const int gm = g - 1, gp = g + 1;
      if (wrap0 || gm >= 0) ok = ok && p > sRow[gm < 0 ? gm + rows : gm];
      if (wrap0 || gp < rows) ok = ok && p >= sRow[gp >= rows ? gp - rows : gp];
      if (ok) insert<KC>(lv, li, p, g);
    }
  } else if constexpr (MODE == kPeakBand) {
    extern __shared__ float sRow[];  // [(H + 2) s1], H = peak_band_rows(s1) >= 1
    const int H = peak_band_rows(s1);
    for (int r0 = 0; r0 < rows; r0 += H) {
      const int hb = min(H, rows - r0);
      // staged row lr is grid row r0 - 1 + lr (wrapped when wrap0; left
      // unset where it does not exist, and then never read)
      const int nl = (hb + 2) * s1;
      // (staged row, column) of this lane's element, advanced by 256 per step
      const int adv_r = 256 / s1, adv_c = 256 - adv_r * s1;
      int lr = tid / s1, i1 = tid - (tid / s1) * s1;
      for (int e0 = 0; e0 < nl; e0 += 8 * 256) {
        float v[8];
        int lrj = lr, i1j = i1;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = e0 + j * 256 + tid;
          int j0 = r0 - 1 + lrj;
          if (wrap0) j0 = wrap_row(j0, rows);
          v[j] = (e < nl && j0 >= 0 && j0 < rows) ? Pb[int64_t(j0) * s1 + i1j] : 0.f;
          lrj += adv_r;
          i1j += adv_c;
          if (i1j >= s1) {
            i1j -= s1;
            ++lrj;
          }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = e0 + j * 256 + tid;
          if (e < nl) sRow[e] = v[j];
        }
        lr = lrj;
        i1 = i1j;
      }
      __syncthreads();
      // each lane tests a run of kPeakRun columns of one row against the
      // three staged rows held in registers
      const int nrun = (s1 + kPeakRun - 1) / kPeakRun;
      for (int w = tid; w < hb * nrun; w += 256) {
        const int rl = w / nrun, c0 = (w - rl * nrun) * kPeakRun;
        const int i0 = r0 + rl;
        const bool has_up = wrap0 || i0 > 0, has_dn = wrap0 || i0 + 1 < rows;
        const float* up = sRow + rl * s1;
        const float* me = up + s1;
        const float* dn = me + s1;
        float u[kPeakRun + 2], m[kPeakRun + 2], d[kPeakRun + 2];
#pragma unroll
        for (int j = 0; j < kPeakRun + 2; ++j) {
          const int c = c0 - 1 + j;
          const bool in = c >= 0 && c < s1;
          m[j] = in ? me[c] : 0.f;
          u[j] = in && has_up ? up[c] : 0.f;
          d[j] = in && has_dn ? dn[c] : 0.f;
        }
#pragma unroll
        for (int j = 1; j <= kPeakRun; ++j) {
          const int c = c0 + j - 1;
          if (c >= s1) break;
          const float p = m[j];
          // the earlier neighbours strictly below, the later ones at most
          // equal, missing ones not compared, NaN never a maximum
          const bool l_ok = c > 0, r_ok = c + 1 < s1;
          bool ok = p == p;
          if (has_up) {
            ok = ok && p > u[j];
            if (l_ok) ok = ok && p > u[j - 1];
            if (r_ok) ok = ok && p > u[j + 1];
          }
          if (l_ok) ok = ok && p > m[j - 1];
          if (r_ok) ok = ok && p >= m[j + 1];
          if (has_dn) {
            ok = ok && p >= d[j];
            if (l_ok) ok = ok && p >= d[j - 1];
            if (r_ok) ok = ok && p >= d[j + 1];
          }
          if (ok) insert<KC>(lv, li, p, i0 * s1 + c);
        }
      }
      __syncthreads();  // the next band reuses the staging
    }
  } else {
    for (int64_t g = tid; g < ncand; g += 256) {
      const float p = Pb[g];
      const int i0 = int(g / s1), i1 = int(g % s1);
      if (is_local_max(Pb, i0, i1, p, s1, rows, wrap0)) insert<KC>(lv, li, p, int(g));
    }
  }

  __shared__ float sv[256 * KC];
  __shared__ int si[256 * KC];
  __shared__ float wv[4];
  __shared__ int wi[4];
  __shared__ float selv[kMaxPeaks];
  __shared__ int seli[kMaxPeaks];
#pragma unroll
  for (int j = 0; j < KC; ++j) {
    sv[tid * KC + j] = lv[j];
    si[tid * KC + j] = li[j];
  }
  __syncthreads();

  int head = 0;
  for (int r = 0; r < k; ++r) {
    float v = head < KC ? sv[tid * KC + head] : -INFINITY;
    int i = head < KC ? si[tid * KC + head] : INT_MAX;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(v, off, 64);
      const int oi = __shfl_xor(i, off, 64);
      if (better(ov, oi, v, i)) {
        v = ov;
        i = oi;
      }
    }
    if (lane == 0) {
      wv[wave] = v;
      wi[wave] = i;
    }
    __syncthreads();
    float bv = wv[0];
    int bi = wi[0];
#pragma unroll
    for (int w = 1; w < 4; ++w)
      if (better(wv[w], wi[w], bv, bi)) {
        bv = wv[w];
        bi = wi[w];
      }
    // every grid index lives in exactly one lane's list
    if (bi != INT_MAX && head < KC && si[tid * KC + head] == bi) ++head;
    if (tid == 0) {
      selv[r] = bv;
      seli[r] = bi;
    }
    __syncthreads();
  }

  if (tid < k) {
    const int g = seli[tid];
    int* ob = idx + b * k;
    float* vb = val + b * k;
    if (g == INT_MAX) {
      ob[tid] = -1;
      vb[tid] = __int_as_float(0x7fc00000);
      if (refined)
        for (int a = 0; a < ndim; ++a) refined[(b * k + tid) * ndim + a] = __longlong_as_double(0x7ff8000000000000LL);
    } else {
      ob[tid] = g;
      vb[tid] = selv[tid];
      if (refined) {
        const int i0 = g / s1, i1 = g % s1;
        const double p0 = double(Pb[g]);
        double d0 = 0.0;
        if (wrap0 || (i0 > 0 && i0 < rows - 1)) {
          const int jm = wrap_row(i0 - 1, rows), jp = wrap_row(i0 + 1, rows);
          d0 = parabolic(double(Pb[int64_t(jm) * s1 + i1]), p0, double(Pb[int64_t(jp) * s1 + i1]));
        }
        refined[(b * k + tid) * ndim + 0] = double(i0) + d0;
        if (ndim == 2) {
          double d1 = 0.0;
          if (i1 > 0 && i1 < s1 - 1)
            d1 = parabolic(double(Pb[int64_t(i0) * s1 + i1 - 1]), p0, double(Pb[int64_t(i0) * s1 + i1 + 1]));
          refined[(b * k + tid) * ndim + 1] = double(i1) + d1;
        }
      }
    }
  }
}

template <int KC, int MODE>
__global__ __launch_bounds__(256) void k_peaks(const float* __restrict__ P, int64_t G, int s1, int rows,
                                               int wrap0, int k, int* __restrict__ idx, float* __restrict__ val,
                                               double* __restrict__ refined, int ndim) {
  peaks_trial<KC, MODE>(blockIdx.x, P, G, s1, rows, wrap0, k, idx, val, refined, ndim);
}

// The same over a batch whose size is only known on the device (*count
// trials): workgroups step through the trials with the grid's stride.
template <int KC, int MODE>
__global__ __launch_bounds__(256) void k_peaks_counted(const float* __restrict__ P, int64_t G, int s1, int rows,
                                                       int wrap0, int k, int* __restrict__ idx,
                                                       float* __restrict__ val, double* __restrict__ refined,
                                                       int ndim, const int* __restrict__ count) {
  const int64_t n = *count;
  for (int64_t b = blockIdx.x; b < n; b += gridDim.x) {
    peaks_trial<KC, MODE>(b, P, G, s1, rows, wrap0, k, idx, val, refined, ndim);
    __syncthreads();  // the next trial reuses the shared staging
  }
}

__device__ __forceinline__ double block_sum(double x, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Proposal moments: w = P / sum P over the distinct points, mu at the first
// global maximum, C = sum w (x - mu)(x - mu)^T with azimuth wrap.
// STAGED: the trial's ncand <= kPeakRowMax values are first copied into LDS
// with 16-byte loads (the row's unaligned head and tail one value at a
// time, so nothing outside the row is read), and both passes read them
// there. Each lane takes the points tid, tid + 256, ... in that order either
// way, so the sums are the same bit for bit.
template <bool STAGED>
__global__ __launch_bounds__(256) void k_moments(const float* __restrict__ P, int64_t G,
                                                 int64_t ncand, const double* __restrict__ X,
                                                 int d, int azwrap, double* __restrict__ out) {
  const int64_t b = blockIdx.x;
  const float* Pb = P + b * G;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double red[4];
  __shared__ float wv[4];
  __shared__ int wi[4];
  extern __shared__ float sP[];  // [ncand] when STAGED
  if constexpr (STAGED) {
    const int n = int(ncand);
    const int off = int((reinterpret_cast<uintptr_t>(Pb) >> 2) & 3);  // floats past a 16-byte boundary
    const int h = min(n, (4 - off) & 3);
    const int nv = (n - h) >> 2;
    const float4* P4 = reinterpret_cast<const float4*>(Pb + h);
    for (int i0 = 0; i0 < nv; i0 += 8 * 256) {
      float4 v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = i0 + j * 256 + tid;
        v[j] = i < nv ? P4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = i0 + j * 256 + tid;
        if (i < nv) {
          float* q = sP + h + 4 * i;
          q[0] = v[j].x;
          q[1] = v[j].y;
          q[2] = v[j].z;
          q[3] = v[j].w;
        }
      }
    }
    const int t0 = h + 4 * nv;
    if (tid < h) sP[tid] = Pb[tid];
    if (tid < n - t0) sP[t0 + tid] = Pb[t0 + tid];
    __syncthreads();
  }
  auto value = [&](int64_t g) { return STAGED ? sP[g] : Pb[g]; };

  double s = 0.0;
  float bv = -INFINITY;
  int bi = INT_MAX;
  for (int64_t g = tid; g < ncand; g += 256) {
    const float p = value(g);
    s += double(p);
    if (better(p, int(g), bv, bi)) {
      bv = p;
      bi = int(g);
    }
  }
  const double S = block_sum(s, red);
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
  float fv = wv[0];
  int gs = wi[0];
  for (int w = 1; w < 4; ++w)
    if (better(wv[w], wi[w], fv, gs)) {
      fv = wv[w];
      gs = wi[w];
    }
  // all-NaN input leaves no maximum: the moments are NaN
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  double mu[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < d; ++a) mu[a] = gs != INT_MAX ? X[int64_t(gs) * d + a] : nan;

  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (d == 1 && !azwrap) {
    // 1-D grids: eight coordinates in flight per lane, same order and arithmetic
    for (int64_t g0 = 0; g0 < ncand; g0 += 8 * 256) {
      double x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t g = g0 + j * 256 + tid;
        x[j] = g < ncand ? X[g] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t g = g0 + j * 256 + tid;
        if (g < ncand) {
          const double p = double(value(g));
          const double D0 = x[j] - mu[0];
          acc[0] += p * D0 * D0;
        }
      }
    }
  } else {
    for (int64_t g = tid; g < ncand; g += 256) {
      const double p = double(value(g));
      double D[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < d; ++a) D[a] = X[g * d + a] - mu[a];
      if (azwrap) {
        double r = fmod(D[0] + 180.0, 360.0);
        if (r < 0.0) r += 360.0;
        D[0] = r - 180.0;
      }
      int c = 0;
      for (int i = 0; i < d; ++i)
        for (int j = i; j < d; ++j) acc[c++] += p * D[i] * D[j];
    }
  }
  double C[6];
  const int nc = d * (d + 1) / 2;
  for (int c = 0; c < nc; ++c) C[c] = block_sum(acc[c], red);
  if (tid == 0) {
    double* o = out + b * int64_t(d + d * d);
    for (int a = 0; a < d; ++a) o[a] = mu[a];
    int c = 0;
    for (int i = 0; i < d; ++i)
      for (int j = i; j < d; ++j) {
        const double v = C[c++] / S;
        o[d + i * d + j] = v;
        o[d + j * d + i] = v;
      }
  }
}

// Merge of the per-range peak candidates of a 1-D grid (one wave per
// trial). The interior maxima come from the ranges' lists; the two end
// columns of every range are tested here against the end values of the
// neighbouring ranges (wrap of the row when wrap0), with the same rule and
// order as k_peaks, so the result is identical to k_peaks on the same P.
constexpr int kMergeCap = kMaxCandRanges * (kMaxPeaks + 2);

__global__ __launch_bounds__(64) void k_peaks_merge(const float4* __restrict__ rec, int nsplit, int64_t span,
                                                    int rows, int wrap0, int k, int* __restrict__ idx,
                                                    float* __restrict__ val, double* __restrict__ refined) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const float4* rb = rec + b * nsplit * (k + 1);
  __shared__ float cv[kMergeCap], cl[kMergeCap], cr[kMergeCap];
  __shared__ int ci[kMergeCap];

  // P at a column next to a range end: one of the four end values of its range
  auto end_val = [&](int64_t g) -> float {
    const int64_t s = g / span, off = g - s * span;
    const int64_t rest = rows - s * span, n = rest < span ? rest : span;
    const float4 e = rb[s * (k + 1) + k];
    return off == 0 ? e.x : off == 1 ? e.y : off == n - 1 ? e.w : e.z;
  };

  const int nlist = nsplit * k;
  for (int e = lane; e < nlist; e += 64) {
    const float4 r = rb[(e / k) * (k + 1) + e % k];
    cv[e] = r.x;
    ci[e] = __float_as_int(r.y);
    cl[e] = r.z;
    cr[e] = r.w;
  }
  // slot nlist + 2 s: first column of range s; nlist + 2 s + 1: its last
  for (int e = lane; e < 2 * nsplit; e += 64) {
    const int s = e >> 1;
    const int64_t g0 = int64_t(s) * span, rest = rows - g0, n = rest < span ? rest : span;
    const int64_t g = (e & 1) ? g0 + n - 1 : g0;
    float v = -INFINITY, l = 0.f, r = 0.f;
    int gi = INT_MAX;
    if (n > 0 && !((e & 1) && n == 1)) {
      const float p = end_val(g);
      bool ok = p == p;
      if (g > 0 || wrap0) {
        l = end_val(g > 0 ? g - 1 : rows - 1);
        ok = ok && p > l;
      }
      if (g + 1 < rows || wrap0) {
        r = end_val(g + 1 < rows ? g + 1 : 0);
        ok = ok && p >= r;
      }
      if (ok) {
        v = p;
        gi = int(g);
      }
    }
    cv[nlist + e] = v;
    ci[nlist + e] = gi;
    cl[nlist + e] = l;
    cr[nlist + e] = r;
  }
  __syncthreads();

  const int ncand = nlist + 2 * nsplit;
  for (int t = 0; t < k; ++t) {
    float bv = -INFINITY;
    int bi = INT_MAX, be = -1;
    for (int e = lane; e < ncand; e += 64)
      if (peak_better(cv[e], ci[e], bv, bi)) {
        bv = cv[e];
        bi = ci[e];
        be = e;
      }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64), oe = __shfl_xor(be, off, 64);
      if (peak_better(ov, oi, bv, bi)) {
        bv = ov;
        bi = oi;
        be = oe;
      }
    }
    if (lane == 0) {
      const int64_t o = b * k + t;
      if (bi == INT_MAX) {
        idx[o] = -1;
        val[o] = __int_as_float(0x7fc00000);
        if (refined) refined[o] = __longlong_as_double(0x7ff8000000000000LL);
      } else {
        idx[o] = bi;
        val[o] = bv;
        if (refined) {
          double d0 = 0.0;
          if (wrap0 || (bi > 0 && bi < rows - 1))
            d0 = peak_parabolic(double(cl[be]), double(bv), double(cr[be]));
          refined[o] = double(bi) + d0;
        }
        ci[be] = INT_MAX;  // taken
        cv[be] = -INFINITY;
      }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_peaks_merge(const Plan& p, int B, int k, const float4* rec, int* idx, float* val,
                              double* refined, hipStream_t s) {
  const CandLayout L = candidate_layout(p, B);
  if (L.nsplit * (k + 2) > kMergeCap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_peaks_merge, dim3(unsigned(B)), dim3(64), 0, s, rec, L.nsplit, L.span, p.rows, p.wrap0, k,
                     idx, val, refined);
  return hipGetLastError();
}

hipError_t launch_peaks(const Plan& p, int B, const float* P, int k, int* idx, float* val,
                        double* refined, hipStream_t s, const int* count) {
  // counted: at most 2048 workgroups step through the device-side count
  const dim3 grid{static_cast<uint32_t>(count ? std::min(B, 2048) : B)}, block{256u};
  // a 1-D candidate row of up to kPeakRowMax points is staged in LDS whole;
  // other grids in bands of dim-0 rows when a band of one row fits
  const bool oned = p.shape1 == 1 && p.rows <= kPeakRowMax;
  const int H = peak_band_rows(p.shape1);
  const bool band = !oned && H >= 1;
  const size_t lds = oned ? size_t(p.rows) * sizeof(float)
                          : (band ? size_t(H + 2) * p.shape1 * sizeof(float) : 0);
#define BA_PK1(KCV, MD)                                                                                     \
  if (count)                                                                                                 \
    hipLaunchKernelGGL((k_peaks_counted<KCV, MD>), grid, block, lds, s, P, p.G, p.shape1, p.rows, p.wrap0,   \
                       k, idx, val, refined, p.ndim, count);                                                 \
  else                                                                                                       \
    hipLaunchKernelGGL((k_peaks<KCV, MD>), grid, block, lds, s, P, p.G, p.shape1, p.rows, p.wrap0, k, idx,   \
                       val, refined, p.ndim)
#define BA_PK(KCV)                \
  if (oned) {                     \
    BA_PK1(KCV, kPeakOneD);       \
  } else if (band) {              \
    BA_PK1(KCV, kPeakBand);       \
  } else {                        \
    BA_PK1(KCV, kPeakGlobal);     \
  }
  if (k <= 1)
    BA_PK(1)
  else if (k <= 2)
    BA_PK(2)
  else if (k <= 4)
    BA_PK(4)
  else if (k <= 8)
    BA_PK(8)
  else
    BA_PK(16)
#undef BA_PK
#undef BA_PK1
  return hipGetLastError();
}

// The same moments over a large point set X [G][3] (no wrap). The maximum
// comes first: every slice of the points reports its best (value, index),
// then every slice workgroup of a trial combines those few entries in index
// order into the same mu and accumulates, in FP64, S0 = sum P and
// S2 = sum P (x - mu)(x - mu)^T about it, so C = S2 / S0 is the weighted
// second moment as defined, with no cancellation against |mu|^2; one
// workgroup per trial sums the slices in index order (deterministic).
constexpr int kPtSlice = 8192;
constexpr int kPtParts = 7;  // S0, S2[6]

__global__ __launch_bounds__(256) void k_point_max(const float* __restrict__ P, int64_t G, int nslice,
                                                   float* __restrict__ part_val, int* __restrict__ part_idx) {
  const int64_t b = blockIdx.x / nslice;
  const int sl = int(blockIdx.x % nslice);
  const float* Pb = P + b * G;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ float wv[4];
  __shared__ int wi[4];
  float bv = -INFINITY;
  int bi = INT_MAX;
  const int64_t g1 = min(G, int64_t(sl + 1) * kPtSlice);
  // each lane takes its points in index order, eight loads in flight
  for (int64_t g0 = int64_t(sl) * kPtSlice; g0 < g1; g0 += 8 * 256) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t g = g0 + j * 256 + tid;
      v[j] = g < g1 ? Pb[g] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t g = g0 + j * 256 + tid;
      if (g < g1 && better(v[j], int(g), bv, bi)) {
        bv = v[j];
        bi = int(g);
      }
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
  if (tid == 0) {
    for (int w = 1; w < 4; ++w)
      if (better(wv[w], wi[w], bv, bi)) {
        bv = wv[w];
        bi = wi[w];
      }
    part_val[b * nslice + sl] = bv;
    part_idx[b * nslice + sl] = bi;
  }
}

// the trial's maximum from its slices' maxima, in slice (index) order
__device__ __forceinline__ int trial_argmax(const float* __restrict__ part_val, const int* __restrict__ part_idx,
                                            int64_t b, int nslice) {
  float bv = -INFINITY;
  int bi = INT_MAX;
  for (int sl = 0; sl < nslice; ++sl) {
    const int i = part_idx[b * nslice + sl];
    const float v = part_val[b * nslice + sl];
    if (i != INT_MAX && better(v, i, bv, bi)) {
      bv = v;
      bi = i;
    }
  }
  return bi;
}

__global__ __launch_bounds__(256) void k_point_partial(const float* __restrict__ P, int64_t G,
                                                       const double* __restrict__ X, int nslice,
                                                       const float* __restrict__ part_val,
                                                       const int* __restrict__ part_idx,
                                                       double* __restrict__ part) {
  const int64_t b = blockIdx.x / nslice;
  const int sl = int(blockIdx.x % nslice);
  const float* Pb = P + b * G;
  const int tid = threadIdx.x;
  __shared__ double red[4];
  const int bi = trial_argmax(part_val, part_idx, b, nslice);
  double* o = part + (b * nslice + sl) * kPtParts;
  if (bi == INT_MAX) {  // every value NaN: no mean
    if (tid < kPtParts) o[tid] = __longlong_as_double(0x7ff8000000000000LL);
    return;
  }
  const double mu0 = X[3 * int64_t(bi)], mu1 = X[3 * int64_t(bi) + 1], mu2 = X[3 * int64_t(bi) + 2];
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t g1 = min(G, int64_t(sl + 1) * kPtSlice);
  // each lane takes its points in index order, four points in flight
  for (int64_t g0 = int64_t(sl) * kPtSlice; g0 < g1; g0 += 4 * 256) {
    float v[4];
    double x[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t g = g0 + j * 256 + tid;
      const bool in = g < g1;
      v[j] = in ? Pb[g] : 0.f;
#pragma unroll
      for (int a = 0; a < 3; ++a) x[j][a] = in ? X[3 * g + a] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (g0 + j * 256 + tid >= g1) continue;
      const double p = double(v[j]);
      const double y0 = x[j][0] - mu0, y1 = x[j][1] - mu1, y2 = x[j][2] - mu2;
      acc[0] += p;
      acc[1] += p * y0 * y0;
      acc[2] += p * y0 * y1;
      acc[3] += p * y0 * y2;
      acc[4] += p * y1 * y1;
      acc[5] += p * y1 * y2;
      acc[6] += p * y2 * y2;
    }
  }
  for (int c = 0; c < kPtParts; ++c) {
    const double v = block_sum(acc[c], red);
    if (tid == 0) o[c] = v;
  }
}

__global__ __launch_bounds__(64) void k_point_combine(const double* __restrict__ part,
                                                      const float* __restrict__ part_val,
                                                      const int* __restrict__ part_idx, int nslice,
                                                      const double* __restrict__ X, double* __restrict__ out) {
  const int64_t b = blockIdx.x;
  if (threadIdx.x != 0) return;
  double S[kPtParts] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int sl = 0; sl < nslice; ++sl) {
    const double* o = part + (b * nslice + sl) * kPtParts;
    for (int c = 0; c < kPtParts; ++c) S[c] += o[c];
  }
  const int bi = trial_argmax(part_val, part_idx, b, nslice);
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  double* o = out + b * 12;
  for (int a = 0; a < 3; ++a) o[a] = bi != INT_MAX ? X[int64_t(bi) * 3 + a] : nan;
  const int q[3][3] = {{1, 2, 3}, {2, 4, 5}, {3, 5, 6}};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) o[3 + i * 3 + j] = S[q[i][j]] / S[0];
}

size_t point_moments_ws_bytes(int B, int64_t G) {
  const int64_t nslice = (G + kPtSlice - 1) / kPtSlice;
  return size_t(B) * nslice * (kPtParts * sizeof(double) + sizeof(float) + sizeof(int)) + 256;
}

hipError_t launch_point_moments(int B, const float* P, int64_t G, const double* X, double* mu_cov, void* ws,
                                hipStream_t s) {
  const int nslice = int((G + kPtSlice - 1) / kPtSlice);
  double* part = static_cast<double*>(ws);
  float* part_val = reinterpret_cast<float*>(part + size_t(B) * nslice * kPtParts);
  int* part_idx = reinterpret_cast<int*>(part_val + size_t(B) * nslice);
  const int64_t nblk = int64_t(nslice) * B;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_point_max, dim3(unsigned(nblk)), dim3(256), 0, s, P, G, nslice, part_val, part_idx);
  hipLaunchKernelGGL(k_point_partial, dim3(unsigned(nblk)), dim3(256), 0, s, P, G, X, nslice, part_val, part_idx,
                     part);
  hipLaunchKernelGGL(k_point_combine, dim3(unsigned(B)), dim3(64), 0, s, part, part_val, part_idx, nslice, X,
                     mu_cov);
  return hipGetLastError();
}

hipError_t launch_moments(const Plan& p, int B, const float* P, double* mu_cov, hipStream_t s) {
  const int64_t ncand = int64_t(p.rows) * p.shape1;
  const int azwrap = p.kind == BA_GRID_AZEL_DEG ? 1 : 0;
  if (ncand <= kPeakRowMax)
    hipLaunchKernelGGL(k_moments<true>, dim3(unsigned(B)), dim3(256), size_t(ncand) * sizeof(float), s, P, p.G,
                       ncand, p.d_coords, p.coord_dim, azwrap, mu_cov);
  else
    hipLaunchKernelGGL(k_moments<false>, dim3(unsigned(B)), dim3(256), 0, s, P, p.G, ncand, p.d_coords,
                       p.coord_dim, azwrap, mu_cov);
  return hipGetLastError();
}

}  // namespace ba
