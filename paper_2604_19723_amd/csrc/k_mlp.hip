// Kernels of the learned proposal network: covariance packing, a strided GEMM
// on the matrix cores with fused epilogues, bias gradients, masked MSE and
// Adam. The network maps the packed sample covariance to coarse directions
// so that only narrow windows of the Bartlett grid (Sec. IV-D.2) are scanned.
//
// GEMM: C[m][n] = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn]: one kernel serves the forward pass (X W^T), the
// input gradient (dZ W) and the weight gradient (dZ^T H). Operands are FP32 in
// memory; a 64 x 64 x 32 tile is staged in LDS k-contiguous (rounded to BF16
// on the way in for the BF16 mode) and multiplied with
// v_mfma_f32_16x16x32_bf16 or v_mfma_f32_16x16x4f32, FP32 accumulate.
#include "ba_internal.h"
#include "mlp.h"

namespace ba {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TM = 64, TN = 64, TK = 32;
constexpr int LDK = TK + 4;  // padded row of the k-contiguous LDS tiles

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float(unsigned(bf16_rne(x)) << 16); }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

template <int PREC>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ float As[TM][LDK];
  __shared__ float Bs[TN][LDK];  // B stored transposed: Bs[n][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += TK) {
    // stage A (64 x 32) and B (32 x 64): iterate along the contiguous dimension
    for (int v = tid; v < TM * TK; v += 256) {
      int mm, kk;
      if (g.sak == 1) { mm = v / TK; kk = v % TK; } else { kk = v / TM; mm = v % TM; }
      const int m = m0 + mm, k = k0 + kk;
      float x = (m < g.M && k < g.K) ? g.A[int64_t(m) * g.sam + int64_t(k) * g.sak] : 0.f;
      As[mm][kk] = PREC == BA_PREC_BF16 ? bf16_round(x) : x;
    }
    for (int v = tid; v < TN * TK; v += 256) {
      int nn, kk;
      if (g.sbk == 1) { nn = v / TK; kk = v % TK; } else { kk = v / TN; nn = v % TN; }
      const int n = n0 + nn, k = k0 + kk;
      float x = (n < g.N && k < g.K) ? g.B[int64_t(k) * g.sbk + int64_t(n) * g.sbn] : 0.f;
      Bs[nn][kk] = PREC == BA_PREC_BF16 ? bf16_round(x) : x;
    }
    __syncthreads();
    if (PREC == BA_PREC_BF16) {
      bf16x8 af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float* ar = &As[wm * 32 + i * 16 + (lane & 15)][8 * (lane >> 4)];
        const float* br = &Bs[wn * 32 + i * 16 + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          af[i][e] = static_cast<__bf16>(ar[e]);  // exact: staged values are already BF16
          bf[i][e] = static_cast<__bf16>(br[e]);
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int s = 0; s < TK / 4; ++s) {
        float af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          af[i] = As[wm * 32 + i * 16 + (lane & 15)][4 * s + (lane >> 4)];
          bf[i] = Bs[wn * 32 + i * 16 + (lane & 15)][4 * s + (lane >> 4)];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // epilogue: acc[i][j][r] = C[m0 + 32 wm + 16 i + 4 (lane/16) + r][n0 + 32 wn + 16 j + lane%16]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][r];
        const int64_t o = int64_t(m) * g.ldc + n;
        switch (g.mode) {
          case kGemmHidden: {
            v += g.bias[n];
            g.Z[o] = v;
            g.C[o] = gelu(v);
            break;
          }
          case kGemmBias: g.C[o] = v + g.bias[n]; break;
          case kGemmGeluGrad: g.C[o] = v * gelu_grad(g.Z[o]); break;
          default: g.C[o] = v; break;
        }
      }
}

// ---------------------------------------------------------------- BF16 GEMM, 128 x 128 or 64 x 64 tiles
//
// 4 waves, each a (BT/2) x (BT/2) sub-tile ((BT/32) x (BT/32) MFMA blocks).
// Operand tiles are stored in LDS as BF16, k-contiguous, rows padded to 40
// elements (80 bytes): a fragment (8 consecutive k of one row) is one
// conflict-free 16-byte read. Global loads go 4 elements at a time along
// whichever dimension is contiguous and are issued one k-tile ahead (double
// buffering through registers). The 64-row tiles serve products too small to
// give the 128-row tiles two workgroups per CU.
constexpr int BK = 32, BLD = 40;

__device__ __forceinline__ void load4(const float* __restrict__ p, int64_t so, int64_t sc, int r, int c,
                                      int nr, int nc, float (&v)[4]) {
  // 4 consecutive elements along the contiguous index c (stride sc == 1 when vectorisable)
  const bool inr = r < nr;
  if (inr && sc == 1 && c + 3 < nc) {
    const float* q = p + int64_t(r) * so + c;
    if ((reinterpret_cast<uintptr_t>(q) & 15) == 0) {
      const float4 x = *reinterpret_cast<const float4*>(q);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = (inr && c + e < nc) ? p[int64_t(r) * so + int64_t(c + e) * sc] : 0.f;
}

// tile loader: operand X(i, k) = P[i si + k sk] for i in [i0, i0+BT), k in [k0, k0+32);
// each of 256 threads loads BT/32 groups of 4 elements
template <int BT>
struct TileLoad {
  static constexpr int NG = BT / 32;  // groups per thread
  static constexpr int IG = BT / 4;   // groups of 4 i per k row
  float v[NG][4];
  __device__ void load(const float* P, int64_t si, int64_t sk, int i0, int k0, int ni, int nk, int tid) {
    if (sk == 1) {  // k contiguous: groups of 4 k
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        const int g = j * 256 + tid, i = g >> 3, k4 = (g & 7) * 4;
        load4(P, si, 1, i0 + i, k0 + k4, ni, nk, v[j]);
      }
    } else {        // i contiguous: groups of 4 i
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        const int g = j * 256 + tid, k = g / IG, i4 = (g % IG) * 4;
        load4(P, sk, si, k0 + k, i0 + i4, nk, ni, v[j]);
      }
    }
  }
  __device__ void store(__bf16 (*S)[BLD], bool kcontig, int tid) const {
    if (kcontig) {
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        const int g = j * 256 + tid, i = g >> 3, k4 = (g & 7) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) S[i][k4 + e] = static_cast<__bf16>(v[j][e]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        const int g = j * 256 + tid, k = g / IG, i4 = (g % IG) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) S[i4 + e][k] = static_cast<__bf16>(v[j][e]);
      }
    }
  }
};

template <int BT>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  constexpr int NI = BT / 32;  // MFMA blocks per wave and dimension
  __shared__ __attribute__((aligned(16))) __bf16 As[2][BT][BLD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BT][BLD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
  const bool a_k = g.sak == 1, b_k = g.sbk == 1;
  floatx4 acc[NI][NI];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  TileLoad<BT> la, lb;
  // B(k, n) = B[k sbk + n sbn]: as an operand indexed (n, k) it has si = sbn, sk = sbk
  la.load(g.A, g.sam, g.sak, m0, 0, g.M, g.K, tid);
  lb.load(g.B, g.sbn, g.sbk, n0, 0, g.N, g.K, tid);
  la.store(As[0], a_k, tid);
  lb.store(Bs[0], b_k, tid);
  __syncthreads();
  const int nk = (g.K + BK - 1) / BK;
  for (int t = 0; t < nk; ++t) {
    const int buf = t & 1;
    const bool more = t + 1 < nk;
    if (more) {
      la.load(g.A, g.sam, g.sak, m0, (t + 1) * BK, g.M, g.K, tid);
      lb.load(g.B, g.sbn, g.sbk, n0, (t + 1) * BK, g.N, g.K, tid);
    }
    bf16x8 af[NI], bfr[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      af[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * (BT / 2) + i * 16 + (lane & 15)][8 * (lane >> 4)]);
      bfr[i] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn * (BT / 2) + i * 16 + (lane & 15)][8 * (lane >> 4)]);
    }
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NI; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    if (more) {
      la.store(As[buf ^ 1], a_k, tid);
      lb.store(Bs[buf ^ 1], b_k, tid);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * (BT / 2) + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn * (BT / 2) + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][r];
        const int64_t o = int64_t(m) * g.ldc + n;
        switch (g.mode) {
          case kGemmHidden: {
            v += g.bias[n];
            g.Z[o] = v;
            g.C[o] = gelu(v);
            break;
          }
          case kGemmBias: g.C[o] = v + g.bias[n]; break;
          case kGemmGeluGrad: g.C[o] = v * gelu_grad(g.Z[o]); break;
          default: g.C[o] = v; break;
        }
      }
}

// db[n] = sum_m dZ[m][n] in a fixed summation order: a workgroup takes 64
// columns; its 16 waves sum interleaved rows (many loads in flight per lane),
// and the 16 partial sums are added in wave order
__global__ __launch_bounds__(1024) void k_colsum(const float* __restrict__ dZ, float* __restrict__ db, int M,
                                                 int N) {
  __shared__ float part[16][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  float s = 0.f;
  if (n < N) {
#pragma unroll 8
    for (int m = g; m < M; m += 16) s += dZ[int64_t(m) * N + n];
  }
  part[g][c] = s;
  __syncthreads();
  if (g == 0 && n < N) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += part[q][c];
    db[n] = t;
  }
}

// masked MSE: loss = sum m (y - t)^2 / sum m, dY = 2 m (y - t) / sum m (one workgroup)
__global__ __launch_bounds__(1024) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                              const float* __restrict__ mask, float* __restrict__ dY,
                                              float* __restrict__ loss, int n) {
  __shared__ float red[2][16];
  float sm = 0.f, se = 0.f;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const float m = mask ? mask[i] : 1.f;
    const float d = Y[i] - T[i];
    sm += m;
    se += m * d * d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sm += __shfl_xor(sm, off, 64);
    se += __shfl_xor(se, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = sm;
    red[1][w] = se;
  }
  __syncthreads();
  float tm = 0.f, te = 0.f;
  for (int i = 0; i < 16; ++i) {
    tm += red[0][i];
    te += red[1][i];
  }
  const float inv = tm > 0.f ? 1.0f / tm : 0.f;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const float m = mask ? mask[i] : 1.f;
    dY[i] = 2.0f * m * (Y[i] - T[i]) * inv;
  }
  if (threadIdx.x == 0 && loss) *loss = te * inv;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n,
                                              float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// packed covariance: [diag re (M)] [strict upper re (M(M-1)/2)] [strict upper im], x M / tr R
// strict-upper index u (row-major) -> (m, n): row m starts at m (2M - m - 1) / 2
__device__ __forceinline__ int2 upper_mn(int u, int M) {
  const double a = 2.0 * M - 1.0;
  int m = int((a - sqrt(a * a - 8.0 * u)) * 0.5);
  m = max(0, min(m, M - 2));
  while (m > 0 && m * (2 * M - m - 1) / 2 > u) --m;
  while ((m + 1) * (2 * M - m - 2) / 2 <= u) ++m;
  const int start = m * (2 * M - m - 1) / 2;
  return make_int2(m, m + 1 + (u - start));
}

__global__ __launch_bounds__(256) void k_pack(const float2* __restrict__ R, float* __restrict__ X, int M) {
  const int64_t b = blockIdx.x;
  const float2* Rb = R + b * int64_t(M) * M;
  __shared__ float red[4];
  float tr = 0.f;
  for (int m = threadIdx.x; m < M; m += 256) tr += Rb[m * M + m].x;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tr;
  __syncthreads();
  const float t = red[0] + red[1] + red[2] + red[3];
  const float s = float(M) / t;
  const int nu = M * (M - 1) / 2;
  float* Xb = X + b * int64_t(M) * M;
  for (int e = threadIdx.x; e < M * M; e += 256) {
    float x;
    if (e < M) {
      x = Rb[e * M + e].x;
    } else if (e < M + nu) {
      const int2 mn = upper_mn(e - M, M);
      x = Rb[mn.x * M + mn.y].x;
    } else {
      const int2 mn = upper_mn(e - M - nu, M);
      x = Rb[mn.x * M + mn.y].y;
    }
    Xb[e] = x * s;
  }
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& g, int prec, hipStream_t s) {
  const dim3 grid(unsigned((g.N + TN - 1) / TN), unsigned((g.M + TM - 1) / TM));
  if (prec == BA_PREC_BF16) {
    // 128-row tiles when they give every CU two workgroups, else 64-row tiles
    const int64_t n128 = int64_t((g.N + 127) / 128) * ((g.M + 127) / 128);
    if (n128 >= 512) {
      const dim3 gb(unsigned((g.N + 127) / 128), unsigned((g.M + 127) / 128));
      hipLaunchKernelGGL(k_gemm_bf16<128>, gb, dim3(256), 0, s, g);
    } else {
      const dim3 gb(unsigned((g.N + 63) / 64), unsigned((g.M + 63) / 64));
      hipLaunchKernelGGL(k_gemm_bf16<64>, gb, dim3(256), 0, s, g);
    }
  } else
    hipLaunchKernelGGL(k_gemm<BA_PREC_F32>, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* dZ, float* db, int M, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3(unsigned((N + 63) / 64)), dim3(1024), 0, s, dZ, db, M, N);
  return hipGetLastError();
}

hipError_t launch_mse(const float* Y, const float* T, const float* mask, float* dY, float* loss, int n,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, s, Y, T, mask, dY, loss, n);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack(const float2* R, float* X, int M, int B, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(unsigned(B)), dim3(256), 0, s, R, X, M);
  return hipGetLastError();
}

}  // namespace ba
