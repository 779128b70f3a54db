// Particle update messages (Sec. IV-C; Supplementary Sec. S-V), FP64.
//
// Every message is a complex Gaussian log-density log CN(z_j; mu, C) whose
// covariance is eta I plus a low-rank part, evaluated with the matrix
// inversion and determinant lemmas so that only S x S systems are factored
// (S = number of features, LOS included).
//
// Steering vectors never exist densely on the per-particle paths. The URA and
// the frequency bins are uniform and centred, so the response of a path is a
// Kronecker product a = g (b (x) y (x) z) of three geometric sequences
// (delay over the bins, horizontal and vertical phase over the elements;
// Sec. II-B). Hence
//   * a^H X for a dense X is a three-level contraction (N_z + N_f N_y + N_f
//     complex MACs);
//   * <a_s, a_t> is a product of three sums of N_f, N_y, N_z terms.
// With these, the MT message's per-pair cost is O(S (N_z + S (N_f + N_y +
// N_z)) + S^3) instead of the O(N_z S^2) of the dense Gram.
//
// Kernels (one launch sequence per time step):
//   k_msg_scalars  rho_s = sum_p w_alpha and the noise prior means eta~_j;
//   k_msg_reduce   particle sums of the low-rank columns and means, per
//                  1024-particle chunk (partials; fixed order);
//   k_msg_combine  chunk partials -> m_s, w_s, m3_s, m4_s per array;
//   k_msg_setup    per (feature, array): Gram, Cholesky of I + G/eta with the
//                  feature's own column removed, the PF message at r = 0 and
//                  the PR message; per array: the noise message's Gram;
//   k_msg_pair     per (particle, array): MT and noise messages, one group of
//                  GS lanes per pair, lane s owning feature s (row s of the
//                  S x S system; Cholesky and solves across the group);
//   k_msg_kappa    per (feature, particle, array): the PF message at r = 1,
//                  one thread per particle contracting its path with every
//                  column (and with z'), columns read wave-uniformly.
#include <hip/hip_runtime.h>

#include <cmath>

#include "messages.h"

namespace ba {
namespace {

constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr int kSub = 64;             // particles per LDS round of the reduction
constexpr int kChunk = 512;          // particles per reduction workgroup
constexpr int kMaxDots = 192;        // inner products of one setup workgroup
constexpr int kSlot = 9;             // double2 per lane in the pair kernel's exchange
constexpr size_t kMaxLds = 160 * 1024;  // LDS of one CU

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double2 cscale(double a, double2 b) { return {a * b.x, a * b.y}; }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return {fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -a.y * b.x)};
}
// acc + a * b and acc + conj(a) * b, four FMAs each
__device__ __forceinline__ double2 cmac(double2 acc, double2 a, double2 b) {
  return {fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y))};
}
__device__ __forceinline__ double2 cmacc(double2 acc, double2 a, double2 b) {
  return {fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y))};
}
__device__ __forceinline__ double2 cconj(double2 a) { return {a.x, -a.y}; }
__device__ __forceinline__ double cabs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ double2 cexpi(double t) {
  double s, c;
  sincos(t, &s, &c);
  return {c, s};
}
// x^n by squaring (n >= 0, uniform across the wave)
__device__ __forceinline__ double2 cpowi(double2 x, int n) {
  double2 r = {1.0, 0.0};
  while (n) {
    if (n & 1) r = cmul(r, x);
    x = cmul(x, x);
    n >>= 1;
  }
  return r;
}

// Read-only vectors that every lane of a wave reads at the same index go
// through the constant address space, so the loads are wave-uniform (scalar
// registers feed the FMAs) instead of one LDS or vector load per lane.
struct cplx {
  double x, y;
};
typedef const __attribute__((address_space(4))) cplx* cvec;
__device__ __forceinline__ cvec uniform_vec(const double2* p) { return (cvec)(p); }
__device__ __forceinline__ double2 ld(cvec p, int i) { return {p[i].x, p[i].y}; }

template <int W>
__device__ __forceinline__ double2 gshfl(double2 v, int src) {
  return {__shfl(v.x, src, W), __shfl(v.y, src, W)};
}
template <int W>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int m = W / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, W);
  return v;
}
template <int W>
__device__ __forceinline__ double2 gsum(double2 v) {
  return {gsum<W>(v.x), gsum<W>(v.y)};
}

// Response of one path at array j in Kronecker form:
//   a[(f N_y + i) N_z + l] = g * (b0 bs^f) * (y0 ys^i) * (z0 zs^l).
// g: path loss lambda / (4 pi d) and carrier phase -2 pi f_c d / c; the delay
// factor exp(-j 2 pi f_k d / c) over the centred bins f_k = (k - (N_f-1)/2) df;
// the spatial factors exp(j pi (i - (N-1)/2) u) for half-wavelength supports,
// u = r_y / d (horizontal) and r_z / d (vertical) of the local vector r
// (eqs. (array-response), (delay-array-response), (spatial-response-y/z)).
// The local vector: LOS r = R^T (x - p_pa); surface with SFV v: virtual
// anchor p_va = p_pa - (2 p_pa.v / |v|^2 - 1) v, Householder mirror of
// x - p_va across v, then R^T (Sec. II-A).
struct Kron {
  double2 g, b0, bs, y0, ys, z0, zs;
};

__device__ Kron path_kron(const MsgGeom& G, int j, const double* __restrict__ x, const double* __restrict__ v) {
  const double* pa = G.pa + 3 * j;
  const double* R = G.rot + 9 * j;
  double w0 = x[0] - pa[0], w1 = x[1] - pa[1], w2 = x[2] - pa[2];
  if (v) {
    const double v0 = v[0], v1 = v[1], v2 = v[2];
    const double vv = v0 * v0 + v1 * v1 + v2 * v2;
    const double k1 = 2.0 * (pa[0] * v0 + pa[1] * v1 + pa[2] * v2) / vv - 1.0;
    const double d0 = w0 + k1 * v0, d1 = w1 + k1 * v1, d2 = w2 + k1 * v2;  // x - p_va
    const double k2 = 2.0 * (d0 * v0 + d1 * v1 + d2 * v2) / vv;
    w0 = d0 - k2 * v0;
    w1 = d1 - k2 * v1;
    w2 = d2 - k2 * v2;
  }
  const double r0 = R[0] * w0 + R[3] * w1 + R[6] * w2;
  const double r1 = R[1] * w0 + R[4] * w1 + R[7] * w2;
  const double r2 = R[2] * w0 + R[5] * w1 + R[8] * w2;
  const double d = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
  const double lam = kC / G.fc;
  Kron k;
  k.g = cscale(lam / (4.0 * kPi * d), cexpi(-2.0 * kPi * G.fc * d / kC));
  // step e^{j theta} = h^2 and first term e^{-j theta (n-1)/2} = conj(h)^(n-1), h = e^{j theta / 2}
  const double2 hf = cexpi(-kPi * G.df * d / kC);
  const double2 hy = cexpi(0.5 * kPi * r1 / d), hz = cexpi(0.5 * kPi * r2 / d);
  k.bs = cmul(hf, hf);
  k.ys = cmul(hy, hy);
  k.zs = cmul(hz, hz);
  k.b0 = cpowi(cconj(hf), G.nf - 1);
  k.y0 = cpowi(cconj(hy), G.ny - 1);
  k.z0 = cpowi(cconj(hz), G.nz - 1);
  return k;
}

// a^H X = conj(g) sum_f conj(b_f) sum_i conj(y_i) sum_l conj(z_l) X[f][i][l],
// X read wave-uniformly; NZ > 0 fixes N_z at compile time (the vertical
// phasors then sit in registers instead of being generated by recurrence).
template <int NZ>
__device__ double2 contract(const Kron& k, cvec X, int nf, int ny, int nzr) {
  const int nz = NZ > 0 ? NZ : nzr;
  const double2 bsc = cconj(k.bs), ysc = cconj(k.ys), zsc = cconj(k.zs);
  double2 zc[NZ > 0 ? NZ : 1];
  if constexpr (NZ > 0) {
    double2 v = cconj(k.z0);
#pragma unroll
    for (int l = 0; l < NZ; ++l) {
      zc[l] = v;
      v = cmul(v, zsc);
    }
  }
  double2 af = {0.0, 0.0};
  double2 bf = cconj(k.b0);
  for (int f = 0; f < nf; ++f) {
    double2 ai = {0.0, 0.0};
    double2 yi = cconj(k.y0);
    for (int i = 0; i < ny; ++i) {
      const int base = (f * ny + i) * nz;
      double2 al = {0.0, 0.0};
      if constexpr (NZ > 0) {
#pragma unroll
        for (int l = 0; l < NZ; ++l) al = cmac(al, zc[l], ld(X, base + l));
      } else {
        double2 zl = cconj(k.z0);
        for (int l = 0; l < nz; ++l) {
          al = cmac(al, zl, ld(X, base + l));
          zl = cmul(zl, zsc);
        }
      }
      ai = cmac(ai, yi, al);
      yi = cmul(yi, ysc);
    }
    af = cmac(af, bf, ai);
    bf = cmul(bf, bsc);
  }
  return cmulc(k.g, af);
}

// sum_k conj(x0 xs^k) (t0 ts^k), k < n; real for centred sequences
__device__ __forceinline__ double seqdot(double2 x0, double2 xs, double2 t0, double2 ts, int n) {
  const double2 r = cmulc(xs, ts);
  double2 t = cmulc(x0, t0);
  double s = 0.0;
  for (int q = 0; q < n; ++q) {
    s += t.x;
    t = cmul(t, r);
  }
  return s;
}

// Cholesky of the Hermitian positive definite matrix whose row `me` lane
// `me` of the group holds in H (H = L L^H; on return H[t], t <= me, is row
// `me` of L, whose diagonal is real); returns L_{me,me}.
template <int GS>
__device__ __forceinline__ double group_cholesky(double2 (&H)[GS], int me) {
  double diag = 1.0;
#pragma unroll
  for (int k = 0; k < GS; ++k) {
    const double lkk = sqrt(__shfl(H[k].x, k, GS));
    if (me == k) {
      H[k] = {lkk, 0.0};
      diag = lkk;
    } else if (me > k) {
      H[k] = cscale(1.0 / lkk, H[k]);
    }
#pragma unroll
    for (int t = k + 1; t < GS; ++t) {
      const double2 ltk = gshfl<GS>(H[k], t);
      if (me >= t) H[t] = csub(H[t], cmul(H[k], cconj(ltk)));
    }
  }
  return diag;
}

// forward substitution L q = b with row `me` of L in Lr (diagonal real)
template <int GS>
__device__ __forceinline__ double2 group_forward(const double2 (&Lr)[GS], double2 b, int me) {
#pragma unroll
  for (int k = 0; k < GS; ++k) {
    if (me == k) b = cscale(1.0 / Lr[k].x, b);
    const double2 bk = gshfl<GS>(b, k);
    if (me > k) b = csub(b, cmul(Lr[k], bk));
  }
  return b;
}

struct MsgWs {
  double* rho;    // [16] PF existence probabilities sum_p w_alpha
  double* etam;   // [16] noise prior means
  double2* part;  // [nchunk][S][J][3][N_z] chunk partial sums
  double2* avg;   // [4][S][J][N_z]: m, w, m3, m4
  double2* zp;    // [S][J][N_z] z minus the other features' means
  double2* L;     // [S][J][GS][GS] Cholesky of I + G_s / eta~ (identity at s)
  double2* wv;    // [S][J][GS] L^{-1} M_s^H z'
  double* kc;     // [S][J][2] z'^H A^{-1} z', log det A
  double2* gnu;   // [J][GS][GS] Gram of all columns
  double2* bnu;   // [J][GS] M^H (z - sum_t m3_t)
  double* jc;     // [J][2] |z - sum_t m3_t|^2, |z|^2
};

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

MsgWs carve(void* base, const MsgGeom& g, int S, int P, size_t* total) {
  const size_t Nz = size_t(g.nf) * g.ny * g.nz, J = g.J, GS = msg_group(S);
  const size_t nchunk = (size_t(P) + kChunk - 1) / kChunk;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += al256(bytes);
    return o;
  };
  const size_t o_rho = take(16 * 8), o_eta = take(16 * 8);
  const size_t o_part = take(nchunk * S * J * 3 * Nz * 16);
  const size_t o_avg = take(4 * S * J * Nz * 16);
  const size_t o_zp = take(S * J * Nz * 16);
  const size_t o_L = take(S * J * GS * GS * 16);
  const size_t o_wv = take(S * J * GS * 16);
  const size_t o_kc = take(S * J * 2 * 8);
  const size_t o_gnu = take(J * GS * GS * 16);
  const size_t o_bnu = take(J * GS * 16);
  const size_t o_jc = take(J * 2 * 8);
  if (total) *total = off;
  char* b = static_cast<char*>(base);
  MsgWs w;
  w.rho = reinterpret_cast<double*>(b + o_rho);
  w.etam = reinterpret_cast<double*>(b + o_eta);
  w.part = reinterpret_cast<double2*>(b + o_part);
  w.avg = reinterpret_cast<double2*>(b + o_avg);
  w.zp = reinterpret_cast<double2*>(b + o_zp);
  w.L = reinterpret_cast<double2*>(b + o_L);
  w.wv = reinterpret_cast<double2*>(b + o_wv);
  w.kc = reinterpret_cast<double*>(b + o_kc);
  w.gnu = reinterpret_cast<double2*>(b + o_gnu);
  w.bnu = reinterpret_cast<double2*>(b + o_bnu);
  w.jc = reinterpret_cast<double*>(b + o_jc);
  return w;
}

// Fixed-order sum over a workgroup of NT threads (result valid in thread 0).
template <int NT>
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int w = NT / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// rho_s = sum_p w_alpha,s^p (workgroups 0..S-1); eta~_j = sum_p w_xi^(j,p)
// eta^(j,p) (workgroups S..S+J-1)
__global__ __launch_bounds__(1024) void k_msg_scalars(MsgIn in, int J, double* __restrict__ rho,
                                                      double* __restrict__ etam) {
  __shared__ double red[1024];
  const int b = blockIdx.x, P = in.P;
  const bool ex = b < in.S;
  const double* w = ex ? in.wa + int64_t(b) * P : in.wxi + int64_t(b - in.S) * P;
  const double* e = ex ? nullptr : in.eta + int64_t(b - in.S) * P;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p0 = threadIdx.x; p0 < P; p0 += 4096) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = p0 + 1024 * q;
      if (p < P) acc[q] += ex ? w[p] : w[p] * e[p];
    }
  }
  const double t = block_sum<1024>((acc[0] + acc[1]) + (acc[2] + acc[3]), red);
  if (threadIdx.x == 0) {
    if (ex)
      rho[b] = t;
    else
      etam[b - in.S] = t;
  }
}

// Partial sums over one chunk of particles, for feature s at array j, of
//   w_beta sqrt(gamma + |mu|^2 (1 - zeta rho)) a,  w_beta sqrt(gamma + |mu|^2 (1 - rho)) a,
//   w_beta mu a.
// Each round puts 64 particles' Kronecker factors in LDS; thread e then
// forms a[e] = (g b_f) y_i z_l for each of its elements (N_z <= 1024).
__global__ __launch_bounds__(256) void k_msg_reduce(MsgGeom G, MsgIn in, const double* __restrict__ rho,
                                                    double2* __restrict__ part) {
  extern __shared__ double2 sm[];
  const int nf = G.nf, ny = G.ny, nz = G.nz, Nz = nf * ny * nz, nt = nf + ny + nz;
  double2* tab = sm;                   // [kSub][nt]
  double2* wt = sm + kSub * nt;        // [kSub][2]: (w1, w2), w3
  const int chunk = blockIdx.x, s = blockIdx.y, j = blockIdx.z, J = G.J;
  const int S = in.S, P = in.P;
  const double zeta = in.zeta[s * J + j], rh = rho[s];
  const double pdd = 1.0 - zeta * rh, pd = 1.0 - rh;
  int fe[4], ie[4], le[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q;
    fe[q] = e / (ny * nz);
    ie[q] = (e / nz) % ny;
    le[q] = e % nz;
  }
  double2 a1[4], a2[4], a3[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) a1[q] = a2[q] = a3[q] = {0.0, 0.0};
  const int p_end = min(P, (chunk + 1) * kChunk);
  for (int p0 = chunk * kChunk; p0 < p_end; p0 += kSub) {
    __syncthreads();
    if (threadIdx.x < kSub) {
      const int p = p0 + threadIdx.x;
      double2* row = tab + threadIdx.x * nt;
      if (p < p_end) {
        const Kron k = path_kron(G, j, in.mt + 3 * int64_t(p), s ? in.sfv + (int64_t(s) * P + p) * 3 : nullptr);
        double2 v = cmul(k.g, k.b0);
        for (int f = 0; f < nf; ++f) {
          row[f] = v;
          v = cmul(v, k.bs);
        }
        v = k.y0;
        for (int i = 0; i < ny; ++i) {
          row[nf + i] = v;
          v = cmul(v, k.ys);
        }
        v = k.z0;
        for (int l = 0; l < nz; ++l) {
          row[nf + ny + l] = v;
          v = cmul(v, k.zs);
        }
        const double wb = in.wb[p];
        const double gm = in.gamma[int64_t(s) * P + p];
        const double2 mu = in.mu[int64_t(s) * P + p];
        const double m2 = cabs2(mu);
        wt[2 * threadIdx.x] = {wb * sqrt(gm + m2 * pdd), wb * sqrt(gm + m2 * pd)};
        wt[2 * threadIdx.x + 1] = cscale(wb, mu);
      } else {
        for (int q = 0; q < nt; ++q) row[q] = {0.0, 0.0};
        wt[2 * threadIdx.x] = {0.0, 0.0};
        wt[2 * threadIdx.x + 1] = {0.0, 0.0};
      }
    }
    __syncthreads();
    const int np = min(kSub, p_end - p0);
    for (int q = 0; q < np; ++q) {
      const double2* row = tab + q * nt;
      const double2 w12 = wt[2 * q], w3 = wt[2 * q + 1];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (threadIdx.x + 256 * r < Nz) {
          const double2 a = cmul(row[fe[r]], cmul(row[nf + ie[r]], row[nf + ny + le[r]]));
          a1[r] = cadd(a1[r], cscale(w12.x, a));
          a2[r] = cadd(a2[r], cscale(w12.y, a));
          a3[r] = cadd(a3[r], cmul(w3, a));
        }
      }
    }
  }
  double2* out = part + ((int64_t(chunk) * S + s) * J + j) * 3 * Nz;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = threadIdx.x + 256 * r;
    if (e < Nz) {
      out[e] = a1[r];
      out[Nz + e] = a2[r];
      out[2 * Nz + e] = a3[r];
    }
  }
}

// The same partial sums as a rank-P update: with U_k,p[f] = W_k,p g_p b_p[f]
// (W_1, W_2 the real square-root weights, W_3 = w_beta mu) and V_p[il] =
// y_p[i] z_p[l], out_k[f][il] = sum_p U_k,p[f] V_p[il]. Each round forms the
// paths of 256 particles (one per thread) as compact phasors in LDS; in
// sub-rounds of 32 particles their U rows and V are expanded into a stage,
// and a thread owns the 3 x kRedCB tile (k = 0..2 at one f, kRedCB
// consecutive il) while groups of nf * ceil(N_y N_z / kRedCB) threads split
// the sub-round's particles. Groups are summed in fixed order.
// Requires nf * ceil(N_y N_z / kRedCB) <= 256 and 3 nf + N_y N_z <= 256.
// LDS row stride of a staged particle: rows of consecutive particles start 16
// dwords apart modulo 32 banks (a row of n complex values is 4n dwords)
__host__ __device__ inline int stage_row(int n) { return n + ((4 - n % 8) + 8) % 8; }
constexpr int kRedR = 128;  // particles per round (paths formed)
constexpr int kRedSub = 32; // particles per expanded sub-round
constexpr int kRedCB = 4;   // il columns of a thread's tile

__global__ __launch_bounds__(256) void k_msg_reduce_tile(MsgGeom G, MsgIn in, const double* __restrict__ rho,
                                                         double2* __restrict__ part) {
  extern __shared__ double2 sm[];
  const int nf = G.nf, ny = G.ny, nz = G.nz, nyz = ny * nz, Nz = nf * nyz, J = G.J;
  const int S = in.S, P = in.P;
  const int ncb = (nyz + kRedCB - 1) / kRedCB;
  const int T = nf * ncb, NG = 256 / T;
  const int per = stage_row(3 * nf + nyz);  // staged complex values per particle (padded)
  Kron* kp = reinterpret_cast<Kron*>(sm);                       // [kRedR]
  double2* wts = reinterpret_cast<double2*>(kp + kRedR);         // [kRedR][2]: (w1, w2), w3
  double2* stage = wts + 2 * kRedR;                              // [kRedSub][per]
  double2* red = stage + kRedSub * per;                          // [3][nf][nyz]
  const int chunk = blockIdx.x, s = blockIdx.y, j = blockIdx.z;
  const double zeta = in.zeta[s * J + j], rh = rho[s];
  const double pdd = 1.0 - zeta * rh, pd = 1.0 - rh;
  const int grp = threadIdx.x / T, rr = threadIdx.x - grp * T;
  const int f = rr / ncb, cb = rr - f * ncb;  // columns cb, cb + ncb, cb + 2 ncb, ...
  const bool act = grp < NG;
  double2 acc[3][kRedCB];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < kRedCB; ++c) acc[k][c] = {0.0, 0.0};
  const int p_end = min(P, (chunk + 1) * kChunk);
  for (int p0 = chunk * kChunk; p0 < p_end; p0 += kRedR) {
    const int nr = min(kRedR, p_end - p0);
    __syncthreads();
    {
      const int q = threadIdx.x, p = p0 + q;
      if (q < nr) {
        kp[q] = path_kron(G, j, in.mt + 3 * int64_t(p), s ? in.sfv + (int64_t(s) * P + p) * 3 : nullptr);
        const double wb = in.wb[p];
        const double gm = in.gamma[int64_t(s) * P + p];
        const double2 mu = in.mu[int64_t(s) * P + p];
        const double m2 = cabs2(mu);
        wts[2 * q] = {wb * sqrt(gm + m2 * pdd), wb * sqrt(gm + m2 * pd)};
        wts[2 * q + 1] = cscale(wb, mu);
      }
    }
    for (int q0 = 0; q0 < nr; q0 += kRedSub) {
      const int np = min(kRedSub, nr - q0);
      __syncthreads();
      {
        // expand: threads [0, 3 kRedSub) write U rows, [3 kRedSub, 4 kRedSub) V
        const int q = threadIdx.x % kRedSub, pt = threadIdx.x / kRedSub;
        if (q < np && pt < 4) {
          const Kron k = kp[q0 + q];
          double2* row = stage + q * per;
          if (pt < 3) {
            const double2 wq = wts[2 * (q0 + q) + (pt == 2 ? 1 : 0)];
            const double2 w = pt == 2 ? wq : double2{pt == 0 ? wq.x : wq.y, 0.0};
            double2 v = cmul(w, cmul(k.g, k.b0));
            for (int ff = 0; ff < nf; ++ff) {
              row[pt * nf + ff] = v;
              v = cmul(v, k.bs);
            }
          } else {
            double2 y = k.y0;
            for (int i = 0; i < ny; ++i) {
              double2 zz = cmul(y, k.z0);
              for (int l = 0; l < nz; ++l) {
                row[3 * nf + i * nz + l] = zz;
                zz = cmul(zz, k.zs);
              }
              y = cmul(y, k.ys);
            }
          }
        }
      }
      __syncthreads();
      if (act) {
        for (int q = grp; q < np; q += NG) {
          const double2* row = stage + q * per;
          const double2 u0 = row[f], u1 = row[nf + f], u2 = row[2 * nf + f];
          const double2* vr = row + 3 * nf + cb;
#pragma unroll
          for (int c = 0; c < kRedCB; ++c) {
            if (cb + c * ncb < nyz) {
              const double2 v = vr[c * ncb];
              acc[0][c] = cmac(acc[0][c], u0, v);
              acc[1][c] = cmac(acc[1][c], u1, v);
              acc[2][c] = cmac(acc[2][c], u2, v);
            }
          }
        }
      }
    }
  }
  // groups in order into red, then out
  for (int g = 0; g < NG; ++g) {
    __syncthreads();
    if (act && grp == g) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < kRedCB; ++c) {
          if (cb + c * ncb < nyz) {
            double2* d = red + (k * nf + f) * nyz + cb + c * ncb;
            *d = g == 0 ? acc[k][c] : cadd(*d, acc[k][c]);
          }
        }
    }
  }
  __syncthreads();
  double2* out = part + ((int64_t(chunk) * S + s) * J + j) * 3 * Nz;
  for (int e = threadIdx.x; e < 3 * Nz; e += 256) out[e] = red[e];
}

// m = rho zeta sum1, w = rho sum2, m4 = rho sum3, m3 = zeta m4. Workgroup
// (feature-array, sum, 64 elements); its four waves take every fourth chunk,
// and the four partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_msg_combine(MsgGeom G, MsgIn in, int nchunk, const double* __restrict__ rho,
                                                     const double2* __restrict__ part, double2* __restrict__ avg) {
  __shared__ double2 red[4][64];
  const int J = G.J, S = in.S, Nz = G.nf * G.ny * G.nz;
  const int sj = blockIdx.x, s = sj / J, j = sj - s * J, kind = blockIdx.y;
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int e = blockIdx.z * 64 + lane;
  double2 acc = {0.0, 0.0};
  if (e < Nz) {
    const int64_t cstride = int64_t(S) * J * 3 * Nz;
    const double2* pc = part + (int64_t(s) * J + j) * 3 * Nz + int64_t(kind) * Nz + e;
#pragma unroll 4
    for (int c = g; c < nchunk; c += 4) acc = cadd(acc, pc[c * cstride]);
  }
  red[g][lane] = acc;
  __syncthreads();
  if (g != 0 || e >= Nz) return;
  const double2 t = cadd(cadd(red[0][lane], red[1][lane]), cadd(red[2][lane], red[3][lane]));
  const double zeta = in.zeta[s * J + j], rh = rho[s];
  const int64_t vec = int64_t(S) * J * Nz;
  const int64_t o = (int64_t(s) * J + j) * Nz + e;
  if (kind == 0) {
    avg[o] = cscale(rh * zeta, t);
  } else if (kind == 1) {
    avg[vec + o] = cscale(rh, t);
  } else {
    const double2 m4 = cscale(rh, t);
    avg[2 * vec + o] = cscale(zeta, m4);
    avg[3 * vec + o] = m4;
  }
}

__device__ void pair_of(int d, int S, int* t, int* u) {
  int r = 0;
  while (d >= S - r) {
    d -= S - r;
    ++r;
  }
  *t = r;
  *u = r + d;
}

// in-place Cholesky of the n x n Hermitian matrix H (row-major, stride 16),
// lower triangle; zeroes the upper triangle
__device__ void serial_cholesky(double2* H, int n) {
  for (int k = 0; k < n; ++k) {
    double d = H[k * 16 + k].x;
    for (int m = 0; m < k; ++m) d -= cabs2(H[k * 16 + m]);
    const double lkk = sqrt(d);
    H[k * 16 + k] = {lkk, 0.0};
    for (int i = k + 1; i < n; ++i) {
      double2 v = H[i * 16 + k];
      for (int m = 0; m < k; ++m) v = csub(v, cmul(H[i * 16 + m], cconj(H[k * 16 + m])));
      H[i * 16 + k] = cscale(1.0 / lkk, v);
    }
    for (int u = k + 1; u < n; ++u) H[k * 16 + u] = {0.0, 0.0};
  }
}

__device__ void serial_forward(const double2* L, double2* b, int n) {
  for (int i = 0; i < n; ++i) {
    double2 v = b[i];
    for (int m = 0; m < i; ++m) v = csub(v, cmul(L[i * 16 + m], b[m]));
    b[i] = cscale(1.0 / L[i * 16 + i].x, v);
  }
}

// Workgroup (s < S, j): the PF message's A = eta~ I + M_s M_s^H (columns of
// every feature but s): Cholesky of I + G_s / eta~ (row and column s replaced
// by the identity), z' = z - sum_{t != s} m3_t, w = L^{-1} M_s^H z',
// z'^H A^{-1} z' and log det A; the PF message at r = 0 and the PR message
// at r = 0, 1 (Sherman-Morrison on top of A).
// Workgroup (S, j): the noise message's Gram of all columns, M^H e and |e|^2
// for e = z - sum_t m3_t, and |z|^2.
__global__ __launch_bounds__(1024) void k_msg_setup(MsgGeom G, int S, int GS, const double2* __restrict__ z,
                                                   MsgWs W, double* __restrict__ kappa0,
                                                   double* __restrict__ omega) {
  extern __shared__ double2 sm[];
  const int Nz = G.nf * G.ny * G.nz, J = G.J;
  const int s = blockIdx.x, j = blockIdx.y;
  const bool nub = s == S;
  double2* v = sm;               // [N_z]
  double2* dots = sm + Nz;       // [kMaxDots]
  double2* H = dots + kMaxDots;  // [16][16]
  double2* rhs = H + 256;        // [3][16]
  const int64_t vec = int64_t(S) * J * Nz;
  auto col = [&](int kind, int t) { return W.avg + kind * vec + (int64_t(t) * J + j) * Nz; };
  for (int e = threadIdx.x; e < Nz; e += 1024) {
    double2 acc = z[int64_t(j) * Nz + e];
    for (int t = 0; t < S; ++t)
      if (t != s) acc = csub(acc, col(2, t)[e]);
    v[e] = acc;
    if (!nub) W.zp[(int64_t(s) * J + j) * Nz + e] = acc;
  }
  __syncthreads();
  const int nG = S * (S + 1) / 2;
  const int nd = nub ? nG + S + 2 : nG + 3 * S + 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int d = wave; d < nd; d += 16) {
    const double2 *x, *y;
    if (d < nG) {
      int t, u;
      pair_of(d, S, &t, &u);
      x = col(0, t);
      y = col(0, u);
    } else if (d < nG + S) {
      x = col(0, d - nG);
      y = v;
    } else if (nub) {
      x = y = (d == nG + S) ? v : z + int64_t(j) * Nz;
    } else if (d < nG + 2 * S) {
      x = col(0, d - nG - S);
      y = col(1, s);
    } else if (d < nG + 3 * S) {
      x = col(0, d - nG - 2 * S);
      y = col(3, s);
    } else {
      const int q = d - nG - 3 * S;
      const double2* ws = col(1, s);
      const double2* m4 = col(3, s);
      const double2* xs[6] = {v, ws, ws, ws, m4, m4};
      const double2* ys[6] = {v, v, ws, m4, v, m4};
      x = xs[q];
      y = ys[q];
    }
    double2 acc = {0.0, 0.0};
    for (int e = lane; e < Nz; e += 64) acc = cmacc(acc, x[e], y[e]);
    acc = gsum<64>(acc);
    if (lane == 0) dots[d] = acc;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  auto gram = [&](int t, int u) {
    int a = t < u ? t : u, b = t < u ? u : t;
    const int d = a * S - a * (a - 1) / 2 + (b - a);
    return t <= u ? dots[d] : cconj(dots[d]);
  };
  const double eta = W.etam[j];
  const double lpi = double(Nz) * log(kPi);
  if (nub) {
    for (int t = 0; t < GS; ++t) {
      for (int u = 0; u < GS; ++u)
        W.gnu[(int64_t(j) * GS + t) * GS + u] = (t < S && u < S) ? gram(t, u) : double2{0.0, 0.0};
      W.bnu[int64_t(j) * GS + t] = t < S ? dots[nG + t] : double2{0.0, 0.0};
    }
    W.jc[2 * j] = dots[nG + S].x;
    W.jc[2 * j + 1] = dots[nG + S + 1].x;
    return;
  }
  for (int t = 0; t < GS; ++t)
    for (int u = 0; u < GS; ++u) {
      double2 h = {t == u ? 1.0 : 0.0, 0.0};
      if (t < S && u < S && t != s && u != s) h = cadd(h, cscale(1.0 / eta, gram(t, u)));
      H[t * 16 + u] = h;
    }
  serial_cholesky(H, GS);
  for (int t = 0; t < GS; ++t) {
    const bool on = t < S && t != s;
    const double2 h = on ? dots[nG + t] : double2{0.0, 0.0};            // m_t^H z'
    const double2 pw = on ? dots[nG + S + t] : double2{0.0, 0.0};       // m_t^H w_s
    const double2 r4 = on ? dots[nG + 2 * S + t] : double2{0.0, 0.0};   // m_t^H m4_s
    rhs[t] = h;
    rhs[16 + t] = pw;
    rhs[32 + t] = csub(h, r4);
  }
  serial_forward(H, rhs, GS);
  serial_forward(H, rhs + 16, GS);
  serial_forward(H, rhs + 32, GS);
  double logdet = double(Nz) * log(eta), ww = 0.0, uww = 0.0, uee = 0.0;
  double2 uwe = {0.0, 0.0};
  for (int t = 0; t < GS; ++t) {
    logdet += 2.0 * log(H[t * 16 + t].x);
    ww += cabs2(rhs[t]);
    uww += cabs2(rhs[16 + t]);
    uee += cabs2(rhs[32 + t]);
    uwe = cadd(uwe, cmulc(rhs[16 + t], rhs[32 + t]));
  }
  const double2* q = dots + nG + 3 * S;  // |z'|^2, w^H z', |w|^2, w^H m4, m4^H z', |m4|^2
  const double qzz = q[0].x / eta - ww / (eta * eta);
  const double k0 = -lpi - logdet - qzz;
  const int sj = s * J + j;
  for (int t = 0; t < GS; ++t) {
    for (int u = 0; u < GS; ++u) W.L[(int64_t(sj) * GS + t) * GS + u] = H[t * 16 + u];
    W.wv[int64_t(sj) * GS + t] = rhs[t];
  }
  W.kc[2 * sj] = qzz;
  W.kc[2 * sj + 1] = logdet;
  if (kappa0) kappa0[sj] = k0;
  if (omega) {
    const double wAw = q[2].x / eta - uww / (eta * eta);
    const double2 wAe = csub(cscale(1.0 / eta, csub(q[1], q[3])), cscale(1.0 / (eta * eta), uwe));
    const double eAe = (q[0].x - 2.0 * q[4].x + q[5].x) / eta - uee / (eta * eta);
    const double den = 1.0 + wAw;
    omega[2 * sj] = k0;
    omega[2 * sj + 1] = cabs2(wAe) / den - eAe - lpi - log(den) - logdet;
  }
}

// MT message (and noise message) at (particle p, array j): group of GS lanes,
// lane s owns feature s.
template <int GS, int NZ>
__global__ __launch_bounds__(256) void k_msg_pair(MsgGeom G, MsgIn in, MsgWs W, double* __restrict__ iota,
                                                  double* __restrict__ nu) {
  __shared__ double2 slot[256 * kSlot];
  const int nf = G.nf, ny = G.ny, nz = G.nz, Nz = nf * ny * nz, J = G.J;
  const int S = in.S, P = in.P;
  const int j = blockIdx.y;
  const int s = threadIdx.x % GS;
  const int gbase = threadIdx.x - s;
  const int64_t p = int64_t(blockIdx.x) * (256 / GS) + threadIdx.x / GS;
  const int64_t pc = p < P ? p : P - 1;
  const double eta = W.etam[j];
  Kron k{};
  double c = 0.0;
  double2 pm = {0.0, 0.0};
  if (s < S) {
    k = path_kron(G, j, in.mt + 3 * pc, s ? in.sfv + (int64_t(s) * P + pc) * 3 : nullptr);
    const double pe = in.zeta[s * J + j] * W.rho[s];
    const double2 mu = in.mu[int64_t(s) * P + pc];
    c = pe * (in.gamma[int64_t(s) * P + pc] + cabs2(mu) * (1.0 - pe));
    pm = cscale(pe, mu);
  }
  // a_s^H z (padded lanes have g = 0)
  const double2 y = contract<NZ>(k, uniform_vec(in.z + int64_t(j) * Nz), nf, ny, nz);
  double2* my = slot + threadIdx.x * kSlot;
  my[0] = k.g;
  my[1] = k.b0;
  my[2] = k.bs;
  my[3] = k.y0;
  my[4] = k.ys;
  my[5] = k.z0;
  my[6] = k.zs;
  my[7] = pm;
  my[8] = {c, 0.0};
  __syncthreads();
  // row s of G0 = [<a_s, a_t>], of I + diag(sqrt c) G0 diag(sqrt c) / eta, and sum_t pm_t G0_st
  double2 H[GS];
  double2 sg = {0.0, 0.0};
  const double sc = sqrt(c);
#pragma unroll
  for (int t = 0; t < GS; ++t) {
    const double2* o = slot + (gbase + t) * kSlot;
    double2 g0 = {0.0, 0.0};
    if (s < S && t < S) {
      const double d = seqdot(k.b0, k.bs, o[1], o[2], nf) * seqdot(k.y0, k.ys, o[3], o[4], ny) *
                       seqdot(k.z0, k.zs, o[5], o[6], nz);
      g0 = cscale(d, cmulc(k.g, o[0]));
    }
    sg = cmac(sg, o[7], g0);
    H[t] = cscale(sc * sqrt(o[8].x) / eta, g0);
    if (t == s) H[t].x += 1.0;
  }
  // b_s = m_s^H (z - sum_t pm_t a_t); |z - sum_t pm_t a_t|^2 summed over the group
  const double2 b = cscale(sc, csub(y, sg));
  const double e2 = W.jc[2 * j + 1] + gsum<GS>(-2.0 * cmulc(pm, y).x + cmulc(pm, sg).x);
  const double lkk = group_cholesky<GS>(H, s);
  const double2 q = group_forward<GS>(H, b, s);
  const double logdet = 2.0 * gsum<GS>(log(lkk));
  const double qq = gsum<GS>(cabs2(q));
  if (iota && s == 0 && p < P)
    iota[int64_t(j) * P + p] = -double(Nz) * log(kPi * eta) - logdet - e2 / eta + qq / (eta * eta);
  if (nu) {
    const double ep = in.eta[int64_t(j) * P + pc];
    double2 Hn[GS];
#pragma unroll
    for (int t = 0; t < GS; ++t) {
      Hn[t] = cscale(1.0 / ep, W.gnu[(int64_t(j) * GS + s) * GS + t]);
      if (t == s) Hn[t].x += 1.0;
    }
    const double ln = group_cholesky<GS>(Hn, s);
    const double2 qn = group_forward<GS>(Hn, W.bnu[int64_t(j) * GS + s], s);
    const double ldn = 2.0 * gsum<GS>(log(ln));
    const double qqn = gsum<GS>(cabs2(qn));
    if (s == 0 && p < P)
      nu[int64_t(j) * P + p] = -double(Nz) * log(kPi * ep) - ldn - W.jc[2 * j] / ep + qqn / (ep * ep);
  }
}

// PF message at r = 1 for (feature s, particle p, array j), one thread per
// particle. The S dense columns (m_t for t != s; z' at t = s) are read
// wave-uniformly, and each element of the path is generated once for all of
// them. SC columns are contracted: SC = S for S <= 8, else 16 (the extra
// columns repeat column 0 and are discarded).
template <int SC, int NZ>
__global__ __launch_bounds__(256) void k_msg_kappa(MsgGeom G, MsgIn in, MsgWs W, int GS, double* __restrict__ kappa) {
  const int nf = G.nf, ny = G.ny, nz = NZ > 0 ? NZ : G.nz, Nz = nf * ny * nz, J = G.J;
  const int S = in.S, P = in.P;
  const int sj = blockIdx.y, s = sj / J, j = sj - s * J;
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t pc = p < P ? p : P - 1;
  const double eta = W.etam[j];
  const Kron k = path_kron(G, j, in.mt + 3 * pc, s ? in.sfv + (int64_t(s) * P + pc) * 3 : nullptr);
  cvec X[SC];
#pragma unroll
  for (int t = 0; t < SC; ++t) {
    const int tt = t < S ? t : 0;
    X[t] = uniform_vec(tt == s ? W.zp + int64_t(sj) * Nz : W.avg + (int64_t(tt) * J + j) * Nz);
  }
  double2 acc[SC];
#pragma unroll
  for (int t = 0; t < SC; ++t) acc[t] = {0.0, 0.0};
  double2 zl[NZ > 0 ? NZ : 1];
  if constexpr (NZ > 0) {
    double2 v = k.z0;
#pragma unroll
    for (int l = 0; l < NZ; ++l) {
      zl[l] = v;
      v = cmul(v, k.zs);
    }
  }
  double2 bf = cmul(k.g, k.b0);
  for (int f = 0; f < nf; ++f) {
    double2 yi = k.y0;
    for (int i = 0; i < ny; ++i) {
      const double2 w = cmul(bf, yi);
      const int base = (f * ny + i) * nz;
      if constexpr (NZ > 0) {
#pragma unroll
        for (int l = 0; l < NZ; ++l) {
          const double2 a = cmul(w, zl[l]);
#pragma unroll
          for (int t = 0; t < SC; ++t) acc[t] = cmacc(acc[t], ld(X[t], base + l), a);
        }
      } else {
        double2 zz = k.z0;
        for (int l = 0; l < nz; ++l) {
          const double2 a = cmul(w, zz);
#pragma unroll
          for (int t = 0; t < SC; ++t) acc[t] = cmacc(acc[t], ld(X[t], base + l), a);
          zz = cmul(zz, k.zs);
        }
      }
      yi = cmul(yi, k.ys);
    }
    bf = cmul(bf, k.bs);
  }
  // acc[t] = X_t^H a: (M_s^H a)_t for t != s, and a^H z' = conj(acc[s]);
  // u = L^{-1} M_s^H a with L of I + G_s / eta~ (identity at s and past S)
  const cvec Lm = uniform_vec(W.L + int64_t(sj) * GS * GS);
  const cvec wv = uniform_vec(W.wv + int64_t(sj) * GS);
  double2 u[SC];
  double uu = 0.0;
  double2 uw = {0.0, 0.0}, aHz = {0.0, 0.0};
#pragma unroll
  for (int t = 0; t < SC; ++t) {
    if (t == s) aHz = cconj(acc[t]);
    double2 r = (t < S && t != s) ? acc[t] : double2{0.0, 0.0};
#pragma unroll
    for (int m = 0; m < t; ++m) r = csub(r, cmul(ld(Lm, t * GS + m), u[m]));
    u[t] = cscale(1.0 / ld(Lm, t * GS + t).x, r);
    uu += cabs2(u[t]);
    uw = cmacc(uw, u[t], ld(wv, t));
  }
  const double aAa = double(Nz) * cabs2(k.g) / eta - uu / (eta * eta);
  const double2 aAz = csub(cscale(1.0 / eta, aHz), cscale(1.0 / (eta * eta), uw));
  const double zeta = in.zeta[s * J + j];
  const double2 mu = in.mu[int64_t(s) * P + pc];
  const double2 cm = cscale(zeta, mu);
  const double q = (in.gamma[int64_t(s) * P + pc] + cabs2(mu) * (1.0 - zeta)) * zeta;
  const double2 aAe = csub(aAz, cscale(aAa, cm));
  const double eAe = W.kc[2 * sj] - 2.0 * cmulc(cm, aAz).x + cabs2(cm) * aAa;
  const double den = 1.0 + q * aAa;
  if (p < P)
    kappa[int64_t(sj) * P + p] =
        q * cabs2(aAe) / den - eAe - double(Nz) * log(kPi) - log(den) - W.kc[2 * sj + 1];
}

template <int GS, int NZ>
hipError_t launch_pair(const MsgGeom& g, const MsgIn& in, const MsgOut& out, const MsgWs& w, hipStream_t st) {
  const int per = 256 / GS;
  const dim3 grid(unsigned((int64_t(in.P) + per - 1) / per), unsigned(g.J));
  k_msg_pair<GS, NZ><<<grid, 256, 0, st>>>(g, in, w, out.iota, out.nu);
  return hipGetLastError();
}

template <int SC, int NZ>
hipError_t launch_kappa(const MsgGeom& g, const MsgIn& in, const MsgOut& out, const MsgWs& w, hipStream_t st) {
  const dim3 grid(unsigned((int64_t(in.P) + 255) / 256), unsigned(in.S * g.J));
  k_msg_kappa<SC, NZ><<<grid, 256, 0, st>>>(g, in, w, msg_group(in.S), out.kappa);
  return hipGetLastError();
}

template <int NZ>
hipError_t launch_per_particle(const MsgGeom& g, const MsgIn& in, const MsgOut& out, const MsgWs& w,
                               hipStream_t st) {
  hipError_t e = hipSuccess;
  if (out.iota || out.nu) {
    const int gs = msg_group(in.S);
    e = gs == 4 ? launch_pair<4, NZ>(g, in, out, w, st)
                : (gs == 8 ? launch_pair<8, NZ>(g, in, out, w, st) : launch_pair<16, NZ>(g, in, out, w, st));
    if (e != hipSuccess) return e;
  }
  if (out.kappa) {
    switch (in.S) {
      case 1: return launch_kappa<1, NZ>(g, in, out, w, st);
      case 2: return launch_kappa<2, NZ>(g, in, out, w, st);
      case 3: return launch_kappa<3, NZ>(g, in, out, w, st);
      case 4: return launch_kappa<4, NZ>(g, in, out, w, st);
      case 5: return launch_kappa<5, NZ>(g, in, out, w, st);
      case 6: return launch_kappa<6, NZ>(g, in, out, w, st);
      case 7: return launch_kappa<7, NZ>(g, in, out, w, st);
      case 8: return launch_kappa<8, NZ>(g, in, out, w, st);
      default: return launch_kappa<16, NZ>(g, in, out, w, st);
    }
  }
  return e;
}

}  // namespace

int msg_group(int S) { return S <= 4 ? 4 : (S <= 8 ? 8 : 16); }

size_t msg_workspace_bytes(const MsgGeom& g, int S, int P) {
  size_t total = 0;
  (void)carve(nullptr, g, S, P, &total);
  return total;
}

hipError_t launch_messages(const MsgGeom& g, const MsgIn& in, const MsgOut& out, void* ws, hipStream_t st) {
  const MsgWs w = carve(ws, g, in.S, in.P, nullptr);
  const int Nz = g.nf * g.ny * g.nz;
  const int nchunk = int((int64_t(in.P) + kChunk - 1) / kChunk);
  k_msg_scalars<<<in.S + g.J, 1024, 0, st>>>(in, g.J, w.rho, w.etam);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid_r(unsigned(nchunk), unsigned(in.S), unsigned(g.J));
  const size_t lds_tile = kRedR * (sizeof(Kron) + 2 * sizeof(double2)) +
                          size_t(kRedSub) * stage_row(3 * g.nf + g.ny * g.nz) * sizeof(double2) +
                          size_t(3) * Nz * sizeof(double2);
  if (g.nf * ((g.ny * g.nz + kRedCB - 1) / kRedCB) <= 256 && 3 * g.nf + g.ny * g.nz <= 256 &&
      lds_tile <= kMaxLds) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_msg_reduce_tile),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_tile));
    if (e != hipSuccess) return e;
    k_msg_reduce_tile<<<grid_r, 256, lds_tile, st>>>(g, in, w.rho, w.part);
  } else {
    // N_f + N_y + N_z + 2 <= 98 complex per particle: at most 100 KB
    const size_t lds_r = size_t(kSub) * (g.nf + g.ny + g.nz + 2) * sizeof(double2);
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_msg_reduce), hipFuncAttributeMaxDynamicSharedMemorySize,
                            int(lds_r));
    if (e != hipSuccess) return e;
    k_msg_reduce<<<grid_r, 256, lds_r, st>>>(g, in, w.rho, w.part);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_msg_combine<<<dim3(unsigned(in.S * g.J), 3u, unsigned((Nz + 63) / 64)), 256, 0, st>>>(g, in, nchunk, w.rho,
                                                                                          w.part, w.avg);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds_s = size_t(Nz + kMaxDots + 256 + 48) * sizeof(double2);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_msg_setup), hipFuncAttributeMaxDynamicSharedMemorySize,
                          int(lds_s));
  if (e != hipSuccess) return e;
  k_msg_setup<<<dim3(unsigned(in.S + 1), unsigned(g.J)), 1024, lds_s, st>>>(g, in.S, msg_group(in.S), in.z, w,
                                                                           out.kappa0, out.omega);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return g.nz == 4 ? launch_per_particle<4>(g, in, out, w, st) : launch_per_particle<0>(g, in, out, w, st);
}

}  // namespace ba
