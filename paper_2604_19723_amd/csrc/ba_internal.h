// Internal declarations shared by the C-ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bartlett.h"

namespace ba {

constexpr int kMaxElem = 256;
constexpr int kMaxPeaks = 16;

struct Plan {
  int device = 0;
  int M = 0;
  int64_t G = 0;
  int kind = 0;
  int shape0 = 0, shape1 = 1, wrap0 = 0;
  int rows = 0;        // candidate rows of dim0 (shape0 - 1 when the last row duplicates the first)
  int ndim = 1;        // refined coordinates per peak
  int coord_dim = 1;   // moment coordinates per grid point
  int precision = BA_PREC_F32;

  std::vector<double> pos;     // [M][3]
  std::vector<double> coords;  // [G][coord_dim]

  // device tables (owned)
  float2* d_A = nullptr;       // [M][G] complex steering, A[m][g] = exp(+j 2 pi p_m . u_g)
  // real-equivalent steering x_g = [Re a_g; Im a_g] (rows padded to 2*Mp) in the
  // MFMA B-fragment order of the projection kernel: [Xblocks][2Mp/16][64 lanes][4]
  float* d_X = nullptr;
  uint16_t* d_Xb = nullptr;    // the same split into BF16 hi/lo (split precisions only)
  int Mp = 0;                  // padded element count of the tables (8 .. 256)
  int64_t Gb = 0;              // 16-column blocks that hold grid points
  int64_t Xblocks = 0;         // 16-column blocks in the tables (Gb padded to a multiple of 32)
  double* d_coords = nullptr;  // [G][coord_dim]
};

// launchers: argument validation happens before these are called
hipError_t launch_covariance(const Plan& p, int B, int T, const float2* Y, float2* R, hipStream_t s);
hipError_t launch_spectrum(const Plan& p, int B, const float2* R, float* P, void* ws, hipStream_t s);
size_t spectrum_ws_bytes(const Plan& p, int B);
size_t qprep_bytes(const Plan& p, int B);
hipError_t launch_spectrum_stream(const Plan& p, int B, const float2* R, void* Qws, float* P,
                                  hipStream_t s);
hipError_t launch_spectrum_valu(const Plan& p, int B, const float2* R, float* P, hipStream_t s);
hipError_t launch_spectrum_mfma(const Plan& p, int B, const float2* R, float* P, hipStream_t s);
// FP32 spectrum of *count trials (read on the device, at most cap), the
// launch sized for `expect` trials at a time
hipError_t launch_spectrum_mfma_counted(const Plan& p, int cap, const int* count, int expect, const float2* R,
                                        float* P, hipStream_t s);
hipError_t launch_spectrum_qb(const Plan& p, int B, const float2* R, float* P, hipStream_t s);
hipError_t launch_spectrum_snapshots(const Plan& p, int B, int T, const float2* Y, float* P,
                                     hipStream_t s);
// count: when non-NULL, the batch is *count trials (read on the device,
// at most B) and the launch is sized without reading it
hipError_t launch_peaks(const Plan& p, int B, const float* P, int k, int* idx, float* val,
                        double* refined, hipStream_t s, const int* count = nullptr);
hipError_t launch_moments(const Plan& p, int B, const float* P, double* mu_cov, hipStream_t s);

// Peak candidates from the projection epilogue (the register-resident paths
// of up to 64 elements, FP32 or the BF16 splits, on 1-D grids): each trial's
// candidate rows are cut into nsplit column ranges of `span` columns (the
// last one shorter); every range leaves k + 1 float4 records (its top-k
// interior maxima, then the values at its two ends).
constexpr int kMaxCandRanges = 64;
struct CandLayout {
  int nsplit = 1;    // column ranges per trial
  int per = 1;       // steering chunks per range
  int64_t span = 0;  // columns per range
};
bool candidates_supported(const Plan& p);
CandLayout candidate_layout(const Plan& p, int B);
size_t candidate_bytes(const Plan& p, int B, int k);
// P may be null (spectrum not written)
hipError_t launch_spectrum_candidates(const Plan& p, int B, const float2* R, float* P, int k, float4* rec,
                                      hipStream_t s);
hipError_t launch_peaks_merge(const Plan& p, int B, int k, const float4* rec, int* idx, float* val,
                              double* refined, hipStream_t s);
// the BF16 register-resident kernel's column split (trial pairs) and its candidate variant
void qb_split(const Plan& p, int B, int max_split, int* nsplit, int* per);
hipError_t launch_spectrum_qb_candidates(const Plan& p, int B, const float2* R, float* P, int k, float4* rec,
                                         hipStream_t s);

// residual covariance R~ = Pi R Pi (Psi given as vectors [B][S][M], or as grid
// indices gidx[b * ld + s] into the plan's steering table, -1 = no column)
hipError_t launch_residual(const Plan& p, int B, const float2* R, int S, const float2* Psi, const int* gidx,
                           int ld, float2* Rout, hipStream_t s);
size_t residual_lds_bytes(int M, int S);
hipError_t launch_put_column(int B, int c, int K, int ndim, const int* i1, const float* v1, const double* r1,
                             int* idx, float* val, double* ref, hipStream_t s);

// search region of the Gaussian proposal, per coordinate: [lo, hi], or
// periodic with the given period (> 0) starting at lo
struct ProposalRegion {
  double lo[3], hi[3], period[3];
};
hipError_t launch_proposal_sample(int B, const double* mu_cov, int d, int N, const double* z,
                                  const ProposalRegion& reg, double* particles, double* weights, hipStream_t s);

void set_error(const std::string& msg);
std::vector<float> plan_x_table(const Plan& p, int Mrows, int Mp, int64_t nblocks);

}  // namespace ba

// the opaque C handle is the plan itself
struct ba_plan_s : public ba::Plan {};
