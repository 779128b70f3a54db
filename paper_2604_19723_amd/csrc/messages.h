// Internal declarations of the particle update messages (Sec. IV-C and
// Supplementary Sec. S-V): the MT state message iota and the noise message nu
// at every (particle, array) pair, the PF state message kappa at every
// (feature, particle, array) triple, and the PR message omega per (feature,
// array).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ba {

// array geometry in device memory (FP64); the URA supports sit at half a
// wavelength and the N_f baseband bins are equally spaced and centred
struct MsgGeom {
  int J, nf, ny, nz;
  double fc;   // carrier (Hz)
  double df;   // bin spacing (Hz); 0 with one bin
  const double* pa;   // [J][3] array positions (m)
  const double* rot;  // [J][3][3] rotations, row-major (local -> global)
};

// one time step's inputs, all in device memory
struct MsgIn {
  int S, P;
  const double2* z;      // [J][N_z] observations
  const double* mt;      // [P][3] MT position particles
  const double* wb;      // [P] MT particle weights
  const double* sfv;     // [S][P][3] SFV particles (row 0 unused: LOS)
  const double* gamma;   // [S][P] amplitude variance particles
  const double2* mu;     // [S][P] amplitude mean particles
  const double* wa;      // [S][P] PF particle weights
  const double* zeta;    // [S][J] PR existence probabilities
  const double* eta;     // [J][P] noise variance particles
  const double* wxi;     // [J][P] noise particle weights
};

struct MsgOut {
  double* iota;    // [J][P] or null
  double* nu;      // [J][P] or null
  double* kappa;   // [S][J][P] (r = 1) or null
  double* kappa0;  // [S][J] (r = 0) or null
  double* omega;   // [S][J][2] or null
};

// lanes per (particle, array) group: the smallest of 4, 8, 16 that holds S
int msg_group(int S);
size_t msg_workspace_bytes(const MsgGeom& g, int S, int P);
hipError_t launch_messages(const MsgGeom& g, const MsgIn& in, const MsgOut& out, void* ws, hipStream_t s);

}  // namespace ba
