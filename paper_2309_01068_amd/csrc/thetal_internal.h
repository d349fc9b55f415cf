// Internal layout of the theta-L evolution object (shared with the warm-start code).
#pragma once

#include "../../include/thetal.h"
#include "common.h"

struct stefan;

namespace kfbi {
constexpr int kTLThreads = 1024;
constexpr int kTLMaxM = 2048;
// scal[] slots (device)
enum { S_L = 0, S_XBX, S_XBY, S_T, S_LPREV, S_MPREV, S_QPX, S_QPY, S_AREA, S_LEN, S_BAD, S_COUNT };
// aux[] planes of M doubles (device)
enum { A_THA = 0, A_HETA, A_NX, A_NY, A_R2, A_U, A_COUNT };
}  // namespace kfbi

struct thetaL {
  thetaL_params prm{};
  kfbi_ctx* kc = nullptr;
  hipStream_t stream = nullptr;
  int M = 0;           // current markers
  int Mcap = 0;        // largest M (refinement limit); buffers are sized for it
  int n = 0;           // steps taken
  int ready = 0;       // thetaL_init or set_state done
  int have_phi = 0;    // phi_prev holds a density
  // phi: density of the last solve, phi2: of the solve before it, phiw: working copy
  // (a step rotates the three buffers instead of copying)
  kfbi::DBuf tw, eta, scal, X, rhs, aux, etahat, nhat, phi, phi2, phiw, dnp, dnm, init;
  double* hscal = nullptr;  // copy of scal in coherent pinned host memory
  double* dscal = nullptr;  // its device address (the step's last kernel writes it)
  hipEvent_t tev[4] = {};   // timing of the phases that end without a host synchronisation
  // The shape pass that opens a step (reconstruction, right-hand side, shape data) is the
  // Stefan problem's when owner is set.  pre_n is the step count for which its outputs are
  // current because a learned guess has just formed them (the step then only copies its
  // initial guess), else -1.
  stefan* owner = nullptr;
  int pre_n = -1;
};


namespace kfbi {
// Recompute the per-marker shape data of the current state (aux planes, markers, rhs)
// without advancing it (used before a learned initial guess is formed).
int thetal_refresh(thetaL* th);
}  // namespace kfbi
