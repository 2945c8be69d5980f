// Adjoint (reverse-mode) state of the quasi-incompressible phase-field LBE
// step and the view of a context that the adjoint entry points use.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qilbm.h"
#include "qilbm_device.hpp"

namespace qilbm {

// Planes of the adjoint scratch fields (compute type), one per node.
enum AdjField : int {
  A_MU1 = 0,                   // mu (collision part)
  A_GMUX, A_GMUY, A_LMU,       // grad mu, lap mu
  A_GPHX, A_GPHY,              // grad phi
  A_PHI2,                      // phi after the velocity/force/pressure stage
  A_LPHI, A_PHI3,              // lap phi; phi after the mu stage
  A_NFIELDS
};

// Parameter cotangent slots, accumulated in FP64.
enum AdjParam : int { AP_BETA = 0, AP_KAPPA = 1, AP_LAMBDA = 2, AP_ALPHA = 3 };

struct AdjointState {
  bool active = false;
  char* ws = nullptr;
  size_t bytes = 0;
  char* hat[2] = {nullptr, nullptr};  // canonical adjoint populations, 18 planes
  int cur = 0;
  char* fld = nullptr;                // forward phi, mu, p
  char* afld = nullptr;               // A_NFIELDS planes
  double* part = nullptr;             // 4 regions x nred x 4
  double* acc = nullptr;              // running totals [4] + final outputs [4]
  int nred = 0;
  int resident = 0;                   // fused adjoint workgroups resident at once
};

struct CtxView {
  const lbm_params* prm;
  double beta, kappa, lam, alpha, gamma, drho;
  Geom geom;
  hipStream_t stream;
  AdjointState* adj;
  int64_t pbytes;
};

CtxView ctx_view(lbm_ctx* c);

}  // namespace qilbm
