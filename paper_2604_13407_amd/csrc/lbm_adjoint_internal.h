// Launch interface of the adjoint kernels (lbm_adjoint.hip) for the host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_params.h"

namespace pplbm {

// One reverse step n.  Arrays are [plane][ny][nx]; D, R and T hold elements
// of type L (float for float storage, double for double storage), the rest
// doubles.
struct AdjStepArgs {
  const uint8_t* mask;      // solid nodes, or NULL
  const double* traj;       // [4]: rho - rho_ref, j_x, j_y, psi of step n's pulled state
  const void* D_next;       // [9] L: dL/d(pulled populations) of step n + 1 through its collision
  const void* R_next;       // [1] L: psi'(rho) dL/dpsi of step n + 1
  void* D;                  // [9] L: output for step n
  void* T;                  // [3] L: dL/dpsi_c, dL/dS_x, dL/dS_y of step n (scratch)
  void* R;                  // [1] L: output for step n
  double* param_acc;        // [blocks][2]: running dL/dG, dL/d|F_ext| per block
  const double* u_target;   // velocity-error loss: target u_x, [ny][nx]
  int32_t have_next;        // 0 for the last step (lambda^N = 0)
  int32_t loss_kind;        // 0 drag window, 1 velocity error
  double cB, cP, cU;        // loss weights of this step's observables
};

int adj_blocks(int nx, int ny);

template <class S>
hipError_t launch_traj(const StepParams& p, const void* f, const uint8_t* mask, double* traj, hipStream_t st);
template <class L>
hipError_t launch_adj_step(const StepParams& p, const AdjStepArgs& a, hipStream_t st);
template <class L>
hipError_t launch_adj_rho0(const StepParams& p, const AdjStepArgs& a, double* grad_rho0, hipStream_t st);
// sum over fluid nodes of (ux - ut)^2 and ut^2 into out[0..1] (partials: adj_blocks * 2 doubles)
hipError_t launch_uerr(const StepParams& p, const uint8_t* mask, const double* ux, const double* ut,
                       double* partials, double* out, hipStream_t st);
hipError_t launch_pair_sum(const double* partials, int n, double* out, hipStream_t st);
hipError_t launch_zero(double* ptr, size_t n, hipStream_t st);

}  // namespace pplbm
