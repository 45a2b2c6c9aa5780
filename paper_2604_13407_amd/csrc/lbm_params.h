// Parameter block shared by the host side of liblbm.so and its kernels.
// Everything a step needs is folded into this struct on the host and passed
// to every kernel by value.
#pragma once

#include <stdint.h>

namespace pplbm {

// Observables of one step, in this order (matches lbm_reduction).
enum Red {
  RED_MASS = 0,
  RED_MOMX,
  RED_MOMY,
  RED_WALLX,
  RED_WALLY,
  RED_UC_NUM,
  RED_UC_DEN,
  RED_BUOY,
  RED_PPHI,
  RED_FAULTS,
  RED_COUNT
};

struct StepParams {
  int32_t nx, ny;
  int32_t periodic_x, periodic_y;
  int32_t eos_kind;    // 0 = van der Waals, 1 = Carnahan-Starling
  int32_t force_mode;  // 0 = constant, 1 = buoyant
  double rho_ref;      // stored deviation reference (0 for the FP64 path)
  // equation of state p = k (rho RT g(rho) - a rho^2)
  double a, b, RT, k_eos;
  double G;            // interaction strength (Eq. 4)
  double psi_solid;    // psi(rho_s), pseudopotential of solid nodes
  // collision rates s_k and (1 - s_k / 2)
  double s[9];
  double h[9];
  // source term coefficients (Eq. 11, Eqs. 13 + 42):
  // Q1 = q1 (Pxx + Pyy), Q2 = q2 Q1, Q7 = q7 (Pxx - Pyy), Q8 = q7 Pxy,
  // Q4 = (qa Pxx - qb Pyy) u_x, Q6 = (qa Pyy - qb Pxx) u_y,  P_ab = F_a F_b / (G psi^2)
  double q1, q2, q7, qa, qb;
  // external force / gravity
  double fx, fy;
  double rho_g, rho_l;
  double gmag, ghx, ghy;  // |(fx, fy)| and its unit vector (observables)
};

}  // namespace pplbm
