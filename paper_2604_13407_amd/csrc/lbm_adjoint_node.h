// Reverse-mode (adjoint) arithmetic of one node's collision, written by hand
// from the forward arithmetic in lbm_node.h (collide_node), statement by
// statement in reverse order.
//
// Forward, at a fluid node: the pulled populations d (deviations), their sums
// drho, j; psi_c of the node and the stencil sums S of its neighbours' psi;
// F_int = -G psi_c S, F_ext (constant or buoyant), u = (j + F/2)/rho; moments
// m = M d; m^eq(rho, u), F_m(F, u), Q_m(G S S, u); mbar; fbar = M^-1 mbar.
//
// Reverse: given obar = dL/dfbar (9) and the loss's direct sensitivities to
// the node's rho, j, F and u, return dL/dd (9, through the collision only;
// the pseudopotential's dependence on rho is added by the caller), dL/dpsi_c,
// dL/dS (2) and the node's contributions to dL/dG and dL/d|F_ext|.
//
// The node functions after it are the per-node bodies of the reverse step's
// kernels (lbm_adjoint.hip), host-callable as well.
#pragma once

#include "lbm_adjoint_internal.h"
#include "lbm_node.h"

namespace pplbm {

// d p_EOS / d rho (van der Waals, Eq. 43; Carnahan-Starling), for psi'(rho).
__host__ __device__ inline double dp_eos(const StepParams& p, double r) {
  if (p.eos_kind == 0) {
    double inv = recip(1.0 - p.b * r);
    return p.k_eos * (p.RT * inv * inv - 2.0 * p.a * r);
  }
  // p = k (rho RT g(eta) - a rho^2), g = (1 + eta + eta^2 - eta^3)/(1 - eta)^3,
  // g' = (4 + 4 eta - 2 eta^2)/(1 - eta)^4, eta = b rho / 4.
  double eta = 0.25 * p.b * r;
  double om = 1.0 - eta;
  double inv = recip(om);
  double inv3 = inv * inv * inv;
  double g = (1.0 + eta * (1.0 + eta * (1.0 - eta))) * inv3;
  double gp = (4.0 + eta * (4.0 - 2.0 * eta)) * inv3 * inv;
  return p.k_eos * (p.RT * g + r * p.RT * gp * 0.25 * p.b - 2.0 * p.a * r);
}

// d psi / d rho with psi^2 = 2 (rho/3 - p): psi' = (1/3 - p')/psi (0 where psi = 0).
__host__ __device__ inline double dpsi_drho(const StepParams& p, double r, double psi) {
  if (!(psi > 0.0)) return 0.0;
  return (1.0 / 3.0 - dp_eos(p, r)) * recip(psi);
}

// Direct sensitivities of the loss to this node's pre-collision observables.
struct LossSens {
  double rho;     // dL/drho (direct)
  double jx, jy;  // dL/dj
  double fx, fy;  // dL/dF (total force)
  double ux, uy;  // dL/du
  double g;       // explicit dL/d|F_ext|
};

struct AdjOut {
  double dd[9];  // dL/d(pulled populations) through the collision
  double psi_c;  // dL/dpsi of this node
  double Sx, Sy; // dL/dS
  double G;      // contribution to dL/dG
  double g;      // contribution to dL/d|F_ext| (F_ext = |F_ext| times its fixed direction)
};

__host__ __device__ inline void collide_node_adjoint(const StepParams& p, double drho, double jx, double jy,
                                                     double psi_c, double Sx, double Sy, const double ob[9],
                                                     const LossSens& ls, AdjOut& out) {
  // ---------------- forward recomputation (the quantities the reverse needs)
  const double G = p.G;
  const double Fix = -G * psi_c * Sx;
  const double Fiy = -G * psi_c * Sy;
  const double r = p.rho_ref + drho;
  double Fex, Fey;
  const bool buoy = (p.force_mode == 1);
  if (buoy) {
    Fex = (r - p.rho_g) * p.fx;
    Fey = (r - p.rho_g) * p.fy;
  } else {
    Fex = p.fx;
    Fey = p.fy;
  }
  const double Fx = Fix + Fex, Fy = Fiy + Fey;
  const double inv_r = recip(r);
  const double ux = (jx + 0.5 * Fx) * inv_r;
  const double uy = (jy + 0.5 * Fy) * inv_r;
  const double U2 = ux * ux + uy * uy;
  const double Pxx = G * Sx * Sx, Pyy = G * Sy * Sy;

  // ---------------- reverse of fbar = M^-1 mbar: mbar_bar_k = (1/D_k) (M obar)_k
  const double s4o = (ob[1] + ob[3]) + (ob[2] + ob[4]);
  const double s8o = (ob[5] + ob[7]) + (ob[6] + ob[8]);
  const double b0 = (ob[0] + s4o + s8o) * (1.0 / 9.0);
  const double b1 = (2.0 * s8o - s4o - 4.0 * ob[0]) * (1.0 / 36.0);
  const double b2 = (4.0 * ob[0] - 2.0 * s4o + s8o) * (1.0 / 36.0);
  const double c57 = ob[5] - ob[7], c86 = ob[8] - ob[6];
  const double s13 = ob[1] - ob[3], s24 = ob[2] - ob[4];
  const double b3 = (s13 + (c57 + c86)) * (1.0 / 6.0);
  const double b4 = ((c57 + c86) - 2.0 * s13) * (1.0 / 12.0);
  const double b5 = (s24 + (c57 - c86)) * (1.0 / 6.0);
  const double b6 = ((c57 - c86) - 2.0 * s24) * (1.0 / 12.0);
  const double b7 = ((ob[1] + ob[3]) - (ob[2] + ob[4])) * 0.25;
  const double b8 = ((ob[5] + ob[7]) - (ob[6] + ob[8])) * 0.25;

  // adjoints of the intermediate quantities
  double a_drho = b0, a_jx = b3, a_jy = b5, a_Fx = b3, a_Fy = b5;
  double a_r = 0.0, a_ux = 0.0, a_uy = 0.0;
  // relaxation, mbar_k = (1 - s_k) m_k + s_k e_k +- h_k F_k + s_k Q_k
  const double am1 = (1.0 - p.s[1]) * b1, am2 = (1.0 - p.s[2]) * b2, am4 = (1.0 - p.s[4]) * b4;
  const double am6 = (1.0 - p.s[6]) * b6, am7 = (1.0 - p.s[7]) * b7, am8 = (1.0 - p.s[8]) * b8;
  const double ae1 = p.s[1] * b1, ae2 = p.s[2] * b2, ae4 = p.s[4] * b4, ae6 = p.s[6] * b6;
  const double ae7 = p.s[7] * b7, ae8 = p.s[8] * b8;
  const double aF1 = p.h[1] * b1 - p.h[2] * b2;
  a_Fx += -p.h[4] * b4;
  a_Fy += -p.h[6] * b6;
  const double aF7 = p.h[7] * b7, aF8 = p.h[8] * b8;
  double aQ1 = p.s[1] * b1;
  const double aQ2 = p.s[2] * b2, aQ4 = p.s[4] * b4, aQ6 = p.s[6] * b6;
  const double aQ7 = p.s[7] * b7, aQ8 = p.s[8] * b8;
  // source moments
  aQ1 += p.q2 * aQ2;
  const double aPxx = p.q1 * aQ1 + p.qa * ux * aQ4 - p.qb * uy * aQ6 + p.q7 * aQ7;
  const double aPyy = p.q1 * aQ1 - p.qb * ux * aQ4 + p.qa * uy * aQ6 - p.q7 * aQ7;
  const double aPxy = p.q7 * aQ8;
  a_ux += (p.qa * Pxx - p.qb * Pyy) * aQ4;
  a_uy += (p.qa * Pyy - p.qb * Pxx) * aQ6;
  double a_Sx = G * (2.0 * Sx * aPxx + Sy * aPxy);
  double a_Sy = G * (2.0 * Sy * aPyy + Sx * aPxy);
  double a_G = Sx * Sx * aPxx + Sy * Sy * aPyy + Sx * Sy * aPxy;
  // force moments: F1 = 6 (Fx ux + Fy uy), F7 = 2 (Fx ux - Fy uy), F8 = Fx uy + Fy ux
  const double aFu = 6.0 * aF1;
  a_Fx += ux * aFu + 2.0 * ux * aF7 + uy * aF8;
  a_Fy += uy * aFu - 2.0 * uy * aF7 + ux * aF8;
  a_ux += Fx * aFu + 2.0 * Fx * aF7 + Fy * aF8;
  a_uy += Fy * aFu - 2.0 * Fy * aF7 + Fx * aF8;
  // equilibria
  const double a12 = ae1 - ae2;  // e1 = -2 drho + 3 r U2, e2 = drho - 3 r U2
  a_drho += -2.0 * ae1 + ae2;
  a_r += 3.0 * U2 * a12;
  const double aU2 = 3.0 * r * a12;
  a_r += -ux * ae4 - uy * ae6 + (ux * ux - uy * uy) * ae7 + ux * uy * ae8;
  a_ux += -r * ae4 + 2.0 * r * ux * ae7 + r * uy * ae8 + 2.0 * ux * aU2;
  a_uy += -r * ae6 - 2.0 * r * uy * ae7 + r * ux * ae8 + 2.0 * uy * aU2;
  // loss sensitivities to u
  a_ux += ls.ux;
  a_uy += ls.uy;
  // u = (j + F/2) / r
  a_jx += inv_r * a_ux;
  a_jy += inv_r * a_uy;
  a_Fx += 0.5 * inv_r * a_ux;
  a_Fy += 0.5 * inv_r * a_uy;
  a_r += -(ux * a_ux + uy * a_uy) * inv_r;
  // loss sensitivities to rho, j
  a_r += ls.rho;
  a_jx += ls.jx;
  a_jy += ls.jy;
  // F = F_int + F_ext
  a_Fx += ls.fx;
  a_Fy += ls.fy;
  const double aFix = a_Fx, aFiy = a_Fy;
  double a_gmag = ls.g;
  if (buoy) {
    a_r += p.fx * a_Fx + p.fy * a_Fy;
    // F_ext = (r - rho_g) |g| ghat
    a_gmag += (r - p.rho_g) * (p.ghx * a_Fx + p.ghy * a_Fy);
  } else {
    a_gmag += p.ghx * a_Fx + p.ghy * a_Fy;
  }
  // F_int = -G psi_c S
  a_G += -psi_c * (Sx * aFix + Sy * aFiy);
  const double a_psi = -G * (Sx * aFix + Sy * aFiy);
  a_Sx += -G * psi_c * aFix;
  a_Sy += -G * psi_c * aFiy;
  // r = rho_ref + drho
  a_drho += a_r;

  // ---------------- into the pulled populations: drho = sum d, j = sum e d, m_k = (M d)_k
  // dd_i = a_drho + e_i . a_j + sum_k M[k][i] am_k
  const double A4 = -am1 - 2.0 * am2;  // common to i = 1..4 from m1, m2
  const double A8 = 2.0 * am1 + am2;   // common to i = 5..8
  out.dd[0] = a_drho - 4.0 * am1 + 4.0 * am2;
  out.dd[1] = a_drho + a_jx + A4 - 2.0 * am4 + am7;
  out.dd[2] = a_drho + a_jy + A4 - 2.0 * am6 - am7;
  out.dd[3] = a_drho - a_jx + A4 + 2.0 * am4 + am7;
  out.dd[4] = a_drho - a_jy + A4 + 2.0 * am6 - am7;
  out.dd[5] = a_drho + a_jx + a_jy + A8 + am4 + am6 + am8;
  out.dd[6] = a_drho - a_jx + a_jy + A8 - am4 + am6 - am8;
  out.dd[7] = a_drho - a_jx - a_jy + A8 - am4 - am6 + am8;
  out.dd[8] = a_drho + a_jx - a_jy + A8 + am4 - am6 - am8;
  out.psi_c = a_psi;
  out.Sx = a_Sx;
  out.Sy = a_Sy;
  out.G = a_G;
  out.g = a_gmag;
}

// ---------------------------------------------------------------- lattice-level reverse step
// The eight neighbours x + e_i of a node (i = 1..8): index (wrapped across
// periodic axes), whether the position is inside the box, whether it is a
// fluid node.  Computed once per node from the wrapped columns x-1, x, x+1 and
// rows y-1, y, y+1.
struct Nbrs {
  size_t k[9];
  bool inside[9];
  bool fluid[9];
};

__host__ __device__ inline void neighbours(const StepParams& p, const uint8_t* __restrict__ mask, int x, int y,
                                           Nbrs& nb) {
  int xs[3], ys[3];
  bool xin[3], yin[3];
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    int xx = x + d, yy = y + d;
    bool xi = true, yi = true;
    if (xx < 0 || xx >= p.nx) {
      xi = p.periodic_x != 0;
      xx = xx < 0 ? xx + p.nx : xx - p.nx;
    }
    if (yy < 0 || yy >= p.ny) {
      yi = p.periodic_y != 0;
      yy = yy < 0 ? yy + p.ny : yy - p.ny;
    }
    xs[d + 1] = xi ? xx : 0;
    ys[d + 1] = yi ? yy : 0;
    xin[d + 1] = xi;
    yin[d + 1] = yi;
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cx = ex(i) + 1, cy = ey(i) + 1;
    nb.inside[i] = xin[cx] && yin[cy];
    nb.k[i] = (size_t)ys[cy] * p.nx + xs[cx];
    nb.fluid[i] = nb.inside[i] && !(mask && mask[nb.k[i]]);
  }
}

// lambda_i(x) = dL/dfbar_i(x) of the state step n + 1 pulls from: the
// transpose of that step's pull.  P = D_next + R_next is the adjoint of the
// pulled populations; fbar_i(x) went to x + e_i when that node is fluid, and
// was bounced back into direction opp(i) at x otherwise.
template <class L>
__host__ __device__ inline double lambda_of(const StepParams& p, const AdjStepArgs& a, const Nbrs& nb, int i) {
  const size_t N = (size_t)p.nx * p.ny;
  const L* Dn = static_cast<const L*>(a.D_next);
  const L* Rn = static_cast<const L*>(a.R_next);
  const size_t k = nb.k[0];
  if (i != 0 && nb.fluid[i]) return (double)Dn[(size_t)i * N + nb.k[i]] + (double)Rn[nb.k[i]];
  return (double)Dn[(size_t)opp(i) * N + k] + (double)Rn[k];
}

// Replay: rho - rho_ref, j and psi of the state f pulled to node (x, y)
// (solid nodes: 0, 0, 0, psi_s).
template <class S>
__host__ __device__ inline void adj_traj_node(const StepParams& p, const S* __restrict__ f,
                                              const uint8_t* __restrict__ mask, double* __restrict__ traj, int x,
                                              int y) {
  const size_t N = (size_t)p.nx * p.ny;
  const size_t k = (size_t)y * p.nx + x;
  double dr = 0.0, jx = 0.0, jy = 0.0, ps = p.psi_solid;
  if (!(mask && mask[k])) {
    double d[9], c;
    pull_node<S>(p, f, mask, nullptr, x, y, d, nullptr, c);
    node_sums<S>(d, c, dr, jx, jy);
    bool bad;
    ps = psi_of(p, p.rho_ref + dr, bad);
  }
  traj[k] = dr;
  traj[N + k] = jx;
  traj[2 * N + k] = jy;
  traj[3 * N + k] = ps;
}

// psi of the replayed step at neighbour i, psi_s outside the box (solid
// nodes inside the box carry psi_s in the trajectory).
__host__ __device__ inline double psi_nbr(const StepParams& p, const double* __restrict__ psi, const Nbrs& nb, int i) {
  return nb.inside[i] ? psi[nb.k[i]] : p.psi_solid;
}

// Reverse of node (x, y)'s step n: gathers lambda^n from step n + 1, adds
// the loss's direct sensitivities at step n, reverses the collision.  Writes
// D^n and T^n of the node (rounded to L); adds its dL/dG, dL/d|F_ext| shares
// to part[0..1].
template <class L>
__host__ __device__ inline void adj_local_node(const StepParams& p, const AdjStepArgs& a, int x, int y,
                                               double part[2]) {
  const size_t N = (size_t)p.nx * p.ny;
  const size_t k = (size_t)y * p.nx + x;
  const bool fluid = !(a.mask && a.mask[k]);
  if (fluid) {
    Nbrs nb;
    neighbours(p, a.mask, x, y, nb);
    // lambda^n(x): transpose of step n+1's pull (zero after the last step)
    double ob[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) ob[i] = a.have_next ? lambda_of<L>(p, a, nb, i) : 0.0;
    const double drho = a.traj[k], jx = a.traj[N + k], jy = a.traj[2 * N + k];
    const double* psi = a.traj + 3 * N;
    const double pc = psi[k];
    double Sx, Sy;
    stencil_sums(psi_nbr(p, psi, nb, 1), psi_nbr(p, psi, nb, 2), psi_nbr(p, psi, nb, 3), psi_nbr(p, psi, nb, 4),
                 psi_nbr(p, psi, nb, 5), psi_nbr(p, psi, nb, 6), psi_nbr(p, psi, nb, 7), psi_nbr(p, psi, nb, 8), Sx,
                 Sy);
    // the loss's direct sensitivities at this step
    LossSens ls = {0, 0, 0, 0, 0, 0, 0, 0};
    const double r = p.rho_ref + drho;
    if (a.loss_kind == 0 && (a.cB != 0.0 || a.cP != 0.0)) {
      const double Fx = -p.G * pc * Sx + (p.force_mode == 1 ? (r - p.rho_g) * p.fx : p.fx);
      const double Fy = -p.G * pc * Sy + (p.force_mode == 1 ? (r - p.rho_g) * p.fy : p.fy);
      const double dl = p.rho_l - p.rho_g;
      const double phi = (r - p.rho_g) / dl;
      const double pg = (jx + 0.5 * Fx) * p.ghx + (jy + 0.5 * Fy) * p.ghy;
      // B = sum phi (rho - rho_g) |g|;  P = sum phi (j + F/2) . ghat
      ls.rho = a.cB * 2.0 * (r - p.rho_g) * p.gmag / dl + a.cP * pg / dl;
      ls.g = a.cB * (r - p.rho_g) * (r - p.rho_g) / dl;
      ls.jx = a.cP * phi * p.ghx;
      ls.jy = a.cP * phi * p.ghy;
      ls.fx = 0.5 * a.cP * phi * p.ghx;
      ls.fy = 0.5 * a.cP * phi * p.ghy;
    } else if (a.loss_kind == 1 && a.cU != 0.0) {
      const double Fx = -p.G * pc * Sx + (p.force_mode == 1 ? (r - p.rho_g) * p.fx : p.fx);
      const double ux = (jx + 0.5 * Fx) * recip(r);
      ls.ux = a.cU * 2.0 * (ux - a.u_target[k]);
    }
    AdjOut o;
    collide_node_adjoint(p, drho, jx, jy, pc, Sx, Sy, ob, ls, o);
#pragma unroll
    for (int i = 0; i < 9; ++i) static_cast<L*>(a.D)[(size_t)i * N + k] = (L)o.dd[i];
    L* T = static_cast<L*>(a.T);
    T[k] = (L)o.psi_c;
    T[N + k] = (L)o.Sx;
    T[2 * N + k] = (L)o.Sy;
    part[0] += o.G;
    part[1] += o.g;
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) static_cast<L*>(a.D)[(size_t)i * N + k] = (L)0;
    L* T = static_cast<L*>(a.T);
    T[k] = (L)0;
    T[N + k] = (L)0;
    T[2 * N + k] = (L)0;
  }
}

// dL/dpsi(x) = T_c(x) + sum_k w_k e_k . T_S(x - e_k), and R^n(x) = psi'(rho) dL/dpsi
// (T and R of type L).
template <class L>
__host__ __device__ inline void adj_psi_node(const StepParams& p, const AdjStepArgs& a, int x, int y) {
  const size_t N = (size_t)p.nx * p.ny;
  const size_t k = (size_t)y * p.nx + x;
  const L* T = static_cast<const L*>(a.T);
  L* R = static_cast<L*>(a.R);
  if (a.mask && a.mask[k]) {
    R[k] = (L)0;
    return;
  }
  // psi(x) enters S(x - e_i) = S(x + e_opp(i)) with weight w_i e_i
  Nbrs nb;
  neighbours(p, a.mask, x, y, nb);
  double pb = (double)T[k];
  const double w1 = 1.0 / 3.0, w2 = 1.0 / 12.0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int o = opp(i);
    if (nb.fluid[o]) {
      const size_t ks = nb.k[o];
      const double w = i <= 4 ? w1 : w2;
      pb += w * (ex(i) * (double)T[N + ks] + ey(i) * (double)T[2 * N + ks]);
    }
  }
  const double r = p.rho_ref + a.traj[k];
  R[k] = (L)(dpsi_drho(p, r, a.traj[3 * N + k]) * pb);
}

// dL/drho0(x) = sum_i w_i lambda^0_i(x), since fbar^0_i = w_i rho0 at rest
// (a.D_next, a.R_next: step 1).
template <class L>
__host__ __device__ inline double adj_rho0_node(const StepParams& p, const AdjStepArgs& a, int x, int y) {
  const size_t k = (size_t)y * p.nx + x;
  if (a.mask && a.mask[k]) return 0.0;
  Nbrs nb;
  neighbours(p, a.mask, x, y, nb);
  double g = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) g += wgt(i) * lambda_of<L>(p, a, nb, i);
  return g;
}


}  // namespace pplbm
